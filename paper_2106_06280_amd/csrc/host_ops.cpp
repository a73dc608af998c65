// Per-element operators of the CSWENO limiter (Section 3.2).  Everything
// here depends on the mesh only, so it is built once per mesh; the
// per-stage kernel applies these operators to the current coefficients.
//
// For element e (= Delta0) and its faces f = 0, 1, 2 (neighbours
// Delta_{f+1}; a periodic neighbour is translated next to e, a
// transmissive face gets the mirror image of e):
//   AVG[f][p][n]  average over piece p of the source element's psi_n, so a
//                 piece average is AVG . (source coefficients).  Pieces:
//                 S1 = (G, w_f', w_f'+1) touching e, S2 = (G, w_f'+1, w_f'+2),
//                 S3 = (G, w_f'+2, w_f'); for N >= 2 also S2' = (G, w_f'+1, F2),
//                 S21 = (G, F2, w_f'+2), S3' = (G, w_f'+2, F3), S31 = (G, F3, w_f')
//                 with F2, F3 the feet of the perpendiculars from the
//                 neighbour's centroid G to its outer sides (Fig. 2).
//   X2, X3, X5    least-squares pseudo-inverses (Householder QR) of the
//                 constrained fits q_2 (linear, rows S1 x 3 faces), q_3
//                 (quadratic, rows S1, S2, S3 x 3) and the top level on T4
//                 (rows S1, S2', S21, S3', S31 x 3): the quartic q_5, or
//                 for the cubic readings the cubic q_4 in X5's first nine
//                 rows, in the scaled monomials
//                 ((x-x0)/h0)^a ((y-y0)/h0)^b, 1 <= a+b, minus their mean
//                 over e; the right-hand side is (piece average - mean of e).
//   BP            the smoothness-indicator matrix of eq. smoothnessIndicator:
//                 c^T B c = sum_{1<=|alpha|<=DTOP} |e|^{|alpha|-1} int_e (D^alpha q)^2
//                 for q = sum c_j phi_j (physical derivatives); lower-degree
//                 levels use its leading block (higher derivatives vanish).
//   MINV          per face, the inverse of the centroid differences of
//                 S2 - S1 and S3 - S1, giving the gradient of the linear
//                 functions of eq. sigmaEqn.
//   PM            (1/J) int_e phi_j psi_i for i >= 1: the L2 projection of
//                 the reconstruction onto the basis.
//   GBASE         b of the linear weights gamma_bar_l = b^(l-1): 1/h0, or 10.
#include <algorithm>
#include <cmath>
#include <thread>
#include <type_traits>

#include "internal.h"

namespace cswdg {

namespace {

struct P2d {
    double x, y;
};

inline P2d operator+(P2d a, P2d b) { return {a.x + b.x, a.y + b.y}; }
inline P2d operator-(P2d a, P2d b) { return {a.x - b.x, a.y - b.y}; }
inline P2d operator*(double s, P2d a) { return {s * a.x, s * a.y}; }
inline double dot(P2d a, P2d b) { return a.x * b.x + a.y * b.y; }
inline double tri_area(P2d a, P2d b, P2d c) {
    return 0.5 * ((b.x - a.x) * (c.y - a.y) - (c.x - a.x) * (b.y - a.y));
}

struct Frame {  // maps placed coordinates to the source element's physical frame
    bool mirror;
    P2d shift;  // subtract (real neighbour)
    P2d P, Q;   // mirror line (ghost)
    P2d apply(P2d x) const {
        if (!mirror) return x - shift;
        P2d d = Q - P;
        double t = dot(x - P, d) / dot(d, d);
        P2d F = P + t * d;
        return 2.0 * F - x;
    }
};

// Householder QR pseudo-inverse X (c x r) of A (r x c), r <= 32.
bool pinv(int r, int c, const double* A, double* X) {
    constexpr int NMAX = 32;
    if (r > NMAX || c > r) return false;
    double R[NMAX][NMAX], QT[NMAX][NMAX];
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j) R[i][j] = A[i * c + j];
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j) QT[i][j] = (i == j) ? 1.0 : 0.0;
    for (int k = 0; k < c; ++k) {
        double nrm = 0;
        for (int i = k; i < r; ++i) nrm += R[i][k] * R[i][k];
        nrm = std::sqrt(nrm);
        if (nrm == 0) continue;
        double alpha = R[k][k] > 0 ? -nrm : nrm;
        double v[NMAX];
        for (int i = 0; i < r; ++i) v[i] = 0;
        for (int i = k; i < r; ++i) v[i] = R[i][k];
        v[k] -= alpha;
        double vv = 0;
        for (int i = k; i < r; ++i) vv += v[i] * v[i];
        if (vv == 0) continue;
        for (int j = 0; j < c; ++j) {
            double s = 0;
            for (int i = k; i < r; ++i) s += v[i] * R[i][j];
            s = 2 * s / vv;
            for (int i = k; i < r; ++i) R[i][j] -= s * v[i];
        }
        for (int j = 0; j < r; ++j) {
            double s = 0;
            for (int i = k; i < r; ++i) s += v[i] * QT[i][j];
            s = 2 * s / vv;
            for (int i = k; i < r; ++i) QT[i][j] -= s * v[i];
        }
    }
    double dmax = 0, dmin = INFINITY;
    for (int k = 0; k < c; ++k) {
        dmax = std::max(dmax, std::fabs(R[k][k]));
        dmin = std::min(dmin, std::fabs(R[k][k]));
    }
    if (!(dmin > 1e-12 * dmax)) return false;
    // X = R^{-1} QT[0:c, :]
    for (int col = 0; col < r; ++col) {
        double y[NMAX];
        for (int i = c - 1; i >= 0; --i) {
            double s = QT[i][col];
            for (int j = i + 1; j < c; ++j) s -= R[i][j] * y[j];
            y[i] = s / R[i][i];
        }
        for (int i = 0; i < c; ++i) X[i * r + col] = y[i];
    }
    return true;
}

constexpr int kMonoMax = 27;  // monomials of degree 1..6

struct MonoList {
    int a[kMonoMax], b[kMonoMax], n;
    explicit MonoList(int d) : n(0) {
        for (int s = 1; s <= d; ++s)
            for (int bb = 0; bb <= s; ++bb) {
                a[n] = s - bb;
                b[n] = bb;
                ++n;
            }
    }
};

template <int N, int QT>
struct OpBuilder {
    using D = Dims<N>;
    using L = OpLayout<N, QT>;
    const HostMesh& m;
    bool constant_gamma;
    bool ghost_extrapolate;  // outflow faces: Delta0's polynomial continued, not mirrored
    std::vector<double> C;  // basis monomial form [NP][NP]
    Rule2D rN, rTop, rBeta, rProj;
    std::vector<double> psiProj;  // [q][NP] on rProj
    MonoList mono{L::DR};

    OpBuilder(const HostMesh& mm, bool cg, bool ge) : m(mm), constant_gamma(cg), ghost_extrapolate(ge) {
        basis_monomial_form(N, C);
        rN = triangle_rule((N + 2) / 2);
        rTop = triangle_rule((L::DR + 2) / 2);
        rBeta = triangle_rule(L::DR);
        rProj = triangle_rule((L::DR + N + 2) / 2);
        psiProj.resize(rProj.w.size() * D::NP);
        for (size_t q = 0; q < rProj.w.size(); ++q) basis_eval(N, rProj.r[q], rProj.s[q], &psiProj[q * D::NP]);
    }

    P2d vert(int64_t e, int k) const { return {m.vx[k * m.K + e], m.vy[k * m.K + e]}; }

    void psi_mono(double r, double s, double* psi) const {
        double pw[D::NP];
        int k = 0;
        for (int d = 0; d <= N; ++d)
            for (int bb = 0; bb <= d; ++bb) {
                int aa = d - bb;
                double v = 1.0;
                for (int t = 0; t < aa; ++t) v *= r;
                for (int t = 0; t < bb; ++t) v *= s;
                pw[k++] = v;
            }
        for (int n = 0; n < D::NP; ++n) {
            double acc = 0;
            for (int kk = 0; kk < D::NP; ++kk) acc += C[n * D::NP + kk] * pw[kk];
            psi[n] = acc;
        }
    }

    // reference coordinates of physical point x in element src
    void to_ref(int64_t src, P2d x, double& r, double& s) const {
        P2d v0 = vert(src, 0), v1 = vert(src, 1), v2 = vert(src, 2);
        double xr = 0.5 * (v1.x - v0.x), xs = 0.5 * (v2.x - v0.x);
        double yr = 0.5 * (v1.y - v0.y), ys = 0.5 * (v2.y - v0.y);
        double J = xr * ys - xs * yr;
        double dx = x.x - v0.x, dy = x.y - v0.y;
        r = -1.0 + (ys * dx - xs * dy) / J;
        s = -1.0 + (-yr * dx + xr * dy) / J;
    }

    static P2d map_tri(const P2d* T, double r, double s) {
        return T[0] + (0.5 * (1.0 + r)) * (T[1] - T[0]) + (0.5 * (1.0 + s)) * (T[2] - T[0]);
    }

    void mono_eval(P2d x, P2d c0, double h0, double* out) const {
        double xi = (x.x - c0.x) / h0, eta = (x.y - c0.y) / h0;
        for (int j = 0; j < mono.n; ++j) {
            double v = 1.0;
            for (int t = 0; t < mono.a[j]; ++t) v *= xi;
            for (int t = 0; t < mono.b[j]; ++t) v *= eta;
            out[j] = v;
        }
    }

    // returns valid flag; counts feet outside their side
    bool build(int64_t e, double* op, int64_t& nfoot) const {
        for (int i = 0; i < L::LEN; ++i) op[i] = 0.0;
        P2d V0[3] = {vert(e, 0), vert(e, 1), vert(e, 2)};
        P2d c0 = (1.0 / 3.0) * (V0[0] + V0[1] + V0[2]);
        double la = std::sqrt(dot(V0[1] - V0[0], V0[1] - V0[0]));
        double lb = std::sqrt(dot(V0[2] - V0[1], V0[2] - V0[1]));
        double lc = std::sqrt(dot(V0[0] - V0[2], V0[0] - V0[2]));
        double h0 = (la + lb + lc) / 3.0;
        double area0 = tri_area(V0[0], V0[1], V0[2]);
        double J0 = 0.5 * area0;

        // monomial means over e
        double mavg0[kMonoMax] = {0};
        {
            double tmp[kMonoMax];
            double wsum = 0;
            for (size_t q = 0; q < rTop.w.size(); ++q) {
                mono_eval(map_tri(V0, rTop.r[q], rTop.s[q]), c0, h0, tmp);
                for (int j = 0; j < mono.n; ++j) mavg0[j] += rTop.w[q] * tmp[j];
                wsum += rTop.w[q];
            }
            for (int j = 0; j < mono.n; ++j) mavg0[j] /= wsum;
        }

        double mavg[3][L::NPC][kMonoMax];
        P2d cen[3][3];
        for (int f = 0; f < 3; ++f) {
            uint8_t inf = m.info[3 * e + f];
            Frame fr;
            P2d W[3];
            int fp;
            int64_t src;
            if (inf & 0x40) {
                fr.mirror = true;
                fr.P = V0[f];
                fr.Q = V0[(f + 1) % 3];
                P2d R = fr.apply(V0[(f + 2) % 3]);
                W[0] = V0[(f + 1) % 3];
                W[1] = V0[f];
                W[2] = R;
                fp = 0;
                src = e;
                if (ghost_extrapolate && (inf & 3) == 0) {
                    // outflow: the ghost triangle carries Delta0's own
                    // polynomial at its points (no reflection)
                    fr.mirror = false;
                    fr.shift = {0.0, 0.0};
                }
            } else {
                int cx = (inf >> 2) & 3, cy = (inf >> 4) & 3;
                double sx = cx == 1 ? m.px : (cx == 2 ? -m.px : 0.0);
                double sy = cy == 1 ? m.py : (cy == 2 ? -m.py : 0.0);
                fr.mirror = false;
                fr.shift = {sx, sy};
                src = m.nbr[3 * e + f];
                for (int k = 0; k < 3; ++k) W[k] = vert(src, k) + fr.shift;
                fp = inf & 3;
            }
            P2d G = (1.0 / 3.0) * (W[0] + W[1] + W[2]);
            P2d wa = W[fp], wb = W[(fp + 1) % 3], wc = W[(fp + 2) % 3];
            P2d pcs[L::NPC][3] = {{G, wa, wb}, {G, wb, wc}, {G, wc, wa}};
            if (L::NPC >= 7) {
                auto foot = [&](P2d p, P2d q) {
                    P2d d = q - p;
                    double t = dot(G - p, d) / dot(d, d);
                    if (!(t > 0.0 && t < 1.0)) {
                        t = 0.5;
                        ++nfoot;
                    }
                    return p + t * d;
                };
                P2d F2 = foot(wb, wc), F3 = foot(wc, wa);
                P2d extra[4][3] = {{G, wb, F2}, {G, F2, wc}, {G, wc, F3}, {G, F3, wa}};
                for (int p = 0; p < 4; ++p)
                    for (int k = 0; k < 3; ++k) pcs[3 + p][k] = extra[p][k];
                if (L::SEXT) {
                    // T5: the boundary divided at the vertices, the feet and
                    // the midpoints of the five segments; fan from G
                    const P2d ring[5] = {wa, wb, F2, wc, F3};
                    P2d pts[10];
                    for (int k = 0; k < 5; ++k) {
                        pts[2 * k] = ring[k];
                        pts[2 * k + 1] = 0.5 * (ring[k] + ring[(k + 1) % 5]);
                    }
                    for (int k = 0; k < 10; ++k) {
                        pcs[7 + k][0] = G;
                        pcs[7 + k][1] = pts[k];
                        pcs[7 + k][2] = pts[(k + 1) % 10];
                    }
                }
            }
            for (int p = 0; p < 3; ++p) cen[f][p] = (1.0 / 3.0) * (pcs[p][0] + pcs[p][1] + pcs[p][2]);
            for (int p = 0; p < L::NPC; ++p) {
                // average of psi_n of the source element
                double acc[D::NP] = {0};
                double wsum = 0, psi[D::NP];
                for (size_t q = 0; q < rN.w.size(); ++q) {
                    P2d x = fr.apply(map_tri(pcs[p], rN.r[q], rN.s[q]));
                    double r, s;
                    to_ref(src, x, r, s);
                    psi_mono(r, s, psi);
                    for (int n = 0; n < D::NP; ++n) acc[n] += rN.w[q] * psi[n];
                    wsum += rN.w[q];
                }
                for (int n = 0; n < D::NP; ++n) op[L::AVG + (f * L::NPC + p) * D::NP + n] = acc[n] / wsum;
                // scaled-monomial averages
                double ma[kMonoMax] = {0}, tmp[kMonoMax];
                wsum = 0;
                for (size_t q = 0; q < rTop.w.size(); ++q) {
                    mono_eval(map_tri(pcs[p], rTop.r[q], rTop.s[q]), c0, h0, tmp);
                    for (int j = 0; j < mono.n; ++j) ma[j] += rTop.w[q] * tmp[j];
                    wsum += rTop.w[q];
                }
                for (int j = 0; j < mono.n; ++j) mavg[f][p][j] = ma[j] / wsum - mavg0[j];
            }
            // gradient of the linear function through the centroid subcells
            double m00 = cen[f][1].x - cen[f][0].x, m01 = cen[f][1].y - cen[f][0].y;
            double m10 = cen[f][2].x - cen[f][0].x, m11 = cen[f][2].y - cen[f][0].y;
            double det = m00 * m11 - m01 * m10;
            double* mi = op + L::MINV + 4 * f;
            mi[0] = m11 / det;
            mi[1] = -m01 / det;
            mi[2] = -m10 / det;
            mi[3] = m00 / det;
        }

        bool valid = true;
        // linear level: rows S1 of faces 0..2, columns monomials of degree 1
        {
            double A[3 * 2];
            for (int f = 0; f < 3; ++f)
                for (int j = 0; j < 2; ++j) A[f * 2 + j] = mavg[f][0][j];
            valid &= pinv(3, 2, A, op + L::X2);
        }
        // quadratic level: rows S1 f0..2, S2 f0..2, S3 f0..2
        {
            double A[9 * 5];
            for (int p = 0; p < 3; ++p)
                for (int f = 0; f < 3; ++f)
                    for (int j = 0; j < 5; ++j) A[(p * 3 + f) * 5 + j] = mavg[f][p][j];
            valid &= pinv(9, 5, A, op + L::X3);
        }
        if (L::FOUR) {
            // top level on T4: rows S1, S2', S21, S3', S31 (pieces 0, 3, 4,
            // 5, 6) x faces; columns the 14 quartic or the 9 cubic monomials;
            // the sextic: rows the ten T5 pieces (7..16) x faces, 27 columns
            const int pl[5] = {0, 3, 4, 5, 6};
            constexpr int nc = L::NT > 0 ? L::NT : 1, nk = L::NROW / 3;
            double A[L::NROW * nc];
            for (int k = 0; k < nk; ++k)
                for (int f = 0; f < 3; ++f)
                    for (int j = 0; j < nc; ++j) A[(k * 3 + f) * nc + j] = mavg[f][L::SEXT ? 7 + k : pl[k]][j];
            valid &= pinv(L::NROW, nc, A, op + L::X5);
        }

        // smoothness-indicator matrix (all derivative orders of the
        // monomials, and orders 1..N only for the literal reading)
        {
            const int nm = mono.n;
            double B[kMonoMax][kMonoMax] = {{0}};
            double BL[kMonoMax][kMonoMax] = {{0}};
            double ihp[L::DR + 1], ap[L::DR + 1];
            ihp[0] = 1.0;
            ap[0] = 1.0 / area0;
            for (int s = 1; s <= L::DR; ++s) {
                ihp[s] = ihp[s - 1] / h0;
                ap[s] = ap[s - 1] * area0;
            }
            for (size_t q = 0; q < rBeta.w.size(); ++q) {
                P2d x = map_tri(V0, rBeta.r[q], rBeta.s[q]);
                double xi = (x.x - c0.x) / h0, eta = (x.y - c0.y) / h0;
                double wq = J0 * rBeta.w[q];
                for (int s = 1; s <= L::DR; ++s)
                    for (int a1 = 0; a1 <= s; ++a1) {
                        int a2 = s - a1;
                        double Dv[kMonoMax];
                        for (int j = 0; j < nm; ++j) {
                            int a = mono.a[j], b = mono.b[j];
                            if (a < a1 || b < a2) {
                                Dv[j] = 0;
                                continue;
                            }
                            double coef = 1.0;
                            for (int t = 0; t < a1; ++t) coef *= (a - t);
                            for (int t = 0; t < a2; ++t) coef *= (b - t);
                            double v = coef * ihp[s];
                            for (int t = 0; t < a - a1; ++t) v *= xi;
                            for (int t = 0; t < b - a2; ++t) v *= eta;
                            Dv[j] = v;
                        }
                        double sc = ap[s] * wq;
                        for (int i = 0; i < nm; ++i)
                            for (int j = 0; j < nm; ++j) B[i][j] += sc * Dv[i] * Dv[j];
                        if (s <= N)
                            for (int i = 0; i < nm; ++i)
                                for (int j = 0; j < nm; ++j) BL[i][j] += sc * Dv[i] * Dv[j];
                    }
            }
            int k = 0;
            for (int i = 0; i < nm; ++i)
                for (int j = i; j < nm; ++j) {
                    op[L::BP + k] = B[i][j];
                    op[L::BPL + k] = BL[i][j];
                    ++k;
                }
        }
        // projection onto psi_1..psi_{NP-1}
        {
            double tmp[kMonoMax];
            for (size_t q = 0; q < rProj.w.size(); ++q) {
                mono_eval(map_tri(V0, rProj.r[q], rProj.s[q]), c0, h0, tmp);
                for (int i = 1; i < D::NP; ++i)
                    for (int j = 0; j < mono.n; ++j)
                        op[L::PM + (i - 1) * L::NM + j] += rProj.w[q] * tmp[j] * psiProj[q * D::NP + i];
            }
        }
        // linear weights gamma_bar_l = b^(l-1) (Section 3.2, Step 2): b = 1/h0,
        // or the constant 10 of the reference cited there
        op[L::GBASE] = constant_gamma ? 10.0 : 1.0 / h0;
        op[L::AREA0] = area0;
        op[L::VALID] = valid ? 1.0 : 0.0;
        return valid;
    }
};

template <int N, int QT>
int build_ops_n(const HostMesh& m, bool constant_gamma, bool ghost_extrapolate, std::vector<double>& ops,
                int64_t& n_rank, int64_t& n_foot) {
    using L = OpLayout<N, QT>;
    OpBuilder<N, QT> b(m, constant_gamma, ghost_extrapolate);
    ops.assign((size_t)m.K * L::LEN, 0.0);
    unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    std::vector<int64_t> rank(nt, 0), foot(nt, 0);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            for (int64_t e = t; e < m.K; e += nt)
                if (!b.build(e, &ops[(size_t)e * L::LEN], foot[t])) ++rank[t];
        });
    for (auto& x : th) x.join();
    n_rank = n_foot = 0;
    for (unsigned t = 0; t < nt; ++t) {
        n_rank += rank[t];
        n_foot += foot[t];
    }
    return CSWDG_OK;
}

// The smoothness-indicator matrix of eq. smoothnessIndicator over the
// derivative orders 1..nd for q = sum_j c_j phi_j in the scaled monomials of
// mono on triangle V0 (centroid c0, mean side h0, area area0): c^T B c =
// sum_{1<=|alpha|<=nd} area0^{|alpha|-1} int (D^alpha q)^2, physical
// derivatives, by the rule rBeta; the packed upper triangle is written.
void smoothness_matrix_packed(int nd, const P2d V0[3], P2d c0, double h0, double area0, const Rule2D& rBeta,
                              const MonoList& mono, double* packed) {
    const int NM = mono.n;
    double B[5][5] = {{0}};
    double ihp[3], ap[3];
    ihp[0] = 1.0;
    ap[0] = 1.0 / area0;
    for (int sd = 1; sd <= nd; ++sd) {
        ihp[sd] = ihp[sd - 1] / h0;
        ap[sd] = ap[sd - 1] * area0;
    }
    const double J0 = 0.5 * area0;
    for (size_t q = 0; q < rBeta.w.size(); ++q) {
        const P2d x = V0[0] + (0.5 * (1.0 + rBeta.r[q])) * (V0[1] - V0[0]) + (0.5 * (1.0 + rBeta.s[q])) * (V0[2] - V0[0]);
        const double xi = (x.x - c0.x) / h0, eta = (x.y - c0.y) / h0;
        const double wq = J0 * rBeta.w[q];
        for (int sd = 1; sd <= nd; ++sd)
            for (int a1 = 0; a1 <= sd; ++a1) {
                const int a2 = sd - a1;
                double Dv[5];
                for (int j = 0; j < NM; ++j) {
                    const int a = mono.a[j], b = mono.b[j];
                    if (a < a1 || b < a2) {
                        Dv[j] = 0;
                        continue;
                    }
                    double coef = 1.0;
                    for (int t = 0; t < a1; ++t) coef *= (a - t);
                    for (int t = 0; t < a2; ++t) coef *= (b - t);
                    double v = coef * ihp[sd];
                    for (int t = 0; t < a - a1; ++t) v *= xi;
                    for (int t = 0; t < b - a2; ++t) v *= eta;
                    Dv[j] = v;
                }
                const double sc = ap[sd] * wq;
                for (int i = 0; i < NM; ++i)
                    for (int j = 0; j < NM; ++j) B[i][j] += sc * Dv[i] * Dv[j];
            }
    }
    int k = 0;
    for (int i = 0; i < NM; ++i)
        for (int j = i; j < NM; ++j) packed[k++] = B[i][j];
}

// The record of the type-I reconstruction (OpLayoutT1): the same stencil
// geometry as the hierarchical one (centroid subcells only), least-squares
// pseudo-inverses of degree N on the central stencil and the three sectors.
template <int N>
struct OpBuilderT1 {
    using D = Dims<N>;
    using L = OpLayoutT1<N>;
    const HostMesh& m;
    std::vector<double> C;
    Rule2D rN, rTop, rBeta, rProj;
    std::vector<double> psiProj;
    MonoList mono{N};

    explicit OpBuilderT1(const HostMesh& mm) : m(mm) {
        basis_monomial_form(N, C);
        rN = triangle_rule((N + 2) / 2);
        rTop = triangle_rule((N + 2) / 2);
        rBeta = triangle_rule(N > 1 ? N : 1);
        rProj = triangle_rule(N + 1);
        psiProj.resize(rProj.w.size() * D::NP);
        for (size_t q = 0; q < rProj.w.size(); ++q) basis_eval(N, rProj.r[q], rProj.s[q], &psiProj[q * D::NP]);
    }

    P2d vert(int64_t e, int k) const { return {m.vx[k * m.K + e], m.vy[k * m.K + e]}; }

    void psi_mono(double r, double s, double* psi) const {
        double pw[D::NP];
        int k = 0;
        for (int d = 0; d <= N; ++d)
            for (int bb = 0; bb <= d; ++bb) {
                double v = 1.0;
                for (int t = 0; t < d - bb; ++t) v *= r;
                for (int t = 0; t < bb; ++t) v *= s;
                pw[k++] = v;
            }
        for (int n = 0; n < D::NP; ++n) {
            double acc = 0;
            for (int kk = 0; kk < D::NP; ++kk) acc += C[n * D::NP + kk] * pw[kk];
            psi[n] = acc;
        }
    }

    void to_ref(int64_t src, P2d x, double& r, double& s) const {
        P2d v0 = vert(src, 0), v1 = vert(src, 1), v2 = vert(src, 2);
        double xr = 0.5 * (v1.x - v0.x), xs = 0.5 * (v2.x - v0.x);
        double yr = 0.5 * (v1.y - v0.y), ys = 0.5 * (v2.y - v0.y);
        double J = xr * ys - xs * yr;
        double dx = x.x - v0.x, dy = x.y - v0.y;
        r = -1.0 + (ys * dx - xs * dy) / J;
        s = -1.0 + (-yr * dx + xr * dy) / J;
    }

    static P2d map_tri(const P2d* T, double r, double s) {
        return T[0] + (0.5 * (1.0 + r)) * (T[1] - T[0]) + (0.5 * (1.0 + s)) * (T[2] - T[0]);
    }

    void mono_eval(P2d x, P2d c0, double h0, double* out) const {
        double xi = (x.x - c0.x) / h0, eta = (x.y - c0.y) / h0;
        for (int j = 0; j < mono.n; ++j) {
            double v = 1.0;
            for (int t = 0; t < mono.a[j]; ++t) v *= xi;
            for (int t = 0; t < mono.b[j]; ++t) v *= eta;
            out[j] = v;
        }
    }

    bool build(int64_t e, double* op) const {
        constexpr int NM = L::NM;
        for (int i = 0; i < L::LEN; ++i) op[i] = 0.0;
        P2d V0[3] = {vert(e, 0), vert(e, 1), vert(e, 2)};
        P2d c0 = (1.0 / 3.0) * (V0[0] + V0[1] + V0[2]);
        double h0 = (std::sqrt(dot(V0[1] - V0[0], V0[1] - V0[0])) + std::sqrt(dot(V0[2] - V0[1], V0[2] - V0[1])) +
                     std::sqrt(dot(V0[0] - V0[2], V0[0] - V0[2]))) / 3.0;
        double area0 = tri_area(V0[0], V0[1], V0[2]);
        double mavg0[5] = {0}, tmp[5];
        {
            double wsum = 0;
            for (size_t q = 0; q < rTop.w.size(); ++q) {
                mono_eval(map_tri(V0, rTop.r[q], rTop.s[q]), c0, h0, tmp);
                for (int j = 0; j < NM; ++j) mavg0[j] += rTop.w[q] * tmp[j];
                wsum += rTop.w[q];
            }
            for (int j = 0; j < NM; ++j) mavg0[j] /= wsum;
        }
        double mavg[3][3][5];
        for (int f = 0; f < 3; ++f) {
            uint8_t inf = m.info[3 * e + f];
            bool mirror = false;
            P2d shift{0.0, 0.0}, P{0, 0}, Q{0, 0}, W[3];
            int fp;
            int64_t src;
            if (inf & 0x40) {
                mirror = true;
                P = V0[f];
                Q = V0[(f + 1) % 3];
                P2d d = Q - P;
                P2d X = V0[(f + 2) % 3];
                P2d F = P + (dot(X - P, d) / dot(d, d)) * d;
                W[0] = Q;
                W[1] = P;
                W[2] = 2.0 * F - X;
                fp = 0;
                src = e;
            } else {
                int cx = (inf >> 2) & 3, cy = (inf >> 4) & 3;
                shift = {cx == 1 ? m.px : (cx == 2 ? -m.px : 0.0), cy == 1 ? m.py : (cy == 2 ? -m.py : 0.0)};
                src = m.nbr[3 * e + f];
                for (int k = 0; k < 3; ++k) W[k] = vert(src, k) + shift;
                fp = inf & 3;
            }
            auto back = [&](P2d x) {
                if (!mirror) return x - shift;
                P2d d = Q - P;
                P2d F = P + (dot(x - P, d) / dot(d, d)) * d;
                return 2.0 * F - x;
            };
            P2d G = (1.0 / 3.0) * (W[0] + W[1] + W[2]);
            P2d wa = W[fp], wb = W[(fp + 1) % 3], wc = W[(fp + 2) % 3];
            P2d pcs[3][3] = {{G, wa, wb}, {G, wb, wc}, {G, wc, wa}};
            for (int p = 0; p < 3; ++p) {
                double acc[D::NP] = {0}, psi[D::NP], wsum = 0;
                for (size_t q = 0; q < rN.w.size(); ++q) {
                    double r, s;
                    to_ref(src, back(map_tri(pcs[p], rN.r[q], rN.s[q])), r, s);
                    psi_mono(r, s, psi);
                    for (int n = 0; n < D::NP; ++n) acc[n] += rN.w[q] * psi[n];
                    wsum += rN.w[q];
                }
                for (int n = 0; n < D::NP; ++n) op[L::AVG + (f * 3 + p) * D::NP + n] = acc[n] / wsum;
                double ma[5] = {0};
                wsum = 0;
                for (size_t q = 0; q < rTop.w.size(); ++q) {
                    mono_eval(map_tri(pcs[p], rTop.r[q], rTop.s[q]), c0, h0, tmp);
                    for (int j = 0; j < NM; ++j) ma[j] += rTop.w[q] * tmp[j];
                    wsum += rTop.w[q];
                }
                for (int j = 0; j < NM; ++j) mavg[f][p][j] = ma[j] / wsum - mavg0[j];
            }
        }
        bool valid = true;
        {
            double A[9 * 5];
            for (int p = 0; p < 3; ++p)
                for (int f = 0; f < 3; ++f)
                    for (int j = 0; j < NM; ++j) A[(p * 3 + f) * NM + j] = mavg[f][p][j];
            valid &= pinv(9, NM, A, op + L::XC);
        }
        for (int k = 0; k < 3; ++k) {
            const int fa[2] = {k, (k + 1) % 3};
            double A[6 * 5];
            for (int p = 0; p < 3; ++p)
                for (int i = 0; i < 2; ++i)
                    for (int j = 0; j < NM; ++j) A[(p * 2 + i) * NM + j] = mavg[fa[i]][p][j];
            valid &= pinv(6, NM, A, op + L::XS + k * NM * 6);
        }
        // smoothness matrix over derivative orders 1..N
        smoothness_matrix_packed(N, V0, c0, h0, area0, rBeta, mono, op + L::BP);
        for (size_t q = 0; q < rProj.w.size(); ++q) {
            mono_eval(map_tri(V0, rProj.r[q], rProj.s[q]), c0, h0, tmp);
            for (int i = 1; i < D::NP; ++i)
                for (int j = 0; j < NM; ++j) op[L::PM + (i - 1) * NM + j] += rProj.w[q] * tmp[j] * psiProj[q * D::NP + i];
        }
        op[L::AREA0] = area0;
        op[L::VALID] = valid ? 1.0 : 0.0;
        return valid;
    }
};

template <int N>
int build_ops_t1(const HostMesh& m, std::vector<double>& ops, int64_t& n_rank) {
    using L = OpLayoutT1<N>;
    OpBuilderT1<N> b(m);
    ops.assign((size_t)m.K * L::LEN, 0.0);
    unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    std::vector<int64_t> rank(nt, 0);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            for (int64_t e = t; e < m.K; e += nt)
                if (!b.build(e, &ops[(size_t)e * L::LEN])) ++rank[t];
        });
    for (auto& x : th) x.join();
    n_rank = 0;
    for (unsigned t = 0; t < nt; ++t) n_rank += rank[t];
    return CSWDG_OK;
}

}  // namespace

int build_type1_ops(const HostMesh& m, int N, std::vector<double>& ops, int64_t& n_rank) {
    if (N == 1) return build_ops_t1<1>(m, ops, n_rank);
    if (N == 2) return build_ops_t1<2>(m, ops, n_rank);
    return CSWDG_EINVAL;
}

// The record of the type-II reconstruction (OpLayoutT2, N = 2): the
// centroid-subcell geometry of the hierarchical one, linear least-squares
// fits on the single-neighbour and sector stencils, and at the 9 points of
// the degree-4 rule the linear weights of minimal distance to 1/6 that make
// the six linear fits reproduce the quadratic fit on T3 (exact for
// quadratic data: sum_j g_j = 1, sum_j g_j L_j[phi_k](x) = phi_k(x) for the
// three quadratic scaled monomials).
//
// The record of the mixed reconstruction (OpLayoutMX) shares the piece
// geometry and the linear fits; in place of the point-wise weights it holds
// the quadratic fit on the nine pieces, the smoothness matrix of a quadratic
// and the projection of the scaled monomials.
template <class L>
struct OpBuilderT2 {
    static constexpr bool MIXED = std::is_same<L, OpLayoutMX>::value;
    static constexpr int N = 2, NP = 6, NM = 5;
    const HostMesh& m;
    std::vector<double> C;
    Rule2D rN, rTop, rQ, rBeta;
    std::vector<double> psiQ;  // [q][NP] at the reference points of rQ
    MonoList mono{2};

    explicit OpBuilderT2(const HostMesh& mm) : m(mm) {
        basis_monomial_form(N, C);
        rN = triangle_rule((N + 2) / 2);
        rTop = triangle_rule((N + 2) / 2);
        rQ = triangle_rule(3);  // degree 4: the points where R is evaluated
        rBeta = triangle_rule(2);
        psiQ.resize(rQ.w.size() * NP);
        for (size_t q = 0; q < rQ.w.size(); ++q) basis_eval(N, rQ.r[q], rQ.s[q], &psiQ[q * NP]);
    }

    P2d vert(int64_t e, int k) const { return {m.vx[k * m.K + e], m.vy[k * m.K + e]}; }

    void psi_mono(double r, double s, double* psi) const {
        double pw[NP];
        int k = 0;
        for (int d = 0; d <= N; ++d)
            for (int bb = 0; bb <= d; ++bb) {
                double v = 1.0;
                for (int t = 0; t < d - bb; ++t) v *= r;
                for (int t = 0; t < bb; ++t) v *= s;
                pw[k++] = v;
            }
        for (int n = 0; n < NP; ++n) {
            double acc = 0;
            for (int kk = 0; kk < NP; ++kk) acc += C[n * NP + kk] * pw[kk];
            psi[n] = acc;
        }
    }

    void to_ref(int64_t src, P2d x, double& r, double& s) const {
        P2d v0 = vert(src, 0), v1 = vert(src, 1), v2 = vert(src, 2);
        double xr = 0.5 * (v1.x - v0.x), xs = 0.5 * (v2.x - v0.x);
        double yr = 0.5 * (v1.y - v0.y), ys = 0.5 * (v2.y - v0.y);
        double J = xr * ys - xs * yr;
        double dx = x.x - v0.x, dy = x.y - v0.y;
        r = -1.0 + (ys * dx - xs * dy) / J;
        s = -1.0 + (-yr * dx + xr * dy) / J;
    }

    static P2d map_tri(const P2d* T, double r, double s) {
        return T[0] + (0.5 * (1.0 + r)) * (T[1] - T[0]) + (0.5 * (1.0 + s)) * (T[2] - T[0]);
    }

    void mono_eval(P2d x, P2d c0, double h0, double* out) const {
        double xi = (x.x - c0.x) / h0, eta = (x.y - c0.y) / h0;
        for (int j = 0; j < mono.n; ++j) {
            double v = 1.0;
            for (int t = 0; t < mono.a[j]; ++t) v *= xi;
            for (int t = 0; t < mono.b[j]; ++t) v *= eta;
            out[j] = v;
        }
    }

    // solves the 4 x 4 system A x = b in place (partial pivoting)
    static bool solve4(double A[4][4], double b[4]) {
        for (int k = 0; k < 4; ++k) {
            int piv = k;
            for (int i = k + 1; i < 4; ++i)
                if (std::fabs(A[i][k]) > std::fabs(A[piv][k])) piv = i;
            if (!(std::fabs(A[piv][k]) > 0.0)) return false;
            if (piv != k) {
                for (int j = 0; j < 4; ++j) std::swap(A[k][j], A[piv][j]);
                std::swap(b[k], b[piv]);
            }
            for (int i = k + 1; i < 4; ++i) {
                const double f = A[i][k] / A[k][k];
                for (int j = k; j < 4; ++j) A[i][j] -= f * A[k][j];
                b[i] -= f * b[k];
            }
        }
        for (int k = 3; k >= 0; --k) {
            double t = b[k];
            for (int j = k + 1; j < 4; ++j) t -= A[k][j] * b[j];
            b[k] = t / A[k][k];
        }
        return true;
    }

    bool build(int64_t e, double* op) const {
        for (int i = 0; i < L::LEN; ++i) op[i] = 0.0;
        P2d V0[3] = {vert(e, 0), vert(e, 1), vert(e, 2)};
        P2d c0 = (1.0 / 3.0) * (V0[0] + V0[1] + V0[2]);
        double h0 = (std::sqrt(dot(V0[1] - V0[0], V0[1] - V0[0])) + std::sqrt(dot(V0[2] - V0[1], V0[2] - V0[1])) +
                     std::sqrt(dot(V0[0] - V0[2], V0[0] - V0[2]))) / 3.0;
        double area0 = tri_area(V0[0], V0[1], V0[2]);
        double mavg0[NM] = {0}, tmp[NM];
        {
            double wsum = 0;
            for (size_t q = 0; q < rTop.w.size(); ++q) {
                mono_eval(map_tri(V0, rTop.r[q], rTop.s[q]), c0, h0, tmp);
                for (int j = 0; j < NM; ++j) mavg0[j] += rTop.w[q] * tmp[j];
                wsum += rTop.w[q];
            }
            for (int j = 0; j < NM; ++j) mavg0[j] /= wsum;
        }
        double mavg[3][3][NM];  // [face][piece][monomial], minus the mean over e
        for (int f = 0; f < 3; ++f) {
            uint8_t inf = m.info[3 * e + f];
            bool mirror = false;
            P2d shift{0.0, 0.0}, P{0, 0}, Q{0, 0}, W[3];
            int fp;
            int64_t src;
            if (inf & 0x40) {
                mirror = true;
                P = V0[f];
                Q = V0[(f + 1) % 3];
                P2d d = Q - P;
                P2d X = V0[(f + 2) % 3];
                P2d F = P + (dot(X - P, d) / dot(d, d)) * d;
                W[0] = Q;
                W[1] = P;
                W[2] = 2.0 * F - X;
                fp = 0;
                src = e;
            } else {
                int cx = (inf >> 2) & 3, cy = (inf >> 4) & 3;
                shift = {cx == 1 ? m.px : (cx == 2 ? -m.px : 0.0), cy == 1 ? m.py : (cy == 2 ? -m.py : 0.0)};
                src = m.nbr[3 * e + f];
                for (int k = 0; k < 3; ++k) W[k] = vert(src, k) + shift;
                fp = inf & 3;
            }
            auto back = [&](P2d x) {
                if (!mirror) return x - shift;
                P2d d = Q - P;
                P2d F = P + (dot(x - P, d) / dot(d, d)) * d;
                return 2.0 * F - x;
            };
            P2d G = (1.0 / 3.0) * (W[0] + W[1] + W[2]);
            P2d wa = W[fp], wb = W[(fp + 1) % 3], wc = W[(fp + 2) % 3];
            P2d pcs[3][3] = {{G, wa, wb}, {G, wb, wc}, {G, wc, wa}};
            for (int p = 0; p < 3; ++p) {
                double acc[NP] = {0}, psi[NP], wsum = 0;
                for (size_t q = 0; q < rN.w.size(); ++q) {
                    double r, s;
                    to_ref(src, back(map_tri(pcs[p], rN.r[q], rN.s[q])), r, s);
                    psi_mono(r, s, psi);
                    for (int n = 0; n < NP; ++n) acc[n] += rN.w[q] * psi[n];
                    wsum += rN.w[q];
                }
                for (int n = 0; n < NP; ++n) op[L::AVG + (f * 3 + p) * NP + n] = acc[n] / wsum;
                double ma[NM] = {0};
                wsum = 0;
                for (size_t q = 0; q < rTop.w.size(); ++q) {
                    mono_eval(map_tri(pcs[p], rTop.r[q], rTop.s[q]), c0, h0, tmp);
                    for (int j = 0; j < NM; ++j) ma[j] += rTop.w[q] * tmp[j];
                    wsum += rTop.w[q];
                }
                for (int j = 0; j < NM; ++j) mavg[f][p][j] = ma[j] / wsum - mavg0[j];
            }
        }
        bool valid = true;
        // the six linear fits: pseudo-inverses, and the fits of the three
        // quadratic monomials' averages, Lq[j][k][c]
        double Lq[6][3][2];
        for (int j = 0; j < 6; ++j) {
            const bool sector = j >= 3;
            const int fa = sector ? j - 3 : j, fb = (fa + 1) % 3;
            const int nr = sector ? 6 : 3;
            double A[6 * 2], X[2 * 6];
            for (int p = 0; p < 3; ++p)
                for (int i = 0; i < (sector ? 2 : 1); ++i) {
                    const int row = sector ? p * 2 + i : p, f = i == 0 ? fa : fb;
                    for (int c = 0; c < 2; ++c) A[row * 2 + c] = mavg[f][p][c];
                }
            valid &= pinv(nr, 2, A, X);
            double* dst = sector ? op + L::XS + (j - 3) * 12 : op + L::XF + j * 6;
            for (int i = 0; i < 2 * nr; ++i) dst[i] = X[i];
            for (int k = 0; k < 3; ++k)
                for (int c = 0; c < 2; ++c) {
                    double t = 0.0;
                    for (int p = 0; p < 3; ++p)
                        for (int i = 0; i < (sector ? 2 : 1); ++i) {
                            const int row = sector ? p * 2 + i : p, f = i == 0 ? fa : fb;
                            t += X[c * nr + row] * mavg[f][p][2 + k];
                        }
                    Lq[j][k][c] = t;
                }
        }
        if constexpr (MIXED) {
            double A[9 * NM];
            for (int p = 0; p < 3; ++p)
                for (int f = 0; f < 3; ++f)
                    for (int j = 0; j < NM; ++j) A[(p * 3 + f) * NM + j] = mavg[f][p][j];
            valid &= pinv(9, NM, A, op + L::X3);
            smoothness_matrix_packed(2, V0, c0, h0, area0, rBeta, mono, op + L::BP);
            for (size_t q = 0; q < rQ.w.size(); ++q) {
                mono_eval(map_tri(V0, rQ.r[q], rQ.s[q]), c0, h0, tmp);
                for (int i = 1; i < NP; ++i)
                    for (int j = 0; j < NM; ++j) op[L::PM + (i - 1) * NM + j] += rQ.w[q] * tmp[j] * psiQ[q * NP + i];
            }
        } else {
            point_weights(V0, c0, h0, mavg0, Lq, op, valid);
        }
        op[L::BSC] = area0 / (h0 * h0);
        op[L::VALID] = valid ? 1.0 : 0.0;
        return valid;
    }

    // the points of the degree-4 rule: linear weights, linear monomials,
    // projection weights (type-II record)
    void point_weights(const P2d V0[3], P2d c0, double h0, const double mavg0[NM], const double Lq[6][3][2],
                       double* op, bool& valid) const {
        for (size_t q = 0; q < rQ.w.size(); ++q) {
            double ph[NM];
            mono_eval(map_tri(V0, rQ.r[q], rQ.s[q]), c0, h0, ph);
            for (int j = 0; j < NM; ++j) ph[j] -= mavg0[j];
            op[L::PHI + q * 2 + 0] = ph[0];
            op[L::PHI + q * 2 + 1] = ph[1];
            double Am[4][6], b[4] = {1.0, ph[2], ph[3], ph[4]};
            for (int j = 0; j < 6; ++j) {
                Am[0][j] = 1.0;
                for (int k = 0; k < 3; ++k) Am[1 + k][j] = ph[0] * Lq[j][k][0] + ph[1] * Lq[j][k][1];
            }
            // g = 1/6 + A^T (A A^T)^{-1} (b - A g0)
            double r4[4], AAt[4][4];
            for (int i = 0; i < 4; ++i) {
                double t = b[i];
                for (int j = 0; j < 6; ++j) t -= Am[i][j] / 6.0;
                r4[i] = t;
                for (int k = 0; k < 4; ++k) {
                    double a = 0.0;
                    for (int j = 0; j < 6; ++j) a += Am[i][j] * Am[k][j];
                    AAt[i][k] = a;
                }
            }
            valid &= solve4(AAt, r4);
            for (int j = 0; j < 6; ++j) {
                double g = 1.0 / 6.0;
                for (int i = 0; i < 4; ++i) g += Am[i][j] * r4[i];
                op[L::GAM + q * 6 + j] = g;
            }
            for (int i = 1; i < NP; ++i) op[L::PMQ + (i - 1) * L::NQ + q] = rQ.w[q] * psiQ[q * NP + i];
        }
    }
};

template <class L>
int build_small_stencil_ops(const HostMesh& m, std::vector<double>& ops, int64_t& n_rank) {
    OpBuilderT2<L> b(m);
    ops.assign((size_t)m.K * L::LEN, 0.0);
    unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    std::vector<int64_t> rank(nt, 0);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            for (int64_t e = t; e < m.K; e += nt)
                if (!b.build(e, &ops[(size_t)e * L::LEN])) ++rank[t];
        });
    for (auto& x : th) x.join();
    n_rank = 0;
    for (unsigned t = 0; t < nt; ++t) n_rank += rank[t];
    return CSWDG_OK;
}

int build_type2_ops(const HostMesh& m, std::vector<double>& ops, int64_t& n_rank) {
    return build_small_stencil_ops<OpLayoutT2>(m, ops, n_rank);
}

int build_mixed_ops(const HostMesh& m, std::vector<double>& ops, int64_t& n_rank) {
    return build_small_stencil_ops<OpLayoutMX>(m, ops, n_rank);
}

// TVB minmod indicator (Cockburn and Shu's limiter for triangles): for each
// element (centroid b0) and face midpoint m_i, coefficients A[3 i + f] with
// m_i - b0 = sum_f A[3 i + f] (b_f - b0), b_f the centroid of the neighbour
// across face f (translated by its periodic shift; across a boundary face
// the mirror image of b0 in the face line).  The neighbour pairs are tried
// in the order (i, i+1), (i, i+2), (i+1, i+2); the first whose two
// coefficients are >= 0 is used, else the one whose smaller coefficient is
// largest (counted in n_neg).
void build_tvb_ops(const HostMesh& m, std::vector<double>& A, int64_t& n_neg) {
    const int64_t K = m.K;
    A.assign((size_t)9 * K, 0.0);
    n_neg = 0;
    for (int64_t e = 0; e < K; ++e) {
        P2d V[3];
        for (int k = 0; k < 3; ++k) V[k] = {m.vx[k * K + e], m.vy[k * K + e]};
        const P2d b0 = (1.0 / 3.0) * (V[0] + V[1] + V[2]);
        P2d d[3];
        for (int f = 0; f < 3; ++f) {
            const uint8_t inf = m.info[3 * e + f];
            P2d bf;
            if (inf & 0x40) {
                const P2d P = V[f], dd = V[(f + 1) % 3] - V[f];
                const double t = dot(b0 - P, dd) / dot(dd, dd);
                bf = 2.0 * (P + t * dd) - b0;
            } else {
                const int cx = (inf >> 2) & 3, cy = (inf >> 4) & 3;
                const P2d sh = {cx == 1 ? m.px : (cx == 2 ? -m.px : 0.0), cy == 1 ? m.py : (cy == 2 ? -m.py : 0.0)};
                const int64_t nb = m.nbr[3 * e + f];
                P2d W[3];
                for (int k = 0; k < 3; ++k) W[k] = {m.vx[k * K + nb], m.vy[k * K + nb]};
                bf = (1.0 / 3.0) * (W[0] + W[1] + W[2]) + sh;
            }
            d[f] = bf - b0;
        }
        for (int i = 0; i < 3; ++i) {
            const P2d mi = 0.5 * (V[i] + V[(i + 1) % 3]) - b0;
            const int pj[3] = {i, i, (i + 1) % 3}, pk[3] = {(i + 1) % 3, (i + 2) % 3, (i + 2) % 3};
            int best = -1;
            double blow = -INFINITY, ba = 0.0, bb = 0.0;
            bool found = false;
            for (int p = 0; p < 3 && !found; ++p) {
                const P2d bj = d[pj[p]], bk = d[pk[p]];
                const double det = bj.x * bk.y - bj.y * bk.x;
                if (det == 0.0) continue;
                const double al = (mi.x * bk.y - mi.y * bk.x) / det;
                const double be = (bj.x * mi.y - bj.y * mi.x) / det;
                const double lo = std::min(al, be);
                if (lo >= 0.0) found = true;
                if (found || lo > blow) {
                    blow = lo;
                    best = p;
                    ba = al;
                    bb = be;
                }
            }
            if (!found) ++n_neg;
            if (best < 0) continue;
            A[(size_t)(3 * i + pj[best]) * K + e] = ba;
            A[(size_t)(3 * i + pk[best]) * K + e] = bb;
        }
    }
}

int build_limiter_ops(const HostMesh& m, int N, int qtop, bool constant_gamma, bool ghost_extrapolate, std::vector<double>& ops,
                      int64_t& n_rank, int64_t& n_foot) {
    auto by_top = [&](auto nc) {
        constexpr int NN = decltype(nc)::value;
        switch (qtop) {
            case kTopQuadratic: return build_ops_n<NN, kTopQuadratic>(m, constant_gamma, ghost_extrapolate, ops, n_rank, n_foot);
            case kTopCubic: return build_ops_n<NN, kTopCubic>(m, constant_gamma, ghost_extrapolate, ops, n_rank, n_foot);
            case kTopCubicTel: return build_ops_n<NN, kTopCubicTel>(m, constant_gamma, ghost_extrapolate, ops, n_rank, n_foot);
            case kTopSextic:
                if constexpr (NN == 3)
                    return build_ops_n<NN, kTopSextic>(m, constant_gamma, ghost_extrapolate, ops, n_rank, n_foot);
                return CSWDG_EINVAL;
            default: return build_ops_n<NN, kTopQuartic>(m, constant_gamma, ghost_extrapolate, ops, n_rank, n_foot);
        }
    };
    if (N == 1) return build_ops_n<1, kTopQuadratic>(m, constant_gamma, ghost_extrapolate, ops, n_rank, n_foot);
    if (N == 2) return by_top(std::integral_constant<int, 2>{});
    if (N == 3) return by_top(std::integral_constant<int, 3>{});
    return CSWDG_EINVAL;
}

}  // namespace cswdg
