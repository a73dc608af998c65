// Adjoint (vector-Jacobian products) of the RKDG stage and of the CSWENO
// limiter with the troubled-cell mask frozen.  Not part of the paper; it
// differentiates exactly the forward operators of kernels.hip:
//
//   k_residual_vjp   prev_bar = [prev_bar] + c_id ybar + L'(u)^T (c_dt dt ybar),
//                    un_bar += a ybar; with (a, c_id, c_dt) = (a, b, b) this is
//                    the stage out = a u_n + b (u + dt L(u)), with (0, 0, 1)
//                    and no dt the plain L'(u)^T.  Gather form: element e collects the
//                    edge-flux adjoints of its own faces and of the faces
//                    its neighbours share with it, so no atomics are used
//                    and the result is deterministic.
//   k_limiter_vjp    per troubled cell (one lane per characteristic
//                    direction and field, as in the forward): recompute the
//                    forward quantities, then run them backwards through
//                    the projection, the weights (omega, tau, beta, sigma),
//                    the least-squares pseudo-inverses, the piece averages
//                    and the characteristic matrices (their derivatives with
//                    respect to the cell mean by forward-mode dual numbers);
//                    the adjoint for the cell itself and for each of its
//                    three sources goes to a compact buffer.
//   k_limiter_gather per element: identity for untroubled cells, the mean
//                    for troubled ones, plus the compact contributions of
//                    the element's own reconstruction and of its troubled
//                    neighbours' reconstructions.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace cswdg {

namespace {

// ubar += (d(F.n)/dU)^T xb, as the gradient of phi(U) = xb . F.n(U): with
// u_n the normal velocity, H the total enthalpy and p the pressure,
// phi = u_n (xb . (rho, m, l, E + p)) + p (xb_1 n_x + xb_2 n_y), so
// grad phi = s (-u_n, n_x, n_y, 0) + u_n xb + w (gamma - 1) (q^2/2, -u, -v, 1)
// with s = xb_0 + xb_1 u + xb_2 v + xb_3 H and w = u_n xb_3 + xb_1 n_x +
// xb_2 n_y (the transposed Jacobian applied without forming it).
template <int EQ>
__device__ __forceinline__ void flux_jacT(const double* U, double nx, double ny, double g, const double* xb,
                                          double* ub) {
    if constexpr (EQ == 0) {
        ub[0] += U[0] * (nx + ny) * xb[0];
    } else {
        const double rho = U[0], m = U[1], l = U[2], E = U[3];
        const double ir = rcp_nr(rho);
        const double u = m * ir, v = l * ir;
        const double q2 = u * u + v * v;
        const double gm = g - 1.0;
        const double p = gm * (E - 0.5 * rho * q2);
        const double H = (E + p) * ir;
        const double un = u * nx + v * ny;
        const double sv = xb[0] + xb[1] * u + xb[2] * v + xb[3] * H;
        const double wg = gm * (un * xb[3] + xb[1] * nx + xb[2] * ny);
        ub[0] += -sv * un + un * xb[0] + wg * (0.5 * q2);
        ub[1] += sv * nx + un * xb[1] - wg * u;
        ub[2] += sv * ny + un * xb[2] - wg * v;
        ub[3] += un * xb[3] + wg;
    }
}

// largest normal wave speed and its gradient (d|x|/dx = 0 at x = 0)
template <int EQ>
__device__ __forceinline__ double speed_grad(const double* U, double nx, double ny, double g, double* dl) {
    if constexpr (EQ == 0) {
        const double s = U[0] * (nx + ny);
        dl[0] = (s > 0.0 ? 1.0 : (s < 0.0 ? -1.0 : 0.0)) * (nx + ny);
        return fabs(s);
    } else {
        const double rho = U[0], m = U[1], l = U[2], E = U[3];
        const double ir = rcp_nr(rho);
        const double u = m * ir, v = l * ir;
        const double q2 = u * u + v * v;
        const double gm = g - 1.0;
        const double p = gm * (E - 0.5 * rho * q2);
        const double c = sqrt_nr(g * p * ir);
        const double un = u * nx + v * ny;
        const double sg = un > 0.0 ? 1.0 : (un < 0.0 ? -1.0 : 0.0);
        const double k = g * rcp_nr(2.0 * c);
        // d(p/rho)
        const double dp0 = gm * (-E * ir * ir + q2 * ir), dp1 = -gm * u * ir, dp2 = -gm * v * ir, dp3 = gm * ir;
        dl[0] = sg * (-un * ir) + k * dp0;
        dl[1] = sg * (nx * ir) + k * dp1;
        dl[2] = sg * (ny * ir) + k * dp2;
        dl[3] = k * dp3;
        return fabs(un) + c;
    }
}

template <int EQ, int N>
__global__ __launch_bounds__(256) void k_residual_vjp(DevMesh msh, const double* __restrict__ u,
                                                      const double* __restrict__ ybar,
                                                      double* __restrict__ prev_bar,
                                                      double* __restrict__ un_bar,
                                                      const double* __restrict__ dtp, double a, double c_id,
                                                      double c_dt, int accumulate, double gamma) {
    using D = Dims<N>;
    constexpr int M = Phys<EQ>::M, NP = D::NP, NE = D::NE, NQ = D::NQ;
    const int K = msh.K;
    const int e = xcd_block(blockIdx.x, gridDim.x, msh.xcd_tiles) * blockDim.x + threadIdx.x;
    const Tab<N>& T = tab<N>();
    // the face-point tables in LDS: the neighbour's side reads them at the
    // neighbour's own face (a per-lane index)
    __shared__ double sPF[3 * NE * NP], sWPF[3 * NE * NP];
    for (int i = threadIdx.x; i < 3 * NE * NP; i += blockDim.x) {
        sPF[i] = (&T.PF[0][0][0])[i];
        sWPF[i] = (&T.wPF[0][0][0])[i];
    }
    __syncthreads();
    if (e >= K) return;
    const double scale = dtp ? c_dt * (*dtp) : c_dt;

    double U[M][NP], Rb[M][NP], Ub[M][NP];
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int n = 0; n < NP; ++n) {
            U[c][n] = u[(size_t)(c * NP + n) * K + e];
            Rb[c][n] = scale * ybar[(size_t)(c * NP + n) * K + e];
            Ub[c][n] = 0.0;
        }
    const double X[3] = {msh.vx[e], msh.vx[K + e], msh.vx[2 * K + e]};
    const double Y[3] = {msh.vy[e], msh.vy[K + e], msh.vy[2 * K + e]};
    const double xr = 0.5 * (X[1] - X[0]), xs = 0.5 * (X[2] - X[0]);
    const double yr = 0.5 * (Y[1] - Y[0]), ys = 0.5 * (Y[2] - Y[0]);
    const double J = xr * ys - xs * yr;
    const double iJ = 1.0 / J;
    const double rx = ys * iJ, ry = -xs * iJ, sx = -yr * iJ, sy = xr * iJ;

    // volume term
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
        double uq[M], Fb[M], Gb[M], ub[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            double s = 0.0, fb = 0.0, gb = 0.0;
#pragma unroll
            for (int n = 0; n < NP; ++n) {
                s += T.V[q][n] * U[c][n];
                fb += Rb[c][n] * (T.wDr[q][n] * rx + T.wDs[q][n] * sx);
                gb += Rb[c][n] * (T.wDr[q][n] * ry + T.wDs[q][n] * sy);
            }
            uq[c] = s;
            Fb[c] = fb;
            Gb[c] = gb;
            ub[c] = 0.0;
        }
        flux_jacT<EQ>(uq, 1.0, 0.0, gamma, Fb, ub);
        flux_jacT<EQ>(uq, 0.0, 1.0, gamma, Gb, ub);
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int n = 0; n < NP; ++n) Ub[c][n] += T.V[q][n] * ub[c];
    }

    // surface terms of the element's own faces and of its neighbours' faces
    const uint32_t info4 = msh.info[e];
#pragma unroll 1
    for (int f = 0; f < 3; ++f) {
        const int f1 = (f == 2) ? 0 : f + 1;
        const double ex = msh.vx[f1 * K + e] - msh.vx[f * K + e], ey = msh.vy[f1 * K + e] - msh.vy[f * K + e];
        const double L = sqrt(ex * ex + ey * ey);
        const double iL = 1.0 / L;
        const double nx = ey * iL, ny = -ex * iL;
        const double sf = 0.5 * L * iJ;
        const uint32_t inf = (info4 >> (8 * f)) & 0xffu;
        const bool bnd = (inf & 0x40u) != 0u;
        const int fp = (int)(inf & 3u);
        const int nb = bnd ? e : msh.nbr[f * K + e];
        double Un[M][NP], Rbn[M][NP];
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int n = 0; n < NP; ++n) {
                Un[c][n] = u[(size_t)(c * NP + n) * K + nb];
                Rbn[c][n] = scale * ybar[(size_t)(c * NP + n) * K + nb];
            }
        double sfn;
        {
            const double a0 = msh.vx[nb], a1 = msh.vx[K + nb], a2 = msh.vx[2 * K + nb];
            const double b0 = msh.vy[nb], b1 = msh.vy[K + nb], b2 = msh.vy[2 * K + nb];
            const double Jn = 0.25 * ((a1 - a0) * (b2 - b0) - (a2 - a0) * (b1 - b0));
            sfn = 0.5 * L / Jn;
        }
#pragma unroll
        for (int g = 0; g < NE; ++g) {
            double um[M], up[M], Fbo[M], Fbn[M], ub[M];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                double s = 0.0, t = 0.0, fo = 0.0, fn = 0.0;
#pragma unroll
                for (int n = 0; n < NP; ++n) {
                    s += T.PF[f][g][n] * U[c][n];
                    t += sPF[(fp * NE + NE - 1 - g) * NP + n] * Un[c][n];
                    fo += Rb[c][n] * T.wPF[f][g][n];
                    fn += Rbn[c][n] * sWPF[(fp * NE + NE - 1 - g) * NP + n];
                }
                um[c] = s;
                up[c] = t;
                Fbo[c] = -sf * fo;
                Fbn[c] = -sfn * fn;
                ub[c] = 0.0;
            }
            if (bnd) {
                // F* = F(u-).n on a transmissive face
                flux_jacT<EQ>(um, nx, ny, gamma, Fbo, ub);
            } else {
                double dlm[M], dlp[M];
                const double lm = speed_grad<EQ>(um, nx, ny, gamma, dlm);
                const double lp = speed_grad<EQ>(up, nx, ny, gamma, dlp);
                const double alpha = fmax(lm, lp);
                double diff[M];
                double dFo = 0.0, dFn = 0.0;
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    diff[c] = up[c] - um[c];
                    dFo += Fbo[c] * diff[c];
                    dFn -= Fbn[c] * diff[c];  // Fbn . (um - up)
                }
                double xb[M];
#pragma unroll
                for (int c = 0; c < M; ++c) xb[c] = 0.5 * (Fbo[c] - Fbn[c]);
                flux_jacT<EQ>(um, nx, ny, gamma, xb, ub);
                const double own_branch = (lm >= lp) ? 1.0 : 0.0;  // ties: first argument
                const double nbr_branch = (lm > lp) ? 1.0 : 0.0;   // neighbour's first argument is up
#pragma unroll
                for (int c = 0; c < M; ++c)
                    ub[c] += 0.5 * alpha * (Fbo[c] - Fbn[c]) - 0.5 * (dFo * own_branch + dFn * nbr_branch) * dlm[c];
            }
#pragma unroll
            for (int c = 0; c < M; ++c)
#pragma unroll
                for (int n = 0; n < NP; ++n) Ub[c][n] += T.PF[f][g][n] * ub[c];
        }
    }

#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int n = 0; n < NP; ++n) {
            const size_t idx = (size_t)(c * NP + n) * K + e;
            const double yb = ybar[idx];
            double v = c_id * yb + Ub[c][n];
            if (accumulate) v += prev_bar[idx];
            prev_bar[idx] = v;
            if (un_bar != nullptr && a != 0.0) un_bar[idx] += a * yb;
        }
}

// mask -> troubled list and the inverse map element -> list position
__global__ __launch_bounds__(256) void k_compact_slots(int K, const uint8_t* __restrict__ mask,
                                                       int32_t* __restrict__ list,
                                                       int32_t* __restrict__ slot,
                                                       uint32_t* __restrict__ count) {
    // segment 0 only (the slots are global list positions); one atomic per block
    __shared__ uint32_t wbase[4];
    __shared__ uint32_t bbase;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const bool tr = (e < K) && mask[e] != 0;
    const unsigned long long bal = __ballot(tr ? 1 : 0);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wbase[w] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0u;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            const uint32_t c = wbase[i];
            wbase[i] = acc;
            acc += c;
        }
        bbase = acc ? atomicAdd(count, acc) : 0u;
    }
    __syncthreads();
    if (e < K) {
        const uint32_t pos = bbase + wbase[w] + (uint32_t)before;
        if (tr && pos < (uint32_t)K) list[pos] = e;
        slot[e] = tr ? (int32_t)pos : -1;
    }
}

template <int EQ, int N, int QTOP>
__global__ __launch_bounds__(64) void k_limiter_vjp(DevMesh msh, const double* __restrict__ u,
                                                    const double* __restrict__ ops,
                                                    const int32_t* __restrict__ list,
                                                    const uint32_t* __restrict__ count,
                                                    const double* __restrict__ ybar,
                                                    double* __restrict__ contrib, double gamma,
                                                    double eps) {
    using D = Dims<N>;
    using LO = OpLayout<N, QTOP>;
    constexpr int M = Phys<EQ>::M, NP = D::NP, NPC = LO::NPC, NM = LO::NM;
    constexpr bool FOUR = LO::FOUR;  // a fourth member on T4
    constexpr int NT = LO::NT > 0 ? LO::NT : 1;
    constexpr int ND = LimLanes<EQ>::ND, LPC = LimLanes<EQ>::LPC;
    constexpr int CPB = 64 / LPC;
    const int K = msh.K;
    uint32_t pre[kListSegs + 1];
    seg_prefix(count, K, pre);
    const uint32_t ncell = pre[kListSegs];
    const int j = threadIdx.x % LPC;
    const int d = j / M;
    const int k = j % M;
    for (uint32_t base = blockIdx.x * CPB; base < ncell; base += gridDim.x * CPB) {
        const uint32_t t = base + threadIdx.x / LPC;
        const bool active = t < ncell;
        const int e = active ? seg_elem(list, pre, K, t) : 0;
        const double* __restrict__ op = ops + (size_t)e * LO::LEN;
        const bool valid = active && op[LO::VALID] != 0.0;

        double ub0[M];
#pragma unroll
        for (int c = 0; c < M; ++c) ub0[c] = u[(size_t)(c * NP) * K + e] * kPsi0;
        // row k of L_d and column k of R_d (their derivatives in ub0 are
        // formed at the end, where they are used)
        double Lr[M], Rc[M];
        if constexpr (EQ == 1) {
            const double nx = d == 0 ? 1.0 : 0.0, ny = d == 0 ? 0.0 : 1.0;
            double Lm[4][4], Rm[4][4];
            euler_eigen<double>(ub0, nx, ny, gamma, Lm, Rm);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double a = Lm[0][c], bb = Rm[c][0];
#pragma unroll
                for (int kk = 1; kk < 4; ++kk) {
                    a = (k == kk) ? Lm[kk][c] : a;
                    bb = (k == kk) ? Rm[c][kk] : bb;
                }
                Lr[c] = a;
                Rc[c] = bb;
            }
        } else {
            Lr[0] = 1.0;
            Rc[0] = 1.0;
        }
        double w0 = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) w0 += Lr[c] * ub0[c];

        // ---- forward recomputation ----
        const uint32_t info4 = msh.info[e];
        int srcs[3];
        double w[3][NPC];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const uint32_t inf = (info4 >> (8 * f)) & 0xffu;
            srcs[f] = (inf & 0x40u) ? e : msh.nbr[f * K + e];
            double ws[NP];
#pragma unroll
            for (int n = 0; n < NP; ++n) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < M; ++c) s += Lr[c] * u[(size_t)(c * NP + n) * K + srcs[f]];
                ws[n] = s;
            }
#pragma unroll
            for (int p = 0; p < NPC; ++p) {
                const double* av = op + LO::AVG + (f * NPC + p) * NP;
                double s = 0.0;
#pragma unroll
                for (int n = 0; n < NP; ++n) s += av[n] * ws[n];
                w[f][p] = s;
            }
        }
        constexpr int pl[5] = {0, 3, 4, 5, 6};
        double c2[2], c3[5], c5[NT];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            double s = 0.0;
#pragma unroll
            for (int f = 0; f < 3; ++f) s += op[LO::X2 + jj * 3 + f] * (w[f][0] - w0);
            c2[jj] = s;
        }
#pragma unroll
        for (int jj = 0; jj < 5; ++jj) {
            double s = 0.0;
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int f = 0; f < 3; ++f) s += op[LO::X3 + jj * 9 + p * 3 + f] * (w[f][p] - w0);
            c3[jj] = s;
        }
#pragma unroll
        for (int jj = 0; jj < NT; ++jj) c5[jj] = 0.0;
        if constexpr (FOUR) {
#pragma unroll 1
            for (int jj = 0; jj < NT; ++jj) {
                double s = 0.0;
#pragma unroll
                for (int kk = 0; kk < 5; ++kk)
#pragma unroll
                    for (int f = 0; f < 3; ++f) s += op[LO::X5 + jj * 15 + kk * 3 + f] * (w[f][pl[kk]] - w0);
                c5[jj] = s;
            }
        }
        const double* bp = op + LO::BP;
        double beta[4];
        beta[1] = quad_form<NM, 2>(bp, c2);
        beta[2] = quad_form<NM, 5>(bp, c3);
        beta[3] = FOUR ? quad_form<NM, NT>(bp, c5) : 0.0;
        const double area0 = op[LO::AREA0];
        double gx[3], gy[3], b1[3], sg[3], ssum, mx, my, num, mm;
        {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const double* mi = op + LO::MINV + 4 * f;
                const double d0 = w[f][1] - w[f][0], d1 = w[f][2] - w[f][0];
                gx[f] = mi[0] * d0 + mi[1] * d1;
                gy[f] = mi[2] * d0 + mi[3] * d1;
                b1[f] = area0 * (gx[f] * gx[f] + gy[f] * gy[f]);
            }
            const double a01 = b1[0] - b1[1], a12 = b1[1] - b1[2], a20 = b1[2] - b1[0];
            mm = (a01 * a01 + a12 * a12 + a20 * a20) / 3.0;
            num = mm * mm;
            ssum = 0.0;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                sg[f] = (1.0 / 3.0) * (1.0 + num / (b1[f] + eps));
                ssum += sg[f];
            }
            mx = 0.0;
            my = 0.0;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                mx += (sg[f] / ssum) * gx[f];
                my += (sg[f] / ssum) * gy[f];
            }
            beta[0] = area0 * (mx * mx + my * my);
        }
        const double ih = op[LO::GBASE];
        const double s2 = 1.0 + ih, s3 = 1.0 + ih + ih * ih, s5 = 1.0 + ih + ih * ih + ih * ih * ih;
        const double g22 = ih / s2, g23 = ih / s3, g33 = ih * ih / s3;
        const double g15 = 1.0 / s5, g25 = ih / s5, g35 = ih * ih / s5, g45 = ih * ih * ih / s5;
        const double g13 = 1.0 / s3;
        constexpr int NL = FOUR ? 4 : 3;
        double gl[4], om[4], ob[4], tau, os;
        if constexpr (!FOUR) {
            gl[0] = g13;
            gl[1] = g23;
            gl[2] = g33;
            gl[3] = 0.0;
            const double d31 = beta[2] - beta[0], d32 = beta[2] - beta[1];
            tau = (d31 * d31 + d32 * d32) / 4.0;
        } else {
            gl[0] = g15;
            gl[1] = g25;
            gl[2] = g35;
            gl[3] = g45;
            const double d1 = beta[3] - beta[0], d2 = beta[3] - beta[1], d3 = beta[3] - beta[2];
            tau = (d1 * d1 + d2 * d2 + d3 * d3) / 16.0;
        }
        os = 0.0;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            ob[l] = gl[l] * (1.0 + tau / (eps + beta[l]));
            os += ob[l];
        }
#pragma unroll
        for (int l = 0; l < NL; ++l) om[l] = ob[l] / os;
        double A2, A3, A5;
        if constexpr (!FOUR) {
            A3 = om[2] / g33;
            A2 = om[1] / g22 - A3 * g23 / g22;
            A5 = 0.0;
        } else if constexpr (QTOP == kTopCubic) {
            // eq. equivalentOrder3: p4 = (c4 - g24 p2)/g34, gamma_{.,4} = gamma_{.,3}
            A5 = om[3] / g33;
            A3 = om[2] / g33;
            A2 = (om[1] - (om[2] + om[3]) * (g23 / g33)) / g22;
        } else {
            A5 = om[3] / g45;
            A3 = (om[2] - A5 * g35) / g33;
            A2 = (om[1] - A5 * g25 - A3 * g23) / g22;
        }
        double Rcoef[NM];
#pragma unroll
        for (int jj = 0; jj < NM; ++jj) {
            double r = 0.0;
            if constexpr (FOUR) r = A5 * c5[jj];
            if (jj < 5) r += A3 * c3[jj];
            if (jj < 2) r += A2 * c2[jj];
            Rcoef[jj] = r;
        }
        double mom[NP - 1];
#pragma unroll
        for (int i = 0; i < NP - 1; ++i) {
            double s = 0.0;
#pragma unroll
            for (int jj = 0; jj < NM; ++jj) s += op[LO::PM + i * NM + jj] * Rcoef[jj];
            mom[i] = s;
        }

        // ---- reverse ----
        double yb[M][NP - 1];
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int i = 0; i < NP - 1; ++i) yb[c][i] = ybar[(size_t)(c * NP + i + 1) * K + e];
        double momb[NP - 1], Rcb[M];
#pragma unroll
        for (int i = 0; i < NP - 1; ++i) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) s += Rc[c] * yb[c][i];
            momb[i] = s / ND;
        }
#pragma unroll
        for (int c = 0; c < M; ++c) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < NP - 1; ++i) s += yb[c][i] * mom[i];
            Rcb[c] = s / ND;
        }
        double Rcoefb[NM];
#pragma unroll 1
        for (int jj = 0; jj < NM; ++jj) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < NP - 1; ++i) s += op[LO::PM + i * NM + jj] * momb[i];
            Rcoefb[jj] = s;
        }
        double c2b[2], c3b[5], c5b[NT];
        double A2b = 0.0, A3b = 0.0, A5b = 0.0;
#pragma unroll
        for (int jj = 0; jj < NT; ++jj) c5b[jj] = 0.0;
        if constexpr (FOUR) {
#pragma unroll
            for (int jj = 0; jj < NT; ++jj) {
                c5b[jj] = A5 * Rcoefb[jj];
                A5b += c5[jj] * Rcoefb[jj];
            }
        }
#pragma unroll
        for (int jj = 0; jj < 5; ++jj) {
            c3b[jj] = A3 * Rcoefb[jj];
            A3b += c3[jj] * Rcoefb[jj];
        }
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            c2b[jj] = A2 * Rcoefb[jj];
            A2b += c2[jj] * Rcoefb[jj];
        }
        double omb[4] = {0.0, 0.0, 0.0, 0.0};
        if constexpr (!FOUR) {
            omb[1] = A2b / g22;
            A3b -= A2b * g23 / g22;
            omb[2] = A3b / g33;
        } else if constexpr (QTOP == kTopCubic) {
            omb[1] = A2b / g22;
            const double tb = A2b * (g23 / g33) / g22;
            omb[2] = A3b / g33 - tb;
            omb[3] = A5b / g33 - tb;
        } else {
            omb[1] = A2b / g22;
            A5b -= A2b * g25 / g22;
            A3b -= A2b * g23 / g22;
            omb[2] = A3b / g33;
            A5b -= A3b * g35 / g33;
            omb[3] = A5b / g45;
        }
        double sdot = 0.0;
#pragma unroll
        for (int l = 0; l < NL; ++l) sdot += omb[l] * om[l];
        double taub = 0.0, betab[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const double obar = (omb[l] - sdot) / os;
            const double ie = 1.0 / (eps + beta[l]);
            taub += obar * gl[l] * ie;
            betab[l] -= obar * gl[l] * tau * ie * ie;
        }
        if constexpr (!FOUR) {
            betab[2] += taub * 0.5 * ((beta[2] - beta[0]) + (beta[2] - beta[1]));
            betab[0] -= taub * 0.5 * (beta[2] - beta[0]);
            betab[1] -= taub * 0.5 * (beta[2] - beta[1]);
        } else {
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const double dd = taub * (2.0 / 16.0) * (beta[3] - beta[l]);
                betab[3] += dd;
                betab[l] -= dd;
            }
        }
        // beta of q_l: c^T B c over the leading blocks -> 2 beta_bar B c
#pragma unroll 1
        for (int i = 0; i < NM; ++i) {
            double s5 = 0.0, s3v = 0.0, s2v = 0.0;
#pragma unroll
            for (int jj = 0; jj < NM; ++jj) {
                const int r0 = i < jj ? i : jj, r1 = i < jj ? jj : i;
                const double Bij = bp[r0 * NM - (r0 * (r0 - 1)) / 2 + (r1 - r0)];
                if constexpr (FOUR) s5 += Bij * c5[jj];
                if (i < 5 && jj < 5) s3v += Bij * c3[jj];
                if (i < 2 && jj < 2) s2v += Bij * c2[jj];
            }
            if constexpr (FOUR) c5b[i] += 2.0 * betab[3] * s5;
            if (i < 5) c3b[i] += 2.0 * betab[2] * s3v;
            if (i < 2) c2b[i] += 2.0 * betab[1] * s2v;
        }
        // beta_1 chain
        double wb[3][NPC];
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int p = 0; p < NPC; ++p) wb[f][p] = 0.0;
        {
            const double mxb = 2.0 * area0 * betab[0] * mx, myb = 2.0 * area0 * betab[0] * my;
            double gxb[3], gyb[3], sb[3], sdt = 0.0;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const double sf = sg[f] / ssum;
                gxb[f] = sf * mxb;
                gyb[f] = sf * myb;
                sb[f] = mxb * gx[f] + myb * gy[f];
                sdt += sb[f] * sf;
            }
            double numb = 0.0, b1b[3];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const double sgb = (sb[f] - sdt) / ssum;
                const double ie = 1.0 / (b1[f] + eps);
                numb += sgb * (1.0 / 3.0) * ie;
                b1b[f] = -sgb * (1.0 / 3.0) * num * ie * ie;
            }
            const double mmb = 2.0 * mm * numb;
            const double a01 = b1[0] - b1[1], a12 = b1[1] - b1[2], a20 = b1[2] - b1[0];
            b1b[0] += mmb * (2.0 / 3.0) * (a01 - a20);
            b1b[1] += mmb * (2.0 / 3.0) * (a12 - a01);
            b1b[2] += mmb * (2.0 / 3.0) * (a20 - a12);
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                gxb[f] += 2.0 * area0 * b1b[f] * gx[f];
                gyb[f] += 2.0 * area0 * b1b[f] * gy[f];
                const double* mi = op + LO::MINV + 4 * f;
                const double d0b = mi[0] * gxb[f] + mi[2] * gyb[f];
                const double d1b = mi[1] * gxb[f] + mi[3] * gyb[f];
                wb[f][1] += d0b;
                wb[f][2] += d1b;
                wb[f][0] -= d0b + d1b;
            }
        }
        // least-squares right-hand sides b = w - w0
        double w0b = 0.0;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            double s = 0.0;
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) s += op[LO::X2 + jj * 3 + f] * c2b[jj];
            wb[f][0] += s;
            w0b -= s;
        }
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                double s = 0.0;
#pragma unroll
                for (int jj = 0; jj < 5; ++jj) s += op[LO::X3 + jj * 9 + p * 3 + f] * c3b[jj];
                wb[f][p] += s;
                w0b -= s;
            }
        if constexpr (FOUR) {
#pragma unroll 1
            for (int kk = 0; kk < 5; ++kk)
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    double s = 0.0;
#pragma unroll
                    for (int jj = 0; jj < NT; ++jj) s += op[LO::X5 + jj * 15 + kk * 3 + f] * c5b[jj];
                    wb[f][pl[kk]] += s;
                    w0b -= s;
                }
        }
        // piece averages and field projection, one face at a time: the
        // cell's contribution to face f's source coefficients is the sum over
        // the cell's lanes of Lr[c] wsb[n]; the lanes' sums are formed face by
        // face so that only one face's block is live
        double Lrb[M], ub0b[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            Lrb[c] = ub0[c] * w0b;
            ub0b[c] = Lr[c] * w0b;
        }
        double* rec = contrib + (size_t)t * (4 * M * NP);
#pragma unroll 1
        for (int f = 0; f < 3; ++f) {
            // this face's row of wb and its source, by selects (a register
            // array indexed by the loop counter would live in scratch)
            double wbf[NPC];
#pragma unroll
            for (int p = 0; p < NPC; ++p) wbf[p] = (f == 0) ? wb[0][p] : ((f == 1) ? wb[1][p] : wb[2][p]);
            const int srcf = (f == 0) ? srcs[0] : ((f == 1) ? srcs[1] : srcs[2]);
            double wsb[NP];
#pragma unroll
            for (int n = 0; n < NP; ++n) {
                double s = 0.0;
#pragma unroll
                for (int p = 0; p < NPC; ++p) s += op[LO::AVG + (f * NPC + p) * NP + n] * wbf[p];
                wsb[n] = s;
            }
            double Usb[M][NP];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                double s = 0.0;
#pragma unroll
                for (int n = 0; n < NP; ++n) {
                    Usb[c][n] = Lr[c] * wsb[n];
                    s += u[(size_t)(c * NP + n) * K + srcf] * wsb[n];
                }
                Lrb[c] += s;
            }
#pragma unroll
            for (int o = 1; o < LPC; o <<= 1)
#pragma unroll
                for (int c = 0; c < M; ++c)
#pragma unroll
                    for (int n = 0; n < NP; ++n) Usb[c][n] += __shfl_xor(Usb[c][n], o, LPC);
            if (active && j < M) {
                // record [slot 0 = the cell][slots 1..3 = sources of faces 0..2][m][Np]
#pragma unroll
                for (int n = 0; n < NP; ++n) {
                    double v = Usb[0][n];
#pragma unroll
                    for (int c = 1; c < M; ++c) v = (j == c) ? Usb[c][n] : v;
                    rec[(1 + f) * M * NP + j * NP + n] = valid ? v : 0.0;
                }
            }
        }
        // characteristic matrices depend on the cell mean: one forward-mode
        // pass per component of ub0 gives d(row k of L_d)/d ub0[cc] and
        // d(column k of R_d)/d ub0[cc]
        if constexpr (EQ == 1) {
            const double nx = d == 0 ? 1.0 : 0.0, ny = d == 0 ? 0.0 : 1.0;
#pragma unroll 1
            for (int cc = 0; cc < 4; ++cc) {
                Dual U4[4], Ld[4][4], Rd[4][4];
#pragma unroll
                for (int c = 0; c < 4; ++c) U4[c] = Dual(ub0[c], c == cc ? 1.0 : 0.0);
                euler_eigen<Dual>(U4, nx, ny, gamma, Ld, Rd);
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    double a = Ld[0][c].d, bb = Rd[c][0].d;
#pragma unroll
                    for (int kk = 1; kk < 4; ++kk) {
                        a = (k == kk) ? Ld[kk][c].d : a;
                        bb = (k == kk) ? Rd[c][kk].d : bb;
                    }
                    s += Lrb[c] * a + Rcb[c] * bb;
                }
                ub0b[cc] += s;
            }
        }
        double U0b[M];
#pragma unroll
        for (int c = 0; c < M; ++c) U0b[c] = kPsi0 * ub0b[c];
#pragma unroll
        for (int o = 1; o < LPC; o <<= 1)
#pragma unroll
            for (int c = 0; c < M; ++c) U0b[c] += __shfl_xor(U0b[c], o, LPC);
        if (active && j < M) {
            double sel0 = U0b[0];
#pragma unroll
            for (int c = 1; c < M; ++c) sel0 = (j == c) ? U0b[c] : sel0;
            rec[j * NP] = valid ? sel0 : 0.0;
#pragma unroll
            for (int n = 1; n < NP; ++n) rec[j * NP + n] = 0.0;
        }
    }
}

template <int EQ, int N>
__global__ __launch_bounds__(256) void k_limiter_gather(DevMesh msh, const uint8_t* __restrict__ mask,
                                                        const int32_t* __restrict__ slot,
                                                        const double* __restrict__ contrib,
                                                        const double* __restrict__ ybar,
                                                        double* __restrict__ wbar) {
    constexpr int M = Phys<EQ>::M, NP = Dims<N>::NP;
    const int K = msh.K;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K) return;
    const bool tr = mask[e] != 0;
    double acc[M][NP];
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int n = 0; n < NP; ++n) {
            const double y = ybar[(size_t)(c * NP + n) * K + e];
            // untroubled: identity; troubled: only the copied mean passes through
            acc[c][n] = (!tr || n == 0) ? y : 0.0;
        }
    const uint32_t info4 = msh.info[e];
    if (tr) {
        const int t = slot[e];
        const double* rec = contrib + (size_t)t * (4 * M * NP);
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int n = 0; n < NP; ++n) acc[c][n] += rec[c * NP + n];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            if ((info4 >> (8 * f)) & 0x40u) {  // mirror ghost: the source is the cell itself
#pragma unroll
                for (int c = 0; c < M; ++c)
#pragma unroll
                    for (int n = 0; n < NP; ++n) acc[c][n] += rec[(1 + f) * M * NP + c * NP + n];
            }
        }
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const uint32_t inf = (info4 >> (8 * f)) & 0xffu;
        if (inf & 0x40u) continue;
        const int nb = msh.nbr[f * K + e];
        if (!mask[nb]) continue;
        const int t = slot[nb];
        const int fn = (int)(inf & 3u);  // the neighbour's face shared with e
        const double* rec = contrib + (size_t)t * (4 * M * NP) + (1 + fn) * M * NP;
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int n = 0; n < NP; ++n) acc[c][n] += rec[c * NP + n];
    }
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int n = 0; n < NP; ++n) wbar[(size_t)(c * NP + n) * K + e] = acc[c][n];
}

}  // namespace

int upload_tables_adjoint() { return upload_tables_here(); }

hipError_t launch_residual_vjp(const LaunchCtx& c, const DevMesh& m, const void* u, const void* ybar,
                               void* prev_bar, void* un_bar, const double* dt, double a, double c_id,
                               double c_dt, int accumulate) {
    const unsigned bs = 256, g = grid_for(m.K, bs);
    CSWDG_DISPATCH_EN(c.eq, c.N, {
        k_residual_vjp<EQ, N><<<g, bs, 0, c.stream>>>(m, (const double*)u, (const double*)ybar, (double*)prev_bar,
                                                      (double*)un_bar, dt, a, c_id, c_dt, accumulate, c.gamma);
    });
    return hipGetLastError();
}

hipError_t launch_compact_slots(const LaunchCtx& c, int K, const uint8_t* mask, int32_t* list, int32_t* slot,
                                uint32_t* count) {
    k_compact_slots<<<grid_for(K, 256), 256, 0, c.stream>>>(K, mask, list, slot, count);
    return hipGetLastError();
}

hipError_t launch_limiter_vjp(const LaunchCtx& c, const DevMesh& m, const void* w, const double* ops,
                              const int32_t* list, const uint32_t* count, const void* ybar, double* contrib,
                              int max_cells) {
    const unsigned bs = 64;
    const int lpc = c.eq == 1 ? LimLanes<1>::LPC : LimLanes<0>::LPC;
    unsigned g = grid_for(max_cells, bs / lpc);
    if (g > 16384u) g = 16384u;
    if (g == 0) g = 1;
    CSWDG_DISPATCH_EN(c.eq, c.N, {
        const int qt = N >= 2 ? c.qtop : kTopQuadratic;
        if (qt == kTopSextic) return hipErrorInvalidValue;  // no adjoint of the sextic top
        if (N == 1 || qt == kTopQuadratic)
            k_limiter_vjp<EQ, N, kTopQuadratic><<<g, bs, 0, c.stream>>>(m, (const double*)w, ops, list, count,
                                                                        (const double*)ybar, contrib, c.gamma, c.eps);
        else if (qt == kTopCubic)
            k_limiter_vjp<EQ, N, kTopCubic><<<g, bs, 0, c.stream>>>(m, (const double*)w, ops, list, count,
                                                                    (const double*)ybar, contrib, c.gamma, c.eps);
        else if (qt == kTopCubicTel)
            k_limiter_vjp<EQ, N, kTopCubicTel><<<g, bs, 0, c.stream>>>(m, (const double*)w, ops, list, count,
                                                                       (const double*)ybar, contrib, c.gamma, c.eps);
        else
            k_limiter_vjp<EQ, N, kTopQuartic><<<g, bs, 0, c.stream>>>(m, (const double*)w, ops, list, count,
                                                                      (const double*)ybar, contrib, c.gamma, c.eps);
    });
    return hipGetLastError();
}

hipError_t launch_limiter_gather(const LaunchCtx& c, const DevMesh& m, const uint8_t* mask, const int32_t* slot,
                                 const double* contrib, const void* ybar, void* wbar) {
    const unsigned g = grid_for(m.K, 256);
    CSWDG_DISPATCH_EN(c.eq, c.N, {
        k_limiter_gather<EQ, N><<<g, 256, 0, c.stream>>>(m, mask, slot, contrib, (const double*)ybar, (double*)wbar);
    });
    return hipGetLastError();
}

}  // namespace cswdg
