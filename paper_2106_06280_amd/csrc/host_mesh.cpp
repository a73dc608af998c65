// Host triangulation checks and connectivity (Section 2, eq. triangulation;
// the neighbour 'across the boundary' of Section 3.1 and the immediate
// neighbours of Section 3.2).
//
// Interior edges are paired by sorting the 3K half-edges on their
// (min vertex id, max vertex id) key.  Periodic boundary edges are paired
// by coordinates: half-edge q is the partner of p when q's start plus a
// period vector equals p's end and q's end plus the same vector equals p's
// start, within 1e-9 times the larger period.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace cswdg {

namespace {

int shift_code(double s) { return s == 0.0 ? 0 : (s > 0.0 ? 1 : 2); }

}  // namespace

int build_mesh(int64_t nv, const double* vxy, int64_t nt, const int32_t* tri_in, int bc, double px,
               double py, HostMesh& m, std::string& msg) {
    if (nv <= 0 || nt <= 0 || !vxy || !tri_in) {
        msg = "mesh: empty or null arrays";
        return CSWDG_EINVAL;
    }
    if (bc != CSWDG_BC_PERIODIC && bc != CSWDG_BC_TRANSMISSIVE) {
        msg = "mesh: unknown boundary condition";
        return CSWDG_EINVAL;
    }
    if (nt > kMaxTriangles) {
        msg = "mesh: more than 715,827,882 triangles (the kernels index the [3][K] vertex and neighbour arrays "
              "with 32-bit integers)";
        return CSWDG_EINVAL;
    }
    const int64_t K = nt;
    m = HostMesh();
    m.K = K;
    m.bc = bc;
    m.px = px;
    m.py = py;
    m.tri.assign(tri_in, tri_in + 3 * K);
    for (int64_t i = 0; i < 3 * K; ++i)
        if (m.tri[i] < 0 || m.tri[i] >= nv) {
            msg = "mesh: vertex id out of range";
            return CSWDG_EBADMESH;
        }
    // counter-clockwise fix
    for (int64_t e = 0; e < K; ++e) {
        int32_t* t = &m.tri[3 * e];
        double x0 = vxy[2 * t[0]], y0 = vxy[2 * t[0] + 1];
        double x1 = vxy[2 * t[1]], y1 = vxy[2 * t[1] + 1];
        double x2 = vxy[2 * t[2]], y2 = vxy[2 * t[2] + 1];
        double a2 = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
        if (a2 == 0.0) {
            msg = "mesh: zero-area triangle " + std::to_string(e);
            return CSWDG_EBADMESH;
        }
        if (a2 < 0.0) {
            std::swap(t[1], t[2]);
            ++m.n_flipped;
        }
    }
    // interior edges by sorted vertex-pair keys
    std::vector<int64_t> key(3 * K);
    std::vector<int64_t> order(3 * K);
    for (int64_t e = 0; e < K; ++e)
        for (int f = 0; f < 3; ++f) {
            int64_t a = m.tri[3 * e + f], b = m.tri[3 * e + (f + 1) % 3];
            int64_t lo = std::min(a, b), hi = std::max(a, b);
            key[3 * e + f] = lo * nv + hi;
        }
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return key[x] < key[y]; });
    m.nbr.assign(3 * K, -1);
    m.info.assign(3 * K, 0);
    std::vector<int64_t> boundary;
    for (int64_t i = 0; i < 3 * K;) {
        int64_t j = i;
        while (j < 3 * K && key[order[j]] == key[order[i]]) ++j;
        int64_t cnt = j - i;
        if (cnt > 2) {
            msg = "mesh: non-manifold edge";
            return CSWDG_EBADMESH;
        }
        if (cnt == 2) {
            int64_t h0 = order[i], h1 = order[i + 1];
            int64_t e0 = h0 / 3, f0 = h0 % 3, e1 = h1 / 3, f1 = h1 % 3;
            if (m.tri[3 * e0 + f0] == m.tri[3 * e1 + f1]) {
                msg = "mesh: neighbours traverse their shared edge in the same direction";
                return CSWDG_EBADMESH;
            }
            m.nbr[h0] = (int32_t)e1;
            m.nbr[h1] = (int32_t)e0;
            m.info[h0] = (uint8_t)f1;
            m.info[h1] = (uint8_t)f0;
        } else {
            boundary.push_back(order[i]);
        }
        i = j;
    }
    if (bc == CSWDG_BC_TRANSMISSIVE) {
        for (int64_t h : boundary) m.info[h] = 0x40;
    } else if (!boundary.empty()) {
        double tol = 1e-9 * std::max(std::fabs(px), std::fabs(py));
        if (!(tol > 0.0)) {
            msg = "mesh: periodic boundary needs positive periods";
            return CSWDG_EINVAL;
        }
        const int64_t B = (int64_t)boundary.size();
        std::vector<double> ax(B), ay(B), bx(B), by(B);
        for (int64_t p = 0; p < B; ++p) {
            int64_t h = boundary[p], e = h / 3, f = h % 3;
            int64_t a = m.tri[3 * e + f], b = m.tri[3 * e + (f + 1) % 3];
            ax[p] = vxy[2 * a];
            ay[p] = vxy[2 * a + 1];
            bx[p] = vxy[2 * b];
            by[p] = vxy[2 * b + 1];
        }
        // index boundary half-edges by their start x (then y) for range queries
        std::vector<int64_t> idx(B);
        std::iota(idx.begin(), idx.end(), 0);
        std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
            return ax[x] < ax[y] || (ax[x] == ax[y] && ay[x] < ay[y]);
        });
        std::vector<double> sax(B);
        for (int64_t k = 0; k < B; ++k) sax[k] = ax[idx[k]];
        const double sh[4][2] = {{px, 0.0}, {-px, 0.0}, {0.0, py}, {0.0, -py}};
        for (int64_t p = 0; p < B; ++p) {
            int matches = 0;
            int64_t q_found = -1;
            int s_found = -1;
            for (int si = 0; si < 4; ++si) {
                if (sh[si][0] == 0.0 && sh[si][1] == 0.0) continue;
                // candidate q: ax[q] + sx == bx[p]
                double target = bx[p] - sh[si][0];
                auto lo = std::lower_bound(sax.begin(), sax.end(), target - 2 * tol);
                for (auto it = lo; it != sax.end() && *it <= target + 2 * tol; ++it) {
                    int64_t q = idx[it - sax.begin()];
                    bool c1 = std::fabs(ax[q] + sh[si][0] - bx[p]) <= tol && std::fabs(ay[q] + sh[si][1] - by[p]) <= tol;
                    bool c2 = std::fabs(bx[q] + sh[si][0] - ax[p]) <= tol && std::fabs(by[q] + sh[si][1] - ay[p]) <= tol;
                    if (c1 && c2) {
                        ++matches;
                        q_found = q;
                        s_found = si;
                    }
                }
            }
            // periodic in one direction only (the other period 0): an edge
            // without a partner stays a boundary face
            if (matches == 0 && (px == 0.0) != (py == 0.0)) {
                m.info[boundary[p]] = 0x40;
                continue;
            }
            if (matches != 1) {
                msg = "mesh: unmatched or ambiguous periodic boundary edge";
                return CSWDG_EBADMESH;
            }
            int64_t hp = boundary[p], hq = boundary[q_found];
            m.nbr[hp] = (int32_t)(hq / 3);
            m.info[hp] = (uint8_t)((hq % 3) | (shift_code(sh[s_found][0]) << 2) | (shift_code(sh[s_found][1]) << 4));
        }
    }
    // element vertices (SoA) and the time-step length scale
    m.vx.resize(3 * K);
    m.vy.resize(3 * K);
    double hmin = INFINITY;
    for (int64_t e = 0; e < K; ++e) {
        for (int k = 0; k < 3; ++k) {
            m.vx[k * K + e] = vxy[2 * m.tri[3 * e + k]];
            m.vy[k * K + e] = vxy[2 * m.tri[3 * e + k] + 1];
        }
        double x0 = m.vx[e], x1 = m.vx[K + e], x2 = m.vx[2 * K + e];
        double y0 = m.vy[e], y1 = m.vy[K + e], y2 = m.vy[2 * K + e];
        double area = 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0));
        double a = std::hypot(x1 - x0, y1 - y0), b = std::hypot(x2 - x1, y2 - y1), c = std::hypot(x0 - x2, y0 - y2);
        double twor = 4.0 * area / (a + b + c);
        hmin = std::min(hmin, twor);
    }
    m.hmin = hmin;
    return CSWDG_OK;
}

int concat_meshes(const std::vector<HostMesh>& parts, HostMesh& out, std::vector<int32_t>& off,
                  std::vector<double>& hmin, std::string& msg) {
    int64_t K = 0;
    for (const HostMesh& p : parts) K += p.K;
    if (parts.empty() || K > (int64_t)0x3fffffff) {
        msg = "mesh: instance count or total size out of range";
        return CSWDG_EINVAL;
    }
    out = HostMesh();
    out.K = K;
    out.bc = parts[0].bc;
    out.px = parts[0].px;
    out.py = parts[0].py;
    out.hmin = INFINITY;
    for (const HostMesh& p : parts) {
        // periodic shifts are applied with the union's period
        if (p.bc == CSWDG_BC_PERIODIC && (p.px != out.px || p.py != out.py)) {
            msg = "mesh: periodic instances must share one period";
            return CSWDG_EINVAL;
        }
    }
    out.tri.resize(3 * K);
    out.nbr.resize(3 * K);
    out.info.resize(3 * K);
    out.vx.resize(3 * K);
    out.vy.resize(3 * K);
    off.assign(parts.size() + 1, 0);
    hmin.assign(parts.size(), 0.0);
    int64_t e0 = 0, v0 = 0;
    for (size_t i = 0; i < parts.size(); ++i) {
        const HostMesh& p = parts[i];
        off[i] = (int32_t)e0;
        hmin[i] = p.hmin;
        out.hmin = std::min(out.hmin, p.hmin);
        out.n_flipped += p.n_flipped;
        int32_t vmax = -1;
        for (int64_t j = 0; j < 3 * p.K; ++j) {
            out.tri[3 * e0 + j] = (int32_t)(p.tri[j] + v0);
            vmax = std::max(vmax, p.tri[j]);
            const bool bnd = (p.info[j] & 0x40) != 0;
            out.nbr[3 * e0 + j] = bnd ? p.nbr[j] : (int32_t)(p.nbr[j] + e0);
            out.info[3 * e0 + j] = p.info[j];
        }
        for (int k = 0; k < 3; ++k)
            for (int64_t e = 0; e < p.K; ++e) {
                out.vx[k * K + e0 + e] = p.vx[k * p.K + e];
                out.vy[k * K + e0 + e] = p.vy[k * p.K + e];
            }
        e0 += p.K;
        v0 += (int64_t)vmax + 1;
    }
    off[parts.size()] = (int32_t)K;
    return CSWDG_OK;
}

}  // namespace cswdg
