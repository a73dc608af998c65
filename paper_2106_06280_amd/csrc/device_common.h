// Device code shared by the forward and the adjoint translation units: the
// constant tables (one copy per translation unit, uploaded by each unit's
// upload function), the XCD tile mapping, fluxes and characteristic
// matrices.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace cswdg {

using ::sqrt;  // keep sqrt(double) visible next to sqrt(Dual)

// forward-mode number for the derivatives of the characteristic matrices
struct Dual {
    double v, d;
    __device__ Dual() : v(0.0), d(0.0) {}
    __device__ Dual(double a) : v(a), d(0.0) {}
    __device__ Dual(double a, double b) : v(a), d(b) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
    const double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
__device__ __forceinline__ Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
__device__ __forceinline__ Dual operator/(double a, Dual b) { return Dual(a, 0.0) / b; }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
__device__ __forceinline__ Dual sqrt(Dual a) {
    const double s = ::sqrt(a.v);
    return Dual(s, 0.5 * a.d / s);
}

namespace {

template <int N>
struct TabIC {
    double r[Dims<N>::NQI], s[Dims<N>::NQI];
    double wV[Dims<N>::NQI][Dims<N>::NP];
};

__constant__ Tab<1> c_tab1;
__constant__ Tab<2> c_tab2;
__constant__ Tab<3> c_tab3;
__constant__ TabF<1> c_tabf1;
__constant__ TabF<2> c_tabf2;
__constant__ TabF<3> c_tabf3;
__constant__ TabIC<1> c_ic1;
__constant__ TabIC<2> c_ic2;
__constant__ TabIC<3> c_ic3;

template <int N>
__device__ __forceinline__ const Tab<N>& tab();
template <>
__device__ __forceinline__ const Tab<1>& tab<1>() { return c_tab1; }
template <>
__device__ __forceinline__ const Tab<2>& tab<2>() { return c_tab2; }
template <>
__device__ __forceinline__ const Tab<3>& tab<3>() { return c_tab3; }
// tables in the residual's arithmetic type
template <int N, typename R>
struct TabOf;
template <int N>
struct TabOf<N, double> {
    __device__ static __forceinline__ const Tab<N>& get() { return tab<N>(); }
};
template <>
struct TabOf<1, float> {
    __device__ static __forceinline__ const TabF<1>& get() { return c_tabf1; }
};
template <>
struct TabOf<2, float> {
    __device__ static __forceinline__ const TabF<2>& get() { return c_tabf2; }
};
template <>
struct TabOf<3, float> {
    __device__ static __forceinline__ const TabF<3>& get() { return c_tabf3; }
};
template <int N>
__device__ __forceinline__ const TabIC<N>& tabic();
template <>
__device__ __forceinline__ const TabIC<1>& tabic<1>() { return c_ic1; }
template <>
__device__ __forceinline__ const TabIC<2>& tabic<2>() { return c_ic2; }
template <>
__device__ __forceinline__ const TabIC<3>& tabic<3>() { return c_ic3; }

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD one
// contiguous range of element tiles so that neighbour gathers stay in its L2.
__device__ __forceinline__ int xcd_block(int b, int G, int on = 1) {
    if (!on) return b;
    int q = G >> 3, r = G & 7, x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// ---------------------------------------------------------------------------
// Troubled-cell lists: kListSegs segments of capacity K (segment x at
// list + x K), each with its own counter at count[x * kCountStride] (one
// 128-byte line each). A block appends with one atomic on its own segment,
// so appends from different XCDs do not serialise on one address.
// Consumers walk a global index t over the concatenated segments.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void seg_prefix(const uint32_t* __restrict__ count, int K, uint32_t pre[kListSegs + 1]) {
    pre[0] = 0u;
#pragma unroll
    for (int x = 0; x < kListSegs; ++x) pre[x + 1] = pre[x] + min(count[x * kCountStride], (uint32_t)K);
}

__device__ __forceinline__ int seg_elem(const int32_t* __restrict__ list, const uint32_t pre[kListSegs + 1], int K,
                                        uint32_t t) {
    int x = 0;
#pragma unroll
    for (int y = 1; y < kListSegs; ++y) x += (t >= pre[y]) ? 1 : 0;
    return list[(size_t)x * K + (t - pre[x])];
}

// block-wide append of the elements with tr set (every thread of the block
// must call it; blockDim.x a multiple of 64, at most 1024)
__device__ __forceinline__ void append_list_block(bool tr, int e, int32_t* __restrict__ list,
                                                  uint32_t* __restrict__ count, int K, int seg) {
    __shared__ uint32_t wbase[16];
    __shared__ uint32_t bbase;
    const unsigned long long mask = __ballot(tr ? 1 : 0);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wbase[w] = (uint32_t)__popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0u;
        const int nw = (int)(blockDim.x >> 6);
        for (int i = 0; i < nw; ++i) {
            const uint32_t c = wbase[i];
            wbase[i] = acc;
            acc += c;
        }
        bbase = acc ? atomicAdd(&count[seg * kCountStride], acc) : 0u;
    }
    __syncthreads();
    const uint32_t pos = bbase + wbase[w] + (uint32_t)before;
    if (tr && pos < (uint32_t)K) list[(size_t)seg * K + pos] = e;
}

// Exterior trace of a boundary face (Section 4, Examples 4-6), given the
// interior trace um and up already set to it (outflow): a reflective wall
// reverses the normal momentum, an inflow face takes the prescribed state.
// The kind is kept in the face bits of the boundary face's info byte.
// side of the moving shock of boundary kind 3 at (x, y) and time t: the
// index of the first component of its post- (behind: n.x < d0 + w t) or
// pre-shock state in the shock record {nx, ny, d0, w, post[4], pre[4]}
__device__ __forceinline__ int shock_state_at(const double* __restrict__ shock, double x, double y, double t) {
    return (shock[0] * x + shock[1] * y < shock[2] + shock[3] * t) ? 4 : 8;
}

// exterior trace of a boundary point (x, y) at time t (kinds: 0 outflow,
// 1 reflective wall, 2 inflow state, 3 moving shock; the point and time are
// read for kind 3 only)
template <int EQ, typename R>
__device__ __forceinline__ void boundary_trace(const R* um, R* up, uint32_t inf, R nx, R ny,
                                               const double* __restrict__ inflow,
                                               const double* __restrict__ shock, double x, double y, double t) {
    // selects rather than branches keep up[] in registers
    constexpr int M = (EQ == 1) ? 4 : 1;
    const uint32_t kind = inf & 3u;
    if constexpr (EQ == 1) {
        const R mn = um[1] * nx + um[2] * ny;
        const R w1 = um[1] - R(2) * mn * nx, w2 = um[2] - R(2) * mn * ny;
        up[1] = (kind == 1u) ? w1 : up[1];
        up[2] = (kind == 1u) ? w2 : up[2];
    }
#pragma unroll
    for (int c = 0; c < M; ++c) up[c] = (kind == 2u) ? (R)inflow[c] : up[c];
    if constexpr (EQ == 1) {
        if (shock != nullptr) {
            const int o = shock_state_at(shock, x, y, t);
#pragma unroll
            for (int c = 0; c < M; ++c) up[c] = (kind == 3u) ? (R)shock[o + c] : up[c];
        }
    }
}


// instance holding element e (binary search over the instance offsets)
__device__ __forceinline__ int inst_of(const DevMesh& m, int e) {
    if (m.n_inst <= 1) return 0;
    int lo = 0, hi = m.n_inst;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (e >= m.inst_off[mid]) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Lax-Friedrichs constant of the element's instance when one global constant
// per residual is set (DevMesh::lf_alpha), else -1 (local: the larger
// normal wave speed of the two traces at each point)
__device__ __forceinline__ double lf_global(const DevMesh& m, int e) {
    return m.lf_alpha ? m.lf_alpha[inst_of(m, e)] : -1.0;
}

// time of a residual's input for the moving-shock boundary: the step's
// start for u^n (modes 0, 1), + dt for u^(1) (mode 2), + dt/2 for u^(2)
// (mode 3)
template <int MODE>
__device__ __forceinline__ double stage_time(const DevMesh& m, int e, const double* __restrict__ dtp) {
    if (m.shock == nullptr) return 0.0;
    const int i = inst_of(m, e);
    if constexpr (MODE == 2) return m.time[i] + dtp[i];
    if constexpr (MODE == 3) return m.time[i] + 0.5 * dtp[i];
    return m.time[i];
}

// ---------------------------------------------------------------------------
// Physics: fluxes and wave speeds (Section 4 eqs. 2dBurgers, 2dEulerEquations)
// ---------------------------------------------------------------------------
// reciprocal: hardware estimate refined by Newton-Raphson (two steps in
// double, one in single precision)
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float rcp_nr(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    const float e = fmaf(-x, r, 1.0f);
    return fmaf(r, e, r);
}
// square root: reciprocal square-root estimate refined by Newton-Raphson
// (Goldschmidt form), then one correction of the root
__device__ __forceinline__ double sqrt_nr(double a) {
    double y = __builtin_amdgcn_rsq(a);
    double h = 0.5 * y;
    double g = a * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, g, a);
    return fma(r, h, g);
}
__device__ __forceinline__ float sqrt_nr(float a) { return __builtin_sqrtf(a); }
__device__ __forceinline__ double abs_r(double a) { return fabs(a); }
__device__ __forceinline__ float abs_r(float a) { return fabsf(a); }
__device__ __forceinline__ double max_r(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float max_r(float a, float b) { return fmaxf(a, b); }

template <int EQ>
struct Phys;

template <>
struct Phys<0> {
    static constexpr int M = 1;
    template <typename R>
    __device__ static __forceinline__ void normal_flux(const R* u, R nx, R ny, R, R* Fn, R& lam) {
        R h = R(0.5) * u[0] * u[0];
        Fn[0] = h * nx + h * ny;
        lam = abs_r(u[0] * (nx + ny));
    }
    template <typename R>
    __device__ static __forceinline__ void flux(const R* u, R, R* F, R* G) {
        F[0] = R(0.5) * u[0] * u[0];
        G[0] = F[0];
    }
};

template <>
struct Phys<1> {
    static constexpr int M = 4;
    template <typename R>
    __device__ static __forceinline__ void flux(const R* U, R g, R* F, R* G) {
        R rho = U[0], mu = U[1], mv = U[2], E = U[3];
        R ir = rcp_nr(rho);
        R u = mu * ir, v = mv * ir;
        R p = (g - R(1)) * (E - R(0.5) * rho * (u * u + v * v));
        F[0] = mu;
        F[1] = mu * u + p;
        F[2] = mv * u;
        F[3] = (E + p) * u;
        G[0] = mv;
        G[1] = mu * v;
        G[2] = mv * v + p;
        G[3] = (E + p) * v;
    }
    template <typename R>
    __device__ static __forceinline__ void normal_flux(const R* U, R nx, R ny, R g, R* Fn, R& lam) {
        R rho = U[0], mu = U[1], mv = U[2], E = U[3];
        R ir = rcp_nr(rho);
        R u = mu * ir, v = mv * ir;
        R p = (g - R(1)) * (E - R(0.5) * rho * (u * u + v * v));
        R un = u * nx + v * ny;
        Fn[0] = rho * un;
        Fn[1] = mu * un + p * nx;
        Fn[2] = mv * un + p * ny;
        Fn[3] = (E + p) * un;
        lam = abs_r(un) + sqrt_nr(g * p * ir);
    }
};


// ---------------------------------------------------------------------------
// Characteristic matrices, quadratic forms, lanes of the limiter
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void euler_eigen(const T* U, double nx, double ny, double g, T L[4][4],
                                            T R[4][4]) {
    const T rho = U[0], u = U[1] / rho, v = U[2] / rho, E = U[3];
    const T q2 = u * u + v * v;
    const T p = (g - 1.0) * (E - 0.5 * rho * q2);
    const T c = sqrt(g * p / rho);
    const T H = (E + p) / rho;
    const T un = u * nx + v * ny;
    // right eigenvectors (columns): u_n - c, u_n (entropy), u_n (shear), u_n + c
    R[0][0] = 1.0;            R[0][1] = 1.0;      R[0][2] = 0.0;              R[0][3] = 1.0;
    R[1][0] = u - c * nx;     R[1][1] = u;        R[1][2] = -ny;              R[1][3] = u + c * nx;
    R[2][0] = v - c * ny;     R[2][1] = v;        R[2][2] = nx;               R[2][3] = v + c * ny;
    R[3][0] = H - c * un;     R[3][1] = 0.5 * q2; R[3][2] = -ny * u + nx * v; R[3][3] = H + c * un;
    // closed-form inverse
    const T b1 = (g - 1.0) / (c * c), b2 = 0.5 * b1 * q2;
    L[0][0] = 0.5 * (b2 + un / c); L[0][1] = 0.5 * (-b1 * u - nx / c); L[0][2] = 0.5 * (-b1 * v - ny / c); L[0][3] = 0.5 * b1;
    L[1][0] = 1.0 - b2;            L[1][1] = b1 * u;                   L[1][2] = b1 * v;                   L[1][3] = -b1;
    L[2][0] = ny * u - nx * v;     L[2][1] = -ny;                      L[2][2] = nx;                       L[2][3] = 0.0;
    L[3][0] = 0.5 * (b2 - un / c); L[3][1] = 0.5 * (-b1 * u + nx / c); L[3][2] = 0.5 * (-b1 * v + ny / c); L[3][3] = 0.5 * b1;
}

// c^T B c over the leading k x k block of the packed upper triangle of an
// nm x nm matrix
template <int NM, int KK>
__device__ __forceinline__ double quad_form(const double* __restrict__ bp, const double* c) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < KK; ++i) {
        const int row = i * NM - (i * (i - 1)) / 2;
        double t = bp[row] * c[i];
#pragma unroll
        for (int j = i + 1; j < KK; ++j) t += 2.0 * bp[row + (j - i)] * c[j];
        s += c[i] * t;
    }
    return s;
}

// One troubled cell is handled by LPC = (number of characteristic
// directions) x (number of fields) lanes: lane (d, k) reconstructs
// characteristic field k of direction d (Euler: 2 x 4 = 8 lanes; Burgers: 1).
// The lanes of a cell read the same operator record and neighbour
// coefficients (one cache line serves all of them) and combine their
// moments with a butterfly over the cell's lanes.
template <int EQ>
struct LimLanes {
    static constexpr int ND = (EQ == 1) ? 2 : 1;
    static constexpr int M = Phys<EQ>::M;
    static constexpr int LPC = ND * M;
};

template <int N>
void fill_ic(TabIC<N>& t) {
    Rule2D r = triangle_rule(Dims<N>::NI1);
    double psi[Dims<N>::NP];
    for (int q = 0; q < Dims<N>::NQI; ++q) {
        t.r[q] = r.r[q];
        t.s[q] = r.s[q];
        basis_eval(N, r.r[q], r.s[q], psi);
        for (int n = 0; n < Dims<N>::NP; ++n) t.wV[q][n] = r.w[q] * psi[n];
    }
}

inline unsigned grid_for(int K, int bs) { return (unsigned)((K + bs - 1) / bs); }

template <int N>
void to_float(const Tab<N>& t, TabF<N>& f) {
    using D = Dims<N>;
    for (int q = 0; q < D::NQ; ++q)
        for (int n = 0; n < D::NP; ++n) {
            f.V[q][n] = (float)t.V[q][n];
            f.wDr[q][n] = (float)t.wDr[q][n];
            f.wDs[q][n] = (float)t.wDs[q][n];
        }
    for (int a = 0; a < 3; ++a)
        for (int g = 0; g < D::NE; ++g)
            for (int n = 0; n < D::NP; ++n) {
                f.PF[a][g][n] = (float)t.PF[a][g][n];
                f.wPF[a][g][n] = (float)t.wPF[a][g][n];
            }
}

inline int upload_tables_here() {
    static Tab<1> t1;
    static Tab<2> t2;
    static Tab<3> t3;
    static TabIC<1> i1;
    static TabIC<2> i2;
    static TabIC<3> i3;
    static bool filled = false;
    if (!filled) {
        fill_tables<1>(t1);
        fill_tables<2>(t2);
        fill_tables<3>(t3);
        fill_ic<1>(i1);
        fill_ic<2>(i2);
        fill_ic<3>(i3);
        filled = true;
    }
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_tab1), &t1, sizeof(t1)) != hipSuccess) return CSWDG_EHIP;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_tab2), &t2, sizeof(t2)) != hipSuccess) return CSWDG_EHIP;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_tab3), &t3, sizeof(t3)) != hipSuccess) return CSWDG_EHIP;
    static TabF<1> f1;
    static TabF<2> f2;
    static TabF<3> f3;
    to_float(t1, f1);
    to_float(t2, f2);
    to_float(t3, f3);
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_tabf1), &f1, sizeof(f1)) != hipSuccess) return CSWDG_EHIP;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_tabf2), &f2, sizeof(f2)) != hipSuccess) return CSWDG_EHIP;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_tabf3), &f3, sizeof(f3)) != hipSuccess) return CSWDG_EHIP;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_ic1), &i1, sizeof(i1)) != hipSuccess) return CSWDG_EHIP;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_ic2), &i2, sizeof(i2)) != hipSuccess) return CSWDG_EHIP;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_ic3), &i3, sizeof(i3)) != hipSuccess) return CSWDG_EHIP;
    return CSWDG_OK;
}

}  // namespace

#define CSWDG_DISPATCH_EN(EQV, NV, ...)                         \
    do {                                                        \
        if ((EQV) == 0 && (NV) == 1) { constexpr int EQ = 0, N = 1; __VA_ARGS__; } \
        else if ((EQV) == 0 && (NV) == 2) { constexpr int EQ = 0, N = 2; __VA_ARGS__; } \
        else if ((EQV) == 0 && (NV) == 3) { constexpr int EQ = 0, N = 3; __VA_ARGS__; } \
        else if ((EQV) == 1 && (NV) == 1) { constexpr int EQ = 1, N = 1; __VA_ARGS__; } \
        else if ((EQV) == 1 && (NV) == 2) { constexpr int EQ = 1, N = 2; __VA_ARGS__; } \
        else if ((EQV) == 1 && (NV) == 3) { constexpr int EQ = 1, N = 3; __VA_ARGS__; } \
        else return hipErrorInvalidValue;                       \
    } while (0)

// the same with the state's storage type S (double, or float for FP32-bulk)
#define CSWDG_DISPATCH_ENP(EQV, NV, PV, ...)                  \
    do {                                                      \
        if ((PV) == 1) {                                      \
            using S = float;                                  \
            CSWDG_DISPATCH_EN(EQV, NV, __VA_ARGS__);          \
        } else {                                              \
            using S = double;                                 \
            CSWDG_DISPATCH_EN(EQV, NV, __VA_ARGS__);          \
        }                                                     \
    } while (0)

}  // namespace cswdg
