// gfx950 kernels of one SSP-RK3 stage with the CSWENO limiter.
//
// Layout: state [m][Np][K] (element index fastest, so a wave of 64
// consecutive elements reads each coefficient with one coalesced access);
// element vertices [3][K] for x and y; neighbours [3][K]; face info packed
// as one uint32 per element (byte f = info of face f).
//
// Kernels
//   k_residual  one thread per element: volume quadrature of
//               grad(psi).F(u_h), traces of the element and of its three
//               neighbours at the edge Gauss points, local Lax-Friedrichs
//               flux, lift, inverse mass matrix (1/J) and the RK combine.
//   k_dt_*      cell-mean wave speeds -> dt (two-pass reduction).
//   k_kxrcf     one thread per element: KXRCF indicator, then a wave ballot
//               and one atomic per wave to append troubled cells to a list.
//   k_tvb       the same with the TVB minmod test (params.indicator = 1).
//   k_limiter   one lane per (troubled cell, characteristic direction,
//               field): subcell averages, the three (four) least-squares
//               levels, smoothness indicators, WENO-Z weights and the
//               projection; a lane butterfly recombines the conserved
//               moments; results to a compact buffer (every cell reads the
//               pre-limit field).
//   k_limiter_t1, k_limiter_t2, k_limiter_mx  the same lanes with the
//               type-I, type-II and mixed WENO reconstructions on the
//               subcell stencils (params.reconstruction = 1, 2, 3).
//   k_scatter   compact results -> state (modes >= 1).
//   k_positivity  optional, not in the paper: Zhang-Shu positivity scaling
//               of every Euler cell at the residual's evaluation points.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "device_common.h"

namespace cswdg {

namespace {

// ---------------------------------------------------------------------------
// Residual and RK stage
// ---------------------------------------------------------------------------
template <int EQ, int N, int MODE>
__device__ __forceinline__ void residual_body(DevMesh msh, const double* __restrict__ u,
                                              const double* __restrict__ un,
                                              double* __restrict__ out,
                                              const double* __restrict__ dtp, double gamma,
                                              uint32_t* __restrict__ cnt_reset) {
    using D = Dims<N>;
    constexpr int M = Phys<EQ>::M, NP = D::NP, NE = D::NE, NQ = D::NQ;
    const int K = msh.K;
    const int e = xcd_block(blockIdx.x, gridDim.x, msh.xcd_tiles) * blockDim.x + threadIdx.x;
    if (cnt_reset != nullptr && blockIdx.x == 0 && threadIdx.x < kListSegs) cnt_reset[threadIdx.x * kCountStride] = 0u;
    if (e >= K) return;
    const double ag = lf_global(msh, e);  // < 0: local Lax-Friedrichs
    const Tab<N>& T = tab<N>();

    double U[M][NP];
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int n = 0; n < NP; ++n) U[c][n] = u[(size_t)(c * NP + n) * K + e];

    const double X[3] = {msh.vx[e], msh.vx[K + e], msh.vx[2 * K + e]};
    const double Y[3] = {msh.vy[e], msh.vy[K + e], msh.vy[2 * K + e]};
    const double xr = 0.5 * (X[1] - X[0]), xs = 0.5 * (X[2] - X[0]);
    const double yr = 0.5 * (Y[1] - Y[0]), ys = 0.5 * (Y[2] - Y[0]);
    const double J = xr * ys - xs * yr;
    const double iJ = 1.0 / J;
    const double rx = ys * iJ, ry = -xs * iJ, sx = -yr * iJ, sy = xr * iJ;

    double acc[M][NP];
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int n = 0; n < NP; ++n) acc[c][n] = 0.0;

    // volume term: sum_q w_q (dpsi/dr (r_x f + r_y g) + dpsi/ds (s_x f + s_y g))
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double uq[M], F[M], G[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            double s = 0.0;
#pragma unroll
            for (int n = 0; n < NP; ++n) s += T.V[q][n] * U[c][n];
            uq[c] = s;
        }
        Phys<EQ>::flux(uq, gamma, F, G);
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const double fr = rx * F[c] + ry * G[c];
            const double fs = sx * F[c] + sy * G[c];
#pragma unroll
            for (int i = 0; i < NP; ++i) acc[c][i] += T.wDr[q][i] * fr + T.wDs[q][i] * fs;
        }
    }

    // surface term
    const uint32_t info4 = msh.info[e];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const int f1 = (f + 1) % 3;
        const double ex = X[f1] - X[f], ey = Y[f1] - Y[f];
        const double L = sqrt(ex * ex + ey * ey);
        const double iL = 1.0 / L;
        const double nx = ey * iL, ny = -ex * iL;
        const double sf = 0.5 * L * iJ;
        const uint32_t inf = (info4 >> (8 * f)) & 0xffu;
        const bool bnd = (inf & 0x40u) != 0u;
        const int fp = bnd ? 0 : (int)(inf & 3u);
        const int nb = bnd ? e : msh.nbr[f * K + e];
        double Un[M][NP];
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int n = 0; n < NP; ++n) Un[c][n] = u[(size_t)(c * NP + n) * K + nb];
#pragma unroll
        for (int g = 0; g < NE; ++g) {
            double um[M], up[M];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                double a = 0.0, b = 0.0;
#pragma unroll
                for (int n = 0; n < NP; ++n) {
                    a += T.PF[f][g][n] * U[c][n];
                    b += T.PF[fp][NE - 1 - g][n] * Un[c][n];
                }
                um[c] = a;
                up[c] = bnd ? a : b;
            }
            if (bnd)
                boundary_trace<EQ>(um, up, inf, nx, ny, msh.inflow, msh.shock, X[f] + tab<N>().es[g] * ex,
                                   Y[f] + tab<N>().es[g] * ey, stage_time<MODE>(msh, e, dtp));
            double Fm[M], Fp[M], lm, lp;
            Phys<EQ>::normal_flux(um, nx, ny, gamma, Fm, lm);
            Phys<EQ>::normal_flux(up, nx, ny, gamma, Fp, lp);
            const double alpha = (ag >= 0.0) ? ag : fmax(lm, lp);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const double Fs = 0.5 * (Fm[c] + Fp[c]) - 0.5 * alpha * (up[c] - um[c]);
                const double sFs = sf * Fs;
#pragma unroll
                for (int i = 0; i < NP; ++i) acc[c][i] -= T.wPF[f][g][i] * sFs;
            }
        }
    }

    double dt = 0.0;
    if (MODE != 0) dt = dtp[inst_of(msh, e)];
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const size_t idx = (size_t)(c * NP + i) * K + e;
            double v;
            if (MODE == 0) {
                v = acc[c][i];
            } else if (MODE == 1) {
                v = U[c][i] + dt * acc[c][i];
            } else if (MODE == 2) {
                v = 0.75 * un[idx] + 0.25 * (U[c][i] + dt * acc[c][i]);
            } else {
                v = (1.0 / 3.0) * un[idx] + (2.0 / 3.0) * (U[c][i] + dt * acc[c][i]);
            }
            out[idx] = v;
        }
}

// Four schedules of the same arithmetic (results agree to rounding): "wide"
// keeps the neighbour coefficients of all faces live (one wave per SIMD for
// P2 Euler), "lean" bounds the live ranges to one face (two waves per SIMD
// without spills), "stream" also re-reads the element's own coefficients per
// face, "compact" (below, the default) rolls the quadrature-point loops.
template <int EQ, int N, int MODE>
__global__ __launch_bounds__(256) void k_residual(DevMesh msh, const double* __restrict__ u,
                                                  const double* __restrict__ un, double* __restrict__ out,
                                                  const double* __restrict__ dtp, double gamma,
                                                  uint32_t* __restrict__ cnt_reset) {
    residual_body<EQ, N, MODE>(msh, u, un, out, dtp, gamma, cnt_reset);
}

// Same arithmetic as residual_body with bounded live ranges: the face loop is
// not unrolled (its tables are read with a uniform face index), and the
// neighbour's traces are formed one conserved variable at a time, so only
// the element's coefficients, the accumulators and one face's traces are
// live at once.
template <int EQ, int N, int MODE>
__device__ __forceinline__ void residual_body_lean(DevMesh msh, const double* __restrict__ u,
                                                   const double* __restrict__ un,
                                                   double* __restrict__ out,
                                                   const double* __restrict__ dtp, double gamma,
                                                   uint32_t* __restrict__ cnt_reset) {
    using D = Dims<N>;
    constexpr int M = Phys<EQ>::M, NP = D::NP, NE = D::NE, NQ = D::NQ;
    const int K = msh.K;
    const int e = xcd_block(blockIdx.x, gridDim.x, msh.xcd_tiles) * blockDim.x + threadIdx.x;
    if (cnt_reset != nullptr && blockIdx.x == 0 && threadIdx.x < kListSegs) cnt_reset[threadIdx.x * kCountStride] = 0u;
    if (e >= K) return;
    const double ag = lf_global(msh, e);  // < 0: local Lax-Friedrichs
    const Tab<N>& T = tab<N>();

    double U[M][NP];
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int n = 0; n < NP; ++n) U[c][n] = u[(size_t)(c * NP + n) * K + e];

    double acc[M][NP];
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int n = 0; n < NP; ++n) acc[c][n] = 0.0;
    {
        const double x0 = msh.vx[e], x1 = msh.vx[K + e], x2 = msh.vx[2 * K + e];
        const double y0 = msh.vy[e], y1 = msh.vy[K + e], y2 = msh.vy[2 * K + e];
        const double xr = 0.5 * (x1 - x0), xs = 0.5 * (x2 - x0);
        const double yr = 0.5 * (y1 - y0), ys = 0.5 * (y2 - y0);
        const double iJ = 1.0 / (xr * ys - xs * yr);
        const double rx = ys * iJ, ry = -xs * iJ, sx = -yr * iJ, sy = xr * iJ;
#pragma unroll 3
        for (int q = 0; q < NQ; ++q) {
            double uq[M], F[M], G[M];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                double s = 0.0;
#pragma unroll
                for (int n = 0; n < NP; ++n) s += T.V[q][n] * U[c][n];
                uq[c] = s;
            }
            Phys<EQ>::flux(uq, gamma, F, G);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const double fr = rx * F[c] + ry * G[c];
                const double fs = sx * F[c] + sy * G[c];
#pragma unroll
                for (int i = 0; i < NP; ++i) acc[c][i] += T.wDr[q][i] * fr + T.wDs[q][i] * fs;
            }
        }
    }

    const uint32_t info4 = msh.info[e];
#pragma unroll 1
    for (int f = 0; f < 3; ++f) {
        const int f1 = (f == 2) ? 0 : f + 1;
        const double xa = msh.vx[f * K + e], ya = msh.vy[f * K + e];
        const double xb = msh.vx[f1 * K + e], yb = msh.vy[f1 * K + e];
        const double ex = xb - xa, ey = yb - ya;
        const double L = sqrt(ex * ex + ey * ey);
        const double iL = 1.0 / L;
        const double nx = ey * iL, ny = -ex * iL;
        // L_f / (2 J) with 2 J = area; recomputed from the vertices
        const double x0 = msh.vx[e], x1 = msh.vx[K + e], x2 = msh.vx[2 * K + e];
        const double y0 = msh.vy[e], y1 = msh.vy[K + e], y2 = msh.vy[2 * K + e];
        const double J = 0.25 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0));
        const double sf = 0.5 * L / J;
        const uint32_t inf = (info4 >> (8 * f)) & 0xffu;
        const bool bnd = (inf & 0x40u) != 0u;
        const int fp = bnd ? 0 : (int)(inf & 3u);
        const int nb = bnd ? e : msh.nbr[f * K + e];
        double up[NE][M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            double w[NP];
#pragma unroll
            for (int n = 0; n < NP; ++n) w[n] = u[(size_t)(c * NP + n) * K + nb];
#pragma unroll
            for (int g = 0; g < NE; ++g) {
                double s = 0.0;
#pragma unroll
                for (int n = 0; n < NP; ++n) s += T.PF[fp][NE - 1 - g][n] * w[n];
                up[g][c] = s;
            }
        }
#pragma unroll
        for (int g = 0; g < NE; ++g) {
            double um[M], upg[M];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                double a = 0.0;
#pragma unroll
                for (int n = 0; n < NP; ++n) a += T.PF[f][g][n] * U[c][n];
                um[c] = a;
                upg[c] = bnd ? a : up[g][c];
            }
            if (bnd)
                boundary_trace<EQ>(um, upg, inf, nx, ny, msh.inflow, msh.shock, xa + tab<N>().es[g] * ex,
                                   ya + tab<N>().es[g] * ey, stage_time<MODE>(msh, e, dtp));
            double Fm[M], Fp[M], lm, lp;
            Phys<EQ>::normal_flux(um, nx, ny, gamma, Fm, lm);
            Phys<EQ>::normal_flux(upg, nx, ny, gamma, Fp, lp);
            const double alpha = (ag >= 0.0) ? ag : fmax(lm, lp);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const double Fs = 0.5 * (Fm[c] + Fp[c]) - 0.5 * alpha * (upg[c] - um[c]);
                const double sFs = sf * Fs;
#pragma unroll
                for (int i = 0; i < NP; ++i) acc[c][i] -= T.wPF[f][g][i] * sFs;
            }
        }
    }

    double dt = 0.0;
    if (MODE != 0) dt = dtp[inst_of(msh, e)];
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const size_t idx = (size_t)(c * NP + i) * K + e;
            double v;
            if (MODE == 0) {
                v = acc[c][i];
            } else if (MODE == 1) {
                v = U[c][i] + dt * acc[c][i];
            } else if (MODE == 2) {
                v = 0.75 * un[idx] + 0.25 * (U[c][i] + dt * acc[c][i]);
            } else {
                v = (1.0 / 3.0) * un[idx] + (2.0 / 3.0) * (U[c][i] + dt * acc[c][i]);
            }
            out[idx] = v;
        }
}

// "compact" (the default): the lean arithmetic with the quadrature-point
// loops rolled, which bounds the live registers to the element's own
// coefficients, the accumulators and one point's values.
template <int EQ, int N, int MODE, typename R>
__device__ __forceinline__ void residual_body_compact(DevMesh msh, const R* __restrict__ u,
                                                   const R* __restrict__ un,
                                                   R* __restrict__ out,
                                                   const double* __restrict__ dtp, double gamma,
                                                   uint32_t* __restrict__ cnt_reset) {
    using D = Dims<N>;
    constexpr int M = Phys<EQ>::M, NP = D::NP, NE = D::NE, NQ = D::NQ;
    const int K = msh.K;
    const int e = xcd_block(blockIdx.x, gridDim.x, msh.xcd_tiles) * blockDim.x + threadIdx.x;
    if (cnt_reset != nullptr && blockIdx.x == 0 && threadIdx.x < kListSegs) cnt_reset[threadIdx.x * kCountStride] = 0u;
    const auto& T = TabOf<N, R>::get();
    // the face-point table in LDS: the neighbour's trace reads it at the
    // neighbour's own face (a per-lane index), which from constant memory
    // would be one vector-memory access per entry
    __shared__ R sPF[3 * NE * NP];
    for (int i = threadIdx.x; i < 3 * NE * NP; i += blockDim.x) sPF[i] = (&T.PF[0][0][0])[i];
    __syncthreads();
    if (e >= K) return;
    const double ag = lf_global(msh, e);  // < 0: local Lax-Friedrichs
    const R gm = (R)gamma;

    R U[M][NP];
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int n = 0; n < NP; ++n) U[c][n] = u[(size_t)(c * NP + n) * K + e];

    R acc[M][NP];
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int n = 0; n < NP; ++n) acc[c][n] = R(0);
    // the vertices, kept for the faces (one load each)
    const double x0 = msh.vx[e], x1 = msh.vx[K + e], x2 = msh.vx[2 * K + e];
    const double y0 = msh.vy[e], y1 = msh.vy[K + e], y2 = msh.vy[2 * K + e];
    {
        const double xr = 0.5 * (x1 - x0), xs = 0.5 * (x2 - x0);
        const double yr = 0.5 * (y1 - y0), ys = 0.5 * (y2 - y0);
        const double iJ = 1.0 / (xr * ys - xs * yr);
        const R rx = (R)(ys * iJ), ry = (R)(-xs * iJ), sx = (R)(-yr * iJ), sy = (R)(xr * iJ);
#pragma unroll 1
        for (int q = 0; q < NQ; ++q) {
            R uq[M], F[M], G[M];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                R s = R(0);
#pragma unroll
                for (int n = 0; n < NP; ++n) s += T.V[q][n] * U[c][n];
                uq[c] = s;
            }
            Phys<EQ>::flux(uq, gm, F, G);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const R fr = rx * F[c] + ry * G[c];
                const R fs = sx * F[c] + sy * G[c];
#pragma unroll
                for (int i = 0; i < NP; ++i) acc[c][i] += T.wDr[q][i] * fr + T.wDs[q][i] * fs;
            }
        }
    }

    const uint32_t info4 = msh.info[e];
    // 1 / J with 2 J = area: the surface scale L_f / (2 J) per face
    const double iJf = 1.0 / (0.25 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)));
    // FP64 P1/P2 keep the vertices in registers for the faces (fewer
    // vector-memory instructions; the registers are there at two waves per
    // SIMD); the others reload them (P3 and FP32-bulk would lose occupancy)
    constexpr bool hold = sizeof(R) == 8 && N <= 2;
#pragma unroll 1
    for (int f = 0; f < 3; ++f) {
        const int f1 = (f == 2) ? 0 : f + 1;
        double xa, ya, xb, yb;
        if constexpr (hold) {
            xa = (f == 0) ? x0 : ((f == 1) ? x1 : x2);
            ya = (f == 0) ? y0 : ((f == 1) ? y1 : y2);
            xb = (f == 0) ? x1 : ((f == 1) ? x2 : x0);
            yb = (f == 0) ? y1 : ((f == 1) ? y2 : y0);
        } else {
            xa = msh.vx[f * K + e];
            ya = msh.vy[f * K + e];
            xb = msh.vx[f1 * K + e];
            yb = msh.vy[f1 * K + e];
        }
        const double ex = xb - xa, ey = yb - ya;
        const double L = sqrt(ex * ex + ey * ey);
        const double iL = 1.0 / L;
        const R nx = (R)(ey * iL), ny = (R)(-ex * iL);
        const R sf = (R)(0.5 * L * iJf);
        const uint32_t inf = (info4 >> (8 * f)) & 0xffu;
        const bool bnd = (inf & 0x40u) != 0u;
        const int fp = bnd ? 0 : (int)(inf & 3u);
        const int nb = bnd ? e : msh.nbr[f * K + e];
        const int gr = NE - 1;
#pragma unroll 1
        for (int g = 0; g < NE; ++g) {
            R um[M], upg[M];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                R a = R(0), b = R(0);
#pragma unroll
                for (int n = 0; n < NP; ++n) {
                    a += T.PF[f][g][n] * U[c][n];
                    b += sPF[(fp * NE + gr - g) * NP + n] * u[(size_t)(c * NP + n) * K + nb];
                }
                um[c] = a;
                upg[c] = bnd ? a : b;
            }
            if (bnd)
                boundary_trace<EQ>(um, upg, inf, nx, ny, msh.inflow, msh.shock, xa + tab<N>().es[g] * ex,
                                   ya + tab<N>().es[g] * ey, stage_time<MODE>(msh, e, dtp));
            R Fm[M], Fp[M], lm, lp;
            Phys<EQ>::normal_flux(um, nx, ny, gm, Fm, lm);
            Phys<EQ>::normal_flux(upg, nx, ny, gm, Fp, lp);
            const R alpha = (ag >= 0.0) ? (R)ag : max_r(lm, lp);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const R Fs = R(0.5) * (Fm[c] + Fp[c]) - R(0.5) * alpha * (upg[c] - um[c]);
                const R sFs = sf * Fs;
#pragma unroll
                for (int i = 0; i < NP; ++i) acc[c][i] -= T.wPF[f][g][i] * sFs;
            }
        }
    }

    R dt = R(0);
    if (MODE != 0) dt = (R)dtp[inst_of(msh, e)];
    // u^n and the output are streamed once: non-temporal accesses keep them
    // from evicting the u^(i-1) lines that neighbouring elements re-read
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const size_t idx = (size_t)(c * NP + i) * K + e;
            R v;
            if (MODE == 0) {
                v = acc[c][i];
            } else if (MODE == 1) {
                v = U[c][i] + dt * acc[c][i];
            } else if (MODE == 2) {
                v = R(0.75) * __builtin_nontemporal_load(&un[idx]) + R(0.25) * (U[c][i] + dt * acc[c][i]);
            } else {
                v = R(1.0 / 3.0) * __builtin_nontemporal_load(&un[idx]) + R(2.0 / 3.0) * (U[c][i] + dt * acc[c][i]);
            }
            __builtin_nontemporal_store(v, &out[idx]);
        }
}

template <int EQ, int N, int MODE, typename R>
__global__ __launch_bounds__(256) void k_residual_compact(DevMesh msh, const R* __restrict__ u,
                                                          const R* __restrict__ un, R* __restrict__ out,
                                                          const double* __restrict__ dtp, double gamma,
                                                          uint32_t* __restrict__ cnt_reset) {
    residual_body_compact<EQ, N, MODE, R>(msh, u, un, out, dtp, gamma, cnt_reset);
}

template <int EQ, int N, int MODE>
__global__ __launch_bounds__(256) void k_residual_compact_d(DevMesh msh, const double* __restrict__ u,
                                                            const double* __restrict__ un, double* __restrict__ out,
                                                            const double* __restrict__ dtp, double gamma,
                                                            uint32_t* __restrict__ cnt_reset) {
    residual_body_compact<EQ, N, MODE, double>(msh, u, un, out, dtp, gamma, cnt_reset);
}

// ---------------------------------------------------------------------------
// Residual on the matrix cores (P2, FP64): the evaluation of the state at the
// quadrature points and the projections onto the test functions are dense
// contractions with the reference-element matrices, batched over elements,
// so they run as v_mfma_f64_16x16x4 products; the fluxes stay on the vector
// ALU.  One wave takes a tile of 16 elements: lane (a = lane / 16,
// r = lane % 16) works on element r of the tile.  Operand layouts of the
// 16x16x4 product D = A B + C: lane (a, r) holds A[r][a] and B[a][r] (k = a)
// and the four entries D[4 i + a][r], i = 0..3.
//   evaluation: A = a table [16 points x 4 basis functions] (two k-steps for
//     the six P2 functions), B = the tile's coefficients of one variable, so
//     register i of lane (a, r) receives the value at row 4 i + a;
//     volume rows: lane group a holds two points of the 9-point rule (the
//     last group three), face rows: lane group a < 3 holds the four points
//     of face a;
//   projection and lift: each lane's flux values are the B operand of one
//     k-step (k = a: the four lane groups' values enter one product), A holds
//     the matching test-function weights (row = output coefficient), and the
//     products accumulate every variable's right-hand side over 6 volume
//     k-steps and 4 face k-steps into D (output coefficient 4 i + a in
//     register i).
// Same quadrature and flux as the other schedules; the sums run in another
// order.
// ---------------------------------------------------------------------------
typedef double mf_v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mf_v4d mf_mma(double a, double b, mf_v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// point of the 9-point volume rule in slot i of lane group a (-1: padding)
__device__ __forceinline__ int mf_vol_point(int a, int i) {
    if (a < 3) return (i < 2) ? 2 * a + i : -1;
    return (i < 3) ? 6 + i : -1;
}

template <int EQ, int MODE>
__global__ __launch_bounds__(256) void k_residual_mfma(DevMesh msh, const double* __restrict__ u,
                                                       const double* __restrict__ un, double* __restrict__ out,
                                                       const double* __restrict__ dtp, double gamma,
                                                       uint32_t* __restrict__ cnt_reset) {
    constexpr int N = 2;
    using D = Dims<N>;
    constexpr int M = Phys<EQ>::M, NP = D::NP, NE = D::NE, NQ = D::NQ;
    static_assert(NP == 6 && NE == 4 && NQ == 9, "tile layout of the P2 rules");
    const int K = msh.K;
    if (cnt_reset != nullptr && blockIdx.x == 0 && threadIdx.x < kListSegs) cnt_reset[threadIdx.x * kCountStride] = 0u;
    if (K <= 0) return;
    const int lane = threadIdx.x & 63, a = lane >> 4, r = lane & 15;
    const int tile = xcd_block(blockIdx.x, gridDim.x, msh.xcd_tiles) * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
    const int e_raw = tile * 16 + r;
    const bool live = e_raw < K;
    const int e = live ? e_raw : K - 1;  // the tail's lanes compute on a copy and store nothing
    const auto& T = TabOf<N, double>::get();
    const double ag = lf_global(msh, e);  // < 0: local Lax-Friedrichs

    const double X0 = msh.vx[e], X1 = msh.vx[K + e], X2 = msh.vx[2 * K + e];
    const double Y0 = msh.vy[e], Y1 = msh.vy[K + e], Y2 = msh.vy[2 * K + e];

    mf_v4d acc[M];
#pragma unroll
    for (int c = 0; c < M; ++c) acc[c] = mf_v4d{0.0, 0.0, 0.0, 0.0};

    // B operands of both evaluations: coefficient n = 4 s + a of element r
    double bu[2][M];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int n = 4 * s + a;
        const int nc = n < NP ? n : 0;
#pragma unroll
        for (int c = 0; c < M; ++c) bu[s][c] = (n < NP) ? u[(size_t)(c * NP + nc) * K + e] : 0.0;
    }

    // ---- volume term ----
    {
        mf_v4d dv[M];
#pragma unroll
        for (int c = 0; c < M; ++c) dv[c] = mf_v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int n = 4 * s + a;  // basis function of k = a in k-step s
            const bool nok = n < NP;
            const int nc = nok ? n : 0;
            const int qa = mf_vol_point(r & 3, r >> 2);  // point of A's row r
            const double av = (nok && qa >= 0) ? T.V[qa >= 0 ? qa : 0][nc] : 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) dv[c] = mf_mma(av, bu[s][c], dv[c]);
        }
        const double xr = 0.5 * (X1 - X0), xs = 0.5 * (X2 - X0);
        const double yr = 0.5 * (Y1 - Y0), ys = 0.5 * (Y2 - Y0);
        const double iJ = 1.0 / (xr * ys - xs * yr);
        const double rx = ys * iJ, ry = -xs * iJ, sx = -yr * iJ, sy = xr * iJ;
        const double gm = gamma;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int q = mf_vol_point(a, i);
            const bool ok = q >= 0;
            const int qc = ok ? q : 0;
            double uq[M], F[M], G[M];
#pragma unroll
            for (int c = 0; c < M; ++c) uq[c] = ok ? dv[c][i] : (c == 0 ? 1.0 : 0.0);  // padding: a harmless state
            Phys<EQ>::flux(uq, gm, F, G);
            const bool rok = r < NP;
            const int rc = rok ? r : 0;
            const double wr = (ok && rok) ? T.wDr[qc][rc] : 0.0;
            const double ws = (ok && rok) ? T.wDs[qc][rc] : 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const double fr = ok ? rx * F[c] + ry * G[c] : 0.0;
                const double fs = ok ? sx * F[c] + sy * G[c] : 0.0;
                acc[c] = mf_mma(wr, fr, acc[c]);
                acc[c] = mf_mma(ws, fs, acc[c]);
            }
        }
    }

    // ---- surface term: lane group a < 3 takes face a ----
    {
        mf_v4d df[M];
#pragma unroll
        for (int c = 0; c < M; ++c) df[c] = mf_v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int n = 4 * s + a;
            const bool nok = n < NP;
            const int nc = nok ? n : 0;
            const int fa = r & 3, ga = r >> 2;  // face and point of A's row r
            const double af = (nok && fa < 3) ? T.PF[fa < 3 ? fa : 0][ga][nc] : 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) df[c] = mf_mma(af, bu[s][c], df[c]);
        }
        const bool fok = a < 3;
        const int f = fok ? a : 0;
        const int f1 = (f == 2) ? 0 : f + 1;
        const double xa = (f == 0) ? X0 : ((f == 1) ? X1 : X2), ya = (f == 0) ? Y0 : ((f == 1) ? Y1 : Y2);
        const double xb = (f1 == 0) ? X0 : ((f1 == 1) ? X1 : X2), yb = (f1 == 0) ? Y0 : ((f1 == 1) ? Y1 : Y2);
        const double ex = xb - xa, ey = yb - ya;
        const double L = sqrt(ex * ex + ey * ey);
        const double iL = 1.0 / L;
        const double nx = ey * iL, ny = -ex * iL;
        const double J = 0.25 * ((X1 - X0) * (Y2 - Y0) - (X2 - X0) * (Y1 - Y0));
        const double sf = 0.5 * L / J;
        const uint32_t inf = (msh.info[e] >> (8 * f)) & 0xffu;
        const bool bnd = (inf & 0x40u) != 0u;
        const int fp = bnd ? 0 : (int)(inf & 3u);
        const int nb = bnd ? e : msh.nbr[f * K + e];
        double Un[M][NP];
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int n = 0; n < NP; ++n) Un[c][n] = u[(size_t)(c * NP + n) * K + nb];
        const double gm = gamma;
        const bool rok = r < NP;
        const int rc = rok ? r : 0;
#pragma unroll
        for (int g = 0; g < NE; ++g) {
            // own trace from the evaluation product, the neighbour's at the
            // same point (its face fp, points in reverse order)
            double um[M], upg[M];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                double b = 0.0;
#pragma unroll
                for (int n = 0; n < NP; ++n) b += T.PF[fp][NE - 1 - g][n] * Un[c][n];
                um[c] = fok ? df[c][g] : (c == 0 ? 1.0 : 0.0);  // lane group 3: a harmless state
                upg[c] = (bnd || !fok) ? um[c] : b;
            }
            if (bnd && fok)
                boundary_trace<EQ>(um, upg, inf, nx, ny, msh.inflow, msh.shock, xa + tab<N>().es[g] * ex,
                                   ya + tab<N>().es[g] * ey, stage_time<MODE>(msh, e, dtp));
            double Fm[M], Fp[M], lm, lp;
            Phys<EQ>::normal_flux(um, nx, ny, gm, Fm, lm);
            Phys<EQ>::normal_flux(upg, nx, ny, gm, Fp, lp);
            const double alpha = (ag >= 0.0) ? ag : fmax(lm, lp);
            const double w = (fok && rok) ? -T.wPF[f][g][rc] : 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const double Fs = 0.5 * (Fm[c] + Fp[c]) - 0.5 * alpha * (upg[c] - um[c]);
                acc[c] = mf_mma(w, fok ? sf * Fs : 0.0, acc[c]);
            }
        }
    }

    // ---- 1/J is in the weights' metric terms; RK combine of the coefficients 4 i + a ----
    double dt = 0.0;
    if (MODE != 0) dt = dtp[inst_of(msh, e)];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int ip = 4 * i + a;
        if (!live || ip >= NP) continue;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const size_t idx = (size_t)(c * NP + ip) * K + e;
            const double rhs = acc[c][i];
            double v;
            if (MODE == 0) {
                v = rhs;
            } else if (MODE == 1) {
                v = u[idx] + dt * rhs;
            } else if (MODE == 2) {
                v = 0.75 * __builtin_nontemporal_load(&un[idx]) + 0.25 * (u[idx] + dt * rhs);
            } else {
                v = (1.0 / 3.0) * __builtin_nontemporal_load(&un[idx]) + (2.0 / 3.0) * (u[idx] + dt * rhs);
            }
            __builtin_nontemporal_store(v, &out[idx]);
        }
    }
}

template <int EQ, int N, int MODE>
__global__ __launch_bounds__(256) void k_residual_lean(DevMesh msh, const double* __restrict__ u,
                                                       const double* __restrict__ un, double* __restrict__ out,
                                                       const double* __restrict__ dtp, double gamma,
                                                       uint32_t* __restrict__ cnt_reset) {
    residual_body_lean<EQ, N, MODE>(msh, u, un, out, dtp, gamma, cnt_reset);
}

template <int EQ, int N, int MODE>
__device__ __forceinline__ void residual_body_stream(DevMesh msh, const double* __restrict__ u,
                                                   const double* __restrict__ un,
                                                   double* __restrict__ out,
                                                   const double* __restrict__ dtp, double gamma,
                                                   uint32_t* __restrict__ cnt_reset) {
    using D = Dims<N>;
    constexpr int M = Phys<EQ>::M, NP = D::NP, NE = D::NE, NQ = D::NQ;
    const int K = msh.K;
    const int e = xcd_block(blockIdx.x, gridDim.x, msh.xcd_tiles) * blockDim.x + threadIdx.x;
    if (cnt_reset != nullptr && blockIdx.x == 0 && threadIdx.x < kListSegs) cnt_reset[threadIdx.x * kCountStride] = 0u;
    if (e >= K) return;
    const double ag = lf_global(msh, e);  // < 0: local Lax-Friedrichs
    const Tab<N>& T = tab<N>();

    // the element's coefficients are re-read (cache hits) in every phase
    // instead of staying live; the opaque copy of the pointer keeps the
    // compiler from reusing the first loads
    const double* __restrict__ us = u;
    double acc[M][NP];
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int n = 0; n < NP; ++n) acc[c][n] = 0.0;
    {
        const double x0 = msh.vx[e], x1 = msh.vx[K + e], x2 = msh.vx[2 * K + e];
        const double y0 = msh.vy[e], y1 = msh.vy[K + e], y2 = msh.vy[2 * K + e];
        const double xr = 0.5 * (x1 - x0), xs = 0.5 * (x2 - x0);
        const double yr = 0.5 * (y1 - y0), ys = 0.5 * (y2 - y0);
        const double iJ = 1.0 / (xr * ys - xs * yr);
        const double rx = ys * iJ, ry = -xs * iJ, sx = -yr * iJ, sy = xr * iJ;
        double U[M][NP];
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int n = 0; n < NP; ++n) U[c][n] = us[(size_t)(c * NP + n) * K + e];
#pragma unroll 3
        for (int q = 0; q < NQ; ++q) {
            double uq[M], F[M], G[M];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                double s = 0.0;
#pragma unroll
                for (int n = 0; n < NP; ++n) s += T.V[q][n] * U[c][n];
                uq[c] = s;
            }
            Phys<EQ>::flux(uq, gamma, F, G);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const double fr = rx * F[c] + ry * G[c];
                const double fs = sx * F[c] + sy * G[c];
#pragma unroll
                for (int i = 0; i < NP; ++i) acc[c][i] += T.wDr[q][i] * fr + T.wDs[q][i] * fs;
            }
        }
    }

    const uint32_t info4 = msh.info[e];
#pragma unroll 1
    for (int f = 0; f < 3; ++f) {
        const int f1 = (f == 2) ? 0 : f + 1;
        const double xa = msh.vx[f * K + e], ya = msh.vy[f * K + e];
        const double xb = msh.vx[f1 * K + e], yb = msh.vy[f1 * K + e];
        const double ex = xb - xa, ey = yb - ya;
        const double L = sqrt(ex * ex + ey * ey);
        const double iL = 1.0 / L;
        const double nx = ey * iL, ny = -ex * iL;
        // L_f / (2 J) with 2 J = area; recomputed from the vertices
        const double x0 = msh.vx[e], x1 = msh.vx[K + e], x2 = msh.vx[2 * K + e];
        const double y0 = msh.vy[e], y1 = msh.vy[K + e], y2 = msh.vy[2 * K + e];
        const double J = 0.25 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0));
        const double sf = 0.5 * L / J;
        const uint32_t inf = (info4 >> (8 * f)) & 0xffu;
        const bool bnd = (inf & 0x40u) != 0u;
        const int fp = bnd ? 0 : (int)(inf & 3u);
        const int nb = bnd ? e : msh.nbr[f * K + e];
        asm volatile("" : "+s"(us));
        double up[NE][M], umf[NE][M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
            double w[NP], wo[NP];
#pragma unroll
            for (int n = 0; n < NP; ++n) {
                w[n] = u[(size_t)(c * NP + n) * K + nb];
                wo[n] = us[(size_t)(c * NP + n) * K + e];
            }
#pragma unroll
            for (int g = 0; g < NE; ++g) {
                double s = 0.0, a = 0.0;
#pragma unroll
                for (int n = 0; n < NP; ++n) {
                    s += T.PF[fp][NE - 1 - g][n] * w[n];
                    a += T.PF[f][g][n] * wo[n];
                }
                up[g][c] = s;
                umf[g][c] = a;
            }
        }
#pragma unroll
        for (int g = 0; g < NE; ++g) {
            double um[M], upg[M];
#pragma unroll
            for (int c = 0; c < M; ++c) {
                um[c] = umf[g][c];
                upg[c] = bnd ? umf[g][c] : up[g][c];
            }
            if (bnd)
                boundary_trace<EQ>(um, upg, inf, nx, ny, msh.inflow, msh.shock, xa + tab<N>().es[g] * ex,
                                   ya + tab<N>().es[g] * ey, stage_time<MODE>(msh, e, dtp));
            double Fm[M], Fp[M], lm, lp;
            Phys<EQ>::normal_flux(um, nx, ny, gamma, Fm, lm);
            Phys<EQ>::normal_flux(upg, nx, ny, gamma, Fp, lp);
            const double alpha = (ag >= 0.0) ? ag : fmax(lm, lp);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const double Fs = 0.5 * (Fm[c] + Fp[c]) - 0.5 * alpha * (upg[c] - um[c]);
                const double sFs = sf * Fs;
#pragma unroll
                for (int i = 0; i < NP; ++i) acc[c][i] -= T.wPF[f][g][i] * sFs;
            }
        }
    }

    double dt = 0.0;
    if (MODE != 0) dt = dtp[inst_of(msh, e)];
    asm volatile("" : "+s"(us));
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const size_t idx = (size_t)(c * NP + i) * K + e;
            double v;
            if (MODE == 0) {
                v = acc[c][i];
            } else if (MODE == 1) {
                v = us[idx] + dt * acc[c][i];
            } else if (MODE == 2) {
                v = 0.75 * un[idx] + 0.25 * (us[idx] + dt * acc[c][i]);
            } else {
                v = (1.0 / 3.0) * un[idx] + (2.0 / 3.0) * (us[idx] + dt * acc[c][i]);
            }
            out[idx] = v;
        }
}

template <int EQ, int N, int MODE>
__global__ __launch_bounds__(256) void k_residual_stream(DevMesh msh, const double* __restrict__ u,
                                                         const double* __restrict__ un, double* __restrict__ out,
                                                         const double* __restrict__ dtp, double gamma,
                                                         uint32_t* __restrict__ cnt_reset) {
    residual_body_stream<EQ, N, MODE>(msh, u, un, out, dtp, gamma, cnt_reset);
}

// ---------------------------------------------------------------------------
// Time step: cell-mean wave speeds (block maxima, then one block)
// ---------------------------------------------------------------------------
template <int EQ, int N, typename S>
__global__ __launch_bounds__(256) void k_dt_partial(int K, const S* __restrict__ u,
                                                    double gamma, double* __restrict__ partial,
                                                    uint32_t* __restrict__ status) {
    constexpr int NP = Dims<N>::NP, M = Phys<EQ>::M;
    double amax = 0.0;
    uint32_t st = 0;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < K; e += gridDim.x * blockDim.x) {
        double ub[M];
#pragma unroll
        for (int c = 0; c < M; ++c) ub[c] = u[(size_t)(c * NP) * K + e] * kPsi0;
        double s;
        if constexpr (EQ == 0) {
            s = 1.41421356237309504880 * fabs(ub[0]);
        } else {
            double rho = ub[0], vx = ub[1] / rho, vy = ub[2] / rho;
            double p = (gamma - 1.0) * (ub[3] - 0.5 * rho * (vx * vx + vy * vy));
            if (!(rho > 0.0) || !(p > 0.0)) st |= CSWDG_STATUS_NEGATIVE;
            s = sqrt(vx * vx + vy * vy) + sqrt(gamma * p / rho);
        }
        if (!isfinite(s)) st |= CSWDG_STATUS_NONFINITE;
        amax = fmax(amax, s);
    }
    __shared__ double red[4];
    for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = red[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) b = fmax(b, red[i]);
        partial[blockIdx.x] = b;
    }
    if (st) atomicOr(status, st);
}

__global__ __launch_bounds__(256) void k_dt_final(int nblocks, const double* __restrict__ partial,
                                                  double cfl, double hmin, double* __restrict__ dt) {
    double a = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) a = fmax(a, partial[i]);
    for (int o = 32; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o));
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = red[0];
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) b = fmax(b, red[i]);
        *dt = cfl * hmin / b;
    }
}

// Per-instance time steps for a mesh holding several independent instances:
// wave maxima go to the instance's slot with an integer atomic max on the bit
// pattern (monotone for non-negative doubles); a wave spanning an instance
// boundary falls back to one atomic per lane. Non-finite speeds are skipped
// (and flagged), as fmax does in the single-mesh reduction.
template <int EQ, int N, typename S>
__global__ __launch_bounds__(256) void k_dt_inst(DevMesh msh, const S* __restrict__ u, double gamma,
                                                 unsigned long long* __restrict__ amax_bits,
                                                 uint32_t* __restrict__ status) {
    constexpr int NP = Dims<N>::NP, M = Phys<EQ>::M;
    const int K = msh.K;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    uint32_t st = 0;
    int ins = msh.n_inst - 1;
    if (e < K) {
        ins = inst_of(msh, e);
        double ub[M];
#pragma unroll
        for (int c = 0; c < M; ++c) ub[c] = u[(size_t)(c * NP) * K + e] * kPsi0;
        if constexpr (EQ == 0) {
            s = 1.41421356237309504880 * fabs(ub[0]);
        } else {
            double rho = ub[0], vx = ub[1] / rho, vy = ub[2] / rho;
            double p = (gamma - 1.0) * (ub[3] - 0.5 * rho * (vx * vx + vy * vy));
            if (!(rho > 0.0) || !(p > 0.0)) st |= CSWDG_STATUS_NEGATIVE;
            s = sqrt(vx * vx + vy * vy) + sqrt(gamma * p / rho);
        }
        if (!isfinite(s)) {
            st |= CSWDG_STATUS_NONFINITE;
            s = 0.0;
        }
    }
    const int i0 = __shfl(ins, 0);
    if (__ballot(ins != i0) == 0ull) {
        double a = s;
        for (int o = 32; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o));
        if ((threadIdx.x & 63) == 0 && a > 0.0) atomicMax(&amax_bits[i0], (unsigned long long)__double_as_longlong(a));
    } else if (s > 0.0) {
        atomicMax(&amax_bits[ins], (unsigned long long)__double_as_longlong(s));
    }
    if (st) atomicOr(status, st);
}

__global__ __launch_bounds__(256) void k_dt_inst_final(int n, unsigned long long* __restrict__ amax_bits,
                                                       double cfl, const double* __restrict__ hmin,
                                                       double* __restrict__ dt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = __longlong_as_double((long long)amax_bits[i]);
    dt[i] = cfl * hmin[i] / a;
    amax_bits[i] = 0ull;
}

// the global Lax-Friedrichs constant of each instance: its largest cell-mean
// wave speed (the reduction of k_dt_inst), left for the residual
__global__ __launch_bounds__(256) void k_lf_alpha_final(int n, unsigned long long* __restrict__ amax_bits,
                                                        double* __restrict__ alpha) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    alpha[i] = __longlong_as_double((long long)amax_bits[i]);
    amax_bits[i] = 0ull;
}

__global__ __launch_bounds__(64) void k_time_advance(int n, double* __restrict__ time,
                                                     const double* __restrict__ dt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) time[i] += dt[i];
}

// ---------------------------------------------------------------------------
// KXRCF indicator + compaction (Section 3.1)
// ---------------------------------------------------------------------------

template <int EQ, int N, typename S>
__global__ __launch_bounds__(256) void k_kxrcf(DevMesh msh, const S* __restrict__ u,
                                               uint8_t* __restrict__ flags, double* __restrict__ Rout,
                                               int32_t* __restrict__ list,
                                               uint32_t* __restrict__ count, double ck, int rms) {
    using D = Dims<N>;
    constexpr int NP = D::NP, NE = D::NE;
    const int K = msh.K;
    const int e = xcd_block(blockIdx.x, gridDim.x, msh.xcd_tiles) * blockDim.x + threadIdx.x;
    bool tr = false;
    // the face-point table in LDS (the neighbour's trace reads it at the
    // neighbour's own face: a per-lane index)
    __shared__ double sPF[3 * NE * NP];
    for (int i = threadIdx.x; i < 3 * NE * NP; i += blockDim.x) sPF[i] = (&tab<N>().PF[0][0][0])[i];
    __syncthreads();
    if (e < K) {
        const Tab<N>& T = tab<N>();
        double U0[NP], U1[NP], U2[NP];
#pragma unroll
        for (int n = 0; n < NP; ++n) {
            U0[n] = u[(size_t)n * K + e];
            if constexpr (EQ == 1) {
                U1[n] = u[(size_t)(NP + n) * K + e];
                U2[n] = u[(size_t)(2 * NP + n) * K + e];
            }
        }
        const double X[3] = {msh.vx[e], msh.vx[K + e], msh.vx[2 * K + e]};
        const double Y[3] = {msh.vy[e], msh.vy[K + e], msh.vy[2 * K + e]};
        const double J = 0.25 * ((X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]));
        const uint32_t info4 = msh.info[e];
        const double ts = (msh.shock != nullptr) ? msh.time[inst_of(msh, e)] : 0.0;
        double num = 0.0, len = 0.0, Ls[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const int f1 = (f + 1) % 3;
            const double ex = X[f1] - X[f], ey = Y[f1] - Y[f];
            const double L = sqrt(ex * ex + ey * ey);
            Ls[f] = L;
            const uint32_t inf = (info4 >> (8 * f)) & 0xffu;
            const bool bnd = (inf & 0x40u) != 0u;
            const int fp = bnd ? 0 : (int)(inf & 3u);
            const int nb = bnd ? e : msh.nbr[f * K + e];
            double Un[NP];
#pragma unroll
            for (int n = 0; n < NP; ++n) Un[n] = u[(size_t)n * K + nb];
#pragma unroll
            for (int g = 0; g < NE; ++g) {
                double um = 0.0, mu = 0.0, mv = 0.0, upv = 0.0;
#pragma unroll
                for (int n = 0; n < NP; ++n) {
                    um += T.PF[f][g][n] * U0[n];
                    if constexpr (EQ == 1) {
                        mu += T.PF[f][g][n] * U1[n];
                        mv += T.PF[f][g][n] * U2[n];
                    }
                    upv += sPF[(fp * NE + NE - 1 - g) * NP + n] * Un[n];
                }
                // inflow point: v.n < 0, tested as the sign of rho (rho v).(L n)
                // with L n = (ey, -ex) (L > 0, rho^2 > 0: the same points,
                // no division); Burgers: v = (u, u)
                double sn;
                if constexpr (EQ == 1) {
                    sn = (mu * ey - mv * ex) * um;
                } else {
                    sn = um * (ey - ex);
                }
                if (sn < 0.0) {
                    // boundary faces: the interior trace (outflow, wall), the
                    // inflow state's indicator variable (inflow), the moving
                    // shock's at the point and the step's start (moving shock)
                    double ub = ((inf & 3u) == 2u) ? msh.inflow[0] : um;
                    if ((inf & 3u) == 3u && msh.shock != nullptr)
                        ub = msh.shock[shock_state_at(msh.shock, X[f] + T.es[g] * ex, Y[f] + T.es[g] * ey, ts)];
                    const double up = bnd ? ub : upv;
                    const double ds = 0.5 * L * T.we[g];
                    num += ds * (um - up);
                    len += ds;
                }
            }
        }
        double ss = 0.0;
#pragma unroll
        for (int n = 0; n < NP; ++n) ss += U0[n] * U0[n];
        // literal L2 norm, or its RMS over the cell (int U^2 dA / (2 J))
        const double norm = rms ? sqrt(0.5 * ss) : sqrt(J * ss);
        const double h = Ls[0] * Ls[1] * Ls[2] / (4.0 * (2.0 * J));
        const double hp = (N == 1) ? h : ((N == 2) ? h * sqrt(h) : h * h);
        double R = 0.0;
        if (len > 0.0 && norm > 0.0) R = fabs(num) / (hp * len * norm);
        tr = R > ck;
        flags[e] = tr ? 1 : 0;
        if (Rout) Rout[e] = R;
    }
    append_list_block(tr, e, list, count, K, blockIdx.x & (kListSegs - 1));
}

// ---------------------------------------------------------------------------
// TVB minmod indicator (not in the paper; Cockburn and Shu's limiter for
// triangles used as a troubled-cell indicator) + compaction
// ---------------------------------------------------------------------------
// One thread per element.  For each face midpoint m_i and variable c: the
// deviation a = u_h(m_i) - ubar0 = sum_{n >= 1} u_n psi_n(m_i) and the
// neighbour-mean difference b = sum_f A[3 i + f] (ubar_f - ubar0) along the
// mesh's midpoint decomposition A (two nonnegative coefficients); the cell
// is troubled when some |a| exceeds max(M h^2, 1e-12 max_c |ubar0_c|) (h the
// circumradius) without a b > 0 and |a| <= 1.5 |b|.  Across a boundary face
// the neighbour mean is the ghost's: ubar0 (outflow), ubar0 with its normal
// momentum reversed (wall), the inflow state, or the moving shock's state
// at the face midpoint and the step's start.
template <int EQ, int N, typename S>
__global__ __launch_bounds__(256) void k_tvb(DevMesh msh, const S* __restrict__ u,
                                             uint8_t* __restrict__ flags, double* __restrict__ Rout,
                                             int32_t* __restrict__ list, uint32_t* __restrict__ count,
                                             double tvb_m) {
    constexpr int M = Phys<EQ>::M, NP = Dims<N>::NP;
    const int K = msh.K;
    const int e = xcd_block(blockIdx.x, gridDim.x, msh.xcd_tiles) * blockDim.x + threadIdx.x;
    bool tr = false;
    if (e < K) {
        const Tab<N>& T = tab<N>();
        double ub0[M], db[3][M];
        double smax = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            ub0[c] = (double)u[(size_t)(c * NP) * K + e] * kPsi0;
            smax = fmax(smax, fabs(ub0[c]));
        }
        const double X[3] = {msh.vx[e], msh.vx[K + e], msh.vx[2 * K + e]};
        const double Y[3] = {msh.vy[e], msh.vy[K + e], msh.vy[2 * K + e]};
        const uint32_t info4 = msh.info[e];
        double Ls[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const int f1 = (f + 1) % 3;
            const double ex = X[f1] - X[f], ey = Y[f1] - Y[f];
            Ls[f] = sqrt(ex * ex + ey * ey);
            const uint32_t inf = (info4 >> (8 * f)) & 0xffu;
            const bool bnd = (inf & 0x40u) != 0u;
            const uint32_t kind = inf & 3u;
            double g[M];
            if (!bnd) {
                const int nb = msh.nbr[f * K + e];
#pragma unroll
                for (int c = 0; c < M; ++c) g[c] = (double)u[(size_t)(c * NP) * K + nb] * kPsi0;
            } else {
#pragma unroll
                for (int c = 0; c < M; ++c) g[c] = ub0[c];
                if constexpr (EQ == 1) {
                    if (kind == 1u) {
                        const double nx = ey / Ls[f], ny = -ex / Ls[f];
                        const double mn = ub0[1] * nx + ub0[2] * ny;
                        g[1] = ub0[1] - 2.0 * mn * nx;
                        g[2] = ub0[2] - 2.0 * mn * ny;
                    }
                }
                if (kind == 2u) {
#pragma unroll
                    for (int c = 0; c < M; ++c) g[c] = msh.inflow[c];
                } else if (kind == 3u && msh.shock != nullptr) {
                    const double xm = 0.5 * (X[f] + X[f1]), ym = 0.5 * (Y[f] + Y[f1]);
                    const int o = shock_state_at(msh.shock, xm, ym, msh.time[inst_of(msh, e)]);
#pragma unroll
                    for (int c = 0; c < M; ++c) g[c] = msh.shock[o + c];
                }
            }
#pragma unroll
            for (int c = 0; c < M; ++c) db[f][c] = g[c] - ub0[c];
        }
        double A[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int f = 0; f < 3; ++f) A[i][f] = msh.tvb[(size_t)(3 * i + f) * K + e];
        const double J2 = (X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]);
        const double h = Ls[0] * Ls[1] * Ls[2] / (2.0 * J2);
        const double thr = fmax(tvb_m * h * h, 1e-12 * smax);
        double rmax = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) {
            double U[NP];
#pragma unroll
            for (int n = 1; n < NP; ++n) U[n] = (double)u[(size_t)(c * NP + n) * K + e];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                double a = 0.0;
#pragma unroll
                for (int n = 1; n < NP; ++n) a += T.PMID[i][n] * U[n];
                const double b = A[i][0] * db[0][c] + A[i][1] * db[1][c] + A[i][2] * db[2][c];
                const double aa = fabs(a);
                const bool same = a * b > 0.0;
                const bool keep = (aa <= thr) || (same && aa <= 1.5 * fabs(b));
                tr = tr || !keep;
                // the ratio of the deviation to the largest one the minmod
                // leaves alone (> 1 exactly for the deviations it changes)
                if (Rout != nullptr && aa > thr) rmax = fmax(rmax, aa / fmax(thr, same ? 1.5 * fabs(b) : 0.0));
            }
        }
        flags[e] = tr ? 1 : 0;
        if (Rout) Rout[e] = rmax;
    }
    append_list_block(tr, e, list, count, K, blockIdx.x & (kListSegs - 1));
}

__global__ __launch_bounds__(256) void k_compact_mask(int K, const uint8_t* __restrict__ mask,
                                                      uint8_t* __restrict__ flags,
                                                      int32_t* __restrict__ list,
                                                      uint32_t* __restrict__ count) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    bool tr = false;
    if (e < K) {
        tr = mask ? (mask[e] != 0) : true;
        if (flags) flags[e] = tr ? 1 : 0;
    }
    append_list_block(tr, e, list, count, K, blockIdx.x & (kListSegs - 1));
}

__global__ void k_zero_u32(uint32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// CSWENO limiter (Section 3.2)
// ---------------------------------------------------------------------------
// waves per SIMD the limiter is compiled for: four for the three-member
// hierarchies (no spills beyond a few bytes), two for a fourth member on T4
// (its quartic least-squares level needs more registers)
template <int N, int QTOP>
struct LimWaves {
    static constexpr int value = OpLayout<N, QTOP>::SEXT ? 1 : (OpLayout<N, QTOP>::FOUR ? 2 : 4);
};

template <int EQ, int N, typename S, int QTOP, bool BLIT>
__global__ __launch_bounds__(64, (LimWaves<N, QTOP>::value)) void k_limiter(DevMesh msh, const S* __restrict__ u,
                                                const double* __restrict__ ops,
                                                const int32_t* __restrict__ list,
                                                const uint32_t* __restrict__ count,
                                                double* __restrict__ compact,
                                                uint32_t* __restrict__ status, double gamma,
                                                double eps, int comp, int lin) {
    using D = Dims<N>;
    using LO = OpLayout<N, QTOP>;
    constexpr int M = Phys<EQ>::M, NP = D::NP, NPC = LO::NPC, NM = LO::NM;
    constexpr int ND = LimLanes<EQ>::ND, LPC = LimLanes<EQ>::LPC;
    constexpr int CPB = 64 / LPC;  // cells per block
    const int K = msh.K;
    uint32_t pre[kListSegs + 1];
    seg_prefix(count, K, pre);
    const uint32_t ncell = pre[kListSegs];
    const int j = threadIdx.x % LPC;  // lane within the cell
    const int d = j / M;              // characteristic direction
    const int k = j % M;              // characteristic field
    for (uint32_t base = blockIdx.x * CPB; base < ncell; base += gridDim.x * CPB) {
        const uint32_t t = base + threadIdx.x / LPC;
        const bool active = t < ncell;
        const int e = active ? seg_elem(list, pre, K, t) : 0;
        const double* __restrict__ op = ops + (size_t)e * LO::LEN;
        const bool valid = active && op[LO::VALID] != 0.0;

        double ub0[M];
#pragma unroll
        for (int c = 0; c < M; ++c) ub0[c] = u[(size_t)(c * NP) * K + e] * kPsi0;
        // row k of L_d and column k of R_d at the mean of Delta0
        double Lr[M], Rc[M];
        if constexpr (EQ == 1) {
            double Lm[4][4], Rm[4][4];
            euler_eigen(ub0, d == 0 ? 1.0 : 0.0, d == 0 ? 0.0 : 1.0, gamma, Lm, Rm);
            if (comp) {
                // conserved variables: both "directions" use the identity
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) Lm[a][b] = Rm[a][b] = (a == b) ? 1.0 : 0.0;
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double a = Lm[0][c], b = Rm[c][0];
#pragma unroll
                for (int kk = 1; kk < 4; ++kk) {
                    a = (k == kk) ? Lm[kk][c] : a;
                    b = (k == kk) ? Rm[c][kk] : b;
                }
                Lr[c] = a;
                Rc[c] = b;
            }
        } else {
            Lr[0] = 1.0;
            Rc[0] = 1.0;
        }
        double w0 = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) w0 += Lr[c] * ub0[c];

        // field-k averages over the pieces of the three neighbours
        const uint32_t info4 = msh.info[e];
        double w[3][NPC];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const uint32_t inf = (info4 >> (8 * f)) & 0xffu;
            const bool bnd = (inf & 0x40u) != 0u;
            const uint32_t kind = bnd ? (inf & 3u) : 0u;
            const int src = bnd ? e : msh.nbr[f * K + e];
            // row of the field for this face's source: a wall's mirror ghost
            // carries the reflected momentum, so its averages map through the
            // reflection (row Lr times the symmetric reflection matrix)
            double Lf[M];
#pragma unroll
            for (int c = 0; c < M; ++c) Lf[c] = Lr[c];
            if constexpr (EQ == 1) {
                if (kind == 1u) {
                    const int f1 = (f == 2) ? 0 : f + 1;
                    const double ex = msh.vx[f1 * K + e] - msh.vx[f * K + e];
                    const double ey = msh.vy[f1 * K + e] - msh.vy[f * K + e];
                    const double iL = 1.0 / sqrt(ex * ex + ey * ey);
                    const double nx = ey * iL, ny = -ex * iL;
                    Lf[1] = Lr[1] * (1.0 - 2.0 * nx * nx) - Lr[2] * (2.0 * nx * ny);
                    Lf[2] = -Lr[1] * (2.0 * nx * ny) + Lr[2] * (1.0 - 2.0 * ny * ny);
                }
            }
            if (kind == 2u || kind == 3u) {
                // inflow ghost: the prescribed state on every piece; moving
                // shock: its state at the face midpoint and the step's start
                const double* st = msh.inflow;
                if (kind == 3u) {
                    const int f1 = (f == 2) ? 0 : f + 1;
                    const double xm = 0.5 * (msh.vx[f * K + e] + msh.vx[f1 * K + e]);
                    const double ym = 0.5 * (msh.vy[f * K + e] + msh.vy[f1 * K + e]);
                    st = msh.shock + shock_state_at(msh.shock, xm, ym, msh.time[inst_of(msh, e)]);
                }
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < M; ++c) s += Lr[c] * st[c];
#pragma unroll
                for (int p = 0; p < NPC; ++p) w[f][p] = s;
                continue;
            }
            double ws[NP];
#pragma unroll
            for (int n = 0; n < NP; ++n) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < M; ++c) s += Lf[c] * u[(size_t)(c * NP + n) * K + src];
                ws[n] = s;
            }
#pragma unroll
            for (int p = 0; p < NPC; ++p) {
                const double* a = op + LO::AVG + (f * NPC + p) * NP;
                double s = 0.0;
#pragma unroll
                for (int n = 0; n < NP; ++n) s += a[n] * ws[n];
                w[f][p] = s;
            }
        }
        // Step 1: least-squares levels (pseudo-inverses applied to
        // piece average - mean of Delta0)
        constexpr bool quartic = LO::FOUR;  // a fourth member on T4
        constexpr int NT = LO::NT > 0 ? LO::NT : 1;
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
        // the top level on T4 for N >= 2 (QTOP = kTopQuadratic: the
        // hierarchy of N = 1); the cubic readings fit 9 monomials, the
        // quartic 14; the sextic (N = 3) 27 on the ten T5 pieces
        if constexpr (quartic) {
            constexpr int pl[5] = {0, 3, 4, 5, 6};
            constexpr int NK = LO::NROW / 3;
#pragma unroll
            for (int jj = 0; jj < NT; ++jj) {
                double s = 0.0;
#pragma unroll
                for (int kk = 0; kk < NK; ++kk)
#pragma unroll
                    for (int f = 0; f < 3; ++f)
                        s += op[LO::X5 + jj * LO::NROW + kk * 3 + f] * (w[f][LO::SEXT ? 7 + kk : pl[kk]] - w0);
                c5[jj] = s;
            }
        }
        // Step 3: smoothness indicators of q_2, q_3 (and the top level), or
        // (BLIT) of the equivalent polynomials p_2, p_3, p_top over derivative
        // orders 1..N (eq. smoothnessIndicator as printed)
        double beta[4];
        if constexpr (!BLIT) {
            const double* bp = op + LO::BP;
            beta[1] = quad_form<NM, 2>(bp, c2);
            beta[2] = quad_form<NM, 5>(bp, c3);
            beta[3] = quartic ? quad_form<NM, NT>(bp, c5) : 0.0;
        } else {
            const double* bpl = op + LO::BPL;
            const double ih = op[LO::GBASE];
            const double s2 = 1.0 + ih, s3 = 1.0 + ih + ih * ih;
            const double g22 = ih / s2, g23 = ih / s3, g33 = ih * ih / s3;
            double p2[2], p3[5], pt[NT];
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) p2[jj] = c2[jj] / g22;
#pragma unroll
            for (int jj = 0; jj < 5; ++jj) p3[jj] = (c3[jj] - (jj < 2 ? g23 * p2[jj] : 0.0)) / g33;
            beta[1] = quad_form<NM, 2>(bpl, p2);
            beta[2] = quad_form<NM, 5>(bpl, p3);
            beta[3] = 0.0;
            if constexpr (quartic) {
                if constexpr (QTOP == kTopCubic) {
                    // eq. equivalentOrder3: p_4 = (q_4 - g24 p_2) / g34, weights gamma_{.,4} = gamma_{.,3}
#pragma unroll
                    for (int jj = 0; jj < NT; ++jj) pt[jj] = (c5[jj] - (jj < 2 ? g23 * p2[jj] : 0.0)) / g33;
                } else {
                    const double s5 = 1.0 + ih + ih * ih + ih * ih * ih;
                    const double g25 = ih / s5, g35 = ih * ih / s5, g45 = ih * ih * ih / s5;
#pragma unroll
                    for (int jj = 0; jj < NT; ++jj)
                        pt[jj] = (c5[jj] - (jj < 2 ? g25 * p2[jj] : 0.0) - (jj < 5 ? g35 * p3[jj] : 0.0)) / g45;
                }
                beta[3] = quad_form<NM, NT>(bpl, pt);
            }
        }
        const double area0 = op[LO::AREA0];
        {
            double gx[3], gy[3], b1[3];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                const double* mi = op + LO::MINV + 4 * f;
                const double d0 = w[f][1] - w[f][0], d1 = w[f][2] - w[f][0];
                gx[f] = mi[0] * d0 + mi[1] * d1;
                gy[f] = mi[2] * d0 + mi[3] * d1;
                b1[f] = area0 * (gx[f] * gx[f] + gy[f] * gy[f]);
            }
            const double a01 = fabs(b1[0] - b1[1]), a12 = fabs(b1[1] - b1[2]), a20 = fabs(b1[2] - b1[0]);
            const double mm = (a01 * a01 + a12 * a12 + a20 * a20) / 3.0;
            const double num = mm * mm;
            double sg[3], ssum = 0.0;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                sg[f] = (1.0 / 3.0) * (1.0 + num / (b1[f] + eps));
                ssum += sg[f];
            }
            double mx = 0.0, my = 0.0;
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                mx += (sg[f] / ssum) * gx[f];
                my += (sg[f] / ssum) * gy[f];
            }
            beta[0] = area0 * (mx * mx + my * my);
        }
        // Steps 2 and 4: linear weights gamma_{l,t} = b^{l-1} / sum with
        // b = 1/h (or the constant b = 10 of the reference cited there; the
        // operator record holds b), WENO-Z weights, R = sum_l omega_l p_l
        // written on c2, c3, c5
        const double ih = op[LO::GBASE];
        double A2, A3, A5;
        {
            const double s2 = 1.0 + ih, s3 = 1.0 + ih + ih * ih;
            const double g22 = ih / s2;
            const double g23 = ih / s3, g33 = ih * ih / s3;
            if constexpr (!quartic) {
                const double g13 = 1.0 / s3;
                const double d31 = fabs(beta[2] - beta[0]), d32 = fabs(beta[2] - beta[1]);
                // tau = 0 gives the linear weights (omega = gamma)
                const double tau = lin ? 0.0 : (d31 * d31 + d32 * d32) / 4.0;
                const double o1 = g13 * (1.0 + tau / (eps + beta[0]));
                const double o2 = g23 * (1.0 + tau / (eps + beta[1]));
                const double o3 = g33 * (1.0 + tau / (eps + beta[2]));
                const double os = o1 + o2 + o3;
                const double w2 = o2 / os, w3 = o3 / os;
                // p2 = c2/g22, p3 = (c3 - g23 p2)/g33
                A3 = w3 / g33;
                A2 = w2 / g22 - A3 * g23 / g22;
                A5 = 0.0;
            } else {
                const double s5 = 1.0 + ih + ih * ih + ih * ih * ih;
                const double g15 = 1.0 / s5, g25 = ih / s5, g35 = ih * ih / s5, g45 = ih * ih * ih / s5;
                const double d1 = fabs(beta[3] - beta[0]), d2 = fabs(beta[3] - beta[1]), d3 = fabs(beta[3] - beta[2]);
                const double tau = lin ? 0.0 : (d1 * d1 + d2 * d2 + d3 * d3) / 16.0;
                const double o1 = g15 * (1.0 + tau / (eps + beta[0]));
                const double o2 = g25 * (1.0 + tau / (eps + beta[1]));
                const double o3 = g35 * (1.0 + tau / (eps + beta[2]));
                const double o4 = g45 * (1.0 + tau / (eps + beta[3]));
                const double os = o1 + o2 + o3 + o4;
                const double w2 = o2 / os, w3 = o3 / os, w4 = o4 / os;
                if constexpr (QTOP == kTopCubic) {
                    // eq. equivalentOrder3: p4 = (c4 - g24 p2)/g34 with the
                    // three weights gamma_{.,4} (equal to gamma_{.,3})
                    A5 = w4 / g33;
                    A3 = w3 / g33;
                    A2 = (w2 - (w3 + w4) * (g23 / g33)) / g22;
                } else {
                    // p4 = (c5 - g25 p2 - g35 p3)/g45; collect the factors of c5, c3, c2
                    A5 = w4 / g45;
                    const double P3 = w3 - A5 * g35;  // factor of p3
                    A3 = P3 / g33;
                    const double P2 = w2 - A5 * g25 - A3 * g23;  // factor of p2
                    A2 = P2 / g22;
                }
            }
        }
        // Step 5: projection of R onto psi_1..psi_{Np-1}
        double mom[NP - 1];
#pragma unroll
        for (int i = 0; i < NP - 1; ++i) {
            const double* pm = op + LO::PM + i * NM;
            double s = 0.0;
#pragma unroll
            for (int jj = 0; jj < NM; ++jj) {
                double r = 0.0;
                if constexpr (quartic) {
                    if (jj < NT) r = A5 * c5[jj];
                }
                if (jj < 5) r += A3 * c3[jj];
                if (jj < 2) r += A2 * c2[jj];
                s += pm[jj] * r;
            }
            mom[i] = s;
        }
        // back to conserved variables: sum over (d, k) of R_d[c][k] mom_dk / ND
        double res[M][NP - 1];
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int i = 0; i < NP - 1; ++i) res[c][i] = (1.0 / ND) * Rc[c] * mom[i];
#pragma unroll
        for (int o = 1; o < LPC; o <<= 1)
#pragma unroll
            for (int c = 0; c < M; ++c)
#pragma unroll
                for (int i = 0; i < NP - 1; ++i) res[c][i] += __shfl_xor(res[c][i], o, LPC);
        if (active && j < M) {
            double* outp = compact + (size_t)t * (M * NP) + j * NP;
            double sel[NP - 1];
#pragma unroll
            for (int i = 0; i < NP - 1; ++i) {
                double v = res[0][i];
#pragma unroll
                for (int c = 1; c < M; ++c) v = (j == c) ? res[c][i] : v;
                sel[i] = v;
            }
            outp[0] = u[(size_t)(j * NP) * K + e];
            if (valid) {
#pragma unroll
                for (int i = 1; i < NP; ++i) outp[i] = sel[i - 1];
            } else {
#pragma unroll
                for (int i = 1; i < NP; ++i) outp[i] = u[(size_t)(j * NP + i) * K + e];
            }
        }
        if (active && !valid && j == 0) atomicOr(status, CSWDG_STATUS_RANK);
    }
}

// Type-I WENO on the same subcell stencils (params.reconstruction = 1; N =
// 1, 2): the lanes, the characteristic fields and the piece averages as in
// k_limiter; then degree-N least-squares fits on the central stencil (the
// nine centroid subcells) and the three sectors (faces k, k+1), the
// smoothness indicators of the four fits, weights lambda_k / (1e-14 +
// beta_k)^4 (lambda 1e5 central, 1 sectors), R = sum_k omega_k q_k, and its
// projection.
template <int EQ, int N, typename S>
__global__ __launch_bounds__(64, 3) void k_limiter_t1(DevMesh msh, const S* __restrict__ u,
                                                const double* __restrict__ ops,
                                                const int32_t* __restrict__ list,
                                                const uint32_t* __restrict__ count,
                                                double* __restrict__ compact,
                                                uint32_t* __restrict__ status, double gamma,
                                                double eps, int comp) {
    using D = Dims<N>;
    using LO = OpLayoutT1<N>;
    constexpr int M = Phys<EQ>::M, NP = D::NP, NPC = 3, NM = LO::NM;
    constexpr int ND = LimLanes<EQ>::ND, LPC = LimLanes<EQ>::LPC;
    constexpr int CPB = 64 / LPC;  // cells per block
    const int K = msh.K;
    uint32_t pre[kListSegs + 1];
    seg_prefix(count, K, pre);
    const uint32_t ncell = pre[kListSegs];
    const int j = threadIdx.x % LPC;  // lane within the cell
    const int d = j / M;              // characteristic direction
    const int k = j % M;              // characteristic field
    for (uint32_t base = blockIdx.x * CPB; base < ncell; base += gridDim.x * CPB) {
        const uint32_t t = base + threadIdx.x / LPC;
        const bool active = t < ncell;
        const int e = active ? seg_elem(list, pre, K, t) : 0;
        const double* __restrict__ op = ops + (size_t)e * LO::LEN;
        const bool valid = active && op[LO::VALID] != 0.0;

        double ub0[M];
#pragma unroll
        for (int c = 0; c < M; ++c) ub0[c] = u[(size_t)(c * NP) * K + e] * kPsi0;
        // row k of L_d and column k of R_d at the mean of Delta0
        double Lr[M], Rc[M];
        if constexpr (EQ == 1) {
            double Lm[4][4], Rm[4][4];
            euler_eigen(ub0, d == 0 ? 1.0 : 0.0, d == 0 ? 0.0 : 1.0, gamma, Lm, Rm);
            if (comp) {
                // conserved variables: both "directions" use the identity
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) Lm[a][b] = Rm[a][b] = (a == b) ? 1.0 : 0.0;
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double a = Lm[0][c], b = Rm[c][0];
#pragma unroll
                for (int kk = 1; kk < 4; ++kk) {
                    a = (k == kk) ? Lm[kk][c] : a;
                    b = (k == kk) ? Rm[c][kk] : b;
                }
                Lr[c] = a;
                Rc[c] = b;
            }
        } else {
            Lr[0] = 1.0;
            Rc[0] = 1.0;
        }
        double w0 = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) w0 += Lr[c] * ub0[c];

        // field-k averages over the pieces of the three neighbours
        const uint32_t info4 = msh.info[e];
        double w[3][NPC];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const uint32_t inf = (info4 >> (8 * f)) & 0xffu;
            const bool bnd = (inf & 0x40u) != 0u;
            const uint32_t kind = bnd ? (inf & 3u) : 0u;
            const int src = bnd ? e : msh.nbr[f * K + e];
            // row of the field for this face's source: a wall's mirror ghost
            // carries the reflected momentum, so its averages map through the
            // reflection (row Lr times the symmetric reflection matrix)
            double Lf[M];
#pragma unroll
            for (int c = 0; c < M; ++c) Lf[c] = Lr[c];
            if constexpr (EQ == 1) {
                if (kind == 1u) {
                    const int f1 = (f == 2) ? 0 : f + 1;
                    const double ex = msh.vx[f1 * K + e] - msh.vx[f * K + e];
                    const double ey = msh.vy[f1 * K + e] - msh.vy[f * K + e];
                    const double iL = 1.0 / sqrt(ex * ex + ey * ey);
                    const double nx = ey * iL, ny = -ex * iL;
                    Lf[1] = Lr[1] * (1.0 - 2.0 * nx * nx) - Lr[2] * (2.0 * nx * ny);
                    Lf[2] = -Lr[1] * (2.0 * nx * ny) + Lr[2] * (1.0 - 2.0 * ny * ny);
                }
            }
            if (kind == 2u || kind == 3u) {
                // inflow ghost: the prescribed state on every piece; moving
                // shock: its state at the face midpoint and the step's start
                const double* st = msh.inflow;
                if (kind == 3u) {
                    const int f1 = (f == 2) ? 0 : f + 1;
                    const double xm = 0.5 * (msh.vx[f * K + e] + msh.vx[f1 * K + e]);
                    const double ym = 0.5 * (msh.vy[f * K + e] + msh.vy[f1 * K + e]);
                    st = msh.shock + shock_state_at(msh.shock, xm, ym, msh.time[inst_of(msh, e)]);
                }
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < M; ++c) s += Lr[c] * st[c];
#pragma unroll
                for (int p = 0; p < NPC; ++p) w[f][p] = s;
                continue;
            }
            double ws[NP];
#pragma unroll
            for (int n = 0; n < NP; ++n) {
                double s = 0.0;
#pragma unroll
                for (int c = 0; c < M; ++c) s += Lf[c] * u[(size_t)(c * NP + n) * K + src];
                ws[n] = s;
            }
#pragma unroll
            for (int p = 0; p < NPC; ++p) {
                const double* a = op + LO::AVG + (f * NPC + p) * NP;
                double s = 0.0;
#pragma unroll
                for (int n = 0; n < NP; ++n) s += a[n] * ws[n];
                w[f][p] = s;
            }
        }
        // degree-N fits: the central stencil (rows piece-major, then face)
        // and the sectors (faces k, k+1; rows piece-major, then the two)
        double cq[4][NM];
#pragma unroll
        for (int jj = 0; jj < NM; ++jj) {
            double s = 0.0;
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int f = 0; f < 3; ++f) s += op[LO::XC + jj * 9 + p * 3 + f] * (w[f][p] - w0);
            cq[0][jj] = s;
        }
#pragma unroll
        for (int sk = 0; sk < 3; ++sk) {
            const int fa = sk, fb = (sk == 2) ? 0 : sk + 1;
#pragma unroll
            for (int jj = 0; jj < NM; ++jj) {
                const double* x = op + LO::XS + (sk * NM + jj) * 6;
                double s = 0.0;
#pragma unroll
                for (int p = 0; p < 3; ++p) s += x[p * 2] * (w[fa][p] - w0) + x[p * 2 + 1] * (w[fb][p] - w0);
                cq[1 + sk][jj] = s;
            }
        }
        // smoothness indicators and weights
        const double* bp = op + LO::BP;
        double om[4], osum = 0.0;
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const double b = quad_form<NM, NM>(bp, cq[st]);
            const double tb = 1e-14 + b, t2 = tb * tb;
            om[st] = (st == 0 ? 1e5 : 1.0) / (t2 * t2);
            osum += om[st];
        }
        // Step 5: projection of R = sum_k omega_k q_k onto psi_1..psi_{Np-1}
        double Rq[NM];
#pragma unroll
        for (int jj = 0; jj < NM; ++jj) {
            double r = 0.0;
#pragma unroll
            for (int st = 0; st < 4; ++st) r += (om[st] / osum) * cq[st][jj];
            Rq[jj] = r;
        }
        double mom[NP - 1];
#pragma unroll
        for (int i = 0; i < NP - 1; ++i) {
            const double* pm = op + LO::PM + i * NM;
            double s = 0.0;
#pragma unroll
            for (int jj = 0; jj < NM; ++jj) s += pm[jj] * Rq[jj];
            mom[i] = s;
        }
        // back to conserved variables: sum over (d, k) of R_d[c][k] mom_dk / ND
        double res[M][NP - 1];
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int i = 0; i < NP - 1; ++i) res[c][i] = (1.0 / ND) * Rc[c] * mom[i];
#pragma unroll
        for (int o = 1; o < LPC; o <<= 1)
#pragma unroll
            for (int c = 0; c < M; ++c)
#pragma unroll
                for (int i = 0; i < NP - 1; ++i) res[c][i] += __shfl_xor(res[c][i], o, LPC);
        if (active && j < M) {
            double* outp = compact + (size_t)t * (M * NP) + j * NP;
            double sel[NP - 1];
#pragma unroll
            for (int i = 0; i < NP - 1; ++i) {
                double v = res[0][i];
#pragma unroll
                for (int c = 1; c < M; ++c) v = (j == c) ? res[c][i] : v;
                sel[i] = v;
            }
            outp[0] = u[(size_t)(j * NP) * K + e];
            if (valid) {
#pragma unroll
                for (int i = 1; i < NP; ++i) outp[i] = sel[i - 1];
            } else {
#pragma unroll
                for (int i = 1; i < NP; ++i) outp[i] = u[(size_t)(j * NP + i) * K + e];
            }
        }
        if (active && !valid && j == 0) atomicOr(status, CSWDG_STATUS_RANK);
    }
}

// What the type-II and the mixed reconstructions share (N = 2), for the
// lane (direction d, field k) of troubled cell e: column k of R_d at the
// mean of Delta0 (Rc), the field's mean w0 on Delta0, its averages w over
// the three pieces of each neighbour (boundary ghosts included) and the six
// linear least-squares fits cl on the single-neighbour stencils (rows: the
// three pieces) and on the sectors (faces k, k+1; rows piece-major, then the
// two faces); the lanes and the characteristic fields as in k_limiter.
template <int EQ, typename S, class LO>
__device__ __forceinline__ void small_stencil_fits(const DevMesh& msh, const S* __restrict__ u,
                                                   const double* __restrict__ op, int e, int d, int k,
                                                   double gamma, int comp, double (&Rc)[Phys<EQ>::M],
                                                   double& w0, double (&w)[3][3], double (&cl)[6][2]) {
    constexpr int M = Phys<EQ>::M, NP = 6, NPC = 3;
    const int K = msh.K;
    double ub0[M];
#pragma unroll
    for (int c = 0; c < M; ++c) ub0[c] = u[(size_t)(c * NP) * K + e] * kPsi0;
    // row k of L_d and column k of R_d at the mean of Delta0
    double Lr[M];
    if constexpr (EQ == 1) {
        double Lm[4][4], Rm[4][4];
        euler_eigen(ub0, d == 0 ? 1.0 : 0.0, d == 0 ? 0.0 : 1.0, gamma, Lm, Rm);
        if (comp) {
            // conserved variables: both "directions" use the identity
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) Lm[a][b] = Rm[a][b] = (a == b) ? 1.0 : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double a = Lm[0][c], b = Rm[c][0];
#pragma unroll
            for (int kk = 1; kk < 4; ++kk) {
                a = (k == kk) ? Lm[kk][c] : a;
                b = (k == kk) ? Rm[c][kk] : b;
            }
            Lr[c] = a;
            Rc[c] = b;
        }
    } else {
        Lr[0] = 1.0;
        Rc[0] = 1.0;
    }
    w0 = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) w0 += Lr[c] * ub0[c];

    // field-k averages over the pieces of the three neighbours
    const uint32_t info4 = msh.info[e];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const uint32_t inf = (info4 >> (8 * f)) & 0xffu;
        const bool bnd = (inf & 0x40u) != 0u;
        const uint32_t kind = bnd ? (inf & 3u) : 0u;
        const int src = bnd ? e : msh.nbr[f * K + e];
        // row of the field for this face's source: a wall's mirror ghost
        // carries the reflected momentum, so its averages map through the
        // reflection (row Lr times the symmetric reflection matrix)
        double Lf[M];
#pragma unroll
        for (int c = 0; c < M; ++c) Lf[c] = Lr[c];
        if constexpr (EQ == 1) {
            if (kind == 1u) {
                const int f1 = (f == 2) ? 0 : f + 1;
                const double ex = msh.vx[f1 * K + e] - msh.vx[f * K + e];
                const double ey = msh.vy[f1 * K + e] - msh.vy[f * K + e];
                const double iL = 1.0 / sqrt(ex * ex + ey * ey);
                const double nx = ey * iL, ny = -ex * iL;
                Lf[1] = Lr[1] * (1.0 - 2.0 * nx * nx) - Lr[2] * (2.0 * nx * ny);
                Lf[2] = -Lr[1] * (2.0 * nx * ny) + Lr[2] * (1.0 - 2.0 * ny * ny);
            }
        }
        if (kind == 2u || kind == 3u) {
            // inflow ghost: the prescribed state on every piece; moving
            // shock: its state at the face midpoint and the step's start
            const double* st = msh.inflow;
            if (kind == 3u) {
                const int f1 = (f == 2) ? 0 : f + 1;
                const double xm = 0.5 * (msh.vx[f * K + e] + msh.vx[f1 * K + e]);
                const double ym = 0.5 * (msh.vy[f * K + e] + msh.vy[f1 * K + e]);
                st = msh.shock + shock_state_at(msh.shock, xm, ym, msh.time[inst_of(msh, e)]);
            }
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) s += Lr[c] * st[c];
#pragma unroll
            for (int p = 0; p < NPC; ++p) w[f][p] = s;
            continue;
        }
        double ws[NP];
#pragma unroll
        for (int n = 0; n < NP; ++n) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < M; ++c) s += Lf[c] * u[(size_t)(c * NP + n) * K + src];
            ws[n] = s;
        }
#pragma unroll
        for (int p = 0; p < NPC; ++p) {
            const double* a = op + LO::AVG + (f * NPC + p) * NP;
            double s = 0.0;
#pragma unroll
            for (int n = 0; n < NP; ++n) s += a[n] * ws[n];
            w[f][p] = s;
        }
    }
    // linear fits on the single-neighbour stencils (rows: the three
    // pieces) and on the sectors (faces k, k+1; rows piece-major, then
    // the two faces)
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            double s = 0.0;
#pragma unroll
            for (int p = 0; p < 3; ++p) s += op[LO::XF + (f * 2 + jj) * 3 + p] * (w[f][p] - w0);
            cl[f][jj] = s;
        }
#pragma unroll
    for (int sk = 0; sk < 3; ++sk) {
        const int fa = sk, fb = (sk == 2) ? 0 : sk + 1;
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const double* x = op + LO::XS + (sk * 2 + jj) * 6;
            double s = 0.0;
#pragma unroll
            for (int p = 0; p < 3; ++p) s += x[p * 2] * (w[fa][p] - w0) + x[p * 2 + 1] * (w[fb][p] - w0);
            cl[3 + sk][jj] = s;
        }
    }
}

// The limited moments of one lane back to conserved variables (the sum over
// the cell's lanes of R_d[c][k] mom_dk / ND) and the store of the cell's
// compact row: the mean copied, the new moments where the record is valid,
// the old ones (and the rank status bit) where it is not.
template <int EQ, typename S>
__device__ __forceinline__ void store_small_stencil(const S* __restrict__ u, int K, int e, uint32_t t, bool active,
                                                    bool valid, int j, const double (&Rc)[Phys<EQ>::M],
                                                    const double (&mom)[5], double* __restrict__ compact,
                                                    uint32_t* __restrict__ status) {
    constexpr int M = Phys<EQ>::M, NP = 6;
    constexpr int ND = LimLanes<EQ>::ND, LPC = LimLanes<EQ>::LPC;
    // back to conserved variables: sum over (d, k) of R_d[c][k] mom_dk / ND
    double res[M][NP - 1];
#pragma unroll
    for (int c = 0; c < M; ++c)
#pragma unroll
        for (int i = 0; i < NP - 1; ++i) res[c][i] = (1.0 / ND) * Rc[c] * mom[i];
#pragma unroll
    for (int o = 1; o < LPC; o <<= 1)
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int i = 0; i < NP - 1; ++i) res[c][i] += __shfl_xor(res[c][i], o, LPC);
    if (active && j < M) {
        double* outp = compact + (size_t)t * (M * NP) + j * NP;
        double sel[NP - 1];
#pragma unroll
        for (int i = 0; i < NP - 1; ++i) {
            double v = res[0][i];
#pragma unroll
            for (int c = 1; c < M; ++c) v = (j == c) ? res[c][i] : v;
            sel[i] = v;
        }
        outp[0] = u[(size_t)(j * NP) * K + e];
        if (valid) {
#pragma unroll
            for (int i = 1; i < NP; ++i) outp[i] = sel[i - 1];
        } else {
#pragma unroll
            for (int i = 1; i < NP; ++i) outp[i] = u[(size_t)(j * NP + i) * K + e];
        }
    }
    if (active && !valid && j == 0) atomicOr(status, CSWDG_STATUS_RANK);
}

// Type-II WENO on the same subcell stencils (params.reconstruction = 2; N
// = 2): the small-stencil fits above, their smoothness indicators, and at
// the nine points of the degree-4 rule the stored linear weights split into
// two positive groups (gamma+- of Shi, Hu and Shu), nonlinear weights
// (gamma+-_j / sigma+-) (1 + (tau / (1e-10 + beta_j))^2) per group with tau
// = max beta - min beta, R(x_q) = sigma+ R+ - sigma- R-, and the projection
// sum_q w_q R(x_q) psi_i(x_q).
template <int EQ, typename S>
__global__ __launch_bounds__(64, 3) void k_limiter_t2(DevMesh msh, const S* __restrict__ u,
                                                const double* __restrict__ ops,
                                                const int32_t* __restrict__ list,
                                                const uint32_t* __restrict__ count,
                                                double* __restrict__ compact,
                                                uint32_t* __restrict__ status, double gamma,
                                                int comp) {
    constexpr int N = 2;
    using D = Dims<N>;
    using LO = OpLayoutT2;
    constexpr int M = Phys<EQ>::M, NP = D::NP, NQ = LO::NQ;
    constexpr double EPS2 = 1e-10;
    constexpr int LPC = LimLanes<EQ>::LPC;
    constexpr int CPB = 64 / LPC;  // cells per block
    const int K = msh.K;
    uint32_t pre[kListSegs + 1];
    seg_prefix(count, K, pre);
    const uint32_t ncell = pre[kListSegs];
    const int j = threadIdx.x % LPC;  // lane within the cell
    const int d = j / M;              // characteristic direction
    const int k = j % M;              // characteristic field
    for (uint32_t base = blockIdx.x * CPB; base < ncell; base += gridDim.x * CPB) {
        const uint32_t t = base + threadIdx.x / LPC;
        const bool active = t < ncell;
        const int e = active ? seg_elem(list, pre, K, t) : 0;
        const double* __restrict__ op = ops + (size_t)e * LO::LEN;
        const bool valid = active && op[LO::VALID] != 0.0;
        double Rc[M], w0, w[3][3], cl[6][2], iw[6];
        small_stencil_fits<EQ, S, LO>(msh, u, op, e, d, k, gamma, comp, Rc, w0, w, cl);
        // WENO-Z form: iw_j = 1 + (tau / (EPS2 + beta_j))^2, tau = max beta - min beta
        const double bsc = op[LO::BSC];
        double bmax = 0.0, bmin = 0.0;
#pragma unroll
        for (int jj = 0; jj < 6; ++jj) {
            const double b = bsc * (cl[jj][0] * cl[jj][0] + cl[jj][1] * cl[jj][1]);
            iw[jj] = b;
            bmax = (jj == 0) ? b : fmax(bmax, b);
            bmin = (jj == 0) ? b : fmin(bmin, b);
        }
        const double tau = bmax - bmin;
#pragma unroll
        for (int jj = 0; jj < 6; ++jj) {
            const double r = tau / (EPS2 + iw[jj]);
            iw[jj] = 1.0 + r * r;
        }
        // at each point: the split linear weights, the nonlinear weights of
        // each group, R(x_q), and its contribution to the moments
        double mom[NP - 1];
#pragma unroll
        for (int i = 0; i < NP - 1; ++i) mom[i] = 0.0;
#pragma unroll 1
        for (int q = 0; q < NQ; ++q) {
            const double phx = op[LO::PHI + q * 2], phy = op[LO::PHI + q * 2 + 1];
            double gp[6], gm[6], sp = 0.0, sm = 0.0;
#pragma unroll
            for (int jj = 0; jj < 6; ++jj) {
                const double g = op[LO::GAM + q * 6 + jj];
                gp[jj] = 0.5 * (g + 3.0 * fabs(g));
                gm[jj] = gp[jj] - g;
                sp += gp[jj];
                sm += gm[jj];
            }
            double ap = 0.0, am = 0.0, rp = 0.0, rm = 0.0;
#pragma unroll
            for (int jj = 0; jj < 6; ++jj) {
                const double Lx = w0 + phx * cl[jj][0] + phy * cl[jj][1];
                const double a1 = (gp[jj] / sp) * iw[jj], a2 = (gm[jj] / sm) * iw[jj];
                ap += a1;
                am += a2;
                rp += a1 * Lx;
                rm += a2 * Lx;
            }
            const double R = sp * (rp / ap) - sm * (rm / am);
#pragma unroll
            for (int i = 0; i < NP - 1; ++i) mom[i] += op[LO::PMQ + i * NQ + q] * R;
        }
        store_small_stencil<EQ, S>(u, K, e, t, active, valid, j, Rc, mom, compact, status);
    }
}

// Mixed WENO on the same subcell stencils (params.reconstruction = 3; N =
// 2): the small-stencil fits above, the quadratic fit Q on the nine pieces,
// p_0 = (Q - gamma_s sum_j L_j) / gamma_0 with gamma_0 = 0.85 and gamma_s =
// 0.025, the smoothness indicators (of p_0 by the stored matrix over the
// derivative orders 1 and 2, of L_j as BSC |c_j|^2), the weights
// gamma_j / (1e-6 + beta_j)^2 normalised, R = omega_0 p_0 + sum_j omega_j L_j
// in the scaled monomials, and its moments by the stored projection.
template <int EQ, typename S>
__global__ __launch_bounds__(64, 3) void k_limiter_mx(DevMesh msh, const S* __restrict__ u,
                                                const double* __restrict__ ops,
                                                const int32_t* __restrict__ list,
                                                const uint32_t* __restrict__ count,
                                                double* __restrict__ compact,
                                                uint32_t* __restrict__ status, double gamma,
                                                int comp) {
    using LO = OpLayoutMX;
    constexpr int M = Phys<EQ>::M, NM = LO::NM;
    constexpr double G0 = 0.85, GS = 0.025, EPS = 1e-6;
    constexpr int LPC = LimLanes<EQ>::LPC;
    constexpr int CPB = 64 / LPC;  // cells per block
    const int K = msh.K;
    uint32_t pre[kListSegs + 1];
    seg_prefix(count, K, pre);
    const uint32_t ncell = pre[kListSegs];
    const int j = threadIdx.x % LPC;  // lane within the cell
    const int d = j / M;              // characteristic direction
    const int k = j % M;              // characteristic field
    for (uint32_t base = blockIdx.x * CPB; base < ncell; base += gridDim.x * CPB) {
        const uint32_t t = base + threadIdx.x / LPC;
        const bool active = t < ncell;
        const int e = active ? seg_elem(list, pre, K, t) : 0;
        const double* __restrict__ op = ops + (size_t)e * LO::LEN;
        const bool valid = active && op[LO::VALID] != 0.0;
        double Rc[M], w0, w[3][3], cl[6][2];
        small_stencil_fits<EQ, S, LO>(msh, u, op, e, d, k, gamma, comp, Rc, w0, w, cl);
        // Q on the nine pieces (row 3 p + f), then p_0
        double c0[NM];
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            double s = 0.0;
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int f = 0; f < 3; ++f) s += op[LO::X3 + i * 9 + p * 3 + f] * (w[f][p] - w0);
            c0[i] = s;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            double s = 0.0;
#pragma unroll
            for (int jj = 0; jj < 6; ++jj) s += cl[jj][i];
            c0[i] -= GS * s;
        }
#pragma unroll
        for (int i = 0; i < NM; ++i) c0[i] /= G0;
        // smoothness indicators and the nonlinear weights
        double b0 = 0.0;
        {
            int q = 0;
#pragma unroll
            for (int a = 0; a < NM; ++a)
#pragma unroll
                for (int b = a; b < NM; ++b, ++q) b0 += (a == b ? 1.0 : 2.0) * op[LO::BP + q] * c0[a] * c0[b];
        }
        const double bsc = op[LO::BSC];
        double om[7];
        om[0] = G0 / ((EPS + b0) * (EPS + b0));
        double osum = om[0];
#pragma unroll
        for (int jj = 0; jj < 6; ++jj) {
            const double b = bsc * (cl[jj][0] * cl[jj][0] + cl[jj][1] * cl[jj][1]);
            om[1 + jj] = GS / ((EPS + b) * (EPS + b));
            osum += om[1 + jj];
        }
        // R = omega_0 p_0 + sum_j omega_j L_j, then its moments
        double cr[NM];
#pragma unroll
        for (int i = 0; i < NM; ++i) cr[i] = (om[0] / osum) * c0[i];
#pragma unroll
        for (int jj = 0; jj < 6; ++jj) {
            cr[0] += (om[1 + jj] / osum) * cl[jj][0];
            cr[1] += (om[1 + jj] / osum) * cl[jj][1];
        }
        double mom[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            double s = 0.0;
#pragma unroll
            for (int kk = 0; kk < NM; ++kk) s += op[LO::PM + i * NM + kk] * cr[kk];
            mom[i] = s;
        }
        store_small_stencil<EQ, S>(u, K, e, t, active, valid, j, Rc, mom, compact, status);
    }
}


template <int N, int M, typename S>
__global__ __launch_bounds__(256) void k_scatter(int K, S* __restrict__ u,
                                                 const int32_t* __restrict__ list,
                                                 const uint32_t* __restrict__ count,
                                                 const double* __restrict__ compact,
                                                 unsigned long long* __restrict__ tstats) {
    constexpr int NP = Dims<N>::NP;
    uint32_t pre[kListSegs + 1];
    seg_prefix(count, K, pre);
    const uint32_t n = pre[kListSegs];
    if (tstats != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
        atomicAdd(&tstats[0], (unsigned long long)n);
        atomicAdd(&tstats[1], 1ull);
    }
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const int e = seg_elem(list, pre, K, t);
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int i = 1; i < NP; ++i) u[(size_t)(c * NP + i) * K + e] = (S)compact[(size_t)t * (M * NP) + c * NP + i];
    }
}

// ---------------------------------------------------------------------------
// Positivity-preserving scaling (not part of the paper's method): Zhang and
// Shu's scaling of the modes above the cell mean, first of the density so
// that rho >= eps, then of all variables so that p >= eps_p, at the volume
// points and the edge Gauss points where the residual evaluates u_h;
// eps = min(1e-13, rhobar, pbar), eps_p = max(eps, 1e-10 pbar) (a floor
// relative to the mean pressure keeps the rounding of the root, large near
// vacuum, from ending below zero).  The pressure factor of a point below
// eps_p is the root in [0, 1] of rho(t) (E(t) - eps_p/(gamma-1)) - |m(t)|^2/2
// along U(t) = Ubar + t (U_q - Ubar), a quadratic in t whose value is >= 0
// at t = 0 and < 0 at t = 1.  One thread per element; cells whose mean is
// not admissible are left alone; a cell is rewritten only when scaled.
// ---------------------------------------------------------------------------
template <int NP>
__device__ __forceinline__ double dot_modes(const double (&c)[NP], const double* __restrict__ phi) {
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) r = fma(c[i], phi[i], r);
    return r;
}

__device__ __forceinline__ double pressure_root(const double (&ub)[4], const double (&uq)[4], double e) {
    const double dr = uq[0] - ub[0], d1 = uq[1] - ub[1], d2 = uq[2] - ub[2], dE = uq[3] - ub[3];
    const double a = dr * dE - 0.5 * (d1 * d1 + d2 * d2);
    const double b = ub[0] * dE + dr * (ub[3] - e) - (ub[1] * d1 + ub[2] * d2);
    const double c = ub[0] * (ub[3] - e) - 0.5 * (ub[1] * ub[1] + ub[2] * ub[2]);
    double t;
    if (fabs(a) <= 1e-14 * (fabs(b) + fabs(c))) {
        t = (b < 0.0) ? -c / b : 0.0;
    } else {
        const double sq = sqrt(fmax(b * b - 4.0 * a * c, 0.0));
        const double q = -0.5 * (b + copysign(sq, b));
        const double r1 = q / a;
        const double r2 = (q != 0.0) ? c / q : 0.0;
        t = (r1 >= 0.0 && r1 <= 1.0) ? r1 : r2;
    }
    return fmin(fmax(t, 0.0), 1.0);
}

template <int N, typename S>
__global__ __launch_bounds__(256) void k_positivity(int K, S* __restrict__ u, double gamma,
                                                    uint32_t* __restrict__ status) {
    using D = Dims<N>;
    constexpr int NP = D::NP, NQ = D::NQ, NE = D::NE;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K) return;
    const Tab<N>& T = tab<N>();
    double c[4][NP];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int i = 0; i < NP; ++i) c[v][i] = (double)u[(size_t)(v * NP + i) * K + e];
    const double psi0 = T.V[0][0];
    double ub[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) ub[v] = c[v][0] * psi0;
    const double gm1 = gamma - 1.0;
    const double pb = gm1 * (ub[3] - 0.5 * (ub[1] * ub[1] + ub[2] * ub[2]) / ub[0]);
    if (!(ub[0] > 0.0) || !(pb > 0.0) || !(pb < INFINITY) || !(ub[0] < INFINITY)) return;
    const double eps = fmin(1e-13, fmin(ub[0], pb));
    // density
    double rmin = INFINITY;
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) rmin = fmin(rmin, dot_modes<NP>(c[0], T.V[q]));
#pragma unroll 1
    for (int fg = 0; fg < 3 * NE; ++fg) rmin = fmin(rmin, dot_modes<NP>(c[0], T.PF[fg / NE][fg % NE]));
    double th1 = 1.0;
    if (rmin < eps) {
        th1 = (ub[0] - eps) / (ub[0] - rmin);
#pragma unroll
        for (int i = 1; i < NP; ++i) c[0][i] *= th1;
    }
    // pressure
    const double eps_p = fmax(eps, 1e-10 * pb);
    const double ee = eps_p / gm1;
    double th2 = 1.0;
#pragma unroll 1
    for (int q = 0; q < NQ + 3 * NE; ++q) {
        const double* phi = (q < NQ) ? T.V[q] : T.PF[(q - NQ) / NE][(q - NQ) % NE];
        double uq[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) uq[v] = dot_modes<NP>(c[v], phi);
        const double pq = gm1 * (uq[3] - 0.5 * (uq[1] * uq[1] + uq[2] * uq[2]) / uq[0]);
        if (pq < eps_p) th2 = fmin(th2, pressure_root(ub, uq, ee));
    }
    if (th1 < 1.0 || th2 < 1.0) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int i = 1; i < NP; ++i) u[(size_t)(v * NP + i) * K + e] = (S)(c[v][i] * th2);
        atomicOr(status, CSWDG_STATUS_SCALED);
    }
}

// ---------------------------------------------------------------------------
// Initial data: quadrature points and L2 projection
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_ic_points(DevMesh msh, double* __restrict__ xy) {
    constexpr int NQI = Dims<N>::NQI;
    const int K = msh.K;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K) return;
    const TabIC<N>& T = tabic<N>();
    const double x0 = msh.vx[e], x1 = msh.vx[K + e], x2 = msh.vx[2 * K + e];
    const double y0 = msh.vy[e], y1 = msh.vy[K + e], y2 = msh.vy[2 * K + e];
    for (int q = 0; q < NQI; ++q) {
        const double l1 = 0.5 * (1.0 + T.r[q]), l2 = 0.5 * (1.0 + T.s[q]);
        xy[(size_t)q * K + e] = x0 + l1 * (x1 - x0) + l2 * (x2 - x0);
        xy[(size_t)(NQI + q) * K + e] = y0 + l1 * (y1 - y0) + l2 * (y2 - y0);
    }
}

template <int N, typename S>
__global__ __launch_bounds__(256) void k_project(int K, int m, const double* __restrict__ vals,
                                                 S* __restrict__ u) {
    constexpr int NQI = Dims<N>::NQI, NP = Dims<N>::NP;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K) return;
    const TabIC<N>& T = tabic<N>();
    for (int c = 0; c < m; ++c) {
        double acc[NP];
#pragma unroll
        for (int n = 0; n < NP; ++n) acc[n] = 0.0;
        for (int q = 0; q < NQI; ++q) {
            const double v = vals[(size_t)(c * NQI + q) * K + e];
#pragma unroll
            for (int n = 0; n < NP; ++n) acc[n] += T.wV[q][n] * v;
        }
#pragma unroll
        for (int n = 0; n < NP; ++n) u[(size_t)(c * NP + n) * K + e] = (S)acc[n];
    }
}

}  // namespace

int ic_points_per_element(int N) {
    return N == 1 ? Dims<1>::NQI : (N == 2 ? Dims<2>::NQI : Dims<3>::NQI);
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free limiter entry point: the troubled-list
// counters, the troubled list and the compact limiter results live in one
// static device array (each device the library runs on holds its own copy
// for the life of the process).  Host code never names the array in a launch:
// init_noalloc_scratch() takes its device address once per device (with that
// device current) and the entry point passes that address to the kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int init_noalloc_scratch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CSWDG_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (g_scratch_ptr[dev] != nullptr) return CSWDG_OK;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) return CSWDG_EHIP;
    g_scratch_ptr[dev] = ptr;
    return CSWDG_OK;
}

void* noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    return g_scratch_ptr[device];
}

int upload_tables_device() {
    int rc = upload_tables_here();
    if (rc != CSWDG_OK) return rc;
    return upload_tables_adjoint();
}


hipError_t launch_residual_reset(const LaunchCtx& c, const DevMesh& m, int mode, const void* u,
                                 const void* un, void* out, const double* dt, uint32_t* reset) {
    const unsigned bs = (c.residual_block == 64 || c.residual_block == 128) ? (unsigned)c.residual_block : 256u;
    const unsigned g = grid_for(m.K, bs);
    const double* U = (const double*)u;
    const double* UN = (const double*)un;
    double* O = (double*)out;
#define CSWDG_RES_LAUNCH(KERN)                                                                   \
    switch (mode) {                                                                              \
        case 0: KERN<EQ, N, 0><<<g, bs, 0, c.stream>>>(m, U, UN, O, dt, c.gamma, reset); break; \
        case 1: KERN<EQ, N, 1><<<g, bs, 0, c.stream>>>(m, U, UN, O, dt, c.gamma, reset); break; \
        case 2: KERN<EQ, N, 2><<<g, bs, 0, c.stream>>>(m, U, UN, O, dt, c.gamma, reset); break; \
        case 3: KERN<EQ, N, 3><<<g, bs, 0, c.stream>>>(m, U, UN, O, dt, c.gamma, reset); break; \
        default: return hipErrorInvalidValue;                                                    \
    }
    if (c.precision == 1) {
        // FP32-bulk: single-precision state and arithmetic, compact schedule
        const float* UF = (const float*)u;
        const float* UNF = (const float*)un;
        float* OF = (float*)out;
        CSWDG_DISPATCH_EN(c.eq, c.N, {
            switch (mode) {
                case 0: k_residual_compact<EQ, N, 0, float><<<g, bs, 0, c.stream>>>(m, UF, UNF, OF, dt, c.gamma, reset); break;
                case 1: k_residual_compact<EQ, N, 1, float><<<g, bs, 0, c.stream>>>(m, UF, UNF, OF, dt, c.gamma, reset); break;
                case 2: k_residual_compact<EQ, N, 2, float><<<g, bs, 0, c.stream>>>(m, UF, UNF, OF, dt, c.gamma, reset); break;
                case 3: k_residual_compact<EQ, N, 3, float><<<g, bs, 0, c.stream>>>(m, UF, UNF, OF, dt, c.gamma, reset); break;
                default: return hipErrorInvalidValue;
            }
        });
        return hipGetLastError();
    }
    CSWDG_DISPATCH_EN(c.eq, c.N, {
        if (c.residual_variant == 1) {
            CSWDG_RES_LAUNCH(k_residual)
        } else if (c.residual_variant == 2) {
            CSWDG_RES_LAUNCH(k_residual_stream)
        } else if (c.residual_variant == 3) {
            CSWDG_RES_LAUNCH(k_residual_compact_d)
        } else if (c.residual_variant == 4) {
            // matrix cores: P2 only, 16 elements per wave
            if constexpr (N == 2) {
                const unsigned gm = grid_for(m.K, bs / 4);
switch (mode) {
                    case 0: k_residual_mfma<EQ, 0><<<gm, bs, 0, c.stream>>>(m, U, UN, O, dt, c.gamma, reset); break;
                    case 1: k_residual_mfma<EQ, 1><<<gm, bs, 0, c.stream>>>(m, U, UN, O, dt, c.gamma, reset); break;
                    case 2: k_residual_mfma<EQ, 2><<<gm, bs, 0, c.stream>>>(m, U, UN, O, dt, c.gamma, reset); break;
                    case 3: k_residual_mfma<EQ, 3><<<gm, bs, 0, c.stream>>>(m, U, UN, O, dt, c.gamma, reset); break;
                    default: return hipErrorInvalidValue;
                }
            } else {
                return hipErrorInvalidValue;
            }
        } else {
            CSWDG_RES_LAUNCH(k_residual_lean)
        }
    });
#undef CSWDG_RES_LAUNCH
    return hipGetLastError();
}

hipError_t launch_max_dt(const LaunchCtx& c, const DevMesh& m, const void* u, double hmin, double* dt,
                         double* partial, uint32_t*, uint32_t* status, int nblocks) {
    CSWDG_DISPATCH_ENP(c.eq, c.N, c.precision, {
        k_dt_partial<EQ, N, S><<<nblocks, 256, 0, c.stream>>>(m.K, (const S*)u, c.gamma, partial, status);
    });
    k_dt_final<<<1, 256, 0, c.stream>>>(nblocks, partial, c.cfl, hmin, dt);
    return hipGetLastError();
}

hipError_t launch_max_dt_inst(const LaunchCtx& c, const DevMesh& m, const void* u, const double* hmin,
                              double* dt, unsigned long long* amax_bits, uint32_t* status) {
    const unsigned g = grid_for(m.K, 256);
    CSWDG_DISPATCH_ENP(c.eq, c.N, c.precision, {
        k_dt_inst<EQ, N, S><<<g, 256, 0, c.stream>>>(m, (const S*)u, c.gamma, amax_bits, status);
    });
    k_dt_inst_final<<<grid_for(m.n_inst, 256), 256, 0, c.stream>>>(m.n_inst, amax_bits, c.cfl, hmin, dt);
    return hipGetLastError();
}

hipError_t launch_lf_alpha(const LaunchCtx& c, const DevMesh& m, const void* u, unsigned long long* amax_bits,
                           double* alpha, uint32_t* status) {
    const unsigned g = grid_for(m.K, 256);
    CSWDG_DISPATCH_ENP(c.eq, c.N, c.precision, {
        k_dt_inst<EQ, N, S><<<g, 256, 0, c.stream>>>(m, (const S*)u, c.gamma, amax_bits, status);
    });
    k_lf_alpha_final<<<grid_for(m.n_inst, 256), 256, 0, c.stream>>>(m.n_inst, amax_bits, alpha);
    return hipGetLastError();
}

hipError_t launch_time_advance(const LaunchCtx& c, int n_inst, double* time, const double* dt) {
    k_time_advance<<<grid_for(n_inst, 64), 64, 0, c.stream>>>(n_inst, time, dt);
    return hipGetLastError();
}

hipError_t launch_kxrcf(const LaunchCtx& c, const DevMesh& m, const void* u, uint8_t* flags, double* R,
                        int32_t* list, uint32_t* count) {
    // one-wave blocks: measured 4% faster than 256 threads at the 1M P2
    // Euler workload (the list append is per block either way)
    const unsigned bs = 64, g = grid_for(m.K, bs);
    if (c.indicator == 1) {
        if (m.tvb == nullptr) return hipErrorInvalidValue;
        CSWDG_DISPATCH_ENP(c.eq, c.N, c.precision, {
            k_tvb<EQ, N, S><<<g, bs, 0, c.stream>>>(m, (const S*)u, flags, R, list, count, c.tvb_m);
        });
    } else {
        CSWDG_DISPATCH_ENP(c.eq, c.N, c.precision, {
            k_kxrcf<EQ, N, S><<<g, bs, 0, c.stream>>>(m, (const S*)u, flags, R, list, count, c.c_k, c.kxrcf_rms);
        });
    }
    return hipGetLastError();
}

hipError_t launch_compact_mask(const LaunchCtx& c, int K, const uint8_t* mask, uint8_t* flags,
                               int32_t* list, uint32_t* count) {
    k_compact_mask<<<grid_for(K, 256), 256, 0, c.stream>>>(K, mask, flags, list, count);
    return hipGetLastError();
}

hipError_t launch_zero_u32(const LaunchCtx& c, uint32_t* p, int n) {
    k_zero_u32<<<grid_for(n, 256), 256, 0, c.stream>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_limiter_t1(const LaunchCtx& c, const DevMesh& m, const void* u, const double* ops,
                             const int32_t* list, const uint32_t* count, double* compact, uint32_t* status,
                             int max_cells);
hipError_t launch_limiter_t2(const LaunchCtx& c, const DevMesh& m, const void* u, const double* ops,
                             const int32_t* list, const uint32_t* count, double* compact, uint32_t* status,
                             int max_cells);

// the limiter's launch with the smoothness-indicator reading as a template
// argument (the literal reading's extra registers stay out of the default)
#define CSWDG_LIMITER_LAUNCH(QT)                                                                             \
    do {                                                                                                     \
        if (c.beta_lit)                                                                                      \
            k_limiter<EQ, N, S, QT, true><<<g, bs, 0, c.stream>>>(m, (const S*)u, ops, list, count, compact,  \
                                                                   status, c.gamma, c.eps, c.char_comp,      \
                                                                   c.weights_linear);                        \
        else                                                                                                 \
            k_limiter<EQ, N, S, QT, false><<<g, bs, 0, c.stream>>>(m, (const S*)u, ops, list, count, compact, \
                                                                    status, c.gamma, c.eps, c.char_comp,     \
                                                                    c.weights_linear);                       \
    } while (0)

hipError_t launch_limiter(const LaunchCtx& c, const DevMesh& m, const void* u, const double* ops,
                          const int32_t* list, const uint32_t* count, double* compact, uint32_t* status,
                          int max_cells) {
    if (c.recon == 1) return launch_limiter_t1(c, m, u, ops, list, count, compact, status, max_cells);
    if (c.recon == 2 || c.recon == 3) return launch_limiter_t2(c, m, u, ops, list, count, compact, status, max_cells);
    const unsigned bs = 64;
    const int lpc = c.eq == 1 ? LimLanes<1>::LPC : LimLanes<0>::LPC;
    // at four waves per SIMD, 4,096 one-wave blocks are resident at once;
    // up to 16,384 blocks so that every troubled cell's wave is in flight
    // (each wave's cells form one chain of dependent loads); blocks beyond
    // the troubled count exit at once
    unsigned g = grid_for(max_cells, bs / lpc);
    if (g > 16384u) g = 16384u;
    if (g == 0) g = 1;
    CSWDG_DISPATCH_ENP(c.eq, c.N, c.precision, {
        const int qt = N >= 2 ? c.qtop : kTopQuartic;
        if (N == 1)
            CSWDG_LIMITER_LAUNCH(kTopQuartic);
        else if (qt == kTopQuadratic)
            CSWDG_LIMITER_LAUNCH(kTopQuadratic);
        else if (qt == kTopCubic)
            CSWDG_LIMITER_LAUNCH(kTopCubic);
        else if (qt == kTopCubicTel)
            CSWDG_LIMITER_LAUNCH(kTopCubicTel);
        else if (qt == kTopSextic) {
            if constexpr (N == 3)
                CSWDG_LIMITER_LAUNCH(kTopSextic);
            else
                return hipErrorInvalidValue;
        } else
            CSWDG_LIMITER_LAUNCH(kTopQuartic);
    });
    return hipGetLastError();
}
#undef CSWDG_LIMITER_LAUNCH

hipError_t launch_limiter_t1(const LaunchCtx& c, const DevMesh& m, const void* u, const double* ops,
                             const int32_t* list, const uint32_t* count, double* compact, uint32_t* status,
                             int max_cells) {
    const unsigned bs = 64;
    const int lpc = c.eq == 1 ? LimLanes<1>::LPC : LimLanes<0>::LPC;
    unsigned g = grid_for(max_cells, bs / lpc);
    if (g > 16384u) g = 16384u;
    if (g == 0) g = 1;
    if (c.N != 1 && c.N != 2) return hipErrorInvalidValue;
    CSWDG_DISPATCH_ENP(c.eq, c.N, c.precision, {
        if constexpr (N <= 2)
            k_limiter_t1<EQ, N, S><<<g, bs, 0, c.stream>>>(m, (const S*)u, ops, list, count, compact, status, c.gamma,
                                                          c.eps, c.char_comp);
    });
    return hipGetLastError();
}

// Type-II WENO on the same subcell stencils (params.reconstruction = 2;
// N = 2): launched like the type-I limiter
hipError_t launch_limiter_t2(const LaunchCtx& c, const DevMesh& m, const void* u, const double* ops,
                             const int32_t* list, const uint32_t* count, double* compact, uint32_t* status,
                             int max_cells) {
    const unsigned bs = 64;
    const int lpc = c.eq == 1 ? LimLanes<1>::LPC : LimLanes<0>::LPC;
    unsigned g = grid_for(max_cells, bs / lpc);
    if (g > 16384u) g = 16384u;
    if (g == 0) g = 1;
    if (c.N != 2) return hipErrorInvalidValue;
    CSWDG_DISPATCH_ENP(c.eq, c.N, c.precision, {
        if constexpr (N == 2) {
            if (c.recon == 3)
                k_limiter_mx<EQ, S><<<g, bs, 0, c.stream>>>(m, (const S*)u, ops, list, count, compact, status,
                                                           c.gamma, c.char_comp);
            else
                k_limiter_t2<EQ, S><<<g, bs, 0, c.stream>>>(m, (const S*)u, ops, list, count, compact, status,
                                                           c.gamma, c.char_comp);
        }
    });
    return hipGetLastError();
}

hipError_t launch_scatter(const LaunchCtx& c, int K, void* u, const int32_t* list, const uint32_t* count,
                          const double* compact, int max_cells, unsigned long long* tstats) {
    const unsigned bs = 256;
    unsigned g = grid_for(max_cells, bs);
    if (g > 4096u) g = 4096u;
    if (g == 0) g = 1;
    CSWDG_DISPATCH_ENP(c.eq, c.N, c.precision, {
        k_scatter<N, Phys<EQ>::M, S><<<g, bs, 0, c.stream>>>(K, (S*)u, list, count, compact, tstats);
    });
    return hipGetLastError();
}

hipError_t launch_positivity(const LaunchCtx& c, const DevMesh& m, void* u, uint32_t* status) {
    if (c.eq != 1) return hipErrorInvalidValue;
    if (m.K == 0) return hipSuccess;
    const unsigned g = grid_for(m.K, 256);
    CSWDG_DISPATCH_ENP(1, c.N, c.precision, {
        (void)EQ;
        k_positivity<N, S><<<g, 256, 0, c.stream>>>(m.K, (S*)u, c.gamma, status);
    });
    return hipGetLastError();
}

hipError_t launch_ic_points(const LaunchCtx& c, const DevMesh& m, double* xy) {
    const unsigned g = grid_for(m.K, 256);
    if (c.N == 1) k_ic_points<1><<<g, 256, 0, c.stream>>>(m, xy);
    else if (c.N == 2) k_ic_points<2><<<g, 256, 0, c.stream>>>(m, xy);
    else if (c.N == 3) k_ic_points<3><<<g, 256, 0, c.stream>>>(m, xy);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_project(const LaunchCtx& c, const DevMesh& m, const double* vals, void* u) {
    const unsigned g = grid_for(m.K, 256);
    const int mv = c.eq == 0 ? 1 : 4;
    CSWDG_DISPATCH_ENP(c.eq, c.N, c.precision, {
        (void)EQ;
        k_project<N, S><<<g, 256, 0, c.stream>>>(m.K, mv, vals, (S*)u);
    });
    return hipGetLastError();
}

}  // namespace cswdg
