// Internal declarations shared by the host sources and the kernel source.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cswdg.h"
#include "tables.h"

namespace cswdg {

constexpr double kPsi0 = 0.70710678118654752440;  // constant mode 1/sqrt(2)

// ----------------------------------------------------------------------------
// host: basis and quadrature (host_tables.cpp)
// ----------------------------------------------------------------------------
struct Rule1D {
    std::vector<long double> x, w;
};
Rule1D gauss_jacobi(int n, double alpha);  // weight (1-x)^alpha on [-1,1]
struct Rule2D {
    std::vector<double> r, s, w;  // reference triangle, sum w = 2
};
Rule2D triangle_rule(int n);
int n_modes(int N);
// psi_n(r,s), dpsi/dr, dpsi/ds for n = 0..Np-1 (orthonormal basis)
void basis_eval(int N, double r, double s, double* psi, double* dr = nullptr, double* ds = nullptr);
// monomial-form coefficients of the basis: psi_n = sum_k C[n][k] r^a_k s^b_k
// with (a_k, b_k) enumerated by total degree, k < Np
void basis_monomial_form(int N, std::vector<double>& C);

template <int N>
void fill_tables(Tab<N>& t);

// ----------------------------------------------------------------------------
// host: mesh (host_mesh.cpp)
// ----------------------------------------------------------------------------
struct HostMesh {
    int64_t K = 0;
    int bc = 0;
    double px = 0, py = 0;
    std::vector<int32_t> tri;   // [K][3] after the CCW fix
    std::vector<int32_t> nbr;   // [K][3]
    std::vector<uint8_t> info;  // [K][3]
    std::vector<double> vx, vy; // [3][K] SoA element vertices
    int64_t n_flipped = 0;
    double hmin = 0;            // min over elements of 2 * inradius
};

// largest mesh: the last index of a [3][K] array, 3 K - 1, fits a 32-bit
// signed integer (the kernels' element indices)
constexpr int64_t kMaxTriangles = 715827882;
// returns CSWDG_OK or an error code with msg filled
int build_mesh(int64_t nv, const double* vxy, int64_t nt, const int32_t* tri, int bc, double px,
               double py, HostMesh& m, std::string& msg);

// disjoint union of independently built meshes (instances): vertex and element
// ids are offset, faces keep their own neighbours; off[i] is the first element
// of instance i (off[n] = K) and hmin[i] its time-step length scale
int concat_meshes(const std::vector<HostMesh>& parts, HostMesh& out, std::vector<int32_t>& off,
                  std::vector<double>& hmin, std::string& msg);

// per-element limiter operators (host_ops.cpp); returns number of
// rank-deficient elements and perpendicular feet that fell outside
// kTop* for degree N from the p2_top parameter: 0 the default reading of N
// (the quadratic top for N = 2, the quartic for N = 3), 1 quadratic, 2
// quartic, 3 the telescoping cubic, 4 the printed cubic
inline int top_for(int N, int p2_top) {
    if (N < 2) return kTopQuadratic;
    switch (p2_top) {
        case 1: return kTopQuadratic;
        case 2: return kTopQuartic;
        case 3: return kTopCubicTel;
        case 4: return kTopCubic;
        case 5: return kTopSextic;  // N = 3 only (the API checks)
        default: return N == 2 ? kTopQuadratic : kTopQuartic;
    }
}

// the per-element record of the type-I reconstruction (OpLayoutT1, N = 1, 2)
int build_type1_ops(const HostMesh& m, int N, std::vector<double>& ops, int64_t& n_rank);
// the per-element record of the type-II reconstruction (OpLayoutT2, N = 2)
int build_type2_ops(const HostMesh& m, std::vector<double>& ops, int64_t& n_rank);
int build_mixed_ops(const HostMesh& m, std::vector<double>& ops, int64_t& n_rank);

int build_limiter_ops(const HostMesh& m, int N, int qtop, bool constant_gamma, bool ghost_extrapolate, std::vector<double>& ops,
                      int64_t& n_rank, int64_t& n_foot);
// the TVB indicator's midpoint decomposition [9][K] (host_ops.cpp); n_neg
// counts midpoints with no pair of nonnegative coefficients
void build_tvb_ops(const HostMesh& m, std::vector<double>& A, int64_t& n_neg);

// ----------------------------------------------------------------------------
// device views and launchers (kernels.hip)
// ----------------------------------------------------------------------------
// troubled-cell list layout: segments and counter stride (in uint32)
constexpr int kListSegs = 8;
constexpr int kCountStride = 32;
constexpr int kCountWords = kListSegs * kCountStride;

struct DevMesh {
    int K;
    const double* vx;      // [3][K]
    const double* vy;      // [3][K]
    const int32_t* nbr;    // [3][K]
    const uint32_t* info;  // [K], face f in byte f
    int xcd_tiles;         // 1: give each XCD a contiguous range of blocks
    const double* inflow;  // [m] state of inflow boundary faces (conserved variables)
    int n_inst;            // independent meshes held (1 for a single mesh)
    const int32_t* inst_off;  // [n_inst + 1] first element of each instance
    const double* lf_alpha;   // [n_inst] global Lax-Friedrichs constants, or null (local)
    const double* time;       // [n_inst] solution time at the start of the step
    const double* shock;      // moving shock of boundary kind 3: nx, ny, d0, w, post[4], pre[4]; or null
    const double* tvb;        // [9][K] TVB indicator: midpoint i along neighbour face f at row 3 i + f; or null
};

struct LaunchCtx {
    hipStream_t stream;
    int eq, N, precision;
    double gamma, cfl, c_k, eps;
    int residual_variant;  // residual schedule: 0 lean, 1 wide, 2 stream, 3 compact (default)
    int residual_block;    // residual threads per block: 64, 128 or 256
    int kxrcf_rms;         // KXRCF norm divided by |Delta|^(1/2)
    int char_comp;         // Euler limiting on the conserved variables
    int weights_linear;    // limiter weights omega = gamma
    int qtop;  // N >= 2: top member of the hierarchy (kTop* below)
    int recon; // 0 the hierarchical reconstruction, 1 type-I WENO, 2 type-II WENO, 3 mixed WENO
    int beta_lit;  // 1: smoothness indicators of p_l over orders 1..N (eq. smoothnessIndicator as printed)
    int indicator;         // troubled-cell indicator: 0 KXRCF, 1 TVB minmod
    double tvb_m;          // TVB constant M
};

int upload_tables_device();   // once per device (both translation units)

// Scratch of cswdg_csweno_limit_noalloc (a static device array in
// kernels.hip): init_noalloc_scratch() takes its address on the current
// device (once per device, at solver creation); noalloc_scratch(device)
// returns that address (nullptr before).  Layout: the troubled-list counters
// (kCountWords u32) at 0, the list (int32 [kListSegs][K], as the solver's
// own) at kNoAllocListOffset, the compact results (double [K][m][Np]) at the
// next 256-byte boundary.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr size_t kNoAllocListOffset = 1024;
constexpr int kMaxDevices = 64;
int init_noalloc_scratch();
void* noalloc_scratch(int device);
int upload_tables_adjoint();  // the adjoint unit's copy of the tables

// residual (mode 0) or RK stage 1..3; dt read from device; reset (may be
// null) is a counter set to zero by the kernel
hipError_t launch_residual_reset(const LaunchCtx& c, const DevMesh& m, int mode, const void* u,
                                 const void* un, void* out, const double* dt, uint32_t* reset);
// wave-speed reduction, dt = cfl * hmin / amax and state checks
hipError_t launch_max_dt(const LaunchCtx& c, const DevMesh& m, const void* u, double hmin,
                         double* dt, double* partial, uint32_t* counter, uint32_t* status,
                         int nblocks);
// the same per instance: dt[i] = cfl * hmin[i] / amax_i; amax_bits ([n_inst],
// zero on entry) is left zero for the next call
hipError_t launch_max_dt_inst(const LaunchCtx& c, const DevMesh& m, const void* u, const double* hmin,
                              double* dt, unsigned long long* amax_bits, uint32_t* status);
// flags of the selected indicator (+ optional R: KXRCF's ratio, or the TVB
// decision as 0/1) and the compacted list of troubled cells
hipError_t launch_kxrcf(const LaunchCtx& c, const DevMesh& m, const void* u, uint8_t* flags,
                        double* R, int32_t* list, uint32_t* count);
// compact a mask (or all cells when mask == nullptr) into the list
hipError_t launch_compact_mask(const LaunchCtx& c, int K, const uint8_t* mask, uint8_t* flags,
                               int32_t* list, uint32_t* count);
hipError_t launch_zero_u32(const LaunchCtx& c, uint32_t* p, int n);
// global Lax-Friedrichs constants: alpha[i] = the largest cell-mean wave
// speed of instance i of u (amax_bits [n_inst] zero on entry and exit)
hipError_t launch_lf_alpha(const LaunchCtx& c, const DevMesh& m, const void* u, unsigned long long* amax_bits,
                           double* alpha, uint32_t* status);
// time[i] += dt[i] for every instance (the end of a step)
hipError_t launch_time_advance(const LaunchCtx& c, int n_inst, double* time, const double* dt);
// positivity-preserving scaling of an Euler state in place (all elements)
hipError_t launch_positivity(const LaunchCtx& c, const DevMesh& m, void* u, uint32_t* status);
// limiter over the list; results to the compact buffer
hipError_t launch_limiter(const LaunchCtx& c, const DevMesh& m, const void* u, const double* ops,
                          const int32_t* list, const uint32_t* count, double* compact,
                          uint32_t* status, int max_cells);
// write the compact results into u (modes >= 1); tstats (may be null)
// accumulates (troubled cells, limiter calls)
hipError_t launch_scatter(const LaunchCtx& c, int K, void* u, const int32_t* list,
                          const uint32_t* count, const double* compact, int max_cells,
                          unsigned long long* tstats);
hipError_t launch_ic_points(const LaunchCtx& c, const DevMesh& m, double* xy);
hipError_t launch_project(const LaunchCtx& c, const DevMesh& m, const double* vals, void* u);
int ic_points_per_element(int N);

// adjoint (adjoint.hip)
hipError_t launch_residual_vjp(const LaunchCtx& c, const DevMesh& m, const void* u, const void* ybar,
                               void* prev_bar, void* un_bar, const double* dt, double a, double c_id,
                               double c_dt, int accumulate);
hipError_t launch_compact_slots(const LaunchCtx& c, int K, const uint8_t* mask, int32_t* list, int32_t* slot,
                                uint32_t* count);
hipError_t launch_limiter_vjp(const LaunchCtx& c, const DevMesh& m, const void* w, const double* ops,
                              const int32_t* list, const uint32_t* count, const void* ybar, double* contrib,
                              int max_cells);
hipError_t launch_limiter_gather(const LaunchCtx& c, const DevMesh& m, const uint8_t* mask, const int32_t* slot,
                                 const double* contrib, const void* ybar, void* wbar);

}  // namespace cswdg
