// C ABI of the library (declared in include/cswdg.h).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace cswdg;

namespace {

thread_local std::string g_err;

const char* kKernelNames[] = {"residual_rk", "max_dt", "kxrcf", "compact_mask", "limiter", "scatter", "copy", "zero", "project",
                              "residual_vjp", "limiter_vjp", "positivity"};
enum KernelId { KID_RESIDUAL = 0, KID_DT, KID_KXRCF, KID_COMPACT, KID_LIMITER, KID_SCATTER, KID_COPY, KID_ZERO, KID_PROJECT,
                KID_RESIDUAL_VJP, KID_LIMITER_VJP, KID_POSITIVITY, KID_COUNT };

std::mutex g_dev_mutex;
std::vector<int> g_dev_tables;  // devices whose constant tables are uploaded

}  // namespace

struct cswdg_solver {
    cswdg_params p{};
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    LaunchCtx ctx{};
    bool has_mesh = false;
    HostMesh mesh;
    DevMesh dm{};
    int M = 1, NP = 3;
    size_t state_elems = 0;
    double* d_vx = nullptr;
    double* d_vy = nullptr;
    int32_t* d_nbr = nullptr;
    uint32_t* d_info = nullptr;
    double* d_ops = nullptr;
    uint8_t* d_flags = nullptr;
    int32_t* d_list = nullptr;
    uint32_t* d_count = nullptr;   // troubled-list segment counters (kCountWords)
    uint32_t* d_status = nullptr;
    unsigned long long* d_tstats = nullptr;  // troubled cells, limiter calls
    double* d_compact = nullptr;
    double* d_partial = nullptr;
    double* d_dt = nullptr;
    void* d_T1 = nullptr;
    void* d_T2 = nullptr;
    // adjoint scratch (allocated by the first adjoint call)
    int32_t* d_slot = nullptr;
    double* d_contrib = nullptr;
    void* d_V = nullptr;
    // instances (a mesh that is a disjoint union of independent meshes)
    int n_inst = 1;
    std::vector<int32_t> inst_off;
    std::vector<double> inst_hmin;
    int32_t* d_inst_off = nullptr;
    double* d_inst_hmin = nullptr;
    unsigned long long* d_amax = nullptr;
    double* d_inflow = nullptr;   // [m] state of inflow boundary faces
    double* d_lfa = nullptr;      // [n_inst] global Lax-Friedrichs constants (lf_mode = 1)
    double* d_time = nullptr;     // [n_inst] solution time (advanced by steps while a moving shock is set)
    double* d_shock = nullptr;    // moving shock of boundary kind 3: nx, ny, d0, w, post[4], pre[4]
    double* d_tvb = nullptr;      // [9][K] TVB midpoint decomposition (indicator = 1 only)
    int64_t n_tvb_neg = 0;        // midpoints without a nonnegative decomposition
    bool shock_set = false;
    int64_t n_special = 0;        // boundary faces of wall or inflow kind
    int dt_blocks = 1024;
    int64_t n_rank = 0, n_foot = 0;
    // profiling
    bool prof = false;
    uint32_t prof_mask = ~0u;  // kernel classes recorded while profiling
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> recs;  // kernel id, event index of the start
};

struct cswdg_graph {
    hipGraphExec_t exec = nullptr;
    int device = 0;
    int64_t nodes = 0;
};

namespace {

int fail(cswdg_solver* s, int code, const std::string& msg) {
    if (s) s->err = msg;
    g_err = msg;
    return code;
}

int hipfail(cswdg_solver* s, hipError_t e, const char* what) {
    return fail(s, CSWDG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void free_mesh(cswdg_solver* s) {
    void* ptrs[] = {s->d_vx, s->d_vy, s->d_nbr, s->d_info, s->d_ops, s->d_flags, s->d_list, s->d_count,
                    s->d_status, s->d_tstats, s->d_compact, s->d_partial, s->d_dt, s->d_T1, s->d_T2,
                    s->d_slot, s->d_contrib, s->d_V, s->d_inst_off, s->d_inst_hmin, s->d_amax, s->d_inflow, s->d_lfa, s->d_time, s->d_shock, s->d_tvb};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    s->d_vx = s->d_vy = nullptr;
    s->d_nbr = nullptr;
    s->d_info = nullptr;
    s->d_ops = nullptr;
    s->d_flags = nullptr;
    s->d_list = nullptr;
    s->d_count = s->d_status = nullptr;
    s->d_tstats = nullptr;
    s->d_compact = s->d_partial = s->d_dt = nullptr;
    s->d_T1 = s->d_T2 = nullptr;
    s->d_slot = nullptr;
    s->d_contrib = nullptr;
    s->d_V = nullptr;
    s->d_inst_off = nullptr;
    s->d_inst_hmin = nullptr;
    s->d_amax = nullptr;
    s->d_inflow = nullptr;
    s->d_lfa = nullptr;
    s->d_time = nullptr;
    s->d_shock = nullptr;
    s->d_tvb = nullptr;
    s->shock_set = false;
    s->n_special = 0;
    s->n_inst = 1;
    s->inst_off.clear();
    s->inst_hmin.clear();
    s->has_mesh = false;
}

template <class F>
hipError_t timed(cswdg_solver* s, int kid, F&& f) {
    if (!s->prof || !((s->prof_mask >> kid) & 1u) || s->ev_used + 2 > s->ev_pool.size()) return f();
    size_t i = s->ev_used;
    s->ev_used += 2;
    (void)hipEventRecord(s->ev_pool[i], s->stream);
    hipError_t r = f();
    (void)hipEventRecord(s->ev_pool[i + 1], s->stream);
    s->recs.push_back({kid, i});
    return r;
}

int check_ready(cswdg_solver* s) {
    if (!s) return fail(nullptr, CSWDG_EINVAL, "null solver");
    if (!s->has_mesh) return fail(s, CSWDG_ESTATE, "no mesh uploaded");
    if (hipSetDevice(s->device) != hipSuccess) return fail(s, CSWDG_EHIP, "hipSetDevice failed");
    return CSWDG_OK;
}

// the adjoint's tape holds one dt: single-instance FP64 solvers only
int check_single(cswdg_solver* s) {
    if (s->n_inst != 1) return fail(s, CSWDG_EINVAL, "adjoint calls take a single-instance mesh");
    if (s->p.precision != 0) return fail(s, CSWDG_EINVAL, "adjoint calls take an FP64 solver");
    if (s->p.char_mode != 0 || s->p.weights_mode != 0)
        return fail(s, CSWDG_EINVAL, "adjoint calls take the default limiter readings (char_mode = weights_mode = 0)");
    if (s->n_special != 0) return fail(s, CSWDG_EINVAL, "adjoint calls take meshes without wall or inflow faces");
    if (s->p.positivity != 0) return fail(s, CSWDG_EINVAL, "adjoint calls take solvers without the positivity scaling");
    if (s->p.lf_mode != 0) return fail(s, CSWDG_EINVAL, "adjoint calls take the local Lax-Friedrichs flux (lf_mode = 0)");
    if (s->p.indicator != 0) return fail(s, CSWDG_EINVAL, "adjoint calls take the KXRCF indicator (indicator = 0)");
    if (s->p.gamma_mode != 0) return fail(s, CSWDG_EINVAL, "adjoint calls take the linear weights (1/h)^(l-1) (gamma_mode = 0)");
    if (s->p.ghost_mode != 0) return fail(s, CSWDG_EINVAL, "adjoint calls take the mirror ghost (ghost_mode = 0)");
    if (s->p.reconstruction != 0)
        return fail(s, CSWDG_EINVAL, "adjoint calls take the hierarchical reconstruction (reconstruction = 0)");
    if (s->ctx.qtop == kTopSextic) return fail(s, CSWDG_EINVAL, "adjoint calls do not take the sextic top (p2_top = 5)");
    if (s->p.beta_mode != 0) return fail(s, CSWDG_EINVAL, "adjoint calls take the smoothness indicators of q_l (beta_mode = 0)");
    return CSWDG_OK;
}

// The wide residual schedule (all loops unrolled) needs more than the 512
// registers of a wave for P3 Euler and spills; that build has produced NaN
// in some elements, so the schedule is not offered there.
bool wide_offered(const cswdg_params& p) { return !(p.equation == CSWDG_EQ_EULER && p.degree == 3); }
// the matrix-core residual is laid out for the P2 rules in FP64
bool matrix_offered(const cswdg_params& p) { return p.degree == 2 && p.precision == 0; }

size_t elem_bytes(const cswdg_solver* s) { return s->p.precision == 1 ? sizeof(float) : sizeof(double); }

// limit `buf` in place: troubled list from mask or KXRCF, limiter reading
// `src` (the pre-limit field), scatter into buf
// The limiter's per-call scratch: troubled-list counters, list, compact
// results (the solver's own buffers, or the static array of the
// allocation-free entry point).
struct LimScratch {
    uint32_t* count;
    int32_t* list;
    double* compact;
};

LimScratch solver_scratch(cswdg_solver* s) { return {s->d_count, s->d_list, s->d_compact}; }

// limit `buf` in place: troubled list from mask or KXRCF, limiter reading
// `src` (the pre-limit field), scatter into buf.  Launches are timed through
// the solver's event pool unless untimed is set (the allocation-free path).
int limit_into_with(cswdg_solver* s, const LimScratch& w, const void* src, void* buf, uint8_t* flags_out,
                    const uint8_t* mask, int mode, bool count_zeroed, bool untimed) {
    hipError_t e;
    const int K = (int)s->mesh.K;
    if (mode == CSWDG_LIMIT_NONE) return CSWDG_OK;
    uint8_t* flags = flags_out ? flags_out : s->d_flags;
    auto run = [&](int kid, auto&& f) { return untimed ? f() : timed(s, kid, f); };
    if (!count_zeroed) {
        e = run(KID_ZERO, [&] { return launch_zero_u32(s->ctx, w.count, kCountWords); });
        if (e != hipSuccess) return hipfail(s, e, "zero");
    }
    if (mask || mode == CSWDG_LIMIT_ALL) {
        e = run(KID_COMPACT, [&] { return launch_compact_mask(s->ctx, K, mask, flags, w.list, w.count); });
    } else {
        e = run(KID_KXRCF, [&] { return launch_kxrcf(s->ctx, s->dm, src, flags, nullptr, w.list, w.count); });
    }
    if (e != hipSuccess) return hipfail(s, e, "troubled-cell list");
    e = run(KID_LIMITER, [&] {
        return launch_limiter(s->ctx, s->dm, src, s->d_ops, w.list, w.count, w.compact, s->d_status, K);
    });
    if (e != hipSuccess) return hipfail(s, e, "limiter");
    e = run(KID_SCATTER, [&] { return launch_scatter(s->ctx, K, buf, w.list, w.count, w.compact, K, s->d_tstats); });
    if (e != hipSuccess) return hipfail(s, e, "scatter");
    return CSWDG_OK;
}

int limit_into(cswdg_solver* s, const void* src, void* buf, uint8_t* flags_out, const uint8_t* mask,
               int mode, bool count_zeroed) {
    return limit_into_with(s, solver_scratch(s), src, buf, flags_out, mask, mode, count_zeroed, false);
}

// the global Lax-Friedrichs constants of u, for a residual of u (lf_mode = 1)
hipError_t lf_prepare(cswdg_solver* s, const void* u) {
    if (!s->p.lf_mode) return hipSuccess;
    return timed(s, KID_DT, [&] { return launch_lf_alpha(s->ctx, s->dm, u, s->d_amax, s->d_lfa, s->d_status); });
}

int rk_stage_impl(cswdg_solver* s, int stage, const void* u_n, const void* u_prev, void* out, const double* dt) {
    hipError_t e = lf_prepare(s, u_prev);
    if (e != hipSuccess) return hipfail(s, e, "Lax-Friedrichs constant");
    e = timed(s, KID_RESIDUAL, [&] {
        return launch_residual_reset(s->ctx, s->dm, stage, u_prev, u_n, out, dt, s->d_count);
    });
    if (e != hipSuccess) return hipfail(s, e, "residual");
    int rc = limit_into(s, out, out, nullptr, nullptr, s->p.limiter_mode, true);
    if (rc || !s->p.positivity) return rc;
    e = timed(s, KID_POSITIVITY, [&] { return launch_positivity(s->ctx, s->dm, out, s->d_status); });
    if (e != hipSuccess) return hipfail(s, e, "positivity");
    return CSWDG_OK;
}

struct TapeView {
    double* st[6];  // u0, w1, u1, w2, u2, w3
    uint8_t* mask[3];
    double* dt;
};

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

size_t tape_bytes(const cswdg_solver* s) {
    const size_t sb = round256(sizeof(double) * s->state_elems);
    const size_t mb = round256((size_t)s->mesh.K);
    return 6 * sb + 3 * mb + 256;
}

TapeView tape_view(const cswdg_solver* s, void* tape) {
    TapeView v;
    char* p = (char*)tape;
    const size_t sb = round256(sizeof(double) * s->state_elems);
    const size_t mb = round256((size_t)s->mesh.K);
    for (int i = 0; i < 6; ++i) v.st[i] = (double*)(p + i * sb);
    for (int i = 0; i < 3; ++i) v.mask[i] = (uint8_t*)(p + 6 * sb + i * mb);
    v.dt = (double*)(p + 6 * sb + 3 * mb);
    return v;
}

// Test hook: CSWDG_FAIL_ADJOINT_ALLOC=i (1..3) makes the allocation of the
// i-th adjoint buffer fail, so that the recovery below can be exercised.
bool adjoint_alloc_fails(int i) {
    const char* v = std::getenv("CSWDG_FAIL_ADJOINT_ALLOC");
    return v != nullptr && std::atoi(v) == i + 1;
}

// The three adjoint buffers are allocated together: on any failure the ones
// that were allocated are freed and all three reset, so a later call retries
// from scratch instead of launching with a missing buffer.
int ensure_adjoint_scratch(cswdg_solver* s) {
    if (s->d_slot && s->d_contrib && s->d_V) return CSWDG_OK;
    const size_t K = (size_t)s->mesh.K;
    void** bufs[3] = {(void**)&s->d_slot, (void**)&s->d_contrib, (void**)&s->d_V};
    const size_t bytes[3] = {sizeof(int32_t) * K, sizeof(double) * 4 * s->state_elems,
                             sizeof(double) * s->state_elems};
    bool ok = true;
    for (int i = 0; i < 3 && ok; ++i) {
        if (*bufs[i]) continue;
        ok = !adjoint_alloc_fails(i) && hipMalloc(bufs[i], bytes[i]) == hipSuccess;
        if (!ok) *bufs[i] = nullptr;
    }
    if (!ok) {
        for (int i = 0; i < 3; ++i) {
            if (*bufs[i]) (void)hipFree(*bufs[i]);
            *bufs[i] = nullptr;
        }
        return fail(s, CSWDG_ENOMEM, "adjoint scratch allocation failed");
    }
    return CSWDG_OK;
}

// wbar = Lambda'(w)^T ybar with the troubled set given by mask
int limiter_vjp_impl(cswdg_solver* s, const void* w, const uint8_t* mask, const void* ybar, void* wbar) {
    const int K = (int)s->mesh.K;
    hipError_t e = launch_zero_u32(s->ctx, s->d_count, kCountWords);
    if (e == hipSuccess) e = launch_compact_slots(s->ctx, K, mask, s->d_list, s->d_slot, s->d_count);
    if (e == hipSuccess)
        e = timed(s, KID_LIMITER_VJP, [&] {
            return launch_limiter_vjp(s->ctx, s->dm, w, s->d_ops, s->d_list, s->d_count, ybar, s->d_contrib, K);
        });
    if (e == hipSuccess)
        e = launch_limiter_gather(s->ctx, s->dm, mask, s->d_slot, s->d_contrib, ybar, wbar);
    return e == hipSuccess ? CSWDG_OK : hipfail(s, e, "limiter vjp");
}

int upload_mesh(cswdg_solver* s);

}  // namespace

extern "C" {

int cswdg_create(const cswdg_params* params, void* hip_stream, cswdg_solver** out) {
    if (!params || !out) return fail(nullptr, CSWDG_EINVAL, "null argument");
    *out = nullptr;
    cswdg_params p = *params;
    if (p.equation != CSWDG_EQ_BURGERS && p.equation != CSWDG_EQ_EULER)
        return fail(nullptr, CSWDG_EINVAL, "equation must be CSWDG_EQ_BURGERS or CSWDG_EQ_EULER");
    if (p.degree < 1 || p.degree > 3) return fail(nullptr, CSWDG_EINVAL, "degree must be 1, 2 or 3");
    if (p.precision != 0 && p.precision != 1) return fail(nullptr, CSWDG_EINVAL, "precision must be 0 (FP64) or 1 (FP32-bulk)");
    if (p.limiter_mode < 0 || p.limiter_mode > 2) return fail(nullptr, CSWDG_EINVAL, "bad limiter_mode");
    if (p.kxrcf_norm < 0 || p.kxrcf_norm > 1 || p.char_mode < 0 || p.char_mode > 1 || p.weights_mode < 0 ||
        p.weights_mode > 1)
        return fail(nullptr, CSWDG_EINVAL, "kxrcf_norm, char_mode and weights_mode must be 0 or 1");
    if (p.positivity < 0 || p.positivity > 1) return fail(nullptr, CSWDG_EINVAL, "positivity must be 0 or 1");
    if (p.lf_mode < 0 || p.lf_mode > 1) return fail(nullptr, CSWDG_EINVAL, "lf_mode must be 0 or 1");
    if (p.p2_top < 0 || p.p2_top > 5) return fail(nullptr, CSWDG_EINVAL, "p2_top must be 0..5");
    if (p.p2_top == 5 && p.degree != 3) return fail(nullptr, CSWDG_EINVAL, "p2_top = 5 (the sextic top) is for degree 3");
    if (p.indicator != CSWDG_INDICATOR_KXRCF && p.indicator != CSWDG_INDICATOR_TVB)
        return fail(nullptr, CSWDG_EINVAL, "indicator must be CSWDG_INDICATOR_KXRCF or CSWDG_INDICATOR_TVB");
    if (!(p.tvb_m >= 0.0) || !std::isfinite(p.tvb_m))
        return fail(nullptr, CSWDG_EINVAL, "tvb_m must be finite and >= 0");
    if (p.gamma_mode < 0 || p.gamma_mode > 1) return fail(nullptr, CSWDG_EINVAL, "gamma_mode must be 0 or 1");
    if (p.ghost_mode < 0 || p.ghost_mode > 1) return fail(nullptr, CSWDG_EINVAL, "ghost_mode must be 0 or 1");
    if (p.reconstruction < 0 || p.reconstruction > 3) return fail(nullptr, CSWDG_EINVAL, "reconstruction must be 0, 1, 2 or 3");
    if (p.reconstruction == 2 && (p.degree != 2 || p.ghost_mode != 0))
        return fail(nullptr, CSWDG_EINVAL, "the type-II reconstruction takes N = 2 and the mirror ghost (ghost_mode = 0)");
    if (p.reconstruction == 3 && (p.degree != 2 || p.ghost_mode != 0))
        return fail(nullptr, CSWDG_EINVAL, "the mixed reconstruction takes N = 2 and the mirror ghost (ghost_mode = 0)");
    if (p.beta_mode < 0 || p.beta_mode > 1) return fail(nullptr, CSWDG_EINVAL, "beta_mode must be 0 or 1");
    if (p.beta_mode == 1 && p.reconstruction != 0)
        return fail(nullptr, CSWDG_EINVAL, "beta_mode = 1 is a reading of the hierarchical reconstruction (reconstruction = 0)");
    if (p.reconstruction == 1 && (p.degree > 2 || p.ghost_mode != 0))
        return fail(nullptr, CSWDG_EINVAL, "the type-I reconstruction takes N = 1, 2 and the mirror ghost (ghost_mode = 0)");
    if (p.positivity && p.equation != CSWDG_EQ_EULER)
        return fail(nullptr, CSWDG_EINVAL, "the positivity scaling is defined for the Euler equations");
    if (!(p.gas_gamma > 0)) p.gas_gamma = 1.4;
    if (!(p.cfl > 0)) p.cfl = 0.3 / (2 * p.degree + 1);
    if (!(p.c_k > 0)) p.c_k = 1.0;
    if (!(p.eps_weno > 0)) p.eps_weno = 1e-10;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, CSWDG_EHIP, "hipGetDevice failed (no GPU?)");
    {
        std::lock_guard<std::mutex> lk(g_dev_mutex);
        if (std::find(g_dev_tables.begin(), g_dev_tables.end(), dev) == g_dev_tables.end()) {
            int rc = upload_tables_device();
            if (rc != CSWDG_OK) return fail(nullptr, rc, "constant table upload failed");
            rc = init_noalloc_scratch();
            if (rc != CSWDG_OK) return fail(nullptr, rc, "address of the allocation-free scratch not available");
            g_dev_tables.push_back(dev);
        }
    }
    cswdg_solver* s = new (std::nothrow) cswdg_solver();
    if (!s) return fail(nullptr, CSWDG_ENOMEM, "out of host memory");
    s->p = p;
    s->stream = (hipStream_t)hip_stream;
    s->device = dev;
    s->M = p.equation == CSWDG_EQ_EULER ? 4 : 1;
    s->NP = n_modes(p.degree);
    s->ctx.stream = s->stream;
    s->ctx.eq = p.equation;
    s->ctx.N = p.degree;
    s->ctx.precision = p.precision;
    s->ctx.gamma = p.gas_gamma;
    s->ctx.cfl = p.cfl;
    s->ctx.c_k = p.c_k;
    s->ctx.eps = p.eps_weno;
    // schedule choice for the residual kernel (a tuning knob; same results)
    const char* rv = std::getenv("CSWDG_RESIDUAL_VARIANT");
    s->ctx.residual_variant = rv ? std::atoi(rv) : 3;
    if (s->ctx.residual_variant == 1 && !wide_offered(p)) s->ctx.residual_variant = 3;
    if (s->ctx.residual_variant == 4 && !matrix_offered(p)) s->ctx.residual_variant = 3;
    if (s->ctx.residual_variant < 0 || s->ctx.residual_variant > 4) s->ctx.residual_variant = 3;
    s->ctx.residual_block = 128;
    s->ctx.kxrcf_rms = p.kxrcf_norm;
    s->ctx.char_comp = p.char_mode;
    s->ctx.weights_linear = p.weights_mode;
    s->ctx.qtop = top_for(p.degree, p.p2_top);
    s->ctx.recon = p.reconstruction;
    s->ctx.beta_lit = p.beta_mode;
    s->ctx.indicator = p.indicator;
    s->ctx.tvb_m = p.tvb_m;
    *out = s;
    return CSWDG_OK;
}

int cswdg_destroy(cswdg_solver* s) {
    if (!s) return CSWDG_OK;
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    free_mesh(s);
    for (hipEvent_t ev : s->ev_pool) (void)hipEventDestroy(ev);
    delete s;
    return CSWDG_OK;
}

const char* cswdg_last_error(const cswdg_solver* s) { return s ? s->err.c_str() : g_err.c_str(); }

int cswdg_host_connectivity(int64_t nv, const double* vxy, int64_t nt, const int32_t* tri, int bc, double px,
                            double py, int32_t* tri_ccw, int32_t* nbr, uint8_t* info) {
    if (!tri_ccw || !nbr || !info) return fail(nullptr, CSWDG_EINVAL, "null output");
    HostMesh m;
    std::string msg;
    int rc = build_mesh(nv, vxy, nt, tri, bc, px, py, m, msg);
    if (rc != CSWDG_OK) return fail(nullptr, rc, msg);
    std::memcpy(tri_ccw, m.tri.data(), sizeof(int32_t) * 3 * nt);
    std::memcpy(nbr, m.nbr.data(), sizeof(int32_t) * 3 * nt);
    std::memcpy(info, m.info.data(), 3 * nt);
    return CSWDG_OK;
}

int cswdg_host_tvb_decomposition(int64_t nv, const double* vxy, int64_t nt, const int32_t* tri, int bc,
                                 double px, double py, double* A, int64_t* n_neg) {
    if (!A) return fail(nullptr, CSWDG_EINVAL, "null output");
    HostMesh m;
    std::string msg;
    int rc = build_mesh(nv, vxy, nt, tri, bc, px, py, m, msg);
    if (rc != CSWDG_OK) return fail(nullptr, rc, msg);
    std::vector<double> soa;
    int64_t neg = 0;
    build_tvb_ops(m, soa, neg);
    for (int64_t e = 0; e < nt; ++e)
        for (int r = 0; r < 9; ++r) A[9 * e + r] = soa[(size_t)r * nt + e];
    if (n_neg) *n_neg = neg;
    return CSWDG_OK;
}

int cswdg_mesh_upload(cswdg_solver* s, int64_t nv, const double* vxy, int64_t nt, const int32_t* tri, int bc,
                      double px, double py) {
    if (!s) return fail(nullptr, CSWDG_EINVAL, "null solver");
    if (hipSetDevice(s->device) != hipSuccess) return fail(s, CSWDG_EHIP, "hipSetDevice failed");
    (void)hipStreamSynchronize(s->stream);
    free_mesh(s);
    std::string msg;
    int rc = build_mesh(nv, vxy, nt, tri, bc, px, py, s->mesh, msg);
    if (rc != CSWDG_OK) return fail(s, rc, msg);
    s->n_inst = 1;
    s->inst_off = {0, (int32_t)s->mesh.K};
    s->inst_hmin = {s->mesh.hmin};
    return upload_mesh(s);
}

int cswdg_mesh_upload_batch(cswdg_solver* s, int32_t n_inst, const int64_t* nv, const double* vxy,
                            const int64_t* nt, const int32_t* tri, const int32_t* bc, double px, double py) {
    if (!s) return fail(nullptr, CSWDG_EINVAL, "null solver");
    if (n_inst < 1 || !nv || !vxy || !nt || !tri || !bc) return fail(s, CSWDG_EINVAL, "bad batch arguments");
    if (hipSetDevice(s->device) != hipSuccess) return fail(s, CSWDG_EHIP, "hipSetDevice failed");
    (void)hipStreamSynchronize(s->stream);
    free_mesh(s);
    std::vector<HostMesh> parts((size_t)n_inst);
    std::string msg;
    int64_t vo = 0, to = 0;
    for (int32_t i = 0; i < n_inst; ++i) {
        if (nv[i] < 3 || nt[i] < 1) return fail(s, CSWDG_EINVAL, "instance " + std::to_string(i) + ": empty mesh");
        int rc = build_mesh(nv[i], vxy + 2 * vo, nt[i], tri + 3 * to, bc[i], px, py, parts[i], msg);
        if (rc != CSWDG_OK) return fail(s, rc, "instance " + std::to_string(i) + ": " + msg);
        vo += nv[i];
        to += nt[i];
        if (to > kMaxTriangles)
            return fail(s, CSWDG_EINVAL, "batch: more than 715,827,882 triangles in all (32-bit element indices)");
    }
    int rc = concat_meshes(parts, s->mesh, s->inst_off, s->inst_hmin, msg);
    if (rc != CSWDG_OK) return fail(s, rc, msg);
    parts.clear();
    s->n_inst = n_inst;
    return upload_mesh(s);
}

int cswdg_instances(const cswdg_solver* s, int32_t* n_inst, int64_t* offsets) {
    if (!s || !s->has_mesh) return fail(const_cast<cswdg_solver*>(s), CSWDG_ESTATE, "no mesh uploaded");
    if (!n_inst) return fail(const_cast<cswdg_solver*>(s), CSWDG_EINVAL, "null pointer");
    *n_inst = s->n_inst;
    if (offsets)
        for (int i = 0; i <= s->n_inst; ++i) offsets[i] = s->inst_off[i];
    return CSWDG_OK;
}

int cswdg_set_boundary(cswdg_solver* s, const uint8_t* kinds, const double* inflow) {
    int rc = check_ready(s);
    if (rc) return rc;
    const int64_t K = s->mesh.K;
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hipfail(s, e, "set_boundary");
    if (kinds) {
        int64_t special = 0;
        for (int64_t i = 0; i < 3 * K; ++i) {
            if (!(s->mesh.info[i] & 0x40)) continue;
            if (kinds[i] > 3)
                return fail(s, CSWDG_EINVAL, "boundary kind must be 0 (outflow), 1 (wall), 2 (inflow) or 3 (moving shock)");
            if (kinds[i] == 3 && !s->shock_set)
                return fail(s, CSWDG_EINVAL, "boundary kind 3 needs cswdg_set_moving_shock first");
            special += kinds[i] != 0;
        }
        std::vector<uint32_t> info4(K);
        for (int64_t el = 0; el < K; ++el) {
            uint32_t w = 0;
            for (int f = 0; f < 3; ++f) {
                uint8_t& b = s->mesh.info[3 * el + f];
                if (b & 0x40) b = (uint8_t)(0x40 | kinds[3 * el + f]);
                w |= (uint32_t)b << (8 * f);
            }
            info4[el] = w;
        }
        e = hipMemcpy(s->d_info, info4.data(), sizeof(uint32_t) * K, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hipfail(s, e, "set_boundary");
        s->n_special = special;
        if (s->p.ghost_mode == 1) {
            // the outflow faces' ghosts differ from the walls': rebuild the
            // stencil operators for the new kinds
            std::vector<double> ops;
            rc = build_limiter_ops(s->mesh, s->p.degree, s->ctx.qtop, s->p.gamma_mode == 1, true, ops, s->n_rank, s->n_foot);
            if (rc != CSWDG_OK) return fail(s, rc, "limiter operator build failed");
            e = hipMemcpy(s->d_ops, ops.data(), sizeof(double) * ops.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) return hipfail(s, e, "set_boundary");
        }
    }
    if (inflow) {
        e = hipMemcpy(s->d_inflow, inflow, sizeof(double) * s->M, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hipfail(s, e, "set_boundary");
    }
    return CSWDG_OK;
}

int cswdg_set_moving_shock(cswdg_solver* s, const double* post, const double* pre, double nx, double ny, double d0,
                           double speed) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (s->p.equation != CSWDG_EQ_EULER) return fail(s, CSWDG_EINVAL, "the moving-shock boundary is an Euler boundary");
    if (!post || !pre) return fail(s, CSWDG_EINVAL, "null state");
    if (!std::isfinite(nx) || !std::isfinite(ny) || !std::isfinite(d0) || !std::isfinite(speed))
        return fail(s, CSWDG_EINVAL, "moving shock: non-finite parameter");
    double rec[12] = {nx, ny, d0, speed};
    for (int c = 0; c < 4; ++c) {
        rec[4 + c] = post[c];
        rec[8 + c] = pre[c];
    }
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipMemcpy(s->d_shock, rec, sizeof(rec), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hipfail(s, e, "set_moving_shock");
    s->shock_set = true;
    s->dm.shock = s->d_shock;
    return CSWDG_OK;
}

int cswdg_set_time(cswdg_solver* s, double t) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!std::isfinite(t)) return fail(s, CSWDG_EINVAL, "non-finite time");
    std::vector<double> tv((size_t)s->n_inst, t);
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipMemcpy(s->d_time, tv.data(), sizeof(double) * tv.size(), hipMemcpyHostToDevice);
    return e == hipSuccess ? CSWDG_OK : hipfail(s, e, "set_time");
}

int cswdg_time(cswdg_solver* s, double* t) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!t) return fail(s, CSWDG_EINVAL, "null pointer");
    hipError_t e = hipMemcpyAsync(t, s->d_time, sizeof(double) * s->n_inst, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    return e == hipSuccess ? CSWDG_OK : hipfail(s, e, "time");
}

int cswdg_mesh_info(const cswdg_solver* s, int64_t* n_elements, int64_t* n_flipped) {
    if (!s || !s->has_mesh) return fail(const_cast<cswdg_solver*>(s), CSWDG_ESTATE, "no mesh uploaded");
    if (n_elements) *n_elements = s->mesh.K;
    if (n_flipped) *n_flipped = s->mesh.n_flipped;
    return CSWDG_OK;
}

int cswdg_connectivity(const cswdg_solver* s, int32_t* nbr, uint8_t* info) {
    if (!s || !s->has_mesh) return fail(const_cast<cswdg_solver*>(s), CSWDG_ESTATE, "no mesh uploaded");
    if (!nbr || !info) return fail(const_cast<cswdg_solver*>(s), CSWDG_EINVAL, "null output");
    std::memcpy(nbr, s->mesh.nbr.data(), sizeof(int32_t) * 3 * s->mesh.K);
    std::memcpy(info, s->mesh.info.data(), 3 * s->mesh.K);
    return CSWDG_OK;
}

int cswdg_stencil(const cswdg_solver* s, int32_t elem, int32_t* ids, int32_t* n) {
    if (!s || !s->has_mesh) return fail(const_cast<cswdg_solver*>(s), CSWDG_ESTATE, "no mesh uploaded");
    if (!ids || !n || elem < 0 || elem >= s->mesh.K) return fail(const_cast<cswdg_solver*>(s), CSWDG_EINVAL, "bad element");
    for (int f = 0; f < 3; ++f) {
        uint8_t inf = s->mesh.info[3 * elem + f];
        if (inf & 0x40) {
            ids[4 * f] = -1;
            ids[4 * f + 1] = ids[4 * f + 2] = ids[4 * f + 3] = 0;
        } else {
            ids[4 * f] = s->mesh.nbr[3 * elem + f];
            ids[4 * f + 1] = inf & 3;
            ids[4 * f + 2] = (inf >> 2) & 3;
            ids[4 * f + 3] = (inf >> 4) & 3;
        }
    }
    *n = 12;
    return CSWDG_OK;
}

int cswdg_ic_points(cswdg_solver* s, double* xy, int32_t* nq) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!nq) return fail(s, CSWDG_EINVAL, "null nq");
    *nq = ic_points_per_element(s->p.degree);
    if (!xy) return CSWDG_OK;
    hipError_t e = launch_ic_points(s->ctx, s->dm, xy);
    return e == hipSuccess ? CSWDG_OK : hipfail(s, e, "ic_points");
}

int cswdg_project(cswdg_solver* s, const double* vals, void* u) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!vals || !u) return fail(s, CSWDG_EINVAL, "null pointer");
    hipError_t e = timed(s, KID_PROJECT, [&] { return launch_project(s->ctx, s->dm, vals, u); });
    return e == hipSuccess ? CSWDG_OK : hipfail(s, e, "project");
}

int cswdg_dg_residual(cswdg_solver* s, const void* u, void* r) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!u || !r || u == r) return fail(s, CSWDG_EINVAL, "u and r must be distinct non-null buffers");
    hipError_t e = lf_prepare(s, u);
    if (e == hipSuccess)
        e = timed(s, KID_RESIDUAL, [&] { return launch_residual_reset(s->ctx, s->dm, 0, u, nullptr, r, nullptr, nullptr); });
    return e == hipSuccess ? CSWDG_OK : hipfail(s, e, "residual");
}

int cswdg_max_dt(cswdg_solver* s, const void* u, double* dt_dev) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!u || !dt_dev) return fail(s, CSWDG_EINVAL, "null pointer");
    int nb = std::min(s->dt_blocks, (int)((s->mesh.K + 255) / 256));
    if (nb < 1) nb = 1;
    hipError_t e = timed(s, KID_DT, [&] {
        if (s->n_inst > 1)
            return launch_max_dt_inst(s->ctx, s->dm, u, s->d_inst_hmin, dt_dev, s->d_amax, s->d_status);
        return launch_max_dt(s->ctx, s->dm, u, s->mesh.hmin, dt_dev, s->d_partial, nullptr, s->d_status, nb);
    });
    return e == hipSuccess ? CSWDG_OK : hipfail(s, e, "max_dt");
}

int cswdg_kxrcf(cswdg_solver* s, const void* u, uint8_t* flags, double* R) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!u || !flags) return fail(s, CSWDG_EINVAL, "null pointer");
    hipError_t e = timed(s, KID_ZERO, [&] { return launch_zero_u32(s->ctx, s->d_count, kCountWords); });
    if (e == hipSuccess)
        e = timed(s, KID_KXRCF, [&] { return launch_kxrcf(s->ctx, s->dm, u, flags, R, s->d_list, s->d_count); });
    return e == hipSuccess ? CSWDG_OK : hipfail(s, e, "kxrcf");
}

int cswdg_csweno_limit(cswdg_solver* s, const void* u_in, void* u_out, uint8_t* flags_out, const uint8_t* mask_in) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!u_in || !u_out || u_in == u_out) return fail(s, CSWDG_EINVAL, "u_in and u_out must be distinct non-null buffers");
    const size_t bytes = elem_bytes(s) * s->state_elems;
    hipError_t e = timed(s, KID_COPY, [&] { return hipMemcpyAsync(u_out, u_in, bytes, hipMemcpyDeviceToDevice, s->stream); });
    if (e != hipSuccess) return hipfail(s, e, "copy");
    int mode = mask_in ? CSWDG_LIMIT_KXRCF : (s->p.limiter_mode == CSWDG_LIMIT_ALL ? CSWDG_LIMIT_ALL : CSWDG_LIMIT_KXRCF);
    return limit_into(s, u_in, u_out, flags_out, mask_in, mode, false);
}

int cswdg_csweno_limit_noalloc(cswdg_solver* s, const void* u_in, void* u_out, uint8_t* flags_out,
                               const uint8_t* mask_in) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!u_in || !u_out || u_in == u_out) return fail(s, CSWDG_EINVAL, "u_in and u_out must be distinct non-null buffers");
    const size_t K = (size_t)s->mesh.K;
    // the troubled list has kListSegs segments of capacity K (as the
    // solver's own list), the compact results one row per element
    const size_t compact_off = (kNoAllocListOffset + sizeof(int32_t) * K * kListSegs + 255) / 256 * 256;
    const size_t need = compact_off + sizeof(double) * K * (size_t)s->M * (size_t)s->NP;
    if (need > kNoAllocScratchBytes)
        return fail(s, CSWDG_EINVAL,
                    "mesh too large for the allocation-free limiter: it needs " + std::to_string(need) +
                        " bytes of scratch, the static array holds " + std::to_string(kNoAllocScratchBytes));
    unsigned char* base = (unsigned char*)noalloc_scratch(s->device);
    if (!base) return fail(s, CSWDG_ESTATE, "allocation-free scratch not initialised on this device");
    const LimScratch w = {(uint32_t*)base, (int32_t*)(base + kNoAllocListOffset), (double*)(base + compact_off)};
    const size_t bytes = elem_bytes(s) * s->state_elems;
    hipError_t e = hipMemcpyAsync(u_out, u_in, bytes, hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return hipfail(s, e, "copy");
    int mode = mask_in ? CSWDG_LIMIT_KXRCF : (s->p.limiter_mode == CSWDG_LIMIT_ALL ? CSWDG_LIMIT_ALL : CSWDG_LIMIT_KXRCF);
    return limit_into_with(s, w, u_in, u_out, flags_out, mask_in, mode, false, true);
}

int cswdg_rk_stage(cswdg_solver* s, int stage, const void* u_n, const void* u_prev, void* out, const double* dt_dev) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (stage < 1 || stage > 3) return fail(s, CSWDG_EINVAL, "stage must be 1, 2 or 3");
    if (!u_prev || !out || !dt_dev || (stage > 1 && !u_n)) return fail(s, CSWDG_EINVAL, "null pointer");
    if (out == u_prev) return fail(s, CSWDG_EINVAL, "out must not alias u_prev");
    return rk_stage_impl(s, stage, u_n, u_prev, out, dt_dev);
}

int cswdg_ssprk3_step(cswdg_solver* s, void* u, const double* dt_dev) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!u) return fail(s, CSWDG_EINVAL, "null state");
    const double* dt = dt_dev;
    if (!dt) {
        rc = cswdg_max_dt(s, u, s->d_dt);
        if (rc) return rc;
        dt = s->d_dt;
    }
    rc = rk_stage_impl(s, 1, nullptr, u, s->d_T1, dt);
    if (rc) return rc;
    rc = rk_stage_impl(s, 2, u, s->d_T1, s->d_T2, dt);
    if (rc) return rc;
    rc = rk_stage_impl(s, 3, u, s->d_T2, u, dt);
    if (rc || !s->shock_set) return rc;
    hipError_t e = launch_time_advance(s->ctx, s->n_inst, s->d_time, dt);
    return e == hipSuccess ? CSWDG_OK : hipfail(s, e, "time advance");
}

int cswdg_positivity(cswdg_solver* s, void* u) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!u) return fail(s, CSWDG_EINVAL, "null state");
    if (s->p.equation != CSWDG_EQ_EULER) return fail(s, CSWDG_EINVAL, "the positivity scaling is defined for the Euler equations");
    hipError_t e = timed(s, KID_POSITIVITY, [&] { return launch_positivity(s->ctx, s->dm, u, s->d_status); });
    if (e != hipSuccess) return hipfail(s, e, "positivity");
    return CSWDG_OK;
}

int cswdg_last_dt(cswdg_solver* s, double** dt_dev) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!dt_dev) return fail(s, CSWDG_EINVAL, "null pointer");
    *dt_dev = s->d_dt;
    return CSWDG_OK;
}

int cswdg_troubled_count(cswdg_solver* s, int64_t* count) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!count) return fail(s, CSWDG_EINVAL, "null pointer");
    uint32_t c[kCountWords];
    hipError_t e = hipMemcpyAsync(c, s->d_count, sizeof(c), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hipfail(s, e, "troubled_count");
    int64_t tot = 0;
    for (int x = 0; x < kListSegs; ++x) tot += std::min<int64_t>(c[x * kCountStride], s->mesh.K);
    *count = tot;
    return CSWDG_OK;
}

int cswdg_troubled_stats(cswdg_solver* s, int64_t* total_cells, int64_t* calls, int reset) {
    int rc = check_ready(s);
    if (rc) return rc;
    unsigned long long v[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(v, s->d_tstats, sizeof(v), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess && reset) {
        unsigned long long zz[2] = {0, 0};
        e = hipMemcpy(s->d_tstats, zz, sizeof(zz), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hipfail(s, e, "troubled_stats");
    if (total_cells) *total_cells = (int64_t)v[0];
    if (calls) *calls = (int64_t)v[1];
    return CSWDG_OK;
}

int cswdg_status(cswdg_solver* s, uint32_t* flags) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!flags) return fail(s, CSWDG_EINVAL, "null pointer");
    uint32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, s->d_status, sizeof(v), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = launch_zero_u32(s->ctx, s->d_status, 1);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hipfail(s, e, "status");
    if (s->n_foot > 0) v |= CSWDG_STATUS_FOOT;
    *flags = v;
    return CSWDG_OK;
}

int cswdg_dg_residual_vjp(cswdg_solver* s, const void* u, const void* r_bar, void* u_bar) {
    int rc = check_ready(s);
    if (rc) return rc;
    rc = check_single(s);
    if (rc) return rc;
    if (!u || !r_bar || !u_bar || u_bar == r_bar) return fail(s, CSWDG_EINVAL, "bad pointers");
    hipError_t e = timed(s, KID_RESIDUAL_VJP, [&] {
        return launch_residual_vjp(s->ctx, s->dm, u, r_bar, u_bar, nullptr, nullptr, 0.0, 0.0, 1.0, 0);
    });
    return e == hipSuccess ? CSWDG_OK : hipfail(s, e, "residual vjp");
}

int cswdg_csweno_limit_vjp(cswdg_solver* s, const void* w, const uint8_t* mask, const void* y_bar, void* w_bar) {
    int rc = check_ready(s);
    if (rc) return rc;
    rc = check_single(s);
    if (rc) return rc;
    if (!w || !y_bar || !w_bar || w_bar == y_bar) return fail(s, CSWDG_EINVAL, "bad pointers");
    rc = ensure_adjoint_scratch(s);
    if (rc) return rc;
    const uint8_t* m = mask;
    if (!m) {
        hipError_t e = launch_zero_u32(s->ctx, s->d_count, kCountWords);
        if (e == hipSuccess) e = launch_kxrcf(s->ctx, s->dm, w, s->d_flags, nullptr, s->d_list, s->d_count);
        if (e != hipSuccess) return hipfail(s, e, "kxrcf");
        m = s->d_flags;
    }
    return limiter_vjp_impl(s, w, m, y_bar, w_bar);
}

int cswdg_tape_bytes(cswdg_solver* s, int64_t* bytes) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!bytes) return fail(s, CSWDG_EINVAL, "null pointer");
    *bytes = (int64_t)tape_bytes(s);
    return CSWDG_OK;
}

int cswdg_ssprk3_step_tape(cswdg_solver* s, void* u, const double* dt_dev, void* tape, int replay) {
    int rc = check_ready(s);
    if (rc) return rc;
    rc = check_single(s);
    if (rc) return rc;
    if (!u || !tape) return fail(s, CSWDG_EINVAL, "null pointer");
    TapeView t = tape_view(s, tape);
    const size_t bytes = sizeof(double) * s->state_elems;
    const int K = (int)s->mesh.K;
    hipError_t e = hipMemcpyAsync(t.st[0], u, bytes, hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return hipfail(s, e, "tape copy");
    if (!replay) {
        if (dt_dev) {
            e = hipMemcpyAsync(t.dt, dt_dev, sizeof(double), hipMemcpyDeviceToDevice, s->stream);
            if (e != hipSuccess) return hipfail(s, e, "dt copy");
        } else {
            rc = cswdg_max_dt(s, u, t.dt);
            if (rc) return rc;
        }
    }
    const double* st_in[3] = {t.st[0], t.st[2], t.st[4]};
    double* st_w[3] = {t.st[1], t.st[3], t.st[5]};
    void* st_out[3] = {t.st[2], t.st[4], u};
    for (int i = 0; i < 3; ++i) {
        e = timed(s, KID_RESIDUAL, [&] {
            return launch_residual_reset(s->ctx, s->dm, i + 1, st_in[i], t.st[0], st_w[i], t.dt, s->d_count);
        });
        if (e == hipSuccess) e = hipMemcpyAsync(st_out[i], st_w[i], bytes, hipMemcpyDeviceToDevice, s->stream);
        if (e != hipSuccess) return hipfail(s, e, "tape stage");
        if (s->p.limiter_mode == CSWDG_LIMIT_NONE) {
            e = launch_zero_u32(s->ctx, (uint32_t*)t.mask[i], (int)(round256((size_t)K) / 4));
            if (e != hipSuccess) return hipfail(s, e, "mask");
            continue;
        }
        if (replay) rc = limit_into(s, st_w[i], st_out[i], nullptr, t.mask[i], CSWDG_LIMIT_KXRCF, true);
        else rc = limit_into(s, st_w[i], st_out[i], t.mask[i], nullptr, s->p.limiter_mode, true);
        if (rc) return rc;
    }
    return CSWDG_OK;
}

int cswdg_ssprk3_step_vjp(cswdg_solver* s, const void* tape, const void* u_next_bar, void* u_n_bar) {
    int rc = check_ready(s);
    if (rc) return rc;
    rc = check_single(s);
    if (rc) return rc;
    if (!tape || !u_next_bar || !u_n_bar || u_n_bar == u_next_bar) return fail(s, CSWDG_EINVAL, "bad pointers");
    rc = ensure_adjoint_scratch(s);
    if (rc) return rc;
    TapeView t = tape_view(s, const_cast<void*>(tape));
    const int nwords = (int)(2 * s->state_elems);  // doubles as pairs of 32-bit words
    hipError_t e = launch_zero_u32(s->ctx, (uint32_t*)u_n_bar, nwords);
    if (e != hipSuccess) return hipfail(s, e, "zero");
    // stage 3: u^{n+1} = Lambda(1/3 u0 + 2/3 (u2 + dt L(u2)))
    rc = limiter_vjp_impl(s, t.st[5], t.mask[2], u_next_bar, s->d_V);
    if (rc) return rc;
    e = timed(s, KID_RESIDUAL_VJP, [&] {
        return launch_residual_vjp(s->ctx, s->dm, t.st[4], s->d_V, s->d_T2, u_n_bar, t.dt, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0, 0);
    });
    if (e != hipSuccess) return hipfail(s, e, "residual vjp");
    // stage 2: u2 = Lambda(3/4 u0 + 1/4 (u1 + dt L(u1)))
    rc = limiter_vjp_impl(s, t.st[3], t.mask[1], s->d_T2, s->d_V);
    if (rc) return rc;
    e = timed(s, KID_RESIDUAL_VJP, [&] {
        return launch_residual_vjp(s->ctx, s->dm, t.st[2], s->d_V, s->d_T2, u_n_bar, t.dt, 0.75, 0.25, 0.25, 0);
    });
    if (e != hipSuccess) return hipfail(s, e, "residual vjp");
    // stage 1: u1 = Lambda(u0 + dt L(u0))
    rc = limiter_vjp_impl(s, t.st[1], t.mask[0], s->d_T2, s->d_V);
    if (rc) return rc;
    e = timed(s, KID_RESIDUAL_VJP, [&] {
        return launch_residual_vjp(s->ctx, s->dm, t.st[0], s->d_V, u_n_bar, nullptr, t.dt, 0.0, 1.0, 1.0, 1);
    });
    return e == hipSuccess ? CSWDG_OK : hipfail(s, e, "residual vjp");
}

int cswdg_set_schedule(cswdg_solver* s, const int32_t* sched) {
    if (!s || !sched) return fail(s, CSWDG_EINVAL, "null argument");
    if (sched[0] < 0 || sched[0] > 4 || (sched[1] != 64 && sched[1] != 128 && sched[1] != 256) ||
        (sched[2] != 0 && sched[2] != 1))
        return fail(s, CSWDG_EINVAL, "schedule: variant 0..4, block 64/128/256, xcd 0/1");
    if (sched[0] == 1 && !wide_offered(s->p))
        return fail(s, CSWDG_EINVAL, "schedule: the wide variant is not offered for P3 Euler");
    if (sched[0] == 4 && !matrix_offered(s->p))
        return fail(s, CSWDG_EINVAL, "schedule: the matrix-core variant is offered for P2 in FP64 only");
    s->ctx.residual_variant = sched[0];
    s->ctx.residual_block = sched[1];
    s->dm.xcd_tiles = sched[2];
    return CSWDG_OK;
}

int cswdg_get_schedule(const cswdg_solver* s, int32_t* sched) {
    if (!s || !sched) return fail(const_cast<cswdg_solver*>(s), CSWDG_EINVAL, "null argument");
    sched[0] = s->ctx.residual_variant;
    sched[1] = s->ctx.residual_block;
    sched[2] = s->dm.xcd_tiles;
    return CSWDG_OK;
}

int cswdg_autotune(cswdg_solver* s, const void* u, int32_t reps, int32_t* sched, double* times_us, int32_t* n_cand) {
    int rc = check_ready(s);
    if (rc) return rc;
    if (!u || reps < 1) return fail(s, CSWDG_EINVAL, "autotune needs a state and reps >= 1");
    const int variants[5] = {0, 1, 2, 3, 4}, blocks[3] = {64, 128, 256}, xcds[2] = {0, 1};
    hipEvent_t ev[2];
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess)
        return fail(s, CSWDG_EHIP, "hipEventCreate failed");
    const bool prof = s->prof;
    s->prof = false;
    const LaunchCtx saved = s->ctx;
    const int saved_xcd = s->dm.xcd_tiles;
    double best = INFINITY;
    int bi = -1, k = 0;
    hipError_t e = lf_prepare(s, u);
    for (int v : variants)
        for (int b : blocks)
            for (int x : xcds) {
                if ((s->p.precision == 1 && v != 3) || (v == 1 && !wide_offered(s->p)) ||
                    (v == 4 && !matrix_offered(s->p))) {
                    // FP32-bulk runs the compact schedule only; P3 Euler has no
                    // wide one; the matrix-core one is P2 FP64
                    if (times_us) times_us[k] = INFINITY;
                    ++k;
                    continue;
                }
                s->ctx.residual_variant = v;
                s->ctx.residual_block = b;
                s->dm.xcd_tiles = x;
                // one untimed launch, then reps timed launches of the residual
                e = launch_residual_reset(s->ctx, s->dm, 0, u, nullptr, s->d_T1, nullptr, nullptr);
                if (e == hipSuccess) e = hipEventRecord(ev[0], s->stream);
                for (int r = 0; r < reps && e == hipSuccess; ++r)
                    e = launch_residual_reset(s->ctx, s->dm, 0, u, nullptr, s->d_T1, nullptr, nullptr);
                if (e == hipSuccess) e = hipEventRecord(ev[1], s->stream);
                if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
                if (e != hipSuccess) break;
                const double us = 1000.0 * ms / reps;
                if (times_us) times_us[k] = us;
                if (us < best) {
                    best = us;
                    bi = k;
                }
                ++k;
            }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    s->prof = prof;
    s->ctx = saved;
    s->dm.xcd_tiles = saved_xcd;
    if (e != hipSuccess) return hipfail(s, e, "autotune");
    if (n_cand) *n_cand = k;
    const int32_t choice[3] = {variants[bi / 6], blocks[(bi / 2) % 3], xcds[bi % 2]};
    if (sched)
        for (int i = 0; i < 3; ++i) sched[i] = choice[i];
    return cswdg_set_schedule(s, choice);
}

int cswdg_graph_capture(int32_t n, cswdg_solver* const* solvers, void* const* states, int32_t nsteps,
                        cswdg_graph** out) {
    if (!out || n < 1 || !solvers || !states || nsteps < 1) return fail(nullptr, CSWDG_EINVAL, "bad capture arguments");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!solvers[i] || !states[i]) return fail(nullptr, CSWDG_EINVAL, "null solver or state");
        int rc = check_ready(solvers[i]);
        if (rc) return rc;
        if (solvers[i]->device != solvers[0]->device) return fail(nullptr, CSWDG_EINVAL, "solvers on different devices");
        for (int j = 0; j < i; ++j)
            if (solvers[j] == solvers[i] || states[j] == states[i])
                return fail(nullptr, CSWDG_EINVAL, "the solvers and their states must be distinct (their branches run concurrently)");
    }
    // capture on private streams of default priority, one per solver: the
    // solvers are independent (own state, own scratch), so each one's steps
    // form a branch of the graph (forked from and joined to the first
    // stream by events) and the branches run concurrently; the members'
    // earlier work is ordered before the capture by a full wait
    std::vector<hipStream_t> cs(n, nullptr);
    std::vector<hipEvent_t> ev(n, nullptr);
    hipError_t e = hipSuccess;
    for (int i = 0; i < n && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&cs[i], hipStreamNonBlocking);
    for (int i = 0; i < n && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
    auto release = [&]() {
        for (int i = 0; i < n; ++i) {
            if (ev[i]) (void)hipEventDestroy(ev[i]);
            if (cs[i]) (void)hipStreamDestroy(cs[i]);
        }
    };
    if (e != hipSuccess) {
        release();
        return fail(nullptr, CSWDG_EHIP, "capture streams");
    }
    for (int i = 0; i < n && e == hipSuccess; ++i) e = hipStreamSynchronize(solvers[i]->stream);
    std::vector<hipStream_t> saved(n);
    std::vector<bool> prof(n);
    for (int i = 0; i < n; ++i) {
        saved[i] = solvers[i]->stream;
        prof[i] = solvers[i]->prof;
        solvers[i]->stream = cs[i];
        solvers[i]->ctx.stream = cs[i];
        solvers[i]->prof = false;
    }
    int rc = CSWDG_OK;
    hipGraph_t graph = nullptr;
    if (e == hipSuccess) e = hipStreamBeginCapture(cs[0], hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        // fork: every other stream joins the capture behind an event of the first
        if (n > 1) e = hipEventRecord(ev[0], cs[0]);
        for (int i = 1; i < n && e == hipSuccess; ++i) e = hipStreamWaitEvent(cs[i], ev[0], 0);
        for (int i = 0; i < n && rc == CSWDG_OK && e == hipSuccess; ++i)
            for (int t = 0; t < nsteps && rc == CSWDG_OK; ++t) rc = cswdg_ssprk3_step(solvers[i], states[i], nullptr);
        // join: the first stream waits for every branch
        for (int i = 1; i < n && e == hipSuccess; ++i) {
            e = hipEventRecord(ev[i], cs[i]);
            if (e == hipSuccess) e = hipStreamWaitEvent(cs[0], ev[i], 0);
        }
        hipError_t e2 = hipStreamEndCapture(cs[0], &graph);
        if (e == hipSuccess) e = e2;
    }
    for (int i = 0; i < n; ++i) {
        solvers[i]->stream = saved[i];
        solvers[i]->ctx.stream = saved[i];
        solvers[i]->prof = prof[i];
    }
    hipGraphExec_t exec = nullptr;
    if (rc == CSWDG_OK && e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    size_t nodes = 0;
    if (rc == CSWDG_OK && e == hipSuccess) e = hipGraphGetNodes(graph, nullptr, &nodes);
    if (graph) (void)hipGraphDestroy(graph);
    release();
    if (rc != CSWDG_OK) {
        if (exec) (void)hipGraphExecDestroy(exec);
        return rc;
    }
    if (e != hipSuccess) {
        if (exec) (void)hipGraphExecDestroy(exec);
        return fail(nullptr, CSWDG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    cswdg_graph* g = new (std::nothrow) cswdg_graph();
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        return fail(nullptr, CSWDG_ENOMEM, "out of host memory");
    }
    g->exec = exec;
    g->device = solvers[0]->device;
    g->nodes = (int64_t)nodes;
    *out = g;
    return CSWDG_OK;
}

int cswdg_graph_launch(cswdg_graph* g, void* hip_stream) {
    if (!g) return fail(nullptr, CSWDG_EINVAL, "null graph");
    if (hipSetDevice(g->device) != hipSuccess) return fail(nullptr, CSWDG_EHIP, "hipSetDevice failed");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)hip_stream);
    return e == hipSuccess ? CSWDG_OK : fail(nullptr, CSWDG_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
}

int cswdg_graph_nodes(const cswdg_graph* g, int64_t* nodes) {
    if (!g || !nodes) return fail(nullptr, CSWDG_EINVAL, "null argument");
    *nodes = g->nodes;
    return CSWDG_OK;
}

int cswdg_graph_destroy(cswdg_graph* g) {
    if (!g) return CSWDG_OK;
    (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();
    (void)hipGraphExecDestroy(g->exec);
    delete g;
    return CSWDG_OK;
}

int cswdg_profile(cswdg_solver* s, int enable) {
    if (!s) return fail(nullptr, CSWDG_EINVAL, "null solver");
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    if (enable && s->ev_pool.empty()) {
        s->ev_pool.resize(1 << 15);
        for (auto& ev : s->ev_pool)
            if (hipEventCreate(&ev) != hipSuccess) return fail(s, CSWDG_EHIP, "hipEventCreate failed");
    }
    s->prof = enable != 0;
    if (enable) {
        s->ev_used = 0;
        s->recs.clear();
    }
    return CSWDG_OK;
}

int cswdg_profile_select(cswdg_solver* s, uint32_t kernel_mask) {
    if (!s) return fail(nullptr, CSWDG_EINVAL, "null solver");
    s->prof_mask = kernel_mask;
    return CSWDG_OK;
}

int cswdg_kernel_times(cswdg_solver* s, const char** names, double* total_ms, int64_t* counts, int cap, int* n) {
    if (!s || !n) return fail(s, CSWDG_EINVAL, "null argument");
    (void)hipSetDevice(s->device);
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hipfail(s, e, "kernel_times");
    double tot[KID_COUNT] = {0};
    int64_t cnt[KID_COUNT] = {0};
    for (auto& r : s->recs) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, s->ev_pool[r.second], s->ev_pool[r.second + 1]) == hipSuccess) {
            tot[r.first] += ms;
            cnt[r.first] += 1;
        }
    }
    *n = KID_COUNT;
    for (int k = 0; k < KID_COUNT && k < cap; ++k) {
        if (names) names[k] = kKernelNames[k];
        if (total_ms) total_ms[k] = tot[k];
        if (counts) counts[k] = cnt[k];
    }
    return CSWDG_OK;
}

}  // extern "C"

namespace {

// device copies of s->mesh (built on the host) and the per-element operators
int upload_mesh(cswdg_solver* s) {
    int rc;
    const int64_t K = s->mesh.K;
    std::vector<double> ops;
    rc = s->p.reconstruction == 1   ? build_type1_ops(s->mesh, s->p.degree, ops, s->n_rank)
         : s->p.reconstruction == 2 ? build_type2_ops(s->mesh, ops, s->n_rank)
         : s->p.reconstruction == 3 ? build_mixed_ops(s->mesh, ops, s->n_rank)
                                    : build_limiter_ops(s->mesh, s->p.degree, s->ctx.qtop, s->p.gamma_mode == 1,
                                                        s->p.ghost_mode == 1, ops, s->n_rank, s->n_foot);
    if (rc != CSWDG_OK) return fail(s, rc, "limiter operator build failed");
    std::vector<double> tvbA;
    s->n_tvb_neg = 0;
    if (s->p.indicator == CSWDG_INDICATOR_TVB) build_tvb_ops(s->mesh, tvbA, s->n_tvb_neg);
    std::vector<int32_t> nbrT(3 * K);
    std::vector<uint32_t> info4(K);
    for (int64_t e = 0; e < K; ++e) {
        uint32_t w = 0;
        for (int f = 0; f < 3; ++f) {
            nbrT[f * K + e] = s->mesh.nbr[3 * e + f];
            w |= (uint32_t)s->mesh.info[3 * e + f] << (8 * f);
        }
        info4[e] = w;
    }
    const size_t NPM = (size_t)s->M * s->NP;
    s->state_elems = NPM * K;
    struct A {
        void** p;
        size_t bytes;
    } allocs[] = {
        {(void**)&s->d_vx, sizeof(double) * 3 * K},
        {(void**)&s->d_vy, sizeof(double) * 3 * K},
        {(void**)&s->d_nbr, sizeof(int32_t) * 3 * K},
        {(void**)&s->d_info, sizeof(uint32_t) * K},
        {(void**)&s->d_ops, sizeof(double) * ops.size()},
        {(void**)&s->d_flags, (size_t)K},
        {(void**)&s->d_list, sizeof(int32_t) * K * kListSegs},
        {(void**)&s->d_count, sizeof(uint32_t) * kCountWords},
        {(void**)&s->d_status, sizeof(uint32_t) * 4},
        {(void**)&s->d_tstats, sizeof(unsigned long long) * 2},
        {(void**)&s->d_compact, sizeof(double) * NPM * K},
        {(void**)&s->d_partial, sizeof(double) * s->dt_blocks},
        {(void**)&s->d_dt, sizeof(double) * std::max(2, s->n_inst)},
        {(void**)&s->d_inst_off, sizeof(int32_t) * (s->n_inst + 1)},
        {(void**)&s->d_inst_hmin, sizeof(double) * s->n_inst},
        {(void**)&s->d_amax, sizeof(unsigned long long) * s->n_inst},
        {(void**)&s->d_inflow, sizeof(double) * 4},
        {(void**)&s->d_lfa, sizeof(double) * s->n_inst},
        {(void**)&s->d_time, sizeof(double) * s->n_inst},
        {(void**)&s->d_shock, sizeof(double) * 12},
        {(void**)&s->d_tvb, sizeof(double) * std::max<size_t>(1, tvbA.size())},
        {(void**)&s->d_T1, sizeof(double) * NPM * K},
        {(void**)&s->d_T2, sizeof(double) * NPM * K},
    };
    for (auto& a : allocs) {
        if (hipMalloc(a.p, a.bytes) != hipSuccess) {
            free_mesh(s);
            return fail(s, CSWDG_ENOMEM, "device allocation failed");
        }
    }
    hipError_t e = hipSuccess;
    auto cp = [&](void* d, const void* h, size_t b) {
        if (e == hipSuccess) e = hipMemcpy(d, h, b, hipMemcpyHostToDevice);
    };
    cp(s->d_vx, s->mesh.vx.data(), sizeof(double) * 3 * K);
    cp(s->d_vy, s->mesh.vy.data(), sizeof(double) * 3 * K);
    cp(s->d_nbr, nbrT.data(), sizeof(int32_t) * 3 * K);
    cp(s->d_info, info4.data(), sizeof(uint32_t) * K);
    cp(s->d_ops, ops.data(), sizeof(double) * ops.size());
    if (!tvbA.empty()) cp(s->d_tvb, tvbA.data(), sizeof(double) * tvbA.size());
    std::vector<uint32_t> zeros(kCountWords, 0u);
    cp(s->d_count, zeros.data(), sizeof(uint32_t) * kCountWords);
    cp(s->d_status, zeros.data(), sizeof(uint32_t) * 4);
    unsigned long long zz[2] = {0, 0};
    cp(s->d_tstats, zz, sizeof(zz));
    cp(s->d_inst_off, s->inst_off.data(), sizeof(int32_t) * (s->n_inst + 1));
    cp(s->d_inst_hmin, s->inst_hmin.data(), sizeof(double) * s->n_inst);
    if (e == hipSuccess) e = hipMemset(s->d_amax, 0, sizeof(unsigned long long) * s->n_inst);
    if (e == hipSuccess) e = hipMemset(s->d_inflow, 0, sizeof(double) * 4);
    if (e == hipSuccess) e = hipMemset(s->d_time, 0, sizeof(double) * s->n_inst);
    if (e == hipSuccess) e = hipMemset(s->d_shock, 0, sizeof(double) * 12);
    if (e != hipSuccess) {
        free_mesh(s);
        return hipfail(s, e, "mesh upload");
    }
    s->dm.K = (int)K;
    s->dm.vx = s->d_vx;
    s->dm.vy = s->d_vy;
    s->dm.nbr = s->d_nbr;
    s->dm.info = s->d_info;
    s->dm.n_inst = s->n_inst;
    s->dm.inflow = s->d_inflow;
    s->n_special = 0;
    s->dm.inst_off = s->d_inst_off;
    s->dm.lf_alpha = s->p.lf_mode ? s->d_lfa : nullptr;
    s->dm.time = s->d_time;
    s->dm.shock = nullptr;
    s->dm.tvb = tvbA.empty() ? nullptr : s->d_tvb;
    s->shock_set = false;
    {
        const char* xt = std::getenv("CSWDG_XCD_TILES");
        s->dm.xcd_tiles = xt ? std::atoi(xt) : 1;
    }
    s->has_mesh = true;
    return CSWDG_OK;
}


}  // namespace
