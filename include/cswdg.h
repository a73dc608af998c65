/*
 * cswdg.h -- C ABI of the MI355X (gfx950) library for one SSP-RK3 stage of
 * the Runge-Kutta discontinuous Galerkin operator on unstructured
 * triangles followed by the compact subcell WENO (CSWENO) limiter
 * (Kochi & Ramakrishna, "A compact subcell WENO limiting strategy using
 * immediate neighbors for Runge-Kutta discontinuous Galerkin methods for
 * unstructured meshes").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every function returns 0 (CSWDG_OK) or a negative CSWDG_E* code;
 * cswdg_last_error() gives a message.  No C++ exception crosses the ABI.
 *
 * Coefficients: modal coefficients in the orthonormal basis of Section 2
 * (eq. triangleBasis; Jacobi polynomials L2-normalised, 1-based index
 * m = j + (N+1) i + 1 - i(i-1)/2 stored at position m-1), on each
 * triangle's affine map x(r,s) = v0 + (1+r)/2 (v1-v0) + (1+s)/2 (v2-v0)
 * from the reference triangle {r,s >= -1, r+s <= 0}, using the vertex order
 * after the counter-clockwise fix of cswdg_mesh_upload.  The cell mean is
 * coefficient 0 divided by sqrt(2).
 *
 * State layout (device memory, caller-owned): [m][Np][K] contiguous, element
 * index fastest; m = 1 (Burgers) or 4 (Euler: rho, rho u, rho v, E);
 * Np = (N+1)(N+2)/2; element type double (precision 0) or float
 * (precision 1, "FP32-bulk": the state is stored in float and the residual
 * and RK combine compute in float; dt, the KXRCF indicator and the limiter
 * compute in double from the float state and the limiter's results are
 * rounded to float; the adjoint calls take FP64 solvers only).
 *
 * Streams: every call that takes device pointers is enqueued on the
 * solver's HIP stream (given at creation; NULL = default stream) and
 * returns without waiting, except the calls marked "synchronous".
 *
 * Mesh conventions: a triangle whose signed area is negative has its local
 * vertices 1 and 2 swapped (reported through cswdg_mesh_info, not an error);
 * a zero-area triangle, an edge shared by more than two triangles, two
 * neighbours traversing their shared edge in the same direction, and (for
 * periodic meshes) a boundary edge without exactly one partner one period
 * away are errors (CSWDG_EBADMESH).  Local face f joins local vertices f and
 * f+1 (mod 3).  Connectivity info byte: bits 0-1 the neighbour's local face,
 * bits 2-3 / 4-5 the x / y shift code (0 none, 1 add +period, 2 add -period
 * to the neighbour's coordinates to place it next to the element), bit 6 set
 * on a boundary face (neighbour id -1), whose bits 0-1 then hold its kind
 * (cswdg_set_boundary: 0 outflow, the default; 1 wall; 2 inflow; 3 moving
 * shock).
 */
#ifndef CSWDG_H
#define CSWDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSWDG_OK 0
#define CSWDG_EINVAL (-1)   /* bad argument (null pointer, size, enum value) */
#define CSWDG_EBADMESH (-2) /* mesh rejected by validation */
#define CSWDG_ERANK (-3)    /* a stencil least-squares system is rank deficient */
#define CSWDG_EHIP (-4)     /* a HIP runtime call failed */
#define CSWDG_ESTATE (-5)   /* call out of order (e.g. no mesh uploaded yet) */
#define CSWDG_ENOMEM (-6)   /* device allocation failed */

#define CSWDG_EQ_BURGERS 0
#define CSWDG_EQ_EULER 1

#define CSWDG_BC_PERIODIC 0
#define CSWDG_BC_TRANSMISSIVE 1

#define CSWDG_LIMIT_KXRCF 0 /* limit the cells the KXRCF indicator flags (Section 3.1) */
#define CSWDG_LIMIT_ALL 1   /* mark every cell troubled (the accuracy tests of Section 4.1) */
#define CSWDG_LIMIT_NONE 2  /* no limiter */

#define CSWDG_INDICATOR_KXRCF 0 /* params.indicator: KXRCF (Section 3.1) */
#define CSWDG_INDICATOR_TVB 1   /* params.indicator: TVB minmod test (not in the paper) */

#define CSWDG_STATUS_NONFINITE 0x1u /* a NaN/Inf coefficient was produced */
#define CSWDG_STATUS_NEGATIVE 0x2u  /* a non-positive Euler cell-mean density or pressure */
#define CSWDG_STATUS_RANK 0x4u      /* a stencil least-squares system was rank deficient */
#define CSWDG_STATUS_FOOT 0x8u      /* a perpendicular foot fell outside its side (midpoint used) */
#define CSWDG_STATUS_SCALED 0x10u   /* the positivity scaling changed a cell (only with positivity = 1) */

typedef struct cswdg_solver cswdg_solver;
typedef struct cswdg_graph cswdg_graph;

/* Parameters.  Zero-initialise and set what you need: for gas_gamma, cfl,
 * c_k and eps_weno a zero/negative value selects the default shown; the
 * integer switches and tvb_m take only the values listed (CSWDG_EINVAL
 * otherwise), zero being the default. */
typedef struct cswdg_params {
    int equation;     /* CSWDG_EQ_BURGERS (eq. 2dBurgers) or CSWDG_EQ_EULER (eq. 2dEulerEquations) */
    int degree;       /* N = 1, 2 or 3 (Section 2, eq. modalForm2D) */
    int precision;    /* 0 FP64 everywhere; 1 FP32-bulk: float state and residual, FP64 dt/indicator/limiter */
    int limiter_mode; /* CSWDG_LIMIT_* used by cswdg_ssprk3_step (default KXRCF) */
    double gas_gamma; /* ratio of specific heats, default 1.4 (Section 4) */
    double cfl;       /* default 0.3/(2N+1) */
    double c_k;       /* KXRCF threshold C_K, default 1 (Section 3.1) */
    double eps_weno;  /* epsilon of the nonlinear weights, default 1e-10 (Section 3.2) */
    /* readings of the paper (0 = the default reading): */
    int kxrcf_norm;   /* ||U_j|| of Section 3.1: 0 the literal (int U^2 dA)^(1/2), 1 divided by |Delta|^(1/2) (RMS) */
    int char_mode;    /* Euler limiting (Section 3.2, last paragraph): 0 characteristic fields, 1 conserved variables */
    int weights_mode; /* Section 3.2 Step 4: 0 nonlinear weights, 1 the linear weights (omega = gamma) */
    /* not in the paper: 1 = after the limiter of every RK stage, the
     * positivity-preserving scaling of cswdg_positivity (Euler only) */
    int positivity;
    /* Lax-Friedrichs constant (end of Section 2): 0 local, the larger normal
     * wave speed of the two traces at each edge point; 1 global, one
     * constant per residual and instance, the largest cell-mean wave speed
     * of the residual's input state (the bound the time step uses) */
    int lf_mode;
    /* fourth member of the N >= 2 reconstruction hierarchy (Section 3.2,
     * Steps 1-2 for P2; the text defines p_4 from the cubic q_4 by eq.
     * equivalentOrder3 and p_5 from the quartic q_5 by eq.
     * equivalentOrder4, then combines four members with gamma_{.,5}):
     *   0 the default reading of the degree: for N = 2 the quadratic top
     *     (value 1: with every cell limited the readings that build a fourth
     *     member on T4 diverge under refinement for the Euler equations),
     *     for N = 3 the quartic (value 2);
     *   1 the quadratic q_3 on top: the three members of N = 1 projected
     *     onto P_N (a third-order reconstruction);
     *   2 the quartic q_5 on the 16-cell stencil T4 by eq. equivalentOrder4;
     *   3 the cubic q_4 in place of q_5 in eq. equivalentOrder4 (so that
     *     the linear weights telescope to q_4);
     *   4 p_4 = (q_4 - gamma_{1,4} p_1 - gamma_{2,4} p_2) / gamma_{3,4} with
     *     the three weights gamma_{.,4} (eq. equivalentOrder3 as printed),
     *     the members p_1..p_4 combined with gamma_{.,5};
     *   5 (N = 3 only: the P3 hierarchy built the same way one level finer,
     *     Section 3.2) the degree-6 q_7 on the 30-piece stencil T5 by eq.
     *     equivalentOrder4, T5 halving each T4 piece by the median from the
     *     neighbour's centroid; no adjoint (CSWDG_EINVAL from the VJP calls).
     * N = 1 is unaffected.  Values outside 0..5, or 5 with N != 3:
     * CSWDG_EINVAL. */
    int p2_top;
    /* troubled-cell indicator (the first step of Section 3; the limiter does
     * not depend on which one marks the cells): CSWDG_INDICATOR_KXRCF (the
     * paper's, Section 3.1) or CSWDG_INDICATOR_TVB (not in the paper: the
     * TVB minmod test of Cockburn and Shu's limiter for triangles, J. Comput.
     * Phys. 141 (1998); cswdg_kxrcf documents it) */
    int indicator;
    /* the TVB constant M of CSWDG_INDICATOR_TVB (>= 0, default 0: the TVD
     * minmod test); deviations up to M h^2 pass, h the circumradius */
    double tvb_m;
    /* linear weights of the reconstruction hierarchy (Section 3.2, Step 2):
     * 0 gamma_bar_{l,m} = (1/h)^(l-1), h the mean side (the paper's);
     * 1 gamma_bar_{l,m} = 10^(l-1), the weights of the reference cited
     * there, which the paper replaces (the same for every h, so the
     * reconstruction does not depend on the length scale of the mesh) */
    int gamma_mode;
    /* the limiter's ghost cell across an outflow face (the paper is silent
     * on boundaries): 0 the mirror image of Delta0 carrying its reflected
     * polynomial; 1 the same triangle carrying Delta0's polynomial continued
     * across the face (linear data then reproduced in boundary cells too).
     * Wall faces keep the mirror image, inflow and moving-shock faces their
     * states.  With 1, cswdg_set_boundary rebuilds the stencil operators
     * (synchronous, host work proportional to K). */
    int ghost_mode;
    /* the reconstruction on the subcell stencils (the paper's stencils work
     * with any WENO reconstruction, Sections 1 and 5): 0 the Zhu-Shu
     * hierarchical reconstruction of Section 3.2 (the paper's); 1 a type-I
     * WENO reconstruction (N = 1, 2 only): degree-N least-squares fits on a
     * central stencil (the nine centroid subcells of the three neighbours)
     * and on three sectors (the six of two neighbours), each with the mean
     * of Delta0 exact, combined with weights lambda_k / (1e-14 + beta_k)^4
     * (lambda 1e5 central, 1 sectors; beta of eq. smoothnessIndicator);
     * the boundary ghosts are those of the hierarchical one (the mirror image
     * and the boundary kinds, ghost_mode 0); 2 a type-II WENO reconstruction
     * (N = 2 only): linear least-squares fits on the three single-neighbour
     * stencils (each neighbour's three centroid subcells) and on the three
     * sectors, combined at each of the 9 points of the degree-4 rule on
     * Delta0 with linear weights of minimal distance to 1/6 that reproduce
     * the quadratic fit on T3, negative weights split into two positive
     * groups (Shi, Hu and Shu), nonlinear weights of the WENO-Z form
     * gamma_j (1 + (tau / (1e-10 + beta_j))^2) per group (tau = max beta -
     * min beta), then projected onto P2; 3 a mixed WENO reconstruction
     * (N = 2 only): the quadratic fit Q on T3 and the six linear fits L_j
     * of reconstruction 2, combined with constant positive linear weights
     * through p_0 = (Q - 0.025 sum_j L_j) / 0.85 (so that 0.85 p_0 +
     * 0.025 sum_j L_j = Q), nonlinear weights gamma_j / (1e-6 + beta_j)^2
     * (beta of eq. smoothnessIndicator: orders 1 and 2 for p_0), R =
     * omega_0 p_0 + sum_j omega_j L_j projected onto P2.  1 with N = 3, 2
     * or 3 with N != 2, ghost_mode 1 with 1, 2 or 3, or the adjoint calls
     * with any but 0: CSWDG_EINVAL. */
    int reconstruction;
    /* the smoothness indicators beta_l, l >= 2, of the hierarchical
     * reconstruction (Section 3.2, Step 3, eq. smoothnessIndicator):
     * 0 of the least-squares levels q_l over derivative orders 1..deg q_l
     * (the default: only then are linear data reproduced, every beta being
     * |Delta0| |grad u|^2); 1 as the equation is printed, of the equivalent
     * polynomials p_l over derivative orders 1..N.  beta_1 (eqs. sigmaEqn,
     * smoothnessIndicatorT1) is the same in both.  1 with reconstruction
     * other than 0 or in the adjoint calls: CSWDG_EINVAL. */
    int beta_mode;
} cswdg_params;

/* Create a solver bound to the current HIP device and to hip_stream
 * (a hipStream_t; NULL = default stream).  *out receives the handle. */
int cswdg_create(const cswdg_params* params, void* hip_stream, cswdg_solver** out);
int cswdg_destroy(cswdg_solver* s);
/* Message of the last error on s (or of the last failed cswdg_create /
 * host-only call when s is NULL).  Valid until the next call on s. */
const char* cswdg_last_error(const cswdg_solver* s);

/* Upload a triangulation (Section 2, eq. triangulation): host arrays
 * vxy [nv][2] (double) and tri [nt][3] (int32 vertex ids), read
 * synchronously and not retained.  bc = CSWDG_BC_*; period_x/period_y are
 * the domain periods for periodic meshes (ignored otherwise); a periodic
 * mesh with one period 0 is periodic in the other direction only, and its
 * unpaired boundary edges become boundary faces (outflow until
 * cswdg_set_boundary says otherwise), as Example 4's sides.  Builds the
 * connectivity on the host, the element geometry and the per-element
 * stencil operators of the limiter on the device.  At most 715,827,882
 * triangles (the kernels index [3][K] arrays with 32-bit integers; a batch
 * counts all its instances): CSWDG_EINVAL beyond.  Synchronous. */
int cswdg_mesh_upload(cswdg_solver* s, int64_t nv, const double* vxy, int64_t nt,
                      const int32_t* tri, int bc, double period_x, double period_y);

/* Upload n_inst independent triangulations (instances) as one mesh, the
 * disjoint union of the instances: vertex and triangle arrays of the
 * instances are concatenated (vxy [sum nv][2], tri [sum nt][3]; the vertex
 * ids in tri are local to their instance), nv[i], nt[i] and bc[i] give
 * instance i's sizes and boundary condition (host arrays of n_inst).  Each
 * instance keeps its own connectivity, element ids are numbered instance
 * after instance, and every periodic instance uses period_x/period_y.  Each
 * instance advances with its own time step (dt arrays of the calls below
 * hold one value per instance); every other call treats the union as one
 * mesh, so one launch serves all instances.  Not for the adjoint calls,
 * which take single-instance meshes.  Same validation as cswdg_mesh_upload
 * per instance.  Synchronous. */
int cswdg_mesh_upload_batch(cswdg_solver* s, int32_t n_inst, const int64_t* nv, const double* vxy,
                            const int64_t* nt, const int32_t* tri, const int32_t* bc, double period_x,
                            double period_y);
/* Number of instances and (when offsets != NULL, host [n_inst + 1]) the
 * first element of each instance, offsets[n_inst] = K.  A mesh from
 * cswdg_mesh_upload is one instance. */
int cswdg_instances(const cswdg_solver* s, int32_t* n_inst, int64_t* offsets);

/* Boundary conditions of the boundary faces (Section 4, Examples 4-6):
 * kinds (host uint8 [K][3], may be NULL to keep them; read for boundary
 * faces only, interior entries ignored): 0 outflow (exterior trace = interior
 * trace, the default), 1 reflective wall (interior trace with its normal
 * momentum reversed; for Burgers the same as outflow), 2 inflow (the state
 * inflow, host double [m] of conserved variables, may be NULL to keep the
 * last one; zero after a mesh upload), 3 moving shock (Example 5's top
 * boundary; cswdg_set_moving_shock first).  The limiter's ghost cell across
 * a boundary face is Delta0's mirror image carrying the same exterior state
 * (the mirrored polynomial, with reversed normal momentum at a wall, the
 * inflow state on every piece, the moving shock's state at the face
 * midpoint on every piece); KXRCF sees the ghost's density.  Adjoint calls
 * reject meshes with faces of kinds 1-3.  Another kind is CSWDG_EINVAL, and
 * so is kind 3 before a moving shock is set.  Synchronous. */
int cswdg_set_boundary(cswdg_solver* s, const uint8_t* kinds, const double* inflow);

/* The moving planar shock of boundary kind 3 (Section 4, Example 5's top
 * boundary, where the exact Mach 10 shock position is imposed): at a
 * boundary point x and time t the exterior state is post (host double [4],
 * conserved variables) where nx x + ny y < d0 + speed t, pre elsewhere.
 * The residual of an SSP-RK3 stage evaluates it at its input's time (the
 * step's start t, t + dt, t + dt/2 for u^n, u^(1), u^(2)); KXRCF and the
 * limiter at the step's start.  Setting it makes cswdg_ssprk3_step (and
 * graphs of it) advance the solution time by dt.  Euler only (otherwise
 * CSWDG_EINVAL).  Synchronous. */
int cswdg_set_moving_shock(cswdg_solver* s, const double* post, const double* pre, double nx, double ny, double d0,
                           double speed);
/* Solution time of every instance: set to t (synchronous; zero after a mesh
 * upload), read into t_host [n_inst] (synchronous). */
int cswdg_set_time(cswdg_solver* s, double t);
int cswdg_time(cswdg_solver* s, double* t_host);

/* Number of elements, number of triangles re-oriented by the CCW fix. */
int cswdg_mesh_info(const cswdg_solver* s, int64_t* n_elements, int64_t* n_flipped);

/* Host-only connectivity builder (no device needed): tri_ccw [nt][3]
 * receives the re-oriented triangles, nbr [nt][3] and info [nt][3] the
 * tables described above.  Same rules as cswdg_mesh_upload. */
int cswdg_host_connectivity(int64_t nv, const double* vxy, int64_t nt, const int32_t* tri, int bc,
                            double period_x, double period_y, int32_t* tri_ccw, int32_t* nbr,
                            uint8_t* info);

/* Host-only builder of the TVB indicator's midpoint decomposition (see
 * cswdg_kxrcf; no device needed): A [nt][3][3] receives, for element e and
 * face midpoint i, the coefficients A[e][i][f] with
 * m_i - b0 = sum_f A[e][i][f] (b_f - b0) (at most two nonzero per i; the
 * pairs of neighbour faces are tried in the order (i, i+1), (i, i+2),
 * (i+1, i+2), the first whose coefficients are both >= 0 is used, else the
 * one whose smaller coefficient is largest); *n_neg (may be NULL) the number
 * of midpoints without a nonnegative pair.  Same mesh rules as
 * cswdg_mesh_upload. */
int cswdg_host_tvb_decomposition(int64_t nv, const double* vxy, int64_t nt, const int32_t* tri, int bc,
                                 double period_x, double period_y, double* A, int64_t* n_neg);

/* Copy the uploaded connectivity to host arrays nbr [nt][3], info [nt][3].
 * Synchronous. */
int cswdg_connectivity(const cswdg_solver* s, int32_t* nbr, uint8_t* info);

/* Limiter stencil of element elem (Section 3.2, Fig. 1): for faces f = 0..2
 * the 4 ints (neighbour id or -1 for the mirror ghost of a transmissive
 * face, neighbour's shared face, x shift code, y shift code); *n = 12.
 * Subcell order per neighbour: Delta_i1 (touching the element), Delta_i2,
 * Delta_i3 in counter-clockwise order; for N >= 2 Delta_i2 and Delta_i3 are
 * cut at the foot of the perpendicular from the neighbour's centroid.
 * ids is a host array of at least 12 ints.  Synchronous. */
int cswdg_stencil(const cswdg_solver* s, int32_t elem, int32_t* ids, int32_t* n);

/* Physical coordinates of the projection quadrature points: xy is a device
 * array [2][nq][K] (double); *nq receives nq.  With xy = NULL only *nq is
 * set.  Used with cswdg_project to load initial data. */
int cswdg_ic_points(cswdg_solver* s, double* xy, int32_t* nq);
/* L2 projection (Section 2, eq. modalForm2D with eq. massMatrix2D) of point
 * values vals [m][nq][K] (device, double) at the cswdg_ic_points onto the
 * basis: u (device, state layout). */
int cswdg_project(cswdg_solver* s, const double* vals, void* u);

/* r = L(u) (Section 2, eq. weakFormScheme2D read as the triangle weak form:
 * volume quadrature of grad psi . F(u_h), edge quadrature of the local
 * Lax-Friedrichs flux, times the inverse mass matrix 1/J).  u, r: device,
 * state layout, distinct buffers. */
int cswdg_dg_residual(cswdg_solver* s, const void* u, void* r);

/* *dt_dev (device double) = CFL * min_e(2 r_e) / max_e a(ubar_e) with r_e the
 * inradius and a the cell-mean wave speed (Burgers sqrt(2)|u|, Euler
 * |v| + c) (the time step of Section 4's examples).  For a mesh of several
 * instances dt_dev is a device array with one dt per instance, the min and
 * max taken over that instance's elements. */
int cswdg_max_dt(cswdg_solver* s, const void* u, double* dt_dev);

/* The troubled-cell indicator of params.indicator.  KXRCF (Section 3.1,
 * eq. troubledCellIndicator): flags [K] (device uint8, 1 = troubled,
 * R > C_K) and optionally R [K] (device double, may be NULL).
 * TVB (CSWDG_INDICATOR_TVB; Cockburn and Shu's limiter for triangles, used
 * as an indicator as by Zhu, Qiu, Shu and Dumbser, J. Comput. Phys. 227
 * (2008)): the midpoint m_i of each face is written as
 * b0 + alpha (b_j - b0) + beta (b_k - b0), alpha, beta >= 0, with b0 the
 * element's centroid and b_j, b_k two neighbours' centroids (a periodic
 * neighbour translated, a boundary face's mirror image; built at mesh
 * upload); per variable (every conserved variable for Euler) the deviation
 * a = u_h(m_i) - ubar0 is compared with b = alpha (ubar_j - ubar0) +
 * beta (ubar_k - ubar0) (a boundary face's ghost mean is its boundary
 * kind's state: ubar0, reversed normal momentum at a wall, the inflow
 * state, the moving shock's state at the face midpoint); a cell is troubled
 * when the TVB minmod would change some a: |a| above
 * max(tvb_m h^2, 1e-12 max_c |ubar0_c|) (h the circumradius) and not
 * (a b > 0 and |a| <= 1.5 |b|).  R then receives the largest ratio of a
 * deviation |a| above that threshold to the largest deviation the minmod
 * leaves alone, max(threshold, 1.5 |b| if a b > 0), over midpoints and
 * variables (0 when every |a| is at or below the threshold); a cell is
 * troubled exactly when R > 1. */
int cswdg_kxrcf(cswdg_solver* s, const void* u, uint8_t* flags, double* R);

/* CSWENO limiter (Section 3.2).  Reads u_in, writes u_out (distinct
 * buffers; every troubled cell reads the pre-limit field).  Troubled cells:
 * mask_in (device uint8 [K], nonzero = troubled) when not NULL, otherwise
 * the flags of params.indicator.  Cell means are copied bitwise; untroubled cells are
 * copied.  flags_out (device uint8 [K]) receives the mask used; may be NULL. */
int cswdg_csweno_limit(cswdg_solver* s, const void* u_in, void* u_out, uint8_t* flags_out,
                       const uint8_t* mask_in);

/* cswdg_csweno_limit for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results, but the call's
 * scratch (troubled-list counters, troubled list, compact limiter results)
 * is a static device array of 64 MiB that every GPU the library runs on
 * holds until the process ends, instead of the solver's buffers; no
 * allocation of any kind.  Limit: 1024 + 32 K (rounded up to 256 bytes) +
 * 8 K m Np bytes must fit in 64 MiB (K <= 299,000 elements for P2 Euler,
 * 1.2 M for P1 Burgers); larger meshes: CSWDG_EINVAL with a message.  The
 * counters are cleared by a kernel at every call.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (on different
 * streams, or from different solvers) race. */
int cswdg_csweno_limit_noalloc(cswdg_solver* s, const void* u_in, void* u_out, uint8_t* flags_out,
                               const uint8_t* mask_in);

/* One stage of the table:tvd third-order RK (end of Section 3) followed by
 * the limiter: out = a u_n + b (u_prev + dt L(u_prev)) with
 * (a, b) = (0, 1), (3/4, 1/4), (1/3, 2/3) for stage = 1, 2, 3, then limited
 * in place according to params.limiter_mode.  dt_dev: device double (one per
 * instance).  out must not alias u_prev; out may alias u_n (stage 3 of an
 * in-place step). */
int cswdg_rk_stage(cswdg_solver* s, int stage, const void* u_n, const void* u_prev, void* out,
                   const double* dt_dev);

/* One full SSP-RK3 step in place on u (device, state layout), limiter after
 * every stage.  dt_dev: device double, or NULL to compute it with
 * cswdg_max_dt from u at the start of the step (kept in the solver; see
 * cswdg_last_dt). */
int cswdg_ssprk3_step(cswdg_solver* s, void* u, const double* dt_dev);
/* Device pointer to the solver's last computed dt (valid for its lifetime). */
int cswdg_last_dt(cswdg_solver* s, double** dt_dev);

/* ---- Adjoint (vector-Jacobian products; not part of the paper) ----------
 * The limiter is differentiated with its troubled-cell set frozen (the KXRCF
 * indicator is a switch, not differentiated); the Lax-Friedrichs max picks
 * the first argument on ties and d|x|/dx = 0 at x = 0.  Deterministic (no
 * floating-point atomics).  All buffers device, state layout.  These calls
 * take FP64 single-instance solvers with the default readings (char_mode,
 * weights_mode, lf_mode, gamma_mode, ghost_mode and positivity 0, the KXRCF
 * indicator; any p2_top but 5; beta_mode 0) and no wall, inflow or moving-shock faces;
 * CSWDG_EINVAL otherwise. */

/* u_bar = L'(u)^T r_bar (the transpose of cswdg_dg_residual linearised at u).
 * u_bar must not alias r_bar. */
int cswdg_dg_residual_vjp(cswdg_solver* s, const void* u, const void* r_bar, void* u_bar);
/* w_bar = Lambda'(w)^T y_bar for the limiter cswdg_csweno_limit applied to w
 * with troubled cells mask (device uint8 [K]; NULL = the KXRCF flags of w). */
int cswdg_csweno_limit_vjp(cswdg_solver* s, const void* w, const uint8_t* mask, const void* y_bar,
                           void* w_bar);
/* Size in bytes of a step tape: the step's input, the three pre-limit stage
 * states, the two limited intermediate states, the three troubled masks and
 * dt. */
int cswdg_tape_bytes(cswdg_solver* s, int64_t* bytes);
/* cswdg_ssprk3_step in place on u, recording the tape (device buffer of
 * cswdg_tape_bytes).  replay = 0: dt from dt_dev (or cswdg_max_dt of u when
 * NULL) and masks from the limiter mode are computed and stored; replay = 1:
 * the tape's dt and masks are reused (a step with frozen decisions). */
int cswdg_ssprk3_step_tape(cswdg_solver* s, void* u, const double* dt_dev, void* tape, int replay);
/* u_n_bar = (d u^{n+1} / d u^n)^T u_next_bar for the step recorded in tape,
 * with its dt and masks frozen.  u_n_bar must not alias u_next_bar. */
int cswdg_ssprk3_step_vjp(cswdg_solver* s, const void* tape, const void* u_next_bar, void* u_n_bar);

/* ---- Schedules, autotuning and graphs (launch configuration only; not part
 * of the paper) ------------------------------------------------------------
 * A schedule is int32 [3]: the residual kernel's variant (0 "lean": one
 * face's neighbour data live at a time, 1 "wide": all three faces live,
 * 2 "stream": own coefficients re-read per face, 3 "compact": quadrature
 * point loops rolled, 4 "matrix": the evaluations at the quadrature points
 * and the projections onto the test functions as FP64 matrix-core products
 * over tiles of 16 elements per wave; the default is {3, 128, 1}), its
 * threads per block
 * (64, 128 or 256) and the XCD-contiguous block order (0 off, 1 on).  All
 * schedules compute the same quantities; variants may differ in the last
 * bits (summation order), block size and block order do not change results.
 * The wide variant is not offered for P3 Euler (its build exceeds a wave's
 * registers and spills; CSWDG_EINVAL), the matrix one is offered for P2 in
 * FP64 only (CSWDG_EINVAL otherwise), and FP32-bulk solvers run the compact
 * one. */
int cswdg_set_schedule(cswdg_solver* s, const int32_t* sched);
int cswdg_get_schedule(const cswdg_solver* s, int32_t* sched);
/* Time every schedule on the residual of the state u (device, reps timed
 * launches each after one untimed launch), keep the fastest and return it
 * in sched (may be NULL); times_us (host, may be NULL, 30 entries) receives
 * the mean microseconds per launch in the order variant-major, then block,
 * then XCD order (infinity for schedules not offered to the solver);
 * *n_cand (may be NULL) the number of schedules timed.
 * Synchronous. */
int cswdg_autotune(cswdg_solver* s, const void* u, int32_t reps, int32_t* sched, double* times_us,
                   int32_t* n_cand);
/* Record nsteps SSP-RK3 steps (cswdg_ssprk3_step with dt computed per step)
 * of each of n solvers on its state states[i] (device, state layout, fixed
 * for the life of the graph) into one HIP graph: each solver's steps form
 * one branch (captured on a private stream of default priority, forked from
 * and joined to the first by events), so the solvers advance concurrently.
 * Solvers and states must be distinct (CSWDG_EINVAL otherwise).  Capture
 * waits for the solvers' streams; nothing is computed.  The schedule and
 * limiter mode in force at capture are used by every launch. */
int cswdg_graph_capture(int32_t n, cswdg_solver* const* solvers, void* const* states, int32_t nsteps,
                        cswdg_graph** out);
/* Enqueue the recorded steps on hip_stream (NULL = default stream): each
 * launch advances every state by nsteps steps in place.  The solvers'
 * scratch is shared with their eager calls: do not overlap the two. */
int cswdg_graph_launch(cswdg_graph* g, void* hip_stream);
/* Number of nodes (kernel launches) in the graph. */
int cswdg_graph_nodes(const cswdg_graph* g, int64_t* nodes);
int cswdg_graph_destroy(cswdg_graph* g);

/* Troubled-cell count of the last limiter call (host int, synchronous). */
int cswdg_troubled_count(cswdg_solver* s, int64_t* count);
/* Troubled cells summed over all limiter calls since the last reset, and the
 * number of limiter calls (host ints; synchronous).  reset != 0 clears both
 * after reading. */
int cswdg_troubled_stats(cswdg_solver* s, int64_t* total_cells, int64_t* calls, int reset);
/* Positivity-preserving scaling of an Euler state u (device [4][Np][K], in
 * place; not part of the paper's method, which has no positivity limiter).
 * Zhang and Shu's scaling (J. Comput. Phys. 229 (2010) 8918-8934; on
 * triangles Zhang, Xia and Shu, J. Sci. Comput. 50 (2012) 29-62) at the
 * points where the residual evaluates the solution (its volume points and
 * the Gauss points of the three edges): with eps = min(1e-13, rhobar,
 * pbar), the density's modes above the mean are multiplied by
 * theta1 = min(1, (rhobar - eps)/(rhobar - min rho)), then every
 * variable's modes above the mean by theta2, the smallest t in [0, 1] at
 * which the pressure of (1 - t) Ubar + t U(x_q) reaches
 * eps_p = max(eps, 1e-10 pbar) over the points below eps_p (1 if none).  Cell means are left bit for bit; a cell
 * whose mean has rho <= 0 or p <= 0 (or is not finite) is left as it is.
 * Sets CSWDG_STATUS_SCALED when a cell changed.  CSWDG_EINVAL for Burgers.
 * With params.positivity = 1, cswdg_ssprk3_step (and graphs of it) apply it
 * after the limiter of every stage. */
int cswdg_positivity(cswdg_solver* s, void* u);

/* Accumulated status bits CSWDG_STATUS_* since the last call (synchronous;
 * clears them). */
int cswdg_status(cswdg_solver* s, uint32_t* flags);

/* Kernel timing with HIP events recorded around every launch on the
 * solver's stream.  enable = 1 starts (and clears) recording.
 * cswdg_kernel_times fills up to cap entries: names (static strings),
 * total milliseconds and launch counts; *n receives the number of kernel
 * classes.  Synchronous. */
int cswdg_profile(cswdg_solver* s, int enable);
/* Restrict the recording to the kernel classes whose bit is set in
 * kernel_mask (bit i = entry i of cswdg_kernel_times: 0 residual_rk,
 * 1 max_dt, 2 kxrcf, 3 compact_mask, 4 limiter, 5 scatter, 6 copy, 7 zero,
 * 8 project, 9 residual_vjp, 10 limiter_vjp, 11 positivity); all classes
 * by default.
 * Fewer events disturb the timed launches less. */
int cswdg_profile_select(cswdg_solver* s, uint32_t kernel_mask);
int cswdg_kernel_times(cswdg_solver* s, const char** names, double* total_ms, int64_t* counts,
                       int cap, int* n);

#ifdef __cplusplus
}
#endif
#endif
