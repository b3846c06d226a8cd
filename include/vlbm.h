/*
 * vlbm.h -- C ABI of the MI355X (gfx950) volumetric curvilinear lattice
 * Boltzmann library (H. Chen, "Volumetric Lattice Boltzmann Models in General
 * Curvilinear Coordinates: Theoretical Formulation", arXiv 2401.17183).
 *
 * Conventions for every call:
 *  - Every function returns an int status: VLBM_OK (0) or a negative
 *    VLBM_ERR_* code; vlbm_last_error() then gives a message (thread-local).
 *    No exception or C++ type crosses this boundary.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device
 *    memory on the current device (e.g. a torch tensor's data_ptr()).  Arrays
 *    passed in are borrowed for the duration of the call and never freed by the
 *    library.  Handles own everything they allocate and free it in *_destroy.
 *  - A "stream" argument is a hipStream_t passed as void* (0 = the null
 *    stream).  A simulation keeps the stream it was created with; all its work
 *    is enqueued there.
 *  - Index space: d axes q = (q^1, .., q^d), n_i real cells per axis; cell
 *    index = q^1 + n_1 (q^2 + n_2 q^3)  (q^1 fastest).  Fields are SoA:
 *    component-major, [component][cell].
 *  - Velocity ordering (Q directions, rest first, then opposite pairs):
 *    D2Q9 : (0,0) (1,0)(-1,0) (0,1)(0,-1) (1,1)(-1,-1) (1,-1)(-1,1)
 *    D3Q19: (0,0,0) (+-1,0,0) (0,+-1,0) (0,0,+-1) (1,1,0)(-1,-1,0) (1,-1,0)(-1,1,0)
 *           (1,0,1)(-1,0,-1) (1,0,-1)(-1,0,1) (0,1,1)(0,-1,-1) (0,1,-1)(0,-1,1)
 *    with weights 4/9,1/9,1/36 (D2Q9) and 1/3,1/18,1/36 (D3Q19), T0 = 1/3
 *    (velocity set and T0: Sec. 2.1 around eq. (iso)).
 *    Sixth-order isotropic sets (eq. (iso) in full), T0 = 2/3, links up to three
 *    cells long, periodic axes only:
 *    D3Q39: (0,0,0); (+-1,0,0) (0,+-1,0) (0,0,+-1); (1,1,1)(-1,-1,-1)
 *           (1,1,-1)(-1,-1,1) (1,-1,1)(-1,1,-1) (1,-1,-1)(-1,1,1); (+-2,0,0)
 *           (0,+-2,0) (0,0,+-2); (2,2,0)(-2,-2,0) (2,-2,0)(-2,2,0) (2,0,2)(-2,0,-2)
 *           (2,0,-2)(-2,0,2) (0,2,2)(0,-2,-2) (0,2,-2)(0,-2,2); (+-3,0,0) (0,+-3,0)
 *           (0,0,+-3); weights per shell 1/12, 1/12, 1/27, 2/135, 1/432, 1/1620;
 *    D2Q21: (0,0); (+-1,0) (0,+-1); (1,1)(-1,-1) (1,-1)(-1,1); (+-2,0) (0,+-2);
 *           (2,2)(-2,-2) (2,-2)(-2,2); (+-3,0) (0,+-3); weights per shell 91/324,
 *           1/12, 2/27, 7/360, 1/432, 1/1620 (the planar projection of D3Q39).
 */
#ifndef VLBM_H
#define VLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { VLBM_D2Q9 = 0, VLBM_D3Q19 = 1, VLBM_D2Q21 = 2, VLBM_D3Q39 = 3 };

/* Storage / arithmetic precision of a simulation:
 *  FP64   populations and geometry stored in FP64, FP64 arithmetic;
 *  FP32   each population stored as the FP32 difference from a per-slot FP16
 *         reference (one reference array, re-based every rebase_every steps),
 *         geometry in FP32 words (g^{ij} as a hi + lo pair; the a_ext words
 *         also cancel the rest-state effect of rounding the link
 *         coefficients), FP64 arithmetic in registers (FP32 arithmetic loses
 *         the small velocity signal to cancellation);
 *  FP32C  FP32 storage and FP32 arithmetic (faster, less accurate);
 *  FP16S / BF16S  the same per-slot deviations stored in 16 bits, FP32
 *         arithmetic (FP16: multiplied by the largest power of two up to 4096
 *         that keeps deviations up to 4 max J inside FP16's range). */
enum { VLBM_FP64 = 0, VLBM_FP32 = 1, VLBM_FP16S = 2, VLBM_BF16S = 3, VLBM_FP32C = 4 };

enum { VLBM_PERIODIC = 0, VLBM_WALL = 1, VLBM_FARFIELD = 2 };

enum {
  VLBM_OK = 0,
  VLBM_ERR_ARG = -1,        /* invalid argument (null, sizes, tau <= 1/2, ...)      */
  VLBM_ERR_MESH = -2,       /* degenerate mesh: beta undefined or J <= 0            */
  VLBM_ERR_NOMEM = -3,      /* device allocation failed                              */
  VLBM_ERR_DEVICE = -4,     /* a HIP call or kernel failed                           */
  VLBM_ERR_NOCONVERGE = -5, /* the collision fixed point hit its iteration cap       */
  VLBM_ERR_STATE = -6,      /* call out of order (e.g. step before init)             */
  VLBM_ERR_NONFINITE = -7,  /* non-finite populations were detected                  */
  VLBM_ERR_UNSUPPORTED = -8 /* combination not built (e.g. precision x lattice)      */
};

typedef struct vlbm_mesh_s* vlbm_mesh;
typedef struct vlbm_sim_s* vlbm_sim;

/* Boundary kinds per index axis and face (0 = low, 1 = high).  An axis is
 * periodic on both faces or on neither.  wrap[i] is the Euclidean translation
 * L_i of a periodic axis: x(q + n_i e_i) = x(q) + L_i (ignored otherwise).
 * Walls are halfway bounce-back; far-field faces impose equilibrium
 * populations (boundary treatment is outside the paper's scope: these are the
 * library's readings). */
typedef struct {
  int32_t face[3][2];
  double wrap[3][3];
} vlbm_topology;

/* Lattice tables.  Q, d: host int32 out; c: host int32 [Q][d] out (may be NULL);
 * w: host double [Q] out (may be NULL). */
int vlbm_lattice_info(int lattice, int32_t* Q, int32_t* d, int32_t* c, double* w);

/* Create a mesh from node coordinates (Sec. 2.1: the node set x(q) on a unit
 * index lattice).
 *  n        host int64[3]: real cells per axis (n[2] = 1 for a 2-D lattice).
 *  coords   double [m_d]..[m_1][d] in device memory (e.g. a mesh generated
 *           on the GPU) or host memory, m_i = n_i + 2 G on non-periodic axes
 *           (G ghost node layers per face: 2 for D2Q9 / D3Q19, 4 for D2Q21 /
 *           D3Q39, one more than the longest link), m_i = n_i on periodic axes.
 *  topo     host, faces and wrap translations.  D2Q21 / D3Q39 take walls on
 *           one axis at most (a link that meets a wall reflects along its own
 *           straight path: halfway bounce-back from the mirrored source cell)
 *           and no far-field faces; every axis needs at least 3 cells.
 *  dx       the representative spacing of the tangent-vector formula (> 0).
 * The ghost layer count is the lattice's (it is not an argument: fewer
 * layers cannot feed the longest link's tangent vectors, more are unused).
 * The coordinates are copied into the mesh (the runtime tells device from
 * host memory by the pointer; the caller keeps its array); nothing is
 * computed yet.  The FP64 geometry arrays are allocated here.
 * Errors: VLBM_ERR_ARG for bad sizes/faces, VLBM_ERR_UNSUPPORTED for faces a
 * lattice does not take, VLBM_ERR_NOMEM. */
int vlbm_mesh_create(int lattice, const int64_t n[3], const double* coords,
                     const vlbm_topology* topo, double dx, vlbm_mesh* out);

typedef struct {
  double min_J, max_J;               /* cell volume range (eq. (jacobian))          */
  double min_gup_eig, max_gup_eig;   /* eigenvalue range of g^{ij} (eq. (inverse))   */
  double min_rest_feq_over_w;        /* min over cells, a of f^eq(rho=1,U=0)/w_a     */
  double max_abs_A;                  /* max |A^i_a|, the contracted Theta           */
} vlbm_geom_report;

/* FP64 geometry precompute on the device, once per mesh (Sec. 2.1 notes that
 * the geometric coefficients depend on the mesh only, so they are computed
 * once, before the time stepping):
 * D_{+-i} (eq. (distance)), beta_i and g_i (eq. (tangent)), J (eq. (jacobian)),
 * g^i (eq. (covectors)), g^{ij} (eq. (inverse)) on real cells and the first
 * ghost layer, then the link coefficients
 *   A^i_a(q) = sum_j c_a^j Theta^i_j(q + c_a, q) = [e_a(q + c_a) - e_a(q)] . g^i(q)
 * (eqs. (lattice), (gamma)) on real cells.  Synchronises the stream and fills
 * rep (host, may be NULL).  The coefficients A are always precomputed and
 * stored (there is no variant that forms them from g_i inside the step: from
 * FP32 g_i their difference of nearly equal tangent vectors would lose to
 * cancellation what the stored FP64-formed A keeps).
 * Errors: VLBM_ERR_MESH when some |D_i - D_-i| = 0 or J <= 0 (reorder axes
 * for a positive handedness), VLBM_ERR_DEVICE. */
int vlbm_geometry_precompute(vlbm_mesh m, void* stream, vlbm_geom_report* rep);

/* vlbm_geometry_precompute for callers that cannot allocate device memory
 * (code in tight loops that re-derive the geometry, harnesses that forbid
 * hipMalloc): the same kernels and the same results, bit for bit, with all
 * scratch (degenerate-cell flag, per-block diagnostics, the g_i box) in a
 * static device array of 32 MiB that every GPU the library runs on holds
 * until the process ends; no device or host allocation.  A mesh needs
 * (d^2 x box cells + 6 x ceil(cells / 256) + 64) doubles of it, the box being
 * the real cells plus one link length of layers on every axis (D3Q19: up to
 * about 440k box cells, e.g. 74^3; D2Q9: about 1M); larger meshes are
 * rejected with VLBM_ERR_ARG.  Calls on one GPU share that array: calls that
 * overlap in time on one GPU (other threads, other streams) race and must
 * not be made.  Synchronises the stream; rep as for vlbm_geometry_precompute.
 * Errors: VLBM_ERR_ARG (null mesh, mesh too large), VLBM_ERR_MESH,
 * VLBM_ERR_DEVICE. */
int vlbm_geometry_precompute_noalloc(vlbm_mesh m, void* stream, vlbm_geom_report* rep);

/* Copy FP64 geometry to device arrays (any may be NULL):
 *  J [cells]; gup [d*d][cells] (full symmetric matrix, row-major ij);
 *  A [Q][d][cells] (A of the rest direction is 0); g [d][d][cells] (g_i
 *  Euclidean components, [i][k]).  Synchronous.  VLBM_ERR_STATE before
 *  vlbm_geometry_precompute. */
int vlbm_geometry_fields(vlbm_mesh m, double* J, double* gup, double* A, double* g);

typedef struct {
  double tau;            /* BGK relaxation time (eq. (collide)); must exceed 1/2      */
  double body_force[3];  /* Euclidean body acceleration G (a reading, not in the paper) */
  double rho_inf;        /* far-field density                                          */
  double u_inf[3];       /* far-field Euclidean velocity                               */
  int32_t precision;     /* VLBM_FP64 / VLBM_FP32 / VLBM_FP16S / VLBM_BF16S            */
  int32_t fp_max_iter;   /* cap of the per-cell collision fixed point (<= 0: 50)       */
  double fp_tol;         /* stop when max_i |F_k - F_(k-1)| <= fp_tol * rho (< 0: default:
                            1e-14 FP64, 1e-10 FP32, 1e-7 FP32C)                         */
  int32_t audit_every;   /* enqueue an audit every k steps (0 = never)                 */
  int32_t stream_only;   /* 1: advection only, no collision (a permutation test mode)  */
  double tau_g;          /* collision matrix of eq. (collide): 0 (or tau) selects BGK,
                            M = -I / tau; otherwise M = -I / tau_g + (1/tau_g - 1/tau) H,
                            H the projector onto the Hermite content of order <= 2, so the
                            stress relaxes at 1/tau (eq. (matrix)) and the rest at 1/tau_g
                            (1: regularised collision); must exceed 1/2                 */
  int32_t rebase_every;  /* FP32 / FP16S / BF16S (deviation storage): every k steps the
                            16-bit references are re-based on the current state, so that
                            the stored deviations restart near zero (0: every 10 steps;
                            < 0: never); ignored for FP64 and FP32C                    */
} vlbm_params;

/* Create a simulation on a precomputed mesh and set the initial state
 * N(0) = J f^eq(rho, U, Ut) with Ut^i = u . g^i and U chosen so that the
 * collision fixed point of N(0) reproduces Ut (the paper gives no initial
 * state: this is the library's reading).
 *  rho  device double [cells] or NULL (rho = 1);
 *  u    device double [d][cells] Euclidean velocity or NULL (u = 0).
 * Errors: VLBM_ERR_ARG (tau <= 1/2, tau_g neither 0 nor above 1/2, bad
 * precision), VLBM_ERR_STATE (geometry not precomputed), VLBM_ERR_NOCONVERGE, VLBM_ERR_NOMEM, VLBM_ERR_DEVICE. */
int vlbm_init(vlbm_mesh m, const vlbm_params* p, const double* rho, const double* u,
              void* stream, vlbm_sim* out);

/* Advance nsteps time steps: the fused pull-advection (eq. (adv)) + collision
 * (eq. (collide), BGK or the general matrix of tau_g) (deviation storage: plus
 * the re-basing of the references every rebase_every steps) + inertial force
 * (eqs. (compo-constr), (delta-flux), (deltaN)) + curvilinear equilibrium
 * (eq. (equilibrium)) update of eq. (lbe), with the implicit force solved per
 * cell as a converged fixed point.  Asynchronous: returns after enqueueing on
 * the sim's stream.  Cells whose fixed point hits fp_max_iter are counted on
 * the device and reported by the next vlbm_sync or vlbm_moments. */
int vlbm_step(vlbm_sim s, int64_t nsteps);

/* One time step on a mesh that moves (the paper's closing discussion names
 * time-varying coordinates as a next step and gives no equations; this is the
 * library's reading): the mesh goes from its current node positions x(q, t)
 * to coords_next = x(q, t + 1) (device FP64, the layout of vlbm_mesh_create)
 * with the periodic translations wrap_next (host double [3][3], row i the
 * vector of axis i; NULL: unchanged).  A population leaving q at t along c_a
 * has the lattice velocity e_a(q, t) and arrives at q + c_a with
 * e_a(q + c_a, t + 1); eqs. (forceI) and (forceO) split the momentum it gains
 * between the two cells, so eq. (compo-constr) takes the outgoing and
 * incoming coefficients
 *   A+^i_a(q, t) = [e_a(q + c_a, t + 1) - e_a(q, t)] . g^i(q, t),
 *   A-^i_a(q, t) = [e_a(q, t) - e_a(q - c_a, t - 1)] . g^i(q, t)
 * (eq. (delta-flux) takes A+ + A-); before its first moving step the mesh is
 * taken as at rest.  The geometry of t + 1 (eqs. (distance) to (gamma)) is
 * computed on the device every step, and the fused step computes each cell's
 * A+ and A- from g_i of the times t - 1, t and t + 1 (no coefficient array
 * goes through HBM); the coefficients of the state at t + 1 (audits, output
 * mapping, a static step that follows) are computed when first needed.  Mass and the mid-link Euclidean
 * momentum with each e_a at the time the particle has it are conserved; the
 * audits report that momentum, the output mapping treats the mesh as
 * momentarily at rest.  FP64 storage, BGK, D2Q9 / D3Q19, periodic axes only,
 * and the mesh must belong to this simulation alone.  Asynchronous; a mesh
 * that becomes degenerate is reported by vlbm_sync (VLBM_ERR_MESH).  The mesh
 * keeps the new positions; a later vlbm_step continues with it at rest.
 * Errors: VLBM_ERR_ARG, VLBM_ERR_UNSUPPORTED, VLBM_ERR_STATE (shared mesh),
 * VLBM_ERR_NOMEM, VLBM_ERR_DEVICE. */
int vlbm_step_moving(vlbm_sim s, const double* coords_next, const double* wrap_next);

/* Wait for the sim's enqueued work.  Returns VLBM_ERR_NOCONVERGE when a step
 * since the last report ran some cell on an inertial force whose fixed point
 * (eq. (compo-constr)) hit fp_max_iter, with the count of such cell-steps in
 * vlbm_last_error(); the count is then reset.  VLBM_ERR_DEVICE on a device
 * error. */
int vlbm_sync(vlbm_sim s);

/* Statistics of the per-cell fixed point of the steps taken while enabled
 * (off by default; enabling it costs a few wavefront ballots and four atomic
 * adds per wavefront and step).  out (host, may be NULL) receives, since the
 * previous read: [0] the sum over cell-steps of the iterations, [1] the sum
 * over wavefront-steps of the wavefront's largest count (the lanes of a
 * wavefront iterate together), [2] the cell-steps and [3] the wavefront-steps
 * counted; the counters are then reset.  Synchronises when out is not NULL. */
int vlbm_step_stats(vlbm_sim s, int enable, uint64_t* out);

/* Durations of the kernels launched by vlbm_step and vlbm_step_moving while
 * enabled, from HIP events recorded on the sim's stream around each launch
 * (off by default).  out (host [6], may be NULL) receives, since the previous
 * read: [0] total milliseconds and [1] count of the fused step launches, [2]
 * and [3] the same for the re-basing launches of the deviation storage, [4]
 * and [5] for the geometry (g_i, J, g^i, g^{ij}) of the next node positions
 * that a moving step computes before its fused step; the record is then
 * cleared.  Synchronises when out is not NULL. */
int vlbm_kernel_timing(vlbm_sim s, int enable, double* out);

/* Change the fixed point's cap and tolerance for the following steps (the
 * meaning of vlbm_params.fp_max_iter and fp_tol, with the same defaults for
 * values <= 0 and < 0).  Host-only; VLBM_ERR_ARG for a null sim. */
int vlbm_set_fixed_point(vlbm_sim s, int32_t max_iter, double tol);

/* Output mapping (eq. (result)) of the current state, computed in FP64 after a
 * dry-run of the collision fixed point:
 *  rho  device double [cells];
 *  u    device double [d][cells]: Euclidean velocity Ut^i g_i (the shifted
 *       velocity Ut = U + F/(2 rho) that obeys the continuity equation);
 *  U    device double [d][cells] or NULL: contravariant first moment U^i.
 * Synchronises the stream.  Errors: VLBM_ERR_NOCONVERGE when the dry run or
 * a step since the last report (see vlbm_sync) hit the fixed point's cap (the
 * outputs are written either way), VLBM_ERR_DEVICE. */
int vlbm_moments(vlbm_sim s, double* rho, double* u, double* U);

/* Current arrived populations N_a(q, t) as FP64 into device double [Q][cells]
 * (converted from the storage precision).  Synchronises. */
int vlbm_populations(vlbm_sim s, double* N);

/* Replace the state by device double [Q][cells] arrived populations
 * (converted to the storage precision).  Synchronises. */
int vlbm_set_populations(vlbm_sim s, const double* N);

typedef struct {
  int64_t step;
  double mass;             /* sum_q sum_a N_a                                        */
  double mom_I[3];         /* mid-link Euclidean momentum 1/2 sum [e_a(q)+e_a(q-c_a)] N_a */
  double wall_impulse[3];  /* impulse taken by bounced links in the step before       */
  double force_impulse[3]; /* body-force impulse per step, G * mass                   */
  double residual;         /* ||u - u_prev|| / ||u|| since the previous audit (NaN first) */
  int32_t max_fp_iters;    /* largest fixed-point iteration count of the dry run      */
  int32_t nonfinite;       /* populations that are NaN or Inf                          */
  int32_t negative;        /* populations below zero                                   */
  int32_t unconverged;     /* cells whose fixed point hit the cap                      */
} vlbm_audit;

/* Enqueue an audit of the current state into the sim's device ring buffer
 * (FP64 wavefront + block reductions, deterministic order; no host sync). */
int vlbm_audit_now(vlbm_sim s);

/* Drain up to cap audits, oldest first, into host out; *n_out = number copied.
 * Synchronises.  Returns VLBM_ERR_NONFINITE if any drained audit saw
 * non-finite populations (the records are still copied). */
int vlbm_audits(vlbm_sim s, vlbm_audit* out, int cap, int* n_out);

/* Checkpoint: raw storage-precision populations, the force cache, the step
 * counter and (16-bit modes) the references into host memory.  With
 * buf == NULL only *used (the size needed) is set. */
int vlbm_save(vlbm_sim s, void* buf, size_t cap, size_t* used);
/* Restore a checkpoint written by vlbm_save for a sim on the same mesh with the
 * same precision.  Errors: VLBM_ERR_ARG on a size or header mismatch. */
int vlbm_restore(vlbm_sim s, const void* buf, size_t size);

/* Re-initialise an existing simulation in place (same mesh, params, stream)
 * with the initial state of vlbm_init from rho / u (device, nullable); resets
 * the step counter.  Synchronises.  Used to warm-start a solve from predicted
 * fields. */
int vlbm_reinit(vlbm_sim s, const double* rho, const double* u);

/* Steps taken since init (host int64 out). */
int vlbm_sim_step_count(vlbm_sim s, int64_t* t);

int vlbm_sim_destroy(vlbm_sim s);
/* A mesh destroyed while simulations still hold it is released with the last
 * of them (the handle must not be used again either way). */
int vlbm_mesh_destroy(vlbm_mesh m);

/* ----------------------------------------------------------------------------
 * Batches: many independent meshes advanced together (growth form of the
 * method's data-parallel step over cells to a data-parallel step over meshes).
 * Every member is an ordinary simulation (vlbm_batch_member returns a
 * borrowed handle; vlbm_moments, vlbm_populations, vlbm_audit_now,
 * vlbm_reinit work on it); all members share the lattice, the precision
 * (FP64, FP32 or FP32C) and the batch's stream.
 * Modes of vlbm_batch_step:
 *   PERSISTENT_GRAPH  one launch per step of a persistent kernel whose blocks
 *                     stride over a table of (mesh, tile) work items of all
 *                     members, captured in a hipGraph per 32 steps (default);
 *   PERSISTENT        the same launches without the graph;
 *   EAGER             one launch per member per step;
 *   EAGER_GRAPH       a hipGraph of the per-member launches.
 * -------------------------------------------------------------------------- */
typedef struct vlbm_batch_s* vlbm_batch;
enum { VLBM_BATCH_PERSISTENT_GRAPH = 0, VLBM_BATCH_PERSISTENT = 1, VLBM_BATCH_EAGER = 2, VLBM_BATCH_EAGER_GRAPH = 3 };

/* meshes: host array of count precomputed meshes; params: host array of count
 * parameter sets (tau may differ per member); stream: a hipStream_t that is
 * not the null stream, or NULL for a stream the batch creates and owns.
 * Members start from rho = 1, u = 0 (use vlbm_reinit on a member to change). */
int vlbm_batch_create(const vlbm_mesh* meshes, const vlbm_params* params, int count, void* stream,
                      vlbm_batch* out);
int vlbm_batch_member(vlbm_batch b, int i, vlbm_sim* out);
/* Host outs (each nullable): member count, total cells, the batch stream, and
 * the launch shape (threads per block, blocks per CU; 0 = one block per tile). */
int vlbm_batch_info(vlbm_batch b, int* count, int64_t* cells, void** stream, int* block, int* grid_per_cu);
int vlbm_batch_set_mode(vlbm_batch b, int mode);
/* block in {64, 128, 256}; grid_per_cu >= 0. */
int vlbm_batch_config(vlbm_batch b, int block, int grid_per_cu);
/* Asynchronous on the batch stream. */
int vlbm_batch_step(vlbm_batch b, int64_t nsteps);
/* Synchronise; VLBM_ERR_NOCONVERGE if any member's fixed point hit its cap. */
int vlbm_batch_sync(vlbm_batch b);
/* Time each launch shape for trial_steps steps (the state is restored
 * afterwards), keep the fastest, and append it to the text cache at
 * cache_path (nullable; a cached entry for the same key is reused). */
int vlbm_batch_autotune(vlbm_batch b, int trial_steps, const char* cache_path, int* block, int* grid_per_cu);
int vlbm_batch_destroy(vlbm_batch b);
/* Audit every active member now (as vlbm_audit_now) and write each member's
 * steady-state residual r = ||u - u_prev||_2 / ||u||_2 (u = output velocity,
 * u_prev = that of the member's previous audit; NaN at a member's first audit)
 * to residual[count] (host); a retired member reports its last audit.
 * Synchronises the batch stream. */
int vlbm_batch_residuals(vlbm_batch b, double* residual);
/* Choose the members vlbm_batch_step advances: active host int32[count],
 * non-zero = stepped (NULL = all).  A retired member keeps its state and step
 * count; the launch covers only the active members' cells, so a batch whose
 * members converge at different times costs what its active cells cost.  The
 * active members must share one step count (VLBM_ERR_STATE otherwise).
 * Synchronises the batch stream. */
int vlbm_batch_set_active(vlbm_batch b, const int32_t* active);

/* ---- Learned warm start: a convolutional surrogate on BF16 MFMA ----------
 *
 * Not part of the paper: a small network that maps a mesh (node coordinates)
 * and a Reynolds number to an approximate steady state, used only as the
 * initial state of a solve that the method then finishes (vlbm_reinit).
 *
 * Tensors are NHWC.  BF16 tensors are passed as raw 16-bit words (uint16_t,
 * the upper half of an IEEE single); FP32 and BF16 pointers are device
 * pointers; weights are [c_out][3][3][c_in + c_skip] and the transposed copy
 * used for input gradients [c_in + c_skip][3][3][c_out].  Calls are
 * asynchronous on `stream` unless stated otherwise.  Channel counts must be
 * multiples of 8 (VLBM_ERR_ARG otherwise). */
typedef struct vlbm_conv_desc {
  int batch, height, width; /* full-resolution input of the convolution */
  int c_in;                 /* channels of the primary input */
  int c_skip;               /* channels of a skip input (height x width) appended after them, or 0 */
  int upsample;             /* 1: the primary input is stored at height/2 x width/2 and read through a
                               nearest-neighbour 2x upsampling (stride must be 1) */
  int stride;               /* 1 or 2; zero padding 1, output ceil(height/stride) x ceil(width/stride) */
  int c_out, relu;
} vlbm_conv_desc;

/* y = relu?(conv3x3(x ++ skip, w) + bias), written as BF16 (y_bf16) and/or FP32
 * (y_f32); either output may be NULL, not both; bias may be NULL. */
int vlbm_conv2d_forward(const vlbm_conv_desc* d, const uint16_t* x, const uint16_t* skip, const uint16_t* w,
                        const float* bias, uint16_t* y_bf16, float* y_f32, void* stream);
/* Input gradients of sum(gy * conv3x3(...)) given gy (BF16, the gradient with
 * respect to the pre-activation output) and the transposed weights:
 * gx += d/dx (at the stored resolution of x, i.e. summed over each 2x2 block
 * when upsampled) and gskip += d/dskip; FP32, either may be NULL. */
int vlbm_conv2d_backward_data(const vlbm_conv_desc* d, const uint16_t* gy, const uint16_t* wt, float* gx,
                              float* gskip, void* stream);
/* gw += d/dw, gb += d/dbias (FP32, the pixel splits accumulated with atomics,
 * so the last bits depend on scheduling; the surrogate object below adds them
 * in a fixed order from its own workspace instead). */
int vlbm_conv2d_backward_weight(const vlbm_conv_desc* d, const uint16_t* x, const uint16_t* skip,
                                const uint16_t* gy, float* gw, float* gb, void* stream);
/* BF16 copies (round to nearest even) of FP32 weights w: w_bf16 in the same
 * layout and wt_bf16 transposed. */
int vlbm_conv2d_pack_weights(const vlbm_conv_desc* d, const float* w, uint16_t* w_bf16, uint16_t* wt_bf16,
                             void* stream);

typedef struct vlbm_adam {
  double lr, beta1, beta2, eps;
} vlbm_adam;
/* One Adam update (Kingma and Ba) of n FP32 parameters p with gradient g and
 * moments m, v at step >= 1 (bias-corrected). */
int vlbm_adam_step(float* p, const float* g, float* m, float* v, int64_t n, const vlbm_adam* hp, int64_t step,
                   void* stream);

/* The network: 5 levels with 32, 64, 128, 256, 256 channels; two 3x3 convs
 * with ReLU per level, stride-2 convs down, nearest 2x upsampling up with the
 * encoder output of each level appended (skip), a 3x3 head.  Input
 * [batch][height][width][3] FP32 features, output [batch][height][width][3]
 * FP32; height and width multiples of 16.  The parameter vector holds, layer
 * by layer (encoder levels 0..4, decoder levels 3..0, head), the FP32 weights
 * [c_out][3][3][c_in + c_skip] and the bias [c_out]; the first layer has 8
 * input channels (features 3..7 are zero) and the head 16 outputs (only the
 * first 3 are trained). */
typedef struct vlbm_surrogate_s* vlbm_surrogate;
int vlbm_surrogate_param_count(int height, int width, int64_t* n);
/* params: device or host FP32 vector of param_count values (copied).  The
 * object owns all its device memory; max_batch bounds the batch of later calls. */
int vlbm_surrogate_create(int height, int width, int max_batch, const float* params, void* stream,
                          vlbm_surrogate* out);
int vlbm_surrogate_forward(vlbm_surrogate s, const float* x, int batch, float* y);
/* Forward + mean squared error over the 3 outputs + backward.  loss (host,
 * nullable; synchronises when given), grad (device, nullable) receives the
 * gradient with respect to the parameter vector; both are bit-reproducible for
 * given weights and inputs (partial sums are added in a fixed order). */
int vlbm_surrogate_gradient(vlbm_surrogate s, const float* x, const float* target, int batch, double* loss,
                            float* grad);
/* Adam update with the last gradient (step count kept by the object). */
int vlbm_surrogate_adam(vlbm_surrogate s, const vlbm_adam* hp);
/* gradient + adam. */
int vlbm_surrogate_train_step(vlbm_surrogate s, const float* x, const float* target, int batch,
                              const vlbm_adam* hp, double* loss);
/* Copy the FP32 parameter vector out (synchronises); step (nullable) = Adam steps taken. */
int vlbm_surrogate_params(vlbm_surrogate s, float* out, int64_t* step);
int vlbm_surrogate_destroy(vlbm_surrogate s);

/* ---------------------------- measurement -------------------------------- */

/* STREAM-style bandwidth of the device: kind 0 read-only, 1 write-only,
 * 2 copy, over device buffers of `bytes` each (allocated and freed by the
 * call; use >= 2 GiB, well beyond the 256 MB last-level cache), 16-byte
 * accesses, regular or non-temporal (nontemporal != 0) loads and stores.
 * Several grid shapes are timed with HIP events over `reps` launches each on
 * `stream`; *gbps receives the best rate in GB/s (copy counts its reads and
 * writes), *best_grid (may be NULL) that launch's block count.  Synchronises.
 * Errors: VLBM_ERR_ARG, VLBM_ERR_NOMEM, VLBM_ERR_DEVICE. */
int vlbm_membench(int kind, int nontemporal, size_t bytes, int reps, void* stream, double* gbps, int* best_grid);

/* Message of the last failing call on this thread ("" if none). */
const char* vlbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VLBM_H */
