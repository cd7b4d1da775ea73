/*
 * fmsolve.h -- C ABI of the MI355X displacement-based FFT mechanical solver.
 *
 * The library solves the small-strain boundary value problem of Sec. 2.2
 * (Eq. GeneralBCtobesolved): div sigma = 0 on a voxel grid, sigma = F(eps),
 * with periodic, Dirichlet or Neumann conditions chosen per face and per
 * displacement component, by the displacement-based fixed point of Sec. 2.3
 * (Eqs. div_pol, div_pol_next_iter, GreenOp) summarised in Algorithm 1
 * (algFFT).  Each iteration evaluates the behaviour law at the integration
 * points, the finite-difference divergence at the nodes (HEX1 or TETRA2,
 * Sec. 2.5), the per-component, per-axis DFT / DCT-I / DST-I / DCT-III /
 * DST-III of Table 1 (Sec. 2.4), the B0 or 2mu0 discrete Green operator
 * (Eqs. NSGO2_HEX1, NSGO2_TETRA2, NSGO1_HEX1, NSGO1_TETRA2) and the inverse
 * transforms, with Anderson acceleration applied to the divergence of the
 * polarization (end of Sec. 2.4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Grid: n[0], n[1], n[2] voxels along x, y, z (cubic voxels of size h).
 *   Node fields have (n0+1)(n1+1)(n2+1) entries per component, voxel fields
 *   n0 n1 n2 entries per component and integration point; x is the fastest
 *   index (index = (z*N1 + y)*N0 + x).
 * - Symmetric tensors use the Voigt order xx, yy, zz, yz, xz, xy with tensor
 *   (not engineering) shear components.  Voxel outputs are component-major:
 *   out[c][ip][voxel].  TETRA2 has 2 integration points per voxel (T1, T2),
 *   HEX1 one.
 * - Memory ownership: the library never allocates device memory.  The caller
 *   passes one device workspace of at least fm_workspace_bytes() bytes (for a
 *   server: one arena) and device pointers for inputs and outputs; host tables
 *   are copied during the call.  All device work is issued on the HIP stream
 *   given at creation (hipStream_t passed as void*; NULL = default stream).
 *   A plan must not be used from two threads at once.
 * - Return codes: 0 = FM_OK; > 0 warnings (FM_W_NOT_CONVERGED: outputs and log
 *   are still written); < 0 errors.  fm_last_error() returns the message of
 *   the calling thread's last error.
 */
#ifndef FMSOLVE_H
#define FMSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FM_OK               0
#define FM_W_NOT_CONVERGED  1
#define FM_E_INVALID_ARG   -1
#define FM_E_BC            -2
#define FM_E_UNSUPPORTED   -3
#define FM_E_WORKSPACE     -4
#define FM_E_HIP           -5
#define FM_E_STATE         -6
#define FM_E_CAPACITY      -7

/* Boundary condition per face and component (Sec. 2.2): periodic (both
 * opposite faces), Dirichlet (u_q = u*_q, anti-symmetric extension of the
 * fluctuation) or Neumann (zero traction component, symmetric extension). */
#define FM_BC_PERIODIC  0
#define FM_BC_DIRICHLET 1
#define FM_BC_NEUMANN   2

/* Finite-difference schemes of Sec. 2.5. */
#define FM_HEX1   0
#define FM_TETRA2 1

/* Discrete Green operators of Sec. 2.6: B0 (Sec. 2.6.3, any BCs), 2mu0
 * (Sec. 2.6.2, lambda0 = 0) and C0 (Sec. 2.6.1 in its small-strain form of
 * Appendix A: the isotropic reference medium on the symmetric gradient,
 * coupling the three components per frequency).  C0 needs normal-mixed
 * conditions (Eq. SGO_BCs): along every axis the tangential components take
 * the condition opposite to the normal one's (Dirichlet <-> Neumann on each
 * face) or all three are periodic; fm_plan_create returns FM_E_BC otherwise. */
#define FM_GREEN_B0   0
#define FM_GREEN_2MU0 1
#define FM_GREEN_C0   2

/* Precision: everything in FP64, or transforms / Green / stencils / laws in
 * FP32 with the displacement accumulator, reductions, the Anderson least
 * squares and the macroscopic updates in FP64. */
#define FM_FP64       0
#define FM_FP32_MIXED 1

/* Behaviour laws (small strain). */
#define FM_LAW_ISO   0  /* p = {lambda, mu}: sigma = 2 mu eps + lambda tr(eps) 1 */
#define FM_LAW_CUBIC 1  /* p = {C11, C12, C44}, quat = crystal -> sample rotation */
#define FM_LAW_J2    2  /* p = {lambda, mu, sy0, H}: J2, sy = sy0 + H p (radial return) */
#define FM_LAW_CP    3  /* p = {C11, C12, C44, gdot0, n, tau0, taus, theta0}, quat:
                           FCC 12 {111}<110> systems, gdot = gdot0 |tau/tc|^n sign(tau),
                           tc = tau0 + (taus-tau0)(1-exp(-theta0 Gamma/(taus-tau0))),
                           backward Euler */
/* Hyperelastic laws of the finite-strain formulation (finite_strain = 1):
 * first Piola-Kirchhoff P = F Pi, F = 1 + grad u, E = (F^T F - 1)/2. */
#define FM_LAW_SVK      4  /* p = {lambda, mu}: Pi = lambda tr(E) 1 + 2 mu E (Sec. 3.1.2) */
#define FM_LAW_NEOHOOKE 5  /* p = {mu, K}: psi = mu/2 (J^-2/3 tr(F F^T) - 3) + K/2 (J - 1)^2
                              (Appendix B) */

typedef struct {
  int32_t n[3];            /* voxels along x, y, z (each >= 2) */
  double  h;               /* voxel size */
  int32_t bc[3][3][2];     /* [component q][axis i][face a], a = 0 at the origin */
  int32_t scheme;          /* FM_HEX1 or FM_TETRA2 */
  int32_t green;           /* FM_GREEN_B0, FM_GREEN_2MU0 or FM_GREEN_C0 */
  double  lambda0, mu0;    /* reference medium (Eq. FourierNSGO2) */
  int32_t prec;            /* FM_FP64 or FM_FP32_MIXED */
  double  tol;             /* equilibrium tolerance (Eq. equilibrium_condition) */
  int32_t max_iter;        /* iteration cap per load increment; an increment also stops,
                              not converged, when its error has not fallen below 0.99 of
                              its best for 200 iterations while within 100 tol (the
                              rounding floor of the precision) */
  int32_t aa_depth;        /* Anderson history depth, 1..4 (1 disables) */
  int32_t aa_period;       /* Anderson applied when m >= 2 and m % period == 0 */
  int32_t max_materials;   /* capacity of the material table */
  int32_t with_state;      /* 1 if any material is J2 or CP (internal variables) */
  int32_t finite_strain;   /* 1: Lagrangian finite strain (Sec. 2.2): the equilibrium of the
                              first Piola-Kirchhoff stress, FM_LAW_SVK / FM_LAW_NEOHOOKE
                              materials only; macro_sigma then holds <P> (P_11, P_22, P_33,
                              P_23, P_13, P_12), eps the Green-Lagrange strain and sig the
                              Cauchy stress, mixed_mask controls those <P> entries.  The C0
                              operator takes its finite-strain form (Eq. FourierSGO). */
} fm_plan_desc;

typedef struct {
  int32_t law;             /* FM_LAW_* */
  int32_t pad_;
  double  p[8];            /* parameters, see FM_LAW_* */
  double  quat[4];         /* unit quaternion (w, x, y, z); CUBIC and CP only */
} fm_material;

/* One load increment.  Prescribed displacement (set-up of Algorithm 1)
 *   u*_q(x) = c[q] + sum_l G[q][l] x_l + 1/2 sum_lm H[q][l][m] x_l x_m
 * at node positions x = (i h, j h, k h).  mixed_mask[c] != 0 makes Voigt
 * component c of sym(G) stress-controlled: it is moved after every iteration
 * so that <sigma>_c reaches mixed_target[c] (Sec. 3.2 normal-mixed loading).
 * traction[i][a][q] is the applied traction T*_q, uniform over face a of axis
 * i (Sec. 2.2: sigma_iq (-1)^(a+1) = T*_q, i.e. the traction vector
 * sigma n); it may be non-zero only where u_q is Neumann on that face
 * (FM_E_BC otherwise).  The solver adds D* = div_d P*, the divergence of the
 * applied stress that is 2 T* on the face's mirror voxels (Fig. NeumannBC).
 * ustar, optional (NULL: none), adds a nodal field to u*: device FP64, 3 x
 * nodes in the layout of fm_outputs.u (component-major, x fastest), read
 * during the increment's begin and the solve's end, so it must stay valid
 * until fm_solve returns (fm_batch_solve: returns; server: the request
 * completes).  As the paper's u* (Sec. 2.2, Algorithm 1 set-up) only its
 * values on the Dirichlet faces of each component shape the solution; the
 * rest is absorbed by u^f. */
typedef struct {
  double  c[3];
  double  G[3][3];
  double  H[3][3][3];
  int32_t mixed_mask[6];
  double  mixed_target[6];
  double  dt;
  double  traction[3][2][3];
  const double* ustar;
} fm_load_step;

/* Outputs; every pointer may be NULL.  u, eps, sig are device pointers
 * (FP64) written after the last increment: u = u^f + u* at the nodes (3 x
 * nodes), eps and sig at the integration points (6 x n_ppv x voxels).
 * macro_sigma (host, n_steps x 6), iters and converged (host, n_steps). */
typedef struct {
  double*  u;
  double*  eps;
  double*  sig;
  double*  macro_sigma;
  int32_t* iters;
  int32_t* converged;
} fm_outputs;

typedef struct {
  int32_t step, iter;
  double  err;             /* equilibrium error before the update (FP64) */
  int32_t aa_applied;      /* Anderson combination used for this update */
  int32_t rs_fp64;         /* 1 if this iterate's strain, law and divergence ran in
                              FP64 (an FP32-mixed plan moves them to FP64 once its
                              error stalls within 100 tol, i.e. at the FP32 rounding
                              floor; 0 for FP64 plans, which always compute in FP64) */
  double  macro_sigma[6];  /* <sigma> of this iterate (FP64) */
  double  t_us;            /* device time from the increment's first control
                              evaluation to this one, microseconds (the
                              difference of two entries is their iterations' time) */
} fm_iter_entry;

typedef struct {
  fm_iter_entry* entries;  /* host array */
  int32_t capacity;
  int32_t count;           /* written by the library */
} fm_iter_log;

typedef struct fm_plan   fm_plan;
typedef struct fm_server fm_server;

/* Bytes of device workspace a plan needs (0 on invalid descriptor). */
size_t fm_workspace_bytes(const fm_plan_desc* desc);

/* Create a plan: validates the BCs (periodic faces must pair, Sec. 2.5.1),
 * classifies each (component, axis) into its Table 1 transform, builds the
 * 1D frequency and twiddle tables inside d_workspace.  d_workspace must stay
 * valid until fm_plan_destroy.  Errors: FM_E_INVALID_ARG, FM_E_BC,
 * FM_E_UNSUPPORTED (grid too small / too large for one pencil), FM_E_WORKSPACE
 * (ws_bytes too small), FM_E_HIP. */
int fm_plan_create(const fm_plan_desc* desc, void* d_workspace, size_t ws_bytes,
                   void* hip_stream, fm_plan** out);

/* Material map: d_mat_id (device, int32 per voxel, values < n_mat) and the
 * host table of n_mat entries (n_mat <= max_materials).  Resets the internal
 * variables and the displacement to zero.  Errors: FM_E_INVALID_ARG,
 * FM_E_CAPACITY, FM_E_UNSUPPORTED (J2/CP without with_state), FM_E_HIP. */
int fm_set_material(fm_plan* plan, const int32_t* d_mat_id, int32_t n_mat,
                    const fm_material* table);

/* Run the load path (Alg. 1, all increments) from the current state.
 * Returns FM_OK, FM_W_NOT_CONVERGED (some increment hit max_iter or stagnated), or an
 * error.  log may be NULL; entries beyond its capacity are dropped. */
int fm_solve(fm_plan* plan, const fm_load_step* steps, int32_t n_steps,
             fm_outputs* out, fm_iter_log* log);

/* Device bytes of the batch descriptors (work lists, per-solve and per-pass
 * descriptors) for fm_batch_solve over these plans. */
size_t fm_batch_workspace_bytes(fm_plan* const* plans, int32_t n_plans);

/* Several independent plans advanced together: every kernel launch covers
 * the tiles of all unfinished solves, and each solve moves through its own
 * load increments.  Arrays have n_plans entries; plans must share one stream
 * and one precision; d_batch_ws holds fm_batch_workspace_bytes() bytes.
 * status[i] receives each solve's return code (FM_OK / FM_W_NOT_CONVERGED);
 * the function returns the worst of them or an error. */
int fm_batch_solve(fm_plan* const* plans, int32_t n_plans,
                   const fm_load_step* const* steps, const int32_t* n_steps,
                   fm_outputs* outs, fm_iter_log* logs, int32_t* status,
                   void* d_batch_ws, size_t ws_bytes);

/* Operator entry points (same kernels as fm_solve), for checking one stage:
 *
 * fm_apply_green: d_w = IDT( DT(d_x) / den ) per component, i.e. minus the
 * B0 / 2mu0 discrete Green operator (Eqs. NSGO2_*, NSGO1_*) applied to the
 * node field d_x, with the transforms of Table 1 and the dismissed points of
 * Sec. 2.7.2 (d_x and d_w: device FP64, 3 x nodes).  Overwrites the plan's
 * displacement and history (call fm_set_material again before fm_solve).
 *
 * fm_residual: for the fluctuation d_uf (device FP64, 3 x nodes) and the
 * load increment *step evaluated against the current internal variables,
 * writes D = div_d sigma at the nodes (Algorithm 1; 0 at dismissed nodes)
 * to d_D (device FP64, 3 x nodes) and the equilibrium error and macroscopic
 * stress to the host (err: 1 double, macro: 6 doubles, either may be NULL).
 * d_uf is u^f alone; a nodal u* of the step is added to it.  Overwrites the
 * plan's displacement. */
int fm_apply_green(fm_plan* plan, const double* d_x, double* d_w);
int fm_residual(fm_plan* plan, const fm_load_step* step, const double* d_uf, double* d_D,
                double* err, double* macro);

/* Per-kernel timing of the iteration (for roofline reporting): runs n_iter
 * iterations of *step with the convergence test disabled, recording HIP
 * events on the plan's stream around each of the FM_N_KERNELS launches, and
 * writes the mean duration in milliseconds per kernel to ms[FM_N_KERNELS]
 * (order: stress+divergence, control, gram, alpha, x-forward, y-forward,
 * z-forward+Green+inverse, y-inverse, x-inverse+update).  Overwrites the
 * plan's displacement. */
#define FM_N_KERNELS 9
int fm_profile_iterations(fm_plan* plan, const fm_load_step* step, int32_t n_iter, double* ms);

/* Launch mode of the iteration chunks of fm_solve, fm_batch_solve and the
 * server (process-wide): enable != 0 (the default) enqueues each chunk of
 * 1, 2, 4, ..., 32 iterations as one HIP graph, captured at first use per
 * plan, batch or server group on a private stream and replayed on the
 * caller's stream; 0 launches the nine kernels of every iteration directly.
 * Results are identical in both modes.  Returns FM_OK. */
int fm_set_graph_launch(int enable);

/* Transform-kernel autotuner (per plan).  Choices are kept for the process
 * per transform signature (grid, per-component transform kinds, precision,
 * scheme, Green operator): a plan whose signature was tuned before takes the
 * stored choice without timing (ms then holds -1 everywhere).  Otherwise, for each of the five axis passes
 * (x forward, y forward, z forward+Green+inverse, y inverse, x inverse),
 * times n_iter iterations of *step with every applicable candidate kernel --
 * 0 the wavefront kernel (pencil lengths 64E, or 32E / 16E for E in {1, 3}),
 * 1..3 the generic LDS kernel with the largest, half and quarter number of
 * transforms per block -- and keeps the fastest per pass for this plan's
 * later solves and batches.  A pass whose launch would hold fewer than
 * about four blocks per compute unit is timed with its tiles repeated up to
 * that fill (time divided by the repetitions): its cost when other solves
 * share the device, as in fm_batch_solve and the server.
 * choice[5] (host, optional) receives the chosen candidate per pass;
 * ms[4*5] (host, optional) the mean time in ms per candidate and pass (-1 if
 * not applicable).  Overwrites the plan's displacement and spectral buffers
 * (reset it with fm_set_material before solving). */
int fm_autotune(fm_plan* plan, const fm_load_step* step, int32_t n_iter, int32_t* choice, double* ms);

/* Iterations performed by the last fm_solve / fm_batch_solve of this plan. */
int64_t fm_plan_total_iterations(const fm_plan* plan);

void fm_plan_destroy(fm_plan* plan);

/* ---- Serving: continuous batching over one device arena -------------- */
typedef struct {
  fm_plan_desc        desc;
  const int32_t*      mat_id;      /* host, n0 n1 n2 voxels */
  int32_t             n_mat;
  const fm_material*  table;       /* host, n_mat entries */
  const fm_load_step* steps;       /* host, n_steps */
  int32_t             n_steps;
  double*             macro_sigma; /* host result buffer, n_steps x 6, may be NULL */
  int32_t*            iters;       /* host, n_steps, may be NULL */
  double              arrival_s;   /* caller clock, used for latency statistics */
} fm_request;

typedef struct {
  int64_t completed, admitted, waiting, active, rejected;
  double  p50_latency_s, p99_latency_s, mean_latency_s;
  double  voxel_iters;           /* sum over completed solves of voxels x iterations */
  size_t  arena_in_use, arena_peak;
} fm_stats;

/* The server owns no memory: d_arena (device, arena_bytes) holds every
 * admitted request's workspace.  Requests are admitted in arrival order when
 * their workspace fits in the arena and fewer than max_active are running. */
int fm_server_create(void* d_arena, size_t arena_bytes, int32_t max_active,
                     void* hip_stream, fm_server** out);
/* Copies the request's host data; returns a ticket.  FM_E_CAPACITY if the
 * request can never fit the arena. */
int fm_server_submit(fm_server* s, const fm_request* req, double now_s, uint64_t* ticket);
/* Advance every active solve by up to `iters` iterations, retire finished
 * ones (results written to the request's host buffers), admit waiting ones.
 * now_s is the caller's clock for latency bookkeeping. */
int fm_server_step(fm_server* s, int32_t iters, double now_s);
/* state: 0 waiting, 1 running, 2 done, 3 failed; latency (s) when done. */
int fm_server_poll(fm_server* s, uint64_t ticket, int32_t* state, double* latency_s);
int fm_server_stats(fm_server* s, fm_stats* out);
void fm_server_destroy(fm_server* s);

/* ---- Allocation-free solve ---------------------------------------------
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid it): fm_solve_static does what fm_plan_create +
 * fm_set_material + fm_solve + fm_plan_destroy do, with the plan's workspace
 * taken from a device array inside the library (FM_STATIC_SCRATCH_BYTES per
 * GPU, held by each GPU the library runs on until the process ends) instead
 * of a caller buffer; iterations are launched directly (no captured graphs).
 * The caller passes the inputs (d_mat_id: device, int32 per voxel; table and
 * steps: host) and the outputs as for fm_solve.  Returns FM_E_CAPACITY when
 * fm_workspace_bytes(desc) exceeds FM_STATIC_SCRATCH_BYTES, otherwise what
 * fm_solve returns.  Every call on one GPU uses that GPU's one array: calls
 * that overlap on a GPU (two threads or two streams) race; the array keeps
 * the last call's contents, and each call initialises what it reads. */
#define FM_STATIC_SCRATCH_BYTES (64u << 20)
int fm_solve_static(const fm_plan_desc* desc, const int32_t* d_mat_id, int32_t n_mat, const fm_material* table,
                    const fm_load_step* steps, int32_t n_steps, fm_outputs* out, fm_iter_log* log,
                    void* hip_stream);

const char* fm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FMSOLVE_H */
