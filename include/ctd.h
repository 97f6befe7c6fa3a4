/*
 * ctd.h -- C-ABI of the MI355X convolution-tensor-decomposition (CTD) solver
 * for the Allen-Cahn equation (Lu, Yuan, Guo, arXiv 2410.15519).
 *
 * One time step of the stabilized semi-implicit scheme (Sec. 2.5,
 * eq. AC-discrete-semi-stable-K) is solved in separated form (Sec. 3.1,
 * eq. CTD): the new field is a sum of rank-one products of 1D convolution-FE
 * functions (Sec. 3.2, App. B/C), built by greedy enrichment with alternating
 * fixed-point sweeps over the directions (Sec. 3.3; directional systems
 * eq. ux/KxQx, derived in App. D).  All arithmetic of a step runs in HIP
 * kernels for gfx950; the host only builds the 1D CFE tables at init and
 * sequences launches.
 *
 * Conventions
 *   - Every function returns an int status: CTD_OK (0) or a negative code.
 *     Nothing aborts or throws; ctd_last_error() gives a message.
 *   - Host arrays passed in are copied during the call; the caller keeps
 *     ownership.  Device memory of an instance comes from the caller's
 *     allocator when ctd_problem.dev_alloc / dev_free are set (e.g. a
 *     framework's caching allocator), else from hipMallocAsync on the
 *     instance's stream; it is held until ctd_destroy / ctd_batch_destroy.
 *   - All device work of a handle is ordered on the HIP stream given at
 *     creation (NULL = the null stream).  One host thread at a time per handle.
 *   - Factor matrices are column-major: column m (one mode) is contiguous,
 *     element (i, m) at [m * nodes + i].  Nodal coefficients equal nodal
 *     values (Kronecker-delta property, Sec. 3.2).
 *   - Dense nodal grids are C-ordered: axis 0 slowest.
 */
#ifndef CTD_H
#define CTD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CTD_ABI_VERSION 4

enum {
  CTD_OK = 0,
  CTD_EINVAL = -1,        /* invalid parameter; nothing allocated           */
  CTD_ENOMEM = -2,        /* device or host allocation failed               */
  CTD_EDEVICE = -3,       /* HIP runtime error                              */
  CTD_ENONFINITE = -4,    /* a mode amplitude became NaN/Inf                */
  CTD_ESTATE = -5,        /* call not valid in the handle's current state   */
  CTD_EUNSUPPORTED = -6,  /* valid but outside what the library supports    */
  CTD_EAGAIN = -7         /* server: not finished / no free slot            */
};

enum { CTD_PREC_FP64 = 0, CTD_PREC_MIXED = 1 };
enum { CTD_SCHED_ADAPTIVE = 0, CTD_SCHED_REPLAY = 1 };
enum { CTD_INIT_HASH = 0, CTD_INIT_WARM = 1 };
enum { CTD_DTYPE_F64 = 0, CTD_DTYPE_F32 = 1 };
/* Directional banded solve: block cyclic reduction (any n), or fast
 * diagonalisation with the axis' generalised eigenvectors (dense n x n FP64
 * per axis shape, host set-up O(n^3) once per process and shape).  AUTO takes
 * fast diagonalisation for 3D instances with n <= 1024 on every axis (many
 * thousands of solves per step amortise the set-up) and cyclic reduction
 * otherwise. */
enum { CTD_SOLVE_AUTO = 0, CTD_SOLVE_BCR = 1, CTD_SOLVE_FD = 2 };

/*
 * Problem statement (Sec. 2.1-2.5, Sec. 3.2 parameters p, a, s; Sec. 3.3
 * tolerances eps1, eps2 and the adaptive mode cap M_c).
 *
 * Coefficients: either the paper form (L, kappa, a0, alpha) or, when all four
 * are NaN, the epsilon form u_t = eps^2 Lap u - (u^3 - u) with stabilizer S,
 * read as L = 1, kappa = eps^2, a0 = 1/4, alpha = S.
 * Mesh: uniform, nodes[d] >= 2*patch_s + 2 nodes on [lo[d], hi[d]].
 * CFE space: patch size patch_s >= 1, reproduction order 0 <= poly_p <=
 *   patch_s, dilation a in natural element units (element = [-1, 1]),
 *   gauss_points Gauss-Legendre points per element for every integral.
 * Stopping: fixed-point sweeps stop when the relative Frobenius change of the
 *   nodal rank-one term is <= fp_tol (from the second sweep) or after
 *   fp_max_iter sweeps; enrichment stops once a mode's nodal max is
 *   <= enrich_tol, or at max_modes (the cap of the adaptive variant).
 * Zero values of dilation_a, gauss_points, fp_tol, fp_max_iter select the
 * defaults 12, 5, 1e-2, 20 (ctd_problem_default fills everything).
 * actd (Sec. 3.3 adaptive algorithm; Sec. 4.2 uses it in 3D): nonzero
 *   makes max_modes the critical mode count M_c of the hybrid CTD/CFE
 *   scheme: a step whose enrichment reaches max_modes with the last mode
 *   still above enrich_tol drops its modes and is computed by the full
 *   tensor-product CFE solve of the same scheme from u^k (exact, by the
 *   generalised eigenbases of (K_d, M_d)); the next step's CTD starts from
 *   that field.  2D: u^{k+1} is held as nodes[1] modes (column j of the
 *   nodal field times the nodal unit vector j of axis 1, amplitude 1), which
 *   is the field itself.  3D: u^{k+1} is held as the nodal tensor (a field
 *   state with no modes: the warm guess falls back to the counter-based
 *   vector); the next step's integrals of u^k come from the tensor
 *   c M3 U - int N w(U) on the tensor Gauss grid, formed once per step.
 *   Needs nodes[d] <= 2048, in 3D also at most 2^30 tensor Gauss points
 *   (about 200 nodes per axis); the set-up computes the axes' eigenbases on
 *   the host (O(n^3)); the device footprint holds nodes[1] modes of u^k
 *   (2D) or the field, its right-hand-side tensor and two Gauss-grid
 *   buffers (3D).
 * dev_alloc / dev_free / alloc_ctx: optional device allocator (both set or
 *   both NULL).  dev_alloc(bytes, hip_stream, ctx) returns device memory
 *   usable in stream order on hip_stream (NULL = out of memory ->
 *   CTD_ENOMEM); dev_free(ptr, bytes, hip_stream, ctx) returns it, called
 *   only after the instance's stream has been synchronised.  The callbacks
 *   may run on the library's worker threads (batch, server) and must be
 *   thread-safe.  Stability: the scheme is energy stable for
 *   alpha >= max(w')/2 = 4 a0 on |u| <= 1 (Sec. 2.5,
 *   eq. AC-discrete-semi-stable-step); a smaller alpha is accepted and
 *   reported by ctd_step_info.stability_warning.
 * rd_tol: reduced integration domain of the 2D M_xy (Sec. 3.3, eq. MxyRD):
 *   an element whose Gauss-point values of w(u^k) = 4 a0 (u^3 - u) all
 *   satisfy |w| <= rd_tol is left out of the integral (an approximation for
 *   rd_tol > 0; 0 = the full integral).  Finite and >= 0; with dim 3 or
 *   actd a positive value is CTD_EUNSUPPORTED (the 3D load is exact in
 *   separated form; the full CFE step integrates the whole domain).
 * w_rank, w_iters: separated integration of the 2D M_xy (Sec. 3.3, eq.
 *   MxySep): the Gauss-grid values of L w(u^k) are replaced by w_rank
 *   rank-one terms a_q(x) b_q(y) of a greedy (PGD) decomposition, each from
 *   w_iters alternating least-squares updates against the residual (b
 *   starting from the counter-based vector of term q), and M_xy becomes the
 *   sum over the terms of products of 1D integrals.  An approximation for
 *   every w_rank below the rank of w; 0 = the full integral.  w_rank in
 *   [0, 256], w_iters in [0, 100000]; w_rank > 0 needs dim 2, no actd and
 *   rd_tol = 0 (CTD_EUNSUPPORTED otherwise).  Holds W and W^T on the Gauss
 *   grid: 16 nq0 nq1 bytes more device memory.
 */
typedef void* (*ctd_dev_alloc_fn)(uint64_t bytes, void* hip_stream, void* ctx);
typedef void (*ctd_dev_free_fn)(void* ptr, uint64_t bytes, void* hip_stream, void* ctx);

typedef struct ctd_problem {
  int32_t abi_version;      /* CTD_ABI_VERSION */
  int32_t dim;              /* 2 or 3 */
  int64_t nodes[3];
  double lo[3], hi[3];
  double eps, S, dt;
  double L, kappa, a0, alpha;
  int32_t patch_s, poly_p;
  double dilation_a;
  int32_t gauss_points;
  int32_t fp_max_iter;
  double fp_tol;
  double enrich_tol;
  int32_t max_modes;
  int32_t precision;        /* CTD_PREC_FP64 | CTD_PREC_MIXED */
  int32_t schedule;         /* CTD_SCHED_ADAPTIVE | CTD_SCHED_REPLAY */
  int32_t init_mode;        /* CTD_INIT_HASH | CTD_INIT_WARM */
  int32_t energy_each_step; /* nonzero: ctd_step fills info.energy */
  int32_t solve_method;     /* CTD_SOLVE_AUTO | CTD_SOLVE_BCR | CTD_SOLVE_FD */
  int32_t actd;             /* nonzero: full CFE solve past max_modes (2D) */
  uint64_t seed;            /* keys the counter-based mode initialisation */
  ctd_dev_alloc_fn dev_alloc;   /* optional device allocator (see above)  */
  ctd_dev_free_fn dev_free;
  void* alloc_ctx;
  double rd_tol;            /* 2D reduced integration domain (see above); 0 */
  int32_t w_rank;           /* 2D separated w: terms (see above); 0 = off  */
  int32_t w_iters;          /* alternating updates per term; 0 = 30        */
} ctd_problem;

/* Per-step report of ctd_step. */
typedef struct ctd_step_info {
  int32_t modes;            /* modes of u^{k+1} */
  int32_t sweeps;           /* fixed-point sweeps summed over modes */
  int32_t capped;           /* 1 if max_modes ended the enrichment */
  int32_t fp_unconverged;   /* modes that hit fp_max_iter */
  int32_t zero_mode;        /* 1 if a zero-amplitude mode ended the step */
  int32_t energy_increase;  /* 1 if energy rose by more than 1e-12 relative */
  int32_t full_solve;       /* 1 if the step was the full CFE solve (actd);
                               modes is then nodes[1] (2D) or 0 (3D field
                               state) */
  int32_t stability_warning;/* 1 if alpha < max(w')/2 = 4 a0: the energy law of
                               App. A is not guaranteed (Sec. 2.5)          */
  double energy;            /* E(u^{k+1}) if energy_each_step, else NaN */
  double last_term_max;     /* nodal max of the last appended mode */
  double ms;                /* wall time of the step on the host clock */
} ctd_step_info;

typedef struct ctd_solver ctd_solver;

/* Fill *p with defaults: dim 2, 64 nodes on [0,1], eps 0.02, S 2, dt 1e-3,
 * s = 2, p = 2, a = 12, 5 Gauss points, fp_tol 1e-2, 20 sweeps,
 * enrich_tol 1e-8, 64 modes, FP64, adaptive, warm initial guess of a mode
 * (mode m of u^k, the counter-based vector past the modes of u^k), library
 * allocation. */
int ctd_problem_default(ctd_problem* p);

/* Validate the problem, build the 1D CFE tables (App. B/C, eq. KxxMxx) on the
 * host in FP64, allocate device memory and load the initial field
 *   u0 = sum_m amp[m] prod_d init[d][:, m]     (eq. CTD),
 * init[d]: host, nodes[d] x m0 column-major; amp: host, m0 values or NULL
 * (all ones).  hip_stream: hipStream_t or NULL.  On error *out stays NULL. */
int ctd_init(const ctd_problem* p, int32_t m0, const double* const* init,
             const double* amp, void* hip_stream, ctd_solver** out);

/* Advance nsteps time steps (Sec. 3.3 algorithm per step).  info: host array
 * of nsteps entries or NULL.  Synchronises the stream before returning. */
int ctd_step(ctd_solver* s, int32_t nsteps, ctd_step_info* info);

/* Discrete energy E(u^k) = int a0 (u^2-1)^2 + kappa/2 |grad u|^2 (Sec. 2.1)
 * on the separated tensor Gauss rule, FP64. */
int ctd_energy(ctd_solver* s, double* E);

/* Dense nodal field of u^k, u[i0, i1(, i2)] = sum_m sigma_m prod_d X_d[i_d, m]
 * (eq. CTD); nodal values equal the nodal coefficients by the Kronecker-delta
 * property of the CFE shape functions (Sec. 3.2), so this is the field at the
 * mesh nodes.  out: caller-owned buffer of dtype CTD_DTYPE_F64 or
 * CTD_DTYPE_F32, device memory if on_device != 0, else host memory.
 * strides: dim element strides (axis d of node index i_d at
 * out[sum_d i_d strides[d]]), all > 0 and such that distinct nodes map to
 * distinct elements (not checked beyond positivity); NULL = C order, axis 0
 * slowest.  Non-contiguous layouts pass through a contiguous device
 * temporary.  Synchronises the stream before returning. */
int ctd_reconstruct(ctd_solver* s, void* out, int32_t dtype, int32_t on_device,
                    const int64_t* strides);

/* Current separated field u^k = sum_m amp[m] prod_d out[d][:, m] (eq. CTD;
 * nodal coefficients = nodal values, Sec. 3.2): *m modes; amp (cap values)
 * and out[d] (nodes[d] x cap, column-major), caller-owned host buffers; any
 * may be NULL to query *m only.  cap < *m with a buffer given: CTD_EINVAL.
 * Factors are unit in the M_d norm except along axis 0, which carries the
 * sign; amp >= 0.  Together with ctd_get_step_index this is a checkpoint:
 * ctd_init(p, m, out, amp, ...) and ctd_set_step_index resume the run.  A
 * 3D field state (actd) is written as nodes[1] nodes[2] modes: mode
 * j nodes[2] + k = U[:, j, k] times the unit vectors e_j and e_k, amplitude
 * 1. */
int ctd_get_modes(ctd_solver* s, int32_t* m, double* amp, double* const* out,
                  int32_t cap);

/* Time-step counter (keys the mode initialisation); settable for resume. */
int ctd_get_step_index(ctd_solver* s, int64_t* k);
int ctd_set_step_index(ctd_solver* s, int64_t k);

/* Decision log of the last ctd_step call: per step, the number of modes
 * followed by the sweep count of each mode (0 modes: the step's first mode
 * had zero amplitude and u^{k+1} = 0), or the single entry -1 for a
 * step computed by the full CFE solve (actd), concatenated.  *len = ints
 * written (or needed, if cap is too small -> CTD_EINVAL). */
int ctd_get_decisions(ctd_solver* s, int32_t* buf, int64_t cap, int64_t* len);

/* Decisions for the next ctd_step call in CTD_SCHED_REPLAY mode, same
 * format; the step then takes no threshold decision of its own. */
int ctd_set_decisions(ctd_solver* s, const int32_t* buf, int64_t len);

/* Message of the last error on this handle (or of the last failed
 * ctd_init when s is NULL); never NULL. */
const char* ctd_last_error(const ctd_solver* s);

void ctd_destroy(ctd_solver* s);   /* NULL-safe; synchronises the stream */

/* Device bytes an instance of this problem with m0 initial modes holds
 * (the allocation ctd_init makes; host tables and pinned scalars excluded).
 * Used for admission by HBM footprint.  Works without a device (then the
 * LDS limit is taken as 64 KiB, which can only over-estimate). */
int ctd_footprint_bytes(const ctd_problem* p, int32_t m0, uint64_t* bytes);

/* ---------------------------------------------------------------------- *
 * Batched execution (many independent, uneven instances).  The instances
 * advance concurrently, either in lockstep rounds of multi-instance launches
 * (2D) or on a pool of worker threads, each with its own non-blocking HIP
 * stream, taking instances longest-first (cost ~ sweeps x directions x
 * per-sweep work, from the shape and mode cap); see ctd_batch_set_mode.
 * Each instance's arithmetic is that of a single ctd_solver: a result does
 * not depend on the batch around it.
 * ---------------------------------------------------------------------- */
typedef struct ctd_batch ctd_batch;

/* problems[i], m0[i], inits[i] (dim pointers), amps[i] (or NULL) as in
 * ctd_init.  Instances are set up on hip_stream; stepping uses the pool. */
int ctd_batch_create(int32_t count, const ctd_problem* problems,
                     const int32_t* m0, const double* const* const* inits,
                     const double* const* amps, void* hip_stream,
                     ctd_batch** out);
/* Worker threads (and streams) of the pool, 1..64; default 8. */
int ctd_batch_set_workers(ctd_batch* b, int32_t workers);
/* Executor.  LOCKSTEP: the instances advance together in rounds, each round
 * one multi-instance launch per phase of a sweep (mode initialisation,
 * right-hand sides, banded solves, Grams) for every instance at that phase,
 * and one read-back of all instances' decision scalars; each instance takes
 * its own decisions (Sec. 3.3 adaptive algorithm) and ends its steps with its
 * own launches.  Needs 2D instances, adaptive schedule, cyclic-reduction
 * solves of one band width (CTD_EUNSUPPORTED otherwise).  STREAMS: the
 * worker pool above.  AUTO (default): LOCKSTEP when every instance allows
 * it, else STREAMS.  Results are the same under either executor. */
enum { CTD_BATCH_AUTO = 0, CTD_BATCH_LOCKSTEP = 1, CTD_BATCH_STREAMS = 2 };
int ctd_batch_set_mode(ctd_batch* b, int32_t mode);
/* Advance every instance nsteps steps; info: count * nsteps entries
 * (instance-major) or NULL.  Returns when all are done (or on the first
 * error, after the running instances reach a step boundary). */
int ctd_batch_step(ctd_batch* b, int32_t nsteps, ctd_step_info* info);
int ctd_batch_get_modes(ctd_batch* b, int32_t i, int32_t* m, double* amp,
                        double* const* out, int32_t cap);
int ctd_batch_reconstruct(ctd_batch* b, int32_t i, void* out, int32_t dtype,
                          int32_t on_device, const int64_t* strides);
const char* ctd_batch_last_error(const ctd_batch* b);
void ctd_batch_destroy(ctd_batch* b);

/* ---------------------------------------------------------------------- *
 * Served execution with continuous batching.  Requests (a problem, its
 * initial modes and a step count) are queued in arrival order, by route.
 * 2D adaptive requests with cyclic-reduction solves (the 2D default) run in
 * lockstep: a server thread admits each as soon as the summed device
 * footprint of the admitted-but-unfetched requests plus its own stays
 * within the HBM budget, adds it to the running set at its first step, and
 * advances the whole set in rounds of multi-instance launches (see
 * ctd_batch_set_mode); a request leaves the set when its steps are done.
 * Other requests go to worker threads, each with its own non-blocking HIP
 * stream, which admit the oldest one as soon as a worker is idle and its
 * footprint fits.  Requests that arrive while others run thus start as
 * memory (and workers) free up, and their work overlaps on the device.
 * Results (the modes) stay device-resident until fetched.  A request's
 * arithmetic is that of a single ctd_solver: the same alone, in any mix and
 * on either route.
 * ---------------------------------------------------------------------- */
typedef struct ctd_server ctd_server;

enum { CTD_REQ_QUEUED = 0, CTD_REQ_RUNNING = 1, CTD_REQ_DONE = 2, CTD_REQ_FAILED = 3 };

typedef struct {
  int32_t state;           /* CTD_REQ_*                                        */
  int32_t steps_done;
  int32_t modes;           /* modes of the current field                        */
  int32_t error;           /* CTD_* code when FAILED                            */
  double t_submit_ms;      /* times on the server's monotonic clock, ms since    */
  double t_start_ms;       /* ctd_server_create; 0 when not reached yet          */
  double t_done_ms;
  uint64_t footprint;      /* admitted device bytes                             */
} ctd_request_status;

typedef struct {
  int64_t submitted, completed, failed, queued, running;
  uint64_t bytes_in_use, budget;
  int64_t steps_done;
  double busy_ms;          /* wall time with at least one request running        */
} ctd_server_stats;

/* budget_bytes: device bytes the admitted requests may hold (0: 80% of the
 * free device memory); workers: 1..64 concurrent requests. */
int ctd_server_create(uint64_t budget_bytes, int32_t workers, ctd_server** out);
/* Copies the problem and the initial modes (host, as in ctd_init).  A
 * request larger than the whole budget fails at once (CTD_ENOMEM). */
int ctd_server_submit(ctd_server* srv, const ctd_problem* p, int32_t m0,
                      const double* const* init, const double* amp,
                      int32_t nsteps, int64_t* ticket);
int ctd_server_status(ctd_server* srv, int64_t ticket, ctd_request_status* st);
/* Block until the request is DONE or FAILED, or timeout_ms passes
 * (< 0: no limit); CTD_EAGAIN on timeout; a FAILED request returns its own
 * error code (its message through ctd_server_last_error). */
int ctd_server_wait(ctd_server* srv, int64_t ticket, double timeout_ms);
/* Modes of a DONE request (host buffers as in ctd_get_modes, cap >= modes);
 * release != 0 frees its device memory and forgets the ticket.  A FAILED
 * request returns its error code; with release != 0 its ticket is forgotten
 * too.  Tickets are claimed under the server's lock, so concurrent fetches of
 * one ticket are safe: the first release wins, later calls get CTD_EINVAL
 * (unknown ticket) or, while a release is in progress, CTD_EAGAIN. */
int ctd_server_fetch(ctd_server* srv, int64_t ticket, int32_t* m, double* amp,
                     double* const* out, int32_t cap, int32_t release);
int ctd_server_get_stats(ctd_server* srv, ctd_server_stats* st);
const char* ctd_server_last_error(const ctd_server* srv);   /* never NULL */
/* Stops admitting, lets running requests finish their current step (or
 * lockstep round), frees everything.  NULL-safe. */
void ctd_server_destroy(ctd_server* srv);
/* on = 0: later submissions all take the worker route (default 1: eligible
 * 2D requests run in lockstep).  Results do not depend on the route. */
int ctd_server_set_lockstep(ctd_server* srv, int32_t on);

/* ---------------------------------------------------------------------- *
 * Low-level kernel entry points on caller device memory (tests, tuning).
 * ---------------------------------------------------------------------- */

/* Generalised eigenvectors of the axis' stiffness and mass matrices (host,
 * FP64): V^T M V = I, V^T K V = diag(mu), used by the fast-diagonalisation
 * directional solve.  Axis as in ctd_problem (nodes, box, patch_s, poly_p,
 * dilation_a, gauss_points; 0 = default).  V: host, n x n row-major (entry i
 * of eigenvector k at V[i*n + k]); mu: host, n values; caller-owned. */
int ctd_axis_fast_diag(int64_t n, double lo, double hi, int32_t s, int32_t p, double a,
                       int32_t ng, double* V, double* mu);

/* Plain device-to-device copy by a kernel (16 bytes per lane and pass; bytes
 * a multiple of 16): a transfer of known size, used to scale hardware
 * traffic counters. */
int ctd_kernel_copy(void* dst, const void* src, uint64_t bytes, void* hip_stream);

/* Symmetric positive definite banded solve, FP64: count independent systems
 * A_k x_k = b_k, A_k = alpha[k] Mb + beta[k] Kb with Mb, Kb in lower band
 * storage ((bw+1) x n, row t holds A[i+t, i] at [t*n + i]).  b, x: device,
 * count x n.  alpha/beta: device, count values.  Block cyclic reduction, one
 * workgroup per system; systems whose block data exceed the LDS use a
 * stream-ordered device workspace allocated and released by the call. */
int ctd_kernel_band_solve(int32_t n, int32_t bw, const double* Mb,
                          const double* Kb, const double* alpha,
                          const double* beta, const double* b, double* x,
                          int32_t count, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as ctd_kernel_band_solve, same arguments and results, allocating
 * nothing.  The cyclic-reduction workspace of systems too large for LDS lives
 * in a static device array of CTD_NOALLOC_SCRATCH_BYTES per device, held
 * until the process ends; a call whose count x per-system workspace exceeds
 * it returns CTD_ENOMEM and launches nothing.  Every call on one device
 * shares that array: calls that overlap on a device (different streams or
 * threads) race and must be serialised by the caller.  The array needs no
 * clearing (each system writes its block data before reading them). */
#define CTD_NOALLOC_SCRATCH_BYTES (16u << 20)
int ctd_kernel_band_solve_noalloc(int32_t n, int32_t bw, const double* Mb,
                                  const double* Kb, const double* alpha,
                                  const double* beta, const double* b, double* x,
                                  int32_t count, void* hip_stream);

/* Per-kernel timing of the handle's launches with HIP events recorded on the
 * handle's stream (enable resets the counters).  For each kernel class:
 * launches, summed device time (ms), and the summed algorithmic flops and
 * bytes of those launches (the minimal work of the operation, counted from
 * the shapes, not the executed instruction count). */
enum {
  CTD_K_CUBIC_G = 0,   /* cubic Gram g_e of a fresh factor (3D, MFMA,
                          split-K partials)                               */
  CTD_K_CUBIC_GRED,    /* split-K reduction of g, S = w g_e g_f          */
  CTD_K_CUBIC_H,       /* cubic evaluation h_d at the Gauss points (MFMA)*/
  CTD_K_RHS,           /* right-hand side assembly + nonlinear projection */
  CTD_K_SOLVE,         /* banded solve (block cyclic reduction) + normalisation */
  CTD_K_SIGNATURE,     /* Grams of a fresh factor, Gauss-point values     */
  CTD_K_GEMV,          /* (no launches: the 2D M_xy product runs inside
                          the RHS launch, booked under CTD_K_RHS)         */
  CTD_K_MXY,           /* M_xy build (2D, once per step)                  */
  CTD_K_ENERGY,        /* separated energy                                */
  CTD_K_QUAD,          /* Gauss-point tables of u^k (once per step)       */
  CTD_K_OTHER,         /* init/append/reset                               */
  CTD_K_FINALIZE,      /* normalisation + fixed-point test after a fast-
                          diagonalisation solve (fused into the cyclic
                          reduction kernel otherwise)                     */
  CTD_K_FULL_SOLVE,    /* full CFE step of actd: dense products in the
                          eigenbases (FP64 MFMA)                          */
  CTD_K_SKIPPED,       /* launches of a sweep enqueued ahead of the host's
                          decision, after which the mode had ended: they
                          returned at once (any class; timed when the
                          class of the launch is selected)                */
  CTD_K_COUNT
};
int ctd_profile_enable(ctd_solver* s, int32_t on);
/* As ctd_profile_enable, timing only the classes whose bit (1u << class) is
 * set in mask (each bracketed launch adds two event records to the stream;
 * timing one class keeps the others' launch cadence). */
int ctd_profile_select(ctd_solver* s, uint32_t mask);
int ctd_profile_read(ctd_solver* s, int32_t kernel, int64_t* launches,
                     double* ms, double* flops, double* bytes);

/* Nonlinear load of the directional system for direction d (the M_xy u_y
 * term of eq. KxQx and its 3D analogue), on the handle's current u^k:
 *   out[i] = int N~_i(x_d) prod_{e != d} u_e(x_e) L w(u^k) dOmega,
 * evaluated by the same kernels as ctd_step (2D: M_xy product; 3D: separated
 * cubic contraction plus the linear part through M X^k).  u: dim host
 * pointers, u[e] of nodes[e] values for e != d (u[d] ignored); out: host,
 * nodes[d] values.  Uses the handle's step scratch; call between steps. */
int ctd_nonlinear_load(ctd_solver* s, int32_t d, const double* const* u,
                       double* out);

/* Tuning table of the 3D cubic contraction (process-wide, thread-safe).
 * An entry gives the split counts for one (precision, nb, nq): precision
 * CTD_PREC_MIXED or CTD_PREC_FP64 (the kernels differ), nb = ceil(M_k / 16)
 * mode tiles, nq = Gauss points of the instance's smallest axis.
 * nsplit_g: Gauss-point splits of the g contraction (workgroups = tile
 * triples x nsplit_g); nsplit_h: tile-triple splits of the h contraction.
 * Handles use an entry from their next step on (ctd_nonlinear_load: from its
 * next call); without one they use the built-in heuristic.  The split counts
 * change the summation order, so results are reproducible for a fixed table.
 * Values are clamped to what the handle allocated.  Set replaces an entry of
 * the same key; returns CTD_EINVAL for non-positive counts or an unknown
 * precision.  The table is measured offline (paper_2410_15519_amd/tune.py)
 * and loaded by the binding. */
int ctd_tuning_set_prec(int32_t precision, int32_t nb, int32_t nq, int32_t nsplit_g,
                        int32_t nsplit_h);
/* The entry of the mixed-precision path (ctd_tuning_set_prec with
 * CTD_PREC_MIXED). */
int ctd_tuning_set(int32_t nb, int32_t nq, int32_t nsplit_g, int32_t nsplit_h);
/* Removes every entry. */
int ctd_tuning_clear(void);
/* The split counts a handle uses for its current M_k (3D; 0 otherwise). */
int ctd_tuning_current(ctd_solver* s, int32_t* nsplit_g, int32_t* nsplit_h);

/* Elements left out by the reduced domain (Sec. 3.3, eq. MxyRD) of the 2D
 * M_xy the next step uses (built from u^k at ctd_init and at the end of each
 * step); 0 with rd_tol = 0 or in 3D.  Waits for the handle's stream. */
int ctd_reduced_domain_excluded(ctd_solver* s, int64_t* count);

#ifdef __cplusplus
}
#endif
#endif /* CTD_H */
