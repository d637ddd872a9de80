/*
 * fem_heat.h -- C ABI of the MI355X (gfx950) assembly-free transient heat solver.
 *
 * The method is that of Loeb & Earls, arXiv:1905.07622: every implicit
 * theta-scheme time step solves
 *     [M + theta*dt*K] U^n = [M - (1-theta)*dt*K] U^{n-1} + dt*F      (Sec. 3.1)
 * with Jacobi-preconditioned conjugate gradient (Algorithm 1, Sec. 3.3).
 * M and K are never assembled: they are applied element by element on a
 * fixed grid of 8-node trilinear hexahedra with per-element heat capacity
 * rho*C_e and conductivity k_e, and the assembly operator is evaluated as a
 * node-centred gather -- each output degree of freedom sums the
 * contributions of the elements around it (the DbD reading of eq. EbEvsDbD
 * and eq. DbD, Sec. 3.2 and 4.2.2).  Every step of that path runs in HIP
 * kernels on the GPU; the host only enqueues work and reads small flags.
 *
 * Conventions shared by every entry point
 *  - Grid: nx*ny*nz elements of size hx*hy*hz, origin 0.  Nodes are numbered
 *    i = ix + (nx+1)*(iy + (ny+1)*iz) (x fastest, as the paper's fixed grid,
 *    Sec. 4.1); N = (nx+1)(ny+1)(nz+1).  Elements e = ex + nx*(ey + ny*ez);
 *    E = nx*ny*nz.  Node arrays have length N, element arrays length E, dense,
 *    in that order.  The library's internal layout never leaks out.
 *  - Faces: 0:-x 1:+x 2:-y 3:+y 4:-z 5:+z.  Bit f of a face mask selects face f.
 *  - Memory: array arguments are HOST pointers unless the handle was created
 *    with FEM_DEVICE_PTRS, in which case they are device pointers on the
 *    handle's device (e.g. torch tensors); the byte layout is the same.
 *    The caller owns every array; create/run copy what they need before
 *    returning, and run writes outputs before returning.  A handle owns its
 *    device memory until fem_heat_destroy.
 *  - Errors: every call returns FEM_OK (0) or a negative FEM_E* code and never
 *    throws across the ABI.  fem_last_error() gives a message for the last
 *    failing call on a handle.
 *  - Threads: a handle belongs to one thread at a time.
 */
#ifndef FEM_HEAT_H
#define FEM_HEAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define FEM_OK 0
#define FEM_EINVAL (-1)      /* invalid argument (nothing was changed)            */
#define FEM_ENOMEM (-2)      /* device or host allocation failed                  */
#define FEM_ENOCONV (-3)     /* some step reached max_iter; outputs still written  */
#define FEM_EBREAKDOWN (-4)  /* CG breakdown (d^T A d <= 0 or non-finite scalar)   */
#define FEM_EDEVICE (-5)     /* a HIP runtime call failed                          */
#define FEM_EBUSY (-6)       /* resource temporarily unavailable                   */
#define FEM_ECANCELED (-7)   /* request cancelled                                  */

/* ---- options ------------------------------------------------------------ */
#define FEM_FP64 0           /* FP64 operator, vectors, dots and scalars           */
#define FEM_FP32_FP64DOT 1   /* FP32 operator and vectors inside FP64 refinement   */

#define FEM_GUESS_EXTRAP 0   /* x0 = 2 T^{n-1} - T^{n-2} (u0_update, App. A.2)     */
#define FEM_GUESS_PREV 1     /* x0 = T^{n-1}                                       */

#define FEM_STOP_RHS 0       /* continue while r^T P^-1 r > rtol^2 b^T P^-1 b      */
#define FEM_STOP_INITIAL 1   /* continue while r^T P^-1 r > rtol^2 r0^T P^-1 r0    */

#define FEM_ELEM_HEX8 0         /* one 8-node trilinear hexahedron per box of the grid */
#define FEM_ELEM_TET6 1         /* the paper's element (Sec. 4.1): every box split into six linear
                                   tetrahedra 0, e_i, e_i + e_j, 7 (one per order of the axes; the
                                   split around the box's 0-7 diagonal, conforming between boxes).
                                   Cubic boxes only (hx = hy = hz).  Face loads come from the
                                   faces' triangles, sensors are linear in their tetrahedron.
                                   Not with FEM_OP_ELEMENTWISE / FEM_OP_ROWWAVE or the Chebyshev
                                   preconditioner (FEM_EINVAL) */

#define FEM_PRECOND_JACOBI 0    /* P = diag(A) (Sec. 3.3)                            */
#define FEM_PRECOND_CHEBYSHEV 1 /* M^-1 = q(D^-1 A) D^-1, D = diag(A), with 1 - lambda q(lambda) the
                                   Chebyshev polynomial of degree m = cheb_degree on
                                   [hi/cheb_ratio, hi], scaled to 1 at 0; hi bounds the spectrum of
                                   D^-1 A for every coefficient field (27/8 for cubic elements).
                                   Applied matrix-free as m steps of the Chebyshev iteration from 0
                                   (m - 1 gathers per application).  Not in the paper, whose GPU
                                   method uses Jacobi only.  The stop rule's norm (P^-1 above) is
                                   M^-1.  FP64 two-kernel form only (FEM_EINVAL with the mixed form
                                   or FEM_ONE_REDUCTION) */

#define FEM_DEVICE_PTRS 0x1u /* array arguments are device pointers               */
#define FEM_TIMING 0x2u      /* time iteration kernels with HIP events (every 64th iteration and every
                                8th residual replacement launched, counted across solves, so the
                                events barely perturb the run) */
#define FEM_ONE_REDUCTION 0x4u /* FP64 PCG in one kernel and one reduction per iteration: the direction
                                  kernel also completes the previous update (r -= alpha q, x += alpha d)
                                  and sums d^T q, q^T P^-1 r, q^T P^-1 q and r^T P^-1 r; alpha and the stop
                                  test are Algorithm 1's, beta uses r'^T P^-1 r' = delta - 2 alpha
                                  q^T P^-1 r + alpha^2 q^T P^-1 q (restarted from the summed delta every
                                  iteration), so the iterates agree with Algorithm 1 to rounding.  One
                                  extra direction kernel per solve.  With FEM_FP32_FP64DOT the FP32
                                  inner solves take this form (sums and scalars in FP64) */

#define FEM_ONE_KERNEL 0x8u /* fem_heat_run: each iteration of Algorithm 1 in one kernel instead of two
                               (direction gather, then the x/r update): the gather's blocks publish
                               d^T q, meet at a grid-wide barrier, and each updates r (and x in FP32)
                               at its own nodes from values it kept on chip.  Used when the gather's
                               blocks all fit the device at once (else two kernels).  The barrier
                               needs all of them resident: work that other streams or processes run
                               on the device at the same time can hold CUs, and then its bounded wait
                               runs out and the run fails with FEM_EDEVICE.  Results agree with the
                               two-kernel form to rounding (the r^T P^-1 r partials are summed per
                               gather block).  Batches and servers always use two kernels, so a
                               simulation's results do not depend on its co-runners */

/* Operators for fem_heat_apply */
#define FEM_OP_A 0           /* y = (M + theta*dt*K) x                              */
#define FEM_OP_L 1           /* y = (M - (1-theta)*dt*K) x                          */
#define FEM_OP_JACOBI 2      /* y = P^-1 x, P = diag(M + theta*dt*K); 0 on Dirichlet */
#define FEM_OP_LOAD 3        /* y = F (boundary load vector); x is ignored          */
#define FEM_OP_FP32 0x100    /* OR-ed in: use the FP32 operator (x rounded to FP32) */
#define FEM_OP_ELEMENTWISE 0x200 /* OR-ed in (FEM_OP_A or FEM_OP_L, FP64 only): apply element by element in
                                    two passes instead of the node-centred gather, after the structure of
                                    the paper's coalesced element-by-element method (Section 4.3, third
                                    implementation): each wavefront integrates a row of elements from the
                                    four node rows along its x-edges and sums neighbouring contributions,
                                    a second pass adds the up to four partial sums per node.  Kept for
                                    comparison; the first use allocates 4 N doubles of partial sums, held
                                    by the handle until fem_heat_destroy */
#define FEM_OP_ROWWAVE 0x400 /* OR-ed in (FEM_OP_A or FEM_OP_L, FP64 only): node-centred apply with one
                                wavefront per node row and no block barrier (x-neighbours through lane
                                shuffles, y- and z-neighbours from nine coalesced row loads), instead of
                                the LDS-tiled z-marching gather.  Kept for comparison */

typedef struct fem_heat fem_heat;

/* Grid: elements per axis and element size per axis (all > 0). */
typedef struct {
  int32_t nx, ny, nz;
  double hx, hy, hz;
} fem_grid;

/* Boundary conditions.  Flux faces carry k dT/dn = q (inward heat flux,
 * Sec. 3.1); Dirichlet faces hold T = value (not in the paper, which uses
 * flux conditions only: imposed by keeping those nodes fixed in every vector,
 * equivalent to symmetric elimination).  A face may not be in both masks.
 * Where two Dirichlet faces meet, the lower-numbered face sets the value.
 * Faces in neither mask are insulated.  The load of step m (1-based global
 * step index) is dt * s_m * F with s_m = flux_schedule[m-1] for
 * 1 <= m <= n_schedule, 0 beyond it, and s_m = 1 for every m when
 * flux_schedule is NULL.  The schedule is copied at create. */
typedef struct {
  uint32_t dirichlet_mask;
  double dirichlet_value[6];
  uint32_t flux_mask;
  double flux[6];
  const double *flux_schedule;  /* host pointer always */
  int32_t n_schedule;
} fem_bc;

/* Device memory of a handle (or of a server's simulations) through the
 * caller's allocator.  alloc returns 0 and sets *ptr to `bytes` of device
 * memory on the handle's device, usable by work enqueued on `stream` after
 * the call (stream-ordered); release hands back a block once the work
 * enqueued on `stream` before the call is done with it.  The library calls
 * them from the thread that uses the handle (a server: from its worker
 * threads, one stream per thread), never concurrently for one stream.  With
 * no allocator, handles use hipMalloc / hipFree; a server uses its own
 * stream-ordered memory pool, so retiring a simulation never synchronises
 * the device. */
typedef struct {
  void *ctx;
  int (*alloc)(void *ctx, void **ptr, size_t bytes, void *stream);
  void (*release)(void *ctx, void *ptr, void *stream);
} fem_allocator;

typedef struct {
  int32_t precision;      /* FEM_FP64 | FEM_FP32_FP64DOT                          */
  int32_t max_iter;       /* i_max of Algorithm 1 (per step; inner per sweep in mixed form); default 10000 */
  int32_t replace_every;  /* residual replacement r = b - A x when i % replace_every == 0 (Algorithm 1 uses 50); 0 = never */
  int32_t guess;          /* FEM_GUESS_*                                           */
  int32_t stop_rule;      /* FEM_STOP_*                                            */
  int32_t max_refine;     /* mixed form: max FP64 refinement sweeps per step (default 4) */
  double inner_rtol;      /* mixed form: floor of the inner FP32 PCG relative tolerance (default 1e-5);
                             each sweep targets half the residual reduction the FP64 stop rule still needs */
  uint32_t flags;         /* FEM_DEVICE_PTRS | FEM_TIMING                          */
  void *hip_stream;       /* hipStream_t to run on; NULL = the library's own stream */
  int32_t device;         /* HIP device ordinal                                    */
  int32_t tile_x, tile_y, tile_z; /* gather tile overrides; 0 = automatic.  tile_x*tile_y <= 512
                             for a handle's own runs (blocks of up to 512 threads), <= 256 for
                             batch members and served simulations, and the (tile_x+2)*(tile_y+2)
                             plane tile must fit two staging slots per thread: FEM_EINVAL
                             otherwise                                                        */
  const fem_allocator *allocator; /* device memory (NULL: see fem_allocator); must outlive
                             every handle and server created with these options          */
  int32_t precond;        /* FEM_PRECOND_* (default Jacobi)                                  */
  int32_t cheb_degree;    /* Chebyshev: 2 .. 8 (default 3)                                   */
  double cheb_ratio;      /* Chebyshev: hi / lo of the interval, > 1 (default 30)            */
  int32_t element;        /* FEM_ELEM_* (default FEM_ELEM_HEX8)                              */
  const char *tune_cache; /* path of the autotuner's tile cache (JSON), or NULL.  When set and no
                             tile override is given, a handle takes the gather tile recorded
                             there for its node grid, precision, element class and launch kind
                             (alone or batch member) on this GPU architecture and HIP runtime;
                             fem_heat_tune records into it (see fem_heat_tune on results). */
  int32_t batch_groups;   /* fem_heat_run_batch: run the simulations as this many batches at once,
                             dealt round-robin, each on its own stream and host thread, so that one
                             batch's last iterations (its slowest members) overlap the others'
                             work; results do not change.  0 = automatic (one batch per 16
                             simulations and per 2^21 nodes in all, at most 3, at least 1);
                             with a caller's stream the batches start after its earlier work.
                             Handles and servers ignore it (server lanes already overlap) */
} fem_opts;

/* Outputs of a run (inputs marked "in").  Every pointer may be NULL.
 * Arrays follow the handle's memory kind (FEM_DEVICE_PTRS). */
typedef struct {
  double *T_final;           /* N: field after the last step                          */
  double *T_saved;           /* (nsteps/save_every)*N: field after every save_every-th step */
  int32_t save_every;        /* in                                                    */
  const double *sensor_xyz;  /* in: 3*S point coordinates                             */
  int32_t n_sensors;         /* in: S                                                 */
  double *traces;            /* nsteps*S, row-major [step][sensor]: field at the points,
                                trilinear in the containing element (lowest-index element on shared faces) */
  int32_t *iters;            /* nsteps: PCG iterations per step (inner FP32 iterations in the mixed form) */
  double *relres;            /* nsteps: final sqrt(r^T P^-1 r / b^T P^-1 b)           */
  int32_t *refine_sweeps;    /* nsteps: FP64 refinement sweeps (mixed form)           */
  int32_t first_step;        /* in: global index of the step preceding this run's first step
                                (0 for a fresh run; the flux schedule is indexed from it) */
  int64_t total_iters;       /* out: sum of iters                                     */
  double device_ms;          /* out: device time of the run's stepping (HIP events)   */
} fem_out;

/* Kernel timing (filled when the handle has FEM_TIMING): launches timed and
 * their summed durations, per kernel kind. */
typedef struct {
  int64_t gather_launches;   /* search-direction + operator-apply kernel (q = A d, d^T q,
                                and the previous iteration's x += alpha d)                  */
  double gather_ms;
  int64_t update_launches;   /* r -= alpha q + preconditioned residual norm kernel        */
  double update_ms;
  int64_t replace_launches;  /* residual-replacement gather kernel                        */
  double replace_ms;
  int32_t grid_blocks;       /* blocks of the gather launch                                */
  int32_t tile_x, tile_y, tile_z;
  int64_t apply_calls;       /* fem_heat_apply calls on a handle created with FEM_TIMING,  */
  double apply_ms;           /* and the device time of their operator kernels (HIP events;
                                the copies of x and y are outside)                          */
  int64_t one_kernel_launches; /* of the sampled direction kernels above, those that also did the
                                x/r update (FEM_ONE_KERNEL) */
} fem_stats;

/* Create a solver for one grid, coefficient field and set of boundary
 * conditions (Sec. 3.2: the element data are prepared once, only the
 * coefficients change between solves).  Validates (FEM_EINVAL): nx,ny,nz >= 1,
 * fewer than 2^29 nodes, h* > 0 and finite, k_e >= 0 and finite, rho*c_e > 0 and finite, masks in 6
 * bits and disjoint, finite boundary values.  Copies k_e, rho*c_e and the
 * schedule to the device, builds the load vector F.  opts may be
 * NULL (defaults).  On success *out owns the device state. */
int fem_heat_create(const fem_grid *grid, const double *k_e, const double *rhoc_e,
                    const fem_bc *bc, const fem_opts *opts, fem_heat **out);

/* Run nsteps theta-scheme steps from T0 (N values; Dirichlet nodes are
 * overwritten by their boundary value).  T_prev (N values or NULL = T0) is
 * the field one step before T0; it feeds the extrapolated initial guess, so
 * a run split into two calls with T_prev = the field before T0 matches the
 * uninterrupted run.  Per step: b = L T^{n-1} + dt*s_n*F, x0 by the guess
 * rule, Algorithm 1 with the Jacobi preconditioner, stop rule, residual
 * replacement and max_iter from the options.  Validates dt > 0,
 * theta in [0,1], rtol > 0, nsteps >= 0 (FEM_EINVAL).  Returns FEM_OK,
 * FEM_ENOCONV (some step hit max_iter: all outputs written, iters = max_iter
 * marks the step) or FEM_EBREAKDOWN (outputs up to the last good step). */
int fem_heat_run(fem_heat *h, const double *T0, const double *T_prev, double dt, double theta,
                 int32_t nsteps, double rtol, fem_out *out);

/* Apply one operator of the method (test hook; see FEM_OP_*) with the given
 * dt and theta: y = op(x).  x and y are N-vectors. */
int fem_heat_apply(fem_heat *h, int32_t which, double dt, double theta, const double *x, double *y);

/* fem_heat_apply for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * which is FEM_OP_A or FEM_OP_L, optionally OR-ed with FEM_OP_ELEMENTWISE
 * (hexahedra only), in FP64.  x and y are DEVICE pointers to N doubles on
 * the handle's device whatever the handle's flags (y must not overlap x).
 * The call only enqueues kernels on the handle's stream and returns: no
 * allocation, copy, event or synchronisation; the caller synchronises the
 * stream before reading y.  The kernels' scratch (the element-by-element
 * form's 4 N partial sums and the gather's sink for lanes without a node) is
 * a static array of the library, one per GPU (32 MiB + 4 KiB, held until the
 * process ends): the element-by-element form takes at most 2^20 nodes
 * (FEM_EINVAL beyond).  Every call on one GPU shares that array, so calls
 * that overlap on one GPU (two streams, two threads) race; calls in one
 * stream's order do not.  Results are bit-identical to fem_heat_apply with
 * the same operator and form.  Returns FEM_EINVAL for other operators, FP32
 * or row-wavefront forms, missing pointers or bad dt/theta. */
int fem_heat_apply_noalloc(fem_heat *h, int32_t which, double dt, double theta, const double *x, double *y);

/* One simulation of a batch: a problem as for fem_heat_create and a run as
 * for fem_heat_run (same meanings, validation and outputs). */
typedef struct {
  fem_grid grid;
  const double *k_e;
  const double *rhoc_e;
  fem_bc bc;
  const double *T0;
  const double *T_prev;      /* NULL = T0 */
  double dt, theta, rtol;
  int32_t nsteps;
  fem_out *out;              /* may be NULL */
} fem_request;

/* Run n independent simulations together on one GPU: the repeated forward
 * solves of a coefficient study (Sec. 5.4), each with its own grid,
 * coefficients, boundary conditions, dt, theta, rtol and step count.  Every
 * kernel launch serves all of them (a simulation's blocks work only on its
 * own data, with its own reductions), they advance one time step per epoch
 * in lockstep, and each leaves the batch after its last step.  A
 * simulation's results do not depend on the others in the batch: they are
 * bit-identical to those of a batch holding it alone.  Large batches run as
 * a few such batches at once (fem_opts.batch_groups).  opts (may be NULL)
 * apply to all: precision, iteration controls, flags (FEM_DEVICE_PTRS covers
 * every array of every request), stream, device and tile overrides; without
 * a tile_z override every simulation marches z-chunks of at most 32 planes.
 * Validates every request first and runs none if one is invalid
 * (FEM_EINVAL, status[i] names it).  Otherwise status[i] (n entries, may be
 * NULL) receives each simulation's outcome as fem_heat_run would return it,
 * and the call returns FEM_OK when all are FEM_OK, else the first other
 * status in request order; FEM_ENOMEM / FEM_EDEVICE abort the whole batch. */
int fem_heat_run_batch(const fem_request *reqs, int32_t n, const fem_opts *opts, int32_t *status);

/* ---- serving: continuous batching of forward simulations ------------------
 *
 * A server groups requests into size classes (the binary order of magnitude
 * of their node count); each class has a lane, a worker thread with its own
 * HIP stream, that advances every admitted simulation of the class one time
 * step per epoch with the batched launches of fem_heat_run_batch, so the
 * classes run concurrently and a small request never waits for the epochs of
 * a large one.  Submitted requests wait in one FIFO queue; at each of its
 * epoch boundaries a lane retires its finished simulations (outputs written,
 * device memory released to the server's stream-ordered pool, completion
 * stamped) and admits queued requests of its class in arrival order while
 * their device footprint fits the free part of the HBM budget and a slot is
 * free (a request that does not fit blocks every later one, so large
 * requests cannot starve).  An admitted simulation
 * keeps its whole PCG state resident until it finishes, and joins the
 * launches at the next epoch while the others continue: its results are
 * bit-identical to those of a batch holding it alone.  The use case is the
 * paper's coefficient study of thousands of forward solves (Sec. 5.4). */

#define FEM_REQ_QUEUED 0
#define FEM_REQ_RUNNING 1
#define FEM_REQ_DONE 2       /* finished: status holds the run's outcome        */
#define FEM_REQ_CANCELED 3

typedef struct fem_server fem_server;

typedef struct {
  uint64_t hbm_budget_bytes; /* device bytes admitted simulations may hold; 0 = 3/4 of free memory at create */
  int32_t max_slots;         /* simulations in flight at most; 0 = 256 */
  fem_opts opts;             /* as for fem_heat_run_batch; FEM_DEVICE_PTRS and FEM_TIMING are not accepted */
} fem_server_opts;

typedef struct {
  int32_t state;             /* FEM_REQ_*                                          */
  int32_t status;            /* DONE: FEM_OK / FEM_ENOCONV / FEM_EBREAKDOWN / FEM_ENOMEM / FEM_EDEVICE;
                                CANCELED: FEM_ECANCELED; otherwise FEM_OK          */
  int32_t steps_done;
  double t_arrive, t_admit, t_done; /* seconds on the server's monotonic clock; < 0 until reached */
  uint64_t bytes;            /* device footprint charged against the budget          */
} fem_status;

typedef struct {
  int64_t submitted, completed, canceled, failed, epochs;
  int32_t queued, running;
  uint64_t budget_bytes, bytes_in_use, peak_bytes_in_use;
  double now;                /* the server's clock                                   */
} fem_server_info;

/* Start a server on opts->opts.device (opts may be NULL: defaults). */
int fem_server_create(const fem_server_opts *opts, fem_server **out);

/* Queue a request (validated as by fem_heat_run_batch; host pointers).  All
 * inputs -- coefficients, fields, schedule, sensor points -- are copied before
 * returning; the output arrays named by req->out (may be NULL) must stay
 * valid until the request is DONE or CANCELED, and are written by then
 * (total_iters and device_ms = time from admission to completion, too).
 * FEM_ENOMEM: the request alone exceeds the budget (nothing queued). */
int fem_server_submit(fem_server *s, const fem_request *req, uint64_t *ticket);

/* Current state of a request (non-blocking).  FEM_EINVAL: unknown ticket. */
int fem_server_poll(fem_server *s, uint64_t ticket, fem_status *st);

/* Wait until the request is DONE or CANCELED or timeout_s passes (< 0: no
 * limit).  Returns its final status, or FEM_EBUSY on timeout; *st (may be
 * NULL) receives the state either way. */
int fem_server_wait(fem_server *s, uint64_t ticket, double timeout_s, fem_status *st);

/* Cancel a queued or running request (a running one leaves at the next epoch
 * boundary; its outputs are not written).  No effect once DONE. */
int fem_server_cancel(fem_server *s, uint64_t ticket);

/* Counters and memory use. */
int fem_server_info_get(fem_server *s, fem_server_info *info);

/* Cancel everything outstanding, stop the worker and release the server. */
void fem_server_destroy(fem_server *s);

/* Autotuner (the project's own; the paper tunes nothing).  Times the
 * hot gather of the PCG iteration -- search-direction update fused with the
 * operator apply q = A d and the previous iteration's x += alpha d, in the
 * handle's precision (FP32 for the mixed form) -- on this handle's grid and
 * coefficients for a set of candidate tiles (x pieces of the node row, block
 * heights, z-chunk lengths for 1 to 4 resident blocks per CU), each with
 * device events over repeated launches, and installs the fastest on the
 * handle.  With FEM_TUNE_BATCH the candidates and the timing are those of a
 * batch member: chunks of 8 to 32 planes or the node column cut into 1 to 6
 * equal chunks, each scored by its time per simulation in a launch with
 * enough copies of the simulation to fill the device plus a sixteenth of a
 * launch holding the simulation alone (a lockstep batch ends each step with
 * launches serving only its slowest members, where the tile's latency
 * counts); the tile is recorded, not installed.  When the
 * handle's options name a tune_cache, the result is recorded there under
 * the key of this grid, precision, element class and launch kind, and later
 * handles (fem_heat_create, fem_heat_run_batch, servers) with the same
 * options take it.  The operator's value at every node does not depend on
 * the tile (its sums are formed in a fixed order), but a run's dot products
 * are summed per block, so another tile changes results at rounding level;
 * the same tile repeats a run bit for bit.  The handle's vectors are overwritten:
 * tune before a run, not between the two halves of a resumed run.  out may
 * be NULL. */
#define FEM_TUNE_BATCH 0x1
typedef struct {
  int32_t tile_x, tile_y, tile_z; /* installed tile                                         */
  int32_t candidates;             /* tiles timed                                            */
  double best_us;                 /* its time per launch (with FEM_TUNE_BATCH: its score, in us) */
  double rule_us;                 /* the same for the tile the handle had before            */
  int32_t recorded;               /* 1: written to the tune_cache                           */
} fem_tune_result;
int fem_heat_tune(fem_heat *h, double dt, double theta, uint32_t flags, fem_tune_result *out);

/* Kernel timing and launch shape of the last run (FEM_TIMING). */
int fem_heat_stats(const fem_heat *h, fem_stats *out);

/* Release a handle (NULL is accepted). */
void fem_heat_destroy(fem_heat *h);

/* Fill *opts with the defaults: FP64, max_iter 10000, replace_every 50,
 * extrapolated guess, RHS stop rule, max_refine 4, inner_rtol 1e-5. */
void fem_heat_default_opts(fem_opts *opts);

const char *fem_strerror(int status);
/* Message of the last failing call on a handle; with NULL, of the last failing
 * fem_heat_create, fem_heat_run_batch or fem_server_* call on the calling thread. */
const char *fem_last_error(const fem_heat *h);

#ifdef __cplusplus
}
#endif
#endif /* FEM_HEAT_H */
