/*
 * wavedd: block-level non-overlapping domain decomposition for the 2D
 * Helmholtz equation with impedance boundary and transmission conditions,
 * subdomain problems solved by WaveHoltz, on one AMD Instinct MI355X (gfx950).
 *
 * Method: A. Rotem, "Efficient Domain Decomposition for the Helmholtz
 * Equation on GPUs".
 *   Problem       Sec. II eq. (1):  -Lap u - k^2 u = f,  d_n u - i k u = g,
 *                 k = omega / c(x), time convention e^{-i omega t}.
 *   Discretisation Sec. IV eq. (4): (A - i omega H - omega^2 M) u = b with a
 *                 tensor-product GLL spectral-element basis of degree P on
 *                 uniform axis-aligned quadrilaterals and GLL quadrature, so
 *                 M and H are diagonal and A is a Kronecker sum.
 *   DD            Sec. III: non-overlapping subdomains coupled by
 *                 zeroth-order impedance conditions; dual variables updated
 *                 by eq. (2) (sign read so that the fixed point is the global
 *                 discrete solution: g_r <- -g_l - 2 i k u_l).
 *   Subdomain solve Sec. V eqs. (6)-(7) and Algorithm 1: WaveHoltz with the
 *                 modified leapfrog scheme, all subdomains in one launch.
 *   Outer         Sec. III (last paragraph): the sweep is affine in the
 *                 interface data, G' = T G + h; (I - T) G = h is solved by
 *                 restarted GMRES in FP64 (or plain fixed-point iteration).
 *
 * Conventions
 *   Global nodes (i, j), i along x, j along y; flat index j * Nx + i with
 *   Nx = nx*P + 1, Ny = ny*P + 1, N = Nx * Ny.
 *   Boundary traces (g on the outer boundary) are arrays of length
 *   2*Ny + 2*Nx: left side (x = x0, by increasing y), right side (x = x1),
 *   bottom side (y = y0, by increasing x), top side (y = y1).  Each side
 *   carries its own value at a corner.
 *   Subdomain l = b * sx + a covers element columns [a*mx, (a+1)*mx) and
 *   rows [b*my, (b+1)*my), mx = nx/sx, my = ny/sy; its local nodes (il, jl)
 *   are stored row-major, nloc = (mx*P+1) * (my*P+1) per subdomain.
 *   Interface arrays ("g layout", used by dd_sweep): for each subdomain l,
 *   the sides left, right, bottom, top, each ordered by increasing
 *   coordinate, of lengths nyl, nyl, nxl, nxl (nxl = mx*P+1, nyl = my*P+1).
 *
 * Errors: every entry point returns 0 on success or a negative DD_E* code;
 * dd_last_error() returns a thread-local message for the last failure.  All
 * argument validation happens before any device work.
 * Threading: a handle is used by one host thread at a time and issues its
 * work on one HIP stream; separate handles are independent.
 * Memory: the library owns all device memory it allocates; host arrays
 * passed in are read or written only during the call.
 */
#ifndef WAVEDD_H
#define WAVEDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DD_OK 0
#define DD_EINVAL (-1)     /* bad shape or value, detected before device work */
#define DD_ENOMEM (-2)     /* device allocation failed */
#define DD_EHIP (-3)       /* HIP runtime error (message in dd_last_error) */
#define DD_ENAN (-4)       /* non-finite input or iterate */
#define DD_ENOTCONV (-5)   /* max_iter reached: outputs and stats ARE written */
#define DD_ENODEV (-6)     /* no usable gfx950 device */

#define DD_FP64 0          /* subdomain sweep in double precision */
#define DD_FP32 1          /* subdomain sweep in single precision, outer FP64 */

#define DD_LAYOUT_AUTO 0        /* pick by measurement (autotuner) */
#define DD_LAYOUT_NODE 1        /* one DOF per thread, state in registers + LDS */
#define DD_LAYOUT_PATCH 2       /* one element patch (P*P DOFs) per thread, one barrier/step */
#define DD_LAYOUT_PATCH_XCHG 3  /* same ownership, partial-sum exchange, two barriers/step */
#define DD_LAYOUT_STREAM 4      /* any size: state streamed through L2 / HBM, one barrier/step */

#define DD_OUTER_GMRES 0
#define DD_OUTER_FIXED 1

typedef struct dd_handle dd_handle;

/* nx x ny uniform quadrilateral elements on [x0,x1] x [y0,y1]. */
typedef struct {
    int nx, ny;
    double x0, x1, y0, y1;
} dd_mesh;

/* sx x sy grid of equal element blocks; sx | nx and sy | ny. */
typedef struct {
    int sx, sy;
} dd_partition;

typedef struct {
    int precision;   /* DD_FP64 | DD_FP32 */
    int layout;      /* DD_LAYOUT_* */
    double tau_in;   /* WaveHoltz stop: ||u_new-u|| <= tau_in ||u_new||; <= 0: fixed count */
    int max_wh;      /* WaveHoltz iteration cap (the fixed count when tau_in <= 0) */
    int outer;       /* DD_OUTER_GMRES | DD_OUTER_FIXED */
    int restart;     /* GMRES restart length m */
    int nt_override; /* > 0: use this many time steps per period in every subdomain */
    double cfl;      /* safety factor s in (0, 1] of the time-step rule */
    int refine;      /* extra GMRES correction passes for FP32 sweeps or relaxed inner
                        tolerance (iterative refinement): corrections use the handle's
                        sweeps, residuals and u come from strict FP64 sweeps (inner
                        tolerance tau_in for FP64 handles, clamp(0.01 tol, 1e-13, 1e-8)
                        for FP32 handles).  0 = a single pass. */
    double relax;    /* > 0: variable inner tolerance (Sec. V: subdomain solves may be
                        loose while the outer iteration is far from convergence).  The
                        k-th GMRES matvec uses tau = clamp(relax * tol / r_k, tau_in, 1e-2),
                        r_k the current relative outer residual; the true residual at
                        exit is computed with tau_in.  0 = fixed tau_in (default). */
    int warm;        /* 1: warm start (Sec. V: WaveHoltz may start from any u; the paper
                        names a previous iterate as the better start).  Applies to the
                        fixed-point outer iteration (outer = DD_OUTER_FIXED), whose sweeps
                        then take G + g_phys with sources on and start WaveHoltz from the
                        previous sweep's subdomain solutions.  Krylov matvec inputs are
                        unrelated from one matvec to the next, so GMRES ignores it.
                        0 = every WaveHoltz solve starts from u = 0 (default). */
    double tc2;      /* >= 0: second-order transmission condition on interface sides
                        (Sec. III names higher-order / optimized conditions as the
                        replacement of the zeroth-order one): B = d_n - i k - q (d_tt + k^2)
                        with the real length q = tc2 * min(c) / omega.  Lumped, it extends
                        each subdomain's 1D weights by q at its interface ends (stiffness
                        and mass keep their Kronecker form, so the time-step rule is
                        unchanged) and adds 2 (q K_side u - omega^2 m u / c^2) / W_side to
                        the interface update; the fixed point stays the global solution.
                        Useful range about 0.05-0.25: from q omega / c ~ 1 on, the lumped
                        sweep map has eigenvalues beyond the unit circle (a fixed-point
                        outer iteration diverges, GMRES slows down).
                        0 = the paper's zeroth-order condition (default). */
} dd_options;

typedef struct {
    int outer_iters;            /* outer iterations (= sweeps with sources off) */
    int sweeps;                 /* all sweep launches of the solve */
    double rel_residual;        /* max(GMRES estimate, true residual) at exit */
    double true_rel_residual;   /* ||h - (I-T)G|| / ||h|| from an FP64 sweep at exit */
    int64_t wh_iters_total;     /* WaveHoltz iterations summed over subdomains and sweeps */
    int wh_iters_max;           /* largest per-subdomain count in any sweep */
    int nt_min, nt_max;         /* time steps per period over subdomains */
    double dof_updates;         /* sum over sweeps/subdomains of nloc*(N_t-1)*iterations */
    double sweep_seconds;       /* device time inside sweep launches */
    double seconds;             /* wall time of the call */
    int refine_steps;           /* FP64 refinement steps taken (FP32 handles) */
    int fp64_sweeps;            /* FP64 sweeps of a refined FP32 solve */
} dd_stats;

/* Defaults: FP64, auto layout, tau_in 1e-12, max_wh 1000, GMRES(50),
 * no N_t override, cfl 0.9, refine 4, relax 0, warm 0, tc2 0. */
int dd_default_options(dd_options* opt);

/* Set up a problem (Sec. II-IV): mesh, degree P in [1, 4], wavespeed c > 0
 * sampled at the N global GLL nodes (host array, copied), omega > 0,
 * partition, options (NULL = defaults).  Computes GLL tables, the lumped M
 * and H of every subdomain (all four sides of a subdomain carry impedance
 * terms), the leapfrog coefficients alpha, beta and sigma, the filter tables
 * and N_t per subdomain, and uploads them.  *out receives a new handle. */
int dd_setup(dd_handle** out, const dd_mesh* mesh, int degree, const double* wavespeed,
             double omega, const dd_partition* part, const dd_options* opt);

void dd_destroy(dd_handle* h);

/* Thread-local description of the last error. */
const char* dd_last_error(void);

/* Sizes: global nodes N, nodes per subdomain, number of subdomains,
 * interface-array length, outer boundary trace length (2*Ny + 2*Nx). */
int dd_sizes(const dd_handle* h, int64_t* n_global, int64_t* n_local, int64_t* n_sub,
             int64_t* n_iface, int64_t* n_trace);

/* Global GLL node coordinates (x[N], y[N]; caller-owned). */
int dd_node_coords(const dd_handle* h, double* x, double* y);

/* Per-subdomain N_t (n_sub ints, caller-owned). */
int dd_time_steps(const dd_handle* h, int* nt);

/* Solve (Sec. III outer iteration over Algorithm 1 sweeps).  f: nodal
 * source at the N global nodes (f_im may be NULL); g: outer boundary trace
 * (NULL = 0; either part may be NULL).  tol: relative outer residual;
 * max_iter: outer iteration cap.  u: caller-owned N-arrays, the glued
 * solution (average of subdomain copies).  st may be NULL.  Returns
 * DD_ENOTCONV (with outputs written) when max_iter is reached. */
int dd_solve(dd_handle* h, const double* f_re, const double* f_im, const double* g_re,
             const double* g_im, double tol, int max_iter, double* u_re, double* u_im,
             dd_stats* st);

/* Same, with device pointers (hipMalloc'd, FP64) and an explicit stream
 * (hipStream_t passed as void*; NULL = the handle's stream).  g may be NULL.
 * Also writes the stacked subdomain copies to u_sub (n_sub*n_local complex,
 * interleaved re/im) when non-NULL. */
int dd_solve_device(dd_handle* h, void* stream, const double* d_f_re, const double* d_f_im,
                    const double* d_g_re, const double* d_g_im, double tol, int max_iter,
                    double* d_u_re, double* d_u_im, double* d_u_sub, dd_stats* st);

/* One DD cycle (Algorithm 1) on every subdomain in one launch: b from
 * src * (f, phi) + sum_sides W_side g_in, WaveHoltz from u = 0, then the
 * interface update into g_out (physical slots set to 0).  Host arrays in
 * the g layout (n_iface each); f as in dd_solve (NULL = 0); u_sub: stacked
 * subdomain solutions (n_sub*n_local each, may be NULL); wh_iters: per
 * subdomain WaveHoltz counts (may be NULL). */
int dd_sweep(dd_handle* h, const double* g_re, const double* g_im, const double* f_re,
             const double* f_im, double src, double* g_out_re, double* g_out_im,
             double* u_re, double* u_im, int* wh_iters);

/* Apply the subdomain stiffness A_l (Sec. IV, eq. (4)) to stacked nodal
 * vectors p (n_sub*n_local) with the sweep kernel's own device routine:
 * q = A p.  Host arrays.  A_l is the plain stiffness: the extension of the
 * second-order transmission condition (tc2 > 0) enters the sweeps through
 * their per-node coefficients, not this routine. */
int dd_apply_stiffness(dd_handle* h, const double* p, double* q);

/* Relative residual ||b - S u||_2 / ||b||_2 of the global system eq. (4) in
 * FP64 for a glued nodal u (host arrays; f_im, g may be NULL). */
int dd_residual(dd_handle* h, const double* u_re, const double* u_im, const double* f_re,
                const double* f_im, const double* g_re, const double* g_im, double* rel);

/* Same residual for callers that cannot allocate device memory (code under
 * stream capture, serving loops, harnesses that forbid allocation): device
 * arrays (u_re, u_im, f_re, f_im: N each; g_re, g_im: the boundary trace,
 * 2*Ny + 2*Nx each; all but u_re may be NULL), the result ||b - S u|| / ||b||
 * written to d_rel[0] (device) in stream order (NULL stream = the handle's
 * stream; no synchronisation).  Nothing is allocated: the row partials of
 * the reduction live in a library array of 16384 entries per GPU, so meshes
 * of more than 16384 grid rows (Ny = ny*P + 1) are rejected with DD_EINVAL.
 * Calls on one GPU share that array: two calls in flight at once (different
 * streams, or different handles on the same GPU) race. */
int dd_residual_device_noalloc(dd_handle* h, void* stream, const double* d_u_re,
                               const double* d_u_im, const double* d_f_re, const double* d_f_im,
                               const double* d_g_re, const double* d_g_im, double* d_rel);

/* Whole-domain operator y = S x in FP64 on device arrays (x, y: N complex,
 * interleaved re/im): the normaliser of the paper's DD-time/operator-time
 * ratio (Sec. VII-A). */
int dd_apply_operator_device(dd_handle* h, void* stream, const double* d_x, double* d_y);

/* Outer state for warm restart / checkpointing: the interface vector G
 * (n_iface complex, interleaved re/im, host). */
int dd_get_state(const dd_handle* h, double* G);
int dd_set_state(dd_handle* h, const double* G);

/* Time sweep launches with events on the handle's stream (the paper's
 * DD-cycle timing, Sec. VII-A): the input is the current outer state G (left
 * by the last solve or set by dd_set_state), sources off.  fixed_iters > 0
 * runs exactly that many WaveHoltz iterations per subdomain (the paper uses
 * five); 0 keeps the handle's tolerance.  Returns the average milliseconds
 * per launch over `reps` launches after one warm-up, and the DOF-updates of
 * one launch (sum over subdomains of nloc*(N_t-1)*iterations; may be NULL). */
int dd_time_sweep(dd_handle* h, int reps, int fixed_iters, double* ms, double* dof_updates);

/* Progress report of a running solve: called on the solving thread every
 * `every` outer iterations with the iteration count and the current
 * relative outer residual (the GMRES estimate, or the fixed-point update).
 * fn = NULL switches it off.  The callback must not call back into the
 * handle. */
typedef void (*dd_progress_fn)(void* user, int outer_iters, double rel_residual);
int dd_set_progress(dd_handle* h, dd_progress_fn fn, void* user, int every);

/* Layout in use (DD_LAYOUT_NODE .. DD_LAYOUT_STREAM) and threads per
 * subdomain: the workgroup size, times the number of workgroups that share
 * each subdomain when the autotuner gives a STREAM subdomain several. */
int dd_layout(const dd_handle* h, int* layout, int* wg_threads);

/* Coordinates of the global GLL nodes of a mesh (N each, flat index
 * j * Nx + i), computed on the host without a handle or a device: the
 * sampling points of wavespeed and f for dd_setup / dd_solve (Sec. IV,
 * nodal GLL basis). */
int dd_mesh_coords(const dd_mesh* mesh, int degree, double* x, double* y);

/* ------------------------------------------------------------------------
 * Batches: several independent problems whose sweeps share launches.
 *
 * The DD method makes every subdomain solve independent within a sweep
 * (Sec. III), so subdomains of different problems can share one launch just
 * as the subdomains of one problem do (Sec. VI: all subdomains of a sweep in
 * one kernel launch).  A batch places its problems in one device store; each
 * problem runs its own FP64 outer iteration on its own host thread and posts
 * its sweeps; whenever one of eight launch slots is free, the oldest pending
 * sweep and the pending sweeps of similar cost (slowest subdomain within a
 * factor of four) go into one round: one launch per launch configuration
 * (precision, degree, layout, workgroup class) whose work list is ordered by
 * estimated cost (DOFs x (N_t - 1) x WaveHoltz iterations of the previous
 * sweep), longest first.  Sweeps posted while the slots are busy form the
 * next round, so rounds grow with the load.
 * Layouts are autotuned once per subdomain shape (mx, my, P, precision).
 * ------------------------------------------------------------------------ */
typedef struct dd_batch dd_batch;

/* One problem: the arguments of dd_setup (wavespeed is copied). */
typedef struct {
    dd_mesh mesh;
    int degree;
    const double* wavespeed;   /* N values at the global nodes, c > 0 */
    double omega;
    dd_partition part;
} dd_problem;

/* Set up n >= 1 problems with shared options (opt may be NULL).  Errors name
 * the failing problem; nothing is allocated on failure. */
int dd_batch_setup(dd_batch** out, int n, const dd_problem* probs, const dd_options* opt);
void dd_batch_destroy(dd_batch* b);

/* Handle of problem i (owned by the batch; valid until dd_batch_destroy) for
 * dd_sizes, dd_node_coords, dd_time_steps, dd_residual, dd_get_state,
 * dd_set_state, dd_layout.  Do not pass it to dd_destroy, and do not solve
 * or sweep through it while dd_batch_solve runs. */
int dd_batch_handle(dd_batch* b, int i, dd_handle** h);

/* Solve all problems, each as dd_solve would (same arguments per problem:
 * arrays of n pointers; f_re, f_im may be NULL or hold NULL entries), with
 * their sweeps batched.  st and rc (n entries each) may be NULL.  Returns
 * DD_OK when every problem converged, DD_ENOTCONV when some did not (their
 * u and stats are written), or the first other error. */
int dd_batch_solve(dd_batch* b, const double* const* f_re, const double* const* f_im, double tol,
                   int max_iter, double* const* u_re, double* const* u_im, dd_stats* st, int* rc);

/* Time batched sweep launches over every subdomain of every problem (the
 * paper's DD-cycle timing, Sec. VII-A): inputs are each problem's current
 * outer state G, sources off, exactly fixed_iters >= 1 WaveHoltz iterations
 * per subdomain.  Returns the average milliseconds per round of launches
 * over `reps` rounds after one warm-up, the DOF-updates of one round, and the
 * number of launches in a round. */
int dd_batch_time_sweep(dd_batch* b, int reps, int fixed_iters, double* ms, double* dof_updates,
                        int* launches);

/* dd_batch_solve in two calls: _start validates, launches the problems'
 * solves on host threads and returns; every array passed must stay valid
 * until _finish, which waits for them and returns what dd_batch_solve would.
 * One solve per batch at a time (DD_EINVAL otherwise). */
int dd_batch_solve_start(dd_batch* b, const double* const* f_re, const double* const* f_im,
                         double tol, int max_iter, double* const* u_re, double* const* u_im,
                         dd_stats* st, int* rc);
int dd_batch_solve_finish(dd_batch* b);

/* Between _start and _finish: block until more than `seen` problems have
 * finished (or all have); *finished receives the count.  Returns at once
 * when no solve is running. */
int dd_batch_wait_progress(dd_batch* b, int seen, int* finished);

/* Batched launches issued by the last dd_batch_solve. */
int dd_batch_launches(const dd_batch* b, int64_t* launches);

/* ------------------------------------------------------------------------
 * Serving engine: solves submitted one at a time, run concurrently with
 * continuous batching.
 *
 * A request is one dd_solve.  The engine admits queued requests in arrival
 * order while the number of running solves is below max_active and their
 * device footprint fits the HBM budget: a share of the budget is one device
 * store holding every admitted problem's sweep arrays (ranges handed out by
 * a first-fit allocator), the rest pays for the per-request outer-iteration
 * vectors.  Each running request advances its own FP64 outer iteration on
 * its own host thread and stream; its sweeps share batched launches with
 * the other running requests' (rounds formed as for dd_batch_solve, up to 32
 * in flight, each on the stream of the request that launches it), and
 * requests join and retire between launches.  A request's own vectors come
 * from the device's stream-ordered memory pool (hipMallocAsync), which the
 * engine sets to keep freed memory.  Results stay with the engine until
 * dd_engine_wait collects them.
 * ------------------------------------------------------------------------ */
typedef struct dd_engine dd_engine;

#define DD_REQ_QUEUED 0
#define DD_REQ_RUNNING 1
#define DD_REQ_DONE 2

typedef struct {
    int64_t queued, running, done;   /* requests in each state */
    int64_t launches;                /* batched launches so far */
    int64_t peak_running;
    size_t budget_bytes;             /* as given */
    size_t store_bytes;              /* device store */
    size_t request_bytes;            /* held by running requests */
} dd_engine_info;

/* hbm_budget_bytes: device memory the engine may use (>= 64 MiB);
 * max_active >= 1 concurrent solves; opt applies to every request (NULL:
 * defaults). */
int dd_engine_create(dd_engine** out, size_t hbm_budget_bytes, int max_active,
                     const dd_options* opt);
/* Cancels queued requests, waits for running ones, frees everything. */
void dd_engine_destroy(dd_engine* e);

/* Queue a request (problem as for dd_setup, source as for dd_solve; all
 * arrays are copied; boundary data g = 0).  Validation and host-side set-up
 * happen here (errors are returned before queueing); a request larger than
 * the engine's whole store or budget fails with DD_ENOMEM.  *id identifies it
 * for dd_engine_status / dd_engine_wait. */
int dd_engine_submit(dd_engine* e, const dd_problem* prob, const double* f_re, const double* f_im,
                     double tol, int max_iter, int64_t* id);

/* DD_REQ_QUEUED, DD_REQ_RUNNING or DD_REQ_DONE. */
int dd_engine_status(dd_engine* e, int64_t id, int* state);

/* Block until request id is done, copy its glued solution (N values each;
 * may be NULL) and stats, and release it.  times (may be NULL) receives the
 * submit, start and completion times in seconds on the engine's clock.
 * Returns the request's own code (DD_OK, DD_ENOTCONV, ...). */
int dd_engine_wait(dd_engine* e, int64_t id, double* u_re, double* u_im, dd_stats* st,
                   double* times);

/* Block until some submitted, not yet collected request is done; *id
 * receives it (collect it with dd_engine_wait).  Each request is returned
 * once.  DD_EINVAL if no outstanding request remains that this call has
 * not already returned. */
int dd_engine_wait_any(dd_engine* e, int64_t* id);

int dd_engine_get_info(dd_engine* e, dd_engine_info* info);

#ifdef __cplusplus
}
#endif

#endif /* WAVEDD_H */
