/*
 * wavedd3: the box (hexahedral) form of the wavedd domain-decomposition
 * sweep, the paper's second workload (Sec. VII-B: constant wavespeed on a
 * cube, DD cycle of a few WaveHoltz iterations timed against one operator
 * evaluation).  Same method as wavedd.h with a third Kronecker factor:
 *   Discretisation Sec. IV eq. (4) on hexahedra: A = Kx (x) Wy (x) Wz +
 *                 Wx (x) Ky (x) Wz + Wx (x) Wy (x) Kz (GLL degree P, lumped M
 *                 and H; H sums W_face / c over the faces through a node).
 *   DD            Sec. III: box subdomains, zeroth-order impedance
 *                 transmission on all six faces, eq. (2) read as
 *                 g_r <- -g_l - 2 i (omega/c) u_l.
 *   Subdomain solve Sec. V eqs. (6)-(7), Algorithm 1: WaveHoltz with the
 *                 modified leapfrog scheme, one workgroup per subdomain, one
 *                 thread per node (subdomains of at most 1024 nodes), all
 *                 subdomains in one launch.  The step count per period adds
 *                 the z term to the spectral bound of Sec. V:
 *                 lambda_max <= cmax^2 mu ((2/hx)^2 + (2/hy)^2 + (2/hz)^2).
 *
 * Conventions
 *   Global nodes (i, j, k): flat index (k * Ny + j) * Nx + i, Nx = nx*P + 1,
 *   Ny = ny*P + 1, Nz = nz*P + 1.
 *   Subdomain l = (c * sy + b) * sx + a covers element blocks
 *   [a*mx, (a+1)*mx) x [b*my, (b+1)*my) x [c*mz, (c+1)*mz), mx = nx/sx etc.;
 *   its local nodes (il, jl, kl) at (kl * nyl + jl) * nxl + il,
 *   nxl = mx*P + 1, nyl = my*P + 1, nzl = mz*P + 1, nloc = nxl*nyl*nzl.
 *   Interface arrays ("g layout"): per subdomain the faces x0, x1 (nodes
 *   (kl, jl), jl fastest), y0, y1 ((kl, il), il fastest), z0, z1 ((jl, il),
 *   il fastest); n_iface = n_sub * (2 nyl nzl + 2 nxl nzl + 2 nxl nyl).
 *   Slots on the outer boundary carry physical impedance data; the sweep
 *   writes 0 there.
 *
 * Options: dd_options from wavedd.h; precision, tau_in, max_wh, cfl,
 * nt_override, restart, refine and relax are used (tau_in <= 0 runs
 * exactly max_wh WaveHoltz iterations); the outer method is always GMRES,
 * and the layout, warm-start and tc2 fields are ignored.  Errors, threading and
 * memory ownership as in wavedd.h.
 */
#ifndef WAVEDD3_H
#define WAVEDD3_H

#include <stdint.h>

#include "wavedd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dd_box {
    double x0, x1, y0, y1, z0, z1;
    int nx, ny, nz; /* elements per direction */
} dd_box;

typedef struct dd_partition3 {
    int sx, sy, sz; /* subdomain blocks per direction; must divide nx, ny, nz */
} dd_partition3;

typedef struct dd3_handle dd3_handle;

/* Build the box problem: per-node coefficients, time steps and filter
 * tables, device buffers.  wavespeed: N positive values at the global nodes
 * (host).  DD_EINVAL when a subdomain exceeds 1024 nodes, its zero-padded
 * double-buffered node grid exceeds the 160 KiB LDS, or an argument is out
 * of range; DD_ENODEV without a device. */
int dd3_setup(dd3_handle** out, const dd_box* box, int degree, const double* wavespeed,
              double omega, const dd_partition3* part, const dd_options* opt);
void dd3_destroy(dd3_handle* h);

/* Problem sizes (any output may be NULL). */
int dd3_sizes(const dd3_handle* h, int64_t* n_global, int64_t* n_local, int64_t* n_sub,
              int64_t* n_iface);

/* Leapfrog steps per period N_t of each subdomain (n_sub ints). */
int dd3_time_steps(const dd3_handle* h, int* nt);

/* GLL node coordinates of the global box grid (N each, host). */
int dd3_mesh_coords(const dd_box* box, int degree, double* x, double* y, double* z);

/* One DD cycle (Algorithm 1) on every box subdomain in one launch:
 * b = src * (f, phi) + sum_faces W_face g_in, WaveHoltz from u = 0, then the
 * interface update into g_out.  Host arrays: g in the g layout (n_iface each,
 * NULL = 0), f at the global nodes (N each; f_re NULL = no source, f_im NULL
 * = 0), u_sub: stacked subdomain solutions (n_sub*n_local each, may be
 * NULL), wh_iters: per-subdomain WaveHoltz counts (may be NULL). */
int dd3_sweep(dd3_handle* h, const double* g_re, const double* g_im, const double* f_re,
              const double* f_im, double src, double* g_out_re, double* g_out_im,
              double* u_re, double* u_im, int* wh_iters);

/* Time sweep launches with events on the handle's stream (Sec. VII-B
 * DD-cycle timing): input = the g of the last dd3_sweep (0 before any),
 * sources off; fixed_iters > 0 runs exactly that many WaveHoltz iterations
 * (the paper uses five).  Returns average milliseconds per launch over reps
 * launches after one warm-up and the DOF-updates of one launch
 * (sum of nloc*(N_t-1)*iterations; may be NULL). */
int dd3_time_sweep(dd3_handle* h, int reps, int fixed_iters, double* ms, double* dof_updates);

/* Solve the box problem (f: N values at the global nodes, f_im may be
 * NULL; no outer boundary data): restarted GMRES (dd_options.restart) in
 * FP64 on (I - T) G = h over box sweeps (Sec. III last paragraph), T the
 * sweep with sources off, h = sweep(0) with sources on, every sweep's
 * WaveHoltz solves to tau_in (cap max_wh) in the handle's precision.  FP32
 * handles with refine > 0 (Sec. VII-A: the DD as a lower-precision
 * operator) run FP64 iterative refinement: h, the residuals
 * r = h - (I - T) G and u come from FP64 sweeps (WaveHoltz tolerance
 * clamp(0.01 tol, 1e-13, 1e-8)), the corrections G += GMRES((I - T) d = r)
 * from FP32 sweeps, at most `refine` extra corrections.  relax > 0 makes
 * the GMRES matvec tolerance variable, clamp(relax tol / rel_k, tau_in,
 * 1e-2) (inexact Krylov), with FP64 refinement passes for FP64 handles too
 * (residual sweeps at tau_in).  u is the sweep of
 * the converged G, glued at the global nodes (mean of the subdomain
 * copies).  u_re, u_im: N host values.  st (may be NULL): outer
 * iterations, sweeps, refine_steps, rel_residual = max(GMRES estimate,
 * true residual), true_rel_residual = ||h - (I - T) G|| / ||h|| from the
 * final sweep, WaveHoltz totals, DOF-updates, seconds.  Returns
 * DD_ENOTCONV (outputs written) when max_iter or the corrections run out
 * first. */
int dd3_solve(dd3_handle* h, const double* f_re, const double* f_im, double tol, int max_iter,
              double* u_re, double* u_im, dd_stats* st);

/* Relative residual ||b - S u||_2 / ||b||_2 of the global box system
 * eq. (4) in FP64, b = (f, phi), for a nodal u (host arrays; f_im may be
 * NULL; f_re NULL means b = 0 and the result is ||S u||). */
int dd3_residual(dd3_handle* h, const double* u_re, const double* u_im, const double* f_re,
                 const double* f_im, double* rel);

/* Whole-box operator y = S x = (A - i omega H - omega^2 M) x in FP64 on
 * device arrays (N complex, interleaved re/im), on `stream` (hipStream_t as
 * void*, NULL = the handle's stream): the normaliser of the DD-time /
 * operator-time ratio. */
int dd3_apply_operator_device(dd3_handle* h, void* stream, const double* d_x, double* d_y);

#ifdef __cplusplus
}
#endif

#endif /* WAVEDD3_H */
