// Internal declarations shared by the host driver and the HIP kernels of
// the wavedd library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace wdd {

constexpr int kMaxP = 4;           // largest supported polynomial degree
constexpr int kMaxWG = 1024;       // largest workgroup
// Reals per node of the STREAM workspace (state triple, coefficient pair,
// side triple); the workspace then holds the interior record {1, 0, 0}
// (padded to kStreamExtra Reals).
constexpr int kStreamRecord = 8;
constexpr int kStreamExtra = 4;

// WaveHoltz stop rule of one subdomain (Sec. V: the fixed-point iteration
// runs until its update is small), given the workgroup sums
// dsum = ||u_new - u||^2 and nsum = ||u_new||^2: stop when
// dsum <= tau^2 nsum (tau <= 0: never, a fixed count).  Sweeps in FP32 also
// stop when the update has stagnated at the FP32 rounding floor, whose level
// depends on how strongly the subdomain amplifies rounding errors: when the
// update is below kWhStallRel ||u|| and did not shrink over the last
// iteration, or when it has not improved on its smallest value for
// kWhStallIters iterations in a row.  Further periods only repeat rounding
// noise; the FP64 refinement of the outer iteration supplies the accuracy.
// Either way the update must already be below kWhStallGate ||u||, so a
// subdomain that is still converging slowly is never cut short.
// State: best (smallest dsum so far, start +inf), prev (last dsum, start
// +inf), stall (iterations since best improved, start 0).  Deterministic:
// all threads hold the same sums.
constexpr double kWhStallRel = 1e-4;
constexpr double kWhStallGate = 1e-3;
constexpr int kWhStallIters = 8;
struct WhStall {
    double best = HUGE_VAL, prev = HUGE_VAL;
    int stall = 0;
};
template <typename Real>
__device__ __forceinline__ bool wh_stop(double tau, double dsum, double nsum, WhStall& s) {
    if (!(tau > 0.0)) return false;
    if (dsum <= tau * tau * nsum) return true;
    if (sizeof(Real) != 4) return false;
    const bool flat = dsum <= kWhStallRel * kWhStallRel * nsum && dsum >= s.prev;
    s.prev = dsum;
    if (dsum < s.best) {
        s.best = dsum;
        s.stall = 0;
    } else {
        s.stall += 1;
    }
    return flat || (s.stall >= kWhStallIters && dsum <= kWhStallGate * kWhStallGate * nsum);
}

// One subdomain work item of a sweep launch.  All offsets index the
// per-node arrays (node_off) or the interface arrays (if_off, nbr_off).
struct SubDesc {
    int mx, my, P;       // elements per side, degree
    int nxl, nyl;        // local node grid
    int nt;              // leapfrog steps per period
    int toff;            // offset of this subdomain's filter tables
    int max_wh;          // > 0: this item's WaveHoltz cap and tolerance (tau) override the launch's
    int64_t node_off;    // first local node in the per-node arrays
    int64_t w_off;       // first entry of its 1D weights: nxl along x, then nyl along y
    int64_t if_off;      // first slot of this subdomain's 4 sides (g layout)
    int64_t nbr_off[4];  // first slot of the neighbour side receiving each side, -1: outer
    double sigma;        // leapfrog step sigma = sin(omega dt / 2) / (omega / 2)
    double pd0c, pd0s;   // omega cos(pi/N_t), omega sin(pi/N_t): pdot^{1/2} from u
    double two_over_nt;  // 2 / N_t
    double sx_ref, sy_ref;  // 2/hx, 2/hy: reference-to-physical stiffness scales
    int64_t ws_off;      // STREAM layout: first element of its two zero-padded p grids
    double tau;          // see max_wh
    int flags;           // bit 0: warm start (first WaveHoltz iteration from the current u)
    int pad1;
    double tc_q;         // > 0: length q of the second-order transmission condition
};

// Per-node coefficient arrays of a sweep in the sweep precision `Real`.
template <typename Real>
struct NodeCoef {
    const Real* alpha;   // (M - theta H) / (M + theta H)
    const Real* betaX;   // beta * (2/hx) * Wy(jl): weight of the x-stiffness sum
    const Real* betaY;   // beta * (2/hy) * Wx(il): weight of the y-stiffness sum
    const Real* beta;    // sigma / (M + theta H)
};

template <typename Real>
struct SweepArgs {
    const SubDesc* desc;     // one per work item
    int n_items;
    NodeCoef<Real> coef;
    const Real* Fre;         // area-weighted source (f, phi) per node, or null
    const Real* Fim;
    const double* w1d;       // physical lumped 1D weights (x then y) at desc.w_off
    const double* kside;     // omega / c per interface slot
    const Real* kap;         // kappa(nu)
    const Real* kaph;        // kappa(nu + 1/2) / omega
    const Real* cs;          // cos(2 pi nu / N_t)
    const Real* sn;          // sin(2 pi nu / N_t)
    const double2* g_in;     // interface data (g layout), FP64 complex
    double2* g_out;          // updated interface data
    double src;              // multiplier of the source term
    double2* u;              // WaveHoltz iterate / result per node (FP64 complex)
    int warm;                // 1: the first WaveHoltz iteration starts from u (else from 0)
    int* wh_iters;           // per item: WaveHoltz iterations performed
    double tau;              // inner tolerance (<= 0: fixed count)
    int max_wh;              // iteration cap / fixed count
    Real* ws_p;              // STREAM layout: padded p grids (2 per subdomain, at desc.ws_off)
    Real* ws_s;              // STREAM layout: 4 Reals per node of state, then 4 of coefficients
    int64_t ws_stride;       // node capacity of ws_s
    // STREAM layout shared by several workgroups (sweep_stream_coop_kernel):
    // xb_k workgroups per item, per-item arrival counters, a launch-wide abort
    // flag and per-item stop-test partial sums (2 * xb_k doubles each); all
    // zeroed before the launch.
    int xb_k;
    int* xb_cnt;
    int* xb_abort;
    double* xb_part;
    size_t lds_bytes;        // dynamic LDS per workgroup of the launch
    int nt_max;              // largest N_t of the launch (sizes the LDS tables)
    double K1[kMaxP + 1][kMaxP + 1][kMaxP + 1];  // K1[P][a][b]: reference D^T W D
};

// Launchers (defined in the .hip kernel sources).
template <typename Real>
hipError_t launch_sweep_patch(const SweepArgs<Real>& a, int P, int wg, hipStream_t s);
template <typename Real>
hipError_t launch_sweep_patch1(const SweepArgs<Real>& a, int P, int wg, hipStream_t s);
template <typename Real>
hipError_t launch_apply_patch1(const SweepArgs<Real>& a, int P, int wg, const Real* p, Real* q,
                               hipStream_t s);
template <typename Real>
hipError_t launch_sweep_node(const SweepArgs<Real>& a, int P, int wg, hipStream_t s);
template <typename Real>
hipError_t launch_apply_patch(const SweepArgs<Real>& a, int P, int wg, const Real* p, Real* q,
                              hipStream_t s);
template <typename Real>
hipError_t launch_apply_node(const SweepArgs<Real>& a, int P, int wg, const Real* p, Real* q,
                             hipStream_t s);
template <typename Real>
hipError_t launch_sweep_stream(const SweepArgs<Real>& a, int P, int wg, hipStream_t s);
// The STREAM sweep with a.xb_k workgroups per item (a cooperative launch, so
// all workgroups are resident together); the caller checks *a.xb_abort.
template <typename Real>
hipError_t launch_sweep_stream_coop(const SweepArgs<Real>& a, int P, int wg, hipStream_t s);
template <typename Real>
hipError_t launch_apply_stream(const SweepArgs<Real>& a, int P, int wg, const Real* p, Real* q,
                               hipStream_t s);
size_t patch_lds_bytes(int mx, int my, int P, int nt_max, size_t real_size);
size_t stream_lds_bytes(int P, int nt_max, size_t real_size);
// Zero-padded p grid of a STREAM subdomain: kMaxP extra nodes on every side.
__host__ __device__ inline int64_t stream_pad_nodes(int nxl, int nyl) {
    return (int64_t)(nxl + 2 * kMaxP) * (nyl + 2 * kMaxP);
}
size_t node_lds_bytes(int nxl, int nyl, int nt_max, size_t real_size);
size_t patch1_lds_bytes(int mx, int my, int P, int wg, int nt_max, size_t real_size);

// FP64 helpers for the outer iteration (blas_kernels.hip).
struct Blas {
    double2* partial = nullptr;   // [max_blocks * (max_vecs)] complex partial sums
    double2* result = nullptr;    // [max_vecs] reduced results
    int max_blocks = 0, max_vecs = 0;
    hipStream_t as = nullptr;     // stream of the pool the buffers came from, or none
};
// With pooled, the buffers come from the stream-ordered pool on s (and go
// back to it on s), else from hipMalloc.
hipError_t blas_init(Blas& b, int max_vecs, hipStream_t s, bool pooled = false);
void blas_free(Blas& b);
// h[i] = <V_i, w> for i < k (V_i = V + i*ld), conjugate-linear in V_i.
hipError_t blas_multidot(Blas& b, const double2* V, int64_t ld, int k, const double2* w, int64_t n,
                         hipStream_t s);
// w -= sum_i h[i] V_i, with h read from device memory (b.result) times `sign`.
hipError_t blas_multiaxpy(Blas& b, const double2* V, int64_t ld, int k, double2* w, int64_t n,
                          hipStream_t s);
hipError_t blas_scale(double2* x, const double2* alpha_dev, int64_t n, int invert, hipStream_t s);
// y = a*x + b*y (host scalars)
hipError_t blas_axpby(double2 a, const double2* x, double2 b, double2* y, int64_t n, hipStream_t s);
// y = sum_i c[i] V_i (host coefficients, copied to a device buffer first)
hipError_t blas_combine(const double2* V, int64_t ld, int k, const double2* c_dev, double2* y,
                        int64_t n, int accumulate, hipStream_t s);

// Per-solve data movement kernels.
hipError_t gather_source(const double* f_re, const double* f_im, const int* gidx,
                         const double* area, int64_t n, void* Fre, void* Fim, int fp32,
                         hipStream_t s);
hipError_t embed_trace(const double* g_re, const double* g_im, const int64_t* trace_idx,
                       int64_t n_if, double2* G, hipStream_t s);
hipError_t glue_solution(const double2* usub, int Nx, int Ny, int P, int mx, int my, int sx,
                         int sy, int64_t nloc, double* u_re, double* u_im, hipStream_t s);
hipError_t mask_interface(double2* G, const int* is_iface, int64_t n_if, hipStream_t s);
hipError_t split_complex(const double2* z, double* re, double* im, int64_t n, hipStream_t s);

// Whole-domain operator y = S x (FP64) on the global node grid.
struct OperatorArgs {
    int Nx, Ny, P, nx, ny;
    double sx_ref, sy_ref;        // 2/hx, 2/hy
    const double* wx;             // assembled physical 1D weights along x (Nx)
    const double* wy;             // along y (Ny)
    const double* M;              // lumped mass per node (N)
    const double* H;              // lumped boundary mass per node (N)
    double omega;
    double K1[kMaxP + 1][kMaxP + 1];
};
hipError_t launch_operator(const OperatorArgs& a, const double2* x, double2* y, hipStream_t s);

// No-allocation residual (noalloc.hip): at most this many grid rows.
constexpr int kNoAllocMaxRows = 16384;
// Device address of the no-allocation scratch array on device dev, which
// must be the current device; looked up once per device, then cached.
hipError_t noalloc_scratch(int dev, double2** ptr);
// out[0] = ||b - S u|| / ||b|| for device planes u, f, g (f, g, u_im may be
// null); part: the scratch array (Ny row partials).  No allocation.
hipError_t launch_residual_noalloc(const OperatorArgs& a, const double* u_re, const double* u_im,
                                   const double* f_re, const double* f_im, const double* g_re,
                                   const double* g_im, double2* part, double* out,
                                   hipStream_t s);
// work[g] = (|b - S u|^2, |b|^2) per global node (f, g may be null).
hipError_t launch_residual(const OperatorArgs& a, const double2* u, const double* f_re,
                           const double* f_im, const double* g_re, const double* g_im,
                           double2* work, hipStream_t s);
// b.result[0] = sum of v (both components), deterministic.
hipError_t blas_sum2(Blas& b, const double2* v, int64_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// 3D box decomposition: one work item per box subdomain, one thread per node.
struct Sub3 {
    int nt;              // leapfrog steps per period
    int toff;            // offset of this subdomain's filter tables
    int64_t node_off;    // first local node in the per-node arrays
    int64_t if_off;      // first slot of its six faces (x0, x1, y0, y1, z0, z1)
    int64_t nbr_off[6];  // first slot of the neighbour face receiving each face, -1: outer
    int64_t gbase;       // global index of its local node (0, 0, 0)
    double sigma;        // leapfrog step sin(omega dt / 2) / (omega / 2)
    double pd0c, pd0s;   // omega cos(pi/N_t), omega sin(pi/N_t)
    double two_over_nt;  // 2 / N_t
};

template <typename Real>
struct Sweep3Args {
    const Sub3* desc;
    int n_items;
    int nxl, nyl, nzl, mx, my, mz, P;
    int per_sub;             // interface slots per subdomain
    const int* perm;         // thread -> local node (nloc entries, shared by all subdomains)
    int face_off[6];         // first slot of each face within a subdomain
    const Real* alpha;       // (M - theta H) / (M + theta H)
    const Real* betaX;       // beta * (2/hx) * Wy * Wz
    const Real* betaY;       // beta * (2/hy) * Wx * Wz
    const Real* betaZ;       // beta * (2/hz) * Wx * Wy
    const Real* beta;        // sigma / (M + theta H)
    int Nx, Ny;              // global node grid (x and y extents) for indexing f
    const double* f_re;      // source f at the global nodes, or null
    const double* f_im;
    const double* w1d;       // physical lumped 1D weights of a subdomain: x, then y, then z
    const double* kside;     // omega / c per interface slot
    const Real* kap;         // kappa(nu)
    const Real* kaph;        // kappa(nu + 1/2) / omega
    const Real* cs;          // cos(2 pi nu / N_t)
    const Real* sn;          // sin(2 pi nu / N_t)
    const double2* g_in;
    double2* g_out;
    double src;
    double2* u;
    int* wh_iters;
    double tau;
    int max_wh;
    size_t lds_bytes;
    double K1[kMaxP + 1][kMaxP + 1];  // reference D^T W D of degree P
};
template <typename Real>
hipError_t launch_sweep3(const Sweep3Args<Real>& a, int wg, hipStream_t s);
size_t sweep3_lds_bytes(int nxl, int nyl, int nzl, int P, int nt_max, size_t real_size);
// Thread -> node order of the 3D sweep for a subdomain shape and sweep
// precision: each aligned group of 256 / real_size lanes reads distinct LDS
// banks in every stencil tap where the shape allows.
void sweep3_thread_order(int nxl, int nyl, int nzl, int P, size_t real_size, int* perm);

// Whole-box operator y = S x (FP64) on the global node grid.
struct Operator3Args {
    int Nx, Ny, Nz, P, nx, ny, nz;
    int kchunk;                     // planes per workgroup along z
    double sx_ref, sy_ref, sz_ref;  // 2/hx, 2/hy, 2/hz
    const double* wx;               // assembled physical 1D weights (Nx, Ny, Nz)
    const double* wy;
    const double* wz;
    const double* M;
    const double* H;
    double omega;
    double K1[kMaxP + 1][kMaxP + 1];
};
hipError_t launch_operator3(const Operator3Args& a, const double2* x, double2* y, hipStream_t s);
// ug = mean of the subdomain copies of every global node.
hipError_t launch_glue3(const Operator3Args& a, const double2* usub, int mx, int my, int mz, int sx,
                        int sy, int sz, double2* ug, hipStream_t s);
// work[g] = (|b - Su|^2, |b|^2), b = (f, phi) at the global nodes (f may be null).
hipError_t launch_residual3(const Operator3Args& a, const double* f_re, const double* f_im,
                            const double2* Su, double2* work, hipStream_t s);

}  // namespace wdd
