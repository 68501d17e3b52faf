// FP64 kernels around the sweep: the outer Krylov iteration's vector
// operations on interface data (Sec. III, last paragraph: the lambda
// iteration accelerated by a Krylov method), per-solve data movement, and
// the whole-domain Helmholtz operator S = A - i omega H - omega^2 M (eq. (4)).
//
// Reductions are deterministic: fixed-size block partials, then one block
// sums the partials in a fixed order.
#include "operator_device.h"

namespace wdd {

namespace {

constexpr int kBT = 256;       // threads per block of the vector kernels
constexpr int kMaxBlocks = 240;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
    return make_double2(a.x + b.x, a.y + b.y);
}
// conj(a) * b
__device__ __forceinline__ double2 cdotc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ double2 block_sum(double2 v, double2* sh) {
    return block_sum_d2(v, sh);
}

// partial[blk * k + i] = sum over this block's chunk of conj(V_i) w
__global__ void __launch_bounds__(kBT) multidot_partial(const double2* V, int64_t ld, int k,
                                                        const double2* w, int64_t n,
                                                        double2* partial) {
    __shared__ double2 sh[kBT / 64];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    for (int i = 0; i < k; ++i) {
        const double2* v = V + (int64_t)i * ld;
        double2 acc = make_double2(0.0, 0.0);
        for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) acc = cadd(acc, cdotc(v[j], w[j]));
        const double2 s = block_sum(acc, sh);
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * k + i] = s;
    }
}

__global__ void reduce_partials(const double2* partial, int nblk, int k, double2* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    double2 s = make_double2(0.0, 0.0);
    for (int b = 0; b < nblk; ++b) s = cadd(s, partial[(int64_t)b * k + i]);
    out[i] = s;
}

// w -= sum_i h_i V_i
__global__ void multiaxpy_kernel(const double2* V, int64_t ld, int k, const double2* h, double2* w,
                                 int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double2 acc = w[j];
    for (int i = 0; i < k; ++i) {
        const double2 v = V[(int64_t)i * ld + j];
        const double2 c = h[i];
        acc.x -= c.x * v.x - c.y * v.y;
        acc.y -= c.x * v.y + c.y * v.x;
    }
    w[j] = acc;
}

// y = sum_i c_i V_i (+ y if accumulate)
__global__ void combine_kernel(const double2* V, int64_t ld, int k, const double2* c, double2* y,
                               int64_t n, int accumulate) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double2 acc = accumulate ? y[j] : make_double2(0.0, 0.0);
    for (int i = 0; i < k; ++i) {
        const double2 v = V[(int64_t)i * ld + j];
        const double2 a = c[i];
        acc.x += a.x * v.x - a.y * v.y;
        acc.y += a.x * v.y + a.y * v.x;
    }
    y[j] = acc;
}

// x *= alpha or x /= alpha (alpha real part only, read from device memory)
__global__ void scale_kernel(double2* x, const double2* alpha, int64_t n, int invert) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double a = invert ? 1.0 / alpha->x : alpha->x;
    x[j] = make_double2(x[j].x * a, x[j].y * a);
}

// y = a x + b y; y is not read when b = 0 (it may hold stale memory, and
// 0 * NaN would poison the result).
__global__ void axpby_kernel(double2 a, const double2* x, double2 b, double2* y, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double2 xv = x[j];
    const double2 yv = (b.x == 0.0 && b.y == 0.0) ? make_double2(0.0, 0.0) : y[j];
    y[j] = make_double2(a.x * xv.x - a.y * xv.y + b.x * yv.x - b.y * yv.y,
                        a.x * xv.y + a.y * xv.x + b.x * yv.y + b.y * yv.x);
}

template <typename T>
__global__ void gather_source_kernel(const double* f_re, const double* f_im, const int* gidx,
                                     const double* area, int64_t n, T* Fre, T* Fim) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int g = gidx[j];
    Fre[j] = (T)(area[j] * f_re[g]);
    Fim[j] = (T)(f_im ? area[j] * f_im[g] : 0.0);
}

__global__ void embed_trace_kernel(const double* g_re, const double* g_im, const int64_t* idx,
                                   int64_t n_if, double2* G) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_if) return;
    const int64_t t = idx[j];
    if (t < 0) {
        G[j] = make_double2(0.0, 0.0);
    } else {
        G[j] = make_double2(g_re ? g_re[t] : 0.0, g_im ? g_im[t] : 0.0);
    }
}

__global__ void mask_kernel(double2* G, const int* is_iface, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (!is_iface[j]) G[j] = make_double2(0.0, 0.0);
}

__global__ void split_kernel(const double2* z, double* re, double* im, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    re[j] = z[j].x;
    im[j] = z[j].y;
}

// u(i, j) = average of the subdomain copies of global node (i, j), summed
// in a fixed order (left-to-right, bottom-to-top).
__global__ void glue_kernel(const double2* usub, int Nx, int Ny, int P, int mx, int my, int sx,
                            int sy, int64_t nloc, double* u_re, double* u_im) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)Nx * Ny) return;
    const int i = (int)(g % Nx), j = (int)(g / Nx);
    const int wx = mx * P, wy = my * P;
    const int nxl = wx + 1;
    int a_lo = i / wx, b_lo = j / wy;
    int a_hi = a_lo, b_hi = b_lo;
    if (a_lo >= sx) a_lo = a_hi = sx - 1;
    else if (i % wx == 0 && a_lo > 0) a_lo = a_lo - 1;
    if (b_lo >= sy) b_lo = b_hi = sy - 1;
    else if (j % wy == 0 && b_lo > 0) b_lo = b_lo - 1;
    double sr = 0.0, si = 0.0;
    int cnt = 0;
    for (int b = b_lo; b <= b_hi; ++b)
        for (int a = a_lo; a <= a_hi; ++a) {
            const int il = i - a * wx, jl = j - b * wy;
            const double2 v = usub[(int64_t)(b * sx + a) * nloc + (int64_t)jl * nxl + il];
            sr += v.x;
            si += v.y;
            ++cnt;
        }
    u_re[g] = sr / cnt;
    u_im[g] = si / cnt;
}

// y = S x on the global grid: (A x)_{ij} = (2/hx) Wy_j sum_k Khat_x[i,k] x_kj
// + (2/hy) Wx_i sum_k Khat_y[j,k] x_ik, then - i omega H x - omega^2 M x.
// One thread per node, blocks of one grid row (no division per thread); the
// degree is a template parameter so the element windows unroll and the
// reference matrix entries stay in scalar registers.

// Node (i, j) of the block's grid row; false past the row's end.
__device__ __forceinline__ bool grid_node(const OperatorArgs& A, int& i, int& j) {
    const int bpr = (A.Nx + kBT - 1) / kBT;
    j = (int)blockIdx.x / bpr;
    i = ((int)blockIdx.x - j * bpr) * kBT + (int)threadIdx.x;
    return i < A.Nx;
}

template <int P>
__global__ void __launch_bounds__(kBT) operator_kernel(const OperatorArgs A, const double2* x,
                                                       double2* y) {
    int i, j;
    if (!grid_node(A, i, j)) return;
    y[(int64_t)j * A.Nx + i] = apply_node<P>(A, Interleaved{x}, i, j);
}

// Per node: r = b - S u with b = (Wx Wy) f + boundary trace terms; writes
// (|r|^2, |b|^2) for a deterministic reduction.
template <int P>
__global__ void __launch_bounds__(kBT) residual_kernel(const OperatorArgs A, const double2* u,
                                                       const double* f_re, const double* f_im,
                                                       const double* g_re, const double* g_im,
                                                       double2* out) {
    int i, j;
    if (!grid_node(A, i, j)) return;
    out[(int64_t)j * A.Nx + i] =
        residual_node<P>(A, Interleaved{u}, f_re, f_im, g_re, g_im, i, j);
}

// partial[blk] = sum of v over this block's chunk (both components)
__global__ void __launch_bounds__(kBT) sum2_partial(const double2* v, int64_t n, double2* partial) {
    __shared__ double2 sh[kBT / 64];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) acc = cadd(acc, v[j]);
    const double2 s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

inline int nblocks(int64_t n, int bt) { return (int)((n + bt - 1) / bt); }

}  // namespace

// Blocks of the operator / residual launches: whole grid rows of kBT-node
// blocks.
static inline unsigned grid_blocks(const OperatorArgs& a) {
    return (unsigned)(((a.Nx + kBT - 1) / kBT) * (int64_t)a.Ny);
}

hipError_t launch_residual(const OperatorArgs& a, const double2* u, const double* f_re,
                           const double* f_im, const double* g_re, const double* g_im,
                           double2* work, hipStream_t s) {
#define L(PP)                                                                                 \
    hipLaunchKernelGGL((residual_kernel<PP>), dim3(grid_blocks(a)), dim3(kBT), 0, s, a, u, \
                       f_re, f_im, g_re, g_im, work)
    switch (a.P) {
        case 1: L(1); break;
        case 2: L(2); break;
        case 3: L(3); break;
        case 4: L(4); break;
        default: return hipErrorInvalidValue;
    }
#undef L
    return hipGetLastError();
}

hipError_t blas_sum2(Blas& b, const double2* v, int64_t n, hipStream_t s) {
    int nblk = nblocks(n, kBT * 4);
    if (nblk > b.max_blocks) nblk = b.max_blocks;
    if (nblk < 1) nblk = 1;
    hipLaunchKernelGGL(sum2_partial, dim3(nblk), dim3(kBT), 0, s, v, n, b.partial);
    hipLaunchKernelGGL(reduce_partials, dim3(1), dim3(64), 0, s, b.partial, nblk, 1, b.result);
    return hipGetLastError();
}

hipError_t blas_init(Blas& b, int max_vecs, hipStream_t s, bool pooled) {
    b.max_blocks = kMaxBlocks;
    b.max_vecs = max_vecs;
    b.as = pooled ? s : nullptr;
    const size_t np = sizeof(double2) * (size_t)kMaxBlocks * max_vecs, nr = sizeof(double2) * (size_t)max_vecs;
    hipError_t e = b.as ? hipMallocAsync(reinterpret_cast<void**>(&b.partial), np, b.as)
                        : hipMalloc(&b.partial, np);
    if (e != hipSuccess) return e;
    return b.as ? hipMallocAsync(reinterpret_cast<void**>(&b.result), nr, b.as) : hipMalloc(&b.result, nr);
}

void blas_free(Blas& b) {
    if (b.partial) (void)(b.as ? hipFreeAsync(b.partial, b.as) : hipFree(b.partial));
    if (b.result) (void)(b.as ? hipFreeAsync(b.result, b.as) : hipFree(b.result));
    b.partial = b.result = nullptr;
    b.as = nullptr;
}

hipError_t blas_multidot(Blas& b, const double2* V, int64_t ld, int k, const double2* w, int64_t n,
                         hipStream_t s) {
    if (k > b.max_vecs) return hipErrorInvalidValue;
    int nblk = nblocks(n, kBT * 4);
    if (nblk > b.max_blocks) nblk = b.max_blocks;
    if (nblk < 1) nblk = 1;
    hipLaunchKernelGGL(multidot_partial, dim3(nblk), dim3(kBT), 0, s, V, ld, k, w, n, b.partial);
    hipLaunchKernelGGL(reduce_partials, dim3(nblocks(k, 64)), dim3(64), 0, s, b.partial, nblk, k,
                       b.result);
    return hipGetLastError();
}

hipError_t blas_multiaxpy(Blas& b, const double2* V, int64_t ld, int k, double2* w, int64_t n,
                          hipStream_t s) {
    hipLaunchKernelGGL(multiaxpy_kernel, dim3(nblocks(n, kBT)), dim3(kBT), 0, s, V, ld, k, b.result,
                       w, n);
    return hipGetLastError();
}

hipError_t blas_scale(double2* x, const double2* alpha_dev, int64_t n, int invert, hipStream_t s) {
    hipLaunchKernelGGL(scale_kernel, dim3(nblocks(n, kBT)), dim3(kBT), 0, s, x, alpha_dev, n, invert);
    return hipGetLastError();
}

hipError_t blas_axpby(double2 a, const double2* x, double2 b, double2* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n, kBT)), dim3(kBT), 0, s, a, x, b, y, n);
    return hipGetLastError();
}

hipError_t blas_combine(const double2* V, int64_t ld, int k, const double2* c_dev, double2* y,
                        int64_t n, int accumulate, hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel, dim3(nblocks(n, kBT)), dim3(kBT), 0, s, V, ld, k, c_dev, y, n,
                       accumulate);
    return hipGetLastError();
}

hipError_t gather_source(const double* f_re, const double* f_im, const int* gidx,
                         const double* area, int64_t n, void* Fre, void* Fim, int fp32,
                         hipStream_t s) {
    if (fp32)
        hipLaunchKernelGGL(gather_source_kernel<float>, dim3(nblocks(n, kBT)), dim3(kBT), 0, s, f_re,
                           f_im, gidx, area, n, (float*)Fre, (float*)Fim);
    else
        hipLaunchKernelGGL(gather_source_kernel<double>, dim3(nblocks(n, kBT)), dim3(kBT), 0, s,
                           f_re, f_im, gidx, area, n, (double*)Fre, (double*)Fim);
    return hipGetLastError();
}

hipError_t embed_trace(const double* g_re, const double* g_im, const int64_t* trace_idx,
                       int64_t n_if, double2* G, hipStream_t s) {
    hipLaunchKernelGGL(embed_trace_kernel, dim3(nblocks(n_if, kBT)), dim3(kBT), 0, s, g_re, g_im,
                       trace_idx, n_if, G);
    return hipGetLastError();
}

hipError_t glue_solution(const double2* usub, int Nx, int Ny, int P, int mx, int my, int sx,
                         int sy, int64_t nloc, double* u_re, double* u_im, hipStream_t s) {
    hipLaunchKernelGGL(glue_kernel, dim3(nblocks((int64_t)Nx * Ny, kBT)), dim3(kBT), 0, s, usub, Nx,
                       Ny, P, mx, my, sx, sy, nloc, u_re, u_im);
    return hipGetLastError();
}

hipError_t mask_interface(double2* G, const int* is_iface, int64_t n_if, hipStream_t s) {
    hipLaunchKernelGGL(mask_kernel, dim3(nblocks(n_if, kBT)), dim3(kBT), 0, s, G, is_iface, n_if);
    return hipGetLastError();
}

hipError_t split_complex(const double2* z, double* re, double* im, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(split_kernel, dim3(nblocks(n, kBT)), dim3(kBT), 0, s, z, re, im, n);
    return hipGetLastError();
}

hipError_t launch_operator(const OperatorArgs& a, const double2* x, double2* y, hipStream_t s) {
#define L(PP) \
    hipLaunchKernelGGL((operator_kernel<PP>), dim3(grid_blocks(a)), dim3(kBT), 0, s, a, x, y)
    switch (a.P) {
        case 1: L(1); break;
        case 2: L(2); break;
        case 3: L(3); break;
        case 4: L(4); break;
        default: return hipErrorInvalidValue;
    }
#undef L
    return hipGetLastError();
}

}  // namespace wdd
