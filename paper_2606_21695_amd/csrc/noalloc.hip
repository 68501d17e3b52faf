// Global residual without device allocation: ||b - S u||_2 / ||b||_2 of the
// system eq. (4) for device arrays, for callers that cannot allocate (code
// under stream capture, tight serving loops).  Its reduction partials live in
// a file-scope device array instead of a buffer allocated by the library.
//
// One workgroup per grid row: each thread sums (|b - S u|^2, |b|^2) over the
// row's nodes at its stride, the workgroup reduces them in a fixed order into
// scratch[row]; a second kernel sums the rows in order and writes the ratio.
// Every launch overwrites the partials of all rows it uses, so nothing needs
// clearing between calls; two calls in flight at once on one GPU share the
// array and race.
#include <mutex>

#include "operator_device.h"

namespace wdd {

namespace {

constexpr int kNaThreads = 256;

// Row partials of the residual reduction (one per grid row, at most
// kNoAllocMaxRows); each GPU holds its own copy.
static __device__ __align__(256) double2 scratch[kNoAllocMaxRows];

template <int P>
__global__ void __launch_bounds__(kNaThreads)
    residual_rows_kernel(const OperatorArgs A, const double* u_re, const double* u_im,
                         const double* f_re, const double* f_im, const double* g_re,
                         const double* g_im, double2* part) {
    __shared__ double2 sh[kNaThreads / 64];
    const int j = blockIdx.x;
    const Planes u{u_re, u_im};
    double2 acc = make_double2(0.0, 0.0);
    for (int i = threadIdx.x; i < A.Nx; i += kNaThreads) {
        const double2 v = residual_node<P>(A, u, f_re, f_im, g_re, g_im, i, j);
        acc.x += v.x;
        acc.y += v.y;
    }
    const double2 s = block_sum_d2(acc, sh);
    if (threadIdx.x == 0) part[j] = s;
}

// out[0] = sqrt(sum |r|^2 / sum |b|^2) (sqrt(sum |r|^2) when b = 0).
__global__ void __launch_bounds__(kNaThreads)
    residual_rows_finish(const double2* part, int rows, double* out) {
    __shared__ double2 sh[kNaThreads / 64];
    double2 acc = make_double2(0.0, 0.0);
    for (int r = threadIdx.x; r < rows; r += kNaThreads) {
        acc.x += part[r].x;
        acc.y += part[r].y;
    }
    const double2 s = block_sum_d2(acc, sh);
    if (threadIdx.x == 0) out[0] = s.y > 0.0 ? sqrt(s.x / s.y) : sqrt(s.x);
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(int dev, double2** ptr) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev) return hipErrorInvalidDevice;  // the caller makes dev current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *ptr = static_cast<double2*>(g_scratch[dev]);
    return hipSuccess;
}

hipError_t launch_residual_noalloc(const OperatorArgs& a, const double* u_re, const double* u_im,
                                   const double* f_re, const double* f_im, const double* g_re,
                                   const double* g_im, double2* part, double* out,
                                   hipStream_t s) {
    if (a.Ny < 1 || a.Ny > kNoAllocMaxRows) return hipErrorInvalidValue;
#define L(PP)                                                                               \
    hipLaunchKernelGGL((residual_rows_kernel<PP>), dim3(a.Ny), dim3(kNaThreads), 0, s, a, u_re, \
                       u_im, f_re, f_im, g_re, g_im, part)
    switch (a.P) {
        case 1: L(1); break;
        case 2: L(2); break;
        case 3: L(3); break;
        case 4: L(4); break;
        default: return hipErrorInvalidValue;
    }
#undef L
    hipLaunchKernelGGL(residual_rows_finish, dim3(1), dim3(kNaThreads), 0, s, part, a.Ny, out);
    return hipGetLastError();
}

}  // namespace wdd
