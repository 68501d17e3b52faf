// Device routines of the whole-domain Helmholtz operator
// S = A - i omega H - omega^2 M (eq. (4), GLL quadrature at the nodes, so
// A = Kx (x) Wy + Wx (x) Ky) at one global node, shared by the operator,
// residual and no-allocation residual kernels.
#pragma once
#include "wavedd_internal.h"

namespace wdd {

// Complex values of a global nodal vector: interleaved (re, im) pairs...
struct Interleaved {
    const double2* x;
    __device__ __forceinline__ double2 operator()(int64_t g) const { return x[g]; }
};
// ... or separate real and imaginary planes (imaginary NULL = 0).
struct Planes {
    const double* re;
    const double* im;
    __device__ __forceinline__ double2 operator()(int64_t g) const {
        return make_double2(re[g], im ? im[g] : 0.0);
    }
};

// Row a of the reference element matrix, selected with compile-time
// indices (a is the node's offset inside its element).
template <int P>
__device__ __forceinline__ double kref(const double (*K)[kMaxP + 1], int a, int q) {
    double v = K[0][q];
#pragma unroll
    for (int r = 1; r <= P; ++r) v = (a == r) ? K[r][q] : v;
    return v;
}

// Assembled 1D stiffness row at node k of a line of n_el elements, applied
// to x along the line (nodes base + m * step).
template <int P, typename X>
__device__ __forceinline__ double2 line1d(const X& x, int64_t base, int64_t step, int k, int n_el,
                                          const double (*K)[kMaxP + 1]) {
    const int e = k / P, a = k - e * P;
    double2 s = make_double2(0.0, 0.0);
    // element e (row a), present unless k is the last node of the line
    if (e < n_el) {
#pragma unroll
        for (int q = 0; q <= P; ++q) {
            const double kv = kref<P>(K, a, q);
            const double2 v = x(base + (int64_t)(e * P + q) * step);
            s.x += kv * v.x;
            s.y += kv * v.y;
        }
    }
    // element e - 1 (row P) at a vertex
    if (a == 0 && e > 0) {
#pragma unroll
        for (int q = 0; q <= P; ++q) {
            const double2 v = x(base + (int64_t)((e - 1) * P + q) * step);
            s.x += K[P][q] * v.x;
            s.y += K[P][q] * v.y;
        }
    }
    return s;
}

// (S x) at global node (i, j).
template <int P, typename X>
__device__ __forceinline__ double2 apply_node(const OperatorArgs& A, const X& x, int i, int j) {
    const int64_t g = (int64_t)j * A.Nx + i;
    const double2 Xs = line1d<P>(x, (int64_t)j * A.Nx, 1, i, A.nx, A.K1);
    const double2 Ys = line1d<P>(x, i, A.Nx, j, A.ny, A.K1);
    const double cx = A.sx_ref * A.wy[j], cy = A.sy_ref * A.wx[i];
    const double2 v = x(g);
    const double m = A.omega * A.omega * A.M[g], h = A.omega * A.H[g];
    // (A - i omega H - omega^2 M) v
    return make_double2(cx * Xs.x + cy * Ys.x - m * v.x + h * v.y,
                        cx * Xs.y + cy * Ys.y - m * v.y - h * v.x);
}

// (|b - S u|^2, |b|^2) at global node (i, j), with b = (Wx Wy) f plus the
// boundary trace terms W_side g (eq. (4)); f and g parts may be NULL.
template <int P, typename U>
__device__ __forceinline__ double2 residual_node(const OperatorArgs& A, const U& u,
                                                 const double* f_re, const double* f_im,
                                                 const double* g_re, const double* g_im, int i,
                                                 int j) {
    const int Nx = A.Nx, Ny = A.Ny;
    const int64_t g = (int64_t)j * Nx + i;
    double br = 0.0, bi = 0.0;
    const double area = A.wx[i] * A.wy[j];
    if (f_re) br = area * f_re[g];
    if (f_im) bi = area * f_im[g];
    // boundary trace (left, right, bottom, top)
    const int64_t tl = j, tr = Ny + j, tb = 2 * (int64_t)Ny + i, tt = 2 * (int64_t)Ny + Nx + i;
    if (i == 0) { if (g_re) br += A.wy[j] * g_re[tl]; if (g_im) bi += A.wy[j] * g_im[tl]; }
    if (i == Nx - 1) { if (g_re) br += A.wy[j] * g_re[tr]; if (g_im) bi += A.wy[j] * g_im[tr]; }
    if (j == 0) { if (g_re) br += A.wx[i] * g_re[tb]; if (g_im) bi += A.wx[i] * g_im[tb]; }
    if (j == Ny - 1) { if (g_re) br += A.wx[i] * g_re[tt]; if (g_im) bi += A.wx[i] * g_im[tt]; }
    const double2 s = apply_node<P>(A, u, i, j);
    const double rr = br - s.x, ri = bi - s.y;
    return make_double2(rr * rr + ri * ri, br * br + bi * bi);
}

// Deterministic sum of a double2 over a workgroup of whole waves (butterfly
// within each wave, then a fixed-order sum over waves); the result is valid
// in thread 0.  All threads must call it; sh holds blockDim.x / 64 entries.
__device__ __forceinline__ double2 block_sum_d2(double2 v, double2* sh) {
    for (int off = 32; off > 0; off >>= 1) {
        v.x += __shfl_xor(v.x, off, 64);
        v.y += __shfl_xor(v.y, off, 64);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double2 s = make_double2(0.0, 0.0);
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            s.x += sh[i].x;
            s.y += sh[i].y;
        }
    }
    __syncthreads();
    return s;
}

}  // namespace wdd
