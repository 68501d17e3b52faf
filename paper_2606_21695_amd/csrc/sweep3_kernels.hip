// 3D box workload (the hexahedral experiments of Sec. VII-B): one DD cycle
// (Algorithm 1: assemble b, WaveHoltz, interface update) for every box
// subdomain in one launch, one workgroup per subdomain and one thread per
// node (the paper's one-DOF-per-thread strategy, up to 1024 nodes per
// subdomain), and the whole-domain operator y = S x.
//
// Stiffness: A = Kx (x) Wy (x) Wz + Wx (x) Ky (x) Wz + Wx (x) Wy (x) Kz applied
// per node as three (2P+1)-point 1D window sums over a zero-padded copy of
// p in LDS (double-buffered: one barrier per step); the weights are folded
// with beta into the per-node coefficients bX, bY, bZ.
#include "wavedd_internal.h"

#include <vector>

namespace wdd {

namespace {

// Deterministic workgroup sum of two FP64 values (butterfly in each wave,
// then a fixed-order sum over the waves).
__device__ __forceinline__ void block_sum2_3(double& a, double& b, double* red) {
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = (blockDim.x + 63) >> 6;
    if (lane == 0) {
        red[2 * w] = a;
        red[2 * w + 1] = b;
    }
    __syncthreads();
    double s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < nw; ++i) {
        s0 += red[2 * i];
        s1 += red[2 * i + 1];
    }
    a = s0;
    b = s1;
    __syncthreads();
}

// Assembled 1D reference stiffness row at node k of a line of n_el
// elements as a (2P+1)-point window centred on k (zero off the line): the
// node is local a of element e = k / P and, when a = 0 and e > 0, also
// local P of element e - 1.
template <typename Real, int P>
__device__ __forceinline__ void window3(Real (&w)[2 * P + 1], int k, int n_el,
                                        const double (*K)[kMaxP + 1]) {
    const int e = k / P, a = k - e * P;
#pragma unroll
    for (int t = 0; t <= 2 * P; ++t) {
        const int d = t - P;
        double v = 0.0;
        if (e < n_el && a + d >= 0 && a + d <= P) v += K[a][a + d];
        if (a == 0 && e > 0 && d <= 0) v += K[P][P + d];
        w[t] = (Real)v;
    }
}

__host__ __device__ inline int box_buf(int nxl, int nyl, int nzl, int P) {
    return (nxl + 2 * P) * (nyl + 2 * P) * (nzl + 2 * P);
}
__host__ __device__ inline int box_tab_off(int nxl, int nyl, int nzl, int P) {
    return (2 * box_buf(nxl, nyl, nzl, P) + 3) & ~3;
}

template <typename Real, int P>
__device__ void sweep3_item(const Sweep3Args<Real>& A, const Sub3& d, int item, Real* lds,
                            double* red) {
    constexpr int W = 2 * P + 1;
    const int nxl = A.nxl, nyl = A.nyl, nzl = A.nzl, tid = threadIdx.x;
    const int px = nxl + 2 * P, py = nyl + 2 * P;
    const int nb = box_buf(nxl, nyl, nzl, P);
    Real* buf0 = lds;
    Real* buf1 = lds + nb;
    Real* TAB = lds + box_tab_off(nxl, nyl, nzl, P);
    for (int i = tid; i < 2 * nb; i += blockDim.x) lds[i] = Real(0);
    for (int nu = tid; nu < d.nt; nu += blockDim.x) {
        TAB[4 * nu + 0] = A.cs[d.toff + nu];
        TAB[4 * nu + 1] = A.sn[d.toff + nu];
        TAB[4 * nu + 2] = A.kap[d.toff + nu];
        TAB[4 * nu + 3] = A.kaph[d.toff + nu];
    }
    const int nloc = nxl * nyl * nzl;
    const bool has = tid < nloc;
    // node of this thread: a permutation that gives the lanes of each group
    // distinct LDS banks (every tap is a fixed offset from the node's slot)
    const int t0 = has ? A.perm[tid] : 0;
    const int il = t0 % nxl, jl = (t0 / nxl) % nyl, kl = t0 / (nxl * nyl);
    const int pidx = ((kl + P) * py + (jl + P)) * px + (il + P);
    const int sy = px, sz = px * py;
    // stiffness windows scaled by the per-node weights beta (2/h) W W: the
    // off-centre taps of the three directions and one merged centre tap
    Real cx[W], cy[W], cz[W];
    window3<Real, P>(cx, il, A.mx, A.K1);
    window3<Real, P>(cy, jl, A.my, A.K1);
    window3<Real, P>(cz, kl, A.mz, A.K1);
    const int64_t n = d.node_off + t0;
    Real al = Real(0), wc = Real(0), bbr = Real(0), bbi = Real(0);
    if (has) {
        al = A.alpha[n];
        const Real bX = A.betaX[n], bY = A.betaY[n], bZ = A.betaZ[n];
        wc = bX * cx[P] + bY * cy[P] + bZ * cz[P];
#pragma unroll
        for (int t = 0; t < W; ++t) {
            cx[t] *= bX;
            cy[t] *= bY;
            cz[t] *= bZ;
        }
        // b = src * (f, phi) + sum over the faces through the node of W_face g
        const double* Wx = A.w1d;
        const double* Wy = Wx + nxl;
        const double* Wz = Wy + nyl;
        double br = 0.0, bi = 0.0;
        if (A.f_re) {
            const int64_t gi = d.gbase + ((int64_t)kl * A.Ny + jl) * A.Nx + il;
            const double v = A.src * (Wx[il] * Wy[jl] * Wz[kl]);
            br = v * A.f_re[gi];
            bi = v * A.f_im[gi];
        }
        const int64_t o = d.if_off;
        double2 g;
        if (il == 0) { g = A.g_in[o + A.face_off[0] + kl * nyl + jl]; br += Wz[kl] * Wy[jl] * g.x; bi += Wz[kl] * Wy[jl] * g.y; }
        if (il == nxl - 1) { g = A.g_in[o + A.face_off[1] + kl * nyl + jl]; br += Wz[kl] * Wy[jl] * g.x; bi += Wz[kl] * Wy[jl] * g.y; }
        if (jl == 0) { g = A.g_in[o + A.face_off[2] + kl * nxl + il]; br += Wz[kl] * Wx[il] * g.x; bi += Wz[kl] * Wx[il] * g.y; }
        if (jl == nyl - 1) { g = A.g_in[o + A.face_off[3] + kl * nxl + il]; br += Wz[kl] * Wx[il] * g.x; bi += Wz[kl] * Wx[il] * g.y; }
        if (kl == 0) { g = A.g_in[o + A.face_off[4] + jl * nxl + il]; br += Wy[jl] * Wx[il] * g.x; bi += Wy[jl] * Wx[il] * g.y; }
        if (kl == nzl - 1) { g = A.g_in[o + A.face_off[5] + jl * nxl + il]; br += Wy[jl] * Wx[il] * g.x; bi += Wy[jl] * Wx[il] * g.y; }
        const double be = (double)A.beta[n];
        bbr = (Real)(be * br);
        bbi = (Real)(be * bi);
    }
    __syncthreads();
    const Real sig = (Real)d.sigma;
    const int nt = d.nt;
    int it = 0;
    Real p = Real(0), pd = Real(0), vr = Real(0), vi = Real(0);
    WhStall stall;
    for (int m = 0; m < A.max_wh; ++m) {
        // p = Re u, pdot^{1/2} = Re{-i omega u e^{-i pi/N_t}}, v = kappa_0 p + (i/omega) kappa_{1/2} pdot
        p = pd = Real(0);
        if (m > 0 && has) {
            const double2 u = A.u[n];
            p = (Real)u.x;
            pd = (Real)(u.y * d.pd0c - u.x * d.pd0s);
        }
        vr = TAB[2] * p;
        vi = TAB[3] * pd;
        for (int nu = 1; nu < nt; ++nu) {
            Real* buf = (nu & 1) ? buf1 : buf0;
            const Real c = TAB[4 * nu + 0], sv = TAB[4 * nu + 1];
            const Real k1 = TAB[4 * nu + 2], k2 = TAB[4 * nu + 3];
            p = fma(sig, pd, p);
            if (has) buf[pidx] = p;
            __syncthreads();
            // the tap addresses are formed anew each step (an opaque copy
            // of the index): hoisting all of them out of the loop costs
            // more registers than the adds it saves
            int ix = pidx;
            asm volatile("" : "+v"(ix));
            const Real* bp = buf + ix;
            Real acc = wc * p;
#pragma unroll
            for (int t = 0; t < W; ++t) {
                if (t == P) continue;
                acc = fma(cx[t], bp[t - P], acc);
                acc = fma(cy[t], bp[(t - P) * sy], acc);
                acc = fma(cz[t], bp[(t - P) * sz], acc);
            }
            Real tt = bbr * c;
            tt = fma(bbi, sv, tt);
            tt -= acc;
            pd = fma(al, pd, tt);
            vr = fma(k1, p, vr);
            vi = fma(k2, pd, vi);
        }
        // u = (2/N_t) v (eq. (7)); fixed-point residual of this iteration
        double dsum = 0.0, nsum = 0.0;
        if (has) {
            const double ur = d.two_over_nt * (double)vr, ui = d.two_over_nt * (double)vi;
            double orr = 0.0, oi = 0.0;
            if (m > 0) {
                const double2 o = A.u[n];
                orr = o.x;
                oi = o.y;
            }
            dsum = (ur - orr) * (ur - orr) + (ui - oi) * (ui - oi);
            nsum = ur * ur + ui * ui;
            A.u[n] = make_double2(ur, ui);
        }
        block_sum2_3(dsum, nsum, red);
        it = m + 1;
        if (!(dsum == dsum)) break;
        if (wh_stop<Real>(A.tau, dsum, nsum, stall)) break;
    }
    __threadfence_block();
    __syncthreads();
    // interface update (eq. (2)): -g - 2 i (omega/c) u into the neighbour's slot
    const int f1 = nzl * nyl, f2 = 2 * f1, f3 = f2 + nzl * nxl, f4 = f3 + nzl * nxl,
              f5 = f4 + nyl * nxl;
    const int64_t* nbr = A.desc[item].nbr_off;
    for (int k = tid; k < A.per_sub; k += blockDim.x) {
        int s, pos, i, j, kk;
        if (k < f2) {
            s = k < f1 ? 0 : 1;
            pos = k - (s ? f1 : 0);
            kk = pos / nyl;
            j = pos - kk * nyl;
            i = s == 0 ? 0 : nxl - 1;
        } else if (k < f4) {
            s = k < f3 ? 2 : 3;
            pos = k - (s == 2 ? f2 : f3);
            kk = pos / nxl;
            i = pos - kk * nxl;
            j = s == 2 ? 0 : nyl - 1;
        } else {
            s = k < f5 ? 4 : 5;
            pos = k - (s == 4 ? f4 : f5);
            j = pos / nxl;
            i = pos - j * nxl;
            kk = s == 4 ? 0 : nzl - 1;
        }
        const int64_t dst = nbr[s];
        if (dst >= 0) {
            const double2 g = A.g_in[d.if_off + k];
            const double K = A.kside[d.if_off + k];
            const double2 u = A.u[d.node_off + ((int64_t)kk * nyl + j) * nxl + i];
            A.g_out[dst + pos] = make_double2(-g.x + 2.0 * K * u.y, -g.y - 2.0 * K * u.x);
        } else {
            A.g_out[d.if_off + k] = make_double2(0.0, 0.0);
        }
    }
    if (tid == 0) A.wh_iters[item] = it;
}

template <typename Real, int P>
__device__ __forceinline__ void sweep3_items(const Sweep3Args<Real>& A) {
    extern __shared__ double smem_d[];
    double* red = smem_d;
    Real* lds = reinterpret_cast<Real*>(smem_d + 40);
    const int item = blockIdx.x;   // one workgroup per item (grid = n_items)
    if (item >= A.n_items) return;
    const Sub3 d = A.desc[item];   // loaded once: kept in registers across the stores below
    sweep3_item<Real, P>(A, d, item, lds, red);
}

template <typename Real, int P>
__global__ void __launch_bounds__(kMaxWG) sweep3_kernel(const Sweep3Args<Real> A) {
    sweep3_items<Real, P>(A);
}

// The same kernel built to allow 6 waves per SIMD (at most 80 VGPRs): 3-4
// small-subdomain workgroups then share a CU.  Only the prologue spills;
// the step loop does not.
template <typename Real, int P>
__global__ void __launch_bounds__(kMaxWG) __attribute__((amdgpu_waves_per_eu(6, 8)))
sweep3_kernel_capped(const Sweep3Args<Real> A) {
    sweep3_items<Real, P>(A);
}

// y = S x on the whole box.  A workgroup owns a 64 x 4 tile of (x, y)
// columns and marches along z over a chunk of planes: each thread keeps the
// 2P+1 values of its column around the current plane in registers (the z
// taps), and takes the x and y taps from the cache (neighbours in the tile
// or in the tiles beside it, read in the same plane step), so x is fetched
// from HBM about once.  Tiles are numbered so that the workgroups the
// hardware places on one XCD (every eighth) hold a contiguous range of
// tiles: tiles side by side in y then share that XCD's L2.
constexpr int kOpTX = 64, kOpTY = 4;

template <int P>
__global__ void __launch_bounds__(kOpTX * kOpTY) operator3_kernel(const Operator3Args A,
                                                                  const double2* x, double2* y) {
    constexpr int W = 2 * P + 1;
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int t = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const int nbx = (A.Nx + kOpTX - 1) / kOpTX, nby = (A.Ny + kOpTY - 1) / kOpTY;
    const int bx = t % nbx, by = (t / nbx) % nby, kc = t / (nbx * nby);
    const int i = bx * kOpTX + (int)(threadIdx.x % kOpTX);
    const int j = by * kOpTY + (int)(threadIdx.x / kOpTX);
    const int k0 = kc * A.kchunk, k1 = min(A.Nz, k0 + A.kchunk);
    if (i >= A.Nx || j >= A.Ny || k0 >= k1) return;
    const int64_t sj = A.Nx, sk = (int64_t)A.Nx * A.Ny;
    double wx[W], wy[W];
    window3<double, P>(wx, i, A.nx, A.K1);
    window3<double, P>(wy, j, A.ny, A.K1);
    const double wxi = A.wx[i], wyj = A.wy[j];
    const int64_t col = (int64_t)j * sj + i;
    // z window: zw[P + d] = x at plane k + d (0 off the box)
    double2 zw[W];
#pragma unroll
    for (int d = -P; d <= P; ++d) {
        const int kk = k0 + d;
        zw[P + d] = (kk >= 0 && kk < A.Nz && d < P) ? x[kk * sk + col] : make_double2(0.0, 0.0);
    }
    for (int k = k0; k < k1; ++k) {
        if (k + P < A.Nz) zw[W - 1] = x[(k + P) * sk + col];
        const int64_t g = k * sk + col;
        double wz[W];
        window3<double, P>(wz, k, A.nz, A.K1);
        double2 X = make_double2(0.0, 0.0), Y = X, Z = X;
#pragma unroll
        for (int tt = 0; tt < W; ++tt) {
            const int d = tt - P;
            const double2 vx = (i + d >= 0 && i + d < A.Nx) ? x[g + d] : make_double2(0.0, 0.0);
            const double2 vy = (j + d >= 0 && j + d < A.Ny) ? x[g + d * sj] : make_double2(0.0, 0.0);
            X.x += wx[tt] * vx.x;
            X.y += wx[tt] * vx.y;
            Y.x += wy[tt] * vy.x;
            Y.y += wy[tt] * vy.y;
            Z.x += wz[tt] * zw[tt].x;
            Z.y += wz[tt] * zw[tt].y;
        }
        const double wzk = A.wz[k];
        const double cx = A.sx_ref * wyj * wzk, cy = A.sy_ref * wxi * wzk, cz = A.sz_ref * wxi * wyj;
        const double2 v = zw[P];
        const double m = A.omega * A.omega * A.M[g], h = A.omega * A.H[g];
        y[g] = make_double2(cx * X.x + cy * Y.x + cz * Z.x - m * v.x + h * v.y,
                            cx * X.y + cy * Y.y + cz * Z.y - m * v.y - h * v.x);
#pragma unroll
        for (int d = 0; d < W - 1; ++d) zw[d] = zw[d + 1];
        zw[W - 1] = make_double2(0.0, 0.0);
    }
}

// Glue: every global node takes the mean of its subdomain copies (up to 8).
__global__ void __launch_bounds__(256) glue3_kernel(const Operator3Args A, const double2* usub,
                                                    int mx, int my, int mz, int sx, int sy, int sz,
                                                    double2* ug) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t N = (int64_t)A.Nx * A.Ny * A.Nz;
    if (g >= N) return;
    const int i = (int)(g % A.Nx), j = (int)((g / A.Nx) % A.Ny), k = (int)(g / ((int64_t)A.Nx * A.Ny));
    const int ex = mx * A.P, ey = my * A.P, ez = mz * A.P;
    const int nxl = ex + 1, nyl = ey + 1, nzl = ez + 1;
    const int64_t nloc = (int64_t)nxl * nyl * nzl;
    const int a1 = min(i / ex, sx - 1), b1 = min(j / ey, sy - 1), c1 = min(k / ez, sz - 1);
    const int a0 = (i == a1 * ex && a1 > 0) ? a1 - 1 : a1;
    const int b0 = (j == b1 * ey && b1 > 0) ? b1 - 1 : b1;
    const int c0 = (k == c1 * ez && c1 > 0) ? c1 - 1 : c1;
    double sr = 0.0, si = 0.0;
    int cnt = 0;
    for (int c = c0; c <= c1; ++c)
        for (int b = b0; b <= b1; ++b)
            for (int a = a0; a <= a1; ++a) {
                const int64_t l = ((int64_t)c * sy + b) * sx + a;
                const int il = i - a * ex, jl = j - b * ey, kl = k - c * ez;
                const double2 v = usub[l * nloc + ((int64_t)kl * nyl + jl) * nxl + il];
                sr += v.x;
                si += v.y;
                ++cnt;
            }
    ug[g] = make_double2(sr / cnt, si / cnt);
}

// work[g] = (|b - Su|^2, |b|^2) with b = (f, phi) = vol * f (f may be null).
__global__ void __launch_bounds__(256) residual3_kernel(const Operator3Args A, const double* f_re,
                                                        const double* f_im, const double2* Su,
                                                        double2* work) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t N = (int64_t)A.Nx * A.Ny * A.Nz;
    if (g >= N) return;
    const int i = (int)(g % A.Nx), j = (int)((g / A.Nx) % A.Ny), k = (int)(g / ((int64_t)A.Nx * A.Ny));
    double br = 0.0, bi = 0.0;
    if (f_re) {
        const double vol = A.wx[i] * A.wy[j] * A.wz[k];
        br = vol * f_re[g];
        bi = f_im ? vol * f_im[g] : 0.0;
    }
    const double rr = br - Su[g].x, ri = bi - Su[g].y;
    work[g] = make_double2(rr * rr + ri * ri, br * br + bi * bi);
}

}  // namespace

size_t sweep3_lds_bytes(int nxl, int nyl, int nzl, int P, int nt_max, size_t real_size) {
    return 40 * sizeof(double) + ((size_t)box_tab_off(nxl, nyl, nzl, P) + 4 * (size_t)nt_max) * real_size;
}

void sweep3_thread_order(int nxl, int nyl, int nzl, int P, size_t real_size, int* perm) {
    // LDS slot of node (il, jl, kl) in the padded grid, as in the kernel;
    // nodes are bucketed by slot mod G and each group of G lanes takes one
    // node per residue, lane j of the group the residue j (so each half of
    // the group also has distinct residues mod G/2); shifting every slot by a
    // tap offset keeps the residues of a group distinct.
    const int G = (int)(256 / real_size);
    const int px = nxl + 2 * P, py = nyl + 2 * P;
    const int n = nxl * nyl * nzl;
    std::vector<std::vector<int>> bucket(G);
    for (int t = n - 1; t >= 0; --t) {
        const int il = t % nxl, jl = (t / nxl) % nyl, kl = t / (nxl * nyl);
        const int slot = ((kl + P) * py + (jl + P)) * px + (il + P);
        bucket[slot % G].push_back(t);
    }
    int filled = 0;
    std::vector<int> rest;
    while (filled < n) {
        int full = 1;
        for (int r = 0; r < G; ++r)
            if (bucket[r].empty()) full = 0;
        if (!full) break;
        for (int r = 0; r < G; ++r) {
            perm[filled++] = bucket[r].back();
            bucket[r].pop_back();
        }
    }
    // the remainder: round-robin over the residues still present
    for (bool any = true; any;) {
        any = false;
        for (int r = 0; r < G; ++r)
            if (!bucket[r].empty()) {
                perm[filled++] = bucket[r].back();
                bucket[r].pop_back();
                any = true;
            }
    }
}

// The register-capped build pays off for FP64 at P <= 3 when a workgroup is
// at most 12 waves (measured: 343- and 729-node subdomains 1.3x faster;
// FP32, P = 4 and 1000-node subdomains were slower with it).
template <typename Real, int P>
void launch_sweep3_p(const Sweep3Args<Real>& a, int wg, hipStream_t s) {
    if constexpr (sizeof(Real) == 8 && P <= 3) {
        if (wg <= 768) {
            hipLaunchKernelGGL((sweep3_kernel_capped<Real, P>), dim3(a.n_items), dim3(wg),
                               a.lds_bytes, s, a);
            return;
        }
    }
    hipLaunchKernelGGL((sweep3_kernel<Real, P>), dim3(a.n_items), dim3(wg), a.lds_bytes, s, a);
}

template <typename Real>
hipError_t launch_sweep3(const Sweep3Args<Real>& a, int wg, hipStream_t s) {
    if (wg > kMaxWG) return hipErrorInvalidValue;
    switch (a.P) {
        case 1: launch_sweep3_p<Real, 1>(a, wg, s); break;
        case 2: launch_sweep3_p<Real, 2>(a, wg, s); break;
        case 3: launch_sweep3_p<Real, 3>(a, wg, s); break;
        case 4: launch_sweep3_p<Real, 4>(a, wg, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_operator3(const Operator3Args& a, const double2* x, double2* y, hipStream_t s) {
    const int64_t tiles = (int64_t)((a.Nx + kOpTX - 1) / kOpTX) * ((a.Ny + kOpTY - 1) / kOpTY);
    const int64_t nkc = (a.Nz + a.kchunk - 1) / a.kchunk;
    const unsigned blocks = (unsigned)(tiles * nkc);
#define L(PP) hipLaunchKernelGGL((operator3_kernel<PP>), dim3(blocks), dim3(kOpTX * kOpTY), 0, s, a, x, y)
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

hipError_t launch_glue3(const Operator3Args& a, const double2* usub, int mx, int my, int mz, int sx,
                        int sy, int sz, double2* ug, hipStream_t s) {
    const int64_t N = (int64_t)a.Nx * a.Ny * a.Nz;
    hipLaunchKernelGGL(glue3_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, a, usub,
                       mx, my, mz, sx, sy, sz, ug);
    return hipGetLastError();
}

hipError_t launch_residual3(const Operator3Args& a, const double* f_re, const double* f_im,
                            const double2* Su, double2* work, hipStream_t s) {
    const int64_t N = (int64_t)a.Nx * a.Ny * a.Nz;
    hipLaunchKernelGGL(residual3_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, a, f_re,
                       f_im, Su, work);
    return hipGetLastError();
}

template hipError_t launch_sweep3<double>(const Sweep3Args<double>&, int, hipStream_t);
template hipError_t launch_sweep3<float>(const Sweep3Args<float>&, int, hipStream_t);

}  // namespace wdd
