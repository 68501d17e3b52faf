// Sweep kernels: one DD cycle (Algorithm 1: assemble b, WaveHoltz, interface
// update) for every subdomain, one workgroup per subdomain, all subdomains
// in one launch.
//
// The stiffness is the assembled GLL-quadrature form A = Kx (x) Wy + Wx (x) Ky
// (Sec. IV: GLL quadrature at the nodes), applied per unique DOF as two 1D
// banded sums (no element redundancy, no atomics, deterministic order):
//   (A p)_{ij} = (2/hx) Wy_j X_ij + (2/hy) Wx_i Y_ij,
//   X_ij = sum_k Khat_x[i,k] p_kj,   Y_ij = sum_k Khat_y[j,k] p_ik,
// Khat the assembled reference 1D stiffness (element blocks D^T W D).  The
// weights are folded with beta into per-node coefficients betaX, betaY.
//
// Layouts:
//  * PATCH_XCHG: thread t = ey*mx + ex owns the P*P nodes (ex*P+a, ey*P+b),
//    a,b < P, of element (ex, ey), in registers; the subdomain's right
//    column and top row of nodes (mx*P + my*P + 1 of them) are an extra
//    one-node "edge" slot on the first threads.  Only element-boundary values
//    cross threads: each step a thread publishes its a=0 column and b=0 row,
//    reads its right neighbour's column and top neighbour's row, and exchanges
//    partial sums for the shared vertex lines (two workgroup barriers per
//    step).  Interior slots finish between the two barriers.
//  * PATCH: the same ownership with one barrier per step: whole patches are
//    published (double-buffered) and each thread computes its left / bottom
//    neighbours' shares of its vertex lines itself.
//  * NODE: one thread per node (<= 1024 nodes); p double-buffered in LDS
//    with zero padding, so the (2P+1)-point 1D windows need no bounds
//    checks (one barrier per step).
//  * STREAM: any subdomain size; the NODE arithmetic with the state in
//    device memory (zero-padded p grids, one barrier per step); waves walk
//    up column segments with the Y windows in registers and exchange X
//    neighbours across lanes.
// All stage the per-step filter / forcing tables of the subdomain in LDS
// (broadcast reads) when the subdomain starts.  The layout of a problem is
// picked by timing the ones that fit (autotuner in the host library).
#include "wavedd_internal.h"

namespace wdd {

namespace {

// Deterministic workgroup sum of two FP64 values (butterfly within each
// wave, then a fixed-order sum over waves).  All threads must call it.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
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

// b_j = src * F_j + sum over the subdomain sides through node (il, jl) of
// W_side(j) * g_side(j)  (b of eq. (4) with the interface data as lambda).
template <typename Real>
__device__ __forceinline__ double2 assemble_b(const SweepArgs<Real>& A, const SubDesc& d, int il,
                                              int jl) {
    const int64_t node = d.node_off + (int64_t)jl * d.nxl + il;
    double br = 0.0, bi = 0.0;
    if (A.Fre) {
        br = A.src * (double)A.Fre[node];
        bi = A.src * (double)A.Fim[node];
    }
    const double* wx = A.w1d + d.w_off;
    const double* wy = wx + d.nxl;
    const int64_t o = d.if_off;
    if (il == 0) {
        const double2 g = A.g_in[o + jl];
        br += wy[jl] * g.x;
        bi += wy[jl] * g.y;
    }
    if (il == d.nxl - 1) {
        const double2 g = A.g_in[o + d.nyl + jl];
        br += wy[jl] * g.x;
        bi += wy[jl] * g.y;
    }
    if (jl == 0) {
        const double2 g = A.g_in[o + 2 * d.nyl + il];
        br += wx[il] * g.x;
        bi += wx[il] * g.y;
    }
    if (jl == d.nyl - 1) {
        const double2 g = A.g_in[o + 2 * d.nyl + d.nxl + il];
        br += wx[il] * g.x;
        bi += wx[il] * g.y;
    }
    return make_double2(br, bi);
}

// Per-node state and coefficients of one owned node (edge and node slots).
template <typename Real>
struct Slot {
    Real p, pd, vr, vi;         // p, pdot^{nu+1/2}, filter sums (Re, Im / omega)
    Real al, bX, bY, bbr, bbi;  // alpha, betaX, betaY, beta*Re b, beta*Im b
    int64_t node;               // index into the per-node arrays
};

template <typename Real>
__device__ __forceinline__ void slot_zero(Slot<Real>& s) {
    s.p = s.pd = s.vr = s.vi = Real(0);
    s.al = s.bX = s.bY = s.bbr = s.bbi = Real(0);
    s.node = 0;
}

template <typename Real>
__device__ __forceinline__ void slot_load(Slot<Real>& s, const SweepArgs<Real>& A,
                                          const SubDesc& d, int il, int jl) {
    s.node = d.node_off + (int64_t)jl * d.nxl + il;
    s.al = A.coef.alpha[s.node];
    s.bX = A.coef.betaX[s.node];
    s.bY = A.coef.betaY[s.node];
    const double be = (double)A.coef.beta[s.node];
    const double2 b = assemble_b(A, d, il, jl);
    s.bbr = (Real)(be * b.x);
    s.bbi = (Real)(be * b.y);
}

// Start of a WaveHoltz iteration (Algorithm 1): p = Re u,
// pdot^{1/2} = Re{-i omega u e^{-i pi/N_t}}, v = kappa_0 p + (i/omega) kappa_{1/2} pdot.
template <typename Real>
__device__ __forceinline__ void slot_init(Slot<Real>& s, const SweepArgs<Real>& A,
                                          const SubDesc& d, bool from_u, Real k0, Real kh0) {
    if (from_u) {
        const double2 u = A.u[s.node];
        s.p = (Real)u.x;
        s.pd = (Real)(u.y * d.pd0c - u.x * d.pd0s);
    } else {
        s.p = Real(0);
        s.pd = Real(0);
    }
    s.vr = k0 * s.p;
    s.vi = kh0 * s.pd;
}

// One leapfrog velocity update plus filter accumulation, given the
// reference x/y stiffness sums X, Y at the node.
template <typename Real>
__device__ __forceinline__ void slot_step(Slot<Real>& s, Real X, Real Y, Real c, Real sn, Real k1,
                                          Real k2) {
    Real t = s.bbr * c;
    t = fma(s.bbi, sn, t);
    t = fma(-s.bX, X, t);
    t = fma(-s.bY, Y, t);
    s.pd = fma(s.al, s.pd, t);
    s.vr = fma(k1, s.p, s.vr);
    s.vi = fma(k2, s.pd, s.vi);
}

// End of a WaveHoltz iteration: u_new = (2/N_t) v (eq. (7)); accumulate
// ||u_new - u_old||^2 and ||u_new||^2.
template <typename Real>
__device__ __forceinline__ void slot_finish(const Slot<Real>& s, const SweepArgs<Real>& A,
                                            const SubDesc& d, bool has_old, double& dsum,
                                            double& nsum) {
    const double ur = d.two_over_nt * (double)s.vr;
    const double ui = d.two_over_nt * (double)s.vi;
    double orr = 0.0, oi = 0.0;
    if (has_old) {
        const double2 o = A.u[s.node];
        orr = o.x;
        oi = o.y;
    }
    dsum += (ur - orr) * (ur - orr) + (ui - oi) * (ui - oi);
    nsum += ur * ur + ui * ui;
    A.u[s.node] = make_double2(ur, ui);
}

// (K_side u)(pos) along one side of the subdomain: the assembled 1D
// stiffness (2/h) sum_e Khat_e of the side's n_el elements (natural ends)
// applied to the complex iterate u at the side nodes base + j * stride.
template <typename Real>
__device__ double2 side_stiffness(const SweepArgs<Real>& A, const double2* u, int64_t base,
                                  int stride, int pos, int n_el, int P, double scale) {
    double sx = 0.0, sy = 0.0;
    const int e0 = pos / P, a0 = pos - e0 * P;
    // element e0 (local row a0), and element e0 - 1 (local row P) at a vertex
    for (int side = 0; side < 2; ++side) {
        const int e = side == 0 ? e0 : e0 - 1;
        const int a = side == 0 ? a0 : P;
        if (e < 0 || e >= n_el || (side == 1 && a0 != 0)) continue;
        for (int q = 0; q <= P; ++q) {
            const double k = A.K1[P][a][q];
            const double2 v = u[base + (int64_t)(e * P + q) * stride];
            sx += k * v.x;
            sy += k * v.y;
        }
    }
    return make_double2(scale * sx, scale * sy);
}

// Interface update (eq. (2), sign read for consistency with b):
// g_{r,s'} = -g_{l,s} - 2 i (omega/c) u_l on each shared side node; outer
// sides get 0.  With the second-order transmission condition (tc_q = q > 0)
// it adds 2 (q K_side u - omega^2 m u / c^2) / W_side, m = q W_side plus
// q^2/2 at an end whose other side is an interface as well.  Cooperative
// over the workgroup, coalesced along sides.
// Receiving slot of side s (a select over constant indices: a per-lane
// index into the descriptor would put the workgroup's copy of it in
// scratch memory).
__device__ __forceinline__ int64_t side_nbr(const SubDesc& d, int s) {
    return s == 0 ? d.nbr_off[0] : s == 1 ? d.nbr_off[1] : s == 2 ? d.nbr_off[2] : d.nbr_off[3];
}

template <typename Real>
__device__ void exchange(const SweepArgs<Real>& A, const SubDesc& d) {
    const int nxl = d.nxl, nyl = d.nyl;
    const int per = 2 * nyl + 2 * nxl;
    for (int k = threadIdx.x; k < per; k += blockDim.x) {
        int s, pos, node;
        if (k < nyl) {
            s = 0; pos = k; node = k * nxl;
        } else if (k < 2 * nyl) {
            s = 1; pos = k - nyl; node = pos * nxl + nxl - 1;
        } else if (k < 2 * nyl + nxl) {
            s = 2; pos = k - 2 * nyl; node = pos;
        } else {
            s = 3; pos = k - 2 * nyl - nxl; node = (nyl - 1) * nxl + pos;
        }
        const int64_t dst = side_nbr(d, s);
        if (dst >= 0) {
            const double2 g = A.g_in[d.if_off + k];
            const double K = A.kside[d.if_off + k];
            const double2 u = A.u[d.node_off + node];
            double gx = -g.x + 2.0 * K * u.y, gy = -g.y - 2.0 * K * u.x;
            if (d.tc_q > 0.0) {
                const double q = d.tc_q;
                const bool vert = s < 2;   // left / right sides run along y
                const int n = vert ? nyl : nxl;
                const double W = A.w1d[d.w_off + (vert ? nxl + pos : pos)];
                double m = q * W;
                // the sides meeting this one at its first / last node
                if (pos == 0 && side_nbr(d, vert ? 2 : 0) >= 0) m += 0.5 * q * q;
                if (pos == n - 1 && side_nbr(d, vert ? 3 : 1) >= 0) m += 0.5 * q * q;
                const int64_t base = d.node_off + (vert ? (s == 0 ? 0 : nxl - 1) : (s == 2 ? 0 : (int64_t)(nyl - 1) * nxl));
                const double2 Ku = side_stiffness(A, A.u, base, vert ? nxl : 1, pos,
                                                  vert ? d.my : d.mx, d.P,
                                                  vert ? d.sy_ref : d.sx_ref);
                const double f = 2.0 / W;
                gx += f * (q * Ku.x - K * K * m * u.x);
                gy += f * (q * Ku.y - K * K * m * u.y);
            }
            A.g_out[dst + pos] = make_double2(gx, gy);
        } else {
            A.g_out[d.if_off + k] = make_double2(0.0, 0.0);
        }
    }
}

// Copy the subdomain's per-step tables into LDS as {cos, sin, kappa,
// kappa_{+1/2}/omega} quadruples (one broadcast read per step).
template <typename Real>
__device__ __forceinline__ void stage_tables(const SweepArgs<Real>& A, const SubDesc& d, Real* tab) {
    for (int nu = threadIdx.x; nu < d.nt; nu += blockDim.x) {
        tab[4 * nu + 0] = A.cs[d.toff + nu];
        tab[4 * nu + 1] = A.sn[d.toff + nu];
        tab[4 * nu + 2] = A.kap[d.toff + nu];
        tab[4 * nu + 3] = A.kaph[d.toff + nu];
    }
}

// Coefficients of the assembled 1D reference stiffness row at node k of a
// line of n_el elements, as a (2P+1)-point window centred on k (KL: the
// reference element matrix in LDS, row-major).
template <typename Real, int P>
__device__ __forceinline__ void window_coeffs(Real (&w)[2 * P + 1], int k, int n_el,
                                              const Real* KL) {
#pragma unroll
    for (int j = 0; j <= 2 * P; ++j) w[j] = Real(0);
    const int e = k / P, a = k - e * P;
    if (a == 0) {
        if (e < n_el) {
#pragma unroll
            for (int q = 0; q <= P; ++q) w[P + q] += KL[q];
        }
        if (e > 0) {
#pragma unroll
            for (int q = 0; q <= P; ++q) w[q] += KL[P * (P + 1) + q];
        }
    } else {
        // row a of element e couples the nodes e*P + q, q = 0..P, which sit
        // at window offset q - a
#pragma unroll
        for (int j = 0; j <= 2 * P; ++j) {
            const int q = j - P + a;
            const int qq = q < 0 ? 0 : (q > P ? P : q);
            const Real kv = KL[a * (P + 1) + qq];
            w[j] = (q == qq) ? kv : Real(0);
        }
    }
}

// ---------------------------------------------------------------------------
// PATCH layout
// ---------------------------------------------------------------------------

// LDS carve-up of the patch layout (in units of Real).  VC, VR, SX, SY hold
// P planes of one value per element (plane k of element e at k * mx*my + e),
// so a wave's lanes touch consecutive words.  The edge lines GC (right
// column) and GR (top row) carry kMaxP zeros on both ends so their windows
// need no bounds checks.
struct PatchLds {
    int vc, vr, sx, sy, gc, gr, zr, corner, sink, kl, tab, total;
};

__host__ __device__ inline PatchLds patch_lds(int mx, int my, int P, int nt_max) {
    PatchLds L;
    const int np = mx * my * P;
    L.vc = 0;
    L.vr = L.vc + np;
    L.sx = L.vr + np;
    L.sy = L.sx + np;
    L.gc = L.sy + np;
    L.gr = L.gc + my * P + 1 + 2 * kMaxP;
    L.zr = L.gr + mx * P + 1 + 2 * kMaxP;
    L.corner = L.zr + 2 * kMaxP + 2;
    L.sink = L.corner + 2;
    L.kl = L.sink + 2 * kMaxP;
    L.tab = L.kl + (kMaxP + 1) * (kMaxP + 1);
    L.tab = (L.tab + 3) & ~3;  // 4-aligned quadruples
    L.total = L.tab + 4 * nt_max;
    return L;
}

// Canonical index of the reference stiffness entry K[a][b]: K is symmetric
// and centrosymmetric (K[a][b] = K[P-a][P-b]), so only the canonical entries
// are ever loaded (6 distinct scalars at P = 3).
template <int P>
__host__ __device__ constexpr int kcan_a(int a, int b) {
    return (a <= b ? a : b) <= P - (a <= b ? b : a) ? (a <= b ? a : b) : P - (a <= b ? b : a);
}
template <int P>
__host__ __device__ constexpr int kcan_b(int a, int b) {
    return (a <= b ? a : b) <= P - (a <= b ? b : a) ? (a <= b ? b : a) : P - (a <= b ? a : b);
}

// Thread context of the patch layout for one subdomain.
template <typename Real, int P>
struct PatchCtx {
    bool hasP, hasE;
    int ex, ey;
    Real* VC; Real* VR; Real* SX; Real* SY; Real* GC; Real* GR; Real* CORN; const Real* TAB;
    // neighbour lines and the strides between their entries (mx*my between
    // planes, 1 along an edge line, 0 on the zero line and the sink)
    const Real* pR; const Real* pT; const Real* pL; const Real* pB;
    int sR, sT, sL, sB;
    Real* wVC; Real* wVR; Real* wSX; Real* wSY;  // own publish targets (a sink without a patch)
    int sW;
    // edge slot
    bool e_col, e_corner, e_wcorner;
    int ek, e_il, e_jl;
    Real* e_pub;               // where the edge value is published
    const Real* e_line;        // its own line, at its own index
    const Real* e_perp;        // partial sum feeding the other direction
    Real ew[2 * P + 1];        // window coefficients on its own line
    const double (*K1)[kMaxP + 1];

    __device__ __forceinline__ Real K(int a, int b) const {
        return (Real)K1[kcan_a<P>(a, b)][kcan_b<P>(a, b)];
    }

    // Carve LDS, zero the padded lines, stage the element matrix.  The
    // caller syncs before setup_windows and before any LDS read.
    __device__ void setup(const SubDesc& d, Real* lds, const double (*K1_)[kMaxP + 1], int nt_max) {
        K1 = K1_;
        const int mx = d.mx, my = d.my, tid = threadIdx.x;
        const PatchLds L = patch_lds(mx, my, P, nt_max);
        VC = lds + L.vc; VR = lds + L.vr; SX = lds + L.sx; SY = lds + L.sy;
        GC = lds + L.gc + kMaxP;
        GR = lds + L.gr + kMaxP;
        CORN = lds + L.corner;
        TAB = lds + L.tab;
        Real* ZR = lds + L.zr;
        Real* KL = lds + L.kl;
        for (int i = L.gc + tid; i < L.kl; i += blockDim.x) lds[i] = Real(0);
        if (tid < (P + 1) * (P + 1)) KL[tid] = (Real)K1[tid / (P + 1)][tid % (P + 1)];
        const int np = mx * my;
        hasP = tid < np;
        ex = hasP ? tid % mx : 0;
        ey = hasP ? tid / mx : 0;
        const int t = hasP ? tid : 0;
        pR = (ex + 1 < mx) ? VC + (t + 1) : GC + ey * P;
        sR = (ex + 1 < mx) ? np : 1;
        pT = (ey + 1 < my) ? VR + (t + mx) : GR + ex * P;
        sT = (ey + 1 < my) ? np : 1;
        pL = (ex > 0) ? SX + (t - 1) : ZR;
        sL = (ex > 0) ? np : 0;
        pB = (ey > 0) ? SY + (t - mx) : ZR;
        sB = (ey > 0) ? np : 0;
        Real* SINK = lds + L.sink;
        wVC = hasP ? VC + tid : SINK;
        wVR = hasP ? VR + tid : SINK;
        wSX = hasP ? SX + tid : SINK;
        wSY = hasP ? SY + tid : SINK;
        sW = hasP ? np : 0;
        const int mxP = mx * P, myP = my * P;
        hasE = tid < mxP + myP + 1;
        e_col = tid <= myP;
        ek = hasE ? (e_col ? tid : tid - (myP + 1)) : 0;
        e_corner = hasE && e_col && ek == myP;
        e_wcorner = hasE && !e_col && ek == (mx - 1) * P;
        if (!hasE) {
            e_il = e_jl = 0;
            e_pub = SINK + kMaxP;
            e_line = ZR + P;        // reads ZR[0..2P] (zeros; never written)
            e_perp = ZR;
        } else if (e_col) {
            e_il = mxP;
            e_jl = ek;
            e_pub = GC + ek;
            e_line = GC + ek;
            const int eyk = ek / P;
            e_perp = e_corner ? CORN : SX + (ek - eyk * P) * np + (eyk * mx + (mx - 1));
        } else {
            e_il = ek;
            e_jl = myP;
            e_pub = GR + ek;
            e_line = GR + ek;
            const int exk = ek / P;
            e_perp = SY + (ek - exk * P) * np + ((my - 1) * mx + exk);
        }
    }

    // Per-thread window coefficients (after K is staged and synced).
    __device__ void setup_windows(const SubDesc& d, const Real* lds, int nt_max) {
        const PatchLds L = patch_lds(d.mx, d.my, P, nt_max);
        window_coeffs<Real, P>(ew, ek, e_col ? d.my : d.mx, lds + L.kl);
        if (!hasE) {
#pragma unroll
            for (int j = 0; j <= 2 * P; ++j) ew[j] = Real(0);
        }
    }

    // Publish the values other threads need: the a=0 column and b=0 row of
    // the patch, and the edge node (the corner is stored in both lines).
    __device__ __forceinline__ void publish(const Real (&p)[P][P], Real ep, int mx) {
#pragma unroll
        for (int b = 0; b < P; ++b) wVC[b * sW] = p[0][b];
#pragma unroll
        for (int a = 0; a < P; ++a) wVR[a * sW] = p[a][0];
        *e_pub = ep;
        if (e_corner) GR[mx * P] = ep;
    }

    // x-sum at (a, b) of this element (right vertex value pr = p(P, b)).
    __device__ __forceinline__ Real xsum(const Real (&p)[P][P], int a, int b, Real pr) const {
        Real s = K(a, P) * pr;
#pragma unroll
        for (int q = 0; q < P; ++q) s = fma(K(a, q), p[q][b], s);
        return s;
    }
    // y-sum at (a, b) of this element (top vertex value pt = p(a, P)).
    __device__ __forceinline__ Real ysum(const Real (&p)[P][P], int a, int b, Real pt) const {
        Real s = K(b, P) * pt;
#pragma unroll
        for (int q = 0; q < P; ++q) s = fma(K(b, q), p[a][q], s);
        return s;
    }

    // Edge node: sum along its own line (and the corner's x partial, written
    // by the row thread at the last top-row vertex).
    __device__ __forceinline__ Real edge_line_sum() const {
        Real w[2 * P + 1];
#pragma unroll
        for (int j = 0; j <= 2 * P; ++j) w[j] = e_line[j - P];
        Real s = Real(0);
#pragma unroll
        for (int j = 0; j <= 2 * P; ++j) s = fma(ew[j], w[j], s);
        if (e_wcorner) {
            Real c = Real(0);
#pragma unroll
            for (int q = 0; q <= P; ++q) c = fma(K(P, q), w[P + q], c);
            *CORN = c;
        }
        return s;
    }
};

// Coefficients of one patch.  Interior slots (a, b >= 1) lie on no
// subdomain side, so alpha = 1 and the interface data contribute nothing
// there; they only carry forcing when the sweep has a source term.
template <typename Real, int P, bool HAS_SRC>
struct PatchCoef {
    Real bX[P][P], bY[P][P];
    Real al[P][P];              // used on vertex-line slots only
    Real bbr[P][P], bbi[P][P];  // vertex-line slots, and all slots with a source
};

template <int P>
__host__ __device__ constexpr bool vline(int a, int b) { return a == 0 || b == 0; }

template <typename Real, int P, bool HAS_SRC>
__device__ void sweep_patch_item(const SweepArgs<Real>& A, const SubDesc& d, int item, Real* lds,
                                 double* red) {
    PatchCtx<Real, P> C;
    C.setup(d, lds, A.K1[P], A.nt_max);
    stage_tables(A, d, lds + patch_lds(d.mx, d.my, P, A.nt_max).tab);
    const int mx = d.mx, nxl = d.nxl;
    PatchCoef<Real, P, HAS_SRC> cf;
    Real p[P][P], pd[P][P], vr[P][P], vi[P][P];
    const int64_t base = d.node_off + (int64_t)(C.ey * P) * nxl + C.ex * P;
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
        for (int b = 0; b < P; ++b) {
            cf.bX[a][b] = cf.bY[a][b] = cf.al[a][b] = cf.bbr[a][b] = cf.bbi[a][b] = Real(0);
            p[a][b] = pd[a][b] = vr[a][b] = vi[a][b] = Real(0);
            if (C.hasP) {
                const int64_t n = base + (int64_t)b * nxl + a;
                cf.bX[a][b] = A.coef.betaX[n];
                cf.bY[a][b] = A.coef.betaY[n];
                if (vline<P>(a, b) || HAS_SRC) {
                    const double be = (double)A.coef.beta[n];
                    const double2 bb = assemble_b(A, d, C.ex * P + a, C.ey * P + b);
                    cf.bbr[a][b] = (Real)(be * bb.x);
                    cf.bbi[a][b] = (Real)(be * bb.y);
                }
                if (vline<P>(a, b)) cf.al[a][b] = A.coef.alpha[n];
            }
        }
    Slot<Real> e;
    slot_zero(e);
    if (C.hasE) slot_load(e, A, d, C.e_il, C.e_jl);
    __syncthreads();
    C.setup_windows(d, lds, A.nt_max);

    const Real sig = (Real)d.sigma;
    const int nt = d.nt;
    const Real* TAB = C.TAB;
    const double pd0c = d.pd0c, pd0s = d.pd0s;
    int it = 0;
    const int max_wh = d.max_wh > 0 ? d.max_wh : A.max_wh;
    const double tau = d.max_wh > 0 ? d.tau : A.tau;
    // warm start: the first WaveHoltz iteration starts from the current u
    const bool warm = A.warm != 0 || (d.flags & 1) != 0;
    WhStall stall;
    for (int m = 0; m < max_wh; ++m) {
        const Real k0 = TAB[2], kh0 = TAB[3];
        // p, pdot from u: read at the first iteration (warm start), after
        // that still in registers from the end of the previous iteration
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
            for (int b = 0; b < P; ++b) {
                if (m == 0) {
                    p[a][b] = Real(0);
                    pd[a][b] = Real(0);
                    if (warm && C.hasP) {
                        const double2 u = A.u[base + (int64_t)b * nxl + a];
                        p[a][b] = (Real)u.x;
                        pd[a][b] = (Real)(u.y * pd0c - u.x * pd0s);
                    }
                }
                vr[a][b] = k0 * p[a][b];
                vi[a][b] = kh0 * pd[a][b];
            }
        if (m == 0) {
            if (C.hasE) slot_init(e, A, d, warm, k0, kh0);
        } else {
            e.vr = k0 * e.p;
            e.vi = kh0 * e.pd;
        }

        for (int nu = 1; nu < nt; ++nu) {
            const Real c = TAB[4 * nu + 0], sv = TAB[4 * nu + 1];
            const Real k1 = TAB[4 * nu + 2], k2 = TAB[4 * nu + 3];
            // p^{nu} = p^{nu-1} + sigma pdot^{nu-1/2}; publish the vertex lines
#pragma unroll
            for (int a = 0; a < P; ++a)
#pragma unroll
                for (int b = 0; b < P; ++b) p[a][b] = fma(sig, pd[a][b], p[a][b]);
            e.p = fma(sig, e.pd, e.p);
            C.publish(p, e.p, mx);
            // own-data work while the writes drain: filter sum and forcing
            Real tv[P][P];
#pragma unroll
            for (int a = 0; a < P; ++a)
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    vr[a][b] = fma(k1, p[a][b], vr[a][b]);
                    if (vline<P>(a, b) || HAS_SRC)
                        tv[a][b] = fma(cf.bbi[a][b], sv, cf.bbr[a][b] * c);
                    else
                        tv[a][b] = Real(0);
                }
            e.vr = fma(k1, e.p, e.vr);
            __syncthreads();

            // neighbour reads first; own-element sums hide their latency, the
            // neighbour term is added last in every sum
            Real pr[P], pt[P], ew[2 * P + 1];
#pragma unroll
            for (int b = 0; b < P; ++b) pr[b] = C.pR[b * C.sR];
#pragma unroll
            for (int a = 0; a < P; ++a) pt[a] = C.pT[a * C.sT];
#pragma unroll
            for (int j = 0; j <= 2 * P; ++j) ew[j] = C.e_line[j - P];
            Real X[P][P], Y[P][P], sx[P], sy[P];
#pragma unroll
            for (int b = 0; b < P; ++b) {
                sx[b] = C.K(P, 0) * p[0][b];
#pragma unroll
                for (int q = 1; q < P; ++q) sx[b] = fma(C.K(P, q), p[q][b], sx[b]);
            }
#pragma unroll
            for (int a = 0; a < P; ++a) {
                sy[a] = C.K(P, 0) * p[a][0];
#pragma unroll
                for (int q = 1; q < P; ++q) sy[a] = fma(C.K(P, q), p[a][q], sy[a]);
            }
#pragma unroll
            for (int a = 0; a < P; ++a)
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    X[a][b] = C.K(a, 0) * p[0][b];
#pragma unroll
                    for (int q = 1; q < P; ++q) X[a][b] = fma(C.K(a, q), p[q][b], X[a][b]);
                    Y[a][b] = C.K(b, 0) * p[a][0];
#pragma unroll
                    for (int q = 1; q < P; ++q) Y[a][b] = fma(C.K(b, q), p[a][q], Y[a][b]);
                }
            // partial sums owed to the right / top neighbours' vertex lines
#pragma unroll
            for (int b = 0; b < P; ++b) C.wSX[b * C.sW] = fma(C.K(P, P), pr[b], sx[b]);
#pragma unroll
            for (int a = 0; a < P; ++a) C.wSY[a * C.sW] = fma(C.K(P, P), pt[a], sy[a]);
            Real eL = Real(0);
#pragma unroll
            for (int j = 0; j <= 2 * P; ++j) eL = fma(C.ew[j], ew[j], eL);
            if (C.e_wcorner) {
                Real cc = Real(0);
#pragma unroll
                for (int q = 0; q <= P; ++q) cc = fma(C.K(P, q), ew[P + q], cc);
                *C.CORN = cc;
            }
#pragma unroll
            for (int a = 0; a < P; ++a)
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    const Real Xf = fma(C.K(a, P), pr[b], X[a][b]);
                    const Real Yf = fma(C.K(b, P), pt[a], Y[a][b]);
                    Real t = fma(-cf.bX[a][b], Xf, tv[a][b]);
                    t = fma(-cf.bY[a][b], Yf, t);
                    if (vline<P>(a, b))
                        tv[a][b] = t;  // finished after the partials arrive
                    else
                        pd[a][b] += t;
                }
            __syncthreads();
            {
                Real pl[P], pbm[P];
#pragma unroll
                for (int b = 0; b < P; ++b) pl[b] = C.pL[b * C.sL];
#pragma unroll
                for (int a = 0; a < P; ++a) pbm[a] = C.pB[a * C.sB];
                const Real eP = *C.e_perp;
                // interior slots: filter sum of the new velocity
#pragma unroll
                for (int a = 0; a < P; ++a)
#pragma unroll
                    for (int b = 0; b < P; ++b)
                        if (!vline<P>(a, b)) vi[a][b] = fma(k2, pd[a][b], vi[a][b]);
#pragma unroll
                for (int b = 0; b < P; ++b) tv[0][b] = fma(-cf.bX[0][b], pl[b], tv[0][b]);
#pragma unroll
                for (int a = 1; a < P; ++a) tv[a][0] = fma(-cf.bY[a][0], pbm[a], tv[a][0]);
                tv[0][0] = fma(-cf.bY[0][0], pbm[0], tv[0][0]);
#pragma unroll
                for (int a = 0; a < P; ++a)
#pragma unroll
                    for (int b = 0; b < P; ++b)
                        if (vline<P>(a, b)) {
                            pd[a][b] = fma(cf.al[a][b], pd[a][b], tv[a][b]);
                            vi[a][b] = fma(k2, pd[a][b], vi[a][b]);
                        }
                const Real eX = C.e_col ? eP : eL;
                const Real eY = C.e_col ? eL : eP;
                Real t = fma(e.bbi, sv, e.bbr * c);
                t = fma(-e.bX, eX, t);
                t = fma(-e.bY, eY, t);
                e.pd = fma(e.al, e.pd, t);
                e.vi = fma(k2, e.pd, e.vi);
            }
        }

        double dsum = 0.0, nsum = 0.0;
        if (C.hasP) {
#pragma unroll
            for (int a = 0; a < P; ++a)
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    const int64_t n = base + (int64_t)b * nxl + a;
                    const double ur = d.two_over_nt * (double)vr[a][b];
                    const double ui = d.two_over_nt * (double)vi[a][b];
                    double orr = 0.0, oi = 0.0;
                    if (m > 0 || warm) {
                        const double2 o = A.u[n];
                        orr = o.x;
                        oi = o.y;
                    }
                    dsum += (ur - orr) * (ur - orr) + (ui - oi) * (ui - oi);
                    nsum += ur * ur + ui * ui;
                    A.u[n] = make_double2(ur, ui);
                    // start of the next iteration (the values a read of u gives)
                    p[a][b] = (Real)ur;
                    pd[a][b] = (Real)(ui * pd0c - ur * pd0s);
                }
        }
        if (C.hasE) {
            slot_finish(e, A, d, m > 0 || warm, dsum, nsum);
            const double ur = d.two_over_nt * (double)e.vr, ui = d.two_over_nt * (double)e.vi;
            e.p = (Real)ur;
            e.pd = (Real)(ui * pd0c - ur * pd0s);
        }
        block_sum2(dsum, nsum, red);
        it = m + 1;
        if (!(dsum == dsum)) break;  // non-finite iterate: stop, reported by the host
        if (wh_stop<Real>(tau, dsum, nsum, stall)) break;
    }
    __threadfence_block();
    __syncthreads();
    exchange(A, d);
    if (threadIdx.x == 0) A.wh_iters[item] = it;
}

template <typename Real, int P, int WG, bool HAS_SRC>
__global__ void __launch_bounds__(WG) sweep_patch_kernel(const SweepArgs<Real> A) {
    extern __shared__ double smem_d[];
    double* red = smem_d;                       // 2 * 16 doubles
    Real* lds = reinterpret_cast<Real*>(smem_d + 40);
    const int item = blockIdx.x;   // one workgroup per item (grid = n_items)
    if (item >= A.n_items) return;
    const SubDesc d = A.desc[item];   // loaded once: kept in registers across the stores below
    sweep_patch_item<Real, P, HAS_SRC>(A, d, item, lds, red);
}

// q = A p on stacked subdomain vectors with the patch routines of the
// sweep (same publish / own-sum / partial-sum sequence).
template <typename Real, int P, int WG>
__global__ void __launch_bounds__(WG) apply_patch_kernel(const SweepArgs<Real> A,
                                                         const Real* pin, Real* qout) {
    extern __shared__ double smem_d[];
    Real* lds = reinterpret_cast<Real*>(smem_d + 40);
    const SubDesc d = A.desc[blockIdx.x];
    PatchCtx<Real, P> C;
    C.setup(d, lds, A.K1[P], A.nt_max);
    const int mx = d.mx, nxl = d.nxl;
    const int64_t base = d.node_off + (int64_t)(C.ey * P) * nxl + C.ex * P;
    Real p[P][P];
    Real ep = Real(0);
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
        for (int b = 0; b < P; ++b) p[a][b] = C.hasP ? pin[base + (int64_t)b * nxl + a] : Real(0);
    if (C.hasE) ep = pin[d.node_off + (int64_t)C.e_jl * nxl + C.e_il];
    __syncthreads();
    C.setup_windows(d, lds, A.nt_max);
    C.publish(p, ep, mx);
    __syncthreads();
    Real X[P][P], Y[P][P];
    if (C.hasP) {
        Real pr[P], pt[P];
#pragma unroll
        for (int b = 0; b < P; ++b) pr[b] = C.pR[b * C.sR];
#pragma unroll
        for (int a = 0; a < P; ++a) pt[a] = C.pT[a * C.sT];
#pragma unroll
        for (int b = 0; b < P; ++b) C.wSX[b * C.sW] = C.xsum(p, P, b, pr[b]);
#pragma unroll
        for (int a = 0; a < P; ++a) C.wSY[a * C.sW] = C.ysum(p, a, P, pt[a]);
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
            for (int b = 0; b < P; ++b) {
                X[a][b] = C.xsum(p, a, b, pr[b]);
                Y[a][b] = C.ysum(p, a, b, pt[a]);
            }
    }
    Real eL = Real(0);
    if (C.hasE) eL = C.edge_line_sum();
    __syncthreads();
    const double* wx = A.w1d + d.w_off;
    const double* wy = wx + d.nxl;
    if (C.hasP) {
#pragma unroll
        for (int b = 0; b < P; ++b) X[0][b] += C.pL[b * C.sL];
#pragma unroll
        for (int a = 0; a < P; ++a) Y[a][0] += C.pB[a * C.sB];
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
            for (int b = 0; b < P; ++b) {
                const int il = C.ex * P + a, jl = C.ey * P + b;
                qout[base + (int64_t)b * nxl + a] =
                    (Real)(d.sx_ref * wy[jl]) * X[a][b] + (Real)(d.sy_ref * wx[il]) * Y[a][b];
            }
    }
    if (C.hasE) {
        const Real eP = *C.e_perp;
        const Real eX = C.e_col ? eP : eL;
        const Real eY = C.e_col ? eL : eP;
        qout[d.node_off + (int64_t)C.e_jl * nxl + C.e_il] =
            (Real)(d.sx_ref * wy[C.e_jl]) * eX + (Real)(d.sy_ref * wx[C.e_il]) * eY;
    }
}

// ---------------------------------------------------------------------------
// PATCH layout, one barrier per step
// ---------------------------------------------------------------------------
// Same ownership as above, but every thread publishes its whole P*P patch
// (structure-of-arrays, double-buffered by step parity) and computes the
// contributions of its left and bottom neighbour elements to its own vertex
// lines itself, so a step needs one barrier and one LDS round trip.  The hot
// loop is branch-free: missing neighbours read a zero column, threads without
// a patch or an edge node publish into unused columns / a sink.
//
// LDS (units of Real): PB[2][P*P][S] with S = WG + 64 (column WG..S-1 is a
// zero column, so S is a multiple of 64), GC[2][myP+1+2kMaxP],
// GR[2][mxP+1+2kMaxP], zero line, sink, K, tables.
struct Patch1Lds {
    int pb, gc, gr, zr, sink, kl, tab, total, S, lgc, lgr;
};

__host__ __device__ inline Patch1Lds patch1_lds(int mx, int my, int P, int WG, int nt_max) {
    Patch1Lds L;
    L.S = WG + 64;
    L.lgc = my * P + 1 + 2 * kMaxP;
    L.lgr = mx * P + 1 + 2 * kMaxP;
    L.pb = 0;
    L.gc = L.pb + 2 * P * P * L.S;
    L.gr = L.gc + 2 * L.lgc;
    L.zr = L.gr + 2 * L.lgr;
    L.sink = L.zr + 2 * kMaxP + 2;
    L.kl = L.sink + 2;
    L.tab = (L.kl + (kMaxP + 1) * (kMaxP + 1) + 3) & ~3;
    L.total = L.tab + 4 * nt_max;
    return L;
}

// Per-thread addressing of the one-barrier patch layout.  Every neighbour
// read is base[k * stride] in buffer (nu & 1), whose offset from buffer 0 is
// `boff` (the two buffers of PB and of each line differ in size).
template <typename Real, int P, int WG>
struct Patch1Ctx {
    Real* lds;
    int own;                        // own PB column
    int rB, rS, rO;                 // right neighbour's a=0 column: base, stride, buffer offset
    int tB, tS, tO;                 // top neighbour's b=0 row
    int lB, bB;                     // left / bottom neighbour PB columns (zero column if absent)
    Real kl, kb;                    // K[P][P] if the left / bottom element exists, else 0
    bool hasP, hasE, e_col, e_corner;
    int ek, e_il, e_jl;
    int pubB, pubO, pub2B, pub2O;   // edge publish (and corner copy into GR; sink otherwise)
    int lnB, lnO;                   // edge: own line (centre)
    int ppB, ppS, ppO;              // edge: perpendicular reads
    Real ew[2 * P + 1];
    const double (*K1)[kMaxP + 1];

    __device__ __forceinline__ Real K(int a, int b) const {
        return (Real)K1[kcan_a<P>(a, b)][kcan_b<P>(a, b)];
    }

    __device__ void setup(const SubDesc& d, Real* lds_, const double (*K1_)[kMaxP + 1],
                          int nt_max) {
        lds = lds_;
        K1 = K1_;
        const int mx = d.mx, my = d.my, tid = threadIdx.x;
        const Patch1Lds L = patch1_lds(mx, my, P, WG, nt_max);
        const int S = L.S, pbO = P * P * S;
        // zero both PB buffers' zero columns, the lines, the zero line
        for (int i = tid; i < 2 * P * P * 64; i += blockDim.x) {
            const int buf = i / (P * P * 64), r = i % (P * P * 64);
            lds[L.pb + buf * pbO + (r / 64) * S + WG + (r % 64)] = Real(0);
        }
        for (int i = L.gc + tid; i < L.kl; i += blockDim.x) lds[i] = Real(0);
        if (tid < (P + 1) * (P + 1)) lds[L.kl + tid] = (Real)K1[tid / (P + 1)][tid % (P + 1)];
        const int np = mx * my;
        hasP = tid < np;
        const int ex = hasP ? tid % mx : 0, ey = hasP ? tid / mx : 0;
        own = L.pb + tid;
        const int zc = L.pb + WG;   // zero column
        if (hasP && ex + 1 < mx) { rB = L.pb + tid + 1; rS = S; rO = pbO; }
        else if (hasP) { rB = L.gc + kMaxP + ey * P; rS = 1; rO = L.lgc; }
        else { rB = zc; rS = S; rO = pbO; }
        if (hasP && ey + 1 < my) { tB = L.pb + tid + mx; tS = P * S; tO = pbO; }
        else if (hasP) { tB = L.gr + kMaxP + ex * P; tS = 1; tO = L.lgr; }
        else { tB = zc; tS = P * S; tO = pbO; }
        lB = (hasP && ex > 0) ? L.pb + tid - 1 : zc;
        bB = (hasP && ey > 0) ? L.pb + tid - mx : zc;
        kl = (hasP && ex > 0) ? K(P, P) : Real(0);
        kb = (hasP && ey > 0) ? K(P, P) : Real(0);
        // edge slot
        const int mxP = mx * P, myP = my * P;
        hasE = tid < mxP + myP + 1;
        e_col = tid <= myP;
        ek = hasE ? (e_col ? tid : tid - (myP + 1)) : 0;
        e_corner = hasE && e_col && ek == myP;
        pub2B = L.sink;
        pub2O = 0;
        if (!hasE) {
            e_il = e_jl = 0;
            pubB = L.sink; pubO = 0;
            lnB = L.zr + kMaxP; lnO = 0;
            ppB = L.zr; ppS = 0; ppO = 0;
        } else if (e_col) {
            e_il = mxP;
            e_jl = ek;
            pubB = L.gc + kMaxP + ek; pubO = L.lgc;
            if (e_corner) {
                pub2B = L.gr + kMaxP + mxP;
                pub2O = L.lgr;
            }
            lnB = L.gc + kMaxP + ek; lnO = L.lgc;
            if (e_corner) {
                ppB = L.gr + kMaxP + (mx - 1) * P; ppS = 1; ppO = L.lgr;
            } else {
                const int eyk = ek / P, b = ek - eyk * P;
                ppB = L.pb + b * S + eyk * mx + (mx - 1); ppS = P * S; ppO = pbO;
            }
        } else {
            e_il = ek;
            e_jl = myP;
            pubB = L.gr + kMaxP + ek; pubO = L.lgr;
            lnB = L.gr + kMaxP + ek; lnO = L.lgr;
            const int exk = ek / P, a = ek - exk * P;
            ppB = L.pb + (a * P) * S + (my - 1) * mx + exk; ppS = S; ppO = pbO;
        }
    }

    __device__ void setup_windows(const SubDesc& d, int nt_max) {
        const Patch1Lds L = patch1_lds(d.mx, d.my, P, WG, nt_max);
        window_coeffs<Real, P>(ew, ek, e_col ? d.my : d.mx, lds + L.kl);
        if (!hasE) {
#pragma unroll
            for (int j = 0; j <= 2 * P; ++j) ew[j] = Real(0);
        }
    }
};

template <typename Real, int P, int WG, bool HAS_SRC>
__device__ void sweep_patch1_item(const SweepArgs<Real>& A, const SubDesc& d, int item, Real* lds,
                                  double* red) {
    Patch1Ctx<Real, P, WG> C;
    C.setup(d, lds, A.K1[P], A.nt_max);
    const Patch1Lds LL = patch1_lds(d.mx, d.my, P, WG, A.nt_max);
    const int S = LL.S, pbO = P * P * S;
    stage_tables(A, d, lds + LL.tab);
    const int nxl = d.nxl;
    PatchCoef<Real, P, HAS_SRC> cf;
    Real p[P][P], pd[P][P], vr[P][P], vi[P][P];
    const int ex = C.hasP ? threadIdx.x % d.mx : 0, ey = C.hasP ? threadIdx.x / d.mx : 0;
    const int64_t base = d.node_off + (int64_t)(ey * P) * nxl + ex * P;
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
        for (int b = 0; b < P; ++b) {
            cf.bX[a][b] = cf.bY[a][b] = cf.al[a][b] = cf.bbr[a][b] = cf.bbi[a][b] = Real(0);
            p[a][b] = pd[a][b] = vr[a][b] = vi[a][b] = Real(0);
            if (C.hasP) {
                const int64_t n = base + (int64_t)b * nxl + a;
                cf.bX[a][b] = A.coef.betaX[n];
                cf.bY[a][b] = A.coef.betaY[n];
                if (vline<P>(a, b) || HAS_SRC) {
                    const double be = (double)A.coef.beta[n];
                    const double2 bb = assemble_b(A, d, ex * P + a, ey * P + b);
                    cf.bbr[a][b] = (Real)(be * bb.x);
                    cf.bbi[a][b] = (Real)(be * bb.y);
                }
                if (vline<P>(a, b)) cf.al[a][b] = A.coef.alpha[n];
            }
        }
    Slot<Real> e;
    slot_zero(e);
    if (C.hasE) slot_load(e, A, d, C.e_il, C.e_jl);
    __syncthreads();
    C.setup_windows(d, A.nt_max);

    const Real sig = (Real)d.sigma;
    const int nt = d.nt;
    const Real* TAB = lds + LL.tab;
    const double pd0c = d.pd0c, pd0s = d.pd0s;
    const Real kPP = C.K(P, P);
    int it = 0;
    const int max_wh = d.max_wh > 0 ? d.max_wh : A.max_wh;
    const double tau = d.max_wh > 0 ? d.tau : A.tau;
    // warm start: the first WaveHoltz iteration starts from the current u
    const bool warm = A.warm != 0 || (d.flags & 1) != 0;
    WhStall stall;
    for (int m = 0; m < max_wh; ++m) {
        const Real k0 = TAB[2], kh0 = TAB[3];
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
            for (int b = 0; b < P; ++b) {
                if ((m > 0 || warm) && C.hasP) {
                    const double2 u = A.u[base + (int64_t)b * nxl + a];
                    p[a][b] = (Real)u.x;
                    pd[a][b] = (Real)(u.y * pd0c - u.x * pd0s);
                } else {
                    p[a][b] = Real(0);
                    pd[a][b] = Real(0);
                }
                vr[a][b] = k0 * p[a][b];
                vi[a][b] = kh0 * pd[a][b];
            }
        if (C.hasE) slot_init(e, A, d, m > 0 || warm, k0, kh0);

        for (int nu = 1; nu < nt; ++nu) {
            const int par = nu & 1;
            const Real c = TAB[4 * nu + 0], sv = TAB[4 * nu + 1];
            const Real k1 = TAB[4 * nu + 2], k2 = TAB[4 * nu + 3];
            // p^{nu} = p^{nu-1} + sigma pdot^{nu-1/2}; publish the patch
            Real* pbuf = lds + C.own + par * pbO;
#pragma unroll
            for (int a = 0; a < P; ++a)
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    p[a][b] = fma(sig, pd[a][b], p[a][b]);
                    pbuf[(a * P + b) * S] = p[a][b];
                }
            e.p = fma(sig, e.pd, e.p);
            lds[C.pubB + par * C.pubO] = e.p;
            lds[C.pub2B + par * C.pub2O] = e.p;
            // own-data work while the writes drain: filter sum and forcing
            Real tf[P][P];
#pragma unroll
            for (int a = 0; a < P; ++a)
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    vr[a][b] = fma(k1, p[a][b], vr[a][b]);
                    if (vline<P>(a, b) || HAS_SRC)
                        tf[a][b] = fma(cf.bbi[a][b], sv, cf.bbr[a][b] * c);
                    else
                        tf[a][b] = Real(0);
                }
            e.vr = fma(k1, e.p, e.vr);
            __syncthreads();

            // neighbour values (right column, top row, left and bottom patches)
            Real pr[P], pt[P], pl[P][P], pb[P][P];
            {
                const Real* r = lds + C.rB + par * C.rO;
                const Real* t = lds + C.tB + par * C.tO;
                const Real* l = lds + C.lB + par * pbO;
                const Real* bo = lds + C.bB + par * pbO;
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    pr[q] = r[q * C.rS];
                    pt[q] = t[q * C.tS];
                }
#pragma unroll
                for (int a = 0; a < P; ++a)
#pragma unroll
                    for (int b = 0; b < P; ++b) {
                        pl[a][b] = l[(a * P + b) * S];
                        pb[a][b] = bo[(a * P + b) * S];
                    }
            }
            Real ew[2 * P + 1], epp[P];
            {
                const Real* ln = lds + C.lnB + C.lnO * par;
                const Real* pp = lds + C.ppB + C.ppO * par;
#pragma unroll
                for (int j = 0; j <= 2 * P; ++j) ew[j] = ln[j - P];
#pragma unroll
                for (int q = 0; q < P; ++q) epp[q] = pp[q * C.ppS];
            }
            // own-element terms first (they hide the LDS latency), neighbour
            // terms last
            Real X[P][P], Y[P][P];
#pragma unroll
            for (int a = 0; a < P; ++a)
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    X[a][b] = C.K(a, 0) * p[0][b];
#pragma unroll
                    for (int q = 1; q < P; ++q) X[a][b] = fma(C.K(a, q), p[q][b], X[a][b]);
                    Y[a][b] = C.K(b, 0) * p[a][0];
#pragma unroll
                    for (int q = 1; q < P; ++q) Y[a][b] = fma(C.K(b, q), p[a][q], Y[a][b]);
                    if (a == 0) X[a][b] = fma(C.kl, p[0][b], X[a][b]);
                    if (b == 0) Y[a][b] = fma(C.kb, p[a][0], Y[a][b]);
                }
#pragma unroll
            for (int a = 0; a < P; ++a)
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    Real Xf = fma(C.K(a, P), pr[b], X[a][b]);
                    Real Yf = fma(C.K(b, P), pt[a], Y[a][b]);
                    if (a == 0) {  // left element's share of this vertex-line node
#pragma unroll
                        for (int q = 0; q < P; ++q) Xf = fma(C.K(P, q), pl[q][b], Xf);
                    }
                    if (b == 0) {  // bottom element's share
#pragma unroll
                        for (int q = 0; q < P; ++q) Yf = fma(C.K(P, q), pb[a][q], Yf);
                    }
                    Real tt = fma(-cf.bX[a][b], Xf, tf[a][b]);
                    tt = fma(-cf.bY[a][b], Yf, tt);
                    if (vline<P>(a, b))
                        pd[a][b] = fma(cf.al[a][b], pd[a][b], tt);
                    else
                        pd[a][b] += tt;
                    vi[a][b] = fma(k2, pd[a][b], vi[a][b]);
                }
            // edge node: window on its own line, and the perpendicular element
            {
                Real sL = Real(0);
#pragma unroll
                for (int j = 0; j <= 2 * P; ++j) sL = fma(C.ew[j], ew[j], sL);
                Real sP = kPP * e.p;
#pragma unroll
                for (int q = 0; q < P; ++q) sP = fma(C.K(P, q), epp[q], sP);
                const Real eX = C.e_col ? sP : sL;
                const Real eY = C.e_col ? sL : sP;
                Real t = fma(e.bbi, sv, e.bbr * c);
                t = fma(-e.bX, eX, t);
                t = fma(-e.bY, eY, t);
                e.pd = fma(e.al, e.pd, t);
                e.vi = fma(k2, e.pd, e.vi);
            }
        }

        double dsum = 0.0, nsum = 0.0;
        if (C.hasP) {
#pragma unroll
            for (int a = 0; a < P; ++a)
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    const int64_t n = base + (int64_t)b * nxl + a;
                    const double ur = d.two_over_nt * (double)vr[a][b];
                    const double ui = d.two_over_nt * (double)vi[a][b];
                    double orr = 0.0, oi = 0.0;
                    if (m > 0 || warm) {
                        const double2 o = A.u[n];
                        orr = o.x;
                        oi = o.y;
                    }
                    dsum += (ur - orr) * (ur - orr) + (ui - oi) * (ui - oi);
                    nsum += ur * ur + ui * ui;
                    A.u[n] = make_double2(ur, ui);
                }
        }
        if (C.hasE) slot_finish(e, A, d, m > 0 || warm, dsum, nsum);
        block_sum2(dsum, nsum, red);
        it = m + 1;
        if (!(dsum == dsum)) break;
        if (wh_stop<Real>(tau, dsum, nsum, stall)) break;
    }
    __threadfence_block();
    __syncthreads();
    exchange(A, d);
    if (threadIdx.x == 0) A.wh_iters[item] = it;
}

template <typename Real, int P, int WG, bool HAS_SRC>
__global__ void __launch_bounds__(WG) sweep_patch1_kernel(const SweepArgs<Real> A) {
    extern __shared__ double smem_d[];
    double* red = smem_d;
    Real* lds = reinterpret_cast<Real*>(smem_d + 40);
    const int item = blockIdx.x;   // one workgroup per item (grid = n_items)
    if (item >= A.n_items) return;
    const SubDesc d = A.desc[item];   // loaded once: kept in registers across the stores below
    sweep_patch1_item<Real, P, WG, HAS_SRC>(A, d, item, lds, red);
}

// q = A p with the one-barrier patch routines (test path).
template <typename Real, int P, int WG>
__global__ void __launch_bounds__(WG) apply_patch1_kernel(const SweepArgs<Real> A,
                                                          const Real* pin, Real* qout) {
    extern __shared__ double smem_d[];
    Real* lds = reinterpret_cast<Real*>(smem_d + 40);
    const SubDesc d = A.desc[blockIdx.x];
    Patch1Ctx<Real, P, WG> C;
    C.setup(d, lds, A.K1[P], A.nt_max);
    const Patch1Lds LL = patch1_lds(d.mx, d.my, P, WG, A.nt_max);
    const int S = LL.S;
    const int nxl = d.nxl;
    const int ex = C.hasP ? threadIdx.x % d.mx : 0, ey = C.hasP ? threadIdx.x / d.mx : 0;
    const int64_t base = d.node_off + (int64_t)(ey * P) * nxl + ex * P;
    Real p[P][P];
    Real ep = Real(0);
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
        for (int b = 0; b < P; ++b) p[a][b] = C.hasP ? pin[base + (int64_t)b * nxl + a] : Real(0);
    if (C.hasE) ep = pin[d.node_off + (int64_t)C.e_jl * nxl + C.e_il];
    __syncthreads();
    C.setup_windows(d, A.nt_max);
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
        for (int b = 0; b < P; ++b) lds[C.own + (a * P + b) * S] = p[a][b];
    lds[C.pubB] = ep;
    lds[C.pub2B] = ep;
    __syncthreads();
    const double* wx = A.w1d + d.w_off;
    const double* wy = wx + d.nxl;
    const Real* r = lds + C.rB;
    const Real* t = lds + C.tB;
    const Real* l = lds + C.lB;
    const Real* bo = lds + C.bB;
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
        for (int b = 0; b < P; ++b) {
            Real X = C.K(a, P) * r[b * C.rS];
#pragma unroll
            for (int q = 0; q < P; ++q) X = fma(C.K(a, q), p[q][b], X);
            Real Y = C.K(b, P) * t[a * C.tS];
#pragma unroll
            for (int q = 0; q < P; ++q) Y = fma(C.K(b, q), p[a][q], Y);
            if (a == 0) {
                X = fma(C.kl, p[0][b], X);
#pragma unroll
                for (int q = 0; q < P; ++q) X = fma(C.K(P, q), l[(q * P + b) * S], X);
            }
            if (b == 0) {
                Y = fma(C.kb, p[a][0], Y);
#pragma unroll
                for (int q = 0; q < P; ++q) Y = fma(C.K(P, q), bo[(a * P + q) * S], Y);
            }
            if (C.hasP) {
                const int il = ex * P + a, jl = ey * P + b;
                qout[base + (int64_t)b * nxl + a] =
                    (Real)(d.sx_ref * wy[jl]) * X + (Real)(d.sy_ref * wx[il]) * Y;
            }
        }
    if (C.hasE) {
        Real sL = Real(0);
#pragma unroll
        for (int j = 0; j <= 2 * P; ++j) sL = fma(C.ew[j], lds[C.lnB + j - P], sL);
        Real sP = C.K(P, P) * ep;
#pragma unroll
        for (int q = 0; q < P; ++q) sP = fma(C.K(P, q), lds[C.ppB + q * C.ppS], sP);
        const Real eX = C.e_col ? sP : sL;
        const Real eY = C.e_col ? sL : sP;
        qout[d.node_off + (int64_t)C.e_jl * nxl + C.e_il] =
            (Real)(d.sx_ref * wy[C.e_jl]) * eX + (Real)(d.sy_ref * wx[C.e_il]) * eY;
    }
}

// ---------------------------------------------------------------------------
// NODE layout (one DOF per thread)
// ---------------------------------------------------------------------------

// Padded LDS grid: rows of nxl + G words (kMaxP zeros on the left, the rest
// on the right) x (nyl + 2kMaxP) rows per buffer, two buffers, then the
// element matrix and the per-step tables.  G = 256 B / word size: a row
// stride equal to nxl modulo G gives consecutive lanes (consecutive nodes,
// across row ends too) consecutive LDS banks in every stencil tap.
__host__ __device__ inline int node_stride(int nxl, int rs) { return nxl + 256 / rs; }
__host__ __device__ inline int node_buf(int nxl, int nyl, int rs) {
    return node_stride(nxl, rs) * (nyl + 2 * kMaxP);
}
__host__ __device__ inline int node_tab_off(int nxl, int nyl, int rs) {
    return (2 * node_buf(nxl, nyl, rs) + (kMaxP + 1) * (kMaxP + 1) + 3) & ~3;
}

template <typename Real, int P>
struct NodeCtx {
    bool has;
    int il, jl, stride, pidx;
    Real* buf0; Real* buf1; const Real* TAB;
    Real wxk[2 * P + 1], wyk[2 * P + 1];

    __device__ void setup(const SubDesc& d, Real* lds, const double (*K1)[kMaxP + 1]) {
        const int nxl = d.nxl, nyl = d.nyl, tid = threadIdx.x;
        const int nb = node_buf(nxl, nyl, (int)sizeof(Real));
        buf0 = lds;
        buf1 = lds + nb;
        Real* kl = lds + 2 * nb;
        TAB = lds + node_tab_off(nxl, nyl, (int)sizeof(Real));
        for (int i = tid; i < 2 * nb; i += blockDim.x) lds[i] = Real(0);
        if (tid < (P + 1) * (P + 1)) kl[tid] = (Real)K1[tid / (P + 1)][tid % (P + 1)];
        __syncthreads();
        has = tid < nxl * nyl;
        il = has ? tid % nxl : 0;
        jl = has ? tid / nxl : 0;
        stride = node_stride(nxl, (int)sizeof(Real));
        pidx = (jl + kMaxP) * stride + il + kMaxP;
        window_coeffs<Real, P>(wxk, il, d.mx, kl);
        window_coeffs<Real, P>(wyk, jl, d.my, kl);
        __syncthreads();
    }

    __device__ __forceinline__ void sums(const Real* buf, Real& X, Real& Y) const {
        Real sx = Real(0), sy = Real(0);
#pragma unroll
        for (int j = 0; j <= 2 * P; ++j) {
            sx = fma(wxk[j], buf[pidx + j - P], sx);
            sy = fma(wyk[j], buf[pidx + (j - P) * stride], sy);
        }
        X = sx;
        Y = sy;
    }
};

template <typename Real, int P>
__device__ void sweep_node_item(const SweepArgs<Real>& A, const SubDesc& d, int item, Real* lds,
                                double* red) {
    NodeCtx<Real, P> C;
    C.setup(d, lds, A.K1[P]);
    stage_tables(A, d, lds + node_tab_off(d.nxl, d.nyl, (int)sizeof(Real)));
    Slot<Real> s;
    slot_zero(s);
    if (C.has) slot_load(s, A, d, C.il, C.jl);
    __syncthreads();
    const Real sig = (Real)d.sigma;
    const int nt = d.nt;
    const Real* TAB = C.TAB;
    int it = 0;
    const int max_wh = d.max_wh > 0 ? d.max_wh : A.max_wh;
    const double tau = d.max_wh > 0 ? d.tau : A.tau;
    // warm start: the first WaveHoltz iteration starts from the current u
    const bool warm = A.warm != 0 || (d.flags & 1) != 0;
    WhStall stall;
    for (int m = 0; m < max_wh; ++m) {
        if (C.has) slot_init(s, A, d, m > 0 || warm, TAB[2], TAB[3]);
        for (int nu = 1; nu < nt; ++nu) {
            Real* buf = (nu & 1) ? C.buf1 : C.buf0;
            const Real c = TAB[4 * nu + 0], sv = TAB[4 * nu + 1];
            const Real k1 = TAB[4 * nu + 2], k2 = TAB[4 * nu + 3];
            if (C.has) {
                s.p = fma(sig, s.pd, s.p);
                buf[C.pidx] = s.p;
            }
            __syncthreads();
            if (C.has) {
                Real X, Y;
                C.sums(buf, X, Y);
                slot_step(s, X, Y, c, sv, k1, k2);
            }
        }
        double dsum = 0.0, nsum = 0.0;
        if (C.has) slot_finish(s, A, d, m > 0 || warm, dsum, nsum);
        block_sum2(dsum, nsum, red);
        it = m + 1;
        if (!(dsum == dsum)) break;
        if (wh_stop<Real>(tau, dsum, nsum, stall)) break;
    }
    __threadfence_block();
    __syncthreads();
    exchange(A, d);
    if (threadIdx.x == 0) A.wh_iters[item] = it;
}

template <typename Real, int P>
__global__ void __launch_bounds__(kMaxWG) sweep_node_kernel(const SweepArgs<Real> A) {
    extern __shared__ double smem_d[];
    double* red = smem_d;
    Real* lds = reinterpret_cast<Real*>(smem_d + 40);
    const int item = blockIdx.x;   // one workgroup per item (grid = n_items)
    if (item >= A.n_items) return;
    const SubDesc d = A.desc[item];   // loaded once: kept in registers across the stores below
    sweep_node_item<Real, P>(A, d, item, lds, red);
}

template <typename Real, int P>
__global__ void __launch_bounds__(kMaxWG) apply_node_kernel(const SweepArgs<Real> A,
                                                            const Real* pin, Real* qout) {
    extern __shared__ double smem_d[];
    Real* lds = reinterpret_cast<Real*>(smem_d + 40);
    const SubDesc d = A.desc[blockIdx.x];
    NodeCtx<Real, P> C;
    C.setup(d, lds, A.K1[P]);
    if (C.has) C.buf0[C.pidx] = pin[d.node_off + (int64_t)C.jl * d.nxl + C.il];
    __syncthreads();
    if (C.has) {
        Real X, Y;
        C.sums(C.buf0, X, Y);
        const double* wx = A.w1d + d.w_off;
        const double* wy = wx + d.nxl;
        qout[d.node_off + (int64_t)C.jl * d.nxl + C.il] =
            (Real)(d.sx_ref * wy[C.jl]) * X + (Real)(d.sy_ref * wx[C.il]) * Y;
    }
}


// ---------------------------------------------------------------------------
// STREAM layout (subdomains larger than one CU's LDS + register file)
// ---------------------------------------------------------------------------
// The workgroup strides over the subdomain's nodes (thread t: nodes t,
// t + WG, ...).  p lives in two zero-padded grids in device memory
// (double-buffered: one barrier per step), pdot and the filter sums in
// node-indexed arrays read and written once per step, so every step moves
// O(1) words per node through L2 / HBM.  The arithmetic per node is the
// NODE layout's, in the same order.

// LDS (after 40 doubles for reductions): window table (kMaxP+2) x
// (2 kMaxP+1), reference element matrix, per-step tables.
constexpr int kStreamWT = (kMaxP + 2) * (2 * kMaxP + 1);
// Workgroup bound: two waves per SIMD leave 256 registers per lane for the
// column windows, the X neighbours in flight and the state addresses.
constexpr int kStreamWG = 512;
constexpr int kStreamTab = (kStreamWT + (kMaxP + 1) * (kMaxP + 1) + 3) & ~3;

// Window class of local node k on a line of nl nodes: 1..P-1 element
// interior offset, 0 interior vertex (two elements), P first node, P+1 last.
template <int P>
__device__ __forceinline__ int stream_class(int k, int nl) {
    return k == 0 ? P : (k == nl - 1 ? P + 1 : k % P);
}

template <typename Real, int P>
__device__ __forceinline__ void stream_tables(Real* lds, const double (*K1)[kMaxP + 1]) {
    constexpr int W = 2 * P + 1;
    Real* KL = lds + kStreamWT;
    const int tid = threadIdx.x;
    if (tid < (P + 1) * (P + 1)) KL[tid] = (Real)K1[tid / (P + 1)][tid % (P + 1)];
    __syncthreads();
    if (tid < P + 2) {
        // representative node of each class: (node, elements on the line)
        const int k = tid == P ? 0 : (tid == P + 1 ? P : (tid == 0 ? P : tid));
        const int nel = tid == 0 ? 2 : 1;
        Real w[W];
        window_coeffs<Real, P>(w, k, nel, KL);
#pragma unroll
        for (int j = 0; j < W; ++j) lds[tid * W + j] = w[j];
    }
}

// Cross-lane read of a value held by another lane of the wave (lane index
// taken modulo 64).
__device__ __forceinline__ double shfl_real(double v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ float shfl_real(float v, int src) { return __shfl(v, src, 64); }

// Work split of the STREAM step loop: wave w takes column group w % CG and
// row segment w / CG.  A column group spans 64 lanes over columns
// g*(64-2P) - P + lane; the P lanes at each end only supply neighbour
// values for the X windows (by cross-lane reads), the others own their
// column's nodes in the segment and walk up it with the Y window in
// registers.
template <typename Real, int P>
struct StreamGeom {
    int lane, i, ic, pcol, j0, j1;
    bool active, colv, own;
    bool side_col;   // every node of this lane's column reads its side record
    Real wx[2 * P + 1];

    // K workgroups share the subdomain; this is number k of them: the waves of
    // all K are numbered consecutively and split the same way.
    __device__ void setup(int nxl, int nyl, const Real* WT, int K = 1, int k = 0) {
        constexpr int OW = 64 - 2 * P;
        const int tid = threadIdx.x, nw1 = blockDim.x >> 6;
        const int wave = k * nw1 + (tid >> 6), nwaves = K * nw1;
        lane = tid & 63;
        const int CG = (nxl + OW - 1) / OW;
        const int RS = nwaves / CG;
        const int g = wave % CG, r = wave / CG;
        const int RL = RS > 0 ? (nyl + RS - 1) / RS : 0;
        j0 = r * RL;
        j1 = min(nyl, j0 + RL);
        active = r < RS && j0 < j1;
        if (!active) j0 = j1 = 0;
        i = g * OW - P + lane;
        ic = min(max(i, 0), nxl - 1);
        colv = i >= -kMaxP && i < nxl + kMaxP;
        own = active && lane >= P && lane < 64 - P && i >= 0 && i < nxl;
        pcol = colv ? i + kMaxP : 0;
        const Real* w = WT + stream_class<P>(own ? i : 1, nxl) * (2 * P + 1);
#pragma unroll
        for (int k = 0; k <= 2 * P; ++k) wx[k] = w[k];
    }
};

// Rows of the STREAM step loop kept in flight per wave (loads issued this
// many rows ahead of their use, so each wave has several rows of memory
// traffic outstanding).
template <typename Real>
constexpr int stream_ahead() { return sizeof(Real) == 8 ? 2 : 4; }

// STREAM workspace per node, in three planes: the state triple {pd, vr, vi}
// (read and written every step), the coefficient pair {betaX, betaY} (read
// every step) and the side triple {alpha, beta Re b, beta Im b}.  The side
// triple differs from {1, 0, 0} only on the subdomain's sides (H != 0
// there; the interface data enter b there) and, in sweeps with a source,
// wherever the source is; every other node reads one shared record
// {1, 0, 0} that the store keeps after the last side triple, so a step
// moves 10 words per node: p in and out, the state triple in and out, the
// pair in.
template <typename Real>
struct alignas(4 * sizeof(Real)) Quad {
    Real a, b, c, d;
};
template <typename Real>
struct Triple {
    Real a, b, c;
};
template <typename Real>
struct alignas(2 * sizeof(Real)) Pair {
    Real a, b;
};

// Planes of the STREAM workspace of a launch (see above).
template <typename Real>
struct StreamPlanes {
    Real* st;          // state triples, 3 per node
    const Real* cf;    // coefficient pairs, 2 per node
    const Real* sd;    // side triples, 3 per node
    const Real* sd1;   // the shared record {1, 0, 0}
};

// One row's loads of one lane: p entering the Y window (row j + P) and the
// node records at row j.  The loads are unconditional (addresses clamped to
// the segment and the grid, values of lanes or rows outside selected away,
// nodes off the sides pointed at the shared record), so no branch separates
// a load from its use and the wait counts let the rows ahead stay in
// flight.
template <typename Real>
struct StreamRow {
    Real pn;
    Triple<Real> st;
    Pair<Real> cf;
    Triple<Real> sd;
};

template <typename Real, int P>
__device__ __forceinline__ void stream_fetch(StreamRow<Real>& r, const StreamGeom<Real, P>& G,
                                             const Real* cur, int stride, int j, int nxl, int nyl,
                                             const StreamPlanes<Real>& N) {
    const bool inrow = j < G.j1;
    const int jc = inrow ? j : G.j1 - 1;
    const Real pn = cur[(jc + P + kMaxP) * stride + G.pcol];
    r.pn = (G.colv && inrow) ? pn : Real(0);
    const size_t n = (size_t)(jc * nxl + G.ic);
    r.st = *reinterpret_cast<const Triple<Real>*>(N.st + 3 * n);
    r.cf = *reinterpret_cast<const Pair<Real>*>(N.cf + 2 * n);
    const bool side = G.side_col || jc == 0 || jc == nyl - 1;
    r.sd = *reinterpret_cast<const Triple<Real>*>(side ? N.sd + 3 * n : N.sd1);
}

// One step of the STREAM layout for the column segment of this lane: walk
// up the rows with the Y window in registers, X neighbours from the lanes
// beside, loads issued stream_ahead rows early.  The body has no branch
// around a load (only the stores are predicated), so the waits keep the
// rows ahead in flight.  LAST: the step that ends a WaveHoltz iteration
// writes u = (2/N_t) v and accumulates the fixed-point residual instead.
template <typename Real, int P, bool LAST>
__device__ __forceinline__ void stream_rows(const StreamGeom<Real, P>& G, const Real* cur, Real* nxt,
                                            int stride, int nxl, int nyl,
                                            const StreamPlanes<Real>& N,
                                            const Real* WT,
                                            const Quad<Real> tb, Real sig, const SweepArgs<Real>& A,
                                            const SubDesc& d, bool has_old, double& dsum,
                                            double& nsum) {
    constexpr int W = 2 * P + 1;
    constexpr int kAhead = stream_ahead<Real>();
    Real win[W];
    win[0] = Real(0);
#pragma unroll
    for (int k = 0; k < 2 * P; ++k) {
        const Real v = cur[(G.j0 - P + k + kMaxP) * stride + G.pcol];
        win[k + 1] = G.colv ? v : Real(0);
    }
    StreamRow<Real> R[kAhead];
#pragma unroll
    for (int q = 0; q < kAhead; ++q)
        stream_fetch(R[q], G, cur, stride, G.j0 + q, nxl, nyl, N);
    for (int jb = G.j0; jb < G.j1; jb += kAhead) {
#pragma unroll
        for (int q = 0; q < kAhead; ++q) {
            const int j = jb + q;
            const StreamRow<Real> r = R[q];
            stream_fetch(R[q], G, cur, stride, j + kAhead, nxl, nyl, N);
#pragma unroll
            for (int k = 0; k < 2 * P; ++k) win[k] = win[k + 1];
            win[2 * P] = r.pn;
            const Real p = win[P];
            const Real* wy = WT + stream_class<P>(min(j, nyl - 1), nyl) * W;
            Real X = Real(0), Y = Real(0);
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const Real nb = k == P ? p : shfl_real(p, G.lane - P + k);
                X = fma(G.wx[k], nb, X);
                Y = fma(wy[k], win[k], Y);
            }
            Real t = r.sd.b * tb.a;
            t = fma(r.sd.c, tb.b, t);
            t = fma(-r.cf.a, X, t);
            t = fma(-r.cf.b, Y, t);
            const Real pd = fma(r.sd.a, r.st.a, t);
            const Real vr = fma(tb.c, p, r.st.b);
            const Real vi = fma(tb.d, pd, r.st.c);
            const bool put = G.own && j < G.j1;
            const int n = j * nxl + G.i;
            if (!LAST) {
                if (put) {
                    *reinterpret_cast<Triple<Real>*>(N.st + 3 * (size_t)n) =
                        Triple<Real>{pd, vr, vi};
                    nxt[(j + kMaxP) * stride + G.pcol] = fma(sig, pd, p);
                }
            } else if (put) {
                // u_new = (2/N_t) v (eq. (7)); fixed-point residual sums
                const double ur = d.two_over_nt * (double)vr;
                const double ui = d.two_over_nt * (double)vi;
                double orr = 0.0, oi = 0.0;
                if (has_old) {
                    const double2 o = A.u[d.node_off + n];
                    orr = o.x;
                    oi = o.y;
                }
                dsum += (ur - orr) * (ur - orr) + (ui - oi) * (ui - oi);
                nsum += ur * ur + ui * ui;
                A.u[d.node_off + n] = make_double2(ur, ui);
            }
        }
    }
}

// Barrier of the K workgroups that share one STREAM subdomain.  They run on
// one XCD (the launch places them so and checks it), whose L2 all their CUs
// share: each wave waits for its own stores to reach L2, one thread per
// workgroup counts itself in with an L2 atomic and polls until all K have
// arrived (bounded: after kXBarSpins polls, or when any workgroup of the
// launch gave up, it sets the launch's abort flag and returns false), then
// drops the CU's L1 lines so that the next loads see what the other
// workgroups wrote.  With K = 1 it is a workgroup barrier.
constexpr int kXBarSpins = 1 << 20;

struct XBar {
    int* cnt;      // arrivals at this item's barriers
    int* abort;    // launch-wide abort flag
    double* part;  // 2 K doubles: per-workgroup partial sums
    int* flag;     // LDS: this workgroup's outcome of the last barrier
    int K, k, epoch;
};

__device__ __forceinline__ bool xbar_sync(XBar& b) {
    if (b.K == 1) {
        __syncthreads();
        return true;
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    b.epoch += 1;
    if (threadIdx.x == 0) {
        atomicAdd(b.cnt, 1);
        const int target = b.epoch * b.K;
        int ok = 1;
        for (int spin = 0; atomicAdd(b.cnt, 0) < target; ++spin) {
            if (spin >= kXBarSpins || atomicAdd(b.abort, 0) != 0) {
                atomicExch(b.abort, 1);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        asm volatile("buffer_inv sc0" ::: "memory");
        *b.flag = ok;
    }
    __syncthreads();
    return *b.flag != 0;
}

// Value another workgroup of the item wrote, read where the barrier's
// atomics are performed (L2): a plain load of a workgroup-uniform address
// may be served by the scalar cache, which the barrier does not invalidate.
__device__ __forceinline__ double xbar_read(double* p) { return atomicAdd(p, 0.0); }

// Sum of the K workgroups' partial sums (a, b) in a fixed order, the same
// in every workgroup (thread 0 reads them and passes the sums on through
// LDS); false if the barrier gave up.
__device__ __forceinline__ bool xbar_sum2(XBar& x, double& a, double& b, double* sh) {
    if (x.K == 1) return true;
    if (threadIdx.x == 0) {
        x.part[2 * x.k] = a;
        x.part[2 * x.k + 1] = b;
    }
    if (!xbar_sync(x)) return false;
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int j = 0; j < x.K; ++j) {
            sa += xbar_read(x.part + 2 * j);
            sb += xbar_read(x.part + 2 * j + 1);
        }
        sh[0] = sa;
        sh[1] = sb;
    }
    __syncthreads();
    a = sh[0];
    b = sh[1];
    __syncthreads();
    return true;
}

__device__ __forceinline__ bool xb_sync_ok(XBar& x) { return xbar_sync(x); }

template <typename Real, int P>
__device__ void sweep_stream_item(const SweepArgs<Real>& A, const SubDesc& d, int item, Real* lds,
                                  double* red, XBar& xb) {
    constexpr int W = 2 * P + 1;
    const int nxl = d.nxl, nyl = d.nyl, bd = xb.K * (int)blockDim.x;
    const int tid = xb.k * (int)blockDim.x + (int)threadIdx.x;  // over the K workgroups
    const int nloc = nxl * nyl, stride = nxl + 2 * kMaxP;
    const int di = bd % nxl, dj = bd / nxl;
    stream_tables<Real, P>(lds, A.K1[P]);
    stage_tables(A, d, lds + kStreamTab);
    const Real* WT = lds;
    const Real* TAB = lds + kStreamTab;
    Real* p0 = A.ws_p + d.ws_off;
    Real* p1 = p0 + stream_pad_nodes(nxl, nyl);
    const size_t cap = (size_t)A.ws_stride;
    Real* NSt = A.ws_s + 3 * (size_t)d.node_off;
    Real* NCf = A.ws_s + 3 * cap + 2 * (size_t)d.node_off;
    Real* NSd = A.ws_s + 5 * cap + 3 * (size_t)d.node_off;
    const StreamPlanes<Real> N{NSt, NCf, NSd, A.ws_s + kStreamRecord * cap};
    // interior nodes carry forcing only in sweeps with a source
    const bool all_sides = A.Fre != nullptr && A.src != 0.0;
    // the coefficient pair, and alpha with beta * b (eq. (4) right-hand side
    // with the interface data) in the side triple
    {
        int il = tid % nxl, jl = tid / nxl;
        for (int n = tid; n < nloc; n += bd) {
            const double be = (double)A.coef.beta[d.node_off + n];
            const double2 b = assemble_b(A, d, il, jl);
            *reinterpret_cast<Pair<Real>*>(NCf + 2 * (size_t)n) =
                Pair<Real>{A.coef.betaX[d.node_off + n], A.coef.betaY[d.node_off + n]};
            *reinterpret_cast<Triple<Real>*>(NSd + 3 * (size_t)n) =
                Triple<Real>{A.coef.alpha[d.node_off + n], (Real)(be * b.x), (Real)(be * b.y)};
            il += di;
            jl += dj;
            if (il >= nxl) { il -= nxl; ++jl; }
        }
    }
    if (!xb_sync_ok(xb)) return;
    StreamGeom<Real, P> G;
    G.setup(nxl, nyl, WT, xb.K, xb.k);
    G.side_col = all_sides || G.ic == 0 || G.ic == nxl - 1;
    const Real sig = (Real)d.sigma;
    const int nt = d.nt;
    int it = 0;
    const int max_wh = d.max_wh > 0 ? d.max_wh : A.max_wh;
    const double tau = d.max_wh > 0 ? d.tau : A.tau;
    // warm start: the first WaveHoltz iteration starts from the current u
    const bool warm = A.warm != 0 || (d.flags & 1) != 0;
    WhStall stall;
    for (int m = 0; m < max_wh; ++m) {
        // u -> (p^1, pdot^{1/2}, v)
        {
            const Real k0 = TAB[2], kh0 = TAB[3];
            int il = tid % nxl, jl = tid / nxl;
            for (int n = tid; n < nloc; n += bd) {
                Real p = Real(0), pd = Real(0);
                if (m > 0 || warm) {
                    const double2 u = A.u[d.node_off + n];
                    p = (Real)u.x;
                    pd = (Real)(u.y * d.pd0c - u.x * d.pd0s);
                }
                *reinterpret_cast<Triple<Real>*>(NSt + 3 * (size_t)n) =
                    Triple<Real>{pd, k0 * p, kh0 * pd};
                p1[(jl + kMaxP) * stride + il + kMaxP] = fma(sig, pd, p);
                il += di;
                jl += dj;
                if (il >= nxl) { il -= nxl; ++jl; }
            }
        }
        double dsum = 0.0, nsum = 0.0;
        for (int nu = 1; nu < nt; ++nu) {
            if (!xb_sync_ok(xb)) return;
            const Real* cur = (nu & 1) ? p1 : p0;
            Real* nxt = (nu & 1) ? p0 : p1;
            if (!G.active) continue;
            const Quad<Real> tb{TAB[4 * nu + 0], TAB[4 * nu + 1], TAB[4 * nu + 2], TAB[4 * nu + 3]};
            if (nu < nt - 1)
                stream_rows<Real, P, false>(G, cur, nxt, stride, nxl, nyl, N, WT, tb, sig, A, d,
                                            m > 0 || warm, dsum, nsum);
            else
                stream_rows<Real, P, true>(G, cur, nxt, stride, nxl, nyl, N, WT, tb, sig, A, d,
                                           m > 0 || warm, dsum, nsum);
        }
        block_sum2(dsum, nsum, red);
        if (!xbar_sum2(xb, dsum, nsum, red + 32)) return;
        it = m + 1;
        if (!(dsum == dsum)) break;
        if (wh_stop<Real>(tau, dsum, nsum, stall)) break;
    }
    __threadfence_block();
    if (!xb_sync_ok(xb)) return;
    if (xb.k != 0) return;
    exchange(A, d);
    if (threadIdx.x == 0) A.wh_iters[item] = it;
}

template <typename Real, int P>
__global__ void __launch_bounds__(kStreamWG) sweep_stream_kernel(const SweepArgs<Real> A) {
    extern __shared__ double smem_d[];
    double* red = smem_d;
    Real* lds = reinterpret_cast<Real*>(smem_d + 40);
    XBar xb{nullptr, nullptr, nullptr, nullptr, 1, 0, 0};
    const int item = blockIdx.x;   // one workgroup per item (grid = n_items)
    if (item >= A.n_items) return;
    const SubDesc d = A.desc[item];   // loaded once: kept in registers across the stores below
    sweep_stream_item<Real, P>(A, d, item, lds, red, xb);
}

// The STREAM sweep with K = A.xb_k workgroups per item.  The hardware hands
// out the workgroups of a launch to the XCDs in turn (workgroup b to XCD
// b mod 8), so item i takes workgroups (i / 8) * 8K + 8k + i mod 8,
// k < K: all on one XCD.  Each workgroup checks that at the start (it
// publishes its XCD number and compares after the first barrier) and the
// launch aborts if they differ; the host then runs the plain STREAM sweep.
template <typename Real, int P>
__global__ void __launch_bounds__(kStreamWG) sweep_stream_coop_kernel(const SweepArgs<Real> A) {
    extern __shared__ double smem_d[];
    double* red = smem_d;
    Real* lds = reinterpret_cast<Real*>(smem_d + 40);
    const int K = A.xb_k, b = blockIdx.x;
    const int item = (b / (8 * K)) * 8 + b % 8, k = (b / 8) % K;
    if (item >= A.n_items) return;
    XBar xb{A.xb_cnt + item, A.xb_abort, A.xb_part + 2 * (size_t)K * item,
            reinterpret_cast<int*>(smem_d + 36), K, k, 0};
    // placement check: every workgroup of the item on the same XCD
    const int xcc = (int)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);  // HW_REG_XCC_ID
    if (threadIdx.x == 0) xb.part[2 * k] = (double)(xcc + 1);
    if (!xbar_sync(xb)) return;
    int* same = reinterpret_cast<int*>(smem_d + 37);
    if (threadIdx.x == 0) {
        int ok = 1;
        for (int j = 0; j < K; ++j) ok &= xbar_read(xb.part + 2 * j) == (double)(xcc + 1);
        if (!ok) atomicExch(xb.abort, 1);
        *same = ok;
    }
    __syncthreads();
    if (!*same) return;
    if (!xbar_sync(xb)) return;  // all have read the placement before part is reused
    const SubDesc d = A.desc[item];
    sweep_stream_item<Real, P>(A, d, item, lds, red, xb);
}

// q = A p per subdomain (node-indexed, unpadded; the windows are bounds
// checked) with the STREAM layout's window tables.
template <typename Real, int P>
__global__ void __launch_bounds__(kMaxWG) apply_stream_kernel(const SweepArgs<Real> A,
                                                              const Real* pin, Real* qout) {
    constexpr int W = 2 * P + 1;
    extern __shared__ double smem_d[];
    Real* lds = reinterpret_cast<Real*>(smem_d + 40);
    const SubDesc d = A.desc[blockIdx.x];
    stream_tables<Real, P>(lds, A.K1[P]);
    __syncthreads();
    const int nxl = d.nxl, nyl = d.nyl, nloc = nxl * nyl;
    const double* wxp = A.w1d + d.w_off;
    const double* wyp = wxp + nxl;
    const Real* p = pin + d.node_off;
    for (int n = threadIdx.x; n < nloc; n += blockDim.x) {
        const int il = n % nxl, jl = n / nxl;
        const Real* wx = lds + stream_class<P>(il, nxl) * W;
        const Real* wy = lds + stream_class<P>(jl, nyl) * W;
        Real X = Real(0), Y = Real(0);
#pragma unroll
        for (int j = 0; j < W; ++j) {
            const int i2 = il + j - P, j2 = jl + j - P;
            const Real px = (i2 >= 0 && i2 < nxl) ? p[jl * nxl + i2] : Real(0);
            const Real py = (j2 >= 0 && j2 < nyl) ? p[j2 * nxl + il] : Real(0);
            X = fma(wx[j], px, X);
            Y = fma(wy[j], py, Y);
        }
        qout[d.node_off + n] = (Real)(d.sx_ref * wyp[jl]) * X + (Real)(d.sy_ref * wxp[il]) * Y;
    }
}

}  // namespace

size_t stream_lds_bytes(int P, int nt_max, size_t real_size) {
    (void)P;
    return 40 * sizeof(double) + ((size_t)kStreamTab + 4 * (size_t)nt_max) * real_size;
}

size_t patch_lds_bytes(int mx, int my, int P, int nt_max, size_t real_size) {
    return 40 * sizeof(double) + (size_t)patch_lds(mx, my, P, nt_max).total * real_size;
}

static inline int patch1_wg_bound(int wg) { return wg <= 256 ? 256 : 512; }

size_t patch1_lds_bytes(int mx, int my, int P, int wg, int nt_max, size_t real_size) {
    return 40 * sizeof(double) +
           (size_t)patch1_lds(mx, my, P, patch1_wg_bound(wg), nt_max).total * real_size;
}

size_t node_lds_bytes(int nxl, int nyl, int nt_max, size_t real_size) {
    return 40 * sizeof(double) +
           ((size_t)node_tab_off(nxl, nyl, (int)real_size) + 4 * (size_t)nt_max) * real_size;
}

#define WDD_DISPATCH_P(P, CALL) \
    switch (P) {                \
        case 1: CALL(1); break; \
        case 2: CALL(2); break; \
        case 3: CALL(3); break; \
        case 4: CALL(4); break; \
        default: return hipErrorInvalidValue; \
    }

template <typename Real>
hipError_t launch_sweep_patch(const SweepArgs<Real>& a, int P, int wg, hipStream_t s) {
    const size_t lds = a.lds_bytes;
    const bool src = a.Fre != nullptr && a.src != 0.0;
#define L(PP, W, S) \
    hipLaunchKernelGGL((sweep_patch_kernel<Real, PP, W, S>), dim3(a.n_items), dim3(wg), lds, s, a)
#define L256(PP) if (src) L(PP, 256, true); else L(PP, 256, false)
#define L512(PP) if (src) L(PP, 512, true); else L(PP, 512, false)
    if (wg <= 256) {
        WDD_DISPATCH_P(P, L256)
    } else if (wg <= 512) {
        WDD_DISPATCH_P(P, L512)
    } else {
        return hipErrorInvalidValue;
    }
#undef L
#undef L256
#undef L512
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_sweep_patch1(const SweepArgs<Real>& a, int P, int wg, hipStream_t s) {
    const size_t lds = a.lds_bytes;
    const bool src = a.Fre != nullptr && a.src != 0.0;
#define L(PP, W, S) \
    hipLaunchKernelGGL((sweep_patch1_kernel<Real, PP, W, S>), dim3(a.n_items), dim3(wg), lds, s, a)
#define L256(PP) if (src) L(PP, 256, true); else L(PP, 256, false)
#define L512(PP) if (src) L(PP, 512, true); else L(PP, 512, false)
    if (wg <= 256) {
        WDD_DISPATCH_P(P, L256)
    } else if (wg <= 512) {
        WDD_DISPATCH_P(P, L512)
    } else {
        return hipErrorInvalidValue;
    }
#undef L
#undef L256
#undef L512
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_apply_patch1(const SweepArgs<Real>& a, int P, int wg, const Real* p, Real* q,
                               hipStream_t s) {
    const size_t lds = a.lds_bytes;
    if (wg <= 256) {
#define L(PP) \
    hipLaunchKernelGGL((apply_patch1_kernel<Real, PP, 256>), dim3(a.n_items), dim3(wg), lds, s, a, p, q)
        WDD_DISPATCH_P(P, L)
#undef L
    } else if (wg <= 512) {
#define L(PP) \
    hipLaunchKernelGGL((apply_patch1_kernel<Real, PP, 512>), dim3(a.n_items), dim3(wg), lds, s, a, p, q)
        WDD_DISPATCH_P(P, L)
#undef L
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_sweep_node(const SweepArgs<Real>& a, int P, int wg, hipStream_t s) {
    const size_t lds = a.lds_bytes;
#define L(PP) hipLaunchKernelGGL((sweep_node_kernel<Real, PP>), dim3(a.n_items), dim3(wg), lds, s, a)
    WDD_DISPATCH_P(P, L)
#undef L
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_apply_patch(const SweepArgs<Real>& a, int P, int wg, const Real* p, Real* q,
                              hipStream_t s) {
    const size_t lds = a.lds_bytes;
    if (wg <= 256) {
#define L(PP) \
    hipLaunchKernelGGL((apply_patch_kernel<Real, PP, 256>), dim3(a.n_items), dim3(wg), lds, s, a, p, q)
        WDD_DISPATCH_P(P, L)
#undef L
    } else if (wg <= 512) {
#define L(PP) \
    hipLaunchKernelGGL((apply_patch_kernel<Real, PP, 512>), dim3(a.n_items), dim3(wg), lds, s, a, p, q)
        WDD_DISPATCH_P(P, L)
#undef L
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_apply_node(const SweepArgs<Real>& a, int P, int wg, const Real* p, Real* q,
                             hipStream_t s) {
    const size_t lds = a.lds_bytes;
#define L(PP) \
    hipLaunchKernelGGL((apply_node_kernel<Real, PP>), dim3(a.n_items), dim3(wg), lds, s, a, p, q)
    WDD_DISPATCH_P(P, L)
#undef L
    return hipGetLastError();
}

template hipError_t launch_sweep_patch<double>(const SweepArgs<double>&, int, int, hipStream_t);
template hipError_t launch_sweep_patch<float>(const SweepArgs<float>&, int, int, hipStream_t);
template hipError_t launch_sweep_patch1<double>(const SweepArgs<double>&, int, int, hipStream_t);
template hipError_t launch_sweep_patch1<float>(const SweepArgs<float>&, int, int, hipStream_t);
template hipError_t launch_apply_patch1<double>(const SweepArgs<double>&, int, int, const double*,
                                                double*, hipStream_t);
template hipError_t launch_apply_patch1<float>(const SweepArgs<float>&, int, int, const float*,
                                               float*, hipStream_t);
template hipError_t launch_sweep_node<double>(const SweepArgs<double>&, int, int, hipStream_t);
template hipError_t launch_sweep_node<float>(const SweepArgs<float>&, int, int, hipStream_t);
template hipError_t launch_apply_patch<double>(const SweepArgs<double>&, int, int, const double*,
                                               double*, hipStream_t);
template hipError_t launch_apply_patch<float>(const SweepArgs<float>&, int, int, const float*,
                                              float*, hipStream_t);
template hipError_t launch_apply_node<double>(const SweepArgs<double>&, int, int, const double*,
                                              double*, hipStream_t);
template hipError_t launch_apply_node<float>(const SweepArgs<float>&, int, int, const float*,
                                             float*, hipStream_t);

template <typename Real>
hipError_t launch_sweep_stream(const SweepArgs<Real>& a, int P, int wg, hipStream_t s) {
    const size_t lds = a.lds_bytes;
    if (wg > kStreamWG) return hipErrorInvalidValue;
#define L(PP) \
    hipLaunchKernelGGL((sweep_stream_kernel<Real, PP>), dim3(a.n_items), dim3(wg), lds, s, a)
    WDD_DISPATCH_P(P, L)
#undef L
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_sweep_stream_coop(const SweepArgs<Real>& a, int P, int wg, hipStream_t s) {
    const size_t lds = a.lds_bytes;
    const int K = a.xb_k;
    if (wg > kStreamWG || K < 2 || !a.xb_cnt || !a.xb_abort || !a.xb_part)
        return hipErrorInvalidValue;
    const unsigned grid = (unsigned)(((a.n_items + 7) / 8) * 8 * K);
    SweepArgs<Real> arg = a;
    void* args[] = {&arg};
#define L(PP)                                                                                 \
    {                                                                                         \
        hipError_t e = hipLaunchCooperativeKernel(                                            \
            reinterpret_cast<const void*>(&sweep_stream_coop_kernel<Real, PP>), dim3(grid),  \
            dim3(wg), args, (unsigned)lds, s);                                                \
        if (e != hipSuccess) return e;                                                        \
    }
    WDD_DISPATCH_P(P, L)
#undef L
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_apply_stream(const SweepArgs<Real>& a, int P, int wg, const Real* p, Real* q,
                               hipStream_t s) {
    const size_t lds = a.lds_bytes;
    if (wg > kMaxWG) return hipErrorInvalidValue;
#define L(PP) \
    hipLaunchKernelGGL((apply_stream_kernel<Real, PP>), dim3(a.n_items), dim3(wg), lds, s, a, p, q)
    WDD_DISPATCH_P(P, L)
#undef L
    return hipGetLastError();
}

template hipError_t launch_sweep_stream<double>(const SweepArgs<double>&, int, int, hipStream_t);
template hipError_t launch_sweep_stream<float>(const SweepArgs<float>&, int, int, hipStream_t);
template hipError_t launch_sweep_stream_coop<double>(const SweepArgs<double>&, int, int,
                                                     hipStream_t);
template hipError_t launch_sweep_stream_coop<float>(const SweepArgs<float>&, int, int,
                                                    hipStream_t);
template hipError_t launch_apply_stream<double>(const SweepArgs<double>&, int, int, const double*,
                                                double*, hipStream_t);
template hipError_t launch_apply_stream<float>(const SweepArgs<float>&, int, int, const float*,
                                               float*, hipStream_t);

}  // namespace wdd
