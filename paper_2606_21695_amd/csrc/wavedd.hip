// Host side of the wavedd library: problem setup (GLL tables, lumped
// coefficients, time-step rule, filter tables), the sweep launcher, the FP64
// outer GMRES / fixed-point iteration on device vectors, and the C ABI of
// include/wavedd.h.
#include "../../include/wavedd.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "wavedd_internal.h"

using cplx = std::complex<double>;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(e_ == hipErrorOutOfMemory ? DD_ENOMEM : DD_EHIP, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);               \
    } while (0)

#define CHK(expr)             \
    do {                      \
        int r_ = (expr);      \
        if (r_ != DD_OK) return r_; \
    } while (0)

// ---------------------------------------------------------------------------
// GLL tables (Sec. IV): nodes = -1, roots of L_P', +1; weights
// 2/(P(P+1) L_P(x)^2); D[a][b] = l_b'(x_a).
// ---------------------------------------------------------------------------
void legendre(int n, double x, double& L, double& dL) {
    double p0 = 1.0, p1 = x;
    if (n == 0) {
        L = 1.0;
        dL = 0.0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    L = p1;
    dL = n * (x * p1 - p0) / (x * x - 1.0);  // valid for |x| < 1
}

struct Gll {
    int P;
    double x[wdd::kMaxP + 1], w[wdd::kMaxP + 1];
    double D[wdd::kMaxP + 1][wdd::kMaxP + 1];
    double K[wdd::kMaxP + 1][wdd::kMaxP + 1];  // D^T W D
    double mu;                                  // largest eigenvalue of W^-1/2 K W^-1/2
};

// Largest eigenvalue of a small symmetric matrix by cyclic Jacobi rotations.
double sym_max_eig(int n, double (*Ain)[wdd::kMaxP + 1]) {
    double A[wdd::kMaxP + 1][wdd::kMaxP + 1];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) A[i][j] = Ain[i][j];
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A[i][j] * A[i][j];
        if (off < 1e-30) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                if (std::fabs(A[p][q]) < 1e-300) continue;
                const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (theta >= 0 ? 1.0 : -1.0) /
                                 (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
            }
    }
    double m = A[0][0];
    for (int i = 1; i < n; ++i) m = std::max(m, A[i][i]);
    return m;
}

Gll make_gll(int P) {
    Gll g{};
    g.P = P;
    g.x[0] = -1.0;
    g.x[P] = 1.0;
    for (int k = 1; k < P; ++k) {
        double x = -std::cos(M_PI * k / P);  // Chebyshev-Gauss-Lobatto start
        for (int it = 0; it < 100; ++it) {
            double L, dL;
            legendre(P, x, L, dL);
            // Legendre ODE: (1-x^2) L'' = 2x L' - P(P+1) L
            const double d2L = (2.0 * x * dL - P * (P + 1.0) * L) / (1.0 - x * x);
            const double dx = dL / d2L;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        g.x[k] = x;
    }
    double LP[wdd::kMaxP + 1];
    for (int a = 0; a <= P; ++a) {
        double L, dL;
        legendre(P, g.x[a], L, dL);
        if (a == 0) L = (P % 2 == 0) ? 1.0 : -1.0;
        if (a == P) L = 1.0;
        LP[a] = L;
        g.w[a] = 2.0 / (P * (P + 1.0) * L * L);
    }
    for (int a = 0; a <= P; ++a)
        for (int b = 0; b <= P; ++b)
            g.D[a][b] = (a != b) ? LP[a] / (LP[b] * (g.x[a] - g.x[b])) : 0.0;
    g.D[0][0] = -P * (P + 1.0) / 4.0;
    g.D[P][P] = P * (P + 1.0) / 4.0;
    for (int a = 0; a <= P; ++a)
        for (int b = 0; b <= P; ++b) {
            double s = 0.0;
            for (int q = 0; q <= P; ++q) s += g.D[q][a] * g.w[q] * g.D[q][b];
            g.K[a][b] = s;
        }
    double S[wdd::kMaxP + 1][wdd::kMaxP + 1];
    for (int a = 0; a <= P; ++a)
        for (int b = 0; b <= P; ++b) S[a][b] = g.K[a][b] / std::sqrt(g.w[a] * g.w[b]);
    g.mu = sym_max_eig(P + 1, S);
    return g;
}

// Time steps per period (Sec. V leapfrog): stable iff sin(pi/N_t) <
// omega / sqrt(lambda_max(M^-1 A)) and lambda_max <= cmax^2 mu ((2/hx)^2 +
// (2/hy)^2); safety factor cfl.
int time_steps(const Gll& g, double hx, double hy, double cmax, double omega, double cfl) {
    const double lam = cmax * cmax * g.mu * ((2.0 / hx) * (2.0 / hx) + (2.0 / hy) * (2.0 / hy));
    const double arg = cfl * omega / std::sqrt(lam);
    if (arg >= 1.0) return 4;
    const int n = (int)std::ceil(M_PI / std::asin(arg));
    return std::max(4, n);
}

// Assembled reference 1D weight at local node il of a line of m elements.
double wref(const Gll& g, int il, int m) {
    const int P = g.P;
    const int e = il / P, a = il - e * P;
    if (a != 0) return g.w[a];
    double s = 0.0;
    if (e < m) s += g.w[0];
    if (e > 0) s += g.w[P];
    return s;
}

template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    hipError_t alloc(size_t count) {
        n = count;
        return hipMalloc(&p, sizeof(T) * std::max<size_t>(count, 1));
    }
    void free() {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
};

}  // namespace

struct dd_handle {
    // problem
    dd_mesh mesh;
    int P;
    double omega;
    dd_partition part;
    dd_options opt;
    Gll gll;
    int mx, my, nxl, nyl, Nx, Ny;
    int64_t N, nloc, L, n_if, n_trace, per_sub;
    double hx, hy;
    std::vector<double> c;           // wavespeed at global nodes
    std::vector<int> nt;             // per subdomain
    int nt_max = 0;
    std::vector<wdd::SubDesc> desc;
    int layout = DD_LAYOUT_PATCH, wg = 256;
    int dev = 0;
    hipStream_t stream = nullptr;
    // device data
    DBuf<wdd::SubDesc> d_desc;
    // per-precision sweep data: [0] FP64 (always), [1] FP32 (FP32 handles)
    struct PrecBuf {
        DBuf<char> coef;             // alpha, betaX, betaY, beta
        DBuf<char> tab;              // kap, kaph, cs, sn
        DBuf<char> F;                // Fre, Fim (per solve)
        size_t lds_bytes = 0;
        bool present = false;
    } pb[2];
    int64_t tab_len = 0;
    DBuf<double> d_w1d, d_kside, d_area;
    DBuf<int> d_gidx, d_iters, d_is_iface;
    DBuf<int64_t> d_trace_idx;
    DBuf<double2> d_u;               // stacked subdomain iterate
    DBuf<double2> d_V;               // GMRES basis (restart + 1) x ld
    DBuf<double2> d_G, d_h, d_tmp, d_g0, d_r, d_coefs, d_D, d_res;
    DBuf<double> d_fre, d_fim, d_gre, d_gim, d_ure, d_uim;  // staging for host API
    DBuf<double> d_wxg, d_wyg, d_Mg, d_Hg;                 // global operator data
    DBuf<double2> d_work;            // N complex scratch
    int64_t ld = 0;
    wdd::Blas blas;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<int> iters_host;
    double K1all[wdd::kMaxP + 1][wdd::kMaxP + 1][wdd::kMaxP + 1];  // reference stiffness per P
    bool has_state = false;
    // stats of the current solve
    dd_stats st{};
};

namespace {

size_t real_size(const dd_handle* h) { return h->opt.precision == DD_FP32 ? 4 : 8; }
size_t prec_size(int prec) { return prec == DD_FP32 ? 4 : 8; }
int prec_index(int prec) { return prec == DD_FP32 ? 1 : 0; }

template <typename Real>
wdd::SweepArgs<Real> make_args(dd_handle* h, const double2* g_in, double2* g_out, double src,
                               bool with_f, double tau, int max_wh) {
    const dd_handle::PrecBuf& B = h->pb[sizeof(Real) == 4 ? 1 : 0];
    wdd::SweepArgs<Real> a{};
    a.desc = h->d_desc.p;
    a.n_items = (int)h->L;
    Real* coef = reinterpret_cast<Real*>(B.coef.p);
    const int64_t n = h->L * h->nloc;
    a.coef.alpha = coef;
    a.coef.betaX = coef + n;
    a.coef.betaY = coef + 2 * n;
    a.coef.beta = coef + 3 * n;
    Real* F = reinterpret_cast<Real*>(B.F.p);
    a.Fre = with_f ? F : nullptr;
    a.Fim = with_f ? F + n : nullptr;
    a.w1d = h->d_w1d.p;
    a.kside = h->d_kside.p;
    Real* tab = reinterpret_cast<Real*>(B.tab.p);
    a.kap = tab;
    a.kaph = tab + h->tab_len;
    a.cs = tab + 2 * h->tab_len;
    a.sn = tab + 3 * h->tab_len;
    a.g_in = g_in;
    a.g_out = g_out;
    a.src = src;
    a.u = h->d_u.p;
    a.wh_iters = h->d_iters.p;
    a.tau = tau;
    a.max_wh = max_wh;
    a.lds_bytes = B.lds_bytes;
    a.nt_max = h->nt_max;
    std::memcpy(a.K1, h->K1all, sizeof(a.K1));
    return a;
}

constexpr size_t kLdsLimit = 160 * 1024;

int patch_threads(const dd_handle* h) {
    return std::max(h->mx * h->my, h->mx * h->P + h->my * h->P + 1);
}

int layout_threads(const dd_handle* h, int layout) {
    const int t = layout == DD_LAYOUT_NODE ? h->nxl * h->nyl : patch_threads(h);
    return ((t + 63) / 64) * 64;
}

size_t layout_lds(const dd_handle* h, int layout, int prec) {
    const size_t rs = prec_size(prec);
    if (layout == DD_LAYOUT_NODE) return wdd::node_lds_bytes(h->nxl, h->nyl, h->nt_max, rs);
    if (layout == DD_LAYOUT_PATCH_XCHG) return wdd::patch_lds_bytes(h->mx, h->my, h->P, h->nt_max, rs);
    return wdd::patch1_lds_bytes(h->mx, h->my, h->P, layout_threads(h, layout), h->nt_max, rs);
}

void layout_config(dd_handle* h, int layout) {
    h->layout = layout;
    h->wg = layout_threads(h, layout);
    for (int prec : {DD_FP64, DD_FP32})
        h->pb[prec_index(prec)].lds_bytes = layout_lds(h, layout, prec);
}

// Fits in one workgroup for every precision the handle carries (FP64
// always, for the refinement residuals of FP32 handles too).
bool layout_fits(const dd_handle* h, int layout) {
    const bool threads_ok = layout == DD_LAYOUT_NODE ? h->nxl * h->nyl <= 1024 : patch_threads(h) <= 512;
    return threads_ok && layout_lds(h, layout, DD_FP64) <= kLdsLimit;
}

// One sweep launch: g_out = sweep(g_in, src), u = subdomain solutions.
int run_sweep(dd_handle* h, const double2* g_in, double2* g_out, double src, bool with_f,
              bool timed, int prec, double tau, int max_wh) {
    hipStream_t s = h->stream;
    if (timed) HIPCHK(hipEventRecord(h->ev0, s));
    hipError_t e;
    if (prec == DD_FP32) {
        auto a = make_args<float>(h, g_in, g_out, src, with_f, tau, max_wh);
        e = h->layout == DD_LAYOUT_NODE    ? wdd::launch_sweep_node<float>(a, h->P, h->wg, s)
            : h->layout == DD_LAYOUT_PATCH ? wdd::launch_sweep_patch1<float>(a, h->P, h->wg, s)
                                           : wdd::launch_sweep_patch<float>(a, h->P, h->wg, s);
    } else {
        auto a = make_args<double>(h, g_in, g_out, src, with_f, tau, max_wh);
        e = h->layout == DD_LAYOUT_NODE    ? wdd::launch_sweep_node<double>(a, h->P, h->wg, s)
            : h->layout == DD_LAYOUT_PATCH ? wdd::launch_sweep_patch1<double>(a, h->P, h->wg, s)
                                           : wdd::launch_sweep_patch<double>(a, h->P, h->wg, s);
    }
    HIPCHK(e);
    if (timed) HIPCHK(hipEventRecord(h->ev1, s));
    HIPCHK(hipMemcpyAsync(h->iters_host.data(), h->d_iters.p, sizeof(int) * h->L,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (timed) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        h->st.sweep_seconds += ms * 1e-3;
    }
    h->st.sweeps += 1;
    if (prec == DD_FP64 && h->opt.precision == DD_FP32) h->st.fp64_sweeps += 1;
    for (int64_t l = 0; l < h->L; ++l) {
        const int it = h->iters_host[l];
        h->st.wh_iters_total += it;
        h->st.wh_iters_max = std::max(h->st.wh_iters_max, it);
        h->st.dof_updates += (double)h->nloc * (h->nt[l] - 1) * it;
    }
    return DD_OK;
}

// Sweep in the handle's own precision and inner tolerance.
int run_sweep(dd_handle* h, const double2* g_in, double2* g_out, double src, bool with_f,
              bool timed) {
    return run_sweep(h, g_in, g_out, src, with_f, timed, h->opt.precision, h->opt.tau_in,
                     h->opt.max_wh);
}

// Hermitian inner products <V_i, w>, i < k, into host array out (device
// reduction, one readback).
int dots(dd_handle* h, const double2* V, int64_t ld, int k, const double2* w, cplx* out) {
    HIPCHK(wdd::blas_multidot(h->blas, V, ld, k, w, h->n_if, h->stream));
    std::vector<double2> tmp(k);
    HIPCHK(hipMemcpyAsync(tmp.data(), h->blas.result, sizeof(double2) * k, hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int i = 0; i < k; ++i) out[i] = cplx(tmp[i].x, tmp[i].y);
    return DD_OK;
}

double norm(dd_handle* h, const double2* x) {
    cplx v;
    if (dots(h, x, 0, 1, x, &v) != DD_OK) return NAN;
    return std::sqrt(std::max(0.0, v.real()));
}

int axpby(dd_handle* h, cplx a, const double2* x, cplx b, double2* y) {
    HIPCHK(wdd::blas_axpby(make_double2(a.real(), a.imag()), x, make_double2(b.real(), b.imag()),
                           y, h->n_if, h->stream));
    return DD_OK;
}


// w = v - T v  (T: sweep with sources off, in the handle's precision, with
// inner tolerance tau); w must not alias v.
int matvec(dd_handle* h, const double2* v, double2* w, double tau) {
    CHK(run_sweep(h, v, w, 0.0, false, true, h->opt.precision, tau, h->opt.max_wh));
    return axpby(h, cplx(1.0, 0.0), v, cplx(-1.0, 0.0), w);
}

// Inner tolerance of the k-th Arnoldi matvec.  Strict (tau_in) unless the
// relaxed mode is on: inexact Krylov theory lets the matvec error grow in
// proportion to 1 / (current residual), so tau_k = relax * tol / rel_k,
// clamped to [tau_in, 1e-2].  The final true residual is always evaluated
// with tau_in.
double matvec_tau(const dd_handle* h, double tol, double rel) {
    if (!(h->opt.relax > 0.0)) return h->opt.tau_in;
    const double t = h->opt.relax * tol / std::max(rel, 1e-300);
    return std::min(1e-2, std::max(h->opt.tau_in, t));
}

// Restarted GMRES(m) for (I - T) x = rhs from x = 0 (the Krylov method of
// the outer iteration, Sec. III last paragraph).  Arnoldi with classical
// Gram-Schmidt applied twice (two block reductions per step instead of j+1
// sequential ones), complex Givens rotations on the host.  Stops when the
// recursive residual <= tol * rnorm0 or after max_iter matvecs; returns the
// iterations and the recursive relative residual.
int gmres(dd_handle* h, const double2* rhs, double2* x, double rnorm0, double tol, int max_iter,
          int* its_out, double* rel_out) {
    const int m = h->opt.restart;
    const int64_t n = h->n_if, ld = h->ld;
    double2* V = h->d_V.p;
    HIPCHK(hipMemsetAsync(x, 0, sizeof(double2) * n, h->stream));
    *its_out = 0;
    *rel_out = rnorm0 == 0.0 ? 0.0 : 1.0;
    if (rnorm0 == 0.0 || max_iter <= 0) return DD_OK;
    std::vector<cplx> H((size_t)(m + 1) * m), g(m + 1), sn(m), y(m);
    std::vector<double> cs(m);
    std::vector<cplx> h1(m + 1), h2(m + 1);
    HIPCHK(hipMemcpyAsync(h->d_r.p, rhs, sizeof(double2) * n, hipMemcpyDeviceToDevice, h->stream));
    double beta = rnorm0;
    int its = 0;
    double rel = 1.0;
    while (true) {
        std::fill(H.begin(), H.end(), cplx(0.0));
        std::fill(g.begin(), g.end(), cplx(0.0));
        g[0] = beta;
        CHK(axpby(h, cplx(1.0 / beta, 0.0), h->d_r.p, cplx(0.0), V));
        int k = 0;
        for (int j = 0; j < m; ++j) {
            double2* w = V + (int64_t)(j + 1) * ld;
            CHK(matvec(h, V + (int64_t)j * ld, w, matvec_tau(h, tol, rel)));
            ++its;
            CHK(dots(h, V, ld, j + 1, w, h1.data()));
            HIPCHK(wdd::blas_multiaxpy(h->blas, V, ld, j + 1, w, n, h->stream));
            CHK(dots(h, V, ld, j + 1, w, h2.data()));
            HIPCHK(wdd::blas_multiaxpy(h->blas, V, ld, j + 1, w, n, h->stream));
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h1[i] + h2[i];
            const double hn = norm(h, w);
            if (!std::isfinite(hn)) return fail(DD_ENAN, "non-finite Krylov vector");
            H[(size_t)(j + 1) * m + j] = hn;
            if (hn > 0.0) CHK(axpby(h, cplx(1.0 / hn, 0.0), w, cplx(0.0), w));
            for (int i = 0; i < j; ++i) {
                const cplx a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
                H[(size_t)(i + 1) * m + j] = -std::conj(sn[i]) * a + cs[i] * b;
            }
            const cplx a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
            const double den = std::sqrt(std::norm(a) + std::norm(b));
            if (std::abs(a) == 0.0) {
                cs[j] = 0.0;
                sn[j] = 1.0;
            } else {
                cs[j] = std::abs(a) / den;
                sn[j] = (a / std::abs(a)) * std::conj(b) / den;
            }
            H[(size_t)j * m + j] = cs[j] * a + sn[j] * b;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -std::conj(sn[j]) * g[j];
            g[j] = cs[j] * g[j];
            rel = std::abs(g[j + 1]) / rnorm0;
            k = j + 1;
            if (!std::isfinite(rel)) return fail(DD_ENAN, "non-finite outer residual");
            if (rel <= tol || its >= max_iter || hn == 0.0) break;
        }
        for (int i = k - 1; i >= 0; --i) {
            cplx sacc = g[i];
            for (int q = i + 1; q < k; ++q) sacc -= H[(size_t)i * m + q] * y[q];
            y[i] = sacc / H[(size_t)i * m + i];
        }
        std::vector<double2> yc(k);
        for (int i = 0; i < k; ++i) yc[i] = make_double2(y[i].real(), y[i].imag());
        HIPCHK(hipMemcpyAsync(h->d_coefs.p, yc.data(), sizeof(double2) * k, hipMemcpyHostToDevice,
                              h->stream));
        HIPCHK(wdd::blas_combine(V, ld, k, h->d_coefs.p, x, n, 1, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (rel <= tol || its >= max_iter) break;
        // r = rhs - (x - T x), with the strict inner tolerance
        CHK(matvec(h, x, h->d_r.p, h->opt.tau_in));
        CHK(axpby(h, cplx(1.0), rhs, cplx(-1.0), h->d_r.p));
        beta = norm(h, h->d_r.p);
        if (!std::isfinite(beta)) return fail(DD_ENAN, "non-finite outer residual");
        rel = beta / rnorm0;
        if (beta == 0.0 || rel <= tol) break;
    }
    *its_out = its;
    *rel_out = rel;
    return DD_OK;
}

// Plain fixed-point iteration G <- T G + h.
int fixed_point(dd_handle* h, double tol, int max_iter, double hnorm) {
    const int64_t n = h->n_if;
    HIPCHK(hipMemsetAsync(h->d_G.p, 0, sizeof(double2) * n, h->stream));
    h->st.outer_iters = 0;
    h->st.rel_residual = hnorm == 0.0 ? 0.0 : 1.0;
    if (hnorm == 0.0) return DD_OK;
    for (int it = 0; it < max_iter; ++it) {
        CHK(run_sweep(h, h->d_G.p, h->d_tmp.p, 0.0, false, true));
        CHK(axpby(h, cplx(1.0), h->d_h.p, cplx(1.0), h->d_tmp.p));   // tmp = T G + h
        CHK(axpby(h, cplx(1.0), h->d_tmp.p, cplx(-1.0), h->d_G.p));  // G = tmp - G
        const double d = norm(h, h->d_G.p);
        HIPCHK(hipMemcpyAsync(h->d_G.p, h->d_tmp.p, sizeof(double2) * n, hipMemcpyDeviceToDevice,
                              h->stream));
        h->st.outer_iters = it + 1;
        h->st.rel_residual = d / hnorm;
        if (!std::isfinite(d)) return fail(DD_ENAN, "non-finite outer residual");
        if (d <= tol * hnorm) break;
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return DD_OK;
}

void reset_stats(dd_handle* h) {
    h->st = dd_stats{};
    h->st.nt_min = *std::min_element(h->nt.begin(), h->nt.end());
    h->st.nt_max = *std::max_element(h->nt.begin(), h->nt.end());
}

// tmp = sweep(G + g0, sources on) = T G + h in precision prec (u left in
// d_u); returns ||tmp - G|| / hnorm, the outer residual of G.
int residual_sweep(dd_handle* h, bool with_f, int prec, double tau, double hnorm, double* rel) {
    CHK(axpby(h, cplx(1.0), h->d_g0.p, cplx(1.0), h->d_G.p));    // G += g0 (disjoint slots)
    CHK(run_sweep(h, h->d_G.p, h->d_tmp.p, 1.0, with_f, true, prec, tau, h->opt.max_wh));
    CHK(axpby(h, cplx(-1.0), h->d_g0.p, cplx(1.0), h->d_G.p));   // G -= g0
    CHK(axpby(h, cplx(-1.0), h->d_G.p, cplx(1.0), h->d_tmp.p));  // tmp = T G + h - G
    const double r = norm(h, h->d_tmp.p);
    if (!std::isfinite(r)) return fail(DD_ENAN, "non-finite outer residual");
    *rel = hnorm > 0.0 ? r / hnorm : 0.0;
    return DD_OK;
}

// Inner tolerance of the FP64 residual sweeps: the handle's own for FP64
// handles, clamp(0.01 tol, 1e-13, 1e-8) for FP32 handles (whose tau_in is an
// FP32-level tolerance).
double residual_tau(const dd_handle* h, double tol) {
    if (h->opt.precision == DD_FP64) return h->opt.tau_in;
    return std::min(1e-8, std::max(1e-13, 0.01 * tol));
}

// GMRES on the interface system inside an iterative-refinement loop:
//   r = h - (I - T) G  with a strict FP64 sweep (which also returns u),
//   G += GMRES((I - T) d = r)  with matvecs in the handle's precision and,
//   optionally, relaxed inner tolerance,
// until the true residual meets tol or `refine` corrections are spent.  A
// strict FP64 solve finishes in one pass (the same iterates as plain GMRES);
// FP32 sweeps and relaxed matvecs are corrected by the FP64 residuals.
int solve_gmres_refined(dd_handle* h, bool with_f, double tol, int max_iter) {
    const double tau64 = residual_tau(h, tol);
    CHK(run_sweep(h, h->d_g0.p, h->d_h.p, 1.0, with_f, true, DD_FP64, tau64, h->opt.max_wh));
    const double hnorm = norm(h, h->d_h.p);
    if (!std::isfinite(hnorm)) return fail(DD_ENAN, "non-finite right-hand side");
    HIPCHK(hipMemsetAsync(h->d_G.p, 0, sizeof(double2) * h->n_if, h->stream));
    HIPCHK(hipMemcpyAsync(h->d_res.p, h->d_h.p, sizeof(double2) * h->n_if,
                          hipMemcpyDeviceToDevice, h->stream));
    const bool fp32 = h->opt.precision == DD_FP32;
    const int passes = 1 + h->opt.refine;
    double rnorm = hnorm;
    int its_total = 0;
    double rel = hnorm > 0.0 ? 1.0 : 0.0;
    double last_rec = rel;
    bool have_u = false;
    for (int k = 0; k < passes && rel > tol && its_total < max_iter; ++k) {
        // FP32 corrections aim at a fixed reduction (their operator is only
        // FP32-accurate); FP64 ones go for the whole way
        const double want = tol * hnorm / rnorm;
        const double inner = fp32 ? std::max(1e-4, want) : want;
        int its = 0;
        double irel = 0.0;
        CHK(gmres(h, h->d_res.p, h->d_D.p, rnorm, inner, max_iter - its_total, &its, &irel));
        its_total += its;
        last_rec = irel * rnorm / hnorm;
        CHK(axpby(h, cplx(1.0), h->d_D.p, cplx(1.0), h->d_G.p));
        CHK(residual_sweep(h, with_f, DD_FP64, tau64, hnorm, &rel));
        HIPCHK(hipMemcpyAsync(h->d_res.p, h->d_tmp.p, sizeof(double2) * h->n_if,
                              hipMemcpyDeviceToDevice, h->stream));
        rnorm = rel * hnorm;
        h->st.refine_steps = k + 1;
        have_u = true;
    }
    if (!have_u) CHK(residual_sweep(h, with_f, DD_FP64, tau64, hnorm, &rel));
    h->st.outer_iters = its_total;
    h->st.rel_residual = std::max(last_rec, rel);
    h->st.true_rel_residual = rel;
    h->has_state = true;
    return DD_OK;
}

// Full solve with the device inputs staged: d_g0 (embedded boundary trace)
// and F (source).  Leaves the stacked u in d_u and G in d_G.
int solve_core(dd_handle* h, bool with_f, double tol, int max_iter) {
    if (h->opt.outer == DD_OUTER_GMRES) return solve_gmres_refined(h, with_f, tol, max_iter);
    CHK(run_sweep(h, h->d_g0.p, h->d_h.p, 1.0, with_f, true));  // h = sweep(g_phys, src)
    const double hnorm = norm(h, h->d_h.p);
    if (!std::isfinite(hnorm)) return fail(DD_ENAN, "non-finite right-hand side");
    CHK(fixed_point(h, tol, max_iter, hnorm));
    // final sweep with G + g_phys and sources: u, and T G + h for the true residual
    double rel = 0.0;
    CHK(residual_sweep(h, with_f, h->opt.precision, h->opt.tau_in, hnorm, &rel));
    h->st.true_rel_residual = rel;
    h->has_state = true;
    return DD_OK;
}

int validate_handle(const dd_handle* h) {
    if (!h) return fail(DD_EINVAL, "null handle");
    return DD_OK;
}

int check_finite(const double* x, int64_t n, const char* name) {
    if (!x) return DD_OK;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return fail(DD_ENAN, "%s[%lld] is not finite", name, (long long)i);
    return DD_OK;
}

int stage_source(dd_handle* h, const double* d_fre, const double* d_fim) {
    const int64_t n = h->L * h->nloc;
    for (int prec : {DD_FP64, DD_FP32}) {
        const dd_handle::PrecBuf& B = h->pb[prec_index(prec)];
        if (!B.present) continue;
        const size_t rs = prec_size(prec);
        char* F = B.F.p;
        HIPCHK(wdd::gather_source(d_fre, d_fim, h->d_gidx.p, h->d_area.p, n, F, F + rs * n,
                                  prec == DD_FP32, h->stream));
    }
    return DD_OK;
}

int ensure_staging(dd_handle* h) {
    if (!h->d_fre.p) {
        HIPCHK(h->d_fre.alloc(h->N));
        HIPCHK(h->d_fim.alloc(h->N));
        HIPCHK(h->d_gre.alloc(h->n_trace));
        HIPCHK(h->d_gim.alloc(h->n_trace));
        HIPCHK(h->d_ure.alloc(h->N));
        HIPCHK(h->d_uim.alloc(h->N));
        HIPCHK(h->d_work.alloc(2 * h->N));
    }
    return DD_OK;
}

wdd::OperatorArgs op_args(const dd_handle* h) {
    wdd::OperatorArgs a{};
    a.Nx = h->Nx;
    a.Ny = h->Ny;
    a.P = h->P;
    a.nx = h->mesh.nx;
    a.ny = h->mesh.ny;
    a.sx_ref = 2.0 / h->hx;
    a.sy_ref = 2.0 / h->hy;
    a.wx = h->d_wxg.p;
    a.wy = h->d_wyg.p;
    a.M = h->d_Mg.p;
    a.H = h->d_Hg.p;
    a.omega = h->omega;
    for (int i = 0; i <= h->P; ++i)
        for (int j = 0; j <= h->P; ++j) a.K1[i][j] = h->gll.K[i][j];
    return a;
}

// Layout autotuner: time every layout that fits on this problem (two
// fixed-count WaveHoltz iterations per subdomain, zero data: the kernels
// have no data-dependent work) and keep the fastest.
int autotune_layout(dd_handle* h) {
    int best = h->layout;
    double best_ms = 1e300;
    for (int lay : {DD_LAYOUT_PATCH, DD_LAYOUT_PATCH_XCHG, DD_LAYOUT_NODE}) {
        if (!layout_fits(h, lay)) continue;
        layout_config(h, lay);
        HIPCHK(hipMemsetAsync(h->d_g0.p, 0, sizeof(double2) * h->n_if, h->stream));
        CHK(run_sweep(h, h->d_g0.p, h->d_tmp.p, 0.0, false, false, h->opt.precision, 0.0, 2));
        reset_stats(h);
        for (int r = 0; r < 3; ++r)
            CHK(run_sweep(h, h->d_g0.p, h->d_tmp.p, 0.0, false, true, h->opt.precision, 0.0, 2));
        const double ms = h->st.sweep_seconds;
        if (ms < best_ms) {
            best_ms = ms;
            best = lay;
        }
    }
    layout_config(h, best);
    reset_stats(h);
    return DD_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* dd_last_error(void) { return g_err.c_str(); }

int dd_default_options(dd_options* o) {
    if (!o) return fail(DD_EINVAL, "null options");
    o->precision = DD_FP64;
    o->layout = DD_LAYOUT_AUTO;
    o->tau_in = 1e-12;
    o->max_wh = 100;
    o->outer = DD_OUTER_GMRES;
    o->restart = 50;
    o->nt_override = 0;
    o->cfl = 0.9;
    o->refine = 4;
    o->relax = 0.0;
    return DD_OK;
}

void dd_destroy(dd_handle* h) {
    if (!h) return;
    (void)hipSetDevice(h->dev);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    h->d_desc.free();
    for (auto& B : h->pb) {
        B.coef.free();
        B.tab.free();
        B.F.free();
    }
    h->d_D.free(); h->d_res.free();
    h->d_w1d.free(); h->d_kside.free(); h->d_area.free();
    h->d_gidx.free(); h->d_iters.free(); h->d_is_iface.free(); h->d_trace_idx.free();
    h->d_u.free(); h->d_V.free(); h->d_G.free(); h->d_h.free(); h->d_tmp.free(); h->d_g0.free();
    h->d_r.free(); h->d_coefs.free();
    h->d_fre.free(); h->d_fim.free(); h->d_gre.free(); h->d_gim.free(); h->d_ure.free();
    h->d_uim.free(); h->d_wxg.free(); h->d_wyg.free(); h->d_Mg.free(); h->d_Hg.free();
    h->d_work.free();
    wdd::blas_free(h->blas);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

int dd_setup(dd_handle** out, const dd_mesh* mesh, int degree, const double* wavespeed,
             double omega, const dd_partition* part, const dd_options* opt) {
    if (!out) return fail(DD_EINVAL, "null output handle pointer");
    *out = nullptr;
    if (!mesh || !part || !wavespeed) return fail(DD_EINVAL, "null mesh, partition or wavespeed");
    if (degree < 1 || degree > wdd::kMaxP)
        return fail(DD_EINVAL, "degree %d not in [1, %d]", degree, wdd::kMaxP);
    if (mesh->nx < 1 || mesh->ny < 1) return fail(DD_EINVAL, "empty mesh");
    if (!(mesh->x1 > mesh->x0) || !(mesh->y1 > mesh->y0) || !std::isfinite(mesh->x0) ||
        !std::isfinite(mesh->x1) || !std::isfinite(mesh->y0) || !std::isfinite(mesh->y1))
        return fail(DD_EINVAL, "degenerate rectangle");
    if (!(omega > 0.0) || !std::isfinite(omega)) return fail(DD_EINVAL, "omega must be > 0");
    if (part->sx < 1 || part->sy < 1 || mesh->nx % part->sx || mesh->ny % part->sy)
        return fail(DD_EINVAL, "partition %dx%d does not divide mesh %dx%d", part->sx, part->sy,
                    mesh->nx, mesh->ny);
    dd_options o;
    if (opt)
        o = *opt;
    else
        dd_default_options(&o);
    if (o.precision != DD_FP64 && o.precision != DD_FP32) return fail(DD_EINVAL, "bad precision");
    if (o.layout < DD_LAYOUT_AUTO || o.layout > DD_LAYOUT_PATCH_XCHG) return fail(DD_EINVAL, "bad layout");
    if (o.max_wh < 1) return fail(DD_EINVAL, "max_wh must be >= 1");
    if (o.outer != DD_OUTER_GMRES && o.outer != DD_OUTER_FIXED)
        return fail(DD_EINVAL, "bad outer method");
    if (o.restart < 1 || o.restart > 400) return fail(DD_EINVAL, "restart must be in [1, 400]");
    if (!(o.cfl > 0.0 && o.cfl <= 1.0)) return fail(DD_EINVAL, "cfl must be in (0, 1]");
    if (o.nt_override < 0 || o.nt_override == 1 || o.nt_override == 2)
        return fail(DD_EINVAL, "nt_override must be 0 or >= 3");
    if (o.refine < 0 || o.refine > 50) return fail(DD_EINVAL, "refine must be in [0, 50]");
    if (!(o.relax >= 0.0) || !std::isfinite(o.relax)) return fail(DD_EINVAL, "relax must be >= 0");
    const int P = degree;
    const int Nx = mesh->nx * P + 1, Ny = mesh->ny * P + 1;
    const int64_t N = (int64_t)Nx * Ny;
    if (N > (int64_t)2000000000) return fail(DD_EINVAL, "mesh too large");
    for (int64_t i = 0; i < N; ++i)
        if (!(wavespeed[i] > 0.0) || !std::isfinite(wavespeed[i]))
            return fail(DD_EINVAL, "wavespeed[%lld] = %g is not a positive number", (long long)i,
                        wavespeed[i]);
    const int mx = mesh->nx / part->sx, my = mesh->ny / part->sy;
    const int nxl = mx * P + 1, nyl = my * P + 1;
    dd_handle* h = new dd_handle();
    h->mesh = *mesh;
    h->P = P;
    h->omega = omega;
    h->part = *part;
    h->opt = o;
    h->gll = make_gll(P);
    std::memset(h->K1all, 0, sizeof(h->K1all));
    for (int q = 1; q <= wdd::kMaxP; ++q) {
        const Gll gq = make_gll(q);
        for (int i = 0; i <= q; ++i)
            for (int j = 0; j <= q; ++j) h->K1all[q][i][j] = gq.K[i][j];
    }
    h->mx = mx;
    h->my = my;
    h->nxl = nxl;
    h->nyl = nyl;
    h->Nx = Nx;
    h->Ny = Ny;
    h->N = N;
    h->nloc = (int64_t)nxl * nyl;
    h->L = (int64_t)part->sx * part->sy;
    h->per_sub = 2 * (int64_t)nyl + 2 * (int64_t)nxl;
    h->n_if = h->L * h->per_sub;
    h->n_trace = 2 * (int64_t)Ny + 2 * (int64_t)Nx;
    h->hx = (mesh->x1 - mesh->x0) / mesh->nx;
    h->hy = (mesh->y1 - mesh->y0) / mesh->ny;
    h->c.assign(wavespeed, wavespeed + N);

    const Gll& g = h->gll;
    const int64_t L = h->L, nloc = h->nloc;
    // per-subdomain time steps and filter tables (deduplicated by N_t)
    h->nt.resize(L);
    std::map<int, int> toff;
    std::vector<double> kap, kaph, cs, sn;
    for (int64_t l = 0; l < L; ++l) {
        const int a = (int)(l % part->sx), b = (int)(l / part->sx);
        double cmax = 0.0;
        for (int jl = 0; jl < nyl; ++jl)
            for (int il = 0; il < nxl; ++il)
                cmax = std::max(cmax, wavespeed[(int64_t)(b * my * P + jl) * Nx + a * mx * P + il]);
        const int n = o.nt_override > 0 ? o.nt_override
                                        : time_steps(g, h->hx, h->hy, cmax, omega, o.cfl);
        h->nt[l] = n;
        if (!toff.count(n)) {
            toff[n] = (int)kap.size();
            const double k0 = -0.25 + 0.25 * std::tan(M_PI / n) * std::tan(M_PI / n);
            for (int nu = 0; nu < n; ++nu) {
                kap.push_back(std::cos(2.0 * M_PI * nu / n) + k0);
                kaph.push_back((std::cos(2.0 * M_PI * (nu + 0.5) / n) + k0) / omega);
                cs.push_back(std::cos(2.0 * M_PI * nu / n));
                sn.push_back(std::sin(2.0 * M_PI * nu / n));
            }
        }
    }
    h->tab_len = (int64_t)kap.size();
    h->nt_max = *std::max_element(h->nt.begin(), h->nt.end());

    // layout choice (validated before any device work)
    const bool node_ok = layout_fits(h, DD_LAYOUT_NODE), patch_ok = layout_fits(h, DD_LAYOUT_PATCH);
    const bool xchg_ok = layout_fits(h, DD_LAYOUT_PATCH_XCHG);
    int lay = o.layout;
    const char* why = nullptr;
    if (lay == DD_LAYOUT_NODE && !node_ok)
        why = "one-DOF-per-thread layout needs <= 1024 nodes per subdomain";
    else if (lay == DD_LAYOUT_PATCH && !patch_ok)
        why = "patch layout needs <= 512 threads (element patches) per subdomain and its LDS";
    else if (lay == DD_LAYOUT_PATCH_XCHG && !xchg_ok)
        why = "patch layout needs <= 512 threads (element patches) per subdomain";
    else if (!node_ok && !patch_ok && !xchg_ok)
        why = "subdomain too large for the on-chip layouts";
    if (why) {
        delete h;
        return fail(DD_EINVAL, "%s (subdomain %dx%d elements, P=%d)", why, mx, my, P);
    }
    if (lay == DD_LAYOUT_AUTO) lay = patch_ok ? DD_LAYOUT_PATCH : xchg_ok ? DD_LAYOUT_PATCH_XCHG : DD_LAYOUT_NODE;
    layout_config(h, lay);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        delete h;
        return fail(DD_ENODEV, "no HIP device");
    }
    (void)hipGetDevice(&h->dev);

    auto bail = [&](int code) {
        dd_destroy(h);
        return code;
    };
#define SCHK(expr)                                                                              \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return bail(fail(e_ == hipErrorOutOfMemory ? DD_ENOMEM : DD_EHIP, "%s: %s", #expr,  \
                             hipGetErrorString(e_)));                                           \
    } while (0)


    // physical lumped 1D weights of a subdomain (the same for all)
    std::vector<double> w1d(nxl + nyl);
    for (int il = 0; il < nxl; ++il) w1d[il] = 0.5 * h->hx * wref(g, il, mx);
    for (int jl = 0; jl < nyl; ++jl) w1d[nxl + jl] = 0.5 * h->hy * wref(g, jl, my);

    // per-node coefficients (Sec. IV lumped M, H; Sec. V alpha, beta)
    const int64_t nn = L * nloc;
    std::vector<double> alpha(nn), betaX(nn), betaY(nn), beta(nn), area(nn);
    std::vector<int> gidx(nn);
    h->desc.resize(L);
    for (int64_t l = 0; l < L; ++l) {
        const int a = (int)(l % part->sx), b = (int)(l / part->sx);
        const int n = h->nt[l];
        const double half = M_PI / n;  // omega dt / 2
        const double theta = std::tan(half) / omega;
        const double sigma = std::sin(half) / (0.5 * omega);
        for (int jl = 0; jl < nyl; ++jl)
            for (int il = 0; il < nxl; ++il) {
                const int64_t k = l * nloc + (int64_t)jl * nxl + il;
                const int64_t gi = (int64_t)(b * my * P + jl) * Nx + a * mx * P + il;
                const double cc = wavespeed[gi];
                const double wx = w1d[il], wy = w1d[nxl + jl];
                const double M = wx * wy / (cc * cc);
                double Hs = 0.0;
                if (il == 0) Hs += wy;
                if (il == nxl - 1) Hs += wy;
                if (jl == 0) Hs += wx;
                if (jl == nyl - 1) Hs += wx;
                const double H = Hs / cc;
                alpha[k] = (M - theta * H) / (M + theta * H);
                beta[k] = sigma / (M + theta * H);
                betaX[k] = beta[k] * (2.0 / h->hx) * wy;
                betaY[k] = beta[k] * (2.0 / h->hy) * wx;
                area[k] = wx * wy;
                gidx[k] = (int)gi;
            }
        wdd::SubDesc& d = h->desc[l];
        d = wdd::SubDesc{};
        d.mx = mx;
        d.my = my;
        d.P = P;
        d.nxl = nxl;
        d.nyl = nyl;
        d.nt = n;
        d.toff = toff[n];
        d.node_off = l * nloc;
        d.w_off = 0;
        d.if_off = l * h->per_sub;
        const int64_t so[4] = {0, nyl, 2 * (int64_t)nyl, 2 * (int64_t)nyl + nxl};
        const int da[4] = {-1, 1, 0, 0}, db[4] = {0, 0, -1, 1}, opp[4] = {1, 0, 3, 2};
        for (int s = 0; s < 4; ++s) {
            const int a2 = a + da[s], b2 = b + db[s];
            if (a2 >= 0 && a2 < part->sx && b2 >= 0 && b2 < part->sy)
                d.nbr_off[s] = ((int64_t)b2 * part->sx + a2) * h->per_sub + so[opp[s]];
            else
                d.nbr_off[s] = -1;
        }
        d.sigma = sigma;
        d.pd0c = omega * std::cos(M_PI / n);
        d.pd0s = omega * std::sin(M_PI / n);
        d.two_over_nt = 2.0 / n;
        d.sx_ref = 2.0 / h->hx;
        d.sy_ref = 2.0 / h->hy;
    }
    // interface bookkeeping: omega/c per slot, outer-trace index of physical
    // slots, interface flags
    std::vector<double> kside(h->n_if);
    std::vector<int64_t> trace_idx(h->n_if);
    std::vector<int> is_iface(h->n_if);
    for (int64_t l = 0; l < L; ++l) {
        const int a = (int)(l % part->sx), b = (int)(l / part->sx);
        const wdd::SubDesc& d = h->desc[l];
        for (int k = 0; k < h->per_sub; ++k) {
            int s, pos, il, jl;
            if (k < nyl) { s = 0; pos = k; il = 0; jl = pos; }
            else if (k < 2 * nyl) { s = 1; pos = k - nyl; il = nxl - 1; jl = pos; }
            else if (k < 2 * nyl + nxl) { s = 2; pos = k - 2 * nyl; il = pos; jl = 0; }
            else { s = 3; pos = k - 2 * nyl - nxl; il = pos; jl = nyl - 1; }
            const int64_t slot = d.if_off + k;
            const int gx = a * mx * P + il, gy = b * my * P + jl;
            kside[slot] = omega / wavespeed[(int64_t)gy * Nx + gx];
            is_iface[slot] = d.nbr_off[s] >= 0;
            if (d.nbr_off[s] >= 0)
                trace_idx[slot] = -1;
            else
                trace_idx[slot] = s == 0 ? gy
                                  : s == 1 ? (int64_t)Ny + gy
                                  : s == 2 ? 2 * (int64_t)Ny + gx
                                           : 2 * (int64_t)Ny + Nx + gx;
        }
    }
    // whole-domain operator data (FP64)
    std::vector<double> wxg(Nx), wyg(Ny), Mg(N), Hg(N);
    for (int i = 0; i < Nx; ++i) wxg[i] = 0.5 * h->hx * wref(g, i, mesh->nx);
    for (int j = 0; j < Ny; ++j) wyg[j] = 0.5 * h->hy * wref(g, j, mesh->ny);
    for (int j = 0; j < Ny; ++j)
        for (int i = 0; i < Nx; ++i) {
            const int64_t gi = (int64_t)j * Nx + i;
            const double cc = wavespeed[gi];
            Mg[gi] = wxg[i] * wyg[j] / (cc * cc);
            double Hs = 0.0;
            if (i == 0) Hs += wyg[j];
            if (i == Nx - 1) Hs += wyg[j];
            if (j == 0) Hs += wxg[i];
            if (j == Ny - 1) Hs += wxg[i];
            Hg[gi] = Hs / cc;
        }

    // device allocation and upload
    SCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    SCHK(hipEventCreate(&h->ev0));
    SCHK(hipEventCreate(&h->ev1));
    const size_t rs = real_size(h);
    SCHK(h->d_desc.alloc(L));
    h->pb[0].present = true;
    h->pb[1].present = o.precision == DD_FP32;
    for (auto& B : h->pb) {
        if (!B.present) continue;
        const size_t bs = (&B == &h->pb[1]) ? 4 : 8;
        SCHK(B.coef.alloc(4 * bs * nn));
        SCHK(B.tab.alloc(4 * bs * h->tab_len));
        SCHK(B.F.alloc(2 * bs * nn));
    }
    SCHK(h->d_D.alloc(h->n_if));
    SCHK(h->d_res.alloc(h->n_if));
    SCHK(h->d_w1d.alloc(nxl + nyl));
    SCHK(h->d_kside.alloc(h->n_if));
    SCHK(h->d_area.alloc(nn));
    SCHK(h->d_gidx.alloc(nn));
    SCHK(h->d_iters.alloc(L));
    SCHK(h->d_is_iface.alloc(h->n_if));
    SCHK(h->d_trace_idx.alloc(h->n_if));
    SCHK(h->d_u.alloc(nn));
    h->ld = ((h->n_if + 63) / 64) * 64;
    SCHK(h->d_V.alloc((size_t)(o.restart + 1) * h->ld));
    SCHK(h->d_G.alloc(h->n_if));
    SCHK(h->d_h.alloc(h->n_if));
    SCHK(h->d_tmp.alloc(h->n_if));
    SCHK(h->d_g0.alloc(h->n_if));
    SCHK(h->d_r.alloc(h->n_if));
    SCHK(h->d_coefs.alloc(o.restart + 1));
    SCHK(h->d_wxg.alloc(Nx));
    SCHK(h->d_wyg.alloc(Ny));
    SCHK(h->d_Mg.alloc(N));
    SCHK(h->d_Hg.alloc(N));
    SCHK(wdd::blas_init(h->blas, o.restart + 2, h->stream));
    h->iters_host.assign(L, 0);

    auto up_real = [&](char* dst, const std::vector<double>& v, size_t bs) -> hipError_t {
        if (bs == 8) return hipMemcpy(dst, v.data(), 8 * v.size(), hipMemcpyHostToDevice);
        std::vector<float> f(v.begin(), v.end());
        return hipMemcpy(dst, f.data(), 4 * f.size(), hipMemcpyHostToDevice);
    };
    SCHK(hipMemcpy(h->d_desc.p, h->desc.data(), sizeof(wdd::SubDesc) * L, hipMemcpyHostToDevice));
    for (auto& B : h->pb) {
        if (!B.present) continue;
        const size_t bs = (&B == &h->pb[1]) ? 4 : 8;
        SCHK(up_real(B.coef.p, alpha, bs));
        SCHK(up_real(B.coef.p + bs * nn, betaX, bs));
        SCHK(up_real(B.coef.p + 2 * bs * nn, betaY, bs));
        SCHK(up_real(B.coef.p + 3 * bs * nn, beta, bs));
        SCHK(up_real(B.tab.p, kap, bs));
        SCHK(up_real(B.tab.p + bs * h->tab_len, kaph, bs));
        SCHK(up_real(B.tab.p + 2 * bs * h->tab_len, cs, bs));
        SCHK(up_real(B.tab.p + 3 * bs * h->tab_len, sn, bs));
        SCHK(hipMemset(B.F.p, 0, 2 * bs * nn));
    }
    SCHK(hipMemcpy(h->d_w1d.p, w1d.data(), 8 * w1d.size(), hipMemcpyHostToDevice));
    SCHK(hipMemcpy(h->d_kside.p, kside.data(), 8 * kside.size(), hipMemcpyHostToDevice));
    SCHK(hipMemcpy(h->d_area.p, area.data(), 8 * area.size(), hipMemcpyHostToDevice));
    SCHK(hipMemcpy(h->d_gidx.p, gidx.data(), 4 * gidx.size(), hipMemcpyHostToDevice));
    SCHK(hipMemcpy(h->d_is_iface.p, is_iface.data(), 4 * is_iface.size(), hipMemcpyHostToDevice));
    SCHK(hipMemcpy(h->d_trace_idx.p, trace_idx.data(), 8 * trace_idx.size(), hipMemcpyHostToDevice));
    SCHK(hipMemcpy(h->d_wxg.p, wxg.data(), 8 * (size_t)Nx, hipMemcpyHostToDevice));
    SCHK(hipMemcpy(h->d_wyg.p, wyg.data(), 8 * (size_t)Ny, hipMemcpyHostToDevice));
    SCHK(hipMemcpy(h->d_Mg.p, Mg.data(), 8 * (size_t)N, hipMemcpyHostToDevice));
    SCHK(hipMemcpy(h->d_Hg.p, Hg.data(), 8 * (size_t)N, hipMemcpyHostToDevice));
    SCHK(hipMemset(h->d_u.p, 0, sizeof(double2) * nn));
    SCHK(hipMemset(h->d_G.p, 0, sizeof(double2) * h->n_if));
    SCHK(hipMemset(h->d_g0.p, 0, sizeof(double2) * h->n_if));
#undef SCHK
    if (o.layout == DD_LAYOUT_AUTO) {
        const int rc = autotune_layout(h);
        if (rc != DD_OK) {
            dd_destroy(h);
            return rc;
        }
    }
    *out = h;
    return DD_OK;
}

int dd_sizes(const dd_handle* h, int64_t* n_global, int64_t* n_local, int64_t* n_sub,
             int64_t* n_iface, int64_t* n_trace) {
    CHK(validate_handle(h));
    if (n_global) *n_global = h->N;
    if (n_local) *n_local = h->nloc;
    if (n_sub) *n_sub = h->L;
    if (n_iface) *n_iface = h->n_if;
    if (n_trace) *n_trace = h->n_trace;
    return DD_OK;
}

int dd_node_coords(const dd_handle* h, double* x, double* y) {
    CHK(validate_handle(h));
    if (!x || !y) return fail(DD_EINVAL, "null output");
    const int P = h->P;
    std::vector<double> xs(h->Nx), ys(h->Ny);
    for (int e = 0; e < h->mesh.nx; ++e)
        for (int a = 0; a <= P; ++a)
            xs[e * P + a] = h->mesh.x0 + e * h->hx + 0.5 * h->hx * (h->gll.x[a] + 1.0);
    xs[h->Nx - 1] = h->mesh.x1;
    for (int e = 0; e < h->mesh.ny; ++e)
        for (int a = 0; a <= P; ++a)
            ys[e * P + a] = h->mesh.y0 + e * h->hy + 0.5 * h->hy * (h->gll.x[a] + 1.0);
    ys[h->Ny - 1] = h->mesh.y1;
    for (int j = 0; j < h->Ny; ++j)
        for (int i = 0; i < h->Nx; ++i) {
            x[(int64_t)j * h->Nx + i] = xs[i];
            y[(int64_t)j * h->Nx + i] = ys[j];
        }
    return DD_OK;
}

int dd_time_steps(const dd_handle* h, int* nt) {
    CHK(validate_handle(h));
    if (!nt) return fail(DD_EINVAL, "null output");
    std::copy(h->nt.begin(), h->nt.end(), nt);
    return DD_OK;
}

int dd_layout(const dd_handle* h, int* layout, int* wg) {
    CHK(validate_handle(h));
    if (layout) *layout = h->layout;
    if (wg) *wg = h->wg;
    return DD_OK;
}

int dd_solve_device(dd_handle* h, void* stream, const double* d_f_re, const double* d_f_im,
                    const double* d_g_re, const double* d_g_im, double tol, int max_iter,
                    double* d_u_re, double* d_u_im, double* d_u_sub, dd_stats* st) {
    CHK(validate_handle(h));
    if (!(tol >= 0.0) || max_iter < 1) return fail(DD_EINVAL, "tol must be >= 0 and max_iter >= 1");
    if (!d_u_re || !d_u_im) return fail(DD_EINVAL, "null output");
    const auto t0 = std::chrono::steady_clock::now();
    HIPCHK(hipSetDevice(h->dev));
    hipStream_t user = (hipStream_t)stream;
    hipEvent_t dep = nullptr;
    if (user) {
        HIPCHK(hipEventCreateWithFlags(&dep, hipEventDisableTiming));
        HIPCHK(hipEventRecord(dep, user));
        HIPCHK(hipStreamWaitEvent(h->stream, dep, 0));
    }
    reset_stats(h);
    const bool with_f = d_f_re != nullptr;
    if (with_f) CHK(stage_source(h, d_f_re, d_f_im));
    HIPCHK(wdd::embed_trace(d_g_re, d_g_im, h->d_trace_idx.p, h->n_if, h->d_g0.p, h->stream));
    const int rc = solve_core(h, with_f, tol, max_iter);
    if (rc != DD_OK) {
        if (dep) (void)hipEventDestroy(dep);
        return rc;
    }
    HIPCHK(wdd::glue_solution(h->d_u.p, h->Nx, h->Ny, h->P, h->mx, h->my, h->part.sx, h->part.sy,
                              h->nloc, d_u_re, d_u_im, h->stream));
    if (d_u_sub)
        HIPCHK(hipMemcpyAsync(d_u_sub, h->d_u.p, sizeof(double2) * h->L * h->nloc,
                              hipMemcpyDeviceToDevice, h->stream));
    if (user) {
        HIPCHK(hipEventRecord(dep, h->stream));
        HIPCHK(hipStreamWaitEvent(user, dep, 0));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    if (dep) (void)hipEventDestroy(dep);
    h->st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = h->st;
    if (h->st.rel_residual > tol || h->st.true_rel_residual > tol)
        return fail(DD_ENOTCONV, "outer iteration stopped at %d iterations, residual %.3e > %.3e",
                    h->st.outer_iters, std::max(h->st.rel_residual, h->st.true_rel_residual), tol);
    return DD_OK;
}

int dd_solve(dd_handle* h, const double* f_re, const double* f_im, const double* g_re,
             const double* g_im, double tol, int max_iter, double* u_re, double* u_im,
             dd_stats* st) {
    CHK(validate_handle(h));
    if (!u_re || !u_im) return fail(DD_EINVAL, "null output");
    if (!(tol >= 0.0) || max_iter < 1) return fail(DD_EINVAL, "tol must be >= 0 and max_iter >= 1");
    if (!f_re && f_im) return fail(DD_EINVAL, "f_im given without f_re");
    CHK(check_finite(f_re, h->N, "f_re"));
    CHK(check_finite(f_im, h->N, "f_im"));
    CHK(check_finite(g_re, h->n_trace, "g_re"));
    CHK(check_finite(g_im, h->n_trace, "g_im"));
    HIPCHK(hipSetDevice(h->dev));
    const auto t0 = std::chrono::steady_clock::now();
    CHK(ensure_staging(h));
    if (f_re) HIPCHK(hipMemcpy(h->d_fre.p, f_re, 8 * h->N, hipMemcpyHostToDevice));
    if (f_im) HIPCHK(hipMemcpy(h->d_fim.p, f_im, 8 * h->N, hipMemcpyHostToDevice));
    if (g_re) HIPCHK(hipMemcpy(h->d_gre.p, g_re, 8 * h->n_trace, hipMemcpyHostToDevice));
    if (g_im) HIPCHK(hipMemcpy(h->d_gim.p, g_im, 8 * h->n_trace, hipMemcpyHostToDevice));
    dd_stats s{};
    const int rc = dd_solve_device(h, nullptr, f_re ? h->d_fre.p : nullptr,
                                   f_im ? h->d_fim.p : nullptr, g_re ? h->d_gre.p : nullptr,
                                   g_im ? h->d_gim.p : nullptr, tol, max_iter, h->d_ure.p,
                                   h->d_uim.p, nullptr, &s);
    if (rc != DD_OK && rc != DD_ENOTCONV) return rc;
    const std::string msg = g_err;
    HIPCHK(hipMemcpy(u_re, h->d_ure.p, 8 * h->N, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(u_im, h->d_uim.p, 8 * h->N, hipMemcpyDeviceToHost));
    s.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = s;
    if (rc == DD_ENOTCONV) g_err = msg;
    return rc;
}

int dd_sweep(dd_handle* h, const double* g_re, const double* g_im, const double* f_re,
             const double* f_im, double src, double* g_out_re, double* g_out_im, double* u_re,
             double* u_im, int* wh_iters) {
    CHK(validate_handle(h));
    if (!g_out_re || !g_out_im) return fail(DD_EINVAL, "null output");
    if (!std::isfinite(src)) return fail(DD_EINVAL, "src must be finite");
    if (!f_re && f_im) return fail(DD_EINVAL, "f_im given without f_re");
    CHK(check_finite(g_re, h->n_if, "g_re"));
    CHK(check_finite(g_im, h->n_if, "g_im"));
    CHK(check_finite(f_re, h->N, "f_re"));
    CHK(check_finite(f_im, h->N, "f_im"));
    HIPCHK(hipSetDevice(h->dev));
    CHK(ensure_staging(h));
    reset_stats(h);
    std::vector<double2> gi(h->n_if);
    for (int64_t i = 0; i < h->n_if; ++i)
        gi[i] = make_double2(g_re ? g_re[i] : 0.0, g_im ? g_im[i] : 0.0);
    HIPCHK(hipMemcpy(h->d_g0.p, gi.data(), sizeof(double2) * h->n_if, hipMemcpyHostToDevice));
    const bool with_f = f_re != nullptr;
    if (with_f) {
        HIPCHK(hipMemcpy(h->d_fre.p, f_re, 8 * h->N, hipMemcpyHostToDevice));
        if (f_im)
            HIPCHK(hipMemcpy(h->d_fim.p, f_im, 8 * h->N, hipMemcpyHostToDevice));
        else
            HIPCHK(hipMemset(h->d_fim.p, 0, 8 * h->N));
        CHK(stage_source(h, h->d_fre.p, h->d_fim.p));
    }
    CHK(run_sweep(h, h->d_g0.p, h->d_tmp.p, src, with_f, true));
    HIPCHK(hipMemcpy(gi.data(), h->d_tmp.p, sizeof(double2) * h->n_if, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < h->n_if; ++i) {
        g_out_re[i] = gi[i].x;
        g_out_im[i] = gi[i].y;
    }
    if (u_re || u_im) {
        std::vector<double2> u(h->L * h->nloc);
        HIPCHK(hipMemcpy(u.data(), h->d_u.p, sizeof(double2) * u.size(), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < u.size(); ++i) {
            if (u_re) u_re[i] = u[i].x;
            if (u_im) u_im[i] = u[i].y;
        }
    }
    if (wh_iters) std::copy(h->iters_host.begin(), h->iters_host.end(), wh_iters);
    return DD_OK;
}

int dd_apply_stiffness(dd_handle* h, const double* p, double* q) {
    CHK(validate_handle(h));
    if (!p || !q) return fail(DD_EINVAL, "null array");
    CHK(check_finite(p, h->L * h->nloc, "p"));
    HIPCHK(hipSetDevice(h->dev));
    const int64_t n = h->L * h->nloc;
    const size_t rs = real_size(h);
    DBuf<char> dp, dq;
    hipError_t e = dp.alloc(rs * n);
    if (e == hipSuccess) e = dq.alloc(rs * n);
    if (e == hipSuccess) {
        if (rs == 8) {
            e = hipMemcpy(dp.p, p, 8 * n, hipMemcpyHostToDevice);
        } else {
            std::vector<float> f(p, p + n);
            e = hipMemcpy(dp.p, f.data(), 4 * n, hipMemcpyHostToDevice);
        }
    }
    if (e == hipSuccess) {
        if (rs == 8) {
            auto a = make_args<double>(h, h->d_g0.p, h->d_tmp.p, 0.0, false, 0.0, 1);
            double* x = (double*)dp.p;
            double* y = (double*)dq.p;
            e = h->layout == DD_LAYOUT_NODE    ? wdd::launch_apply_node<double>(a, h->P, h->wg, x, y, h->stream)
                : h->layout == DD_LAYOUT_PATCH ? wdd::launch_apply_patch1<double>(a, h->P, h->wg, x, y, h->stream)
                                               : wdd::launch_apply_patch<double>(a, h->P, h->wg, x, y, h->stream);
        } else {
            auto a = make_args<float>(h, h->d_g0.p, h->d_tmp.p, 0.0, false, 0.0, 1);
            float* x = (float*)dp.p;
            float* y = (float*)dq.p;
            e = h->layout == DD_LAYOUT_NODE    ? wdd::launch_apply_node<float>(a, h->P, h->wg, x, y, h->stream)
                : h->layout == DD_LAYOUT_PATCH ? wdd::launch_apply_patch1<float>(a, h->P, h->wg, x, y, h->stream)
                                               : wdd::launch_apply_patch<float>(a, h->P, h->wg, x, y, h->stream);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) {
        if (rs == 8) {
            e = hipMemcpy(q, dq.p, 8 * n, hipMemcpyDeviceToHost);
        } else {
            std::vector<float> f(n);
            e = hipMemcpy(f.data(), dq.p, 4 * n, hipMemcpyDeviceToHost);
            std::copy(f.begin(), f.end(), q);
        }
    }
    dp.free();
    dq.free();
    HIPCHK(e);
    return DD_OK;
}

int dd_apply_operator_device(dd_handle* h, void* stream, const double* d_x, double* d_y) {
    CHK(validate_handle(h));
    if (!d_x || !d_y) return fail(DD_EINVAL, "null array");
    HIPCHK(hipSetDevice(h->dev));
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    HIPCHK(wdd::launch_operator(op_args(h), (const double2*)d_x, (double2*)d_y, s));
    return DD_OK;
}

int dd_residual(dd_handle* h, const double* u_re, const double* u_im, const double* f_re,
                const double* f_im, const double* g_re, const double* g_im, double* rel) {
    CHK(validate_handle(h));
    if (!u_re || !u_im || !rel) return fail(DD_EINVAL, "null array");
    CHK(check_finite(u_re, h->N, "u_re"));
    CHK(check_finite(u_im, h->N, "u_im"));
    HIPCHK(hipSetDevice(h->dev));
    CHK(ensure_staging(h));
    const int64_t N = h->N;
    std::vector<double2> u(N);
    for (int64_t i = 0; i < N; ++i) u[i] = make_double2(u_re[i], u_im[i]);
    double2* du = h->d_work.p;
    double2* out = h->d_work.p + N;
    HIPCHK(hipMemcpy(du, u.data(), sizeof(double2) * N, hipMemcpyHostToDevice));
    if (f_re) HIPCHK(hipMemcpy(h->d_fre.p, f_re, 8 * N, hipMemcpyHostToDevice));
    if (f_im) HIPCHK(hipMemcpy(h->d_fim.p, f_im, 8 * N, hipMemcpyHostToDevice));
    if (g_re) HIPCHK(hipMemcpy(h->d_gre.p, g_re, 8 * h->n_trace, hipMemcpyHostToDevice));
    if (g_im) HIPCHK(hipMemcpy(h->d_gim.p, g_im, 8 * h->n_trace, hipMemcpyHostToDevice));
    HIPCHK(wdd::launch_residual(op_args(h), du, f_re ? h->d_fre.p : nullptr,
                                f_im ? h->d_fim.p : nullptr, g_re ? h->d_gre.p : nullptr,
                                g_im ? h->d_gim.p : nullptr, out, h->stream));
    HIPCHK(wdd::blas_sum2(h->blas, out, N, h->stream));
    double2 r;
    HIPCHK(hipMemcpyAsync(&r, h->blas.result, sizeof(double2), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    *rel = r.y > 0.0 ? std::sqrt(r.x / r.y) : std::sqrt(r.x);
    return DD_OK;
}

int dd_get_state(const dd_handle* h, double* G) {
    CHK(validate_handle(h));
    if (!G) return fail(DD_EINVAL, "null array");
    HIPCHK(hipMemcpy(G, h->d_G.p, sizeof(double2) * h->n_if, hipMemcpyDeviceToHost));
    return DD_OK;
}

int dd_set_state(dd_handle* h, const double* G) {
    CHK(validate_handle(h));
    if (!G) return fail(DD_EINVAL, "null array");
    CHK(check_finite(G, 2 * h->n_if, "G"));
    HIPCHK(hipMemcpy(h->d_G.p, G, sizeof(double2) * h->n_if, hipMemcpyHostToDevice));
    h->has_state = true;
    return DD_OK;
}

int dd_time_sweep(dd_handle* h, int reps, int fixed_iters, double* ms, double* dof_updates) {
    CHK(validate_handle(h));
    if (reps < 1 || !ms || fixed_iters < 0) return fail(DD_EINVAL, "reps must be >= 1, fixed_iters >= 0, ms non-null");
    HIPCHK(hipSetDevice(h->dev));
    const double tau = h->opt.tau_in;
    const int mwh = h->opt.max_wh;
    if (fixed_iters > 0) {
        h->opt.tau_in = 0.0;
        h->opt.max_wh = fixed_iters;
    }
    reset_stats(h);
    int rc = run_sweep(h, h->d_G.p, h->d_tmp.p, 0.0, false, false);
    if (rc == DD_OK) {
        reset_stats(h);
        for (int r = 0; r < reps && rc == DD_OK; ++r)
            rc = run_sweep(h, h->d_G.p, h->d_tmp.p, 0.0, false, true);
    }
    h->opt.tau_in = tau;
    h->opt.max_wh = mwh;
    if (rc != DD_OK) return rc;
    *ms = h->st.sweep_seconds * 1e3 / reps;
    if (dof_updates) *dof_updates = h->st.dof_updates / reps;
    return DD_OK;
}

}  // extern "C"
