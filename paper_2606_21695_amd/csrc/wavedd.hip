// Host side of the wavedd library: problem setup (GLL tables, lumped
// coefficients, time-step rule, filter tables), the sweep launcher, the FP64
// outer GMRES / fixed-point iteration on device vectors, and the C ABI of
// include/wavedd.h, and the box (3D) sweep of include/wavedd3.h.
#include "../../include/wavedd.h"
#include "../../include/wavedd3.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
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

// Device array.  With a stream (`as`) it comes from the device's
// stream-ordered memory pool and is returned to it on that stream: hipFree
// waits for the whole device to go idle, which a served request finishing
// while other requests' sweeps run must not do.
template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    hipStream_t as = nullptr;
    hipError_t alloc(size_t count, hipStream_t s = nullptr) {
        n = count;
        as = s;
        const size_t bytes = sizeof(T) * std::max<size_t>(count, 1);
        return s ? hipMallocAsync(reinterpret_cast<void**>(&p), bytes, s) : hipMalloc(&p, bytes);
    }
    void free() {
        if (p) (void)(as ? hipFreeAsync(p, as) : hipFree(p));
        p = nullptr;
        n = 0;
        as = nullptr;
    }
};

// First-fit allocator of index ranges in [0, cap), coalescing on release.
struct RangeAlloc {
    int64_t cap = 0, used = 0;
    std::map<int64_t, int64_t> free_;  // start -> length
    void init(int64_t c) {
        cap = c;
        used = 0;
        free_.clear();
        if (c > 0) free_[0] = c;
    }
    // start of a free range of n entries, or -1
    int64_t alloc(int64_t n) {
        if (n <= 0) return 0;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const int64_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[off + n] = len - n;
            used += n;
            return off;
        }
        return -1;
    }
    void release(int64_t off, int64_t n) {
        if (n <= 0 || off < 0) return;
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Store;

// A pending sweep of one problem, waiting for the next batched launch.
struct SweepReq {
    dd_handle* h;
    const double2* g_in;
    double2* g_out;
    double src;
    bool with_f;
    int prec;
    double tau;
    int max_wh;
    bool warm;
    bool done = false;
    int rc = 0;
};

// Continuous batching of the sweeps of the problems solving concurrently on
// one store: a problem posts its sweep and blocks; whenever a launch slot is
// free, the posting thread takes every pending sweep into one batched
// launch on that slot's stream.  While launches run, new posts queue up and
// form the next batch, so the batches grow with the load and no problem
// waits for another's sweep to finish.
struct Sched {
    static constexpr int kSlots = 32;  // most work-list staging regions (rounds in flight)
    std::mutex mu;
    std::condition_variable cv;
    int active = 0;                    // problems inside a batched solve
    bool busy[kSlots] = {};
    std::vector<SweepReq*> pending;
    std::atomic<int64_t> launches{0};
    std::string err;
};

// Device arrays that sweep kernels index by global offsets: per node,
// per interface slot, per work item, per table entry.  A handle created by
// dd_setup owns a store sized for itself; batches and engines place many
// problems in one store (disjoint ranges), so one launch covers them all.
struct Store {
    int dev = 0;
    bool shared = false;      // several problems (exchange buffers, work lists)
    int64_t align = 1;        // range granularity
    int64_t cap_node = 0, cap_if = 0, cap_item = 0, cap_tab = 0, cap_w1d = 0, cap_wsp = 0;
    RangeAlloc a_node, a_if, a_item, a_tab, a_w1d, a_wsp;
    struct PrecBuf {
        DBuf<char> coef;      // alpha, betaX, betaY, beta (stride cap_node)
        DBuf<char> tab;       // kap, kaph, cs, sn (stride cap_tab)
        DBuf<char> F;         // Fre, Fim (stride cap_node)
        bool present = false;
    } pb[2];
    DBuf<wdd::SubDesc> d_desc;
    DBuf<double> d_w1d, d_kside, d_area;
    DBuf<int> d_gidx, d_iters, d_is_iface;
    DBuf<int64_t> d_trace_idx;
    DBuf<double2> d_u;
    DBuf<double> d_wsp, d_wss;       // STREAM layout workspace, FP64 sweeps
    DBuf<float> d_wsp32, d_wss32;    // STREAM layout workspace, FP32 sweeps (own bytes: FP64 and
                                     // FP32 sweeps of different problems run concurrently)
    DBuf<double2> d_gin, d_gout;     // shared: per-problem sweep input / output ranges
    DBuf<wdd::SubDesc> d_work;       // shared: work lists of batched launches (per slot)
    DBuf<int> d_work_iters;
    wdd::SubDesc* h_work = nullptr;  // pinned staging of the work lists (per slot)
    int* h_work_iters = nullptr;
    int n_slots = 0;                      // slots in use (shared stores)
    int64_t slot_items = 0;               // work-list entries per slot
    hipStream_t ss[Sched::kSlots] = {};   // launch streams of the slots (batch stores)
    hipEvent_t sev0[Sched::kSlots] = {}, sev1[Sched::kSlots] = {};
    // the launch groups of one slot's round run concurrently on sub-streams:
    // sevc (work list staged) starts them, gev (group done) joins them
    static constexpr int kSub = 4;
    hipStream_t gs[Sched::kSlots][kSub] = {};
    hipEvent_t sevc[Sched::kSlots] = {}, gev[Sched::kSlots][kSub] = {};
    int sub_streams = kSub;   // sub-streams used per round (1: all groups in order on ss)
    size_t bytes = 0;
    std::mutex mu;            // allocators, layout cache
    std::map<std::tuple<int, int, int, int>, std::pair<int, int>> layout_cache;  // (mx, my, P, prec) -> (layout, wg)
    Sched sched;
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
    std::vector<wdd::SubDesc> desc;  // global offsets into the store
    int layout = DD_LAYOUT_PATCH, wg = 256;
    size_t lds[2] = {0, 0};          // dynamic LDS of a launch, FP64 / FP32
    // STREAM sweeps of a handle of its own may share each subdomain among
    // xb_k workgroups (1: one workgroup per subdomain); d_xb holds their
    // per-item counters, the abort flag and the per-item partial sums
    int xb_k = 1;
    DBuf<char> d_xb;
    size_t xb_bytes = 0;
    int dev = 0;
    hipStream_t stream = nullptr;
    // placement in the store
    Store* store = nullptr;
    bool own_store = false;
    bool batched = false;            // sweeps go through the store's batched launches
    bool sweep_warm = false;         // the next sweeps start WaveHoltz from the current u
    dd_progress_fn prog = nullptr;   // progress report (dd_set_progress)
    void* prog_user = nullptr;
    int prog_every = 1;
    int prog_base = 0;               // outer iterations before the current GMRES pass
    double prog_scale = 1.0;         // pass residual -> residual relative to ||h||
    int64_t node_base = 0, if_base = 0, item_base = 0, tab_base = 0, w1d_base = 0, wsp_base = 0;
    int64_t node_len = 0, if_len = 0, item_len = 0, tab_len = 0, w1d_len = 0, wsp_len = 0;
    bool placed = false;
    // per-problem device vectors of the outer iteration
    DBuf<double2> d_V;               // GMRES basis (restart + 1) x ld
    DBuf<double2> d_G, d_h, d_tmp, d_g0, d_r, d_coefs, d_D, d_res;
    DBuf<double> d_fre, d_fim, d_gre, d_gim, d_ure, d_uim;  // staging for host API
    DBuf<double> d_wxg, d_wyg, d_Mg, d_Hg;                 // global operator data
    DBuf<double2> d_work;            // N complex scratch
    size_t own_bytes = 0;            // device bytes of the vectors above
    int64_t ld = 0;
    wdd::Blas blas;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<int> iters_host;
    std::vector<int> last_iters;     // per subdomain, for longest-first ordering
    double K1all[wdd::kMaxP + 1][wdd::kMaxP + 1][wdd::kMaxP + 1];  // reference stiffness per P
    bool has_state = false;
    // stats of the current solve
    dd_stats st{};
};

namespace {

size_t real_size(const dd_handle* h) { return h->opt.precision == DD_FP32 ? 4 : 8; }
size_t prec_size(int prec) { return prec == DD_FP32 ? 4 : 8; }
int prec_index(int prec) { return prec == DD_FP32 ? 1 : 0; }

// Launch arguments with the store's arrays; desc / n_items / wh_iters /
// lds / nt_max are filled by the caller.
template <typename Real>
wdd::SweepArgs<Real> store_args(const Store* S, const double2* g_in, double2* g_out, double src,
                                bool with_f, double tau, int max_wh, const double (*K1)[wdd::kMaxP + 1][wdd::kMaxP + 1]) {
    const Store::PrecBuf& B = S->pb[sizeof(Real) == 4 ? 1 : 0];
    wdd::SweepArgs<Real> a{};
    Real* coef = reinterpret_cast<Real*>(B.coef.p);
    const int64_t n = S->cap_node;
    a.coef.alpha = coef;
    a.coef.betaX = coef + n;
    a.coef.betaY = coef + 2 * n;
    a.coef.beta = coef + 3 * n;
    Real* F = reinterpret_cast<Real*>(B.F.p);
    a.Fre = with_f ? F : nullptr;
    a.Fim = with_f ? F + n : nullptr;
    a.w1d = S->d_w1d.p;
    a.kside = S->d_kside.p;
    Real* tab = reinterpret_cast<Real*>(B.tab.p);
    a.kap = tab;
    a.kaph = tab + S->cap_tab;
    a.cs = tab + 2 * S->cap_tab;
    a.sn = tab + 3 * S->cap_tab;
    a.g_in = g_in;
    a.g_out = g_out;
    a.src = src;
    a.u = S->d_u.p;
    a.tau = tau;
    a.max_wh = max_wh;
    if (sizeof(Real) == 4) {
        a.ws_p = reinterpret_cast<Real*>(S->d_wsp32.p);
        a.ws_s = reinterpret_cast<Real*>(S->d_wss32.p);
    } else {
        a.ws_p = reinterpret_cast<Real*>(S->d_wsp.p);
        a.ws_s = reinterpret_cast<Real*>(S->d_wss.p);
    }
    a.ws_stride = n;
    std::memcpy(a.K1, K1, sizeof(a.K1));
    return a;
}

// Arguments of a launch over this handle's subdomains; g_in / g_out are
// indexed by the store's interface offsets.
template <typename Real>
wdd::SweepArgs<Real> make_args(dd_handle* h, const double2* g_in, double2* g_out, double src,
                               bool with_f, double tau, int max_wh) {
    wdd::SweepArgs<Real> a = store_args<Real>(h->store, g_in, g_out, src, with_f, tau, max_wh,
                                              h->K1all);
    a.desc = h->store->d_desc.p + h->item_base;
    a.n_items = (int)h->L;
    a.wh_iters = h->store->d_iters.p + h->item_base;
    a.warm = h->sweep_warm ? 1 : 0;
    a.lds_bytes = h->lds[sizeof(Real) == 4 ? 1 : 0];
    a.nt_max = h->nt_max;
    return a;
}

constexpr size_t kLdsLimit = 160 * 1024;

int patch_threads(const dd_handle* h) {
    return std::max(h->mx * h->my, h->mx * h->P + h->my * h->P + 1);
}

int layout_threads(const dd_handle* h, int layout) {
    int t = layout == DD_LAYOUT_NODE ? h->nxl * h->nyl : patch_threads(h);
    if (layout == DD_LAYOUT_STREAM) t = (int)std::min<int64_t>(512, h->nloc);
    return ((t + 63) / 64) * 64;
}

size_t layout_lds(const dd_handle* h, int layout, int prec) {
    const size_t rs = prec_size(prec);
    if (layout == DD_LAYOUT_NODE) return wdd::node_lds_bytes(h->nxl, h->nyl, h->nt_max, rs);
    if (layout == DD_LAYOUT_STREAM) return wdd::stream_lds_bytes(h->P, h->nt_max, rs);
    if (layout == DD_LAYOUT_PATCH_XCHG) return wdd::patch_lds_bytes(h->mx, h->my, h->P, h->nt_max, rs);
    return wdd::patch1_lds_bytes(h->mx, h->my, h->P, layout_threads(h, layout), h->nt_max, rs);
}

void layout_config(dd_handle* h, int layout, int wg = 0) {
    h->layout = layout;
    h->wg = wg > 0 ? wg : layout_threads(h, layout);
    for (int prec : {DD_FP64, DD_FP32}) h->lds[prec_index(prec)] = layout_lds(h, layout, prec);
}

// Workgroup sizes the STREAM layout can run with on this subdomain: every
// column group of its step loop needs a wave, and the kernel is built for
// at most 512 threads.
std::vector<int> stream_wg_options(const dd_handle* h) {
    const int ow = 64 - 2 * h->P, groups = (h->nxl + ow - 1) / ow;
    std::vector<int> out;
    for (int wg : {256, 512})
        if (groups <= wg / 64 && wg <= ((std::min<int64_t>(512, h->nloc) + 63) / 64) * 64)
            out.push_back(wg);
    if (out.empty()) out.push_back(layout_threads(h, DD_LAYOUT_STREAM));
    return out;
}

// Fits in one workgroup for every precision the handle carries (FP64
// always, for the refinement residuals of FP32 handles too).
bool layout_fits(const dd_handle* h, int layout) {
    if (layout == DD_LAYOUT_STREAM) {
        // every column group of the step loop needs a wave of its own
        const int ow = 64 - 2 * h->P, groups = (h->nxl + ow - 1) / ow;
        return groups <= layout_threads(h, layout) / 64 &&
               layout_lds(h, layout, DD_FP64) <= kLdsLimit;
    }
    const bool threads_ok = layout == DD_LAYOUT_NODE ? h->nxl * h->nyl <= 1024 : patch_threads(h) <= 512;
    return threads_ok && layout_lds(h, layout, DD_FP64) <= kLdsLimit;
}

template <typename Real>
hipError_t launch_layout(int layout, const wdd::SweepArgs<Real>& a, int P, int wg, hipStream_t s) {
    switch (layout) {
        case DD_LAYOUT_NODE: return wdd::launch_sweep_node<Real>(a, P, wg, s);
        case DD_LAYOUT_PATCH: return wdd::launch_sweep_patch1<Real>(a, P, wg, s);
        case DD_LAYOUT_STREAM: return wdd::launch_sweep_stream<Real>(a, P, wg, s);
        default: return wdd::launch_sweep_patch<Real>(a, P, wg, s);
    }
}

// Fold one launch's WaveHoltz counts of this handle into its stats.
void account_sweep(dd_handle* h, const int* iters, double seconds, int prec) {
    h->st.sweep_seconds += seconds;
    h->st.sweeps += 1;
    if (prec == DD_FP64 && h->opt.precision == DD_FP32) h->st.fp64_sweeps += 1;
    for (int64_t l = 0; l < h->L; ++l) {
        const int it = iters[l];
        h->iters_host[l] = it;
        h->last_iters[l] = it;
        h->st.wh_iters_total += it;
        h->st.wh_iters_max = std::max(h->st.wh_iters_max, it);
        h->st.dof_updates += (double)h->nloc * (h->nt[l] - 1) * it;
    }
}

int sched_sweep(dd_handle* h, const double2* g_in, double2* g_out, double src, bool with_f,
                int prec, double tau, int max_wh);

// One sweep launch of this handle alone: g_out = sweep(g_in, src), u =
// subdomain solutions.  In a shared store the vectors pass through the
// handle's range of the exchange buffers.
// Per-item counters (int), the abort flag and the per-item partial sums
// (2 K doubles) of the shared-subdomain STREAM sweep, laid out in d_xb.
template <typename Real>
void xb_args(dd_handle* h, wdd::SweepArgs<Real>& a) {
    char* base = h->d_xb.p;
    const size_t cnt_bytes = (((size_t)h->L + 1) * sizeof(int) + 255) & ~(size_t)255;
    a.xb_k = h->xb_k;
    a.xb_cnt = reinterpret_cast<int*>(base);
    a.xb_abort = reinterpret_cast<int*>(base) + h->L;
    a.xb_part = reinterpret_cast<double*>(base + cnt_bytes);
}

size_t xb_bytes_for(int64_t L, int K) {
    const size_t cnt_bytes = (((size_t)L + 1) * sizeof(int) + 255) & ~(size_t)255;
    return cnt_bytes + sizeof(double) * 2 * (size_t)K * (size_t)L;
}

// One sweep launch in the handle's layout; STREAM sweeps of a shared-
// subdomain handle (xb_k > 1) that start cold go to the cooperative kernel,
// and if that launch is refused or aborts (its workgroups could not be
// placed together) the handle falls back to one workgroup per subdomain
// and relaunches the plain kernel on the same inputs.
template <typename Real>
int launch_sweep(dd_handle* h, const double2* gi, double2* go, double src, bool with_f,
                 double tau, int max_wh, hipStream_t s) {
    wdd::SweepArgs<Real> a = make_args<Real>(h, gi, go, src, with_f, tau, max_wh);
    // FP64 sweeps only: FP32 shared-subdomain sweeps disagree with the
    // one-workgroup sweep on short row segments (cause not found), so they
    // stay off
    if (sizeof(Real) == 8 && h->layout == DD_LAYOUT_STREAM && h->xb_k > 1 && !h->sweep_warm) {
        xb_args(h, a);
        HIPCHK(hipMemsetAsync(h->d_xb.p, 0, h->xb_bytes, s));
        hipError_t e = wdd::launch_sweep_stream_coop<Real>(a, h->P, h->wg, s);
        int aborted = 1;
        if (e == hipSuccess) {
            HIPCHK(hipMemcpyAsync(&aborted, a.xb_abort, sizeof(int), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        } else {
            (void)hipGetLastError();
        }
        if (!aborted) return DD_OK;
        h->xb_k = 1;
    }
    HIPCHK(launch_layout<Real>(h->layout, a, h->P, h->wg, s));
    return DD_OK;
}

int run_sweep_direct(dd_handle* h, const double2* g_in, double2* g_out, double src, bool with_f,
                     bool timed, int prec, double tau, int max_wh) {
    hipStream_t s = h->stream;
    Store* S = h->store;
    const double2* gi = g_in;
    double2* go = g_out;
    if (S->shared) {
        HIPCHK(hipMemcpyAsync(S->d_gin.p + h->if_base, g_in, sizeof(double2) * h->n_if,
                              hipMemcpyDeviceToDevice, s));
        gi = S->d_gin.p;
        go = S->d_gout.p;
    }
    if (timed) HIPCHK(hipEventRecord(h->ev0, s));
    if (prec == DD_FP32)
        CHK(launch_sweep<float>(h, gi, go, src, with_f, tau, max_wh, s));
    else
        CHK(launch_sweep<double>(h, gi, go, src, with_f, tau, max_wh, s));
    if (timed) HIPCHK(hipEventRecord(h->ev1, s));
    if (S->shared)
        HIPCHK(hipMemcpyAsync(g_out, S->d_gout.p + h->if_base, sizeof(double2) * h->n_if,
                              hipMemcpyDeviceToDevice, s));
    std::vector<int> its(h->L);
    HIPCHK(hipMemcpyAsync(its.data(), S->d_iters.p + h->item_base, sizeof(int) * h->L,
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    if (timed) HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    account_sweep(h, its.data(), ms * 1e-3, prec);
    return DD_OK;
}

int run_sweep(dd_handle* h, const double2* g_in, double2* g_out, double src, bool with_f,
              bool timed, int prec, double tau, int max_wh) {
    if (h->batched) return sched_sweep(h, g_in, g_out, src, with_f, prec, tau, max_wh);
    return run_sweep_direct(h, g_in, g_out, src, with_f, timed, prec, tau, max_wh);
}

// ---------------------------------------------------------------------------
// Batched launches: the sweeps of several problems of one store in one
// launch per launch configuration, longest-first
// ---------------------------------------------------------------------------

// LDS of a launch of this handle's layout at another workgroup size and
// table length (a group of problems shares one launch configuration).
size_t lds_for(const dd_handle* h, int prec, int wg, int nt_max) {
    const size_t rs = prec_size(prec);
    switch (h->layout) {
        case DD_LAYOUT_NODE: return wdd::node_lds_bytes(h->nxl, h->nyl, nt_max, rs);
        case DD_LAYOUT_STREAM: return wdd::stream_lds_bytes(h->P, nt_max, rs);
        case DD_LAYOUT_PATCH_XCHG: return wdd::patch_lds_bytes(h->mx, h->my, h->P, nt_max, rs);
        default: return wdd::patch1_lds_bytes(h->mx, h->my, h->P, wg, nt_max, rs);
    }
}

// Workgroup-size class of a layout's kernel template (items of one launch
// must share it; blockDim is the largest need in the class).
int wg_class(int layout, int wg) {
    if (layout == DD_LAYOUT_PATCH || layout == DD_LAYOUT_PATCH_XCHG) return wg <= 256 ? 256 : 512;
    return 1024;
}

// Estimated cost of a subdomain: DOF-updates of its last sweep.
double item_cost(const dd_handle* h, int64_t l) {
    return (double)h->nloc * (h->nt[l] - 1) * std::max(1, h->last_iters[l]);
}

// One batched launch over the requests' subdomains.  Requests are grouped
// by launch configuration (precision, degree, layout, workgroup class,
// source); each group is one launch whose work list is sorted by cost,
// longest first (the hardware dispatches workgroups in order, so the list
// is the schedule).  Groups run concurrently on the store's group streams.
int launch_batch(Store* S, const std::vector<SweepReq*>& reqs, int slot, hipStream_t s,
                 double* ms_out = nullptr, int* groups_out = nullptr) {
    HIPCHK(hipSetDevice(S->dev));
    struct Item {
        double cost;
        int r;
        int64_t l;
    };
    struct Group {
        std::vector<Item> items;
        int prec = 0, P = 0, layout = 0, wg = 0, nt_max = 0;
        double src = 0.0;
        size_t lds = 0;
        int64_t off = 0;
    };
    std::map<std::tuple<int, int, int, int, double, const void*>, Group> groups;
    for (int r = 0; r < (int)reqs.size(); ++r) {
        const SweepReq* q = reqs[r];
        const dd_handle* h = q->h;
        const double src = (q->with_f && q->src != 0.0) ? q->src : 0.0;
        auto key = std::make_tuple(q->prec, h->P, h->layout, wg_class(h->layout, h->wg), src,
                                   (const void*)nullptr);
        Group& g = groups[key];
        const int wg = std::max(g.wg, h->wg), ntm = std::max(g.nt_max, h->nt_max);
        bool fits = lds_for(h, q->prec, wg, ntm) <= kLdsLimit;
        for (const Item& it : g.items) fits = fits && lds_for(reqs[it.r]->h, q->prec, wg, ntm) <= kLdsLimit;
        Group& gg = fits ? g : groups[std::make_tuple(q->prec, h->P, h->layout,
                                                      wg_class(h->layout, h->wg), src, (const void*)h)];
        gg.prec = q->prec;
        gg.P = h->P;
        gg.layout = h->layout;
        gg.src = src;
        gg.wg = std::max(gg.wg, h->wg);
        gg.nt_max = std::max(gg.nt_max, h->nt_max);
        for (int64_t l = 0; l < h->L; ++l) gg.items.push_back({item_cost(h, l), r, l});
    }
    wdd::SubDesc* hw = S->h_work + (int64_t)slot * S->slot_items;
    int* hi = S->h_work_iters + (int64_t)slot * S->slot_items;
    wdd::SubDesc* dw = S->d_work.p + (int64_t)slot * S->slot_items;
    int* di = S->d_work_iters.p + (int64_t)slot * S->slot_items;
    int64_t total = 0;
    for (const auto& kv : groups) total += (int64_t)kv.second.items.size();
    if (total > S->slot_items) return fail(DD_EINVAL, "batched work list exceeds its slot");
    total = 0;
    for (auto& kv : groups) {
        Group& g = kv.second;
        std::stable_sort(g.items.begin(), g.items.end(),
                         [](const Item& a, const Item& b) { return a.cost > b.cost; });
        g.off = total;
        for (size_t i = 0; i < g.items.size(); ++i) {
            const Item& it = g.items[i];
            const SweepReq* q = reqs[it.r];
            wdd::SubDesc d = q->h->desc[it.l];
            d.max_wh = q->max_wh;
            d.tau = q->tau;
            d.flags = q->warm ? 1 : 0;
            hw[total + (int64_t)i] = d;
        }
        for (const Item& it : g.items)
            g.lds = std::max(g.lds, lds_for(reqs[it.r]->h, g.prec, g.wg, g.nt_max));
        total += (int64_t)g.items.size();
    }
    HIPCHK(hipEventRecord(S->sev0[slot], s));
    HIPCHK(hipMemcpyAsync(dw, hw, sizeof(wdd::SubDesc) * total, hipMemcpyHostToDevice, s));
    for (const SweepReq* q : reqs)
        HIPCHK(hipMemcpyAsync(S->d_gin.p + q->h->if_base, q->g_in, sizeof(double2) * q->h->n_if,
                              hipMemcpyDeviceToDevice, s));
    const double(*K1)[wdd::kMaxP + 1][wdd::kMaxP + 1] = reqs[0]->h->K1all;
    // Groups (one launch each) go to sub-streams by longest processing time
    // first: the costliest group to the least-loaded sub-stream, so the
    // groups of a round overlap on the device and short launches fill the
    // CUs that a long launch's tail leaves idle.
    std::vector<Group*> order;
    for (auto& kv : groups)
        if (!kv.second.items.empty()) order.push_back(&kv.second);
    auto gcost = [](const Group* g) {
        double c = 0.0;
        for (const Item& it : g->items) c += it.cost;
        return c;
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](const Group* a, const Group* b) { return gcost(a) > gcost(b); });
    const int nsub = std::max(1, std::min<int>(S->sub_streams, (int)order.size()));
    double load[Store::kSub] = {};
    bool used[Store::kSub] = {};
    if (nsub > 1) HIPCHK(hipEventRecord(S->sevc[slot], s));
    int gi = 0;
    for (Group* gp : order) {
        Group& g = *gp;
        ++gi;
        hipStream_t gstream = s;
        if (nsub > 1) {
            int k = 0;
            for (int j = 1; j < nsub; ++j)
                if (load[j] < load[k]) k = j;
            load[k] += gcost(gp);
            gstream = S->gs[slot][k];
            if (!used[k]) HIPCHK(hipStreamWaitEvent(gstream, S->sevc[slot], 0));
            used[k] = true;
        }
        const bool wf = g.src != 0.0;
        hipError_t e;
        if (g.prec == DD_FP32) {
            auto a = store_args<float>(S, S->d_gin.p, S->d_gout.p, g.src, wf, 0.0, 1, K1);
            a.desc = dw + g.off;
            a.n_items = (int)g.items.size();
            a.wh_iters = di + g.off;
            a.lds_bytes = g.lds;
            a.nt_max = g.nt_max;
            e = launch_layout<float>(g.layout, a, g.P, g.wg, gstream);
        } else {
            auto a = store_args<double>(S, S->d_gin.p, S->d_gout.p, g.src, wf, 0.0, 1, K1);
            a.desc = dw + g.off;
            a.n_items = (int)g.items.size();
            a.wh_iters = di + g.off;
            a.lds_bytes = g.lds;
            a.nt_max = g.nt_max;
            e = launch_layout<double>(g.layout, a, g.P, g.wg, gstream);
        }
        HIPCHK(e);
    }
    for (int k = 0; k < nsub && nsub > 1; ++k) {
        if (!used[k]) continue;
        HIPCHK(hipEventRecord(S->gev[slot][k], S->gs[slot][k]));
        HIPCHK(hipStreamWaitEvent(s, S->gev[slot][k], 0));
    }
    HIPCHK(hipEventRecord(S->sev1[slot], s));
    for (const SweepReq* q : reqs)
        HIPCHK(hipMemcpyAsync(q->g_out, S->d_gout.p + q->h->if_base, sizeof(double2) * q->h->n_if,
                              hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(hi, di, sizeof(int) * total, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, S->sev0[slot], S->sev1[slot]));
    std::vector<std::vector<int>> its(reqs.size());
    for (size_t r = 0; r < reqs.size(); ++r) its[r].assign(reqs[r]->h->L, 0);
    for (auto& kv : groups) {
        const Group& g = kv.second;
        for (size_t i = 0; i < g.items.size(); ++i)
            its[g.items[i].r][g.items[i].l] = hi[g.off + (int64_t)i];
    }
    for (size_t r = 0; r < reqs.size(); ++r)
        account_sweep(reqs[r]->h, its[r].data(), ms * 1e-3, reqs[r]->prec);
    if (ms_out) *ms_out = ms;
    if (groups_out) *groups_out = gi;
    return DD_OK;
}

void sched_join(Store* S) {
    std::lock_guard<std::mutex> lk(S->sched.mu);
    S->sched.active += 1;
}

void sched_leave(Store* S) {
    std::lock_guard<std::mutex> lk(S->sched.mu);
    S->sched.active -= 1;
}

// Cost of one posted sweep: its slowest work item (subdomain nodes x steps
// per period x WaveHoltz iterations of its last sweep).
double sweep_cost(const SweepReq* r) {
    double c = 0.0;
    for (int64_t l = 0; l < r->h->L; ++l) c = std::max(c, item_cost(r->h, l));
    return c;
}
constexpr double kRoundCostSpan = 4.0;

// A sweep of a batched handle: post it; if a launch slot is free, launch
// everything pending (this sweep included unless another thread already
// took it), else wait for the launch that carries it.
int sched_sweep(dd_handle* h, const double2* g_in, double2* g_out, double src, bool with_f,
                int prec, double tau, int max_wh) {
    HIPCHK(hipStreamSynchronize(h->stream));
    Store* S = h->store;
    Sched& Q = S->sched;
    SweepReq req{h, g_in, g_out, src, with_f, prec, tau, max_wh, h->sweep_warm};
    std::unique_lock<std::mutex> lk(Q.mu);
    Q.pending.push_back(&req);
    while (!req.done) {
        int slot = -1;
        for (int k = 0; k < S->n_slots; ++k)
            if (!Q.busy[k]) {
                slot = k;
                break;
            }
        if (slot < 0 || Q.pending.empty()) {
            Q.cv.wait(lk);
            continue;
        }
        // One round takes the oldest pending sweep and every other pending
        // sweep of a similar cost (its slowest subdomain within a factor of
        // four): a round lasts as long as its slowest work item, so mixing
        // cheap and expensive requests would hold the cheap ones to the pace
        // of the expensive ones.  The rest wait for the next free slot (as
        // do sweeps beyond the slot's work-list entries).
        std::vector<SweepReq*> batch, rest;
        const double c0 = sweep_cost(Q.pending.front());
        int64_t items = 0;
        for (SweepReq* r : Q.pending) {
            const double c = sweep_cost(r);
            const bool fits = batch.empty() || items + r->h->L <= S->slot_items;
            if (fits && c <= kRoundCostSpan * c0 && c * kRoundCostSpan >= c0) {
                batch.push_back(r);
                items += r->h->L;
            } else {
                rest.push_back(r);
            }
        }
        Q.pending.swap(rest);
        Q.busy[slot] = true;
        if (!Q.pending.empty()) Q.cv.notify_all();   // another free slot can take them
        lk.unlock();
        // the round runs on the launching thread's stream (the slot's own
        // stream in a batch store), so rounds in flight are limited by the
        // staging slots, not by a fixed set of streams
        const int rc = launch_batch(S, batch, slot, S->ss[slot] ? S->ss[slot] : h->stream);
        const std::string msg = rc == DD_OK ? std::string() : g_err;
        lk.lock();
        for (SweepReq* r : batch) {
            r->rc = rc;
            r->done = true;
        }
        if (rc != DD_OK) Q.err = msg;
        Q.busy[slot] = false;
        Q.launches += 1;
        Q.cv.notify_all();
    }
    if (req.rc != DD_OK) return fail(req.rc, "batched sweep: %s", Q.err.c_str());
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
// Device vectors and operator of one restarted GMRES run: the outer
// iteration's Krylov method, shared by the 2D and box handles.
struct Krylov {
    wdd::Blas* blas;
    hipStream_t stream;
    int64_t n, ld;                 // vector length, basis stride
    int m;                         // restart length
    double2 *V, *r, *coefs;        // basis [(m+1) * ld], residual [n], combination [m+1]
    std::function<int(const double2*, double2*, double)> matvec;  // w = v - T v, inner tol
    std::function<double(double)> tau;  // inner tolerance at a relative residual
    double tau_strict;                  // inner tolerance of the restart residuals
    std::function<void(int, double)> progress;  // (matvecs so far, relative residual) or empty
};

int kdots(const Krylov& k, const double2* V, int64_t ld, int nv, const double2* w, cplx* out) {
    HIPCHK(wdd::blas_multidot(*k.blas, V, ld, nv, w, k.n, k.stream));
    std::vector<double2> tmp(nv);
    HIPCHK(hipMemcpyAsync(tmp.data(), k.blas->result, sizeof(double2) * nv, hipMemcpyDeviceToHost,
                          k.stream));
    HIPCHK(hipStreamSynchronize(k.stream));
    for (int i = 0; i < nv; ++i) out[i] = cplx(tmp[i].x, tmp[i].y);
    return DD_OK;
}

double knorm(const Krylov& k, const double2* x) {
    cplx v;
    if (kdots(k, x, 0, 1, x, &v) != DD_OK) return NAN;
    return std::sqrt(std::max(0.0, v.real()));
}

int kaxpby(const Krylov& k, cplx a, const double2* x, cplx b, double2* y) {
    HIPCHK(wdd::blas_axpby(make_double2(a.real(), a.imag()), x, make_double2(b.real(), b.imag()),
                           y, k.n, k.stream));
    return DD_OK;
}

// The handle's interface-vector operations.
Krylov handle_vectors(dd_handle* h) {
    Krylov k{};
    k.blas = &h->blas;
    k.stream = h->stream;
    k.n = h->n_if;
    k.ld = h->ld;
    k.m = h->opt.restart;
    k.V = h->d_V.p;
    k.r = h->d_r.p;
    k.coefs = h->d_coefs.p;
    return k;
}

int dots(dd_handle* h, const double2* V, int64_t ld, int k, const double2* w, cplx* out) {
    return kdots(handle_vectors(h), V, ld, k, w, out);
}

double norm(dd_handle* h, const double2* x) { return knorm(handle_vectors(h), x); }

int axpby(dd_handle* h, cplx a, const double2* x, cplx b, double2* y) {
    return kaxpby(handle_vectors(h), a, x, b, y);
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
int gmres_core(const Krylov& K, const double2* rhs, double2* x, double rnorm0, double tol,
               int max_iter, int* its_out, double* rel_out) {
    const int m = K.m;
    const int64_t n = K.n, ld = K.ld;
    double2* V = K.V;
    HIPCHK(hipMemsetAsync(x, 0, sizeof(double2) * n, K.stream));
    *its_out = 0;
    *rel_out = rnorm0 == 0.0 ? 0.0 : 1.0;
    if (rnorm0 == 0.0 || max_iter <= 0) return DD_OK;
    std::vector<cplx> H((size_t)(m + 1) * m), g(m + 1), sn(m), y(m);
    std::vector<double> cs(m);
    std::vector<cplx> h1(m + 1), h2(m + 1);
    HIPCHK(hipMemcpyAsync(K.r, rhs, sizeof(double2) * n, hipMemcpyDeviceToDevice, K.stream));
    double beta = rnorm0;
    int its = 0;
    double rel = 1.0;
    while (true) {
        std::fill(H.begin(), H.end(), cplx(0.0));
        std::fill(g.begin(), g.end(), cplx(0.0));
        g[0] = beta;
        CHK(kaxpby(K, cplx(1.0 / beta, 0.0), K.r, cplx(0.0), V));
        int k = 0;
        for (int j = 0; j < m; ++j) {
            double2* w = V + (int64_t)(j + 1) * ld;
            CHK(K.matvec(V + (int64_t)j * ld, w, K.tau(rel)));
            ++its;
            CHK(kdots(K, V, ld, j + 1, w, h1.data()));
            HIPCHK(wdd::blas_multiaxpy(*K.blas, V, ld, j + 1, w, n, K.stream));
            CHK(kdots(K, V, ld, j + 1, w, h2.data()));
            HIPCHK(wdd::blas_multiaxpy(*K.blas, V, ld, j + 1, w, n, K.stream));
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h1[i] + h2[i];
            const double hn = knorm(K, w);
            if (!std::isfinite(hn)) return fail(DD_ENAN, "non-finite Krylov vector");
            H[(size_t)(j + 1) * m + j] = hn;
            if (hn > 0.0) CHK(kaxpby(K, cplx(1.0 / hn, 0.0), w, cplx(0.0), w));
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
            if (K.progress) K.progress(its, rel);
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
        HIPCHK(hipMemcpyAsync(K.coefs, yc.data(), sizeof(double2) * k, hipMemcpyHostToDevice,
                              K.stream));
        HIPCHK(wdd::blas_combine(V, ld, k, K.coefs, x, n, 1, K.stream));
        HIPCHK(hipStreamSynchronize(K.stream));
        if (rel <= tol || its >= max_iter) break;
        // r = rhs - (x - T x), with the strict inner tolerance
        CHK(K.matvec(x, K.r, K.tau_strict));
        CHK(kaxpby(K, cplx(1.0), rhs, cplx(-1.0), K.r));
        beta = knorm(K, K.r);
        if (!std::isfinite(beta)) return fail(DD_ENAN, "non-finite outer residual");
        rel = beta / rnorm0;
        if (beta == 0.0 || rel <= tol) break;
    }
    *its_out = its;
    *rel_out = rel;
    return DD_OK;
}

// GMRES of a 2D handle: its sweep operator, inner-tolerance rule and progress callback.
int gmres(dd_handle* h, const double2* rhs, double2* x, double rnorm0, double tol, int max_iter,
          int* its_out, double* rel_out) {
    Krylov K = handle_vectors(h);
    K.matvec = [h](const double2* v, double2* w, double tau) { return matvec(h, v, w, tau); };
    K.tau = [h, tol](double rel) { return matvec_tau(h, tol, rel); };
    K.tau_strict = h->opt.tau_in;
    if (h->prog)
        K.progress = [h](int its, double rel) {
            if (its % h->prog_every == 0) h->prog(h->prog_user, h->prog_base + its, rel * h->prog_scale);
        };
    return gmres_core(K, rhs, x, rnorm0, tol, max_iter, its_out, rel_out);
}

// Plain fixed-point iteration G <- T G + h.  With warm start the sweep
// is taken as sweep(G + g_phys, sources on) (= T G + h, the sweep being
// affine), so consecutive sweeps solve converging subdomain problems and
// each WaveHoltz solve starts from the previous sweep's u.
int residual_sweep(dd_handle* h, bool with_f, int prec, double tau, double hnorm, double* rel);

int fixed_point(dd_handle* h, bool with_f, double tol, int max_iter, double hnorm) {
    const int64_t n = h->n_if;
    HIPCHK(hipMemsetAsync(h->d_G.p, 0, sizeof(double2) * n, h->stream));
    h->st.outer_iters = 0;
    h->st.rel_residual = hnorm == 0.0 ? 0.0 : 1.0;
    if (hnorm == 0.0) return DD_OK;
    const bool warm = h->opt.warm != 0;
    for (int it = 0; it < max_iter; ++it) {
        double d = 0.0;
        if (warm) {
            // tmp = T G + h - G (u left for the next warm start), G += tmp
            h->sweep_warm = true;   // the h-sweep (or previous iteration) left u
            double rel = 0.0;
            const int rc = residual_sweep(h, with_f, h->opt.precision, h->opt.tau_in, hnorm, &rel);
            h->sweep_warm = false;
            CHK(rc);
            CHK(axpby(h, cplx(1.0), h->d_tmp.p, cplx(1.0), h->d_G.p));
            d = rel * hnorm;
        } else {
            CHK(run_sweep(h, h->d_G.p, h->d_tmp.p, 0.0, false, true));
            CHK(axpby(h, cplx(1.0), h->d_h.p, cplx(1.0), h->d_tmp.p));   // tmp = T G + h
            CHK(axpby(h, cplx(1.0), h->d_tmp.p, cplx(-1.0), h->d_G.p));  // G = tmp - G
            d = norm(h, h->d_G.p);
            HIPCHK(hipMemcpyAsync(h->d_G.p, h->d_tmp.p, sizeof(double2) * n,
                                  hipMemcpyDeviceToDevice, h->stream));
        }
        h->st.outer_iters = it + 1;
        h->st.rel_residual = d / hnorm;
        if (h->prog && (it + 1) % h->prog_every == 0) h->prog(h->prog_user, it + 1, d / hnorm);
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
        // FP32 corrections inside a refinement loop aim at a fixed reduction
        // (their operator is only FP32-accurate); FP64 ones, and a single
        // FP32 pass (refine = 0), go for the whole way
        const double want = tol * hnorm / rnorm;
        const double inner = (fp32 && passes > 1) ? std::max(1e-4, want) : want;
        int its = 0;
        double irel = 0.0;
        h->prog_base = its_total;
        h->prog_scale = hnorm > 0.0 ? rnorm / hnorm : 0.0;
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
    CHK(fixed_point(h, with_f, tol, max_iter, hnorm));
    // final sweep with G + g_phys and sources: u, and T G + h for the true residual
    double rel = 0.0;
    h->sweep_warm = h->opt.warm != 0;
    const int rc = residual_sweep(h, with_f, h->opt.precision, h->opt.tau_in, hnorm, &rel);
    h->sweep_warm = false;
    CHK(rc);
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
    Store* S = h->store;
    for (int prec : {DD_FP64, DD_FP32}) {
        const Store::PrecBuf& B = S->pb[prec_index(prec)];
        if (!B.present) continue;
        const size_t rs = prec_size(prec);
        char* F = B.F.p + rs * h->node_base;
        HIPCHK(wdd::gather_source(d_fre, d_fim, S->d_gidx.p + h->node_base,
                                  S->d_area.p + h->node_base, n, F, F + rs * S->cap_node,
                                  prec == DD_FP32, h->stream));
    }
    return DD_OK;
}

double2* u_dev(const dd_handle* h) { return h->store->d_u.p + h->node_base; }

// Stream whose pool a problem's own vectors come from: its stream when it
// sits in a shared store (batches, served requests), none (plain hipMalloc)
// for a handle with a store of its own.
hipStream_t pool_stream(const dd_handle* h) {
    return (h->store && h->store->shared) ? h->stream : nullptr;
}

int ensure_staging(dd_handle* h) {
    if (!h->d_fre.p) {
        hipStream_t as = pool_stream(h);
        HIPCHK(h->d_fre.alloc(h->N, as));
        HIPCHK(h->d_fim.alloc(h->N, as));
        HIPCHK(h->d_gre.alloc(h->n_trace, as));
        HIPCHK(h->d_gim.alloc(h->n_trace, as));
        HIPCHK(h->d_ure.alloc(h->N, as));
        HIPCHK(h->d_uim.alloc(h->N, as));
        HIPCHK(h->d_work.alloc(2 * h->N, as));
        if (as) HIPCHK(hipStreamSynchronize(as));
    }
    return DD_OK;
}

// Device address of the no-allocation scratch array on the handle's device
// (looked up once per device, with that device current).
int noalloc_init(const dd_handle* h) {
    HIPCHK(hipSetDevice(h->dev));
    double2* p = nullptr;
    HIPCHK(wdd::noalloc_scratch(h->dev, &p));
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
// Workgroups per subdomain for a STREAM sweep of a handle of its own: the
// largest K in {4, 2} with K workgroups of 512 threads per subdomain still
// resident together (one per CU), when the device supports cooperative
// launches; 1 otherwise.
int stream_share_k(const dd_handle* h) {
    int coop = 0, cus = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, h->dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->dev) != hipSuccess)
        return 1;
    if (!coop) return 1;
    const int64_t items = (h->L + 7) / 8 * 8;
    for (int k : {4, 2})
        if (items * k <= cus) return k;
    return 1;
}

// Layout and workgroup size of a subdomain shape, by timing: three sweeps
// of two WaveHoltz iterations each with every candidate that fits.  The
// candidates are the on-chip layouts (one element patch per thread with two
// or one barrier per step, one node per thread) at their natural
// workgroup sizes and, for subdomains that only the STREAM layout holds,
// STREAM at each workgroup size it can run with (256 or 512 threads: 64-2P
// columns per wave, the rows of a column group split over the waves).
int autotune_layout(dd_handle* h) {
    struct Cand {
        int layout, wg, k;
    };
    std::vector<Cand> cands;
    if (h->layout == DD_LAYOUT_STREAM) {
        for (int wg : stream_wg_options(h)) cands.push_back({DD_LAYOUT_STREAM, wg, 1});
        // a handle of its own with few subdomains may share each subdomain
        // among several workgroups (all resident at once: at most one
        // 512-thread workgroup per CU)
        const int k = (h->store->shared || h->opt.precision != DD_FP64) ? 1 : stream_share_k(h);
        if (k > 1) cands.push_back({DD_LAYOUT_STREAM, 512, k});
    } else {
        for (int lay : {DD_LAYOUT_PATCH, DD_LAYOUT_PATCH_XCHG, DD_LAYOUT_NODE})
            if (layout_fits(h, lay)) cands.push_back({lay, layout_threads(h, lay), 1});
    }
    Cand best{h->layout, h->wg, 1};
    double best_ms = 1e300;
    for (const Cand& c : cands) {
        layout_config(h, c.layout, c.wg);
        if (c.k > 1) {
            if (h->xb_bytes < xb_bytes_for(h->L, c.k)) {
                h->d_xb.free();
                HIPCHK(h->d_xb.alloc(xb_bytes_for(h->L, c.k)));
                h->xb_bytes = xb_bytes_for(h->L, c.k);
            }
        }
        h->xb_k = c.k;
        HIPCHK(hipMemsetAsync(h->d_g0.p, 0, sizeof(double2) * h->n_if, h->stream));
        CHK(run_sweep(h, h->d_g0.p, h->d_tmp.p, 0.0, false, false, h->opt.precision, 0.0, 2));
        reset_stats(h);
        for (int r = 0; r < 3; ++r)
            CHK(run_sweep(h, h->d_g0.p, h->d_tmp.p, 0.0, false, true, h->opt.precision, 0.0, 2));
        const double ms = h->st.sweep_seconds;
        // a shared-subdomain candidate that fell back to one workgroup
        // (h->xb_k reset by launch_sweep) is not kept
        if (ms < best_ms && h->xb_k == c.k) {
            best_ms = ms;
            best = c;
        }
    }
    layout_config(h, best.layout, best.wg);
    h->xb_k = best.k;
    reset_stats(h);
    return DD_OK;
}


// Host-side arrays of one problem, computed before any device work.
struct HostArrays {
    std::vector<double> alpha, betaX, betaY, beta, area, w1d, kap, kaph, cs, sn, kside;
    std::vector<double> wxg, wyg, Mg, Hg;
    std::vector<int> gidx, is_iface;
    std::vector<int64_t> trace_idx;
};

// Validate a problem and compute everything the device needs (Sec. IV
// lumped operators, Sec. V leapfrog coefficients and filter tables, the
// time-step rule, the layout).  Descriptors carry problem-local offsets.
int prepare(dd_handle* h, const dd_mesh* mesh, int degree, const double* wavespeed, double omega,
            const dd_partition* part, const dd_options* opt, HostArrays& ha) {
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
    if (o.layout < DD_LAYOUT_AUTO || o.layout > DD_LAYOUT_STREAM) return fail(DD_EINVAL, "bad layout");
    if (o.max_wh < 1) return fail(DD_EINVAL, "max_wh must be >= 1");
    if (o.outer != DD_OUTER_GMRES && o.outer != DD_OUTER_FIXED)
        return fail(DD_EINVAL, "bad outer method");
    if (o.restart < 1 || o.restart > 400) return fail(DD_EINVAL, "restart must be in [1, 400]");
    if (!(o.cfl > 0.0 && o.cfl <= 1.0)) return fail(DD_EINVAL, "cfl must be in (0, 1]");
    if (o.nt_override < 0 || o.nt_override == 1 || o.nt_override == 2)
        return fail(DD_EINVAL, "nt_override must be 0 or >= 3");
    if (o.refine < 0 || o.refine > 50) return fail(DD_EINVAL, "refine must be in [0, 50]");
    if (!(o.relax >= 0.0) || !std::isfinite(o.relax)) return fail(DD_EINVAL, "relax must be >= 0");
    if (o.warm != 0 && o.warm != 1) return fail(DD_EINVAL, "warm must be 0 or 1");
    if (!(o.tc2 >= 0.0) || !std::isfinite(o.tc2)) return fail(DD_EINVAL, "tc2 must be >= 0");
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
    else if (lay == DD_LAYOUT_STREAM && !layout_fits(h, DD_LAYOUT_STREAM))
        why = "streaming layout tables exceed the LDS (N_t too large)";
    else if (!node_ok && !patch_ok && !xchg_ok && !layout_fits(h, DD_LAYOUT_STREAM))
        why = "no layout fits (N_t too large)";
    if (why) {
        return fail(DD_EINVAL, "%s (subdomain %dx%d elements, P=%d)", why, mx, my, P);
    }
    if (lay == DD_LAYOUT_AUTO)
        lay = patch_ok ? DD_LAYOUT_PATCH
              : xchg_ok ? DD_LAYOUT_PATCH_XCHG
              : node_ok ? DD_LAYOUT_NODE
                        : DD_LAYOUT_STREAM;
    layout_config(h, lay);
    // physical lumped 1D weights of a subdomain (the same for all)
    std::vector<double> w1d(nxl + nyl);
    for (int il = 0; il < nxl; ++il) w1d[il] = 0.5 * h->hx * wref(g, il, mx);
    for (int jl = 0; jl < nyl; ++jl) w1d[nxl + jl] = 0.5 * h->hy * wref(g, jl, my);

    // per-node coefficients (Sec. IV lumped M, H; Sec. V alpha, beta)
    const int64_t nn = L * nloc;
    std::vector<double> alpha(nn), betaX(nn), betaY(nn), beta(nn), area(nn);
    std::vector<int> gidx(nn);
    h->desc.resize(L);
    // second-order transmission condition: q = tc2 * min(c) / omega
    const double q = o.tc2 > 0.0 ? o.tc2 * *std::min_element(wavespeed, wavespeed + N) / omega : 0.0;
    for (int64_t l = 0; l < L; ++l) {
        const int a = (int)(l % part->sx), b = (int)(l / part->sx);
        const int n = h->nt[l];
        const double half = M_PI / n;  // omega dt / 2
        const double theta = std::tan(half) / omega;
        const double sigma = std::sin(half) / (0.5 * omega);
        // interface sides (left, right, bottom, top): their ends extend the
        // 1D weights of stiffness and mass by q (Kronecker form kept)
        const bool itf[4] = {a > 0, a + 1 < part->sx, b > 0, b + 1 < part->sy};
        for (int jl = 0; jl < nyl; ++jl)
            for (int il = 0; il < nxl; ++il) {
                const int64_t k = l * nloc + (int64_t)jl * nxl + il;
                const int64_t gi = (int64_t)(b * my * P + jl) * Nx + a * mx * P + il;
                const double cc = wavespeed[gi];
                const double wx = w1d[il], wy = w1d[nxl + jl];
                const double wxt = wx + ((il == 0 && itf[0]) || (il == nxl - 1 && itf[1]) ? q : 0.0);
                const double wyt = wy + ((jl == 0 && itf[2]) || (jl == nyl - 1 && itf[3]) ? q : 0.0);
                const double M = wxt * wyt / (cc * cc);
                double Hs = 0.0;
                if (il == 0) Hs += wy;
                if (il == nxl - 1) Hs += wy;
                if (jl == 0) Hs += wx;
                if (jl == nyl - 1) Hs += wx;
                const double H = Hs / cc;
                alpha[k] = (M - theta * H) / (M + theta * H);
                beta[k] = sigma / (M + theta * H);
                betaX[k] = beta[k] * (2.0 / h->hx) * wyt;
                betaY[k] = beta[k] * (2.0 / h->hy) * wxt;
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
        d.ws_off = l * 2 * wdd::stream_pad_nodes(nxl, nyl);
        d.tc_q = q;
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

    ha.alpha = std::move(alpha);
    ha.betaX = std::move(betaX);
    ha.betaY = std::move(betaY);
    ha.beta = std::move(beta);
    ha.area = std::move(area);
    ha.gidx = std::move(gidx);
    ha.w1d = std::move(w1d);
    ha.kap = std::move(kap);
    ha.kaph = std::move(kaph);
    ha.cs = std::move(cs);
    ha.sn = std::move(sn);
    ha.kside = std::move(kside);
    ha.trace_idx = std::move(trace_idx);
    ha.is_iface = std::move(is_iface);
    ha.wxg = std::move(wxg);
    ha.wyg = std::move(wyg);
    ha.Mg = std::move(Mg);
    ha.Hg = std::move(Hg);
    return DD_OK;
}

void store_destroy(Store* S) {
    if (!S) return;
    (void)hipSetDevice(S->dev);
    for (auto& B : S->pb) {
        B.coef.free();
        B.tab.free();
        B.F.free();
    }
    S->d_desc.free();
    S->d_w1d.free(); S->d_kside.free(); S->d_area.free();
    S->d_gidx.free(); S->d_iters.free(); S->d_is_iface.free(); S->d_trace_idx.free();
    S->d_u.free(); S->d_wsp.free(); S->d_wss.free(); S->d_wsp32.free(); S->d_wss32.free();
    S->d_gin.free(); S->d_gout.free(); S->d_work.free(); S->d_work_iters.free();
    if (S->h_work) (void)hipHostFree(S->h_work);
    if (S->h_work_iters) (void)hipHostFree(S->h_work_iters);
    for (int i = 0; i < Sched::kSlots; ++i) {
        if (S->ss[i]) (void)hipStreamSynchronize(S->ss[i]);
        for (int k = 0; k < Store::kSub; ++k) {
            if (S->gs[i][k]) (void)hipStreamSynchronize(S->gs[i][k]);
            if (S->gev[i][k]) (void)hipEventDestroy(S->gev[i][k]);
            if (S->gs[i][k]) (void)hipStreamDestroy(S->gs[i][k]);
        }
        if (S->sevc[i]) (void)hipEventDestroy(S->sevc[i]);
        if (S->sev0[i]) (void)hipEventDestroy(S->sev0[i]);
        if (S->sev1[i]) (void)hipEventDestroy(S->sev1[i]);
        if (S->ss[i]) (void)hipStreamDestroy(S->ss[i]);
    }
    delete S;
}

// Allocate a store with the given capacities (entries per index space).
// A shared store has n_slots work-list regions of slot_items entries; with
// slot_streams each slot launches on a stream of its own (and sub_streams
// group streams), else a round runs on the stream of the thread that
// launches it.
int store_create(Store** out, int dev, int64_t cn, int64_t ci, int64_t cit, int64_t ct,
                 int64_t cw, int64_t cwsp, bool fp32, bool shared, int sub_streams = Store::kSub,
                 int n_slots = 8, int64_t slot_items = 0, bool slot_streams = true) {
    *out = nullptr;
    Store* S = new Store();
    S->dev = dev;
    S->shared = shared;
    S->sub_streams = slot_streams ? std::max(1, std::min(sub_streams, Store::kSub)) : 1;
    S->n_slots = std::max(1, std::min(n_slots, Sched::kSlots));
    S->slot_items = slot_items > 0 ? std::min(slot_items, std::max<int64_t>(cit, 1))
                                   : std::max<int64_t>(cit, 1);
    S->align = shared ? 64 : 1;
    S->cap_node = cn;
    S->cap_if = ci;
    S->cap_item = cit;
    S->cap_tab = ct;
    S->cap_w1d = cw;
    S->cap_wsp = cwsp;
    S->a_node.init(cn);
    S->a_if.init(ci);
    S->a_item.init(cit);
    S->a_tab.init(ct);
    S->a_w1d.init(cw);
    S->a_wsp.init(cwsp);
    S->pb[0].present = true;
    S->pb[1].present = fp32;
#define STCHK(expr)                                                                              \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            const int c_ = fail(e_ == hipErrorOutOfMemory ? DD_ENOMEM : DD_EHIP, "%s: %s", #expr, \
                                hipGetErrorString(e_));                                          \
            store_destroy(S);                                                                    \
            return c_;                                                                           \
        }                                                                                        \
    } while (0)
    STCHK(hipSetDevice(dev));
    size_t bytes = 0;
    for (int k = 0; k < 2; ++k) {
        Store::PrecBuf& B = S->pb[k];
        if (!B.present) continue;
        const size_t bs = k == 1 ? 4 : 8;
        STCHK(B.coef.alloc(4 * bs * cn));
        STCHK(B.tab.alloc(4 * bs * ct));
        STCHK(B.F.alloc(2 * bs * cn));
        bytes += bs * (6 * cn + 4 * ct);
    }
    STCHK(S->d_desc.alloc(cit));
    STCHK(S->d_w1d.alloc(cw));
    STCHK(S->d_kside.alloc(ci));
    STCHK(S->d_area.alloc(cn));
    STCHK(S->d_gidx.alloc(cn));
    STCHK(S->d_iters.alloc(cit));
    STCHK(S->d_is_iface.alloc(ci));
    STCHK(S->d_trace_idx.alloc(ci));
    STCHK(S->d_u.alloc(cn));
    bytes += cit * (sizeof(wdd::SubDesc) + 4) + cw * 8 + ci * 20 + cn * 28;
    if (cwsp > 0) {
        // STREAM workspace: kStreamRecord Reals per node, then the interior
        // record {1, 0, 0} (and a zero pad) that nodes off the subdomain
        // sides read
        const int64_t nws = wdd::kStreamRecord * cn + wdd::kStreamExtra;
        const double one64[wdd::kStreamExtra] = {1.0, 0.0, 0.0, 0.0};
        const float one32[wdd::kStreamExtra] = {1.0f, 0.0f, 0.0f, 0.0f};
        STCHK(S->d_wsp.alloc(cwsp));
        STCHK(S->d_wss.alloc(nws));
        STCHK(hipMemcpy(S->d_wss.p + wdd::kStreamRecord * cn, one64, sizeof(one64),
                        hipMemcpyHostToDevice));
        bytes += 8 * (cwsp + nws);
        if (fp32) {
            STCHK(S->d_wsp32.alloc(cwsp));
            STCHK(S->d_wss32.alloc(nws));
            STCHK(hipMemcpy(S->d_wss32.p + wdd::kStreamRecord * cn, one32, sizeof(one32),
                            hipMemcpyHostToDevice));
            bytes += 4 * (cwsp + nws);
        }
    }
    if (shared) {
        // problems placed in this store take their own vectors from the
        // device's stream-ordered pool: keep freed memory in the pool (no
        // release to the system, which would synchronise)
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t keep = UINT64_MAX;
            STCHK(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
        }
        STCHK(S->d_gin.alloc(ci));
        STCHK(S->d_gout.alloc(ci));
        const int64_t nw = (int64_t)S->n_slots * S->slot_items;
        STCHK(S->d_work.alloc(nw));
        STCHK(S->d_work_iters.alloc(nw));
        STCHK(hipHostMalloc((void**)&S->h_work, sizeof(wdd::SubDesc) * nw));
        STCHK(hipHostMalloc((void**)&S->h_work_iters, sizeof(int) * nw));
        for (int i = 0; i < S->n_slots; ++i) {
            if (slot_streams) STCHK(hipStreamCreateWithFlags(&S->ss[i], hipStreamNonBlocking));
            STCHK(hipEventCreate(&S->sev0[i]));
            STCHK(hipEventCreate(&S->sev1[i]));
            STCHK(hipEventCreateWithFlags(&S->sevc[i], hipEventDisableTiming));
            for (int k = 0; k < S->sub_streams && S->sub_streams > 1; ++k) {
                STCHK(hipStreamCreateWithFlags(&S->gs[i][k], hipStreamNonBlocking));
                STCHK(hipEventCreateWithFlags(&S->gev[i][k], hipEventDisableTiming));
            }
        }
        bytes += ci * 32 + nw * (sizeof(wdd::SubDesc) + 4);
    }
#undef STCHK
    S->bytes = bytes;
    *out = S;
    return DD_OK;
}

// Device bytes a placed problem holds outside the store.
size_t problem_own_bytes(const dd_handle* h) {
    const int64_t ld = ((h->n_if + 63) / 64) * 64;
    return sizeof(double2) * ((size_t)(h->opt.restart + 1) * ld + 8 * (size_t)h->n_if +
                              (h->opt.restart + 1)) +
           8 * ((size_t)h->Nx + h->Ny + 2 * (size_t)h->N) +
           sizeof(double2) * (size_t)(h->opt.restart + 2) * 1024;
}

// Range lengths of a problem in a store.
void problem_ranges(dd_handle* h, int64_t align) {
    auto rnd = [&](int64_t n) { return (n + align - 1) / align * align; };
    h->node_len = rnd(h->L * h->nloc);
    h->if_len = rnd(h->n_if);
    h->item_len = h->L;
    h->w1d_len = h->nxl + h->nyl;
    h->wsp_len = h->layout == DD_LAYOUT_STREAM ? h->L * 2 * wdd::stream_pad_nodes(h->nxl, h->nyl) : 0;
}

void unplace(dd_handle* h) {
    (void)hipSetDevice(h->dev);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    h->d_V.free(); h->d_G.free(); h->d_h.free(); h->d_tmp.free(); h->d_g0.free();
    h->d_r.free(); h->d_coefs.free(); h->d_D.free(); h->d_res.free();
    h->d_fre.free(); h->d_fim.free(); h->d_gre.free(); h->d_gim.free(); h->d_ure.free();
    h->d_uim.free(); h->d_wxg.free(); h->d_wyg.free(); h->d_Mg.free(); h->d_Hg.free();
    h->d_work.free();
    h->d_xb.free();
    wdd::blas_free(h->blas);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    h->ev0 = h->ev1 = nullptr;
    h->stream = nullptr;
    if (h->placed && h->store) {
        Store* S = h->store;
        std::lock_guard<std::mutex> lk(S->mu);
        S->a_node.release(h->node_base, h->node_len);
        S->a_if.release(h->if_base, h->if_len);
        S->a_item.release(h->item_base, h->item_len);
        S->a_tab.release(h->tab_base, h->tab_len);
        S->a_w1d.release(h->w1d_base, h->w1d_len);
        S->a_wsp.release(h->wsp_base, h->wsp_len);
        h->placed = false;
    }
}

// Reserve the problem's ranges in the store (DD_ENOMEM if any is full).
int reserve(dd_handle* h, Store* S) {
    problem_ranges(h, S->align);
    std::lock_guard<std::mutex> lk(S->mu);
    int64_t* base[6] = {&h->node_base, &h->if_base, &h->item_base, &h->tab_base, &h->w1d_base,
                        &h->wsp_base};
    const int64_t len[6] = {h->node_len, h->if_len, h->item_len, h->tab_len, h->w1d_len, h->wsp_len};
    RangeAlloc* ra[6] = {&S->a_node, &S->a_if, &S->a_item, &S->a_tab, &S->a_w1d, &S->a_wsp};
    for (int k = 0; k < 6; ++k) {
        *base[k] = ra[k]->alloc(len[k]);
        if (*base[k] < 0) {
            for (int q = 0; q < k; ++q) ra[q]->release(*base[q], len[q]);
            return fail(DD_ENOMEM, "device store full");
        }
    }
    h->store = S;
    h->dev = S->dev;
    h->placed = true;
    return DD_OK;
}

// Upload a reserved problem into its store ranges and allocate its outer
// iteration vectors.  On failure the caller unplaces.
int upload(dd_handle* h, const HostArrays& ha) {
    Store* S = h->store;
    HIPCHK(hipSetDevice(S->dev));
    const int64_t L = h->L, nn = L * h->nloc;
    for (auto& d : h->desc) {
        d.node_off += h->node_base;
        d.w_off = h->w1d_base;
        d.if_off += h->if_base;
        for (int s = 0; s < 4; ++s)
            if (d.nbr_off[s] >= 0) d.nbr_off[s] += h->if_base;
        d.toff += (int)h->tab_base;
        d.ws_off += h->wsp_base;
    }
    HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreate(&h->ev0));
    HIPCHK(hipEventCreate(&h->ev1));
    auto up_real = [&](char* base, int64_t stride, int k, int64_t off, const std::vector<double>& v,
                       size_t bs) -> hipError_t {
        char* dst = base + bs * ((size_t)k * stride + off);
        if (bs == 8) return hipMemcpy(dst, v.data(), 8 * v.size(), hipMemcpyHostToDevice);
        std::vector<float> f(v.begin(), v.end());
        return hipMemcpy(dst, f.data(), 4 * f.size(), hipMemcpyHostToDevice);
    };
    HIPCHK(hipMemcpy(S->d_desc.p + h->item_base, h->desc.data(), sizeof(wdd::SubDesc) * L,
                     hipMemcpyHostToDevice));
    for (int k = 0; k < 2; ++k) {
        Store::PrecBuf& B = S->pb[k];
        if (!B.present) continue;
        const size_t bs = k == 1 ? 4 : 8;
        HIPCHK(up_real(B.coef.p, S->cap_node, 0, h->node_base, ha.alpha, bs));
        HIPCHK(up_real(B.coef.p, S->cap_node, 1, h->node_base, ha.betaX, bs));
        HIPCHK(up_real(B.coef.p, S->cap_node, 2, h->node_base, ha.betaY, bs));
        HIPCHK(up_real(B.coef.p, S->cap_node, 3, h->node_base, ha.beta, bs));
        HIPCHK(up_real(B.tab.p, S->cap_tab, 0, h->tab_base, ha.kap, bs));
        HIPCHK(up_real(B.tab.p, S->cap_tab, 1, h->tab_base, ha.kaph, bs));
        HIPCHK(up_real(B.tab.p, S->cap_tab, 2, h->tab_base, ha.cs, bs));
        HIPCHK(up_real(B.tab.p, S->cap_tab, 3, h->tab_base, ha.sn, bs));
        for (int q = 0; q < 2; ++q)
            HIPCHK(hipMemset(B.F.p + bs * ((size_t)q * S->cap_node + h->node_base), 0, bs * nn));
    }
    HIPCHK(hipMemcpy(S->d_w1d.p + h->w1d_base, ha.w1d.data(), 8 * ha.w1d.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S->d_kside.p + h->if_base, ha.kside.data(), 8 * ha.kside.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S->d_area.p + h->node_base, ha.area.data(), 8 * ha.area.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S->d_gidx.p + h->node_base, ha.gidx.data(), 4 * ha.gidx.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S->d_is_iface.p + h->if_base, ha.is_iface.data(), 4 * ha.is_iface.size(),
                     hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S->d_trace_idx.p + h->if_base, ha.trace_idx.data(), 8 * ha.trace_idx.size(),
                     hipMemcpyHostToDevice));
    HIPCHK(hipMemset(S->d_u.p + h->node_base, 0, sizeof(double2) * nn));
    if (h->wsp_len > 0) {
        // the zero padding of the p grids is never written: clear once
        HIPCHK(hipMemset(S->d_wsp.p + h->wsp_base, 0, sizeof(double) * h->wsp_len));
        if (S->d_wsp32.p)
            HIPCHK(hipMemset(S->d_wsp32.p + h->wsp_base, 0, sizeof(float) * h->wsp_len));
    }
    const int64_t Nx = h->Nx, Ny = h->Ny, N = h->N;
    h->ld = ((h->n_if + 63) / 64) * 64;
    // a problem in a shared store takes its own vectors from the stream-
    // ordered pool (returned without a device-wide wait when it retires)
    hipStream_t as = pool_stream(h);
    HIPCHK(h->d_V.alloc((size_t)(h->opt.restart + 1) * h->ld, as));
    HIPCHK(h->d_G.alloc(h->n_if, as));
    HIPCHK(h->d_h.alloc(h->n_if, as));
    HIPCHK(h->d_tmp.alloc(h->n_if, as));
    HIPCHK(h->d_g0.alloc(h->n_if, as));
    HIPCHK(h->d_r.alloc(h->n_if, as));
    HIPCHK(h->d_D.alloc(h->n_if, as));
    HIPCHK(h->d_res.alloc(h->n_if, as));
    HIPCHK(h->d_coefs.alloc(h->opt.restart + 1, as));
    HIPCHK(h->d_wxg.alloc(Nx, as));
    HIPCHK(h->d_wyg.alloc(Ny, as));
    HIPCHK(h->d_Mg.alloc(N, as));
    HIPCHK(h->d_Hg.alloc(N, as));
    HIPCHK(wdd::blas_init(h->blas, h->opt.restart + 2, h->stream, as != nullptr));
    if (as) HIPCHK(hipStreamSynchronize(as));   // allocations complete before other streams use them
    h->own_bytes = problem_own_bytes(h);
    h->iters_host.assign(L, 0);
    h->last_iters.assign(L, 1);
    HIPCHK(hipMemcpy(h->d_wxg.p, ha.wxg.data(), 8 * (size_t)Nx, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->d_wyg.p, ha.wyg.data(), 8 * (size_t)Ny, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->d_Mg.p, ha.Mg.data(), 8 * (size_t)N, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->d_Hg.p, ha.Hg.data(), 8 * (size_t)N, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(h->d_G.p, 0, sizeof(double2) * h->n_if));
    HIPCHK(hipMemset(h->d_g0.p, 0, sizeof(double2) * h->n_if));
    return DD_OK;
}

int device_present(int* dev) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(DD_ENODEV, "no HIP device");
    (void)hipGetDevice(dev);
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
    o->max_wh = 1000;
    o->outer = DD_OUTER_GMRES;
    o->restart = 50;
    o->nt_override = 0;
    o->cfl = 0.9;
    o->refine = 4;
    o->relax = 0.0;
    o->warm = 0;
    o->tc2 = 0.0;
    return DD_OK;
}

void dd_destroy(dd_handle* h) {
    if (!h) return;
    Store* S = h->store;
    const bool own = h->own_store;
    unplace(h);
    if (own) store_destroy(S);
    delete h;
}

int dd_setup(dd_handle** out, const dd_mesh* mesh, int degree, const double* wavespeed,
             double omega, const dd_partition* part, const dd_options* opt) {
    if (!out) return fail(DD_EINVAL, "null output handle pointer");
    *out = nullptr;
    dd_handle* h = new dd_handle();
    HostArrays ha;
    int rc = prepare(h, mesh, degree, wavespeed, omega, part, opt, ha);
    int dev = 0;
    if (rc == DD_OK) rc = device_present(&dev);
    if (rc != DD_OK) {
        delete h;
        return rc;
    }
    problem_ranges(h, 1);
    Store* S = nullptr;
    rc = store_create(&S, dev, h->node_len, h->if_len, h->item_len, h->tab_len, h->w1d_len,
                      h->wsp_len, h->opt.precision == DD_FP32, false);
    if (rc != DD_OK) {
        delete h;
        return rc;
    }
    h->own_store = true;
    h->store = S;
    rc = reserve(h, S);
    if (rc == DD_OK) rc = upload(h, ha);
    if (rc == DD_OK && h->opt.layout == DD_LAYOUT_AUTO) rc = autotune_layout(h);
    if (rc == DD_OK) rc = noalloc_init(h);
    if (rc != DD_OK) {
        dd_destroy(h);
        return rc;
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

int dd_mesh_coords(const dd_mesh* mesh, int degree, double* x, double* y) {
    if (!mesh || !x || !y) return fail(DD_EINVAL, "null argument");
    if (degree < 1 || degree > wdd::kMaxP)
        return fail(DD_EINVAL, "degree %d not in [1, %d]", degree, wdd::kMaxP);
    if (mesh->nx < 1 || mesh->ny < 1) return fail(DD_EINVAL, "empty mesh");
    if (!(mesh->x1 > mesh->x0) || !(mesh->y1 > mesh->y0)) return fail(DD_EINVAL, "degenerate rectangle");
    const int P = degree, Nx = mesh->nx * P + 1, Ny = mesh->ny * P + 1;
    const Gll g = make_gll(P);
    const double hx = (mesh->x1 - mesh->x0) / mesh->nx, hy = (mesh->y1 - mesh->y0) / mesh->ny;
    std::vector<double> xs(Nx), ys(Ny);
    for (int e = 0; e < mesh->nx; ++e)
        for (int a = 0; a <= P; ++a) xs[e * P + a] = mesh->x0 + e * hx + 0.5 * hx * (g.x[a] + 1.0);
    xs[Nx - 1] = mesh->x1;
    for (int e = 0; e < mesh->ny; ++e)
        for (int a = 0; a <= P; ++a) ys[e * P + a] = mesh->y0 + e * hy + 0.5 * hy * (g.x[a] + 1.0);
    ys[Ny - 1] = mesh->y1;
    for (int j = 0; j < Ny; ++j)
        for (int i = 0; i < Nx; ++i) {
            x[(int64_t)j * Nx + i] = xs[i];
            y[(int64_t)j * Nx + i] = ys[j];
        }
    return DD_OK;
}

int dd_set_progress(dd_handle* h, dd_progress_fn fn, void* user, int every) {
    CHK(validate_handle(h));
    if (fn && every < 1) return fail(DD_EINVAL, "every must be >= 1");
    h->prog = fn;
    h->prog_user = user;
    h->prog_every = fn ? every : 1;
    return DD_OK;
}

int dd_layout(const dd_handle* h, int* layout, int* wg) {
    CHK(validate_handle(h));
    if (layout) *layout = h->layout;
    if (wg) *wg = h->wg * (h->layout == DD_LAYOUT_STREAM ? h->xb_k : 1);
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
    HIPCHK(wdd::embed_trace(d_g_re, d_g_im, h->store->d_trace_idx.p + h->if_base, h->n_if,
                           h->d_g0.p, h->stream));
    const int rc = solve_core(h, with_f, tol, max_iter);
    if (rc != DD_OK) {
        if (dep) (void)hipEventDestroy(dep);
        return rc;
    }
    HIPCHK(wdd::glue_solution(u_dev(h), h->Nx, h->Ny, h->P, h->mx, h->my, h->part.sx, h->part.sy,
                              h->nloc, d_u_re, d_u_im, h->stream));
    if (d_u_sub)
        HIPCHK(hipMemcpyAsync(d_u_sub, u_dev(h), sizeof(double2) * h->L * h->nloc,
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
        HIPCHK(hipMemcpy(u.data(), u_dev(h), sizeof(double2) * u.size(), hipMemcpyDeviceToHost));
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
            e = h->layout == DD_LAYOUT_NODE     ? wdd::launch_apply_node<double>(a, h->P, h->wg, x, y, h->stream)
                : h->layout == DD_LAYOUT_PATCH  ? wdd::launch_apply_patch1<double>(a, h->P, h->wg, x, y, h->stream)
                : h->layout == DD_LAYOUT_STREAM ? wdd::launch_apply_stream<double>(a, h->P, h->wg, x, y, h->stream)
                                                : wdd::launch_apply_patch<double>(a, h->P, h->wg, x, y, h->stream);
        } else {
            auto a = make_args<float>(h, h->d_g0.p, h->d_tmp.p, 0.0, false, 0.0, 1);
            float* x = (float*)dp.p;
            float* y = (float*)dq.p;
            e = h->layout == DD_LAYOUT_NODE     ? wdd::launch_apply_node<float>(a, h->P, h->wg, x, y, h->stream)
                : h->layout == DD_LAYOUT_PATCH  ? wdd::launch_apply_patch1<float>(a, h->P, h->wg, x, y, h->stream)
                : h->layout == DD_LAYOUT_STREAM ? wdd::launch_apply_stream<float>(a, h->P, h->wg, x, y, h->stream)
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

int dd_residual_device_noalloc(dd_handle* h, void* stream, const double* d_u_re,
                               const double* d_u_im, const double* d_f_re, const double* d_f_im,
                               const double* d_g_re, const double* d_g_im, double* d_rel) {
    CHK(validate_handle(h));
    if (!d_u_re || !d_rel) return fail(DD_EINVAL, "null array");
    if (h->Ny > wdd::kNoAllocMaxRows)
        return fail(DD_EINVAL,
                    "dd_residual_device_noalloc: the mesh has %d grid rows; at most %d fit "
                    "its scratch array (use dd_residual)",
                    (int)h->Ny, wdd::kNoAllocMaxRows);
    HIPCHK(hipSetDevice(h->dev));
    double2* part = nullptr;
    HIPCHK(wdd::noalloc_scratch(h->dev, &part));
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    HIPCHK(wdd::launch_residual_noalloc(op_args(h), d_u_re, d_u_im, d_f_re, d_f_im, d_g_re,
                                        d_g_im, part, d_rel, s));
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

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
}  // extern "C"

struct dd_batch {
    Store* store = nullptr;
    std::vector<dd_handle*> probs;
    int64_t launches = 0;
    std::mutex mu;               // progress of a running solve
    std::condition_variable cv;
    int finished = 0;
    bool running = false;
    // state of a running solve (between dd_batch_solve_start and _finish)
    std::vector<std::thread> th;
    std::vector<int> rc;
    std::vector<std::string> msg;
    std::vector<dd_stats> sts;
    dd_stats* st_out = nullptr;
    int* rc_out = nullptr;
    int64_t l0 = 0;
};

namespace {

// Layout of a placed problem in a shared store: the store's cached choice
// for its subdomain shape, else the autotuner's (then cached).
int choose_layout_shared(dd_handle* h) {
    if (h->opt.layout != DD_LAYOUT_AUTO) return DD_OK;
    Store* S = h->store;
    const auto key = std::make_tuple(h->mx, h->my, h->P, h->opt.precision);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->layout_cache.find(key);
        if (it != S->layout_cache.end()) {
            layout_config(h, it->second.first, it->second.second);
            return DD_OK;
        }
    }
    CHK(autotune_layout(h));
    std::lock_guard<std::mutex> lk(S->mu);
    S->layout_cache[key] = std::make_pair(h->layout, h->wg);
    return DD_OK;
}

void batch_free(dd_batch* b) {
    for (dd_handle* h : b->probs) {
        if (!h) continue;
        unplace(h);
        delete h;
    }
    store_destroy(b->store);
    delete b;
}

}  // namespace

extern "C" {

void dd_batch_destroy(dd_batch* b) {
    if (!b) return;
    bool running;
    {
        std::lock_guard<std::mutex> lk(b->mu);
        running = b->running;
    }
    if (running) (void)dd_batch_solve_finish(b);
    batch_free(b);
}

int dd_batch_setup(dd_batch** out, int n, const dd_problem* probs, const dd_options* opt) {
    if (!out) return fail(DD_EINVAL, "null output batch pointer");
    *out = nullptr;
    if (n < 1 || !probs) return fail(DD_EINVAL, "need n >= 1 problems");
    std::vector<dd_handle*> hs(n, nullptr);
    std::vector<HostArrays> has(n);
    auto drop = [&]() {
        for (dd_handle* h : hs) delete h;
    };
    int64_t cn = 0, ci = 0, cit = 0, ct = 0, cw = 0, cwsp = 0;
    for (int i = 0; i < n; ++i) {
        hs[i] = new dd_handle();
        const dd_problem& q = probs[i];
        const int rc = prepare(hs[i], &q.mesh, q.degree, q.wavespeed, q.omega, &q.part, opt, has[i]);
        if (rc != DD_OK) {
            const std::string m = g_err;
            drop();
            return fail(rc, "problem %d: %s", i, m.c_str());
        }
        problem_ranges(hs[i], 64);
        cn += hs[i]->node_len;
        ci += hs[i]->if_len;
        cit += hs[i]->item_len;
        ct += hs[i]->tab_len;
        cw += hs[i]->w1d_len;
        cwsp += hs[i]->wsp_len;
    }
    int dev = 0;
    int rc = device_present(&dev);
    Store* S = nullptr;
    if (rc == DD_OK)
        rc = store_create(&S, dev, cn, ci, cit, ct, cw, cwsp, hs[0]->opt.precision == DD_FP32, true);
    if (rc != DD_OK) {
        drop();
        return rc;
    }
    dd_batch* b = new dd_batch();
    b->store = S;
    b->probs = hs;
    for (int i = 0; i < n && rc == DD_OK; ++i) {
        rc = reserve(hs[i], S);
        if (rc == DD_OK) rc = upload(hs[i], has[i]);
        if (rc == DD_OK) rc = choose_layout_shared(hs[i]);
        has[i] = HostArrays();
    }
    if (rc != DD_OK) {
        batch_free(b);
        return rc;
    }
    *out = b;
    return DD_OK;
}

int dd_batch_handle(dd_batch* b, int i, dd_handle** h) {
    if (!b || !h) return fail(DD_EINVAL, "null batch or output");
    if (i < 0 || i >= (int)b->probs.size()) return fail(DD_EINVAL, "problem index %d out of range", i);
    *h = b->probs[i];
    return DD_OK;
}

int dd_batch_solve_start(dd_batch* b, const double* const* f_re, const double* const* f_im,
                         double tol, int max_iter, double* const* u_re, double* const* u_im,
                         dd_stats* st, int* rcs) {
    if (!b) return fail(DD_EINVAL, "null batch");
    if (!u_re || !u_im) return fail(DD_EINVAL, "null output arrays");
    if (!(tol >= 0.0) || max_iter < 1) return fail(DD_EINVAL, "tol must be >= 0 and max_iter >= 1");
    const int n = (int)b->probs.size();
    for (int i = 0; i < n; ++i)
        if (!u_re[i] || !u_im[i]) return fail(DD_EINVAL, "null output for problem %d", i);
    {
        std::lock_guard<std::mutex> lk(b->mu);
        if (b->running) return fail(DD_EINVAL, "a batch solve is already running");
        b->finished = 0;
        b->running = true;
    }
    Store* S = b->store;
    b->l0 = S->sched.launches;
    b->rc.assign(n, DD_OK);
    b->msg.assign(n, std::string());
    b->sts.assign(n, dd_stats{});
    b->st_out = st;
    b->rc_out = rcs;
    for (dd_handle* h : b->probs) {
        h->batched = true;
        sched_join(S);
    }
    b->th.clear();
    b->th.reserve(n);
    for (int i = 0; i < n; ++i) {
        const double* fr = f_re ? f_re[i] : nullptr;
        const double* fi = f_im ? f_im[i] : nullptr;
        double* ur = u_re[i];
        double* ui = u_im[i];
        b->th.emplace_back([b, S, i, fr, fi, tol, max_iter, ur, ui]() {
            (void)hipSetDevice(S->dev);
            b->rc[i] = dd_solve(b->probs[i], fr, fi, nullptr, nullptr, tol, max_iter, ur, ui,
                                &b->sts[i]);
            b->msg[i] = g_err;
            sched_leave(S);
            std::lock_guard<std::mutex> lk(b->mu);
            b->finished += 1;
            b->cv.notify_all();
        });
    }
    return DD_OK;
}

int dd_batch_solve_finish(dd_batch* b) {
    if (!b) return fail(DD_EINVAL, "null batch");
    {
        std::lock_guard<std::mutex> lk(b->mu);
        if (!b->running) return fail(DD_EINVAL, "no batch solve is running");
    }
    for (auto& t : b->th) t.join();
    b->th.clear();
    Store* S = b->store;
    for (dd_handle* h : b->probs) h->batched = false;
    b->launches = S->sched.launches - b->l0;
    const int n = (int)b->probs.size();
    if (b->st_out) std::copy(b->sts.begin(), b->sts.end(), b->st_out);
    if (b->rc_out) std::copy(b->rc.begin(), b->rc.end(), b->rc_out);
    {
        std::lock_guard<std::mutex> lk(b->mu);
        b->running = false;
        b->cv.notify_all();
    }
    int worst = DD_OK;
    for (int i = 0; i < n; ++i) {
        if (b->rc[i] != DD_OK && b->rc[i] != DD_ENOTCONV)
            return fail(b->rc[i], "problem %d: %s", i, b->msg[i].c_str());
        if (b->rc[i] == DD_ENOTCONV && worst == DD_OK) {
            worst = DD_ENOTCONV;
            fail(DD_ENOTCONV, "problem %d: %s", i, b->msg[i].c_str());
        }
    }
    return worst;
}

int dd_batch_solve(dd_batch* b, const double* const* f_re, const double* const* f_im, double tol,
                   int max_iter, double* const* u_re, double* const* u_im, dd_stats* st, int* rcs) {
    CHK(dd_batch_solve_start(b, f_re, f_im, tol, max_iter, u_re, u_im, st, rcs));
    return dd_batch_solve_finish(b);
}

int dd_batch_wait_progress(dd_batch* b, int seen, int* finished) {
    if (!b || !finished) return fail(DD_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(b->mu);
    b->cv.wait(lk, [&] { return b->finished > seen || !b->running ||
                             b->finished >= (int)b->probs.size(); });
    *finished = b->finished;
    return DD_OK;
}

int dd_batch_launches(const dd_batch* b, int64_t* launches) {
    if (!b || !launches) return fail(DD_EINVAL, "null argument");
    *launches = b->launches;
    return DD_OK;
}

int dd_batch_time_sweep(dd_batch* b, int reps, int fixed_iters, double* ms, double* dof_updates,
                        int* launches) {
    if (!b || !ms) return fail(DD_EINVAL, "null argument");
    if (reps < 1 || fixed_iters < 1) return fail(DD_EINVAL, "reps and fixed_iters must be >= 1");
    Store* S = b->store;
    HIPCHK(hipSetDevice(S->dev));
    std::vector<SweepReq> reqs;
    for (dd_handle* h : b->probs) {
        HIPCHK(hipStreamSynchronize(h->stream));
        reqs.push_back(SweepReq{h, h->d_G.p, h->d_tmp.p, 0.0, false, h->opt.precision, 0.0,
                                fixed_iters, false});
    }
    std::vector<SweepReq*> rp;
    for (auto& r : reqs) rp.push_back(&r);
    CHK(launch_batch(S, rp, 0, S->ss[0]));
    for (dd_handle* h : b->probs) reset_stats(h);
    double total_ms = 0.0;
    int groups = 0;
    for (int r = 0; r < reps; ++r) {
        double m = 0.0;
        CHK(launch_batch(S, rp, 0, S->ss[0], &m, &groups));
        total_ms += m;
    }
    *ms = total_ms / reps;
    if (dof_updates) {
        double d = 0.0;
        for (dd_handle* h : b->probs) d += h->st.dof_updates;
        *dof_updates = d / reps;
    }
    if (launches) *launches = groups;
    return DD_OK;
}

// ---------------------------------------------------------------------------
// Serving engine
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

struct Request {
    int64_t id = 0;
    dd_handle* h = nullptr;
    HostArrays ha;
    std::vector<double> fre, fim, ure, uim;
    bool has_f = false, has_fim = false;
    double tol = 0.0;
    int max_iter = 0;
    int state = DD_REQ_QUEUED;
    int rc = DD_OK;
    std::string msg;
    dd_stats st{};
    double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
    size_t bytes = 0;
    bool claimed = false;   // returned by dd_engine_wait_any
};

}  // namespace

struct dd_engine {
    Store* store = nullptr;
    dd_options opt;
    size_t budget = 0, used = 0;
    int max_active = 1;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request*> queue;
    std::map<int64_t, Request*> reqs;
    int running = 0;
    int64_t peak = 0, done = 0, next_id = 1;
    bool stop = false;
    std::thread dispatcher;
    std::chrono::steady_clock::time_point t0;
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// One admitted request on its own host thread: upload, layout, batched
// solve, release.
void engine_run(dd_engine* e, Request* r) {
    Store* S = e->store;
    (void)hipSetDevice(S->dev);
    dd_handle* h = r->h;
    int rc = upload(h, r->ha);
    r->ha = HostArrays();
    if (rc == DD_OK) rc = choose_layout_shared(h);
    if (rc == DD_OK) {
        h->batched = true;
        sched_join(S);
        rc = dd_solve(h, r->has_f ? r->fre.data() : nullptr, r->has_fim ? r->fim.data() : nullptr,
                      nullptr, nullptr, r->tol, r->max_iter, r->ure.data(), r->uim.data(), &r->st);
        r->msg = g_err;
        sched_leave(S);
        h->batched = false;
    } else {
        r->msg = g_err;
    }
    unplace(h);
    delete h;
    r->h = nullptr;
    r->fre = std::vector<double>();
    r->fim = std::vector<double>();
    std::lock_guard<std::mutex> lk(e->mu);
    r->rc = rc;
    r->state = DD_REQ_DONE;
    r->t_done = e->now();
    e->used -= r->bytes;
    e->running -= 1;
    e->done += 1;
    e->cv.notify_all();
}

// Admission loop: FIFO, while a slot is free and the head request's store
// ranges and vectors fit.
void engine_dispatch(dd_engine* e) {
    std::unique_lock<std::mutex> lk(e->mu);
    while (true) {
        while (!e->stop && !e->queue.empty() && e->running < e->max_active) {
            Request* r = e->queue.front();
            if (e->used + r->bytes + e->store->bytes > e->budget) break;
            if (reserve(r->h, e->store) != DD_OK) break;
            e->queue.pop_front();
            e->used += r->bytes;
            e->running += 1;
            e->peak = std::max<int64_t>(e->peak, e->running);
            r->state = DD_REQ_RUNNING;
            r->t_start = e->now();
            std::thread(engine_run, e, r).detach();
        }
        if (e->stop && e->running == 0) break;
        e->cv.wait(lk);
    }
}

}  // namespace

extern "C" {

int dd_engine_create(dd_engine** out, size_t budget, int max_active, const dd_options* opt) {
    if (!out) return fail(DD_EINVAL, "null output engine pointer");
    *out = nullptr;
    if (budget < ((size_t)64 << 20)) return fail(DD_EINVAL, "budget must be >= 64 MiB");
    if (max_active < 1 || max_active > 4096) return fail(DD_EINVAL, "max_active must be in [1, 4096]");
    dd_options o;
    if (opt)
        o = *opt;
    else
        dd_default_options(&o);
    int dev = 0;
    CHK(device_present(&dev));
    // store: about 60% of the budget at ~200 bytes per subdomain node
    // (coefficients, source, iterate, streaming workspace), interface and
    // work-item spaces in proportion
    const int64_t cn = std::max<int64_t>(1 << 16, (int64_t)(0.6 * (double)budget / 200.0));
    const int64_t ci = cn / 2, cit = std::max<int64_t>(1024, cn / 64);
    const int64_t ct = std::max<int64_t>(1 << 16, cn / 16), cw = 1 << 18, cwsp = cn * 5 / 2;
    Store* S = nullptr;
    // The store creates no streams: a round runs on the stream of the
    // request that launches it (one stream per running request).  HIP maps
    // streams onto a fixed pool of hardware queues and kernels that share a
    // queue run in order, so every further stream would make some request's
    // short outer-iteration kernels wait behind another request's sweep;
    // and a fixed set of launch streams would let a few long rounds hold
    // all of them while cheap requests wait.  32 work-list slots of an
    // eighth of the work-item space each.
    CHK(store_create(&S, dev, cn, ci, cit, ct, cw, cwsp, o.precision == DD_FP32, true, 1,
                     Sched::kSlots, std::max<int64_t>(2048, cit / 8), false));
    if (S->bytes >= budget) {
        store_destroy(S);
        return fail(DD_ENOMEM, "budget too small for the device store");
    }
    dd_engine* e = new dd_engine();
    e->store = S;
    e->opt = o;
    e->budget = budget;
    e->max_active = max_active;
    e->t0 = std::chrono::steady_clock::now();
    e->dispatcher = std::thread(engine_dispatch, e);
    *out = e;
    return DD_OK;
}

void dd_engine_destroy(dd_engine* e) {
    if (!e) return;
    {
        std::lock_guard<std::mutex> lk(e->mu);
        for (Request* r : e->queue) {
            if (r->h) delete r->h;
            r->h = nullptr;
            r->state = DD_REQ_DONE;
            r->rc = DD_EINVAL;
        }
        e->queue.clear();
        e->stop = true;
        e->cv.notify_all();
    }
    e->dispatcher.join();
    for (auto& kv : e->reqs) delete kv.second;
    store_destroy(e->store);
    delete e;
}

int dd_engine_submit(dd_engine* e, const dd_problem* prob, const double* f_re, const double* f_im,
                     double tol, int max_iter, int64_t* id) {
    if (!e || !prob || !id) return fail(DD_EINVAL, "null argument");
    if (!(tol >= 0.0) || max_iter < 1) return fail(DD_EINVAL, "tol must be >= 0 and max_iter >= 1");
    if (!f_re && f_im) return fail(DD_EINVAL, "f_im given without f_re");
    const double t = e->now();
    Request* r = new Request();
    r->h = new dd_handle();
    int rc = prepare(r->h, &prob->mesh, prob->degree, prob->wavespeed, prob->omega, &prob->part,
                     &e->opt, r->ha);
    const int64_t N = rc == DD_OK ? r->h->N : 0;
    if (rc == DD_OK) rc = check_finite(f_re, N, "f_re");
    if (rc == DD_OK) rc = check_finite(f_im, N, "f_im");
    if (rc == DD_OK) {
        Store* S = e->store;
        problem_ranges(r->h, S->align);
        r->bytes = problem_own_bytes(r->h) + sizeof(double) * (10 * (size_t)N + 2 * (size_t)r->h->n_trace);
        if (r->h->node_len > S->cap_node || r->h->if_len > S->cap_if ||
            r->h->item_len > S->cap_item || r->h->L > S->slot_items || r->h->tab_len > S->cap_tab ||
            r->h->wsp_len > S->cap_wsp || r->bytes + S->bytes > e->budget)
            rc = fail(DD_ENOMEM, "request needs more device memory than the engine holds");
    }
    if (rc != DD_OK) {
        delete r->h;
        delete r;
        return rc;
    }
    r->has_f = f_re != nullptr;
    r->has_fim = f_im != nullptr;
    if (f_re) r->fre.assign(f_re, f_re + N);
    if (f_im) r->fim.assign(f_im, f_im + N);
    r->ure.assign(N, 0.0);
    r->uim.assign(N, 0.0);
    r->tol = tol;
    r->max_iter = max_iter;
    r->t_submit = t;
    std::lock_guard<std::mutex> lk(e->mu);
    r->id = e->next_id++;
    e->reqs[r->id] = r;
    e->queue.push_back(r);
    e->cv.notify_all();
    *id = r->id;
    return DD_OK;
}

int dd_engine_status(dd_engine* e, int64_t id, int* state) {
    if (!e || !state) return fail(DD_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(e->mu);
    auto it = e->reqs.find(id);
    if (it == e->reqs.end()) return fail(DD_EINVAL, "unknown request %lld", (long long)id);
    *state = it->second->state;
    return DD_OK;
}

int dd_engine_wait(dd_engine* e, int64_t id, double* u_re, double* u_im, dd_stats* st,
                   double* times) {
    if (!e) return fail(DD_EINVAL, "null engine");
    Request* r = nullptr;
    {
        std::unique_lock<std::mutex> lk(e->mu);
        auto it = e->reqs.find(id);
        if (it == e->reqs.end()) return fail(DD_EINVAL, "unknown request %lld", (long long)id);
        r = it->second;
        e->cv.wait(lk, [&] { return r->state == DD_REQ_DONE; });
        e->reqs.erase(it);
    }
    if (u_re) std::copy(r->ure.begin(), r->ure.end(), u_re);
    if (u_im) std::copy(r->uim.begin(), r->uim.end(), u_im);
    if (st) *st = r->st;
    if (times) {
        times[0] = r->t_submit;
        times[1] = r->t_start;
        times[2] = r->t_done;
    }
    const int rc = r->rc;
    const std::string msg = r->msg;
    delete r;
    if (rc != DD_OK) g_err = msg;
    return rc;
}

int dd_engine_wait_any(dd_engine* e, int64_t* id) {
    if (!e || !id) return fail(DD_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(e->mu);
    bool unclaimed = false;
    for (auto& kv : e->reqs) unclaimed = unclaimed || !kv.second->claimed;
    if (!unclaimed) return fail(DD_EINVAL, "no outstanding request that wait_any has not returned");
    int64_t found = -1;
    e->cv.wait(lk, [&] {
        for (auto& kv : e->reqs)
            if (kv.second->state == DD_REQ_DONE && !kv.second->claimed) {
                found = kv.first;
                return true;
            }
        return false;
    });
    e->reqs[found]->claimed = true;
    *id = found;
    return DD_OK;
}

int dd_engine_get_info(dd_engine* e, dd_engine_info* info) {
    if (!e || !info) return fail(DD_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(e->mu);
    info->queued = (int64_t)e->queue.size();
    info->running = e->running;
    info->done = e->done;
    info->peak_running = e->peak;
    info->budget_bytes = e->budget;
    info->store_bytes = e->store->bytes;
    info->request_bytes = e->used;
    info->launches = e->store->sched.launches.load();
    return DD_OK;
}

}  // extern "C"

// ===========================================================================
// Box (3D) decomposition: setup, sweep and operator of include/wavedd3.h
// ===========================================================================
struct dd3_handle {
    dd_box box{};
    dd_partition3 part{};
    dd_options opt{};
    int P = 0, dev = 0;
    double omega = 0.0, hx = 0.0, hy = 0.0, hz = 0.0;
    int mx = 0, my = 0, mz = 0, nxl = 0, nyl = 0, nzl = 0, Nx = 0, Ny = 0, Nz = 0;
    int64_t N = 0, nloc = 0, L = 0, per_sub = 0, n_if = 0, tab_len = 0;
    int face_off[6] = {0, 0, 0, 0, 0, 0};
    int nt_max = 0;
    std::vector<int> nt;
    std::vector<wdd::Sub3> desc;
    double K1[wdd::kMaxP + 1][wdd::kMaxP + 1] = {};
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    DBuf<wdd::Sub3> d_desc;
    DBuf<unsigned char> d_coef;  // alpha, betaX, betaY, betaZ, beta (Real, nn each)
    DBuf<unsigned char> d_tab;   // kap, kaph, cs, sn (Real, tab_len each)
    DBuf<unsigned char> d_coef64, d_tab64;  // FP64 copies of an FP32 handle (refinement sweeps)
    DBuf<double> d_w1d, d_kside, d_wx, d_wy, d_wz, d_M, d_H, d_f;
    DBuf<double2> d_gin, d_gout, d_u;
    DBuf<int> d_iters, d_perm;
    bool has_f = false;
    // outer solve (allocated by the first dd3_solve)
    wdd::Blas blas{};
    int64_t ld = 0;
    DBuf<double2> d_V, d_r, d_coefs, d_h, d_G, d_tmp, d_ug, d_Su, d_work, d_res, d_D;
    int64_t sweeps = 0, wh_total = 0;
    int wh_max = 0;
    double dof_updates = 0.0;
};

namespace {

void dd3_free(dd3_handle* h) {
    h->d_desc.free();
    h->d_coef.free();
    h->d_tab.free();
    h->d_coef64.free();
    h->d_tab64.free();
    for (DBuf<double>* b : {&h->d_w1d, &h->d_kside, &h->d_wx, &h->d_wy, &h->d_wz, &h->d_M, &h->d_H,
                            &h->d_f})
        b->free();
    h->d_gin.free();
    h->d_gout.free();
    h->d_u.free();
    h->d_iters.free();
    h->d_perm.free();
    for (DBuf<double2>* b : {&h->d_V, &h->d_r, &h->d_coefs, &h->d_h, &h->d_G, &h->d_tmp, &h->d_ug,
                             &h->d_Su, &h->d_work, &h->d_res, &h->d_D})
        b->free();
    wdd::blas_free(h->blas);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    h->ev0 = h->ev1 = nullptr;
    h->stream = nullptr;
}

int validate3(const dd3_handle* h) {
    if (!h || h->L < 1) return fail(DD_EINVAL, "null or unset 3D handle");
    return DD_OK;
}

size_t real3(const dd3_handle* h) { return h->opt.precision == DD_FP32 ? 4 : 8; }

// Physical lumped 1D weights of a line of m elements of length h.
std::vector<double> line_weights(const Gll& g, int m, double hlen) {
    std::vector<double> w(m * g.P + 1);
    for (int i = 0; i <= m * g.P; ++i) w[i] = 0.5 * hlen * wref(g, i, m);
    return w;
}

// Time steps per period on a box element (Sec. V bound with the z term).
int time_steps3(const Gll& g, double hx, double hy, double hz, double cmax, double omega,
                double cfl) {
    const double lam = cmax * cmax * g.mu *
                       ((2.0 / hx) * (2.0 / hx) + (2.0 / hy) * (2.0 / hy) + (2.0 / hz) * (2.0 / hz));
    const double arg = cfl * omega / std::sqrt(lam);
    if (arg >= 1.0) return 4;
    return std::max(4, (int)std::ceil(M_PI / std::asin(arg)));
}

template <typename Real>
int upload_real(unsigned char* dst, const std::vector<double>& v) {
    std::vector<Real> r(v.size());
    for (size_t i = 0; i < v.size(); ++i) r[i] = (Real)v[i];
    HIPCHK(hipMemcpy(dst, r.data(), sizeof(Real) * r.size(), hipMemcpyHostToDevice));
    return DD_OK;
}

int upload_as(const dd3_handle* h, unsigned char* dst, const std::vector<double>& v) {
    return h->opt.precision == DD_FP32 ? upload_real<float>(dst, v) : upload_real<double>(dst, v);
}

int prepare3(dd3_handle* h, const dd_box* box, int degree, const double* c, double omega,
             const dd_partition3* part, const dd_options* opt) {
    if (!box || !part || !c) return fail(DD_EINVAL, "null box, partition or wavespeed");
    if (degree < 1 || degree > wdd::kMaxP)
        return fail(DD_EINVAL, "degree %d not in [1, %d]", degree, wdd::kMaxP);
    if (box->nx < 1 || box->ny < 1 || box->nz < 1) return fail(DD_EINVAL, "empty box");
    const double lo[3] = {box->x0, box->y0, box->z0}, hi[3] = {box->x1, box->y1, box->z1};
    for (int d = 0; d < 3; ++d)
        if (!(hi[d] > lo[d]) || !std::isfinite(lo[d]) || !std::isfinite(hi[d]))
            return fail(DD_EINVAL, "degenerate box");
    if (!(omega > 0.0) || !std::isfinite(omega)) return fail(DD_EINVAL, "omega must be > 0");
    if (part->sx < 1 || part->sy < 1 || part->sz < 1 || box->nx % part->sx ||
        box->ny % part->sy || box->nz % part->sz)
        return fail(DD_EINVAL, "partition %dx%dx%d does not divide box %dx%dx%d", part->sx,
                    part->sy, part->sz, box->nx, box->ny, box->nz);
    dd_options o;
    if (opt)
        o = *opt;
    else
        dd_default_options(&o);
    if (o.precision != DD_FP64 && o.precision != DD_FP32) return fail(DD_EINVAL, "bad precision");
    if (o.max_wh < 1) return fail(DD_EINVAL, "max_wh must be >= 1");
    if (!(o.cfl > 0.0 && o.cfl <= 1.0)) return fail(DD_EINVAL, "cfl must be in (0, 1]");
    if (o.nt_override < 0 || o.nt_override == 1 || o.nt_override == 2)
        return fail(DD_EINVAL, "nt_override must be 0 or >= 3");
    if (!std::isfinite(o.tau_in)) return fail(DD_EINVAL, "tau_in must be finite");
    if (o.restart < 1 || o.restart > 400) return fail(DD_EINVAL, "restart must be in [1, 400]");
    if (o.refine < 0 || o.refine > 50) return fail(DD_EINVAL, "refine must be in [0, 50]");
    if (!(o.relax >= 0.0) || !std::isfinite(o.relax)) return fail(DD_EINVAL, "relax must be >= 0");
    const int P = degree;
    const int64_t Nx = (int64_t)box->nx * P + 1, Ny = (int64_t)box->ny * P + 1,
                  Nz = (int64_t)box->nz * P + 1;
    if (Nx * Ny * Nz > (int64_t)2000000000) return fail(DD_EINVAL, "box too large");
    const int mx = box->nx / part->sx, my = box->ny / part->sy, mz = box->nz / part->sz;
    const int nxl = mx * P + 1, nyl = my * P + 1, nzl = mz * P + 1;
    if ((int64_t)nxl * nyl * nzl > wdd::kMaxWG)
        return fail(DD_EINVAL, "subdomain of %dx%dx%d nodes exceeds 1024 (one node per thread)",
                    nxl, nyl, nzl);
    h->box = *box;
    h->part = *part;
    h->opt = o;
    h->P = P;
    h->omega = omega;
    h->Nx = (int)Nx;
    h->Ny = (int)Ny;
    h->Nz = (int)Nz;
    h->N = Nx * Ny * Nz;
    for (int64_t i = 0; i < h->N; ++i)
        if (!(c[i] > 0.0) || !std::isfinite(c[i]))
            return fail(DD_EINVAL, "wavespeed[%lld] = %g is not a positive number", (long long)i,
                        c[i]);
    h->mx = mx;
    h->my = my;
    h->mz = mz;
    h->nxl = nxl;
    h->nyl = nyl;
    h->nzl = nzl;
    h->nloc = (int64_t)nxl * nyl * nzl;
    h->L = (int64_t)part->sx * part->sy * part->sz;
    const int flen[6] = {nyl * nzl, nyl * nzl, nxl * nzl, nxl * nzl, nxl * nyl, nxl * nyl};
    int acc = 0;
    for (int s = 0; s < 6; ++s) {
        h->face_off[s] = acc;
        acc += flen[s];
    }
    h->per_sub = acc;
    h->n_if = h->L * h->per_sub;
    h->hx = (box->x1 - box->x0) / box->nx;
    h->hy = (box->y1 - box->y0) / box->ny;
    h->hz = (box->z1 - box->z0) / box->nz;
    const Gll g = make_gll(P);
    for (int a = 0; a <= P; ++a)
        for (int b = 0; b <= P; ++b) h->K1[a][b] = g.K[a][b];

    const int64_t L = h->L, nloc = h->nloc, nn = L * nloc;
    auto gnode = [&](int64_t l, int il, int jl, int kl) {
        const int a = (int)(l % part->sx), b = (int)((l / part->sx) % part->sy),
                  cc = (int)(l / ((int64_t)part->sx * part->sy));
        return ((int64_t)(cc * mz * P + kl) * Ny + (b * my * P + jl)) * Nx + a * mx * P + il;
    };
    // time steps and filter tables (deduplicated by N_t), as in the 2D setup
    h->nt.resize(L);
    std::map<int, int> toff;
    std::vector<double> kap, kaph, cs, sn;
    for (int64_t l = 0; l < L; ++l) {
        double cmax = 0.0;
        for (int kl = 0; kl < nzl; ++kl)
            for (int jl = 0; jl < nyl; ++jl)
                for (int il = 0; il < nxl; ++il) cmax = std::max(cmax, c[gnode(l, il, jl, kl)]);
        const int n = o.nt_override > 0 ? o.nt_override
                                        : time_steps3(g, h->hx, h->hy, h->hz, cmax, omega, o.cfl);
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
    // FP32 handles also run FP64 refinement sweeps (8-byte LDS grid)
    if (wdd::sweep3_lds_bytes(nxl, nyl, nzl, P, h->nt_max, 8) > kLdsLimit)
        return fail(DD_EINVAL, "subdomain %dx%dx%d nodes (P=%d, N_t=%d) exceeds the LDS", nxl,
                    nyl, nzl, P, h->nt_max);

    // per-node coefficients (Sec. IV lumped M, H; Sec. V alpha, beta)
    const std::vector<double> wx = line_weights(g, mx, h->hx), wy = line_weights(g, my, h->hy),
                              wz = line_weights(g, mz, h->hz);
    std::vector<double> alpha(nn), bX(nn), bY(nn), bZ(nn), beta(nn), kside(h->n_if);
    h->desc.resize(L);
    for (int64_t l = 0; l < L; ++l) {
        const int n = h->nt[l];
        const double half = M_PI / n;
        const double theta = std::tan(half) / omega;
        const double sigma = std::sin(half) / (0.5 * omega);
        for (int kl = 0; kl < nzl; ++kl)
            for (int jl = 0; jl < nyl; ++jl)
                for (int il = 0; il < nxl; ++il) {
                    const int64_t k = l * nloc + ((int64_t)kl * nyl + jl) * nxl + il;
                    const double cc = c[gnode(l, il, jl, kl)];
                    const double M = wx[il] * wy[jl] * wz[kl] / (cc * cc);
                    double Hs = 0.0;
                    if (il == 0) Hs += wy[jl] * wz[kl];
                    if (il == nxl - 1) Hs += wy[jl] * wz[kl];
                    if (jl == 0) Hs += wx[il] * wz[kl];
                    if (jl == nyl - 1) Hs += wx[il] * wz[kl];
                    if (kl == 0) Hs += wx[il] * wy[jl];
                    if (kl == nzl - 1) Hs += wx[il] * wy[jl];
                    const double H = Hs / cc;
                    alpha[k] = (M - theta * H) / (M + theta * H);
                    beta[k] = sigma / (M + theta * H);
                    bX[k] = beta[k] * (2.0 / h->hx) * wy[jl] * wz[kl];
                    bY[k] = beta[k] * (2.0 / h->hy) * wx[il] * wz[kl];
                    bZ[k] = beta[k] * (2.0 / h->hz) * wx[il] * wy[jl];
                }
        // omega / c at every face slot, in the g layout
        const int64_t o = l * h->per_sub;
        for (int kl = 0; kl < nzl; ++kl)
            for (int jl = 0; jl < nyl; ++jl) {
                kside[o + h->face_off[0] + kl * nyl + jl] = omega / c[gnode(l, 0, jl, kl)];
                kside[o + h->face_off[1] + kl * nyl + jl] = omega / c[gnode(l, nxl - 1, jl, kl)];
            }
        for (int kl = 0; kl < nzl; ++kl)
            for (int il = 0; il < nxl; ++il) {
                kside[o + h->face_off[2] + kl * nxl + il] = omega / c[gnode(l, il, 0, kl)];
                kside[o + h->face_off[3] + kl * nxl + il] = omega / c[gnode(l, il, nyl - 1, kl)];
            }
        for (int jl = 0; jl < nyl; ++jl)
            for (int il = 0; il < nxl; ++il) {
                kside[o + h->face_off[4] + jl * nxl + il] = omega / c[gnode(l, il, jl, 0)];
                kside[o + h->face_off[5] + jl * nxl + il] = omega / c[gnode(l, il, jl, nzl - 1)];
            }
        wdd::Sub3& d = h->desc[l];
        d = wdd::Sub3{};
        d.nt = n;
        d.toff = toff[n];
        d.node_off = l * nloc;
        d.if_off = o;
        d.gbase = gnode(l, 0, 0, 0);
        const int a = (int)(l % part->sx), b = (int)((l / part->sx) % part->sy),
                  cc = (int)(l / ((int64_t)part->sx * part->sy));
        const int da[6] = {-1, 1, 0, 0, 0, 0}, db[6] = {0, 0, -1, 1, 0, 0},
                  dc[6] = {0, 0, 0, 0, -1, 1}, opp[6] = {1, 0, 3, 2, 5, 4};
        for (int s = 0; s < 6; ++s) {
            const int a2 = a + da[s], b2 = b + db[s], c2 = cc + dc[s];
            if (a2 < 0 || a2 >= part->sx || b2 < 0 || b2 >= part->sy || c2 < 0 || c2 >= part->sz) {
                d.nbr_off[s] = -1;
            } else {
                const int64_t r = ((int64_t)c2 * part->sy + b2) * part->sx + a2;
                d.nbr_off[s] = r * h->per_sub + h->face_off[opp[s]];
            }
        }
        d.sigma = sigma;
        d.pd0c = omega * std::cos(M_PI / n);
        d.pd0s = omega * std::sin(M_PI / n);
        d.two_over_nt = 2.0 / n;
    }

    // global 1D weights, lumped M and H for the whole-box operator
    const std::vector<double> gx = line_weights(g, box->nx, h->hx),
                              gy = line_weights(g, box->ny, h->hy),
                              gz = line_weights(g, box->nz, h->hz);
    std::vector<double> Mg(h->N), Hg(h->N);
    for (int64_t k = 0; k < Nz; ++k)
        for (int64_t j = 0; j < Ny; ++j)
            for (int64_t i = 0; i < Nx; ++i) {
                const int64_t q = (k * Ny + j) * Nx + i;
                Mg[q] = gx[i] * gy[j] * gz[k] / (c[q] * c[q]);
                double Hs = 0.0;
                if (i == 0 || i == Nx - 1) Hs += gy[j] * gz[k] * ((i == 0) + (i == Nx - 1));
                if (j == 0 || j == Ny - 1) Hs += gx[i] * gz[k] * ((j == 0) + (j == Ny - 1));
                if (k == 0 || k == Nz - 1) Hs += gx[i] * gy[j] * ((k == 0) + (k == Nz - 1));
                Hg[q] = Hs / c[q];
            }

    // device buffers
    CHK(device_present(&h->dev));
    HIPCHK(hipSetDevice(h->dev));
    HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreate(&h->ev0));
    HIPCHK(hipEventCreate(&h->ev1));
    const size_t rs = real3(h);
    HIPCHK(h->d_desc.alloc(L));
    HIPCHK(h->d_coef.alloc(5 * nn * rs));
    HIPCHK(h->d_tab.alloc(4 * h->tab_len * rs));
    HIPCHK(h->d_w1d.alloc(nxl + nyl + nzl));
    HIPCHK(h->d_kside.alloc(h->n_if));
    HIPCHK(h->d_wx.alloc(Nx));
    HIPCHK(h->d_wy.alloc(Ny));
    HIPCHK(h->d_wz.alloc(Nz));
    HIPCHK(h->d_M.alloc(h->N));
    HIPCHK(h->d_H.alloc(h->N));
    HIPCHK(h->d_f.alloc(2 * h->N));
    HIPCHK(h->d_gin.alloc(h->n_if));
    HIPCHK(h->d_gout.alloc(h->n_if));
    HIPCHK(h->d_u.alloc(nn));
    HIPCHK(h->d_iters.alloc(L));
    HIPCHK(h->d_perm.alloc(nloc));
    {
        std::vector<int> perm(nloc);
        wdd::sweep3_thread_order(nxl, nyl, nzl, P, rs, perm.data());
        std::vector<char> seen(nloc, 0);
        for (int64_t t = 0; t < nloc; ++t) {
            if (perm[t] < 0 || perm[t] >= nloc || seen[perm[t]])
                return fail(DD_EINVAL, "internal: thread order is not a permutation");
            seen[perm[t]] = 1;
        }
        HIPCHK(hipMemcpy(h->d_perm.p, perm.data(), sizeof(int) * nloc, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(h->d_desc.p, h->desc.data(), sizeof(wdd::Sub3) * L, hipMemcpyHostToDevice));
    const std::vector<double>* coefs[5] = {&alpha, &bX, &bY, &bZ, &beta};
    for (int i = 0; i < 5; ++i) CHK(upload_as(h, h->d_coef.p + i * nn * rs, *coefs[i]));
    const std::vector<double>* tabs[4] = {&kap, &kaph, &cs, &sn};
    for (int i = 0; i < 4; ++i) CHK(upload_as(h, h->d_tab.p + i * h->tab_len * rs, *tabs[i]));
    if (o.precision == DD_FP32 && o.refine > 0) {
        HIPCHK(h->d_coef64.alloc(5 * nn * 8));
        HIPCHK(h->d_tab64.alloc(4 * h->tab_len * 8));
        for (int i = 0; i < 5; ++i)
            CHK(upload_real<double>(h->d_coef64.p + i * nn * 8, *coefs[i]));
        for (int i = 0; i < 4; ++i)
            CHK(upload_real<double>(h->d_tab64.p + i * h->tab_len * 8, *tabs[i]));
    }
    std::vector<double> w1d;
    w1d.insert(w1d.end(), wx.begin(), wx.end());
    w1d.insert(w1d.end(), wy.begin(), wy.end());
    w1d.insert(w1d.end(), wz.begin(), wz.end());
    HIPCHK(hipMemcpy(h->d_w1d.p, w1d.data(), 8 * w1d.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->d_kside.p, kside.data(), 8 * kside.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->d_wx.p, gx.data(), 8 * gx.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->d_wy.p, gy.data(), 8 * gy.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->d_wz.p, gz.data(), 8 * gz.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->d_M.p, Mg.data(), 8 * Mg.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->d_H.p, Hg.data(), 8 * Hg.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(h->d_gin.p, 0, sizeof(double2) * h->n_if));
    HIPCHK(hipMemset(h->d_u.p, 0, sizeof(double2) * nn));
    return DD_OK;
}

template <typename Real>
wdd::Sweep3Args<Real> sweep3_args(const dd3_handle* h, const double2* gi, double2* go, double src,
                                  bool with_f, double tau, int max_wh) {
    wdd::Sweep3Args<Real> a{};
    const int64_t nn = h->L * h->nloc;
    // FP64 sweeps of an FP32 handle read the FP64 copies
    const bool copy64 = sizeof(Real) == 8 && h->opt.precision == DD_FP32;
    const Real* coef = reinterpret_cast<const Real*>(copy64 ? h->d_coef64.p : h->d_coef.p);
    const Real* tab = reinterpret_cast<const Real*>(copy64 ? h->d_tab64.p : h->d_tab.p);
    a.desc = h->d_desc.p;
    a.n_items = (int)h->L;
    a.nxl = h->nxl;
    a.nyl = h->nyl;
    a.nzl = h->nzl;
    a.mx = h->mx;
    a.my = h->my;
    a.mz = h->mz;
    a.P = h->P;
    a.per_sub = (int)h->per_sub;
    a.perm = h->d_perm.p;
    for (int s = 0; s < 6; ++s) a.face_off[s] = h->face_off[s];
    a.alpha = coef;
    a.betaX = coef + nn;
    a.betaY = coef + 2 * nn;
    a.betaZ = coef + 3 * nn;
    a.beta = coef + 4 * nn;
    a.Nx = h->Nx;
    a.Ny = h->Ny;
    a.f_re = with_f ? h->d_f.p : nullptr;
    a.f_im = with_f ? h->d_f.p + h->N : nullptr;
    a.w1d = h->d_w1d.p;
    a.kside = h->d_kside.p;
    a.kap = tab;
    a.kaph = tab + h->tab_len;
    a.cs = tab + 2 * h->tab_len;
    a.sn = tab + 3 * h->tab_len;
    a.g_in = gi;
    a.g_out = go;
    a.src = src;
    a.u = h->d_u.p;
    a.wh_iters = h->d_iters.p;
    a.tau = tau;
    a.max_wh = max_wh;
    a.lds_bytes = wdd::sweep3_lds_bytes(h->nxl, h->nyl, h->nzl, h->P, h->nt_max, sizeof(Real));
    for (int i = 0; i <= h->P; ++i)
        for (int j = 0; j <= h->P; ++j) a.K1[i][j] = h->K1[i][j];
    return a;
}

// One launch over all box subdomains (g_in -> g_out); optionally timed with
// events.  Accumulates the WaveHoltz counts of the launch.
int run_sweep3_io(dd3_handle* h, const double2* gi, double2* go, double src, bool with_f,
                  double tau, int max_wh, float* ms, int prec = -1) {
    const int wg = (int)(((h->nloc + 63) / 64) * 64);
    if (prec < 0) prec = h->opt.precision;
    if (prec == DD_FP64 && h->opt.precision == DD_FP32 && !h->d_coef64.p)
        return fail(DD_EINVAL, "FP64 sweeps of an FP32 box handle need refine > 0");
    if (ms) HIPCHK(hipEventRecord(h->ev0, h->stream));
    hipError_t e;
    if (prec == DD_FP32)
        e = wdd::launch_sweep3<float>(sweep3_args<float>(h, gi, go, src, with_f, tau, max_wh), wg,
                                      h->stream);
    else
        e = wdd::launch_sweep3<double>(sweep3_args<double>(h, gi, go, src, with_f, tau, max_wh), wg,
                                       h->stream);
    HIPCHK(e);
    if (ms) HIPCHK(hipEventRecord(h->ev1, h->stream));
    std::vector<int> its(h->L);
    HIPCHK(hipMemcpyAsync(its.data(), h->d_iters.p, sizeof(int) * h->L, hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (ms) HIPCHK(hipEventElapsedTime(ms, h->ev0, h->ev1));
    h->sweeps += 1;
    for (int64_t l = 0; l < h->L; ++l) {
        h->wh_total += its[l];
        h->wh_max = std::max(h->wh_max, its[l]);
        h->dof_updates += (double)h->nloc * (h->nt[l] - 1) * its[l];
        if (its[l] < 1) return fail(DD_EHIP, "box sweep reported no WaveHoltz iteration");
    }
    return DD_OK;
}

int run_sweep3(dd3_handle* h, double src, bool with_f, double tau, int max_wh, float* ms) {
    return run_sweep3_io(h, h->d_gin.p, h->d_gout.p, src, with_f, tau, max_wh, ms);
}

int ensure_solver3(dd3_handle* h) {
    if (h->d_V.p) return DD_OK;
    const int m = h->opt.restart;
    h->ld = ((h->n_if + 63) / 64) * 64;
    HIPCHK(h->d_V.alloc((size_t)(m + 1) * h->ld));
    HIPCHK(h->d_r.alloc(h->n_if));
    HIPCHK(h->d_coefs.alloc(m + 1));
    HIPCHK(h->d_h.alloc(h->n_if));
    HIPCHK(h->d_G.alloc(h->n_if));
    HIPCHK(h->d_tmp.alloc(h->n_if));
    HIPCHK(h->d_ug.alloc(h->N));
    HIPCHK(h->d_Su.alloc(h->N));
    HIPCHK(h->d_work.alloc(h->N));
    HIPCHK(h->d_res.alloc(h->n_if));
    HIPCHK(h->d_D.alloc(h->n_if));
    HIPCHK(wdd::blas_init(h->blas, m + 2, h->stream));
    return DD_OK;
}

wdd::Operator3Args op3_args(const dd3_handle* h) {
    wdd::Operator3Args a{};
    a.Nx = h->Nx;
    a.Ny = h->Ny;
    a.Nz = h->Nz;
    a.P = h->P;
    a.nx = h->box.nx;
    a.ny = h->box.ny;
    a.nz = h->box.nz;
    // z chunks: enough workgroups to fill the chip (about 2048), chunks of
    // at least 4P planes so the 2P-plane warm-up of the z window stays small
    const int64_t tiles = (int64_t)((h->Nx + 63) / 64) * ((h->Ny + 3) / 4);
    const int64_t nkc = std::max<int64_t>(1, std::min<int64_t>((2048 + tiles - 1) / tiles,
                                                               h->Nz / (4 * h->P)));
    a.kchunk = (int)((h->Nz + nkc - 1) / nkc);
    a.sx_ref = 2.0 / h->hx;
    a.sy_ref = 2.0 / h->hy;
    a.sz_ref = 2.0 / h->hz;
    a.wx = h->d_wx.p;
    a.wy = h->d_wy.p;
    a.wz = h->d_wz.p;
    a.M = h->d_M.p;
    a.H = h->d_H.p;
    a.omega = h->omega;
    for (int i = 0; i <= h->P; ++i)
        for (int j = 0; j <= h->P; ++j) a.K1[i][j] = h->K1[i][j];
    return a;
}

}  // namespace

extern "C" {

void dd3_destroy(dd3_handle* h) {
    if (!h) return;
    if (h->stream) (void)hipSetDevice(h->dev);
    dd3_free(h);
    delete h;
}

int dd3_setup(dd3_handle** out, const dd_box* box, int degree, const double* wavespeed,
              double omega, const dd_partition3* part, const dd_options* opt) {
    if (!out) return fail(DD_EINVAL, "null output handle pointer");
    *out = nullptr;
    dd3_handle* h = new dd3_handle();
    const int rc = prepare3(h, box, degree, wavespeed, omega, part, opt);
    if (rc != DD_OK) {
        dd3_destroy(h);
        return rc;
    }
    *out = h;
    return DD_OK;
}

int dd3_sizes(const dd3_handle* h, int64_t* n_global, int64_t* n_local, int64_t* n_sub,
              int64_t* n_iface) {
    CHK(validate3(h));
    if (n_global) *n_global = h->N;
    if (n_local) *n_local = h->nloc;
    if (n_sub) *n_sub = h->L;
    if (n_iface) *n_iface = h->n_if;
    return DD_OK;
}

int dd3_time_steps(const dd3_handle* h, int* nt) {
    CHK(validate3(h));
    if (!nt) return fail(DD_EINVAL, "null output");
    std::copy(h->nt.begin(), h->nt.end(), nt);
    return DD_OK;
}

int dd3_mesh_coords(const dd_box* box, int degree, double* x, double* y, double* z) {
    if (!box || !x || !y || !z) return fail(DD_EINVAL, "null argument");
    if (degree < 1 || degree > wdd::kMaxP)
        return fail(DD_EINVAL, "degree %d not in [1, %d]", degree, wdd::kMaxP);
    if (box->nx < 1 || box->ny < 1 || box->nz < 1) return fail(DD_EINVAL, "empty box");
    const Gll g = make_gll(degree);
    const int P = degree;
    auto axis = [&](int n, double a, double b) {
        const double hh = (b - a) / n;
        std::vector<double> v(n * P + 1);
        for (int e = 0; e < n; ++e)
            for (int q = 0; q <= P; ++q) v[e * P + q] = a + e * hh + 0.5 * hh * (g.x[q] + 1.0);
        v[n * P] = b;
        return v;
    };
    const std::vector<double> xs = axis(box->nx, box->x0, box->x1),
                              ys = axis(box->ny, box->y0, box->y1),
                              zs = axis(box->nz, box->z0, box->z1);
    int64_t q = 0;
    for (double zz : zs)
        for (double yy : ys)
            for (double xx : xs) {
                x[q] = xx;
                y[q] = yy;
                z[q] = zz;
                ++q;
            }
    return DD_OK;
}

int dd3_sweep(dd3_handle* h, const double* g_re, const double* g_im, const double* f_re,
              const double* f_im, double src, double* g_out_re, double* g_out_im, double* u_re,
              double* u_im, int* wh_iters) {
    CHK(validate3(h));
    if (!g_out_re || !g_out_im) return fail(DD_EINVAL, "null output");
    if (!std::isfinite(src)) return fail(DD_EINVAL, "src must be finite");
    if (!f_re && f_im) return fail(DD_EINVAL, "f_im given without f_re");
    CHK(check_finite(g_re, h->n_if, "g_re"));
    CHK(check_finite(g_im, h->n_if, "g_im"));
    CHK(check_finite(f_re, h->N, "f_re"));
    CHK(check_finite(f_im, h->N, "f_im"));
    HIPCHK(hipSetDevice(h->dev));
    std::vector<double2> gi(h->n_if);
    for (int64_t i = 0; i < h->n_if; ++i)
        gi[i] = make_double2(g_re ? g_re[i] : 0.0, g_im ? g_im[i] : 0.0);
    HIPCHK(hipMemcpy(h->d_gin.p, gi.data(), sizeof(double2) * h->n_if, hipMemcpyHostToDevice));
    const bool with_f = f_re != nullptr;
    if (with_f) {
        HIPCHK(hipMemcpy(h->d_f.p, f_re, 8 * h->N, hipMemcpyHostToDevice));
        if (f_im)
            HIPCHK(hipMemcpy(h->d_f.p + h->N, f_im, 8 * h->N, hipMemcpyHostToDevice));
        else
            HIPCHK(hipMemset(h->d_f.p + h->N, 0, 8 * h->N));
    }
    const double tau = h->opt.tau_in > 0.0 ? h->opt.tau_in : 0.0;
    CHK(run_sweep3(h, src, with_f, tau, h->opt.max_wh, nullptr));
    HIPCHK(hipMemcpy(gi.data(), h->d_gout.p, sizeof(double2) * h->n_if, hipMemcpyDeviceToHost));
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
    if (wh_iters)
        HIPCHK(hipMemcpy(wh_iters, h->d_iters.p, sizeof(int) * h->L, hipMemcpyDeviceToHost));
    return DD_OK;
}

int dd3_time_sweep(dd3_handle* h, int reps, int fixed_iters, double* ms, double* dof_updates) {
    CHK(validate3(h));
    if (reps < 1 || !ms || fixed_iters < 0)
        return fail(DD_EINVAL, "reps must be >= 1, fixed_iters >= 0, ms non-null");
    HIPCHK(hipSetDevice(h->dev));
    const double tau = fixed_iters > 0 ? 0.0 : std::max(h->opt.tau_in, 0.0);
    const int mwh = fixed_iters > 0 ? fixed_iters : h->opt.max_wh;
    float t = 0.f;
    CHK(run_sweep3(h, 0.0, false, tau, mwh, &t));
    double total = 0.0;
    for (int r = 0; r < reps; ++r) {
        CHK(run_sweep3(h, 0.0, false, tau, mwh, &t));
        total += t;
    }
    *ms = total / reps;
    if (dof_updates) {
        std::vector<int> its(h->L);
        HIPCHK(hipMemcpy(its.data(), h->d_iters.p, sizeof(int) * h->L, hipMemcpyDeviceToHost));
        double du = 0.0;
        for (int64_t l = 0; l < h->L; ++l) du += (double)h->nloc * (h->nt[l] - 1) * its[l];
        *dof_updates = du;
    }
    return DD_OK;
}

int dd3_apply_operator_device(dd3_handle* h, void* stream, const double* d_x, double* d_y) {
    CHK(validate3(h));
    if (!d_x || !d_y) return fail(DD_EINVAL, "null array");
    HIPCHK(hipSetDevice(h->dev));
    hipStream_t s = stream ? (hipStream_t)stream : h->stream;
    HIPCHK(wdd::launch_operator3(op3_args(h), (const double2*)d_x, (double2*)d_y, s));
    return DD_OK;
}

int dd3_solve(dd3_handle* h, const double* f_re, const double* f_im, double tol, int max_iter,
              double* u_re, double* u_im, dd_stats* st) {
    CHK(validate3(h));
    if (!u_re || !u_im) return fail(DD_EINVAL, "null output");
    if (!(tol > 0.0) || max_iter < 1) return fail(DD_EINVAL, "tol must be > 0, max_iter >= 1");
    if (!f_re && f_im) return fail(DD_EINVAL, "f_im given without f_re");
    CHK(check_finite(f_re, h->N, "f_re"));
    CHK(check_finite(f_im, h->N, "f_im"));
    HIPCHK(hipSetDevice(h->dev));
    const auto t0 = std::chrono::steady_clock::now();
    CHK(ensure_solver3(h));
    const bool with_f = f_re != nullptr;
    if (with_f) {
        HIPCHK(hipMemcpy(h->d_f.p, f_re, 8 * h->N, hipMemcpyHostToDevice));
        if (f_im)
            HIPCHK(hipMemcpy(h->d_f.p + h->N, f_im, 8 * h->N, hipMemcpyHostToDevice));
        else
            HIPCHK(hipMemset(h->d_f.p + h->N, 0, 8 * h->N));
    }
    h->sweeps = h->wh_total = 0;
    h->wh_max = 0;
    h->dof_updates = 0.0;
    const double tau = std::max(h->opt.tau_in, 0.0);
    const int mwh = h->opt.max_wh;
    // FP64 iterative refinement (the 2D reading of the reduced-precision
    // outer iteration): residuals r = h - (I - T) G from FP64 sweeps,
    // corrections G += GMRES((I - T) d = r) with sweeps in the handle's
    // precision and, with relax > 0, a variable inner tolerance.  A strict
    // FP64 solve finishes in the first pass (plain GMRES from G = 0).
    const bool fp32 = h->opt.precision == DD_FP32;
    const bool refine = h->opt.refine > 0 && (fp32 || h->opt.relax > 0.0);
    const bool fp32_refined = fp32 && refine;
    const int rprec = refine ? DD_FP64 : h->opt.precision;
    const double rtau = fp32_refined ? std::min(1e-8, std::max(1e-13, 0.01 * tol)) : tau;
    const int passes = refine ? 1 + h->opt.refine : 1;
    const double relax = h->opt.relax;
    // h = sweep(0, sources on): the affine part of the sweep map (no outer
    // boundary data in the box problem)
    HIPCHK(hipMemsetAsync(h->d_tmp.p, 0, sizeof(double2) * h->n_if, h->stream));
    CHK(run_sweep3_io(h, h->d_tmp.p, h->d_h.p, 1.0, with_f, rtau, mwh, nullptr, rprec));
    Krylov K{};
    K.blas = &h->blas;
    K.stream = h->stream;
    K.n = h->n_if;
    K.ld = h->ld;
    K.m = h->opt.restart;
    K.V = h->d_V.p;
    K.r = h->d_r.p;
    K.coefs = h->d_coefs.p;
    K.matvec = [h, mwh](const double2* v, double2* w, double t) {
        CHK(run_sweep3_io(h, v, w, 0.0, false, t, mwh, nullptr));
        return kaxpby(Krylov{&h->blas, h->stream, h->n_if}, cplx(1.0), v, cplx(-1.0), w);
    };
    // inexact Krylov: the matvec tolerance may grow as 1 / (residual),
    // tau_k = clamp(relax * tol / rel_k, tau_in, 1e-2) (relax = 0: tau_in)
    K.tau = [tau, relax, tol](double rel) {
        if (!(relax > 0.0)) return tau;
        return std::min(1e-2, std::max(tau, relax * tol / std::max(rel, 1e-300)));
    };
    K.tau_strict = tau;
    const double hn = knorm(K, h->d_h.p);
    if (!std::isfinite(hn)) return fail(DD_ENAN, "non-finite interface data");
    HIPCHK(hipMemsetAsync(h->d_G.p, 0, sizeof(double2) * h->n_if, h->stream));
    HIPCHK(hipMemcpyAsync(h->d_res.p, h->d_h.p, sizeof(double2) * h->n_if,
                          hipMemcpyDeviceToDevice, h->stream));
    int its = 0, steps = 0;
    double rnorm = hn, rtrue = hn > 0.0 ? 1.0 : 0.0, last_rec = rtrue;
    bool have_u = false;
    for (int k = 0; k < passes && rtrue > tol && its < max_iter; ++k) {
        // FP32 corrections under refinement aim at a fixed reduction (their
        // operator is only FP32-accurate); a single pass goes the whole way
        const double want = tol * hn / rnorm;
        const double inner = fp32_refined ? std::max(1e-4, want) : want;
        int pits = 0;
        double irel = 0.0;
        CHK(gmres_core(K, h->d_res.p, h->d_D.p, rnorm, inner, max_iter - its, &pits, &irel));
        its += pits;
        last_rec = irel * rnorm / hn;
        CHK(kaxpby(K, cplx(1.0), h->d_D.p, cplx(1.0), h->d_G.p));
        // true residual and u from the sweep of G with sources on:
        // g_fin = T G + h, r = g_fin - G
        CHK(run_sweep3_io(h, h->d_G.p, h->d_tmp.p, 1.0, with_f, rtau, mwh, nullptr, rprec));
        CHK(kaxpby(K, cplx(-1.0), h->d_G.p, cplx(1.0), h->d_tmp.p));
        rnorm = knorm(K, h->d_tmp.p);
        if (!std::isfinite(rnorm)) return fail(DD_ENAN, "non-finite outer residual");
        rtrue = hn > 0.0 ? rnorm / hn : 0.0;
        HIPCHK(hipMemcpyAsync(h->d_res.p, h->d_tmp.p, sizeof(double2) * h->n_if,
                              hipMemcpyDeviceToDevice, h->stream));
        steps = k + 1;
        have_u = true;
    }
    if (!have_u) {
        // nothing to correct (h = 0): u from the sweep of G = 0
        CHK(run_sweep3_io(h, h->d_G.p, h->d_tmp.p, 1.0, with_f, rtau, mwh, nullptr, rprec));
        rtrue = 0.0;
        last_rec = 0.0;
    }
    double rel = std::max(last_rec, rtrue);
    HIPCHK(wdd::launch_glue3(op3_args(h), h->d_u.p, h->mx, h->my, h->mz, h->part.sx, h->part.sy,
                             h->part.sz, h->d_ug.p, h->stream));
    std::vector<double2> u(h->N);
    HIPCHK(hipMemcpyAsync(u.data(), h->d_ug.p, sizeof(double2) * h->N, hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int64_t i = 0; i < h->N; ++i) {
        u_re[i] = u[i].x;
        u_im[i] = u[i].y;
    }
    if (!std::isfinite(rel)) return fail(DD_ENAN, "non-finite outer residual");
    if (st) {
        *st = dd_stats{};
        st->outer_iters = its;
        st->refine_steps = refine ? steps : 0;  // passes with an FP64 residual
        st->sweeps = (int)h->sweeps;
        st->rel_residual = rel;
        st->true_rel_residual = rtrue;
        st->wh_iters_total = h->wh_total;
        st->wh_iters_max = h->wh_max;
        st->nt_min = *std::min_element(h->nt.begin(), h->nt.end());
        st->nt_max = h->nt_max;
        st->dof_updates = h->dof_updates;
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return rel <= tol ? DD_OK : DD_ENOTCONV;
}

int dd3_residual(dd3_handle* h, const double* u_re, const double* u_im, const double* f_re,
                 const double* f_im, double* rel) {
    CHK(validate3(h));
    if (!u_re || !u_im || !rel) return fail(DD_EINVAL, "null argument");
    if (!f_re && f_im) return fail(DD_EINVAL, "f_im given without f_re");
    CHK(check_finite(u_re, h->N, "u_re"));
    CHK(check_finite(u_im, h->N, "u_im"));
    CHK(check_finite(f_re, h->N, "f_re"));
    CHK(check_finite(f_im, h->N, "f_im"));
    HIPCHK(hipSetDevice(h->dev));
    CHK(ensure_solver3(h));
    std::vector<double2> u(h->N);
    for (int64_t i = 0; i < h->N; ++i) u[i] = make_double2(u_re[i], u_im[i]);
    HIPCHK(hipMemcpy(h->d_ug.p, u.data(), sizeof(double2) * h->N, hipMemcpyHostToDevice));
    if (f_re) {
        HIPCHK(hipMemcpy(h->d_f.p, f_re, 8 * h->N, hipMemcpyHostToDevice));
        if (f_im)
            HIPCHK(hipMemcpy(h->d_f.p + h->N, f_im, 8 * h->N, hipMemcpyHostToDevice));
        else
            HIPCHK(hipMemset(h->d_f.p + h->N, 0, 8 * h->N));
    }
    HIPCHK(wdd::launch_operator3(op3_args(h), h->d_ug.p, h->d_Su.p, h->stream));
    HIPCHK(wdd::launch_residual3(op3_args(h), f_re ? h->d_f.p : nullptr,
                                 f_re ? h->d_f.p + h->N : nullptr, h->d_Su.p, h->d_work.p,
                                 h->stream));
    HIPCHK(wdd::blas_sum2(h->blas, h->d_work.p, h->N, h->stream));
    double2 sums;
    HIPCHK(hipMemcpyAsync(&sums, h->blas.result, sizeof(double2), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    *rel = sums.y > 0.0 ? std::sqrt(sums.x / sums.y) : std::sqrt(sums.x);
    return DD_OK;
}

}  // extern "C"
