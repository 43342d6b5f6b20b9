// extern "C" entry points of the device side: argument validation on the
// host, workspace carving, launch sequencing and optional per-kernel timing.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "apply.h"
#include "fused_kernel.h"
#include "status.h"
#include "tangent.h"
#include <rocprofiler-sdk-roctx/roctx.h>

using namespace vk;

// FP32 path: a point is recomputed in double when one of its pivots falls
// below 2^-kDefaultRedoLog2 * K_ii (view->redo_log2 == 0).  Emulated on the
// CPU (exact solves of float-rounded K_cc on the radial Matern and clumped
// squared-exponential clouds), the points kept in float below 2^-8 move the
// forward result by up to ~1e-5 of max|v|; at 2^-16 by up to ~1e-3.
constexpr int kDefaultRedoLog2 = 8;

namespace {

// ---- per-kernel timing with HIP events on the launch stream ---------------
struct Pending {
    const char* name;
    hipEvent_t a, b;
};
struct KernelTotal {
    std::string name;
    double ms = 0.0;
    int64_t launches = 0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_event_pool;
std::vector<KernelTotal> g_totals;

hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

template <class F>
hipError_t timed(const char* name, hipStream_t s, F&& launch) {
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        on = g_prof_on;
    }
    if (!on) return launch();
    hipEvent_t a, b;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        a = take_event();
        b = take_event();
    }
    if (!a || !b) return launch();
    (void)hipEventRecord(a, s);
    hipError_t err = launch();
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_pending.push_back(Pending{name, a, b});
    return err;
}

int hip_fail(hipError_t e, const char* where) {
    return vecchia_set_error(VECCHIA_EHIP, "%s: %s", where, hipGetErrorString(e));
}

// A named roctx range around each call of the path (shown by a marker trace,
// e.g. rocprofv3 --marker-trace; a flag check when no tool is attached).
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

int check_kernel(const vecchia_kernel* k) {
    if (!k) return vecchia_set_error(VECCHIA_EINVAL, "kernel is NULL");
    if (k->kind < 0 || k->kind > 4) return vecchia_set_error(VECCHIA_EINVAL, "kernel kind %d not in {0,...,4}", k->kind);
    if (k->kind == 4 && !(k->nu >= VECCHIA_NU_MIN && k->nu <= VECCHIA_NU_MAX))
        return vecchia_set_error(VECCHIA_EINVAL, "kernel nu must lie in [%g, %g]", VECCHIA_NU_MIN, VECCHIA_NU_MAX);
    if (!(k->sigma > 0.0) || !std::isfinite(k->sigma)) return vecchia_set_error(VECCHIA_EINVAL, "kernel sigma must be > 0");
    if (!(k->ell > 0.0) || !std::isfinite(k->ell)) return vecchia_set_error(VECCHIA_EINVAL, "kernel ell must be > 0");
    if (!(k->nugget >= 0.0) || !std::isfinite(k->nugget)) return vecchia_set_error(VECCHIA_EINVAL, "kernel nugget must be >= 0");
    return VECCHIA_OK;
}

// The general Matern kernel is built into the factor kernels that evaluate
// covariances in double (FP64 views, and k = 64 for both precisions) only;
// the entry points with their own kernel evaluations refuse it.
int check_closed_form(const vecchia_kernel* k, const char* who) {
    if (k->kind == 4)
        return vecchia_set_error(VECCHIA_EUNSUPPORTED, "%s: the general Matern kernel is supported by vecchia_factor "
                                 "(FP64 views, or k = 64) only", who);
    return VECCHIA_OK;
}

// Checks shared by the stored-factor view and the fused forward's view
// (everything but the workspace size).
int check_view_common(const vecchia_view* v, const char* who) {
    if (!v) return vecchia_set_error(VECCHIA_EINVAL, "%s: view is NULL", who);
    if (v->n < 1 || v->n >= (int64_t(1) << 31)) return vecchia_set_error(VECCHIA_EINVAL, "%s: need 1 <= N < 2^31", who);
    if (v->k < 1) return vecchia_set_error(VECCHIA_EINVAL, "%s: need k >= 1", who);
    if (v->k > VECCHIA_KMAX)
        return vecchia_set_error(VECCHIA_EUNSUPPORTED, "%s: k=%d exceeds the compiled maximum %d", who, v->k, VECCHIA_KMAX);
    if (v->kp != vecchia_padded_k(v->k))
        return vecchia_set_error(VECCHIA_EINVAL, "%s: kp=%d does not match k=%d (expected %d)", who, v->kp, v->k,
                                 vecchia_padded_k(v->k));
    if (v->n0 < 1 || v->n0 > v->n) return vecchia_set_error(VECCHIA_EINVAL, "%s: need 1 <= n0 <= N", who);
    if (v->n0 > VECCHIA_N0MAX)
        return vecchia_set_error(VECCHIA_EUNSUPPORTED, "%s: n0=%d exceeds the compiled maximum %d", who, v->n0, VECCHIA_N0MAX);
    if (v->precision != VECCHIA_FP64 && v->precision != VECCHIA_FP32)
        return vecchia_set_error(VECCHIA_EINVAL, "%s: precision must be VECCHIA_FP64 or VECCHIA_FP32", who);
    if (!v->x || !v->nbr || !v->level_ptr || !v->workspace)
        return vecchia_set_error(VECCHIA_EINVAL, "%s: x, nbr, level_ptr and workspace must be set", who);
    if (v->n_levels < 0) return vecchia_set_error(VECCHIA_EINVAL, "%s: n_levels < 0", who);
    const int32_t* lp = v->level_ptr;
    if (lp[0] != 0 || lp[1] != v->n0 || lp[v->n_levels + 1] != v->n)
        return vecchia_set_error(VECCHIA_EINVAL, "%s: level_ptr must start 0, n0 and end at N", who);
    for (int l = 1; l <= v->n_levels; ++l)
        if (lp[l + 1] < lp[l]) return vecchia_set_error(VECCHIA_EINVAL, "%s: level_ptr not ascending at %d", who, l);
    if (reinterpret_cast<uintptr_t>(v->workspace) & 255)
        return vecchia_set_error(VECCHIA_EINVAL, "%s: workspace must be 256-byte aligned", who);
    return VECCHIA_OK;
}

int check_view(const vecchia_view* v, Layout* lay, const char* who) {
    const int rc = check_view_common(v, who);
    if (rc) return rc;
    *lay = workspace_layout(v->n, v->kp, v->n0, v->precision);
    if (v->workspace_bytes < lay->total)
        return vecchia_set_error(VECCHIA_ENOMEM, "%s: workspace has %zu bytes, needs %zu", who, v->workspace_bytes, lay->total);
    return VECCHIA_OK;
}

int check_fused_view(const vecchia_view* v, FusedLayout* lay, const char* who) {
    const int rc = check_view_common(v, who);
    if (rc) return rc;
    *lay = fused_layout(v->n, v->n0);
    if (v->workspace_bytes < lay->total)
        return vecchia_set_error(VECCHIA_ENOMEM, "%s: workspace has %zu bytes, needs %zu", who, v->workspace_bytes, lay->total);
    return VECCHIA_OK;
}

template <typename T>
T* ws(const vecchia_view* v, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(v->workspace) + off);
}

}  // namespace

extern "C" int vecchia_workspace_bytes(int64_t n, int32_t k, int32_t n0, int32_t precision, size_t* bytes) {
    if (!bytes) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_workspace_bytes: bytes is NULL");
    if (k < 1) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_workspace_bytes: need k >= 1");
    if (k > VECCHIA_KMAX)
        return vecchia_set_error(VECCHIA_EUNSUPPORTED, "vecchia_workspace_bytes: k=%d exceeds the compiled maximum %d", k,
                                 VECCHIA_KMAX);
    const int kp = vecchia_padded_k(k);
    if (n < 1 || n0 < 1 || n0 > n) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_workspace_bytes: need 1 <= n0 <= N");
    if (precision != VECCHIA_FP64 && precision != VECCHIA_FP32)
        return vecchia_set_error(VECCHIA_EINVAL, "vecchia_workspace_bytes: bad precision");
    *bytes = workspace_layout(n, kp, n0, precision).total;
    return VECCHIA_OK;
}

extern "C" int vecchia_factor(vecchia_view* view, const vecchia_kernel* kern, void* stream) {
    vecchia_clear_error();
    TraceRange trace_range("vecchia_factor");
    Layout lay;
    int rc = check_view(view, &lay, "vecchia_factor");
    if (rc) return rc;
    if ((rc = check_kernel(kern))) return rc;
    if (kern->kind == 4 && view->precision != VECCHIA_FP64 && view->kp != 64)
        return vecchia_set_error(VECCHIA_EUNSUPPORTED, "vecchia_factor: the general Matern kernel needs an FP64 view "
                                 "or k = 64 (whose factor is in FP64 for both storage precisions)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    view->kernel = *kern;
    hipError_t e = timed("factor_dense", s, [&] {
        return launch_factor_dense(view->precision, kern->kind, view->x, view->n0, *kern, ws<double>(view, lay.l0),
                                   ws<double>(view, lay.ld0), ws<uint64_t>(view, lay.status), s);
    });
    if (e != hipSuccess) return hip_fail(e, "vecchia_factor (dense block)");
    FactorLaunch a;
    a.precision = view->precision;
    a.kp = view->kp;
    a.kind = kern->kind;
    a.n = view->n;
    a.ns = lay.ns;
    a.n0 = view->n0;
    a.x = view->x;
    a.nbr = view->nbr;
    a.b = ws<char>(view, lay.b);
    a.sigma = ws<char>(view, lay.sigma);
    a.ldpart = ws<double>(view, lay.ldpart);
    a.ldfix = ws<long long>(view, lay.ldfix);
    a.status = ws<uint64_t>(view, lay.status);
    a.redo = ws<uint32_t>(view, lay.redo);
    {
        const int bits = view->redo_log2 == 0 ? kDefaultRedoLog2 : view->redo_log2;
        a.redo_ratio = bits < 0 ? 0.0 : std::ldexp(1.0, -bits);
    }
    a.kern = *kern;
    if (lay.ns > 0) {
        // FP32: the policy sample, the float pass and the double pass are
        // timed apart; FP64 has the main pass only
        if (view->precision == VECCHIA_FP32 && a.redo_ratio > 0.0) {
            a.stages = kStageProbe;
            e = timed("factor_probe", s, [&] { return launch_factor_sparse(a, s); });
            if (e != hipSuccess) return hip_fail(e, "vecchia_factor (precision sample)");
        }
        a.stages = kStageMain;
        e = timed("factor_sparse", s, [&] { return launch_factor_sparse(a, s); });
        if (e != hipSuccess) return hip_fail(e, "vecchia_factor (sparse points)");
        if (view->precision == VECCHIA_FP32) {
            a.stages = kStageRedo;
            e = timed("factor_redo", s, [&] { return launch_factor_sparse(a, s); });
            if (e != hipSuccess) return hip_fail(e, "vecchia_factor (points recomputed in double)");
        }
    }
    return VECCHIA_OK;
}

extern "C" int vecchia_forward(const vecchia_view* view, const void* xi, void* v, void* stream) {
    vecchia_clear_error();
    TraceRange trace_range("vecchia_forward");
    Layout lay;
    int rc = check_view(view, &lay, "vecchia_forward");
    if (rc) return rc;
    if (!xi || !v) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_forward: xi and v must be set");
    if (xi == v) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_forward: xi and v must not alias");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = timed("forward_dense", s, [&] {
        return launch_forward_dense(view->precision, ws<double>(view, lay.l0), view->n0, xi, v, s);
    });
    if (e != hipSuccess) return hip_fail(e, "vecchia_forward (dense block)");
    const int32_t* lp = view->level_ptr;
    const int L = view->n_levels;
    const int64_t lds_cap = kRunLdsBytes / (view->precision == VECCHIA_FP32 ? 4 : 8);
    for (int l = 1; l <= L;) {
        // A run of at least two consecutive small batches goes to one
        // workgroup.  Its LDS holds positions [lo, run_end): the whole prefix
        // (lo = 0) while that fits, else the run's own positions (lo = its
        // first position); the run stops before it would outgrow the LDS.
        int run_end = l;
        if (view->level_ptr_dev) {
            while (run_end <= L && lp[run_end + 1] - lp[run_end] <= kRunMaxPoints) {
                const int64_t end_pos = lp[run_end + 1];
                if (end_pos > lds_cap && end_pos - lp[l] > lds_cap) break;
                ++run_end;
            }
        }
        if (run_end - l >= 2) {
            const int l0 = l;
            const int64_t end_pos = lp[run_end];
            const int64_t lo = end_pos <= lds_cap ? 0 : (int64_t)lp[l];
            e = timed("forward_run", s, [&] {
                return launch_forward_run(view->precision, view->kp, view->nbr, ws<char>(view, lay.b),
                                          ws<char>(view, lay.sigma), xi, v, view->n0, view->level_ptr_dev, l0, run_end,
                                          lo, end_pos, s);
            });
            if (e != hipSuccess) return hip_fail(e, "vecchia_forward (run of small batches)");
            l = run_end;
            continue;
        }
        const int64_t a = lp[l] - view->n0, b = lp[l + 1] - view->n0;
        e = timed("forward_level", s, [&] {
            return launch_forward_level(view->precision, view->kp, view->nbr, ws<char>(view, lay.b),
                                        ws<char>(view, lay.sigma), xi, v, view->n0, a, b, s);
        });
        if (e != hipSuccess) return hip_fail(e, "vecchia_forward (level)");
        ++l;
    }
    return VECCHIA_OK;
}

extern "C" int vecchia_inverse(const vecchia_view* view, const void* v, void* xi, void* stream) {
    vecchia_clear_error();
    TraceRange trace_range("vecchia_inverse");
    Layout lay;
    int rc = check_view(view, &lay, "vecchia_inverse");
    if (rc) return rc;
    if (!xi || !v) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_inverse: xi and v must be set");
    if (xi == v) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_inverse: xi and v must not alias");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = timed("inverse_dense", s, [&] {
        return launch_inverse_dense(view->precision, ws<double>(view, lay.l0), view->n0, v, xi, s);
    });
    if (e != hipSuccess) return hip_fail(e, "vecchia_inverse (dense block)");
    e = timed("inverse_sparse", s, [&] {
        return launch_inverse_sparse(view->precision, view->kp, view->nbr, ws<char>(view, lay.b),
                                     ws<char>(view, lay.sigma), v, xi, view->n0, lay.ns, s);
    });
    if (e != hipSuccess) return hip_fail(e, "vecchia_inverse (sparse points)");
    return VECCHIA_OK;
}

extern "C" int vecchia_logdet(const vecchia_view* view, double* out, void* stream) {
    vecchia_clear_error();
    TraceRange trace_range("vecchia_logdet");
    Layout lay;
    int rc = check_view(view, &lay, "vecchia_logdet");
    if (rc) return rc;
    if (!out) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_logdet: out is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = timed("logdet", s, [&] {
        return launch_logdet(ws<double>(view, lay.ldpart), ws<long long>(view, lay.ldfix), lay.ns > 0 ? lay.nparts : 0,
                             ws<double>(view, lay.ld0), ws<double>(view, lay.ldstage), out, s);
    });
    if (e != hipSuccess) return hip_fail(e, "vecchia_logdet");
    return VECCHIA_OK;
}

extern "C" int vecchia_status(const vecchia_view* view, void* stream, int64_t* first_bad_slot) {
    vecchia_clear_error();
    Layout lay;
    int rc = check_view(view, &lay, "vecchia_status");
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint64_t st[2] = {0, 0};
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "vecchia_status (stream)");
    e = hipMemcpy(st, ws<uint64_t>(view, lay.status), sizeof(st), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "vecchia_status (copy)");
    if (first_bad_slot) *first_bad_slot = st[0] == kStatusNone ? -1 : (int64_t)st[0];
    if (st[0] != kStatusNone)
        return vecchia_set_error(VECCHIA_ENOTPD, "covariance not positive definite at storage position %llu (%llu points)",
                                 (unsigned long long)st[0], (unsigned long long)st[1]);
    return VECCHIA_OK;
}

extern "C" int vecchia_factor_counts(const vecchia_view* view, void* stream, int64_t* not_pd, int64_t* recomputed) {
    vecchia_clear_error();
    Layout lay;
    int rc = check_view(view, &lay, "vecchia_factor_counts");
    if (rc) return rc;
    uint64_t st[4] = {0, 0, 0, 0};
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e == hipSuccess) e = hipMemcpy(st, ws<uint64_t>(view, lay.status), sizeof(st), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "vecchia_factor_counts");
    if (not_pd) *not_pd = (int64_t)st[1];
    if (recomputed) *recomputed = (int64_t)st[2];
    return VECCHIA_OK;
}

extern "C" int vecchia_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return VECCHIA_OK;
}

static int drain_pending() {
    std::vector<Pending> todo;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        todo.swap(g_pending);
    }
    for (const Pending& p : todo) {
        hipError_t e = hipEventSynchronize(p.b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e != hipSuccess) return hip_fail(e, "vecchia_profile_read");
        std::lock_guard<std::mutex> lk(g_prof_mu);
        KernelTotal* t = nullptr;
        for (auto& k : g_totals)
            if (k.name == p.name) t = &k;
        if (!t) {
            g_totals.push_back(KernelTotal{p.name, 0.0, 0});
            t = &g_totals.back();
        }
        t->ms += ms;
        t->launches += 1;
        g_event_pool.push_back(p.a);
        g_event_pool.push_back(p.b);
    }
    return VECCHIA_OK;
}

extern "C" int vecchia_profile_read(char* names, size_t cap, double* total_ms, int64_t* launches, int32_t max_kernels,
                                    int32_t* n_kernels) {
    int rc = drain_pending();
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    std::string joined;
    int n = 0;
    for (const auto& t : g_totals) {
        if (n >= max_kernels) break;
        if (total_ms) total_ms[n] = t.ms;
        if (launches) launches[n] = t.launches;
        joined += t.name;
        joined += '\n';
        ++n;
    }
    if (n_kernels) *n_kernels = n;
    if (names && cap > 0) {
        const size_t m = std::min(cap - 1, joined.size());
        std::memcpy(names, joined.data(), m);
        names[m] = 0;
    }
    return VECCHIA_OK;
}

extern "C" int vecchia_profile_reset(void) {
    int rc = drain_pending();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_totals.clear();
    return rc;
}

extern "C" int vecchia_backward_scratch_bytes(const vecchia_view* view, size_t* bytes) {
    vecchia_clear_error();
    Layout lay;
    int rc = check_view(view, &lay, "vecchia_backward_scratch_bytes");
    if (rc) return rc;
    if (!bytes) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_backward_scratch_bytes: bytes is NULL");
    *bytes = backward_scratch(view->n, view->kp, view->n0, view->precision).total;
    return VECCHIA_OK;
}

extern "C" int vecchia_backward(const vecchia_view* view, const vecchia_kernel* kern, const void* xi, const void* v,
                                const void* v_bar, const void* xi_bar_in, double logdet_bar, void* xi_bar,
                                void* v_bar_out, double* theta_bar, void* scratch, size_t scratch_bytes,
                                void* stream) {
    vecchia_clear_error();
    TraceRange trace_range("vecchia_backward");
    Layout lay;
    int rc = check_view(view, &lay, "vecchia_backward");
    if (rc) return rc;
    if ((rc = check_kernel(kern))) return rc;
    if ((rc = check_closed_form(kern, "vecchia_backward"))) return rc;
    if (!view->child_ptr || !view->child)
        return vecchia_set_error(VECCHIA_EINVAL, "vecchia_backward: the view needs child_ptr and child");
    if (!xi || !v || !theta_bar || !scratch)
        return vecchia_set_error(VECCHIA_EINVAL, "vecchia_backward: xi, v, theta_bar and scratch must be set");
    if (v_bar && !xi_bar) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_backward: v_bar given without xi_bar");
    if (xi_bar_in && !v_bar_out)
        return vecchia_set_error(VECCHIA_EINVAL, "vecchia_backward: xi_bar_in given without v_bar_out");
    if (!std::isfinite(logdet_bar)) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_backward: logdet_bar not finite");
    const BackwardScratch sc = backward_scratch(view->n, view->kp, view->n0, view->precision);
    if (scratch_bytes < sc.total)
        return vecchia_set_error(VECCHIA_ENOMEM, "vecchia_backward: scratch has %zu bytes, needs %zu", scratch_bytes,
                                 sc.total);
    if (reinterpret_cast<uintptr_t>(scratch) & 255)
        return vecchia_set_error(VECCHIA_EINVAL, "vecchia_backward: scratch must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* sb = static_cast<char*>(scratch);
    BackwardLaunch p;
    p.precision = view->precision;
    p.kp = view->kp;
    p.n0 = view->n0;
    p.n_levels = view->n_levels;
    p.n = view->n;
    p.ns = lay.ns;
    p.level_ptr = view->level_ptr;
    p.x = view->x;
    p.xi = xi;
    p.v = v;
    p.vbar = v_bar;
    p.xibar_in = xi_bar_in;
    p.b = ws<char>(view, lay.b);
    p.sigma = ws<char>(view, lay.sigma);
    p.nbr = view->nbr;
    p.child_ptr = view->child_ptr;
    p.child = view->child;
    p.l0 = ws<double>(view, lay.l0);
    p.w = sb + sc.w;
    p.xibar = xi_bar;
    p.vbar_out = v_bar_out;
    p.t0 = reinterpret_cast<double*>(sb + sc.t0);
    p.theta_part = reinterpret_cast<double*>(sb + sc.part);
    p.theta_dense = reinterpret_cast<double*>(sb + sc.dense);
    p.theta_out = theta_bar;
    p.ldbar = logdet_bar;
    p.kern = *kern;
    hipError_t e = timed("backward", s, [&] { return launch_backward(p, s); });
    if (e != hipSuccess) return hip_fail(e, "vecchia_backward");
    return VECCHIA_OK;
}

extern "C" int vecchia_backward_x_scratch_bytes(const vecchia_view* view, size_t* bytes) {
    vecchia_clear_error();
    Layout lay;
    int rc = check_view(view, &lay, "vecchia_backward_x_scratch_bytes");
    if (rc) return rc;
    if (!bytes) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_backward_x_scratch_bytes: bytes is NULL");
    *bytes = backward_x_scratch(view->n, view->kp, view->n0, view->precision).total;
    return VECCHIA_OK;
}

extern "C" int vecchia_backward_x(const vecchia_view* view, const vecchia_kernel* kern, const void* xi, const void* v,
                                  const void* v_bar, const void* xi_bar_in, double logdet_bar, double* x_bar,
                                  void* scratch, size_t scratch_bytes, void* stream) {
    vecchia_clear_error();
    TraceRange trace_range("vecchia_backward_x");
    Layout lay;
    int rc = check_view(view, &lay, "vecchia_backward_x");
    if (rc) return rc;
    if ((rc = check_kernel(kern))) return rc;
    if ((rc = check_closed_form(kern, "vecchia_backward_x"))) return rc;
    if (!view->child_ptr || !view->child)
        return vecchia_set_error(VECCHIA_EINVAL, "vecchia_backward_x: the view needs child_ptr and child");
    if (!xi || !v || !x_bar || !scratch)
        return vecchia_set_error(VECCHIA_EINVAL, "vecchia_backward_x: xi, v, x_bar and scratch must be set");
    if (!std::isfinite(logdet_bar)) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_backward_x: logdet_bar not finite");
    const BackwardScratch sc = backward_scratch(view->n, view->kp, view->n0, view->precision);
    const BackwardXScratch sx = backward_x_scratch(view->n, view->kp, view->n0, view->precision);
    if (scratch_bytes < sx.total)
        return vecchia_set_error(VECCHIA_ENOMEM, "vecchia_backward_x: scratch has %zu bytes, needs %zu", scratch_bytes,
                                 sx.total);
    if (reinterpret_cast<uintptr_t>(scratch) & 255)
        return vecchia_set_error(VECCHIA_EINVAL, "vecchia_backward_x: scratch must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* sb = static_cast<char*>(scratch);
    BackwardLaunch p;
    p.precision = view->precision;
    p.kp = view->kp;
    p.n0 = view->n0;
    p.n_levels = view->n_levels;
    p.n = view->n;
    p.ns = lay.ns;
    p.level_ptr = view->level_ptr;
    p.x = view->x;
    p.xi = xi;
    p.v = v;
    p.vbar = v_bar;
    p.xibar_in = xi_bar_in;
    p.b = ws<char>(view, lay.b);
    p.sigma = ws<char>(view, lay.sigma);
    p.nbr = view->nbr;
    p.child_ptr = view->child_ptr;
    p.child = view->child;
    p.l0 = ws<double>(view, lay.l0);
    p.w = sb + sc.w;
    p.xibar = sb + sx.xibar;
    p.vbar_out = sb + sx.vbar;
    p.t0 = reinterpret_cast<double*>(sb + sc.t0);
    p.theta_part = reinterpret_cast<double*>(sb + sc.part);
    p.theta_dense = reinterpret_cast<double*>(sb + sc.dense);
    p.theta_out = nullptr;
    p.ldbar = logdet_bar;
    p.kern = *kern;
    hipError_t e = timed("backward_x", s, [&] {
        return launch_backward_x(p, x_bar, reinterpret_cast<double*>(sb + sx.contrib), s);
    });
    if (e != hipSuccess) return hip_fail(e, "vecchia_backward_x");
    return VECCHIA_OK;
}

extern "C" int vecchia_fused_workspace_bytes(int64_t n, int32_t k, int32_t n0, int32_t precision, size_t* bytes) {
    if (!bytes) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_fused_workspace_bytes: bytes is NULL");
    if (k < 1) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_fused_workspace_bytes: need k >= 1");
    if (k > VECCHIA_KMAX)
        return vecchia_set_error(VECCHIA_EUNSUPPORTED, "vecchia_fused_workspace_bytes: k=%d exceeds the compiled maximum %d",
                                 k, VECCHIA_KMAX);
    if (n < 1 || n0 < 1 || n0 > n) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_fused_workspace_bytes: need 1 <= n0 <= N");
    if (precision != VECCHIA_FP64 && precision != VECCHIA_FP32)
        return vecchia_set_error(VECCHIA_EINVAL, "vecchia_fused_workspace_bytes: bad precision");
    *bytes = fused_layout(n, n0).total;
    return VECCHIA_OK;
}

extern "C" int vecchia_forward_fused(const vecchia_view* view, const vecchia_kernel* kern, const void* xi, void* v,
                                     double* logdet, void* stream) {
    vecchia_clear_error();
    TraceRange trace_range("vecchia_forward_fused");
    FusedLayout lay;
    int rc = check_fused_view(view, &lay, "vecchia_forward_fused");
    if (rc) return rc;
    if ((rc = check_kernel(kern))) return rc;
    if ((rc = check_closed_form(kern, "vecchia_forward_fused"))) return rc;
    if (!xi || !v) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_forward_fused: xi and v must be set");
    if (xi == v) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_forward_fused: xi and v must not alias");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(view->workspace);
    double* l0 = reinterpret_cast<double*>(w + lay.l0);
    double* ld0 = reinterpret_cast<double*>(w + lay.ld0);
    uint64_t* status = reinterpret_cast<uint64_t*>(w + lay.status);
    long long* ldfix = reinterpret_cast<long long*>(w + lay.ldfix);
    hipError_t e = timed("fused_zero", s, [&] { return launch_zero_u64(w + lay.ldpart, 2 * lay.ntiles, s); });
    if (e != hipSuccess) return hip_fail(e, "vecchia_forward_fused (clear)");
    e = timed("factor_dense", s, [&] {
        return launch_factor_dense(view->precision, kern->kind, view->x, view->n0, *kern, l0, ld0, status, s);
    });
    if (e != hipSuccess) return hip_fail(e, "vecchia_forward_fused (dense block)");
    e = timed("forward_dense", s, [&] { return launch_forward_dense(view->precision, l0, view->n0, xi, v, s); });
    if (e != hipSuccess) return hip_fail(e, "vecchia_forward_fused (dense forward)");
    FusedLaunch f;
    f.precision = view->precision;
    f.kp = view->kp;
    f.kind = kern->kind;
    f.n0 = view->n0;
    f.x = view->x;
    f.nbr = view->nbr;
    f.xi = xi;
    f.v = v;
    f.ldfix = ldfix;
    f.status = status;
    f.diag = kern->sigma * kern->sigma + kern->nugget;
    f.kern = *kern;
    const int32_t* lp = view->level_ptr;
    for (int l = 1; l <= view->n_levels; ++l) {
        f.s_begin = lp[l] - view->n0;
        f.s_end = lp[l + 1] - view->n0;
        if (f.s_end <= f.s_begin) continue;
        e = timed("forward_fused", s, [&] {
            switch (view->kp) {
                case 8: return launch_forward_fused_k8(f, s);
                case 16: return launch_forward_fused_k16(f, s);
                case 32: return launch_forward_fused_k32(f, s);
                case 64: return launch_forward_fused_k64(f, s);
                default: return hipErrorInvalidValue;
            }
        });
        if (e != hipSuccess) return hip_fail(e, "vecchia_forward_fused (batch)");
    }
    if (logdet) {
        e = timed("logdet", s, [&] {
            return launch_logdet(reinterpret_cast<double*>(w + lay.ldpart), ldfix, lay.ns > 0 ? lay.ntiles : 0, ld0,
                                 reinterpret_cast<double*>(w + lay.ldstage), logdet, s);
        });
        if (e != hipSuccess) return hip_fail(e, "vecchia_forward_fused (logdet)");
    }
    return VECCHIA_OK;
}

extern "C" int vecchia_fused_status(const vecchia_view* view, void* stream, int64_t* first_bad_slot) {
    vecchia_clear_error();
    FusedLayout lay;
    int rc = check_fused_view(view, &lay, "vecchia_fused_status");
    if (rc) return rc;
    uint64_t st[2] = {0, 0};
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e == hipSuccess)
        e = hipMemcpy(st, static_cast<char*>(view->workspace) + lay.status, sizeof(st), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "vecchia_fused_status");
    if (first_bad_slot) *first_bad_slot = st[0] == kStatusNone ? -1 : (int64_t)st[0];
    if (st[0] != kStatusNone)
        return vecchia_set_error(VECCHIA_ENOTPD, "covariance not positive definite at storage position %llu (%llu points)",
                                 (unsigned long long)st[0], (unsigned long long)st[1]);
    return VECCHIA_OK;
}

extern "C" int vecchia_jvp_scratch_bytes(const vecchia_view* view, size_t* bytes) {
    vecchia_clear_error();
    Layout lay;
    int rc = check_view(view, &lay, "vecchia_jvp_scratch_bytes");
    if (rc) return rc;
    if (!bytes) return vecchia_set_error(VECCHIA_EINVAL, "vecchia_jvp_scratch_bytes: bytes is NULL");
    *bytes = tangent_scratch(view->n, view->kp, view->n0, view->precision).total;
    return VECCHIA_OK;
}

extern "C" int vecchia_forward_jvp(const vecchia_view* view, const vecchia_kernel* kern, const void* xi, const void* v,
                                   const void* xi_dot, double sigma_dot, double ell_dot, void* v_dot,
                                   double* logdet_dot, void* scratch, size_t scratch_bytes, void* stream) {
    vecchia_clear_error();
    TraceRange trace_range("vecchia_forward_jvp");
    Layout lay;
    int rc = check_view(view, &lay, "vecchia_forward_jvp");
    if (rc) return rc;
    if ((rc = check_kernel(kern))) return rc;
    if ((rc = check_closed_form(kern, "vecchia_forward_jvp"))) return rc;
    if (!xi || !v || !v_dot || !scratch)
        return vecchia_set_error(VECCHIA_EINVAL, "vecchia_forward_jvp: xi, v, v_dot and scratch must be set");
    if (v_dot == v || v_dot == xi || (xi_dot && v_dot == xi_dot))
        return vecchia_set_error(VECCHIA_EINVAL, "vecchia_forward_jvp: v_dot must not alias an input");
    if (!std::isfinite(sigma_dot) || !std::isfinite(ell_dot))
        return vecchia_set_error(VECCHIA_EINVAL, "vecchia_forward_jvp: the direction must be finite");
    const TangentScratch sc = tangent_scratch(view->n, view->kp, view->n0, view->precision);
    if (scratch_bytes < sc.total)
        return vecchia_set_error(VECCHIA_ENOMEM, "vecchia_forward_jvp: scratch has %zu bytes, needs %zu", scratch_bytes,
                                 sc.total);
    if (reinterpret_cast<uintptr_t>(scratch) & 255)
        return vecchia_set_error(VECCHIA_EINVAL, "vecchia_forward_jvp: scratch must be 256-byte aligned");
    char* sb = static_cast<char*>(scratch);
    TangentLaunch t;
    t.precision = view->precision;
    t.kp = view->kp;
    t.kind = kern->kind;
    t.n0 = view->n0;
    t.n_levels = view->n_levels;
    t.n = view->n;
    t.ns = lay.ns;
    t.level_ptr = view->level_ptr;
    t.x = view->x;
    t.b = ws<char>(view, lay.b);
    t.sigma = ws<char>(view, lay.sigma);
    t.xi = xi;
    t.v = v;
    t.xi_dot = xi_dot;
    t.nbr = view->nbr;
    t.l0 = ws<double>(view, lay.l0);
    t.bdot = sb + sc.bdot;
    t.sigdot = sb + sc.sigdot;
    t.v_dot = v_dot;
    t.part = reinterpret_cast<double*>(sb + sc.part);
    t.fixzero = reinterpret_cast<double*>(sb + sc.fixzero);
    t.ld0dot = reinterpret_cast<double*>(sb + sc.ld0dot);
    t.stage = reinterpret_cast<double*>(sb + sc.stage);
    t.logdet_dot = logdet_dot;
    t.diag = kern->sigma * kern->sigma + kern->nugget;
    t.sigma_amp = kern->sigma;
    t.sdot = sigma_dot;
    t.ldot = ell_dot;
    t.kern = *kern;
    hipError_t e = timed("forward_jvp", static_cast<hipStream_t>(stream),
                         [&] { return launch_forward_tangent(t, static_cast<hipStream_t>(stream)); });
    if (e != hipSuccess) return hip_fail(e, "vecchia_forward_jvp");
    return VECCHIA_OK;
}
