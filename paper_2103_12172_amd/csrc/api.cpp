// C-ABI entry points (include/mdp.h): context, projector cache, the three
// algorithm steps of paper Sec. 3.5 and the AP solve itself.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "ap_solver.h"
#include "ls_solver.h"

using namespace mdp;

namespace {

// Device buffers of released projectors, kept for the next builds so that a
// rebuild allocates nothing (hipMalloc/hipFree stall the host and the device).
// A kept buffer is handed out only to a later call, whose work is ordered after
// every earlier call's work (same stream, or the wait in begin_call).
struct BufPool {
    int device = 0;
    std::mutex mu;
    std::vector<DevBuf> bufs;
    size_t held = 0;
    static constexpr size_t cap = (size_t)8 << 30;
    // a kept buffer of at least `bytes` (at most twice that), else a new one
    DevBuf take(size_t bytes) {
        {
            std::lock_guard<std::mutex> g(mu);
            int best = -1;
            for (int i = 0; i < (int)bufs.size(); ++i)
                if (bufs[i].bytes >= bytes && bufs[i].bytes <= 2 * std::max<size_t>(bytes, 4096) &&
                    (best < 0 || bufs[i].bytes < bufs[best].bytes))
                    best = i;
            if (best >= 0) {
                DevBuf b = std::move(bufs[best]);
                bufs.erase(bufs.begin() + best);
                held -= b.bytes;
                return b;
            }
        }
        return DevBuf(bytes);
    }
    void give(DevBuf&& b) {
        if (!b.p) return;
        std::lock_guard<std::mutex> g(mu);
        if (held + b.bytes > cap) {
            (void)hipDeviceSynchronize();
            b.release();
            return;
        }
        held += b.bytes;
        bufs.push_back(std::move(b));
    }
    ~BufPool() {
        (void)hipSetDevice(device);
        (void)hipDeviceSynchronize();
        bufs.clear();
    }
};

}  // namespace

// The grid sets and gamma of one rectangle size and n with their device tables, shared
// by every projector of that geometry whatever its k (the tables are uploaded, and the
// node map written, by the first build that needs them).
struct GeomShared {
    Geometry g;
    DevBuf meta;   // gamma nodes: gm, gq, side (int), then rho, t, side length (double)
    DevBuf gidx;   // (n+1)^2 node -> gamma index, -1 off gamma
    const int *gm = nullptr, *gq = nullptr, *gside = nullptr;
    const double *grho = nullptr, *gt = nullptr, *gslen = nullptr;
    bool on_device = false;
    explicit GeomShared(Geometry&& geo) : g(std::move(geo)) {}
};

struct mdp_projector {
    std::atomic<int> refs{1};
    int device = 0;
    unsigned long long serial = 0;   // unique per build in its context (the interface factor's key)
    std::shared_ptr<GeomShared> geo;
    const Geometry& g;
    double k = 0.0;
    int m_star = 0, precision = 0;
    DevBuf Q;      // n_gamma x 8M* complex, column-major
    DevBuf E;      // n_gamma x 8M* real
    const int* gidx = nullptr;   // the geometry's node map and gamma tables (device)
    const int *gm = nullptr, *gq = nullptr, *gside = nullptr;
    const double *grho = nullptr, *gt = nullptr, *gslen = nullptr;
    std::shared_ptr<BufPool> pool;   // where the buffers go on release
    explicit mdp_projector(std::shared_ptr<GeomShared> s)
        : geo(std::move(s)), g(geo->g), gidx(geo->gidx.as<int>()), gm(geo->gm), gq(geo->gq), gside(geo->gside),
          grho(geo->grho), gt(geo->gt), gslen(geo->gslen) {}
};

namespace {

using PlanKey = std::tuple<int, double, double>;
using ProjKey = std::tuple<double, double, int, double, int, int>;
using GeomKey = std::tuple<double, double, int>;

}  // namespace

namespace {

// Offsets of the interface solve's tables in its upload.
struct IfaceOffs {
    size_t qsrc, qld, roff, cmap, coef, kcol, kval, koff, esrc, ecoef, eknown, sf, sjet, sgoff, sfoff;
};

// The host side of the last interface solve without sources (packed description, elimination tree and the
// device tables of both), kept for the next call with the same layout, side kinds and coefficients and M*.
// The tables hold workspace addresses (the packed matrix, the factor arena): they are valid while those
// buffers are the ones recorded here.
struct IfaceCache {
    bool valid = false;
    std::vector<double> key;
    PackedHost ph;
    HostBlob blob;
    PackedTables tabs{};
    IfaceOffs o{};
    size_t dyn_end = 0;   // the per-call part (projector addresses, known coefficients) is blob[0, dyn_end)
    DevBuf image;         // the device copy of blob
    const void* ap = nullptr;
    const void* mf = nullptr;
};

}  // namespace

struct mdp_ctx {
    int device = 0;
    std::string err;
    std::map<PlanKey, std::unique_ptr<APPlan>> plans;
    std::map<ProjKey, mdp_projector*> cache;
    std::map<GeomKey, std::shared_ptr<GeomShared>> geoms;   // per rectangle size and n (position-free)
    std::shared_ptr<BufPool> pool = std::make_shared<BufPool>();
    Workspace ws;
    size_t ws_cap = (size_t)24 << 30;
    int projector_path = MDP_PATH_AUTO;
    int sweep_cols = 0;        // mode columns per lane of the fused sweep (0: chosen per batch)
    int last_sweep_cols = 0;   // what the last fused build used
    int interface_path = MDP_IFACE_AUTO;
    unsigned long long next_serial = 1;
    // key of the interface system whose Gram factor the workspaces hold (projector builds, side
    // kinds and coefficients, M*, route); empty when none is valid
    std::vector<double> iface_key;
    IfaceCache icache;
    void* scratch = nullptr;     // this device's static scratch array (mdp_ap_solve_noalloc)
    hipEvent_t last = nullptr;   // end of the previous call's work (workspaces are shared)
    hipStream_t last_stream = nullptr;
    bool have_last = false;
};

namespace {

std::string g_create_error;

int fail(mdp_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    else g_create_error = msg;
    return code;
}

template <class F>
int guarded(mdp_ctx* ctx, F&& f) {
    try {
        if (ctx) {
            hipError_t e = hipSetDevice(ctx->device);
            if (e != hipSuccess) return fail(ctx, MDP_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
        }
        return f();
    } catch (const Error& e) {
        return fail(ctx, e.code, e.what());
    } catch (const std::bad_alloc&) {
        return fail(ctx, MDP_ERR_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(ctx, MDP_ERR_HIP, e.what());
    }
}

// Order this call after the previous one (it may have used another stream).
void begin_call(mdp_ctx* ctx, hipStream_t st) {
    if (ctx->have_last && ctx->last_stream != st) MDP_HIP(hipStreamWaitEvent(st, ctx->last, 0));
}

// The device work of one call, from its first launch to its return: opening it orders the
// call after the previous one; leaving it (normal return or an error thrown after some work
// was queued) records the end of the queued work, so that the next call, on any stream,
// waits for it before reusing the shared workspaces.  If the record itself fails the
// device is drained instead.
struct CallScope {
    mdp_ctx* ctx = nullptr;
    hipStream_t st = nullptr;
    CallScope() = default;
    CallScope(mdp_ctx* c, hipStream_t s) { open(c, s); }
    CallScope(const CallScope&) = delete;
    CallScope& operator=(const CallScope&) = delete;
    void open(mdp_ctx* c, hipStream_t s) {
        if (ctx) return;
        begin_call(c, s);
        ctx = c;
        st = s;
    }
    bool is_open() const { return ctx != nullptr; }
    ~CallScope() {
        if (!ctx) return;
        if (hipEventRecord(ctx->last, st) == hipSuccess) {
            ctx->last_stream = st;
            ctx->have_last = true;
        } else {
            (void)hipDeviceSynchronize();
            ctx->have_last = false;
        }
    }
};

APPlan& get_plan(mdp_ctx* ctx, int n, double h, double k) {
    PlanKey key{n, h, k};
    auto it = ctx->plans.find(key);
    if (it != ctx->plans.end()) return *it->second;
    auto p = std::make_unique<APPlan>(n, h, k);
    APPlan& ref = *p;
    ctx->plans.emplace(key, std::move(p));
    return ref;
}

void check_precision(int p) {
    if (p != MDP_C128 && p != MDP_C64 && p != MDP_C64_REFINED) throw Error(MDP_ERR_ARG, "unknown precision");
}

template <class T>
void upload(DevBuf& d, const std::vector<T>& v) {
    d.alloc(std::max<size_t>(v.size(), 1) * sizeof(T));
    if (!v.empty()) MDP_HIP(hipMemcpy(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

// Grow a workspace buffer (after the device has drained, since earlier work
// may still use the old allocation; contents are not kept).
void ensure(DevBuf& d, size_t bytes) {
    if (bytes > d.bytes) {
        MDP_HIP(hipDeviceSynchronize());
        d.reserve(bytes);
    }
}

// Copy a host vector into a grow-only workspace buffer on the stream.  The
// host vector must stay alive until the stream has consumed it.
template <class T>
void upload_ws(DevBuf& d, const std::vector<T>& v, hipStream_t st) {
    ensure(d, std::max<size_t>(v.size(), 1) * sizeof(T));
    if (!v.empty()) MDP_HIP(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

// Grow the batch workspaces before a solve so that no buffer is freed while
// earlier work may still use it.
void prepare_ws(mdp_ctx* ctx, const APPlan& P, int precision, int R) {
    const size_t elem = (precision == MDP_C128) ? 8 : 4;
    const size_t need = (size_t)R * 2 * (P.n + 1) * P.f.W * elem;
    const size_t needc = (precision == MDP_C64_REFINED) ? (size_t)R * 2 * (P.n + 1) * P.f.W * 4 : 0;
    if (need > ctx->ws.a.bytes || need > ctx->ws.b.bytes || needc > ctx->ws.c.bytes) {
        MDP_HIP(hipDeviceSynchronize());
        ctx->ws.a.reserve(need);
        ctx->ws.b.reserve(need);
        if (needc) ctx->ws.c.reserve(needc);
    }
}


// Rows m_lo-1..m_hi+1 of the M+ box: they hold gamma and N+, and a right-hand
// side supported on M+ vanishes outside them, so the AP solve may stop there
// (twisted pivot at the last row); the full grid if that pivot is too small.
Band box_band(const APPlan& plan, const Geometry& G) {
    const int t = G.m_hi + 1;
    if (G.m_lo < 1 || t > G.n || !(plan.twist_ratio[t] > 1e-13)) return Band{0, G.n + 1};
    return Band{G.m_lo - 1, G.m_hi - G.m_lo + 3};
}

// A projector whose Q the fused route computes.
struct FusedItem {
    const APPlan* plan;
    mdp_projector* P;
};

// Mode columns per lane of the fused sweep when none is set: two (independent recurrences
// side by side, half the cross-lane reduction per column; 150 VGPRs in FP64, three
// wavefronts per SIMD) when the batch still gives about two wavefronts per SIMD of the
// chip at two columns per lane, else one (small batches: more wavefronts hide more
// latency); or what the autotuner measured fastest.
int sweep_lanes_cols(long waves_one_col) { return waves_one_col >= 2L * 4096 ? 2 : 1; }

// Q of every item by the support-in / gamma-out route, T the arithmetic of the build
// (double for complex128, float for complex64), the columns of all items through each
// stage together.  Per batch of columns (as many as the workspace holds): the ring RHS
// and the folded special rows, their sine GEMM (one launch per n), the fused sweep with
// the gamma-row reductions, the inverse GEMM of the four full gamma rows (one launch
// per n) and the gather into Q (FP64).
template <class T>
void build_q_fused_t(mdp_ctx* ctx, std::vector<FusedItem> items, hipStream_t st) {
    if (items.empty()) return;
    constexpr bool f64 = sizeof(T) == 8;
    std::stable_sort(items.begin(), items.end(),
                     [](const FusedItem& a, const FusedItem& b) { return a.plan->n < b.plan->n; });
    struct Per { size_t a, b; int ncol; };
    std::vector<Per> per(items.size());
    for (size_t i = 0; i < items.size(); ++i) {
        const Geometry& G = items[i].P->g;
        const Fold& f = items[i].plan->f;
        const int nseg = fused_segments(G.m_lo, G.m_hi), rows_pad = nseg * FUSED_K, nb = f.W / 64;
        per[i].a = (size_t)nseg * 2 * f.W + (size_t)nb * rows_pad * 4;      // ckpt + thin
        per[i].b = (size_t)(G.n + 1) * 4 + (size_t)(4 + 4 + 8 + 8) * f.W;    // gc, spec, spec_hat, xs, us
        per[i].ncol = 8 * items[i].P->m_star;
    }
    const size_t cap = ctx->ws_cap / sizeof(T);
    Profiler& pr = ctx->ws.prof;
    struct JobHost { size_t item; int col0, R; };
    size_t it = 0;
    int next_col = 0;
    while (it < items.size()) {
        // the next batch: whole or partial items in order, within the workspace and the grid limit
        std::vector<JobHost> jh;
        size_t sa = 0, sb = 0;
        int total = 0;
        while (it < items.size()) {
            const Per& q = per[it];
            const size_t used = sa + sb, each = q.a + q.b;
            const size_t room = used < cap ? (cap - used) / each : 0;
            const int R = (int)std::min<size_t>({room, (size_t)(q.ncol - next_col)});
            if (R <= 0) break;
            jh.push_back({it, next_col, R});
            sa += (size_t)R * q.a;
            sb += (size_t)R * q.b;
            total += R;
            next_col += R;
            if (next_col == q.ncol) { ++it; next_col = 0; }
        }
        if (jh.empty()) throw Error(MDP_ERR_OOM, "workspace too small for one projector column");
        if (sa * sizeof(T) > ctx->ws.a.bytes || sb * sizeof(T) > ctx->ws.b.bytes) {
            MDP_HIP(hipDeviceSynchronize());
            ctx->ws.a.reserve(std::max<size_t>(sa, 1) * sizeof(T));
            ctx->ws.b.reserve(std::max<size_t>(sb, 1) * sizeof(T));
        }
        // regions: ws.b = gc | spec | spec_hat | xs | us, ws.a = ckpt | thin, each in job order
        size_t n_gc = 0, n_sp = 0, n_x = 0, n_ck = 0;
        for (const JobHost& j : jh) {
            const Geometry& G = items[j.item].P->g;
            const Fold& f = items[j.item].plan->f;
            n_gc += (size_t)j.R * (G.n + 1) * 4;
            n_sp += (size_t)j.R * 4 * f.W;
            n_x += (size_t)j.R * 8 * f.W;
            n_ck += (size_t)j.R * fused_segments(G.m_lo, G.m_hi) * 2 * f.W;
        }
        T* B = ctx->ws.b.as<T>();
        T* A = ctx->ws.a.as<T>();
        T *gc = B, *spec = gc + n_gc, *spec_hat = spec + n_sp, *xs = spec_hat + n_sp, *us = xs + n_x;
        T *ckpt = A, *thin = ckpt + n_ck;
        auto dp = [](T* p) { return reinterpret_cast<double*>(p); };
        auto cdp = [](const void* p) { return reinterpret_cast<const double*>(p); };
        std::vector<FusedJob> jobs(jh.size());
        int b0 = 0, max_n = 0, max_w = 0, max_ng = 0;
        long groups[3] = {0, 0, 0};
        long waves_one_col = 0;
        double fold_bytes = 0.0, sweep_flops = 0.0, sweep_bytes = 0.0, gather_bytes = 0.0;
        for (size_t q = 0; q < jh.size(); ++q) {
            const JobHost& j = jh[q];
            const FusedItem& itm = items[j.item];
            const APPlan& plan = *itm.plan;
            const Geometry& G = itm.P->g;
            const Fold& f = plan.f;
            const int n = G.n, ng = G.n_gamma, R = j.R;
            const int nseg = fused_segments(G.m_lo, G.m_hi);
            FusedJob& J = jobs[q];
            J.src = SrcDesc{};
            J.src.kind = Src::STENCIL_E;
            J.src.E = itm.P->E.as<double>();
            J.src.ldE = ng;
            J.src.col0 = j.col0;
            J.src.gidx = itm.P->gidx;
            J.src.m_lo = G.m_lo; J.src.m_hi = G.m_hi; J.src.q_lo = G.q_lo; J.src.q_hi = G.q_hi;
            J.sc = plan.sc;
            J.f = f;
            J.nseg = nseg;
            J.rows_pad = nseg * FUSED_K;
            J.ng = ng;
            J.ldq = ng;
            J.b0 = b0;
            J.R = R;
            for (int lg = 0; lg < 3; ++lg) {
                J.g0[lg] = (int)groups[lg];
                groups[lg] += (R + (1 << lg) - 1) >> lg;
            }
            J.Sf = cdp(f64 ? plan.Sf64.p : plan.Sf32.p);
            J.Si = cdp(f64 ? plan.Si64.p : plan.Si32.p);
            J.rf = cdp(f64 ? plan.rf64.p : plan.rf32.p);
            J.tf = cdp(f64 ? plan.tf64.p : plan.tf32.p);
            J.colc = cdp(f64 ? plan.colc64.p : plan.colc32.p);
            J.gc = dp(gc); gc += (size_t)R * (n + 1) * 4;
            J.spec = dp(spec); spec += (size_t)R * 4 * f.W;
            J.spec_hat = dp(spec_hat); spec_hat += (size_t)R * 4 * f.W;
            J.xs = dp(xs); xs += (size_t)R * 8 * f.W;
            J.us = dp(us); us += (size_t)R * 8 * f.W;
            J.ckpt = dp(ckpt); ckpt += (size_t)R * nseg * 2 * f.W;
            J.thin = dp(thin); thin += (size_t)R * (f.W / 64) * J.rows_pad * 4;
            J.Q = itm.P->Q.as<double>();
            J.gm = itm.P->gm;
            J.gq = itm.P->gq;
            b0 += R;
            max_n = std::max(max_n, n);
            max_w = std::max(max_w, f.W);
            max_ng = std::max(max_ng, ng);
            waves_one_col += (long)R * (f.W / 64);
            // algorithmic flops per column element of the swept band (rows m_lo-1..m_hi+1): forward
            // elimination 7, back substitution 10, synthesis products and sums 8; ring transform 3 (box rows)
            const int box_rows = G.m_hi - G.m_lo + 3;
            fold_bytes += (double)R * ((n + 1) * 4.0 + 4.0 * (n - 1)) * sizeof(T);
            sweep_flops += (double)R * ((double)box_rows * (n - 1) * 25.0 + (double)(G.m_hi - G.m_lo + 1) * (n - 1) * 3.0);
            sweep_bytes += (double)R * ((G.m_hi - G.m_lo + 1) * 4.0 + 4.0 * (n - 1) + 8.0 * (n - 1) +
                                        (double)box_rows * 4) * sizeof(T);
            gather_bytes += (double)ng * R * 16.0 * 2.0;
        }
        HostBlob blob;
        const size_t o_jobs = blob.put(jobs);
        const FusedJob* dj = reinterpret_cast<const FusedJob*>(ctx->ws.stage.upload(blob, st) + o_jobs);
        const int nj = (int)jobs.size();
        // the sine GEMMs: one per run of jobs with the same n (their rows are consecutive)
        auto gemms = [&](bool forward) {
            for (size_t q0 = 0; q0 < jobs.size();) {
                size_t q1 = q0;
                long rows = 0;
                while (q1 < jobs.size() && jobs[q1].f.n == jobs[q0].f.n) rows += jobs[q1++].R;
                const Fold& f = jobs[q0].f;
                const double row_flops = 2.0 * ((double)f.p * f.p + (double)(f.p - 1) * (f.p - 1));
                const int mult = forward ? 4 : 8;
                pr.run(f64 ? "gemm_sine_f64" : "gemm_sine_f32", st, mult * rows * row_flops,
                       2.0 * mult * rows * (f.n - 1) * sizeof(T), [&] {
                    if (forward)
                        launch_gemm_bd<T>(reinterpret_cast<const T*>(jobs[q0].spec),
                                          reinterpret_cast<const T*>(jobs[q0].Sf),
                                          reinterpret_cast<T*>(jobs[q0].spec_hat), rows * 4, f, st);
                    else
                        launch_gemm_bd<T>(reinterpret_cast<const T*>(jobs[q0].xs),
                                          reinterpret_cast<const T*>(jobs[q0].Si),
                                          reinterpret_cast<T*>(jobs[q0].us), rows * 8, f, st);
                });
                q0 = q1;
            }
        };
        const int L = ctx->sweep_cols > 0 ? ctx->sweep_cols : sweep_lanes_cols(waves_one_col);
        pr.run("fold_ring", st, 0.0, fold_bytes, [&] { launch_fold_ring_jobs<T>(dj, nj, total, max_n, st); });
        gemms(true);
        pr.run(f64 ? "ap_fused_f64" : "ap_fused_f32", st, sweep_flops, sweep_bytes, [&] {
            ctx->last_sweep_cols =
                launch_proj_sweep_jobs<T>(dj, nj, total, groups, max_w, waves_one_col, L, ctx->sweep_cols == 0, st);
        });
        gemms(false);
        pr.run("gather_q", st, 0.0, gather_bytes,
               [&] { launch_gather_q_fused_jobs<T>(dj, nj, total, max_ng, ctx->last_sweep_cols, st); });
    }
}

void build_q_fused(mdp_ctx* ctx, const std::vector<FusedItem>& items, int precision, hipStream_t st) {
    if (precision == MDP_C128) build_q_fused_t<double>(ctx, items, st);
    else build_q_fused_t<float>(ctx, items, st);
}

// Band solves of several plans' entries in one launch per stage: jobs in order of n (their
// A and B regions are assigned here, back to back, so one sine GEMM per n covers a run of
// jobs), job.b0 set by the caller.  Fold (job.src), forward GEMMs, mode solves (or their
// conjugate transposes), inverse GEMMs, unfold into job.out or in place (w - u into `grids`).
void batched_band_solve(mdp_ctx* ctx, std::vector<SolveJob>& jobs, const std::vector<const APPlan*>& plans,
                        double* grids, hipStream_t st) {
    if (jobs.empty()) return;
    Profiler& pr = ctx->ws.prof;
    size_t elems = 0;
    int total = 0, max_w = 0, max_nr = 0, max_n = 0;
    double rhs_bytes = 0.0, tri_pts = 0.0, unfold_bytes = 0.0;
    for (SolveJob& J : jobs) {
        J.A = reinterpret_cast<double*>(elems);   // offsets for now
        elems += (size_t)J.R * 2 * J.bd.nr * J.f.W;
        total += J.R;
        max_w = std::max(max_w, J.f.W);
        max_nr = std::max(max_nr, J.bd.nr);
        max_n = std::max(max_n, J.f.n);
        rhs_bytes += (double)J.R * 2 * J.bd.nr * (J.f.n - 1) * 8.0;
        tri_pts += (double)J.R * J.bd.nr * (J.f.n - 1);
        unfold_bytes += (double)J.R * J.bd.nr * (J.f.n + 1) * 16.0 * 3.0;
    }
    if (elems * sizeof(double) > ctx->ws.a.bytes || elems * sizeof(double) > ctx->ws.b.bytes) {
        MDP_HIP(hipDeviceSynchronize());
        ctx->ws.a.reserve(elems * sizeof(double));
        ctx->ws.b.reserve(elems * sizeof(double));
    }
    for (SolveJob& J : jobs) {
        const size_t o = reinterpret_cast<size_t>(J.A);
        J.A = ctx->ws.a.as<double>() + o;
        J.B = ctx->ws.b.as<double>() + o;
    }
    HostBlob jb;
    const size_t o_jobs = jb.put(jobs);
    ensure(ctx->ws.cw.jobs, jb.size());
    ctx->ws.stage.copy(ctx->ws.cw.jobs.p, jb, st);
    const SolveJob* dj = reinterpret_cast<const SolveJob*>(ctx->ws.cw.jobs.as<char>() + o_jobs);
    const int nj = (int)jobs.size();
    auto gemms = [&](bool forward) {
        for (size_t q0 = 0; q0 < jobs.size();) {
            size_t q1 = q0;
            long rows = 0;
            while (q1 < jobs.size() && jobs[q1].f.n == jobs[q0].f.n) {
                rows += (long)jobs[q1].R * 2 * jobs[q1].bd.nr;
                ++q1;
            }
            const Fold& f = jobs[q0].f;
            const double row_flops = 2.0 * ((double)f.p * f.p + (double)(f.p - 1) * (f.p - 1));
            pr.run("gemm_sine_f64", st, rows * row_flops, 2.0 * rows * (f.n - 1) * 8.0, [&] {
                launch_gemm_bd<double>(jobs[q0].A, (forward ? plans[q0]->Sf64 : plans[q0]->Si64).as<double>(),
                                       jobs[q0].B, rows, f, st);
            });
            q0 = q1;
        }
    };
    pr.run("fold_rhs", st, 0.0, rhs_bytes, [&] { launch_fold_rhs_jobs(dj, nj, total, max_w, max_nr, st); });
    gemms(true);
    const bool adj = jobs[0].adjoint != 0;
    pr.run(adj ? "tridiag_adj" : "tridiag_f64", st, tri_pts * 22.0, tri_pts * 4.0 * 8.0,
           [&] { launch_tridiag_jobs(dj, nj, total, max_w, st); });
    gemms(false);
    pr.run("unfold_grid", st, 0.0, unfold_bytes, [&] { launch_unfold_jobs(dj, nj, total, max_n, max_nr, grids, st); });
}

}  // namespace

extern "C" {

const char* mdp_version(void) { return "mdp-gfx950 0.1"; }

int mdp_create(mdp_ctx** out, int device) {
    if (!out) return fail(nullptr, MDP_ERR_ARG, "ctx pointer is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(nullptr, MDP_ERR_NODEVICE, "no HIP device available");
    if (device < 0 || device >= count) return fail(nullptr, MDP_ERR_NODEVICE, "device index out of range");
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, MDP_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    auto* ctx = new (std::nothrow) mdp_ctx;
    if (!ctx) return fail(nullptr, MDP_ERR_OOM, "host allocation failed");
    ctx->device = device;
    if (const char* s = std::getenv("MDP_WORKSPACE_GB")) {
        double gb = std::atof(s);
        if (gb > 0) ctx->ws_cap = (size_t)(gb * (1ull << 30));
    }
    e = hipEventCreateWithFlags(&ctx->last, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete ctx;
        return fail(nullptr, MDP_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
    }
    // the device address of the static scratch array of mdp_ap_solve_noalloc (with the device current)
    try {
        ctx->scratch = noalloc_scratch(device);
    } catch (const Error& err) {
        (void)hipEventDestroy(ctx->last);
        delete ctx;
        return fail(nullptr, err.code, err.what());
    }
    *out = ctx;
    return MDP_OK;
}

void mdp_destroy(mdp_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : ctx->cache) mdp_projector_release(kv.second);
    ctx->cache.clear();
    ctx->plans.clear();
    if (ctx->last) (void)hipEventDestroy(ctx->last);
    delete ctx;
}

int mdp_set_projector_path(mdp_ctx* ctx, int path) {
    if (!ctx) return fail(nullptr, MDP_ERR_ARG, "ctx is NULL");
    if (path != MDP_PATH_AUTO && path != MDP_PATH_DENSE) return fail(ctx, MDP_ERR_ARG, "unknown projector path");
    ctx->projector_path = path;
    return MDP_OK;
}

int mdp_set_autotune(mdp_ctx* ctx, int enable) {
    if (!ctx) return fail(nullptr, MDP_ERR_ARG, "ctx is NULL");
    set_gemm_autotune(enable);
    set_sweep_autotune(enable);
    return MDP_OK;
}

int mdp_set_fused_schedule(mdp_ctx* ctx, int cols_per_lane) {
    if (!ctx) return fail(nullptr, MDP_ERR_ARG, "ctx is NULL");
    if (cols_per_lane != 0 && cols_per_lane != 1 && cols_per_lane != 2 && cols_per_lane != 4)
        return fail(ctx, MDP_ERR_ARG, "columns per lane must be 0, 1, 2 or 4");
    ctx->sweep_cols = cols_per_lane;
    return MDP_OK;
}

int mdp_fused_schedule_used(const mdp_ctx* ctx) { return ctx ? ctx->last_sweep_cols : 0; }

int mdp_set_interface_path(mdp_ctx* ctx, int path) {
    if (!ctx) return fail(nullptr, MDP_ERR_ARG, "ctx is NULL");
    if (path != MDP_IFACE_AUTO && path != MDP_IFACE_DENSE && path != MDP_IFACE_MULTIFRONTAL)
        return fail(ctx, MDP_ERR_ARG, "unknown interface path");
    ctx->interface_path = path;
    return MDP_OK;
}

const char* mdp_last_error(const mdp_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

int mdp_build_projectors(mdp_ctx* ctx, int count, const mdp_subdomain* sds, int m_star, int precision, void* stream,
                         mdp_projector** out) {
    if (!ctx) return fail(nullptr, MDP_ERR_ARG, "ctx is NULL");
    if (out && count > 0) std::memset(out, 0, sizeof(mdp_projector*) * count);
    return guarded(ctx, [&]() -> int {
        if (count < 1) throw Error(MDP_ERR_ARG, "count must be >= 1");
        if (!sds || !out) throw Error(MDP_ERR_ARG, "null subdomain or output pointer");
        if (m_star < 1) throw Error(MDP_ERR_ARG, "M* must be >= 1");
        check_precision(precision);
        for (int i = 0; i < count; ++i)
            if (!std::isfinite(sds[i].k) || !(sds[i].k > 0)) throw Error(MDP_ERR_NONFINITE, "k must be finite and > 0");
        hipStream_t st = (hipStream_t)stream;
        std::vector<mdp_projector*> res(count, nullptr);
        std::vector<FusedItem> fused;
        std::vector<std::pair<ProjKey, mdp_projector*>> fresh;   // built by this call, not yet cached
        CallScope scope;
        try {
            // the gamma tables of geometries new to the context in one upload; E of every fresh
            // projector and the new geometries' node maps in one launch pair
            struct SetupSrc { GeomShared* geo; size_t base, o_gm, o_gq, o_side, o_rho, o_t, o_slen; };
            HostBlob setup;
            std::vector<SetupSrc> gnew;                     // geometries uploaded by this call
            std::vector<std::pair<mdp_projector*, int>> ejobs;   // projector, its geometry in gnew (-1: resident)
            int max_nodes = 0;
            std::vector<std::pair<mdp_projector*, APPlan*>> dense;   // the full-solve route, after the set-up
            for (int i = 0; i < count; ++i) {
                const mdp_subdomain* sd = &sds[i];
                ProjKey key{sd->lx, sd->ly, sd->n, sd->k, m_star, precision};
                auto it = ctx->cache.find(key);
                if (it != ctx->cache.end()) { res[i] = it->second; continue; }
                bool dup = false;
                for (auto& kv : fresh)
                    if (kv.first == key) { res[i] = kv.second; dup = true; }
                if (dup) continue;
                scope.open(ctx, st);
                // the grid sets relative to the rectangle depend on its size and n only
                GeomKey gk{sd->lx, sd->ly, sd->n};
                auto git = ctx->geoms.find(gk);
                if (git == ctx->geoms.end())
                    git = ctx->geoms
                              .emplace(gk, std::make_shared<GeomShared>(
                                               make_geometry(sd->x0, sd->y0, sd->lx, sd->ly, sd->n)))
                              .first;
                GeomShared& gs = *git->second;
                int gi = -1;
                if (!gs.on_device) {
                    for (size_t q = 0; q < gnew.size(); ++q)
                        if (gnew[q].geo == &gs) gi = (int)q;
                    if (gi < 0) {
                        const Geometry& g = gs.g;
                        HostBlob blob;
                        SetupSrc ss{&gs, 0, 0, 0, 0, 0, 0, 0};
                        ss.o_gm = blob.put(g.gm);
                        ss.o_gq = blob.put(g.gq);
                        ss.o_side = blob.put(g.side);
                        ss.o_rho = blob.put(g.rho);
                        ss.o_t = blob.put(g.t);
                        ss.o_slen = blob.put(g.slen);
                        if (blob.size() % 4) throw Error(MDP_ERR_ARG, "gamma tables not in 4-byte words");
                        ss.base = setup.put(blob.data(), blob.size());
                        gs.meta.alloc(blob.size());
                        const char* mb = gs.meta.as<char>();
                        gs.gm = reinterpret_cast<const int*>(mb + ss.o_gm);
                        gs.gq = reinterpret_cast<const int*>(mb + ss.o_gq);
                        gs.gside = reinterpret_cast<const int*>(mb + ss.o_side);
                        gs.grho = reinterpret_cast<const double*>(mb + ss.o_rho);
                        gs.gt = reinterpret_cast<const double*>(mb + ss.o_t);
                        gs.gslen = reinterpret_cast<const double*>(mb + ss.o_slen);
                        gs.gidx.alloc((size_t)(g.n + 1) * (g.n + 1) * sizeof(int));
                        max_nodes = std::max(max_nodes, (g.n + 1) * (g.n + 1));
                        gi = (int)gnew.size();
                        gnew.push_back(ss);
                    }
                }
                APPlan& plan = get_plan(ctx, gs.g.n, gs.g.h, sd->k);
                std::unique_ptr<mdp_projector> P(new mdp_projector(git->second));
                P->device = ctx->device;
                P->serial = ctx->next_serial++;
                P->k = sd->k;
                P->m_star = m_star;
                P->precision = precision;
                P->pool = ctx->pool;
                BufPool& pool = *ctx->pool;
                const int ng = gs.g.n_gamma, ncol = 8 * m_star;
                P->E = pool.take((size_t)ng * ncol * sizeof(double));
                P->Q = pool.take((size_t)ng * ncol * 2 * sizeof(double));
                max_nodes = std::max(max_nodes, ng);
                const Geometry& G = P->g;
                mdp_projector* raw = P.release();
                fresh.push_back({key, raw});
                ejobs.push_back({raw, gi});
                res[i] = raw;
                if ((precision == MDP_C128 || precision == MDP_C64) && ctx->projector_path == MDP_PATH_AUTO &&
                    fused_projector_supported(plan.f, G.m_lo, G.m_hi, G.q_lo, G.q_hi) &&
                    plan.twist_ratio[G.m_hi + 1] > 1e-13) {
                    fused.push_back({&plan, raw});
                    continue;
                }
                dense.push_back({raw, &plan});
            }
            if (!ejobs.empty()) {
                // the job table holds device addresses inside the upload: the image is sized first
                std::vector<GeomJob> jobs;
                const size_t o_jobs = (setup.size() + 255) / 256 * 256;
                char* img =
                    ctx->ws.stage.image_for(o_jobs + (gnew.size() + ejobs.size()) * sizeof(GeomJob));
                auto tables = [&](GeomJob& jb, const SetupSrc& ss) {
                    const char* b = img + ss.base;
                    jb.gm = reinterpret_cast<const int*>(b + ss.o_gm);
                    jb.gq = reinterpret_cast<const int*>(b + ss.o_gq);
                    jb.side = reinterpret_cast<const int*>(b + ss.o_side);
                    jb.rho = reinterpret_cast<const double*>(b + ss.o_rho);
                    jb.t = reinterpret_cast<const double*>(b + ss.o_t);
                    jb.slen = reinterpret_cast<const double*>(b + ss.o_slen);
                };
                for (const SetupSrc& ss : gnew) {   // tables to the geometry's buffer, its node map
                    GeomJob jb{};
                    tables(jb, ss);
                    jb.src = img + ss.base;
                    jb.meta = ss.geo->meta.as<char>();
                    jb.meta_words = (long)(ss.geo->meta.bytes / 4);
                    jb.ng = ss.geo->g.n_gamma;
                    jb.n = ss.geo->g.n;
                    jb.gidx = ss.geo->gidx.as<int>();
                    jobs.push_back(jb);
                }
                for (const auto& ej : ejobs) {   // E of each fresh projector
                    const mdp_projector* P = ej.first;
                    GeomJob jb{};
                    if (ej.second >= 0) {
                        tables(jb, gnew[ej.second]);   // the geometry arrives with this call
                    } else {
                        jb.gm = P->gm; jb.gq = P->gq; jb.side = P->gside;
                        jb.rho = P->grho; jb.t = P->gt; jb.slen = P->gslen;
                    }
                    jb.ng = P->g.n_gamma;
                    jb.n = P->g.n;
                    jb.M = m_star;
                    jb.k = P->k;
                    jb.E = P->E.as<double>();
                    jobs.push_back(jb);
                }
                if (setup.put(jobs) != o_jobs) throw Error(MDP_ERR_ARG, "set-up table layout");
                if (ctx->ws.stage.upload(setup, st) != img) throw Error(MDP_ERR_ARG, "set-up image moved");
                launch_geom_setup(reinterpret_cast<const GeomJob*>(img + o_jobs), (int)jobs.size(), max_nodes, st);
                for (const SetupSrc& ss : gnew) ss.geo->on_device = true;
            }
            for (auto& dp : dense) {
                // dense route: full AP solves of the columns, gathered onto gamma
                mdp_projector* raw = dp.first;
                APPlan& plan = *dp.second;
                const Geometry& G = raw->g;
                const int ng = G.n_gamma, ncol = 8 * m_star;
                const int chunk = chunk_size(plan, precision, ctx->ws_cap, ncol);
                prepare_ws(ctx, plan, precision, chunk);
                for (int col0 = 0; col0 < ncol; col0 += chunk) {
                    const int R = std::min(chunk, ncol - col0);
                    SrcDesc src{};
                    src.kind = Src::STENCIL_E;
                    src.E = raw->E.as<double>();
                    src.ldE = ng;
                    src.col0 = col0;
                    src.gidx = raw->gidx;
                    src.m_lo = G.m_lo; src.m_hi = G.m_hi; src.q_lo = G.q_lo; src.q_hi = G.q_hi;
                    double* Qd = raw->Q.as<double>();
                    const int* gmd = raw->gm;
                    const int* gqd = raw->gq;
                    const int n = G.n;
                    const Fold f = plan.f;
                    solve_batch(plan, ctx->ws, precision, src, false, R, box_band(plan, G),
                                [&](const void* u, const float* du, Band bd) {
                                    ctx->ws.prof.run("gather_q", st, 0.0, (double)ng * R * 16.0 * 2.0, [&] {
                                        if (precision == MDP_C128)
                                            launch_gather_q<double>((const double*)u, du, n, f, bd, gmd, gqd, ng, R,
                                                                    Qd, ng, col0, st);
                                        else
                                            launch_gather_q<float>((const float*)u, du, n, f, bd, gmd, gqd, ng, R,
                                                                   Qd, ng, col0, st);
                                    });
                                },
                                st);
                }
            }
            build_q_fused(ctx, fused, precision, st);
        } catch (...) {
            // nothing built by this call is handed out; its projectors are dropped after the device drains
            (void)hipDeviceSynchronize();
            for (auto& kv : fresh) mdp_projector_release(kv.second);
            throw;
        }
        for (auto& kv : fresh) {
            kv.second->refs.store(1);   // the cache's reference; the callers' follow
            ctx->cache[kv.first] = kv.second;
        }
        for (int i = 0; i < count; ++i) {
            res[i]->refs.fetch_add(1);
            out[i] = res[i];
        }
        return MDP_OK;
    });
}

int mdp_build_projector(mdp_ctx* ctx, const mdp_subdomain* sd, int m_star, int precision, void* stream,
                        mdp_projector** out) {
    if (!ctx) return fail(nullptr, MDP_ERR_ARG, "ctx is NULL");
    if (!sd || !out) return fail(ctx, MDP_ERR_ARG, "null subdomain or output pointer");
    return mdp_build_projectors(ctx, 1, sd, m_star, precision, stream, out);
}

int mdp_projector_info(const mdp_projector* P, int* n_gamma, const int** gamma_mq, const mdp_c128** q_dev) {
    if (!P) return MDP_ERR_ARG;
    if (n_gamma) *n_gamma = P->g.n_gamma;
    if (gamma_mq) *gamma_mq = P->g.gmq.data();
    if (q_dev) *q_dev = P->Q.as<const mdp_c128>();
    return MDP_OK;
}

int mdp_ap_grid(const mdp_subdomain* sd, double* xa, double* ya, double* h) {
    if (!sd || !xa || !ya || !h) return MDP_ERR_ARG;
    try {
        const Geometry g = make_geometry(sd->x0, sd->y0, sd->lx, sd->ly, sd->n);
        *xa = g.xa;
        *ya = g.ya;
        *h = g.h;
        return MDP_OK;
    } catch (const Error& e) {
        return e.code;
    }
}

int mdp_projector_gamma_feet(const mdp_projector* P, const mdp_subdomain* sd, double* xy_out, int* side_out) {
    if (!P || !sd || !xy_out) return MDP_ERR_ARG;
    const Geometry& g = P->g;
    if (sd->lx != g.lx || sd->ly != g.ly) return MDP_ERR_ARG;
    for (int i = 0; i < g.n_gamma; ++i) {
        const int s = g.side[i];
        const double t = g.t[i];
        double x, y;
        if (s == 0 || s == 1) {
            x = sd->x0 + 0.5 * (t + 1.0) * sd->lx;
            y = (s == 0) ? sd->y0 : sd->y0 + sd->ly;
        } else {
            y = sd->y0 + 0.5 * (t + 1.0) * sd->ly;
            x = (s == 2) ? sd->x0 : sd->x0 + sd->lx;
        }
        xy_out[2 * i] = x;
        xy_out[2 * i + 1] = y;
        if (side_out) side_out[i] = s;
    }
    return MDP_OK;
}

void mdp_projector_release(mdp_projector* P) {
    if (!P) return;
    if (P->refs.fetch_sub(1) == 1) {
        (void)hipSetDevice(P->device);
        // the buffers go back to the context's pool (freed with it)
        P->pool->give(std::move(P->Q));
        P->pool->give(std::move(P->E));
        delete P;
    }
}

// ---------------------------------------------------------------------------- step 2
namespace {

struct Contrib { int sub, side, kind; double2 coef; };
struct Block { int type; std::vector<Contrib> c; };  // type 0 Dirichlet, 1 Neumann, 2 Robin, 3 interface

bool same(double a, double b) { return std::fabs(a - b) <= 1e-12 * std::max(1.0, std::max(std::fabs(a), std::fabs(b))); }

// endpoints of side s of subdomain sd: (x, y) of both ends
void side_segment(const mdp_subdomain& sd, int s, double* seg) {
    double x0 = sd.x0, y0 = sd.y0, x1 = sd.x0 + sd.lx, y1 = sd.y0 + sd.ly;
    switch (s) {
        case 0: seg[0] = x0; seg[1] = y0; seg[2] = x1; seg[3] = y0; break;
        case 1: seg[0] = x0; seg[1] = y1; seg[2] = x1; seg[3] = y1; break;
        case 2: seg[0] = x0; seg[1] = y0; seg[2] = x0; seg[3] = y1; break;
        default: seg[0] = x1; seg[1] = y0; seg[2] = x1; seg[3] = y1; break;
    }
}

}  // namespace

namespace {

// Receivers and outputs of a gradient call (host arrays).
struct GradArgs {
    int n_rcv;
    const int* rcv_sub;
    const int* rcv_node;
    const mdp_c128* ubar;
    double* grad_k2;
    mdp_c128* grad_d;
};

// Reverse pass of Phi = Re sum_r conj(ubar_r) u_r (u the reconstruction of eq. potential_solution_homo,
// f = 0) through the three steps of Sec. 3.5, after the interface solve left x, Fbar and the Gram factor:
//   u_i = w_i - A_i^{-1}(L w_i |M+), w_i = E_i c_i on gamma:
//       cbar_i = E_i^T [ubar_i - L^T (A_i^{-H} ubar_i)|M+] on gamma;
//   c = K x + known(d):  xbar = K^* cbar;
//   x = (Qbar^* Qbar)^{-1} Qbar^* Fbar:  z = (Qbar^* Qbar)^{-1} xbar, Fbb = Qbar z, r = Fbar - Qbar x;
//   boundary data: dPhi/dd = (cbar_known - Q_known^* Fbb) / (alpha or beta);
//   k_i^2: Re[ <ubar, du/dk^2>_c fixed - <Fbb_i, dQ_i c_i> + <r_i, dQ_i cz_i> ] with cz = K z, where
//       for a density c: v = A^{-1}(L w|M+), h = -dA v + (dL w + L dw)|M+ (dw = dE c), y = A^{-1} h,
//       dQ c = -y|gamma and du/dk^2 = dw - y.
void interface_gradient(mdp_ctx* ctx, int n_sub, const mdp_subdomain* sd, const mdp_projector* const* P,
                        const mdp_side* sides, int M, const PackedHost& ph, const PackedTables& tabs, const char* img,
                        const double2* F, const double2* x, const double2* c_full, const int* esrc, const double2* ecoef, const std::vector<int>& row_off, const GradArgs& ga,
                        hipStream_t st);

// The interface solve of step 2; with ga set, the reverse pass of the receiver functional follows.
int solve_interface_impl(mdp_ctx* ctx, int n_sub, const mdp_subdomain* subs, const mdp_projector* const* P,
                         const mdp_side* sides, int m_star, const mdp_source* sources, void* stream, mdp_c128* c_out,
                         double* rel_residual_out, double* cond_estimate_out, const GradArgs* ga) {
    if (!ctx) return fail(nullptr, MDP_ERR_ARG, "ctx is NULL");
    return guarded(ctx, [&]() -> int {
        if (n_sub < 1 || !subs || !P || !sides || !c_out) throw Error(MDP_ERR_ARG, "null or empty arguments");
        if (m_star < 1) throw Error(MDP_ERR_ARG, "M* must be >= 1");
        hipStream_t st = (hipStream_t)stream;
        for (int i = 0; i < n_sub; ++i) {
            if (!P[i]) throw Error(MDP_ERR_ARG, "null projector");
            if (P[i]->m_star != m_star) throw Error(MDP_ERR_ARG, "projector built with a different M*");
        }
        const int M = m_star;
        std::vector<mdp_subdomain> sd(subs, subs + n_sub);
        for (int i = 0; i < n_sub; ++i) {
            const Geometry& g = P[i]->g;
            if (sd[i].lx != g.lx || sd[i].ly != g.ly || sd[i].n != g.n || sd[i].k != P[i]->k)
                throw Error(MDP_ERR_ARG, "projector does not match its subdomain (size, n or k)");
        }
        // unknown blocks (Sec. 3.3.3): boundary sides keep one M*-block, interfaces two
        std::vector<Block> blocks;
        for (int i = 0; i < n_sub; ++i) {
            for (int s = 0; s < 4; ++s) {
                const mdp_side& sd_ = sides[4 * i + s];
                if (sd_.kind == 0) {
                    const double a = sd_.alpha, b = sd_.beta;
                    if (!std::isfinite(a) || !std::isfinite(b)) throw Error(MDP_ERR_NONFINITE, "non-finite alpha/beta");
                    if (a == 0.0 && b == 0.0) throw Error(MDP_ERR_ARG, "boundary side with alpha = beta = 0");
                    if (!sd_.d) throw Error(MDP_ERR_ARG, "boundary side without data coefficients");
                    for (int j = 0; j < M; ++j)
                        if (!std::isfinite(sd_.d[j].re) || !std::isfinite(sd_.d[j].im))
                            throw Error(MDP_ERR_NONFINITE, "non-finite boundary coefficient");
                    if (b == 0.0) blocks.push_back({0, {{i, s, 1, {1.0, 0.0}}}});
                    else if (a == 0.0) blocks.push_back({1, {{i, s, 0, {1.0, 0.0}}}});
                    else blocks.push_back({2, {{i, s, 0, {1.0, 0.0}}, {i, s, 1, {-a / b, 0.0}}}});
                } else if (sd_.kind == 1) {
                    const int j = sd_.nbr, t = sd_.nbr_side;
                    if (j < 0 || j >= n_sub || t < 0 || t > 3 || j == i) throw Error(MDP_ERR_ARG, "bad interface neighbour");
                    const mdp_side& o = sides[4 * j + t];
                    if (o.kind != 1 || o.nbr != i || o.nbr_side != s) throw Error(MDP_ERR_ARG, "interface sides do not match");
                    double a[4], b[4];
                    side_segment(sd[i], s, a);
                    side_segment(sd[j], t, b);
                    for (int e = 0; e < 4; ++e)
                        if (!same(a[e], b[e])) throw Error(MDP_ERR_ARG, "interface segments differ");
                    if (std::make_pair(i, s) < std::make_pair(j, t)) {
                        blocks.push_back({3, {{i, s, 0, {1.0, 0.0}}, {j, t, 0, {1.0, 0.0}}}});
                        blocks.push_back({3, {{i, s, 1, {1.0, 0.0}}, {j, t, 1, {-1.0, 0.0}}}});
                    }
                } else {
                    throw Error(MDP_ERR_ARG, "side kind must be 0 (boundary) or 1 (interface)");
                }
            }
        }
        const int ncol = (int)blocks.size() * M;
        const bool multifrontal = ctx->interface_path == MDP_IFACE_MULTIFRONTAL ||
                                  (ctx->interface_path == MDP_IFACE_AUTO && ncol > 4096 && n_sub > 1);
        // Column order of the unknowns and the steps of the interface Cholesky.  The unknowns are cut into
        // slices of at most 64 columns: each subdomain's private unknowns (its boundary sides), and the
        // unknowns of each interface.  Two slices couple in the Gram matrix only if some subdomain's rows
        // touch both, i.e. if they share a subdomain.  A symbolic elimination groups the slices into steps:
        // each step takes slices that are mutually uncoupled in the current (filled) coupling graph, so that
        // their diagonal blocks factor independently in one launch; eliminating a slice couples all its
        // remaining neighbours.  A step takes, fewest couplings first, only slices with at most `slack` times
        // the smallest current coupling count (eliminating a well-connected slice early fills the graph);
        // the slack giving the fewest steps is kept.  perm maps the column b*M + j of block b to its place.
        std::vector<int> perm(ncol);
        CholPlan chol_steps;
        if (multifrontal) {
            // the elimination tree orders the columns itself
            for (int c = 0; c < ncol; ++c) perm[c] = c;
        } else {
            struct Slice { std::vector<int> cols; std::vector<int> subs; };
            std::vector<Slice> slices;
            std::map<std::pair<int, int>, std::vector<int>> groups;   // (sub, sub) -> columns (sub, -1: private)
            for (size_t b = 0; b < blocks.size(); ++b) {
                const Block& B = blocks[b];
                int s0 = B.c[0].sub, s1 = -1;
                for (const Contrib& c : B.c)
                    if (c.sub != s0) s1 = c.sub;
                auto& g = groups[{s0, s1}];
                for (int j = 0; j < M; ++j) g.push_back((int)b * M + j);
            }
            for (auto& kv : groups) {
                const std::vector<int>& cols = kv.second;
                for (size_t lo = 0; lo < cols.size(); lo += 64) {
                    Slice sl;
                    sl.cols.assign(cols.begin() + lo, cols.begin() + std::min(cols.size(), lo + 64));
                    sl.subs.push_back(kv.first.first);
                    if (kv.first.second >= 0) sl.subs.push_back(kv.first.second);
                    slices.push_back(std::move(sl));
                }
            }
            const int ns = (int)slices.size();
            std::vector<std::vector<char>> adj0(ns, std::vector<char>(ns, 0));
            for (int u = 0; u < ns; ++u)
                for (int v = 0; v < ns; ++v)
                    if (u != v)
                        for (int a1 : slices[u].subs)
                            for (int a2 : slices[v].subs)
                                if (a1 == a2) adj0[u][v] = 1;
            auto schedule = [&](double slack) {
                std::vector<std::vector<int>> steps;
                std::vector<std::vector<char>> adj = adj0;
                std::vector<char> done(ns, 0);
                for (int left = ns; left > 0;) {
                    std::vector<int> order, deg(ns, 0);
                    for (int u = 0; u < ns; ++u) {
                        if (done[u]) continue;
                        order.push_back(u);
                        for (int v = 0; v < ns; ++v) deg[u] += (!done[v] && adj[u][v]);
                    }
                    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return deg[x] < deg[y]; });
                    const double cap = slack * std::max(deg[order[0]], 1);
                    std::vector<int> pick;
                    for (int u : order) {
                        if (deg[u] > cap) break;
                        bool ok = true;
                        for (int v : pick) ok = ok && !adj[u][v];
                        if (ok) pick.push_back(u);
                    }
                    for (int u : pick) {   // the eliminated slice's remaining neighbours become coupled
                        done[u] = 1;
                        --left;
                        for (int v = 0; v < ns; ++v)
                            for (int w2 = 0; w2 < ns; ++w2)
                                if (v != w2 && !done[v] && !done[w2] && adj[u][v] && adj[u][w2]) adj[v][w2] = 1;
                    }
                    steps.push_back(pick);
                }
                return steps;
            };
            std::vector<std::vector<int>> best;
            for (double slack : {1.0, 1.5, 2.0, 3.0, 1e9}) {
                auto st = schedule(slack);
                if (best.empty() || st.size() < best.size()) best = st;
            }
            int next = 0;
            for (const auto& step : best) {
                std::vector<int> widths;
                for (int u : step) {
                    for (int c : slices[u].cols) perm[c] = next++;
                    widths.push_back((int)slices[u].cols.size());
                }
                chol_steps.push_back(widths);
            }
        }
        std::vector<int> row_off(n_sub + 1, 0);
        for (int i = 0; i < n_sub; ++i) row_off[i + 1] = row_off[i] + P[i]->g.n_gamma;
        const int m = row_off[n_sub];
        if (m < ncol) throw Error(MDP_ERR_ARG, "fewer gamma rows than unknowns");
        // column map per (subdomain, Qbar column): the dense route's fallback assembles Qbar from it
        std::vector<int4> colmap(multifrontal ? 0 : (size_t)n_sub * ncol, int4{-1, -1, 0, 0});
        std::vector<double2> coefs(multifrontal ? 0 : (size_t)n_sub * ncol * 2, double2{0.0, 0.0});
        for (size_t b = 0; b < blocks.size() && !multifrontal; ++b) {
            for (const Contrib& c : blocks[b].c) {
                for (int j = 0; j < M; ++j) {
                    const size_t idx = (size_t)c.sub * ncol + perm[b * M + j];
                    const int qcol = c.kind * 4 * M + c.side * M + j;
                    if (colmap[idx].x < 0) { colmap[idx].x = qcol; coefs[2 * idx] = c.coef; }
                    else { colmap[idx].y = qcol; coefs[2 * idx + 1] = c.coef; }
                }
            }
        }
        // known coefficients moved to the right-hand side
        std::vector<int> kcol, koff(n_sub + 1, 0);
        std::vector<double2> kval;
        for (int i = 0; i < n_sub; ++i) {
            for (int s = 0; s < 4; ++s) {
                const mdp_side& sd_ = sides[4 * i + s];
                if (sd_.kind != 0) continue;
                const double a = sd_.alpha, b = sd_.beta;
                const int kind = (b == 0.0) ? 0 : 1;          // Dirichlet: known c0 = d/alpha; else c1 part d/beta
                const double div = (b == 0.0) ? a : b;
                for (int j = 0; j < M; ++j) {
                    kcol.push_back(kind * 4 * M + s * M + j);
                    kval.push_back(double2{sd_.d[j].re / div, sd_.d[j].im / div});
                }
            }
            koff[i + 1] = (int)kcol.size();
        }
        // the full coefficient vectors from the unknowns: c[e] = known[e] + coef[e] x[src[e]]
        const int nce = n_sub * 8 * M;
        std::vector<int> esrc(nce, -1);
        std::vector<double2> ecoef(nce, double2{0.0, 0.0}), eknown(nce, double2{0.0, 0.0});
        auto E = [&](int i, int kind, int s, int j) { return (size_t)i * 8 * M + kind * 4 * M + s * M + j; };
        for (size_t b = 0; b < blocks.size(); ++b) {
            const Block& B = blocks[b];
            for (int j = 0; j < M; ++j) {
                if (B.type == 2) {
                    const size_t e = E(B.c[0].sub, 0, B.c[0].side, j);
                    esrc[e] = perm[b * M + j];
                    ecoef[e] = double2{1.0, 0.0};
                    continue;
                }
                for (const Contrib& ct : B.c) {
                    const size_t e = E(ct.sub, ct.kind, ct.side, j);
                    esrc[e] = perm[b * M + j];
                    ecoef[e] = ct.coef;
                }
            }
        }
        for (int i = 0; i < n_sub; ++i)
            for (int s = 0; s < 4; ++s) {
                const mdp_side& sd_ = sides[4 * i + s];
                if (sd_.kind != 0) continue;
                const double a = sd_.alpha, b = sd_.beta;
                for (int j = 0; j < M; ++j) {
                    const double2 d{sd_.d[j].re, sd_.d[j].im};
                    if (b == 0.0) eknown[E(i, 0, s, j)] = double2{d.x / a, d.y / a};
                    else if (a == 0.0) eknown[E(i, 1, s, j)] = double2{d.x / b, d.y / b};
                    else {   // c1 = d/beta - (alpha/beta) c0
                        const size_t e = E(i, 1, s, j);
                        esrc[e] = esrc[E(i, 0, s, j)];
                        ecoef[e] = double2{-a / b, 0.0};
                        eknown[e] = double2{d.x / b, d.y / b};
                    }
                }
            }
        std::vector<const double2*> qsrc(n_sub);
        std::vector<int> qld(n_sub);
        for (int i = 0; i < n_sub; ++i) { qsrc[i] = P[i]->Q.as<const double2>(); qld[i] = P[i]->g.n_gamma; }
        // The host side below (packed description, elimination tree, tables) depends on the layout, the side
        // kinds and coefficients and M* only: it is kept from the last call of the same structure (without
        // sources), whose tables then get this call's projector addresses and boundary data.
        bool has_src = false;
        for (int i = 0; sources && i < n_sub; ++i) has_src = has_src || sources[i].f != nullptr;
        std::vector<double> skey{(double)M, multifrontal ? 1.0 : 0.0, (double)n_sub};
        for (int i = 0; i < n_sub; ++i) {
            skey.insert(skey.end(), {sd[i].x0, sd[i].y0, sd[i].lx, sd[i].ly, (double)sd[i].n, (double)qld[i]});
            for (int s = 0; s < 4; ++s) {
                const mdp_side& q = sides[4 * i + s];
                skey.insert(skey.end(), {(double)q.kind, q.kind == 0 ? q.alpha : (double)q.nbr,
                                         q.kind == 0 ? q.beta : (double)q.nbr_side});
            }
        }
        IfaceCache& ic = ctx->icache;
        const bool plan_hit = !has_src && ic.valid && ic.key == skey && ic.ap == ctx->ws.pk.Ap.p &&
                              ic.mf == ctx->ws.pk.mf.p;
        if (!plan_hit) ic.valid = false;
        // block-sparse description: subdomain i's rows touch only the unknown blocks with a contribution from i
        PackedHost ph_new;
        if (!plan_hit) {
        PackedHost& ph = ph_new;
        ph.n_sub = n_sub;
        ph.nc = ncol;
        ph.steps = chol_steps;
        ph.Q = qsrc;
        ph.m = qld;
        long off = 0;
        for (int i = 0; i < n_sub; ++i) {
            ph.off.push_back(off);
            ph.roff.push_back(row_off[i]);
            ph.pc_start.push_back((int)ph.pc_sub.size());
            int si = 0;
            for (size_t b = 0; b < blocks.size(); ++b) {
                std::vector<const Contrib*> mine;
                for (const Contrib& c : blocks[b].c)
                    if (c.sub == i) mine.push_back(&c);
                if (mine.empty()) continue;
                for (int j = 0; j < M; ++j) {
                    int4 cm{-1, -1, 0, 0};
                    double2 w0{0.0, 0.0}, w1{0.0, 0.0};
                    cm.x = mine[0]->kind * 4 * M + mine[0]->side * M + j;
                    w0 = mine[0]->coef;
                    if (mine.size() > 1) {
                        cm.y = mine[1]->kind * 4 * M + mine[1]->side * M + j;
                        w1 = mine[1]->coef;
                    }
                    ph.pc_sub.push_back(i);
                    ph.pc_p.push_back(si);
                    ph.pc_gcol.push_back(perm[b * M + j]);
                    ph.pc_cols.push_back(cm);
                    ph.pc_coef.push_back(w0);
                    ph.pc_coef.push_back(w1);
                    ++si;
                }
            }
            ph.s.push_back(si);
            ph.max_s = std::max(ph.max_s, si);
            ph.max_m = std::max(ph.max_m, qld[i]);
            off += (long)qld[i] * si;
        }
        ph.total_pc = (int)ph.pc_sub.size();
        if (multifrontal) {
            for (int i = 0; i < n_sub; ++i) {
                ph.cx.push_back(sd[i].x0 + 0.5 * sd[i].lx);
                ph.cy.push_back(sd[i].y0 + 0.5 * sd[i].ly);
            }
            ph.mf = mf_plan(ph);
            if (ph.mf.lds_fwd > 4096 || ph.mf.lds_bwd > 4096)
                throw Error(MDP_ERR_ARG, "interface front too large for the multifrontal solve");
            ph.multifrontal = true;
        }
        }

        // step 1c: subdomains with a source, grouped by projector (one batched AP solve per group)
        struct SrcGroup { const mdp_projector* P; int R; size_t e0; };
        std::vector<SrcGroup> src_groups;
        std::vector<const double*> s_f, s_jet;
        std::vector<long> s_goff, s_foff;
        long srcw_elems = 0;
        if (sources) {
            std::vector<bool> used(n_sub, false);
            for (int i = 0; i < n_sub; ++i) {
                if (!sources[i].f || used[i]) continue;
                SrcGroup sg{P[i], 0, s_f.size()};
                const long npts = (long)(P[i]->g.n + 1) * (P[i]->g.n + 1);
                for (int j = i; j < n_sub; ++j) {
                    if (P[j] != P[i] || !sources[j].f) continue;
                    if (!sources[j].jet) throw Error(MDP_ERR_ARG, "source without its boundary jet");
                    used[j] = true;
                    s_f.push_back(reinterpret_cast<const double*>(sources[j].f));
                    s_jet.push_back(reinterpret_cast<const double*>(sources[j].jet));
                    s_goff.push_back(srcw_elems);
                    s_foff.push_back(row_off[j]);
                    srcw_elems += npts;
                    ++sg.R;
                }
                src_groups.push_back(sg);
            }
        }

        CallScope scope(ctx, st);
        CallWork& cw = ctx->ws.cw;
        DevBuf &F = cw.F, &x = cw.x;
        ensure(F, (size_t)m * sizeof(double2));
        ensure(x, (size_t)ncol * sizeof(double2));
        if (srcw_elems) ensure(cw.srcw, (size_t)srcw_elems * sizeof(double2));
        // every table of the call in one upload
        HostBlob blob_new;
        PackedTables tabs_new{};
        IfaceOffs o_new{};
        if (!plan_hit) {
            HostBlob& blob = blob_new;
            // the per-call part first (one contiguous range to rewrite when the tables are kept)
            o_new.qsrc = blob.put(qsrc);
            o_new.kval = blob.put(kval);
            o_new.eknown = blob.put(eknown);
            const size_t dyn_end = blob.size();
            o_new.qld = blob.put(qld);
            o_new.roff = blob.put(row_off);
            o_new.cmap = blob.put(colmap);
            o_new.coef = blob.put(coefs);
            o_new.kcol = blob.put(kcol);
            o_new.koff = blob.put(koff);
            o_new.esrc = blob.put(esrc);
            o_new.ecoef = blob.put(ecoef);
            o_new.sf = blob.put(s_f);
            o_new.sjet = blob.put(s_jet);
            o_new.sgoff = blob.put(s_goff);
            o_new.sfoff = blob.put(s_foff);
            tabs_new = ls_packed_tables(ctx->ws, ph_new, blob);
            tabs_new.Q = o_new.qsrc;   // the same projector addresses, kept in the per-call part
            if (!has_src) {
                ic.key = skey;
                ic.ph = std::move(ph_new);
                ic.blob = std::move(blob_new);
                ic.tabs = tabs_new;
                ic.o = o_new;
                ic.dyn_end = dyn_end;
                ic.ap = ctx->ws.pk.Ap.p;
                ic.mf = ctx->ws.pk.mf.p;
                if (ic.image.bytes < ic.blob.size()) {
                    MDP_HIP(hipDeviceSynchronize());   // earlier calls may still read the old copy
                    ic.image.alloc(ic.blob.size());
                }
                ctx->ws.stage.copy(ic.image.p, ic.blob, st);
                ic.valid = true;
            }
        } else {   // this call's projectors and known coefficients into the kept tables and their device copy
            ic.ph.Q = qsrc;
            ic.blob.put_at(ic.o.qsrc, qsrc);
            ic.blob.put_at(ic.o.kval, kval);
            ic.blob.put_at(ic.o.eknown, eknown);
            ctx->ws.stage.copy(ic.image.p, ic.blob.data(), ic.dyn_end, st);
        }
        const PackedHost& ph = ic.valid ? ic.ph : ph_new;
        const PackedTables& tabs = ic.valid ? ic.tabs : tabs_new;
        const IfaceOffs& O = ic.valid ? ic.o : o_new;
        const size_t o_qsrc = O.qsrc, o_qld = O.qld, o_roff = O.roff, o_cmap = O.cmap, o_coef = O.coef,
                     o_kcol = O.kcol, o_kval = O.kval, o_koff = O.koff, o_esrc = O.esrc, o_ecoef = O.ecoef,
                     o_eknown = O.eknown, o_sf = O.sf, o_sjet = O.sjet, o_sgoff = O.sgoff, o_sfoff = O.sfoff;
        const char* img = ic.valid ? ic.image.as<const char>() : ctx->ws.stage.upload(blob_new, st);
        auto dq = reinterpret_cast<const double2* const*>(img + o_qsrc);
        auto dld = reinterpret_cast<const int*>(img + o_qld);
        auto droff = reinterpret_cast<const int*>(img + o_roff);
        launch_known_rhs(dq, dld, n_sub, droff, m, reinterpret_cast<const int*>(img + o_kcol),
                         reinterpret_cast<const double2*>(img + o_kval), reinterpret_cast<const int*>(img + o_koff),
                         F.as<double2>(), st);
        // F^(i) = Tr G((L w_I - B f)|M+) with w_I = Ex^(I) f on gamma (eq. linear_system_equations:
        // (I - P_gamma) Ex^(I) f = Tr G(L w_I|M+)), added to subdomain i's rows of Fbar
        for (const SrcGroup& sg : src_groups) {
            const mdp_projector* Pi = sg.P;
            const Geometry& G = Pi->g;
            const int n = G.n, ng = G.n_gamma;
            const long npts = (long)(n + 1) * (n + 1);
            APPlan& plan = get_plan(ctx, n, G.h, Pi->k);
            double* wb = cw.srcw.as<double>();
            const long* go = reinterpret_cast<const long*>(img + o_sgoff) + sg.e0;
            const long* fo = reinterpret_cast<const long*>(img + o_sfoff) + sg.e0;
            const double* const* fs = reinterpret_cast<const double* const*>(img + o_sf) + sg.e0;
            const double* const* js = reinterpret_cast<const double* const*>(img + o_sjet) + sg.e0;
            MDP_HIP(hipMemsetAsync(wb + 2 * s_goff[sg.e0], 0, (size_t)sg.R * npts * sizeof(double2), st));
            launch_source_extension(Pi->grho, Pi->gm, Pi->gq, ng, n, Pi->k, js, sg.R, wb, go, false, st);
            const int chunk = chunk_size(plan, Pi->precision, ctx->ws_cap, sg.R);
            prepare_ws(ctx, plan, Pi->precision, chunk);
            const Fold f = plan.f;
            const int prec = Pi->precision;
            for (int r0 = 0; r0 < sg.R; r0 += chunk) {
                const int Rc = std::min(chunk, sg.R - r0);
                SrcDesc src{};
                src.kind = Src::STENCIL_GRID;
                src.grid = wb;
                src.goff = go + r0;
                src.fsrc = fs + r0;
                src.m_lo = G.m_lo; src.m_hi = G.m_hi; src.q_lo = G.q_lo; src.q_hi = G.q_hi;
                solve_batch(plan, ctx->ws, prec, src, true, Rc, box_band(plan, G),
                            [&](const void* u, const float* du, Band bd) {
                                double* Fd = reinterpret_cast<double*>(F.p);
                                if (prec == MDP_C128)
                                    launch_gather_add<double>((const double*)u, n, f, bd, Pi->gm, Pi->gq, ng, Rc, Fd,
                                                              fo + r0, st);
                                else
                                    launch_gather_add<float>((const float*)u, n, f, bd, Pi->gm, Pi->gq, ng, Rc, Fd,
                                                             fo + r0, st);
                                if (du)   // the FP32 correction of a refined solve
                                    launch_gather_add<float>(du, n, f, bd, Pi->gm, Pi->gq, ng, Rc, Fd, fo + r0, st);
                            },
                            st);
            }
        }
        // the system matrix depends on the projectors, the side kinds and coefficients and the route only:
        // when they match the last factored system, its Gram factor is reused (new data or sources change
        // the right-hand side alone; Sec. 3.5 factors Qbar once)
        std::vector<double> key;
        key.push_back((double)m_star);
        key.push_back(multifrontal ? 1.0 : 0.0);
        for (int i = 0; i < n_sub; ++i) {
            key.push_back((double)P[i]->serial);
            for (int s = 0; s < 4; ++s) {
                const mdp_side& q = sides[4 * i + s];
                key.push_back((double)q.kind);
                key.push_back(q.kind == 0 ? q.alpha : (double)q.nbr);
                key.push_back(q.kind == 0 ? q.beta : (double)q.nbr_side);
            }
        }
        const bool reuse = !ctx->iface_key.empty() && ctx->iface_key == key;
        ctx->iface_key.clear();   // set again below once this call's factor is in place
        LSResult r;
        bool fallback = false;
        {
            // the whole least-squares solve as one profiled span (it synchronises internally)
            Profiler& pr = ctx->ws.prof;
            hipEvent_t a = nullptr, b = nullptr;
            const bool span = pr.wants("interface_ls");
            if (span) { a = pr.get(); b = pr.get(); MDP_HIP(hipEventRecord(a, st)); }
            // algorithmic work of the least squares: the semi-normal path's own count, or a Householder QR
            // of the m x ncol matrix for the dense fallback
            double ls_flops = 8.0 * ((double)m * ncol * ncol - (double)ncol * ncol * ncol / 3.0);
            r = ls_solve_packed(ctx->ws, ph, img, tabs, F.as<double2>(), x.as<double2>(), cond_estimate_out != nullptr,
                                st, &fallback, reuse);
            if (fallback && multifrontal)
                throw Error(MDP_ERR_SINGULAR, "interface least squares: the multifrontal Gram factor broke down or "
                                              "the refinement did not converge");
            if (fallback) {
                // dense Cholesky-QR passes on the assembled matrix
                DevBuf Qbar((size_t)m * ncol * sizeof(double2));
                launch_assemble_qbar(dq, dld, n_sub, droff, m, reinterpret_cast<const int4*>(img + o_cmap),
                                     reinterpret_cast<const double2*>(img + o_coef), ncol, Qbar.as<double2>(), m, st);
                r = ls_solve(ctx->ws, Qbar.as<double2>(), F.as<double2>(), m, ncol, x.as<double2>(),
                             cond_estimate_out != nullptr, st);
                MDP_HIP(hipStreamSynchronize(st));
            } else {
                ls_flops = r.flops;
                ctx->iface_key = key;
            }
            if (span) {
                MDP_HIP(hipEventRecord(b, st));
                pr.recs.push_back({"interface_ls", a, b, ls_flops, (double)m * ncol * 16.0});
            }
        }
        // known and solved coefficients into the caller's vector (column order of Q), on the stream
        launch_expand_coeffs(nce, reinterpret_cast<const int*>(img + o_esrc),
                             reinterpret_cast<const double2*>(img + o_ecoef),
                             reinterpret_cast<const double2*>(img + o_eknown), x.as<double2>(),
                             reinterpret_cast<double2*>(c_out), st);
        if (ga) {
            if (fallback) throw Error(MDP_ERR_SINGULAR, "gradient: the interface system needed the dense fallback");
            interface_gradient(ctx, n_sub, sd.data(), P, sides, M, ph, tabs, img, F.as<double2>(), x.as<double2>(),
                               reinterpret_cast<const double2*>(c_out), reinterpret_cast<const int*>(img + o_esrc),
                               reinterpret_cast<const double2*>(img + o_ecoef), row_off, *ga, st);
        }
        if (rel_residual_out) *rel_residual_out = r.rel_residual;
        if (cond_estimate_out) *cond_estimate_out = r.cond;
        return MDP_OK;
    });
}

// refinement steps of the gradient's normal solve (each: two products with the packed matrix and
// one solve with the kept Gram factor)
constexpr int kGradRefineSteps = 2;

void interface_gradient(mdp_ctx* ctx, int n_sub, const mdp_subdomain* sd, const mdp_projector* const* P,
                        const mdp_side* sides, int M, const PackedHost& ph, const PackedTables& tabs, const char* img,
                        const double2* F, const double2* x, const double2* c_full, const int* esrc,
                        const double2* ecoef, const std::vector<int>& row_off, const GradArgs& ga, hipStream_t st) {
    const int nc = ph.nc, ncol = 8 * M, nce = n_sub * ncol;
    const long m_rows = row_off[n_sub];
    // grid offsets (complex elements) of every subdomain in the ubar and lambda grids
    std::vector<long> goff(n_sub + 1, 0);
    int max_ng = 0;
    for (int i = 0; i < n_sub; ++i) {
        goff[i + 1] = goff[i] + (long)(P[i]->g.n + 1) * (P[i]->g.n + 1);
        max_ng = std::max(max_ng, P[i]->g.n_gamma);
    }
    // receivers: values summed per node, grouped by subdomain
    std::map<std::pair<int, int>, double2> acc;
    for (int t = 0; t < ga.n_rcv; ++t) {
        const int i = ga.rcv_sub[t], node = ga.rcv_node[t];   // checked by mdp_dd_gradient
        double2& v = acc[{i, node}];
        v.x += ga.ubar[t].re;
        v.y += ga.ubar[t].im;
    }
    std::vector<long> r_off_all, r_node;   // ubar grid offsets; node within the subdomain's grid
    std::vector<double2> r_val;
    std::vector<int> r_first(n_sub + 1, 0);
    for (const auto& kv : acc) {
        r_off_all.push_back(goff[kv.first.first] + kv.first.second);
        r_node.push_back(kv.first.second);
        r_val.push_back(kv.second);
        ++r_first[kv.first.first + 1];
    }
    for (int i = 0; i < n_sub; ++i) r_first[i + 1] += r_first[i];
    // known coefficients: (subdomain, side, j) of every boundary side
    std::vector<const double2*> kq;
    std::vector<int> krows, kcolv, keidx;
    std::vector<long> kroff;
    std::vector<double> kdiv;
    std::vector<size_t> kout;   // index into grad_d
    for (int i = 0; i < n_sub; ++i)
        for (int s = 0; s < 4; ++s) {
            const mdp_side& sdd = sides[4 * i + s];
            if (sdd.kind != 0) continue;
            const double a = sdd.alpha, b = sdd.beta;
            const int kind = (b == 0.0) ? 0 : 1;   // Dirichlet: c0 = d/alpha; otherwise c1 holds d/beta
            for (int j = 0; j < M; ++j) {
                kq.push_back(P[i]->Q.as<const double2>());
                krows.push_back(P[i]->g.n_gamma);
                kcolv.push_back(kind * 4 * M + s * M + j);
                keidx.push_back(i * ncol + kind * 4 * M + s * M + j);
                kroff.push_back(row_off[i]);
                kdiv.push_back(b == 0.0 ? a : b);
                kout.push_back(((size_t)i * 4 + s) * M + j);
            }
        }
    const int nk = (int)kq.size();
    std::vector<long> entry_off(2 * n_sub);   // JVP scratch offsets: entries 0 (c_full), 1 (cz)
    HostBlob blob;
    const size_t o_roff = blob.put(r_off_all), o_rnode = blob.put(r_node), o_rval = blob.put(r_val),
                 o_goff = blob.put(goff), o_kq = blob.put(kq), o_krows = blob.put(krows), o_kcol = blob.put(kcolv),
                 o_keidx = blob.put(keidx), o_kroff = blob.put(kroff), o_kdiv = blob.put(kdiv);
    std::vector<int> one_idx(n_sub);
    for (int i = 0; i < n_sub; ++i) one_idx[i] = i;
    const size_t o_idx = blob.put(one_idx);
    // subdomains in order of n (the batched solves' GEMMs go per n)
    std::vector<int> ord(n_sub);
    for (int i = 0; i < n_sub; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return P[a]->g.n < P[b]->g.n; });
    // JVP grids: two entries per subdomain (densities c and cz) at goff2[2i + e]; dE per subdomain at de_off[i];
    // the two coefficient sets [c | cz] side by side (entry (i, e) reads vector i + e n_sub)
    std::vector<long> goff2(2 * n_sub), de_off(n_sub + 1, 0);
    std::vector<int> cidx2(2 * n_sub);
    for (int i = 0; i < n_sub; ++i) {
        const long gs = (long)(P[i]->g.n + 1) * (P[i]->g.n + 1);
        goff2[2 * i] = 2 * goff[i];
        goff2[2 * i + 1] = 2 * goff[i] + gs;
        cidx2[2 * i] = i;
        cidx2[2 * i + 1] = n_sub + i;
        de_off[i + 1] = de_off[i] + (long)P[i]->g.n_gamma * ncol;
    }
    // the job-table form of these index arrays follows the job order (ord)
    std::vector<long> goff2_o, goff_o;
    std::vector<int> cidx2_o;
    for (int i : ord) {
        goff2_o.push_back(goff2[2 * i]);
        goff2_o.push_back(goff2[2 * i + 1]);
        cidx2_o.push_back(cidx2[2 * i]);
        cidx2_o.push_back(cidx2[2 * i + 1]);
        goff_o.push_back(goff[i]);
    }
    const size_t o_g2 = blob.put(goff2_o), o_c2 = blob.put(cidx2_o), o_go = blob.put(goff_o),
                 o_g2s = blob.put(goff2);
    // device buffers: grids ubar, lambda; JVP grids w, dw, v, h, y (two per subdomain); dE; wbar; vectors
    CallWork& cw = ctx->ws.cw;
    const long gtot = goff[n_sub];
    size_t off = 0;
    auto take = [&](size_t elems) { const size_t o = off; off += (elems + 15) / 16 * 16; return o; };
    const size_t b_ubar = take(gtot), b_lam = take(gtot), b_w = take(2 * gtot), b_dw = take(2 * gtot),
                 b_v = take(2 * gtot), b_h = take(2 * gtot), b_y = take(2 * gtot),
                 b_dE = take(((size_t)de_off[n_sub] + 1) / 2), b_wbar = take(max_ng), b_cbar = take(nce),
                 b_cc = take(2 * (size_t)nce), b_zero = take(nce), b_xbar = take(nc), b_xs = take(nc),
                 b_zs = take(nc), b_z = take(nc), b_Fbb = take(m_rows), b_r = take(m_rows), b_k = take(n_sub),
                 b_dg = take(nk), b_tab = take((blob.size() + 15) / 16);
    ensure(cw.grad, off * sizeof(double2));
    double2* G0 = cw.grad.as<double2>();
    auto at = [&](size_t o) { return G0 + o; };
    char* tab = reinterpret_cast<char*>(at(b_tab));
    ctx->ws.stage.copy(tab, blob, st);
    auto T = [&](size_t o) { return tab + o; };
    const long* d_goff = reinterpret_cast<const long*>(T(o_goff));
    const int* d_idx = reinterpret_cast<const int*>(T(o_idx));
    const long* d_g2 = reinterpret_cast<const long*>(T(o_g2));
    const int* d_c2 = reinterpret_cast<const int*>(T(o_c2));
    const long* d_go = reinterpret_cast<const long*>(T(o_go));
    const long* d_g2s = reinterpret_cast<const long*>(T(o_g2s));   // subdomain order
    double* ubar = reinterpret_cast<double*>(at(b_ubar));
    double* lam = reinterpret_cast<double*>(at(b_lam));
    Profiler& pr = ctx->ws.prof;
    // (1) ubar grids
    MDP_HIP(hipMemsetAsync(ubar, 0, (size_t)gtot * sizeof(double2), st));
    launch_scatter_values(reinterpret_cast<const long*>(T(o_roff)), reinterpret_cast<const double*>(T(o_rval)),
                          (int)r_val.size(), ubar, st);
    // (2) lambda = A^{-H} ubar for every subdomain in one batched solve; then per subdomain wbar on gamma
    // and cbar = E^T wbar
    std::vector<const APPlan*> plans(n_sub);
    for (int i = 0; i < n_sub; ++i) plans[i] = &get_plan(ctx, P[i]->g.n, P[i]->g.h, P[i]->k);
    {
        std::vector<SolveJob> jobs;
        std::vector<const APPlan*> jp;
        for (int q = 0; q < n_sub; ++q) {
            const int i = ord[q];
            const APPlan& plan = *plans[i];
            SolveJob J{};
            J.src.kind = Src::GRID;
            J.src.grid = ubar;
            J.src.goff = d_go + q;
            J.sc = plan.sc;
            J.f = plan.f;
            J.bd = Band{0, plan.n + 1};
            J.b0 = q;
            J.R = 1;
            J.fac = plan.fac64.as<double>();
            J.colc = plan.colc64.as<double>();
            J.adjoint = 1;
            J.out = lam;
            J.ooff = d_go + q;
            jobs.push_back(J);
            jp.push_back(&plan);
        }
        batched_band_solve(ctx, jobs, jp, nullptr, st);
    }
    double2* cbar = at(b_cbar);
    for (int i = 0; i < n_sub; ++i) {
        const mdp_projector* Pi = P[i];
        const Geometry& G = Pi->g;
        pr.run("adjoint", st, 0.0, 0.0, [&] {
            launch_gamma_adjoint(ubar, lam, d_goff + i, 1, G.n, plans[i]->sc, G.m_lo, G.m_hi, G.q_lo, G.q_hi,
                                 Pi->gm, Pi->gq, G.n_gamma, reinterpret_cast<double*>(at(b_wbar)), 0, st);
            launch_et_apply(Pi->E.as<double>(), G.n_gamma, ncol, reinterpret_cast<const double*>(at(b_wbar)), 0, 1,
                            d_idx + i, reinterpret_cast<double*>(cbar), st);
        });
    }
    // (3) xbar = K^* cbar; z = (Qbar^* Qbar)^{-1} xbar = D^{-1} G^{-1} D^{-1} xbar with the column
    // equilibration D of the packed matrix Ap = Qbar D^{-1} and its Gram matrix G = Ap^* Ap (the forward
    // call's factor), refined like the forward solve (corrected semi-normal steps): the error of one
    // solve with the Gram factor grows like cond(Ap)^2 u, each step against the true normal residual
    // rho = D^{-1} xbar - Ap^*(Ap zs) contracts it by about that factor again
    const double* norms = ctx->ws.ls.norms.as<double>() + nc;
    double2* xbar = at(b_xbar);
    double2* xs = at(b_xs);
    double2* zs = at(b_zs);
    double2* z = at(b_z);
    const char* pimg = img;
    auto pat = [&](size_t o) { return pimg + o; };
    PackedDevice d{reinterpret_cast<const double2* const*>(pat(tabs.Q)), reinterpret_cast<const int*>(pat(tabs.m)),
                   reinterpret_cast<const long*>(pat(tabs.off)), reinterpret_cast<const int*>(pat(tabs.s)),
                   reinterpret_cast<const int*>(pat(tabs.sub)), reinterpret_cast<const int*>(pat(tabs.p)),
                   reinterpret_cast<const int*>(pat(tabs.gcol)), reinterpret_cast<const int4*>(pat(tabs.cols)),
                   reinterpret_cast<const double2*>(pat(tabs.coef)), reinterpret_cast<const long*>(pat(tabs.roff)),
                   reinterpret_cast<const int*>(pat(tabs.start)), reinterpret_cast<const int*>(pat(tabs.gc_start)),
                   reinterpret_cast<const int*>(pat(tabs.gc_list))};
    const double2* Ap = ctx->ws.pk.Ap.as<double2>();
    double2* Fbb = at(b_Fbb);
    double2* r = at(b_r);
    const double2 one{1.0, 0.0}, mone{-1.0, 0.0};
    MDP_HIP(hipMemsetAsync(xbar, 0, (size_t)nc * sizeof(double2), st));
    launch_expand_adj(nce, esrc, ecoef, cbar, xbar, st);
    MDP_HIP(hipMemcpyAsync(xs, xbar, (size_t)nc * sizeof(double2), hipMemcpyDeviceToDevice, st));
    launch_scale_cols(xs, 1, nc, 1, norms, 1, st);
    ls_packed_factor_solve(ctx->ws, ph, img, tabs, xs, zs, st);
    for (int step = 0; step < kGradRefineSteps; ++step) {
        launch_packed_axpy(d, n_sub, ph.max_m, Ap, zs, one, nullptr, Fbb, nullptr, nullptr, st);   // Ap zs
        launch_packed_ahx_set(d, nc, Ap, Fbb, z, st);                                             // Ap^* Ap zs
        launch_zsub(nc, xs, z, z, st);                                                            // rho
        ls_packed_factor_solve(ctx->ws, ph, img, tabs, z, xbar, st);                              // G^{-1} rho
        launch_zaxpy_norms(nc, xbar, zs, nullptr, nullptr, st);
    }
    MDP_HIP(hipMemcpyAsync(z, zs, (size_t)nc * sizeof(double2), hipMemcpyDeviceToDevice, st));
    launch_scale_cols(z, 1, nc, 1, norms, 1, st);
    // (4) Fbb = Qbar z = Ap zs; r = Fbar - Qbar x = Fbar - Ap (D x)
    launch_packed_axpy(d, n_sub, ph.max_m, Ap, zs, one, nullptr, Fbb, nullptr, nullptr, st);
    MDP_HIP(hipMemcpyAsync(xs, x, (size_t)nc * sizeof(double2), hipMemcpyDeviceToDevice, st));
    launch_scale_cols(xs, 1, nc, 1, norms, 0, st);
    launch_packed_axpy(d, n_sub, ph.max_m, Ap, xs, mone, F, r, nullptr, nullptr, st);
    // (5) boundary-data gradient
    double2* dg = at(b_dg);
    launch_data_grad(nk, reinterpret_cast<const double2* const*>(T(o_kq)), reinterpret_cast<const int*>(T(o_krows)),
                     reinterpret_cast<const int*>(T(o_kcol)), reinterpret_cast<const long*>(T(o_kroff)),
                     reinterpret_cast<const int*>(T(o_keidx)), reinterpret_cast<const double*>(T(o_kdiv)), cbar, Fbb,
                     dg, st);
    // (6) the two density sets side by side: [c | cz], cz = K z (no known part)
    double2* cc = at(b_cc);
    double2* zero = at(b_zero);
    MDP_HIP(hipMemcpyAsync(cc, c_full, (size_t)nce * sizeof(double2), hipMemcpyDeviceToDevice, st));
    MDP_HIP(hipMemsetAsync(zero, 0, (size_t)nce * sizeof(double2), st));
    launch_expand_coeffs(nce, esrc, ecoef, zero, z, cc + nce, st);
    // (7) k^2 of every subdomain, both densities of all subdomains in the same launches:
    //     w = E c, dw = dE c; v = A^{-1}(L w|M+); h = -dA v + (dL w + L dw)|M+; y = A^{-1} h
    double* W = reinterpret_cast<double*>(at(b_w));
    double* DW = reinterpret_cast<double*>(at(b_dw));
    double* V = reinterpret_cast<double*>(at(b_v));
    double* H = reinterpret_cast<double*>(at(b_h));
    double* Y = reinterpret_cast<double*>(at(b_y));
    double* dE = reinterpret_cast<double*>(at(b_dE));
    double2* kres = at(b_k);
    const StencilCoef dsc{2.0 / 3.0, 1.0 / 12.0, 0.0};
    MDP_HIP(hipMemsetAsync(dE, 0, (size_t)de_off[n_sub] * sizeof(double), st));
    MDP_HIP(hipMemsetAsync(W, 0, (size_t)2 * gtot * sizeof(double2), st));
    MDP_HIP(hipMemsetAsync(DW, 0, (size_t)2 * gtot * sizeof(double2), st));
    for (int i = 0; i < n_sub; ++i)
        launch_extension(P[i]->gside, P[i]->grho, P[i]->gt, P[i]->gslen, P[i]->g.n_gamma, P[i]->k, M, dE + de_off[i],
                         st, 1);
    auto jvp_jobs = [&](Src kind, const double* grid, double* out, bool density_dE) {
        std::vector<SolveJob> jobs;
        std::vector<const APPlan*> jp;
        for (int q = 0; q < n_sub; ++q) {
            const int i = ord[q];
            const mdp_projector* Pi = P[i];
            const Geometry& G = Pi->g;
            const APPlan& plan = *plans[i];
            SolveJob J{};
            J.src.kind = kind;
            J.src.grid = grid;
            J.src.goff = d_g2 + 2 * q;
            J.src.m_lo = G.m_lo; J.src.m_hi = G.m_hi; J.src.q_lo = G.q_lo; J.src.q_hi = G.q_hi;
            J.sc = plan.sc;
            J.f = plan.f;
            J.bd = Band{0, plan.n + 1};
            J.b0 = 2 * q;
            J.R = 2;
            J.fac = plan.fac64.as<double>();
            J.colc = plan.colc64.as<double>();
            J.E = density_dE ? dE + de_off[i] : Pi->E.as<double>();
            J.ng = G.n_gamma;
            J.ncol = ncol;
            J.gm = Pi->gm; J.gq = Pi->gq; J.gside = Pi->gside;
            J.cidx = d_c2 + 2 * q;
            J.out = out;
            J.ooff = d_g2 + 2 * q;
            jobs.push_back(J);
            jp.push_back(&plan);
        }
        return std::make_pair(jobs, jp);
    };
    // densities w (E) and dw (dE) of both coefficient sets
    for (int which = 0; which < 2; ++which) {
        auto jj = jvp_jobs(Src::STENCIL_GRID, nullptr, nullptr, which == 1);
        HostBlob jb;
        const size_t o_j = jb.put(jj.first);
        ensure(cw.jobs, jb.size());
        ctx->ws.stage.copy(cw.jobs.p, jb, st);
        launch_extend_density_jobs(reinterpret_cast<const SolveJob*>(cw.jobs.as<char>() + o_j), n_sub, 2 * n_sub,
                                   max_ng, which == 0 ? W : DW, reinterpret_cast<const double*>(cc), st);
    }
    {
        auto jj = jvp_jobs(Src::STENCIL_GRID, W, V, false);
        batched_band_solve(ctx, jj.first, jj.second, nullptr, st);
    }
    for (int i = 0; i < n_sub; ++i) {
        const Geometry& G = P[i]->g;
        launch_jvp_rhs(V, W, DW, d_g2s + 2 * i, 2, G.n, G.h, P[i]->k, plans[i]->sc, dsc, G.m_lo, G.m_hi, G.q_lo,
                       G.q_hi, H, st);
    }
    {
        auto jj = jvp_jobs(Src::GRID_ALL, H, Y, false);
        batched_band_solve(ctx, jj.first, jj.second, nullptr, st);
    }
    for (int i = 0; i < n_sub; ++i) {
        const Geometry& G = P[i]->g;
        const int r0 = r_first[i], rc = r_first[i + 1] - r_first[i];
        launch_kappa_dot(Y + 2 * goff2[2 * i], Y + 2 * goff2[2 * i + 1], DW + 2 * goff2[2 * i], P[i]->gm, P[i]->gq,
                         G.n_gamma, G.n, Fbb, r, row_off[i], reinterpret_cast<const long*>(T(o_rnode)) + r0,
                         reinterpret_cast<const double*>(T(o_rval)) + 2 * r0, rc, kres + i, st);
    }
    // (8) results to the host
    std::vector<double2> hk(n_sub), hd(nk);
    MDP_HIP(hipMemcpyAsync(hk.data(), kres, (size_t)n_sub * sizeof(double2), hipMemcpyDeviceToHost, st));
    if (nk) MDP_HIP(hipMemcpyAsync(hd.data(), dg, (size_t)nk * sizeof(double2), hipMemcpyDeviceToHost, st));
    MDP_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < n_sub; ++i) ga.grad_k2[i] = hk[i].x;
    std::memset(ga.grad_d, 0, sizeof(mdp_c128) * (size_t)n_sub * 4 * M);
    for (int t = 0; t < nk; ++t) ga.grad_d[kout[t]] = mdp_c128{hd[t].x, hd[t].y};
}

}  // namespace

int mdp_solve_interface(mdp_ctx* ctx, int n_sub, const mdp_subdomain* subs, const mdp_projector* const* P,
                        const mdp_side* sides, int m_star, const mdp_source* sources, void* stream, mdp_c128* c_out,
                        double* rel_residual_out, double* cond_estimate_out) {
    return solve_interface_impl(ctx, n_sub, subs, P, sides, m_star, sources, stream, c_out, rel_residual_out,
                                cond_estimate_out, nullptr);
}

int mdp_dd_gradient(mdp_ctx* ctx, int n_sub, const mdp_subdomain* subs, const mdp_projector* const* P,
                    const mdp_side* sides, int m_star, int n_rcv, const int* rcv_sub, const int* rcv_node,
                    const mdp_c128* ubar, void* stream, double* grad_k2, mdp_c128* grad_d) {
    if (!ctx) return fail(nullptr, MDP_ERR_ARG, "ctx is NULL");
    if (n_sub < 1 || !grad_k2 || !grad_d || n_rcv < 0 || (n_rcv > 0 && (!rcv_sub || !rcv_node || !ubar)))
        return fail(ctx, MDP_ERR_ARG, "null or empty gradient arguments");
    if (!P || !subs || !sides) return fail(ctx, MDP_ERR_ARG, "null or empty gradient arguments");
    // everything the reverse pass checks, before the forward solve queues any work
    for (int i = 0; i < n_sub; ++i) {
        if (!P[i]) return fail(ctx, MDP_ERR_ARG, "null projector");
        if (P[i]->precision != MDP_C128) return fail(ctx, MDP_ERR_ARG, "gradient: projectors must be complex128");
    }
    for (int t = 0; t < n_rcv; ++t) {
        if (rcv_sub[t] < 0 || rcv_sub[t] >= n_sub) return fail(ctx, MDP_ERR_ARG, "receiver subdomain out of range");
        const int n = P[rcv_sub[t]]->g.n;
        if (rcv_node[t] < 0 || rcv_node[t] >= (n + 1) * (n + 1))
            return fail(ctx, MDP_ERR_ARG, "receiver node out of range");
        if (!std::isfinite(ubar[t].re) || !std::isfinite(ubar[t].im))
            return fail(ctx, MDP_ERR_NONFINITE, "non-finite receiver weight");
    }
    GradArgs ga{n_rcv, rcv_sub, rcv_node, ubar, grad_k2, grad_d};
    int rc = MDP_OK;
    {
        DevBuf c;
        try {
            c.alloc((size_t)n_sub * 8 * std::max(m_star, 1) * sizeof(mdp_c128));
        } catch (const Error& e) {
            return fail(ctx, e.code, e.what());
        }
        rc = solve_interface_impl(ctx, n_sub, subs, P, sides, m_star, nullptr, stream, c.as<mdp_c128>(), nullptr,
                                  nullptr, &ga);
        (void)hipStreamSynchronize((hipStream_t)stream);
    }
    return rc;
}

// ---------------------------------------------------------------------------- step 3
int mdp_reconstruct(mdp_ctx* ctx, int n_sub, const mdp_projector* const* P, const mdp_c128* c,
                    const mdp_source* sources, void* stream, mdp_c128* u_out) {
    if (!ctx) return fail(nullptr, MDP_ERR_ARG, "ctx is NULL");
    return guarded(ctx, [&]() -> int {
        if (n_sub < 1 || !P || !c || !u_out) throw Error(MDP_ERR_ARG, "null or empty arguments");
        hipStream_t st = (hipStream_t)stream;
        std::vector<long> off(n_sub + 1, 0);
        for (int i = 0; i < n_sub; ++i) {
            if (!P[i]) throw Error(MDP_ERR_ARG, "null projector");
            off[i + 1] = off[i] + (long)(P[i]->g.n + 1) * (P[i]->g.n + 1);
        }
        // group subdomains by projector: one batched solve per distinct projector
        std::vector<std::vector<int>> groups;
        std::vector<bool> done(n_sub, false);
        for (int i = 0; i < n_sub; ++i) {
            if (done[i]) continue;
            std::vector<int> grp;
            for (int j = i; j < n_sub; ++j)
                if (P[j] == P[i]) { grp.push_back(j); done[j] = true; }
            groups.push_back(std::move(grp));
        }
        // groups of one n next to each other (the batched route's sine GEMMs go per n)
        std::stable_sort(groups.begin(), groups.end(), [&](const std::vector<int>& a, const std::vector<int>& b) {
            return P[a[0]]->g.n < P[b[0]]->g.n;
        });
        bool any_source = false;
        for (int i = 0; i < n_sub; ++i) any_source = any_source || (sources && sources[i].f);
        // several distinct projectors, no source: every group's solve in the same launches, in FP64
        // whatever the projectors' precision (one AP solve per subdomain; the precision of a build
        // is that of its 8M* solves per projector)
        const bool batched = groups.size() > 1 && !any_source;
        // per batch entry: the subdomain (its coefficients in c), its grid's offset in u_out and its source
        std::vector<int> cidx;
        std::vector<long> goff;
        std::vector<const double*> sf, sjet;
        for (const auto& grp : groups)
            for (int i : grp) {
                cidx.push_back(i);
                goff.push_back(off[i]);
                const bool has = sources && sources[i].f;
                if (has && !sources[i].jet) throw Error(MDP_ERR_ARG, "source without its boundary jet");
                sf.push_back(has ? reinterpret_cast<const double*>(sources[i].f) : nullptr);
                sjet.push_back(has ? reinterpret_cast<const double*>(sources[i].jet) : nullptr);
            }
        CallScope scope(ctx, st);
        HostBlob blob;
        const size_t o_cidx = blob.put(cidx), o_goff = blob.put(goff), o_sf = blob.put(sf), o_sjet = blob.put(sjet);
        const char* img = ctx->ws.stage.upload(blob, st);
        // u_out holds the density w (zero off gamma), then u = w - G(L w |M+) in place
        MDP_HIP(hipMemsetAsync(u_out, 0, (size_t)off[n_sub] * sizeof(mdp_c128), st));
        double* uo = reinterpret_cast<double*>(u_out);
        if (batched) {
            std::vector<SolveJob> jobs;
            std::vector<const APPlan*> plans;
            size_t e = 0;
            int total = 0, max_ng = 0;
            for (const auto& grp : groups) {
                const mdp_projector* Pi = P[grp[0]];
                const Geometry& G = Pi->g;
                const APPlan& plan = get_plan(ctx, G.n, G.h, Pi->k);
                SolveJob J{};
                J.src.kind = Src::STENCIL_GRID;
                J.src.grid = uo;
                J.src.goff = reinterpret_cast<const long*>(img + o_goff) + e;
                J.src.m_lo = G.m_lo; J.src.m_hi = G.m_hi; J.src.q_lo = G.q_lo; J.src.q_hi = G.q_hi;
                J.sc = plan.sc;
                J.f = plan.f;
                J.bd = box_band(plan, G);
                J.b0 = total;
                J.R = (int)grp.size();
                J.fac = plan.fac64.as<double>();
                J.colc = plan.colc64.as<double>();
                J.E = Pi->E.as<double>();
                J.ng = G.n_gamma;
                J.ncol = 8 * Pi->m_star;
                J.gm = Pi->gm; J.gq = Pi->gq; J.gside = Pi->gside;
                J.cidx = reinterpret_cast<const int*>(img + o_cidx) + e;
                jobs.push_back(J);
                plans.push_back(&plan);
                total += J.R;
                e += grp.size();
                max_ng = std::max(max_ng, G.n_gamma);
            }
            // the densities first (the table goes up with the solve's; the density step reads the same fields)
            {
                HostBlob jb;
                const size_t o_j = jb.put(jobs);
                ensure(ctx->ws.cw.jobs, jb.size());
                ctx->ws.stage.copy(ctx->ws.cw.jobs.p, jb, st);
                launch_extend_density_jobs(reinterpret_cast<const SolveJob*>(ctx->ws.cw.jobs.as<char>() + o_j),
                                           (int)jobs.size(), total, max_ng, uo, reinterpret_cast<const double*>(c), st);
            }
            batched_band_solve(ctx, jobs, plans, uo, st);
            return MDP_OK;
        }
        size_t e0 = 0;
        for (const auto& grp : groups) {
            const mdp_projector* Pi = P[grp[0]];
            const Geometry& G = Pi->g;
            const int n = G.n, ng = G.n_gamma, ncol = 8 * Pi->m_star, R = (int)grp.size();
            APPlan& plan = get_plan(ctx, n, G.h, Pi->k);
            const int* ci = reinterpret_cast<const int*>(img + o_cidx) + e0;
            const long* go = reinterpret_cast<const long*>(img + o_goff) + e0;
            launch_extend_density(Pi->E.as<double>(), ng, ncol, reinterpret_cast<const double*>(c), ci, R, Pi->gm,
                                  Pi->gq, Pi->gside, n, uo, 0, go, st);
            // xi_gamma also holds Ex^(I) f where there is a source (eq. extension_split)
            bool any_src = false;
            for (size_t e = e0; e < e0 + grp.size(); ++e) any_src = any_src || sf[e];
            const double* const* fs = reinterpret_cast<const double* const*>(img + o_sf) + e0;
            if (any_src)
                launch_source_extension(Pi->grho, Pi->gm, Pi->gq, ng, n, Pi->k,
                                        reinterpret_cast<const double* const*>(img + o_sjet) + e0, R, uo, go, true,
                                        st);
            const int chunk = chunk_size(plan, Pi->precision, ctx->ws_cap, R);
            prepare_ws(ctx, plan, Pi->precision, chunk);
            for (int r0 = 0; r0 < R; r0 += chunk) {
                const int Rc = std::min(chunk, R - r0);
                SrcDesc src{};
                src.kind = Src::STENCIL_GRID;
                src.grid = uo;
                src.goff = go + r0;
                src.fsrc = any_src ? fs + r0 : nullptr;   // right-hand side L w - B f (eq. potential_solution)
                src.m_lo = G.m_lo; src.m_hi = G.m_hi; src.q_lo = G.q_lo; src.q_hi = G.q_hi;
                const Fold f = plan.f;
                const int prec = Pi->precision;
                const Band rows = box_band(plan, G);
                solve_batch(plan, ctx->ws, prec, src, true, Rc, rows,
                            [&](const void* u, const float* du, Band bd) {
                                // u_out = w - G(L w |M+) on the band, in place (zero on the other rows)
                                ctx->ws.prof.run("unfold_grid", st, 0.0, (double)Rc * rows.nr * (n + 1) * 16.0 * 3.0,
                                                 [&] {
                                    if (prec == MDP_C128)
                                        launch_unfold_grid<double>((const double*)u, du, n, f, bd, rows, Rc, uo, 0, uo,
                                                                   0, go + r0, st);
                                    else
                                        launch_unfold_grid<float>((const float*)u, du, n, f, bd, rows, Rc, uo, 0, uo, 0,
                                                                  go + r0, st);
                                });
                            },
                            st);
            }
            e0 += grp.size();
        }
        return MDP_OK;
    });
}

// ---------------------------------------------------------------------------- G^(h)
int mdp_ap_solve(mdp_ctx* ctx, int n, double h, double k, int precision, int batch, const mdp_c128* g, mdp_c128* u,
                 void* stream) {
    if (!ctx) return fail(nullptr, MDP_ERR_ARG, "ctx is NULL");
    return guarded(ctx, [&]() -> int {
        if (batch < 0 || (batch > 0 && (!g || !u))) throw Error(MDP_ERR_ARG, "null grid pointers");
        if (!std::isfinite(k) || !(k > 0)) throw Error(MDP_ERR_NONFINITE, "k must be finite and > 0");
        check_precision(precision);
        APPlan& plan = get_plan(ctx, n, h, k);
        if (batch == 0) return MDP_OK;
        hipStream_t st = (hipStream_t)stream;
        const long npts = (long)(n + 1) * (n + 1);
        CallScope scope(ctx, st);
        const int chunk = chunk_size(plan, precision, ctx->ws_cap, batch);
        prepare_ws(ctx, plan, precision, chunk);
        for (int b0 = 0; b0 < batch; b0 += chunk) {
            const int R = std::min(chunk, batch - b0);
            SrcDesc src{};
            src.kind = Src::GRID;
            src.grid = reinterpret_cast<const double*>(g) + 2 * (size_t)b0 * npts;
            src.grid_stride = npts;
            double* out = reinterpret_cast<double*>(u) + 2 * (size_t)b0 * npts;
            const Fold f = plan.f;
            const Band all{0, n + 1};
            solve_batch(plan, ctx->ws, precision, src, true, R, all,
                        [&](const void* uu, const float* du, Band bd) {
                            if (precision == MDP_C128)
                                launch_unfold_grid<double>((const double*)uu, du, n, f, bd, all, R, nullptr, 0, out,
                                                           npts, nullptr, st);
                            else
                                launch_unfold_grid<float>((const float*)uu, du, n, f, bd, all, R, nullptr, 0, out,
                                                          npts, nullptr, st);
                        },
                        st);
        }
        return MDP_OK;
    });
}

// ---------------------------------------------------------------------------- G^(h) without allocation
int mdp_ap_solve_noalloc(mdp_ctx* ctx, int n, double h, double k, int precision, int batch, const mdp_c128* g,
                         mdp_c128* u, void* stream) {
    if (!ctx) return fail(nullptr, MDP_ERR_ARG, "ctx is NULL");
    return guarded(ctx, [&]() -> int {
        if (batch < 0 || (batch > 0 && (!g || !u))) throw Error(MDP_ERR_ARG, "null grid pointers");
        if (!std::isfinite(k) || !(k > 0)) throw Error(MDP_ERR_NONFINITE, "k must be finite and > 0");
        check_precision(precision);
        if (!ctx->scratch) throw Error(MDP_ERR_HIP, "the scratch array of this device was not resolved");
        // the plan must exist already: creating one allocates its device tables
        auto it = ctx->plans.find(PlanKey{n, h, k});
        if (it == ctx->plans.end())
            throw Error(MDP_ERR_ARG, "no plan for this (n, h, k) on the context: call mdp_ap_solve with the same "
                                     "n, h and k first (a batch of 0 creates it)");
        const APPlan& plan = *it->second;
        if (batch == 0) return MDP_OK;
        const size_t one = solve_scratch_bytes(plan, precision, 1);
        if (one > kNoAllocScratchBytes)
            throw Error(MDP_ERR_ARG, "n = " + std::to_string(n) + " needs " + std::to_string(one) +
                                         " bytes of scratch per right-hand side in this precision, more than the " +
                                         std::to_string(kNoAllocScratchBytes) + " bytes of the allocation-free solve");
        const int chunk = (int)std::min<size_t>((size_t)batch, kNoAllocScratchBytes / one);
        hipStream_t st = (hipStream_t)stream;
        const long npts = (long)(n + 1) * (n + 1);
        CallScope scope(ctx, st);
        for (int b0 = 0; b0 < batch; b0 += chunk) {   // chunks reuse the scratch in stream order
            const int R = std::min(chunk, batch - b0);
            SrcDesc src{};
            src.kind = Src::GRID;
            src.grid = reinterpret_cast<const double*>(g) + 2 * (size_t)b0 * npts;
            src.grid_stride = npts;
            double* out = reinterpret_cast<double*>(u) + 2 * (size_t)b0 * npts;
            const Fold f = plan.f;
            const Band all{0, n + 1};
            solve_batch_scratch(plan, precision, ctx->scratch, src, true, R,
                                [&](const void* uu, const float* du, Band bd) {
                                    if (precision == MDP_C128)
                                        launch_unfold_grid<double>((const double*)uu, du, n, f, bd, all, R, nullptr, 0,
                                                                   out, npts, nullptr, st);
                                    else
                                        launch_unfold_grid<float>((const float*)uu, du, n, f, bd, all, R, nullptr, 0,
                                                                  out, npts, nullptr, st);
                                },
                                st);
        }
        return MDP_OK;
    });
}

// ---------------------------------------------------------------------------- cache / profiling
int mdp_cache_clear(mdp_ctx* ctx) {
    if (!ctx) return MDP_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        // released buffers are reused only by later calls, in stream order after this context's work
        for (auto& kv : ctx->cache) mdp_projector_release(kv.second);
        ctx->cache.clear();
        return MDP_OK;
    });
}

int mdp_profile_enable(mdp_ctx* ctx, int enable) {
    if (!ctx) return MDP_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        MDP_HIP(hipDeviceSynchronize());
        ctx->ws.prof.reset();
        ctx->ws.prof.on = enable != 0;
        return MDP_OK;
    });
}

int mdp_profile_select(mdp_ctx* ctx, const char* classes) {
    if (!ctx) return MDP_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        ctx->ws.prof.only.clear();
        if (classes) {
            std::string all(classes), cur;
            for (char ch : all + ",") {
                if (ch == ',') {
                    if (!cur.empty()) ctx->ws.prof.only.push_back(cur);
                    cur.clear();
                } else if (ch != ' ') {
                    cur += ch;
                }
            }
        }
        return MDP_OK;
    });
}

int mdp_profile_report(mdp_ctx* ctx, char* buf, int buflen) {
    if (!ctx || !buf || buflen < 3) return MDP_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        MDP_HIP(hipDeviceSynchronize());
        struct Acc { int count = 0; double ms = 0, flops = 0, bytes = 0; };
        std::map<std::string, Acc> acc;
        for (auto& r : ctx->ws.prof.recs) {
            float ms = 0.f;
            MDP_HIP(hipEventElapsedTime(&ms, r.a, r.b));
            Acc& a = acc[r.name];
            a.count += 1;
            a.ms += ms;
            a.flops += r.flops;
            a.bytes += r.bytes;
        }
        std::string out = "{";
        bool first = true;
        char tmp[512];
        for (auto& kv : acc) {
            std::snprintf(tmp, sizeof tmp, "%s\"%s\": {\"count\": %d, \"total_ms\": %.6f, \"flops\": %.6e, \"bytes\": %.6e}",
                          first ? "" : ", ", kv.first.c_str(), kv.second.count, kv.second.ms, kv.second.flops,
                          kv.second.bytes);
            out += tmp;
            first = false;
        }
        out += "}";
        if ((int)out.size() + 1 > buflen) throw Error(MDP_ERR_ARG, "profile report buffer too small");
        std::memcpy(buf, out.c_str(), out.size() + 1);
        return MDP_OK;
    });
}

// ---------------------------------------------------------------------------- Chebyshev helpers
int mdp_cheb_points(int m_star, double* t) {
    if (m_star < 1 || !t) return MDP_ERR_ARG;
    for (int i = 0; i < m_star; ++i) t[i] = std::cos(M_PI * (i + 0.5) / m_star);
    return MDP_OK;
}

int mdp_cheb_coeffs(int m_star, const mdp_c128* samples, mdp_c128* d) {
    if (m_star < 1 || !samples || !d) return MDP_ERR_ARG;
    for (int j = 0; j < m_star; ++j) {
        double re = 0.0, im = 0.0;
        for (int i = 0; i < m_star; ++i) {
            // T_j(cos theta_i) = cos(j theta_i), theta_i = pi (i + 1/2)/M*
            double tj = std::cos(j * M_PI * (i + 0.5) / m_star);
            re += samples[i].re * tj;
            im += samples[i].im * tj;
        }
        double w = (j == 0 ? 1.0 : 2.0) / m_star;
        d[j].re = re * w;
        d[j].im = im * w;
    }
    return MDP_OK;
}

}  // extern "C"
