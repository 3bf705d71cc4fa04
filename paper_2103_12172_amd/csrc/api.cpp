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

struct mdp_projector {
    std::atomic<int> refs{1};
    int device = 0;
    Geometry g;
    double k = 0.0;
    int m_star = 0, precision = 0;
    DevBuf Q;      // n_gamma x 8M* complex, column-major
    DevBuf E;      // n_gamma x 8M* real
    DevBuf gidx;   // (n+1)^2 node -> gamma index
    DevBuf meta;   // gamma nodes: gm, gq, side (int), then rho, t, side length (double)
    std::vector<char> meta_host;  // host copy the upload reads from
    const int *gm = nullptr, *gq = nullptr, *gside = nullptr;
    const double *grho = nullptr, *gt = nullptr, *gslen = nullptr;
};

namespace {

using PlanKey = std::tuple<int, double, double>;
using ProjKey = std::tuple<double, double, int, double, int, int>;

}  // namespace

struct mdp_ctx {
    int device = 0;
    std::string err;
    std::map<PlanKey, std::unique_ptr<APPlan>> plans;
    std::map<ProjKey, mdp_projector*> cache;
    Workspace ws;
    size_t ws_cap = (size_t)24 << 30;
    int projector_path = MDP_PATH_AUTO;
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
void end_call(mdp_ctx* ctx, hipStream_t st) {
    MDP_HIP(hipEventRecord(ctx->last, st));
    ctx->last_stream = st;
    ctx->have_last = true;
}

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


// Q by the support-in / gamma-out route (FP64): per chunk of columns, the
// ring RHS and the folded special rows, their sine GEMM, the fused sweep with
// the gamma-row reductions, the inverse GEMM of the four full gamma rows and
// the gather into Q.
void build_q_fused(mdp_ctx* ctx, const APPlan& plan, mdp_projector* P, hipStream_t st) {
    const Geometry& G = P->g;
    const Fold& f = plan.f;
    const int n = G.n, W = f.W, ng = G.n_gamma, ncol = 8 * P->m_star;
    const int nseg = fused_segments(n), rows_pad = nseg * FUSED_K, nb = W / 64;
    const size_t per_a = (size_t)nseg * 2 * W + (size_t)nb * rows_pad * 4;      // ckpt + thin
    const size_t per_b = (size_t)(n + 1) * 4 + (size_t)(4 + 4 + 8 + 8) * W;       // gc, spec, spec_hat, xs, us
    size_t chunk = ctx->ws_cap / ((per_a + per_b) * sizeof(double));
    chunk = std::max<size_t>(1, std::min<size_t>({chunk, (size_t)65535, (size_t)ncol}));
    const size_t need_a = chunk * per_a * sizeof(double), need_b = chunk * per_b * sizeof(double);
    if (need_a > ctx->ws.a.bytes || need_b > ctx->ws.b.bytes) {
        MDP_HIP(hipDeviceSynchronize());
        ctx->ws.a.reserve(need_a);
        ctx->ws.b.reserve(need_b);
    }
    Profiler& pr = ctx->ws.prof;
    const double elems_useful = (double)(n + 1) * (n - 1);
    const double gemm_row_flops = 2.0 * ((double)f.p * f.p + (double)(f.p - 1) * (f.p - 1));
    const int box_rows = G.m_hi - G.m_lo + 3;
    for (int col0 = 0; col0 < ncol; col0 += (int)chunk) {
        const int R = std::min((int)chunk, ncol - col0);
        double* ckpt = ctx->ws.a.as<double>();
        double* thin = ckpt + (size_t)R * nseg * 2 * W;
        double* gc = ctx->ws.b.as<double>();
        double* spec = gc + (size_t)R * (n + 1) * 4;
        double* spec_hat = spec + (size_t)R * 4 * W;
        double* xs = spec_hat + (size_t)R * 4 * W;
        double* us = xs + (size_t)R * 8 * W;
        SrcDesc src{};
        src.kind = Src::STENCIL_E;
        src.E = P->E.as<double>();
        src.ldE = ng;
        src.col0 = col0;
        src.gidx = P->gidx.as<int>();
        src.m_lo = G.m_lo; src.m_hi = G.m_hi; src.q_lo = G.q_lo; src.q_hi = G.q_hi;
        pr.run("fold_ring", st, 0.0, (double)R * ((n + 1) * 4.0 + 4.0 * (n - 1)) * 8.0,
               [&] { launch_fold_ring(src, n, f, plan.sc, R, gc, spec, st); });
        pr.run("gemm_sine_f64", st, 4.0 * R * gemm_row_flops, 2.0 * 4.0 * R * (n - 1) * 8.0,
               [&] { launch_gemm_bd<double>(spec, plan.Sf64.as<double>(), spec_hat, (long)R * 4, f, st); });
        // algorithmic flops per column element: forward elimination 7, back substitution 10, ring transform 3
        // (box rows), synthesis products and sums 8 (gamma rows)
        pr.run("ap_fused_f64", st,
               (double)R * (elems_useful * 17.0 + (double)(G.m_hi - G.m_lo + 1) * (n - 1) * 3.0 +
                            (double)box_rows * (n - 1) * 8.0),
               (double)R * ((G.m_hi - G.m_lo + 1) * 32.0 + 4.0 * (n - 1) * 8.0 + 8.0 * (n - 1) * 8.0 +
                            (double)box_rows * 4 * 8.0),
               [&] {
                   launch_proj_fused(gc, spec_hat, plan.Sf64.as<double>(), plan.Si64.as<double>(), f, G.m_lo,
                                     G.m_hi, G.q_lo, G.q_hi, plan.lf64.as<double>(), plan.rf64.as<double>(),
                                     plan.colc64.as<double>(), ckpt, xs, thin, R, st);
               });
        pr.run("gemm_sine_f64", st, 8.0 * R * gemm_row_flops, 2.0 * 8.0 * R * (n - 1) * 8.0,
               [&] { launch_gemm_bd<double>(xs, plan.Si64.as<double>(), us, (long)R * 8, f, st); });
        pr.run("gather_q", st, 0.0, (double)ng * R * 16.0 * 2.0, [&] {
            launch_gather_q_fused(us, thin, f, G.m_lo, G.m_hi, G.q_lo, G.q_hi, P->gm, P->gq, ng,
                                  R, P->Q.as<double>(), ng, col0, st);
        });
    }
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

const char* mdp_last_error(const mdp_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

int mdp_build_projector(mdp_ctx* ctx, const mdp_subdomain* sd, int m_star, int precision, void* stream,
                        mdp_projector** out) {
    if (!ctx) return fail(nullptr, MDP_ERR_ARG, "ctx is NULL");
    return guarded(ctx, [&]() -> int {
        if (!sd || !out) throw Error(MDP_ERR_ARG, "null subdomain or output pointer");
        *out = nullptr;
        if (m_star < 1) throw Error(MDP_ERR_ARG, "M* must be >= 1");
        check_precision(precision);
        if (!std::isfinite(sd->k) || !(sd->k > 0)) throw Error(MDP_ERR_NONFINITE, "k must be finite and > 0");
        ProjKey key{sd->lx, sd->ly, sd->n, sd->k, m_star, precision};
        auto it = ctx->cache.find(key);
        if (it != ctx->cache.end()) {
            it->second->refs.fetch_add(1);
            *out = it->second;
            return MDP_OK;
        }
        hipStream_t st = (hipStream_t)stream;
        Geometry g = make_geometry(sd->x0, sd->y0, sd->lx, sd->ly, sd->n);
        APPlan& plan = get_plan(ctx, g.n, g.h, sd->k);
        std::unique_ptr<mdp_projector> P(new mdp_projector);
        P->device = ctx->device;
        P->k = sd->k;
        P->m_star = m_star;
        P->precision = precision;
        const int ng = g.n_gamma, ncol = 8 * m_star;
        begin_call(ctx, st);
        // gamma node lists in one upload; E and the node -> gamma map are built on the device
        const size_t ints = ((3 * (size_t)ng + 1) / 2) * 2, meta_bytes = ints * sizeof(int) + 3 * (size_t)ng * sizeof(double);
        P->meta_host.assign(meta_bytes, 0);
        int* hi = reinterpret_cast<int*>(P->meta_host.data());
        double* hd = reinterpret_cast<double*>(hi + ints);
        std::copy(g.gm.begin(), g.gm.end(), hi);
        std::copy(g.gq.begin(), g.gq.end(), hi + ng);
        std::copy(g.side.begin(), g.side.end(), hi + 2 * ng);
        std::copy(g.rho.begin(), g.rho.end(), hd);
        std::copy(g.t.begin(), g.t.end(), hd + ng);
        std::copy(g.slen.begin(), g.slen.end(), hd + 2 * ng);
        P->meta.alloc(meta_bytes);
        MDP_HIP(hipMemcpyAsync(P->meta.p, P->meta_host.data(), meta_bytes, hipMemcpyHostToDevice, st));
        const int* di = P->meta.as<int>();
        const double* dd = reinterpret_cast<const double*>(di + ints);
        P->gm = di;
        P->gq = di + ng;
        P->gside = di + 2 * ng;
        P->grho = dd;
        P->gt = dd + ng;
        P->gslen = dd + 2 * ng;
        P->E.alloc((size_t)ng * ncol * sizeof(double));
        MDP_HIP(hipMemsetAsync(P->E.p, 0, (size_t)ng * ncol * sizeof(double), st));
        launch_extension(P->gside, P->grho, P->gt, P->gslen, ng, sd->k, m_star, P->E.as<double>(), st);
        const size_t nodes = (size_t)(g.n + 1) * (g.n + 1);
        P->gidx.alloc(nodes * sizeof(int));
        MDP_HIP(hipMemsetAsync(P->gidx.p, 0xff, nodes * sizeof(int), st));   // -1 everywhere
        launch_gamma_index(P->gm, P->gq, ng, g.n, P->gidx.as<int>(), st);
        P->Q.alloc((size_t)ng * ncol * 2 * sizeof(double));
        P->g = std::move(g);
        const Geometry& G = P->g;

        if (precision == MDP_C128 && ctx->projector_path == MDP_PATH_AUTO &&
            fused_projector_supported(plan.f, G.m_lo, G.m_hi, G.q_lo, G.q_hi)) {
            build_q_fused(ctx, plan, P.get(), st);
            end_call(ctx, st);
            mdp_projector* raw = P.release();
            raw->refs.store(2);
            ctx->cache[key] = raw;
            *out = raw;
            return MDP_OK;
        }
        const int chunk = chunk_size(plan, precision, ctx->ws_cap, ncol);
        prepare_ws(ctx, plan, precision, chunk);
        for (int col0 = 0; col0 < ncol; col0 += chunk) {
            const int R = std::min(chunk, ncol - col0);
            SrcDesc src{};
            src.kind = Src::STENCIL_E;
            src.E = P->E.as<double>();
            src.ldE = ng;
            src.col0 = col0;
            src.gidx = P->gidx.as<int>();
            src.m_lo = G.m_lo; src.m_hi = G.m_hi; src.q_lo = G.q_lo; src.q_hi = G.q_hi;
            double* Qd = P->Q.as<double>();
            const int* gmd = P->gm;
            const int* gqd = P->gq;
            const int n = G.n;
            const Fold f = plan.f;
            solve_batch(plan, ctx->ws, precision, src, false, R,
                        [&](const void* u, const float* du) {
                            ctx->ws.prof.run("gather_q", st, 0.0, (double)ng * R * 16.0 * 2.0, [&] {
                                if (precision == MDP_C128)
                                    launch_gather_q<double>((const double*)u, du, n, f, gmd, gqd, ng, R, Qd, ng, col0,
                                                            st);
                                else
                                    launch_gather_q<float>((const float*)u, du, n, f, gmd, gqd, ng, R, Qd, ng, col0,
                                                           st);
                            });
                        },
                        st);
        }
        end_call(ctx, st);
        mdp_projector* raw = P.release();
        raw->refs.store(2);  // one for the cache, one for the caller
        ctx->cache[key] = raw;
        *out = raw;
        return MDP_OK;
    });
}

int mdp_projector_info(const mdp_projector* P, int* n_gamma, const int** gamma_mq, const mdp_c128** q_dev) {
    if (!P) return MDP_ERR_ARG;
    if (n_gamma) *n_gamma = P->g.n_gamma;
    if (gamma_mq) *gamma_mq = P->g.gmq.data();
    if (q_dev) *q_dev = P->Q.as<const mdp_c128>();
    return MDP_OK;
}

void mdp_projector_release(mdp_projector* P) {
    if (!P) return;
    if (P->refs.fetch_sub(1) == 1) {
        (void)hipSetDevice(P->device);
        (void)hipDeviceSynchronize();
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

int mdp_solve_interface(mdp_ctx* ctx, int n_sub, const mdp_subdomain* subs, const mdp_projector* const* P,
                        const mdp_side* sides, int m_star, void* stream, mdp_c128* c_out, double* rel_residual_out,
                        double* cond_estimate_out) {
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
        std::vector<int> row_off(n_sub + 1, 0);
        for (int i = 0; i < n_sub; ++i) row_off[i + 1] = row_off[i] + P[i]->g.n_gamma;
        const int m = row_off[n_sub];
        if (m < ncol) throw Error(MDP_ERR_ARG, "fewer gamma rows than unknowns");
        // column map per (subdomain, Qbar column)
        std::vector<int4> colmap((size_t)n_sub * ncol, int4{-1, -1, 0, 0});
        std::vector<double2> coefs((size_t)n_sub * ncol * 2, double2{0.0, 0.0});
        for (size_t b = 0; b < blocks.size(); ++b) {
            for (const Contrib& c : blocks[b].c) {
                for (int j = 0; j < M; ++j) {
                    const size_t idx = (size_t)c.sub * ncol + b * M + j;
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
        begin_call(ctx, st);
        std::vector<const double2*> qsrc(n_sub);
        std::vector<int> qld(n_sub);
        for (int i = 0; i < n_sub; ++i) { qsrc[i] = P[i]->Q.as<const double2>(); qld[i] = P[i]->g.n_gamma; }
        CallWork& cw = ctx->ws.cw;
        DevBuf &d_qsrc = cw.qsrc, &d_qld = cw.qld, &d_roff = cw.roff, &d_cmap = cw.cmap, &d_coef = cw.coef,
               &d_kcol = cw.kcol, &d_kval = cw.kval, &d_koff = cw.koff, &F = cw.F, &x = cw.x;
        upload_ws(d_qsrc, qsrc, st);
        upload_ws(d_qld, qld, st);
        upload_ws(d_roff, row_off, st);
        upload_ws(d_cmap, colmap, st);
        upload_ws(d_coef, coefs, st);
        upload_ws(d_kcol, kcol, st);
        upload_ws(d_kval, kval, st);
        upload_ws(d_koff, koff, st);
        ensure(F, (size_t)m * sizeof(double2));
        ensure(x, (size_t)ncol * sizeof(double2));
        launch_known_rhs(d_qsrc.as<const double2* const>(), d_qld.as<int>(), n_sub, d_roff.as<int>(), m,
                         d_kcol.as<int>(), d_kval.as<double2>(), d_koff.as<int>(), F.as<double2>(), st);
        // block-sparse description: subdomain i's rows touch only the unknown blocks with a contribution from i
        PackedHost ph;
        ph.n_sub = n_sub;
        ph.nc = ncol;
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
                    ph.pc_gcol.push_back((int)b * M + j);
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
        LSResult r;
        {
            // the whole least-squares solve as one profiled span (it synchronises internally)
            Profiler& pr = ctx->ws.prof;
            hipEvent_t a = nullptr, b = nullptr;
            const bool span = pr.wants("interface_ls");
            if (span) { a = pr.get(); b = pr.get(); MDP_HIP(hipEventRecord(a, st)); }
            // algorithmic work of the least squares: a Householder QR of the m x ncol matrix
            const double qr_flops = 8.0 * ((double)m * ncol * ncol - (double)ncol * ncol * ncol / 3.0);
            bool fallback = false;
            r = ls_solve_packed(ctx->ws, ph, F.as<double2>(), x.as<double2>(), cond_estimate_out != nullptr, st,
                                &fallback);
            if (fallback) {
                // dense Cholesky-QR passes on the assembled matrix
                DevBuf Qbar((size_t)m * ncol * sizeof(double2));
                launch_assemble_qbar(d_qsrc.as<const double2* const>(), d_qld.as<int>(), n_sub, d_roff.as<int>(), m,
                                     d_cmap.as<int4>(), d_coef.as<double2>(), ncol, Qbar.as<double2>(), m, st);
                r = ls_solve(ctx->ws, Qbar.as<double2>(), F.as<double2>(), m, ncol, x.as<double2>(),
                             cond_estimate_out != nullptr, st);
                MDP_HIP(hipStreamSynchronize(st));
            }
            if (span) {
                MDP_HIP(hipEventRecord(b, st));
                pr.recs.push_back({"interface_ls", a, b, qr_flops, (double)m * ncol * 16.0});
            }
        }
        // expand the unknowns to the full coefficient vectors (column order of Q)
        std::vector<double2> hx(ncol);
        MDP_HIP(hipMemcpyAsync(hx.data(), x.p, ncol * sizeof(double2), hipMemcpyDeviceToHost, st));
        MDP_HIP(hipStreamSynchronize(st));
        std::vector<double2> c((size_t)n_sub * 8 * M, double2{0.0, 0.0});
        auto C = [&](int i, int kind, int s, int j) -> double2& { return c[(size_t)i * 8 * M + kind * 4 * M + s * M + j]; };
        for (size_t b = 0; b < blocks.size(); ++b) {
            const Block& B = blocks[b];
            for (int j = 0; j < M; ++j) {
                double2 v = hx[b * M + j];
                if (B.type == 2) { C(B.c[0].sub, 0, B.c[0].side, j) = v; continue; }
                for (const Contrib& ct : B.c) {
                    double2 w = ct.coef;
                    C(ct.sub, ct.kind, ct.side, j) = double2{w.x * v.x - w.y * v.y, w.x * v.y + w.y * v.x};
                }
            }
        }
        for (int i = 0; i < n_sub; ++i)
            for (int s = 0; s < 4; ++s) {
                const mdp_side& sd_ = sides[4 * i + s];
                if (sd_.kind != 0) continue;
                const double a = sd_.alpha, b = sd_.beta;
                for (int j = 0; j < M; ++j) {
                    double2 d{sd_.d[j].re, sd_.d[j].im};
                    if (b == 0.0) C(i, 0, s, j) = double2{d.x / a, d.y / a};
                    else if (a == 0.0) C(i, 1, s, j) = double2{d.x / b, d.y / b};
                    else {
                        double2 c0 = C(i, 0, s, j);
                        C(i, 1, s, j) = double2{d.x / b - (a / b) * c0.x, d.y / b - (a / b) * c0.y};
                    }
                }
            }
        MDP_HIP(hipMemcpyAsync(c_out, c.data(), c.size() * sizeof(double2), hipMemcpyHostToDevice, st));
        MDP_HIP(hipStreamSynchronize(st));
        end_call(ctx, st);
        if (rel_residual_out) *rel_residual_out = r.rel_residual;
        if (cond_estimate_out) *cond_estimate_out = r.cond;
        return MDP_OK;
    });
}

// ---------------------------------------------------------------------------- step 3
int mdp_reconstruct(mdp_ctx* ctx, int n_sub, const mdp_projector* const* P, const mdp_c128* c, void* stream,
                    mdp_c128* u_out) {
    if (!ctx) return fail(nullptr, MDP_ERR_ARG, "ctx is NULL");
    return guarded(ctx, [&]() -> int {
        if (n_sub < 1 || !P || !c || !u_out) throw Error(MDP_ERR_ARG, "null or empty arguments");
        hipStream_t st = (hipStream_t)stream;
        std::vector<long> off(n_sub + 1, 0);
        for (int i = 0; i < n_sub; ++i) {
            if (!P[i]) throw Error(MDP_ERR_ARG, "null projector");
            off[i + 1] = off[i] + (long)(P[i]->g.n + 1) * (P[i]->g.n + 1);
        }
        begin_call(ctx, st);
        // group subdomains by projector: one batched solve per distinct projector
        std::vector<bool> done(n_sub, false);
        for (int i = 0; i < n_sub; ++i) {
            if (done[i]) continue;
            const mdp_projector* Pi = P[i];
            std::vector<int> grp;
            for (int j = i; j < n_sub; ++j)
                if (P[j] == Pi) { grp.push_back(j); done[j] = true; }
            const Geometry& G = Pi->g;
            const int n = G.n, ng = G.n_gamma, ncol = 8 * Pi->m_star, R = (int)grp.size();
            const long npts = (long)(n + 1) * (n + 1);
            APPlan& plan = get_plan(ctx, n, G.h, Pi->k);
            DevBuf& cb = ctx->ws.cw.rc_c;
            DevBuf& wb = ctx->ws.cw.rc_w;
            ensure(cb, (size_t)R * ncol * sizeof(mdp_c128));
            ensure(wb, (size_t)R * npts * sizeof(mdp_c128));
            for (int r = 0; r < R; ++r)
                MDP_HIP(hipMemcpyAsync(cb.as<mdp_c128>() + (size_t)r * ncol, c + (size_t)grp[r] * ncol,
                                       ncol * sizeof(mdp_c128), hipMemcpyDeviceToDevice, st));
            MDP_HIP(hipMemsetAsync(wb.p, 0, (size_t)R * npts * sizeof(mdp_c128), st));
            launch_extend_density(Pi->E.as<double>(), ng, ncol, cb.as<double>(), R, Pi->gm, Pi->gq, Pi->gside, n,
                                  wb.as<double>(), npts, st);
            const int chunk = chunk_size(plan, Pi->precision, ctx->ws_cap, R);
            prepare_ws(ctx, plan, Pi->precision, chunk);
            for (int r0 = 0; r0 < R; r0 += chunk) {
                const int Rc = std::min(chunk, R - r0);
                SrcDesc src{};
                src.kind = Src::STENCIL_GRID;
                src.grid = wb.as<double>() + 2 * (size_t)r0 * npts;
                src.grid_stride = npts;
                src.m_lo = G.m_lo; src.m_hi = G.m_hi; src.q_lo = G.q_lo; src.q_hi = G.q_hi;
                double* w = wb.as<double>() + 2 * (size_t)r0 * npts;
                const Fold f = plan.f;
                const int prec = Pi->precision;
                solve_batch(plan, ctx->ws, prec, src, true, Rc,
                            [&](const void* u, const float* du) {
                                // u_out = w - G(L w |M+), written in place over w
                                ctx->ws.prof.run("unfold_grid", st, 0.0, (double)Rc * npts * 16.0 * 3.0, [&] {
                                    if (prec == MDP_C128)
                                        launch_unfold_grid<double>((const double*)u, du, n, f, Rc, w, npts, w, npts,
                                                                   st);
                                    else
                                        launch_unfold_grid<float>((const float*)u, du, n, f, Rc, w, npts, w, npts, st);
                                });
                            },
                            st);
            }
            for (int r = 0; r < R; ++r)
                MDP_HIP(hipMemcpyAsync(u_out + off[grp[r]], wb.as<mdp_c128>() + (size_t)r * npts,
                                       npts * sizeof(mdp_c128), hipMemcpyDeviceToDevice, st));
        }
        end_call(ctx, st);
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
        begin_call(ctx, st);
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
            solve_batch(plan, ctx->ws, precision, src, true, R,
                        [&](const void* uu, const float* du) {
                            if (precision == MDP_C128)
                                launch_unfold_grid<double>((const double*)uu, du, n, f, R, nullptr, 0, out, npts, st);
                            else
                                launch_unfold_grid<float>((const float*)uu, du, n, f, R, nullptr, 0, out, npts, st);
                        },
                        st);
        }
        end_call(ctx, st);
        return MDP_OK;
    });
}

// ---------------------------------------------------------------------------- cache / profiling
int mdp_cache_clear(mdp_ctx* ctx) {
    if (!ctx) return MDP_ERR_ARG;
    return guarded(ctx, [&]() -> int {
        MDP_HIP(hipDeviceSynchronize());
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
