// Host side of the batched auxiliary-problem solve G^(h) (paper Sec. 3.2.1).
//
// The discrete AP (compact scheme at interior nodes, u = 0 at q = 0 and n,
// fourth-order Sommerfeld-type rows at m = 0 and n) is diagonalised in y by the
// type-I sine transform (the Dirichlet ends make every y second difference act
// on mode j as multiplication by -lambda_j, lambda_j = 4 sin^2(pi j/(2n))), so
// one solve is: forward sine transform of every grid row, one complex
// tridiagonal system in x per mode, inverse sine transform.  The plan holds the
// device constants of one (n, h, k): the block-diagonal sine matrices of the
// folded layout and the LU factors of the per-mode tridiagonal matrices.
#include "ap_solver.h"

#include <cmath>
#include <complex>
#include <cstring>

namespace mdp {

using cd = std::complex<double>;

StencilCoef stencil_coef(double h, double k) {
    // eq. FD_scheme: (1/h^2)(E - 4u) + (1/(6h^2))(C + 4u - 2E) + (k^2/12)(E + 8u)
    StencilCoef s;
    s.c0 = -10.0 / (3.0 * h * h) + 2.0 * k * k / 3.0;
    s.ce = 2.0 / (3.0 * h * h) + k * k / 12.0;
    s.cc = 1.0 / (6.0 * h * h);
    return s;
}

EndRowCoef end_row_coef(double h, double k) {
    // x-end rows at the half node: D/h + d2(D)/(24h) + (k^2 h/24) D +- i k [A + d2(A)/8 + (k^2 h^2/8) A] = 0
    EndRowCoef e;
    e.wD = 1.0 / h + k * k * h / 24.0;
    e.wD2 = 1.0 / (24.0 * h);
    e.wA = 1.0 + k * k * h * h / 8.0;
    e.wA2 = 1.0 / 8.0;
    e.k = k;
    return e;
}

namespace {

// mode j of folded column c (0 = padding)
int mode_of(const Fold& f, int c) {
    if (c < f.P1) return (c < f.p) ? 2 * c + 1 : 0;
    int cc = c - f.P1;
    return (cc < f.p - 1) ? 2 * cc + 2 : 0;
}

// sine value sin(pi j q / n) with the argument reduced exactly mod 2n
double sine(int j, int q, int n) {
    long a = ((long)j * q) % (2L * n);
    return std::sin(M_PI * (double)a / (double)n);
}

template <class T>
void upload(DevBuf& d, const std::vector<double>& h) {
    std::vector<T> t(h.begin(), h.end());
    d.alloc(t.size() * sizeof(T));
    MDP_HIP(hipMemcpy(d.p, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice));
}

}  // namespace

APPlan::APPlan(int n_, double h_, double k_) : n(n_), h(h_), k(k_) {
    if (n < 8 || (n & 1)) throw Error(MDP_ERR_ARG, "n must be even and >= 8");
    if (!std::isfinite(h) || !(h > 0)) throw Error(MDP_ERR_ARG, "grid step must be positive and finite");
    if (!std::isfinite(k) || !(k > 0)) throw Error(MDP_ERR_NONFINITE, "wavenumber must be positive and finite");
    f = Fold::make(n);
    sc = stencil_coef(h, k);
    ec = end_row_coef(h, k);
    const int W = f.W;

    // block-diagonal sine matrices, row-major W x W.
    // forward: B[kcol][c] = (2/n) sin(pi j q/n) for kcol = folded physical column of q, c = folded mode of j
    // inverse: B[c][kcol] = sin(pi j q/n)
    std::vector<double> Sf((size_t)W * W, 0.0), Si((size_t)W * W, 0.0);
    for (int c = 0; c < W; ++c) {
        int j = mode_of(f, c);
        if (!j) continue;
        bool odd = (c < f.P1);
        int qmax = odd ? f.p : f.p - 1;
        int base = odd ? 0 : f.P1;
        for (int q = 1; q <= qmax; ++q) {
            double s = sine(j, q, n);
            int kc = base + q - 1;
            Sf[(size_t)kc * W + c] = (2.0 / n) * s;
            Si[(size_t)c * W + kc] = s;
        }
    }

    // tridiagonal matrices per mode, rows m = 0..n:
    //   m = 0:      (-wD - i k wA/2) U0 + (wD - i k wA/2) U1 = rhs0
    //   0 < m < n:  a U(m-1) + (b - 2a) U(m) + a U(m+1) = rhs
    //   m = n:      (-wD + i k wA/2) U(n-1) + (wD + i k wA/2) Un = rhsn
    // with a = 1/h^2 - lambda/(6h^2) + k^2/12, b = k^2 - lambda (1/h^2 + k^2/12),
    // wD = 1/h - lambda/(24h) + k^2 h/24, wA = 1 - lambda/8 + k^2 h^2/8.
    // Thomas factors: d'_0 = diag_0, l_m = sub_m/d'_{m-1}, d'_m = diag_m - l_m sup_{m-1}; r_m = 1/d'_m.
    // Twisted pivots (projector sweep over a band of rows m0..t with a zero right-hand side
    // below t): with the bottom-up elimination e_n = diag_n, e_m = diag_m - sup_m sub_{m+1}/e_{m+1},
    // row t reduces to gamma_t x_t = y_t, gamma_t = d'_t - sup_t sub_{t+1}/e_{t+1} (gamma_n = d'_n);
    // tw_m = 1/gamma_m.
    const size_t plane = (size_t)(n + 1) * W;
    std::vector<double> fac(6 * plane, 0.0), colc(3 * (size_t)W, 0.0), tw(2 * plane, 0.0);
    std::vector<cd> dpiv(n + 1);
    twist_ratio.assign(n + 1, 1e300);
    const double h2 = h * h, k2 = k * k;
    min_pivot_ratio = 1e300;
    for (int c = 0; c < W; ++c) {
        int j = mode_of(f, c);
        if (!j) continue;
        double sj = std::sin(M_PI * j / (2.0 * n));
        double lam = 4.0 * sj * sj;
        double a = 1.0 / h2 - lam / (6.0 * h2) + k2 / 12.0;
        double b = k2 - lam * (1.0 / h2 + k2 / 12.0);
        double wD = 1.0 / h - lam / (24.0 * h) + k2 * h / 24.0;
        double wA = 1.0 - lam / 8.0 + k2 * h2 / 8.0;
        cd ik(0.0, k);
        cd diag0 = -wD - ik * wA * 0.5, sup0 = wD - ik * wA * 0.5;
        cd subn = -wD + ik * wA * 0.5, diagn = wD + ik * wA * 0.5;
        double scale = std::abs(a) + std::abs(b - 2 * a) + std::abs(wD) + k * std::abs(wA);
        cd dprev = diag0;
        auto put = [&](int m, cd l, cd r) {
            fac[0 * plane + (size_t)m * W + c] = l.real();
            fac[1 * plane + (size_t)m * W + c] = l.imag();
            fac[2 * plane + (size_t)m * W + c] = r.real();
            fac[3 * plane + (size_t)m * W + c] = r.imag();
        };
        double minp = std::abs(dprev);
        put(0, 0.0, 1.0 / dprev);
        dpiv[0] = dprev;
        for (int m = 1; m <= n; ++m) {
            cd sub = (m < n) ? cd(a) : subn;
            cd sup = (m - 1 == 0) ? sup0 : cd(a);
            cd diag = (m < n) ? cd(b - 2 * a) : diagn;
            cd l = sub / dprev;
            cd d = diag - l * sup;
            minp = std::min(minp, std::abs(d));
            put(m, l, 1.0 / d);
            dprev = d;
            dpiv[m] = d;
        }
        min_pivot_ratio = std::min(min_pivot_ratio, minp / scale);
        cd e = diagn;
        for (int m = n; m >= 0; --m) {
            cd gam = dpiv[m];
            if (m < n) {
                const cd sup = (m == 0) ? sup0 : cd(a);
                const cd sub1 = (m + 1 < n) ? cd(a) : subn;
                gam -= sup * sub1 / e;
                const cd diag = (m == 0) ? diag0 : cd(b - 2 * a);
                e = diag - sup * sub1 / e;
            }
            const cd r = 1.0 / gam;
            tw[2 * ((size_t)m * W + c)] = r.real();
            tw[2 * ((size_t)m * W + c) + 1] = r.imag();
            fac[4 * plane + (size_t)m * W + c] = r.real();
            fac[5 * plane + (size_t)m * W + c] = r.imag();
            twist_ratio[m] = std::min(twist_ratio[m], std::abs(gam) / scale);
        }
        colc[c] = a;
        colc[W + c] = sup0.real();
        colc[2 * (size_t)W + c] = sup0.imag();
    }
    if (!(min_pivot_ratio > 1e-13))
        throw Error(MDP_ERR_SINGULAR, "a tridiagonal mode pivot of the auxiliary problem vanished");

    upload<double>(Sf64, Sf);
    upload<double>(Si64, Si);
    upload<float>(Sf32, Sf);
    upload<float>(Si32, Si);
    upload<double>(fac64, fac);
    upload<float>(fac32, fac);
    upload<double>(colc64, colc);
    // the fused sweep's tables, in the unknowns scaled by the interior off-diagonal a of the
    // mode (q_m = a p_m, x~_m = a x_m): a r_m on every row and a tw_m, interleaved complex
    std::vector<double> rf(2 * plane), tf(2 * plane);
    for (int m = 0; m <= n; ++m)
        for (int c = 0; c < W; ++c) {
            const size_t e = (size_t)m * W + c;
            const double a = colc[c];
            rf[2 * e] = a * fac[2 * plane + e];
            rf[2 * e + 1] = a * fac[3 * plane + e];
            tf[2 * e] = a * tw[2 * e];
            tf[2 * e + 1] = a * tw[2 * e + 1];
        }
    upload<double>(rf64, rf);
    upload<double>(tf64, tf);
    upload<float>(rf32, rf);
    upload<float>(tf32, tf);
    upload<float>(colc32, colc);
}

// One batched solve: R right-hand sides from `src` (complex if src_cplx), result
// handed to `consume(u, du)` as folded synthesis rows in T (u) plus, for the
// refined precision, the FP32 correction (du).  A, B: batch buffers of
// R * 2 * rows * W elements of T each; C (refined only): R * 2 * rows * W floats.
// pr null: no per-launch profiling and no GEMM autotuning (nothing is allocated).
template <class T>
static void solve_batch_bufs(const APPlan& P, T* A, T* B, float* C, Profiler* pr, const SrcDesc& src, bool src_cplx,
                             int R, bool refine, Band bd,
                             const std::function<void(const void*, const float*, Band)>& consume, hipStream_t st) {
    const Fold& f = P.f;
    const int n = P.n;
    const size_t rows = (size_t)bd.nr;
    const int pin = src_cplx ? 2 : 1;
    const bool tune = pr != nullptr;
    const T* Sf = (const T*)(sizeof(T) == 8 ? P.Sf64.p : P.Sf32.p);
    const T* Si = (const T*)(sizeof(T) == 8 ? P.Si64.p : P.Si32.p);
    const T* fac = (const T*)(sizeof(T) == 8 ? P.fac64.p : P.fac32.p);
    const T* colc = (const T*)(sizeof(T) == 8 ? P.colc64.p : P.colc32.p);
    auto run = [&](const char* name, double flops, double bytes, auto&& f_) {
        if (pr) pr->run(name, st, flops, bytes, f_);
        else f_();
    };

    // algorithmic work per launch: only the p + (p-1) = n-1 useful columns of a
    // folded row count, padding does not
    const double useful = (double)(n - 1);
    const double gemm_row_flops = 2.0 * ((double)f.p * f.p + (double)(f.p - 1) * (f.p - 1));
    const double rows_in = (double)R * pin * rows, rows_c = (double)R * 2 * rows;
    const double tri_pts = (double)R * rows * useful;
    run("fold_rhs", 0.0, rows_in * useful * sizeof(T), [&] { launch_fold_rhs<T>(src, n, f, P.sc, R, src_cplx, bd, A, st); });
    run(sizeof(T) == 8 ? "gemm_sine_f64" : "gemm_sine_f32", rows_in * gemm_row_flops,
        2.0 * rows_in * useful * sizeof(T), [&] { launch_gemm_bd<T>(A, Sf, B, (long)R * pin * rows, f, st, tune); });
    run(sizeof(T) == 8 ? "tridiag_f64" : "tridiag_f32", tri_pts * 22.0,
        tri_pts * (pin + 2) * sizeof(T) + 4.0 * rows * useful * sizeof(T),
        [&] { launch_tridiag<T>(B, pin, A, fac, colc, n, f, R, bd, st); });
    run(sizeof(T) == 8 ? "gemm_sine_f64" : "gemm_sine_f32", rows_c * gemm_row_flops,
        2.0 * rows_c * useful * sizeof(T), [&] { launch_gemm_bd<T>(A, Si, B, (long)R * 2 * rows, f, st, tune); });
    const float* du = nullptr;
    if (refine) {
        // r = g - A u in FP64 (u = the FP32 solution in B), correction solved in FP32
        float* Af = reinterpret_cast<float*>(A);
        const double tri_c = (double)R * rows * useful;
        run("residual", tri_c * 9.0 * 8.0, tri_c * 2.0 * 2.0 * sizeof(float),
            [&] { launch_residual(src, n, f, P.sc, P.ec, R, src_cplx, reinterpret_cast<const float*>(B), Af, st); });
        run("gemm_sine_f32", rows_c * gemm_row_flops, 2.0 * rows_c * useful * sizeof(float),
            [&] { launch_gemm_bd<float>(Af, P.Sf32.as<float>(), C, (long)R * 2 * rows, f, st, tune); });
        run("tridiag_f32", tri_c * 22.0, tri_c * 4.0 * sizeof(float) + 4.0 * rows * useful * sizeof(float),
            [&] { launch_tridiag<float>(C, 2, Af, P.fac32.as<float>(), P.colc32.as<float>(), n, f, R, bd, st); });
        run("gemm_sine_f32", rows_c * gemm_row_flops, 2.0 * rows_c * useful * sizeof(float),
            [&] { launch_gemm_bd<float>(Af, P.Si32.as<float>(), C, (long)R * 2 * rows, f, st, tune); });
        du = C;
    }
    consume(B, du, bd);
}

template <class T>
static void solve_batch_t(const APPlan& P, Workspace& ws, const SrcDesc& src, bool src_cplx, int R, bool refine,
                          Band bd, const std::function<void(const void*, const float*, Band)>& consume,
                          hipStream_t st) {
    if (refine) bd = Band{0, P.n + 1};   // the FP64 residual needs every row of the AP
    const size_t elems = (size_t)R * 2 * bd.nr * P.f.W;
    ws.a.reserve(elems * sizeof(T));
    ws.b.reserve(elems * sizeof(T));
    if (refine) ws.c.reserve(elems * sizeof(float));
    solve_batch_bufs<T>(P, ws.a.as<T>(), ws.b.as<T>(), refine ? ws.c.as<float>() : nullptr, &ws.prof, src, src_cplx, R,
                        refine, bd, consume, st);
}

size_t solve_scratch_bytes(const APPlan& P, int precision, int R) {
    const size_t elems = (size_t)R * 2 * (P.n + 1) * P.f.W;
    if (precision == MDP_C128) return 2 * elems * sizeof(double);
    return 2 * elems * sizeof(float) + (precision == MDP_C64_REFINED ? elems * sizeof(float) : 0);
}

void solve_batch_scratch(const APPlan& P, int precision, void* scratch, const SrcDesc& src, bool src_cplx, int R,
                         const std::function<void(const void*, const float*, Band)>& consume, hipStream_t st) {
    if (R <= 0) return;
    const Band all{0, P.n + 1};
    const size_t elems = (size_t)R * 2 * (P.n + 1) * P.f.W;
    if (precision == MDP_C128) {
        double* A = static_cast<double*>(scratch);
        solve_batch_bufs<double>(P, A, A + elems, nullptr, nullptr, src, src_cplx, R, false, all, consume, st);
    } else {
        float* A = static_cast<float*>(scratch);
        solve_batch_bufs<float>(P, A, A + elems, precision == MDP_C64_REFINED ? A + 2 * elems : nullptr, nullptr, src,
                                src_cplx, R, precision == MDP_C64_REFINED, all, consume, st);
    }
}

int chunk_size(const APPlan& P, int precision, size_t cap_bytes, int R) {
    const size_t elem = (precision == MDP_C128) ? 8 : 4;
    const size_t per_rhs = 2 * (size_t)(P.n + 1) * P.f.W * elem * (precision == MDP_C64_REFINED ? 3 : 2);
    size_t r = cap_bytes / per_rhs;
    if (r < 1) r = 1;
    if (r > 65535) r = 65535;
    return (int)std::min<size_t>(r, (size_t)R);
}

void solve_batch(const APPlan& P, Workspace& ws, int precision, const SrcDesc& src, bool src_cplx, int R, Band bd,
                 const std::function<void(const void*, const float*, Band)>& consume, hipStream_t st) {
    if (R <= 0) return;
    if (precision == MDP_C128)
        solve_batch_t<double>(P, ws, src, src_cplx, R, false, bd, consume, st);
    else if (precision == MDP_C64)
        solve_batch_t<float>(P, ws, src, src_cplx, R, false, bd, consume, st);
    else if (precision == MDP_C64_REFINED)
        solve_batch_t<float>(P, ws, src, src_cplx, R, true, bd, consume, st);
    else
        throw Error(MDP_ERR_ARG, "unknown precision");
}

}  // namespace mdp
