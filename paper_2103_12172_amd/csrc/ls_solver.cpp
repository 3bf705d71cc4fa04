// Interface least squares on the device (paper Sec. 3.5, steps 2b-2c):
// min ||Qbar c - Fbar||_2 through a QR factorisation Qbar = Q R and
// c = R^{-1} Q^* Fbar.
//
// The factorisation is Cholesky-QR with re-orthogonalisation (CholeskyQR2;
// shifted CholeskyQR3 when the first Gram matrix is numerically indefinite):
// after scaling every column to unit norm, each pass forms the Gram matrix
// G = A^* A, its Cholesky factor G = L L^*, and A <- A L^{-*}.  Two passes give
// columns orthonormal to working precision when cond(A) is below ~1e7; the
// shifted first pass (G + s I, s = 11 (m n + n(n+1)) u ||A||^2) extends this to
// cond(A) ~ 1/u at the price of a third pass.  R is the product of the L^*
// factors.  Every pass is complex FP64 GEMM on the matrix cores (Gram, the
// blocked triangular inverse, the product with it) plus one small Cholesky per
// 64-column diagonal block, instead of the long chain of column-by-column
// reflector kernels a Householder factorisation would need on a GPU.  One step
// of least-squares refinement with the same factors follows.
#include "ls_solver.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace mdp {

namespace {

constexpr int NB = 64;
const double2 ONE = {1.0, 0.0}, ZERO = {0.0, 0.0}, MONE = {-1.0, 0.0};

struct LSBufs {
    DevBuf G, L, Linv[3], T, A0, Aw, Aq, F, y, z, x, r, info, norms;
};

// Blocked lower Cholesky G = L L^* (G is overwritten by the trailing updates)
// and the blocked inverse Linv = L^{-1}.  Returns the 1-based index of the
// first failing pivot, 0 on success.
int cholesky_and_inverse(double2* G, double2* L, double2* Linv, double2* T, int* info_dev, int nc, double shift,
                         Workspace& ws, hipStream_t st) {
    MDP_HIP(hipMemsetAsync(info_dev, 0, sizeof(int), st));
    MDP_HIP(hipMemsetAsync(L, 0, sizeof(double2) * (size_t)nc * nc, st));
    MDP_HIP(hipMemsetAsync(Linv, 0, sizeof(double2) * (size_t)nc * nc, st));
    for (int kb = 0; kb < nc; kb += NB) {
        const int nbk = std::min(NB, nc - kb);
        launch_chol_block(G + kb + (size_t)kb * nc, nc, nbk, shift, L + kb + (size_t)kb * nc, nc,
                          Linv + kb + (size_t)kb * nc, nc, info_dev, kb, st);
        const int rest = nc - kb - nbk;
        if (rest > 0) {
            // panel: L(below, k) = G(below, k) L_kk^{-*}
            launch_zgemm('N', 'C', rest, nbk, nbk, ONE, G + (kb + nbk) + (size_t)kb * nc, nc,
                         Linv + kb + (size_t)kb * nc, nc, ZERO, L + (kb + nbk) + (size_t)kb * nc, nc, ws.zg, st);
            // trailing update: G(below, below) -= L(below, k) L(below, k)^*
            launch_zgemm('N', 'C', rest, rest, nbk, MONE, L + (kb + nbk) + (size_t)kb * nc, nc,
                         L + (kb + nbk) + (size_t)kb * nc, nc, ONE, G + (kb + nbk) + (size_t)(kb + nbk) * nc, nc,
                         ws.zg, st);
        }
    }
    // block rows of the inverse: Linv(i, 0:i) = -Linv_ii L(i, 0:i) Linv(0:i, 0:i)
    for (int ib = NB; ib < nc; ib += NB) {
        const int nbi = std::min(NB, nc - ib);
        launch_zgemm('N', 'N', nbi, ib, ib, ONE, L + ib, nc, Linv, nc, ZERO, T, nbi, ws.zg, st);
        launch_zgemm('N', 'N', nbi, ib, nbi, MONE, Linv + ib + (size_t)ib * nc, nc, T, nbi, ZERO, Linv + ib, nc,
                     ws.zg, st);
    }
    int info = 0;
    MDP_HIP(hipMemcpyAsync(&info, info_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    MDP_HIP(hipStreamSynchronize(st));
    return info;
}

double host_norm(const double2* dev, int m, hipStream_t st) {
    std::vector<double2> h(m);
    MDP_HIP(hipMemcpyAsync(h.data(), dev, sizeof(double2) * m, hipMemcpyDeviceToHost, st));
    MDP_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (auto& v : h) s += v.x * v.x + v.y * v.y;
    return std::sqrt(s);
}

}  // namespace

// A: m x nc (ld m, device) -- overwritten; F: m (device); x_out: nc (device).
LSResult ls_solve(Workspace& ws, double2* A, const double2* F, int m, int nc, double2* x_out, bool want_cond,
                  hipStream_t st) {
    if (m < nc) throw Error(MDP_ERR_ARG, "least squares needs at least as many rows as unknowns");
    LSResult res{};
    LSBufs b;
    const size_t nn = (size_t)nc * nc, mn = (size_t)m * nc;
    b.G.alloc(nn * sizeof(double2));
    b.L.alloc(nn * sizeof(double2));
    for (auto& l : b.Linv) l.alloc(nn * sizeof(double2));
    b.T.alloc((size_t)NB * nc * sizeof(double2));
    b.A0.alloc(mn * sizeof(double2));
    b.Aq.alloc(mn * sizeof(double2));
    b.y.alloc(nc * sizeof(double2));
    b.z.alloc(nc * sizeof(double2));
    b.x.alloc(nc * sizeof(double2));
    b.r.alloc(m * sizeof(double2));
    b.info.alloc(sizeof(int));
    b.norms.alloc(nc * sizeof(double));

    // column equilibration
    launch_col_norms(A, m, nc, m, b.norms.as<double>(), st);
    std::vector<double> norms(nc);
    MDP_HIP(hipMemcpyAsync(norms.data(), b.norms.p, nc * sizeof(double), hipMemcpyDeviceToHost, st));
    MDP_HIP(hipStreamSynchronize(st));
    for (int c = 0; c < nc; ++c) {
        if (!std::isfinite(norms[c])) throw Error(MDP_ERR_NONFINITE, "non-finite entry in the interface matrix");
        if (!(norms[c] > 0.0)) throw Error(MDP_ERR_SINGULAR, "zero column in the interface matrix");
    }
    launch_scale_cols(A, m, nc, m, b.norms.as<double>(), 1, st);
    MDP_HIP(hipMemcpyAsync(b.A0.p, A, mn * sizeof(double2), hipMemcpyDeviceToDevice, st));

    double2* cur = A;
    double2* nxt = b.Aq.as<double2>();
    int passes = 2;
    double shift = 0.0;
    for (int pass = 0; pass < passes; ++pass) {
        launch_zgemm('C', 'N', nc, nc, m, ONE, cur, m, cur, m, ZERO, b.G.as<double2>(), nc, ws.zg, st);
        int info = cholesky_and_inverse(b.G.as<double2>(), b.L.as<double2>(), b.Linv[pass].as<double2>(),
                                        b.T.as<double2>(), b.info.as<int>(), nc, pass == 0 ? shift : 0.0, ws, st);
        if (info && pass == 0 && shift == 0.0) {
            // numerically indefinite Gram matrix: shifted first pass, one extra pass
            const double u = 1.1102230246251565e-16;
            shift = 11.0 * ((double)m * nc + (double)nc * (nc + 1)) * u * (double)nc;
            passes = 3;
            launch_zgemm('C', 'N', nc, nc, m, ONE, cur, m, cur, m, ZERO, b.G.as<double2>(), nc, ws.zg, st);
            info = cholesky_and_inverse(b.G.as<double2>(), b.L.as<double2>(), b.Linv[0].as<double2>(),
                                        b.T.as<double2>(), b.info.as<int>(), nc, shift, ws, st);
        }
        if (info) throw Error(MDP_ERR_SINGULAR, "interface least squares: Cholesky-QR broke down (rank deficient)");
        // A <- A L^{-*}
        launch_zgemm('N', 'C', m, nc, nc, ONE, cur, m, b.Linv[pass].as<double2>(), nc, ZERO, nxt, m, ws.zg, st);
        std::swap(cur, nxt);
    }
    res.shifted = shift != 0.0;
    res.passes = passes;

    // x = R^{-1} Q^* F with R^{-1} = Linv_0^* Linv_1^* ... Linv_{p-1}^* (apply the last pass first);
    // `accumulate` adds the result to `out` instead of overwriting it.
    DevBuf s1(nc * sizeof(double2)), s2(nc * sizeof(double2));
    auto apply_rinv = [&](const double2* v, double2* out, bool accumulate) {
        const double2* src = v;
        double2* bufs[2] = {s1.as<double2>(), s2.as<double2>()};
        int t = 0;
        for (int p = passes - 1; p >= 0; --p) {
            double2* dst = (p == 0) ? out : bufs[t];
            launch_zgemm('C', 'N', nc, 1, nc, ONE, b.Linv[p].as<double2>(), nc, src, nc,
                         (p == 0 && accumulate) ? ONE : ZERO, dst, nc, ws.zg, st);
            src = dst;
            t ^= 1;
        }
    };
    double2* Qf = cur;
    DevBuf qtf(nc * sizeof(double2));
    launch_zgemm('C', 'N', nc, 1, m, ONE, Qf, m, F, m, ZERO, qtf.as<double2>(), nc, ws.zg, st);
    apply_rinv(qtf.as<double2>(), b.x.as<double2>(), false);
    // one refinement step: r = F - A0 x, x += R^{-1} Q^* r
    MDP_HIP(hipMemcpyAsync(b.r.p, F, m * sizeof(double2), hipMemcpyDeviceToDevice, st));
    launch_zgemm('N', 'N', m, 1, nc, MONE, b.A0.as<double2>(), m, b.x.as<double2>(), nc, ONE, b.r.as<double2>(), m,
                 ws.zg, st);
    launch_zgemm('C', 'N', nc, 1, m, ONE, Qf, m, b.r.as<double2>(), m, ZERO, qtf.as<double2>(), nc, ws.zg, st);
    apply_rinv(qtf.as<double2>(), b.x.as<double2>(), true);
    // residual
    MDP_HIP(hipMemcpyAsync(b.r.p, F, m * sizeof(double2), hipMemcpyDeviceToDevice, st));
    launch_zgemm('N', 'N', m, 1, nc, MONE, b.A0.as<double2>(), m, b.x.as<double2>(), nc, ONE, b.r.as<double2>(), m,
                 ws.zg, st);
    const double nf = host_norm(F, m, st);
    res.rel_residual = host_norm(b.r.as<double2>(), m, st) / (nf > 0 ? nf : 1.0);

    // unscale: c = x / norms
    launch_scale_cols(b.x.as<double2>(), 1, nc, 1, b.norms.as<double>(), 1, st);
    MDP_HIP(hipMemcpyAsync(x_out, b.x.p, nc * sizeof(double2), hipMemcpyDeviceToDevice, st));

    if (want_cond) {
        // power iterations for sigma_max(A0) (on A0^* A0) and sigma_min (on R^{-1} R^{-*})
        std::vector<double2> hv(nc);
        for (int i = 0; i < nc; ++i) hv[i] = make_double2(1.0 + 0.001 * (i % 7), 0.37 * ((i * 13) % 5));
        DevBuf v(nc * sizeof(double2)), w(nc * sizeof(double2)), t(m * sizeof(double2));
        auto normalize = [&](DevBuf& vec) {
            std::vector<double2> h(nc);
            MDP_HIP(hipMemcpyAsync(h.data(), vec.p, nc * sizeof(double2), hipMemcpyDeviceToHost, st));
            MDP_HIP(hipStreamSynchronize(st));
            double s = 0;
            for (auto& e : h) s += e.x * e.x + e.y * e.y;
            s = std::sqrt(s);
            for (auto& e : h) { e.x /= s; e.y /= s; }
            MDP_HIP(hipMemcpyAsync(vec.p, h.data(), nc * sizeof(double2), hipMemcpyHostToDevice, st));
            MDP_HIP(hipStreamSynchronize(st));
            return s;
        };
        MDP_HIP(hipMemcpyAsync(v.p, hv.data(), nc * sizeof(double2), hipMemcpyHostToDevice, st));
        normalize(v);
        double lmax = 0.0;
        for (int it = 0; it < 12; ++it) {
            launch_zgemm('N', 'N', m, 1, nc, ONE, b.A0.as<double2>(), m, v.as<double2>(), nc, ZERO, t.as<double2>(), m,
                         ws.zg, st);
            launch_zgemm('C', 'N', nc, 1, m, ONE, b.A0.as<double2>(), m, t.as<double2>(), m, ZERO, v.as<double2>(), nc,
                         ws.zg, st);
            lmax = normalize(v);
        }
        MDP_HIP(hipMemcpyAsync(w.p, hv.data(), nc * sizeof(double2), hipMemcpyHostToDevice, st));
        normalize(w);
        double lmin_inv = 0.0;
        for (int it = 0; it < 12; ++it) {
            // w <- R^{-1} R^{-*} w with R^{-*} = Linv_{p-1} ... Linv_1 Linv_0 (Linv_0 applied first)
            const double2* src = w.as<double2>();
            double2* bufs[2] = {b.z.as<double2>(), b.y.as<double2>()};
            int tt = 0;
            for (int p = 0; p < passes; ++p) {
                launch_zgemm('N', 'N', nc, 1, nc, ONE, b.Linv[p].as<double2>(), nc, src, nc, ZERO, bufs[tt], nc,
                             ws.zg, st);
                src = bufs[tt];
                tt ^= 1;
            }
            apply_rinv(src, w.as<double2>(), false);
            lmin_inv = normalize(w);
        }
        res.cond = std::sqrt(lmax * lmin_inv);
    }
    MDP_HIP(hipStreamSynchronize(st));
    return res;
}

}  // namespace mdp
