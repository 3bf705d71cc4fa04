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
// reflector kernels a Householder factorisation needs.  One step of
// least-squares refinement with the same factors follows.  The host waits for
// the device once, at the end (and once more when the shift is needed).
#include "ls_solver.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <functional>
#include <limits>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace mdp {

namespace {

constexpr int NB = 64;
const double2 ONE = {1.0, 0.0}, ZERO = {0.0, 0.0}, MONE = {-1.0, 0.0};

// device scalars written by the kernels and read back once
struct Flags {
    int info;      // first failing Cholesky pivot (1-based) of any pass
    int badcol;    // 1: zero column, 2: non-finite column
    double r2;     // ||F - A x||^2
    double f2;     // ||F||^2
    double pw[2];  // power-iteration norms
};

void grow(DevBuf& b, size_t bytes) {
    if (bytes > b.bytes) {
        MDP_HIP(hipDeviceSynchronize());
        b.reserve(bytes);
    }
}

}  // namespace

CholPlan chol_plan_uniform(int nc) {
    CholPlan p;
    for (int kb = 0; kb < nc; kb += NB) p.push_back({std::min(NB, nc - kb)});
    return p;
}

// Blocked Cholesky G + shift I = L L^* and Linv = L^{-1}, two launches per
// step of the plan (diagonal sub-blocks + panel + inverse block rows, then the
// trailing and inverse updates); W (nc x nc) is the inverse's accumulator.
// G's lower triangle is overwritten by the trailing updates.
double cholesky_and_inverse(double2* G, double2* L, double2* Linv, double2* W, int* info_dev, int nc, double shift,
                            hipStream_t st, Profiler* pr, const CholPlan* plan) {
    MDP_HIP(hipMemsetAsync(L, 0, sizeof(double2) * (size_t)nc * nc, st));
    MDP_HIP(hipMemsetAsync(Linv, 0, sizeof(double2) * (size_t)nc * nc, st));
    MDP_HIP(hipMemsetAsync(W, 0, sizeof(double2) * (size_t)nc * nc, st));
    Profiler none;
    Profiler& p = pr ? *pr : none;
    const CholPlan uniform = plan ? CholPlan{} : chol_plan_uniform(nc);
    const CholPlan& steps = plan ? *plan : uniform;
    int kb = 0;
    double total = 0.0;
    for (const std::vector<int>& widths : steps) {
        // a step with more sub-blocks than one launch takes is split (the sub-blocks do not couple)
        for (size_t q0 = 0; q0 < widths.size(); q0 += CholStepDev::kMaxQ) {
            CholStepDev sp{};
            sp.kb = kb;
            sp.nq = (int)std::min<size_t>(CholStepDev::kMaxQ, widths.size() - q0);
            sp.off[0] = 0;
            double diag_flops = 0.0, diag_bytes = 0.0, panel_flops = 0.0, panel_bytes = 0.0;
            for (int q = 0; q < sp.nq; ++q) sp.off[q + 1] = sp.off[q] + widths[q0 + q];
            sp.wtot = sp.off[sp.nq];
            if (sp.wtot < 1 || kb + sp.wtot > nc) throw Error(MDP_ERR_ARG, "Cholesky plan does not cover the matrix");
            const double wt = sp.wtot, rest = nc - kb - sp.wtot;
            for (int q = 0; q < sp.nq; ++q) {
                // algorithmic flops (complex = 4 real multiply-adds): Cholesky and triangular inverse of the
                // diagonal sub-block (4/3 b^3 each), its panel of L (8 rest b^2), its block row of Z (8 kb b^2)
                const double b = widths[q0 + q];
                diag_flops += 8.0 / 3.0 * b * b * b;
                diag_bytes += 16.0 * 2.0 * b * b;
                panel_flops += 8.0 * rest * b * b + 8.0 * kb * b * b;
                panel_bytes += 16.0 * (b * b + rest * b + 2.0 * kb * b);
            }
            p.run("chol_diag", st, diag_flops, diag_bytes,
                  [&] { launch_chol_diag(G, nc, sp, shift, L, Linv, info_dev, st); });
            if (rest > 0 || kb > 0)
                p.run("chol_panel", st, panel_flops, panel_bytes,
                      [&] { launch_chol_slabs(G, nc, sp, L, Linv, W, st); });
            total += diag_flops + panel_flops;
            // then the trailing update (4 rest^2 w, lower half) and the inverse accumulation (8 rest (kb+w) w)
            if (rest > 0) {
                const double uf = 4.0 * rest * rest * wt + 8.0 * rest * (kb + wt) * wt;
                p.run("chol_update", st, uf, 16.0 * (rest * rest + 2.0 * rest * wt + 2.0 * rest * (kb + wt)),
                      [&] { launch_chol_update(G, nc, kb, sp.wtot, L, Linv, W, st); });
                total += uf;
            }
            kb += sp.wtot;
        }
    }
    if (kb != nc) throw Error(MDP_ERR_ARG, "Cholesky plan does not cover the matrix");
    return total;
}

LSResult ls_solve(Workspace& ws, double2* A, const double2* F, int m, int nc, double2* x_out, bool want_cond,
                  hipStream_t st) {
    if (m < nc) throw Error(MDP_ERR_ARG, "least squares needs at least as many rows as unknowns");
    LSResult res{};
    LSWork& w = ws.ls;
    const size_t nn = (size_t)nc * nc, mn = (size_t)m * nc;
    grow(w.G, nn * sizeof(double2));
    grow(w.L, nn * sizeof(double2));
    for (auto& l : w.Linv) grow(l, nn * sizeof(double2));
    grow(w.T, nn * sizeof(double2));
    grow(w.A0, mn * sizeof(double2));
    grow(w.Aq, mn * sizeof(double2));
    grow(w.vec, (size_t)(6 * nc + 2 * m) * sizeof(double2));
    grow(w.norms, nc * sizeof(double));
    grow(w.flags, sizeof(Flags));
    double2* y = w.vec.as<double2>();
    double2* z = y + nc;
    double2* xv = z + nc;
    double2* s1 = xv + nc;
    double2* s2 = s1 + nc;
    double2* s3 = s2 + nc;
    double2* r = s3 + nc;
    double2* t = r + m;
    Flags* fl = w.flags.as<Flags>();

    auto run = [&](double shift, int passes) {
        MDP_HIP(hipMemsetAsync(&fl->info, 0, sizeof(int), st));
        MDP_HIP(hipMemcpyAsync(A, w.A0.p, mn * sizeof(double2), hipMemcpyDeviceToDevice, st));
        double2* cur = A;
        double2* nxt = w.Aq.as<double2>();
        for (int pass = 0; pass < passes; ++pass) {
            launch_zgemm('C', 'N', nc, nc, m, ONE, cur, m, cur, m, ZERO, w.G.as<double2>(), nc, ws.zg, st, 1);
            cholesky_and_inverse(w.G.as<double2>(), w.L.as<double2>(), w.Linv[pass].as<double2>(), w.T.as<double2>(),
                                 &fl->info, nc, pass == 0 ? shift : 0.0, st, &ws.prof);
            // A <- A L^{-*}  (L^{-*} is upper triangular)
            launch_zgemm('N', 'C', m, nc, nc, ONE, cur, m, w.Linv[pass].as<double2>(), nc, ZERO, nxt, m, ws.zg, st, 2);
            std::swap(cur, nxt);
        }
        return cur;   // Q, orthonormal columns
    };
    // R^{-1} v = Linv_0^* Linv_1^* ... Linv_{p-1}^* v (last pass first)
    auto apply_rinv = [&](int passes, const double2* v, double2* out, bool accumulate) {
        const double2* src = v;
        double2* bufs[2] = {s1, s2};
        int tt = 0;
        for (int p = passes - 1; p >= 0; --p) {
            double2* dst = (p == 0) ? out : bufs[tt];
            launch_zgemm('C', 'N', nc, 1, nc, ONE, w.Linv[p].as<double2>(), nc, src, nc,
                         (p == 0 && accumulate) ? ONE : ZERO, dst, nc, ws.zg, st);
            src = dst;
            tt ^= 1;
        }
    };

    // column equilibration (A0 keeps the scaled matrix)
    MDP_HIP(hipMemsetAsync(fl, 0, sizeof(Flags), st));
    launch_col_norms(A, m, nc, m, w.norms.as<double>(), st);
    launch_scale_cols_checked(A, m, nc, m, w.norms.as<double>(), &fl->badcol, st);
    MDP_HIP(hipMemcpyAsync(w.A0.p, A, mn * sizeof(double2), hipMemcpyDeviceToDevice, st));

    int passes = 2;
    double shift = 0.0;
    Flags hf{};
    for (int attempt = 0; attempt < 2; ++attempt) {
        double2* Q = run(shift, passes);
        // x = R^{-1} Q^* F, then one refinement step x += R^{-1} Q^* (F - A0 x)
        launch_zgemm('C', 'N', nc, 1, m, ONE, Q, m, F, m, ZERO, y, nc, ws.zg, st);
        apply_rinv(passes, y, xv, false);
        MDP_HIP(hipMemcpyAsync(r, F, m * sizeof(double2), hipMemcpyDeviceToDevice, st));
        launch_zgemm('N', 'N', m, 1, nc, MONE, w.A0.as<double2>(), m, xv, nc, ONE, r, m, ws.zg, st);
        launch_zgemm('C', 'N', nc, 1, m, ONE, Q, m, r, m, ZERO, y, nc, ws.zg, st);
        apply_rinv(passes, y, xv, true);
        // final residual
        MDP_HIP(hipMemcpyAsync(r, F, m * sizeof(double2), hipMemcpyDeviceToDevice, st));
        launch_zgemm('N', 'N', m, 1, nc, MONE, w.A0.as<double2>(), m, xv, nc, ONE, r, m, ws.zg, st);
        MDP_HIP(hipMemsetAsync(&fl->r2, 0, 2 * sizeof(double), st));
        launch_znorm2(m, r, &fl->r2, st);
        launch_znorm2(m, F, &fl->f2, st);
        MDP_HIP(hipMemcpyAsync(&hf, fl, sizeof(Flags), hipMemcpyDeviceToHost, st));
        MDP_HIP(hipStreamSynchronize(st));
        if (hf.badcol & 2) throw Error(MDP_ERR_NONFINITE, "non-finite entry in the interface matrix");
        if (hf.badcol & 1) throw Error(MDP_ERR_SINGULAR, "zero column in the interface matrix");
        if (!hf.info) break;
        if (attempt == 1) throw Error(MDP_ERR_SINGULAR, "interface least squares: Cholesky-QR broke down");
        // numerically indefinite Gram matrix: shifted first pass and one extra pass
        const double u = 1.1102230246251565e-16;
        shift = 11.0 * ((double)m * nc + (double)nc * (nc + 1)) * u * (double)nc;
        passes = 3;
    }
    res.shifted = shift != 0.0;
    res.passes = passes;
    res.rel_residual = std::sqrt(hf.r2) / (hf.f2 > 0 ? std::sqrt(hf.f2) : 1.0);

    // unscale: c = x / norms
    launch_scale_cols(xv, 1, nc, 1, w.norms.as<double>(), 1, st);
    MDP_HIP(hipMemcpyAsync(x_out, xv, nc * sizeof(double2), hipMemcpyDeviceToDevice, st));

    if (want_cond) {
        // power iterations: sigma_max(A0)^2 on A0^* A0, 1/sigma_min^2 on R^{-1} R^{-*}
        std::vector<double2> hv(nc);
        for (int i = 0; i < nc; ++i) hv[i] = make_double2(1.0 + 0.001 * (i % 7), 0.37 * ((i * 13) % 5));
        double2* v = s3;
        MDP_HIP(hipMemcpyAsync(v, hv.data(), nc * sizeof(double2), hipMemcpyHostToDevice, st));
        launch_znormalize(nc, v, &fl->pw[0], st);
        for (int it = 0; it < 12; ++it) {
            launch_zgemm('N', 'N', m, 1, nc, ONE, w.A0.as<double2>(), m, v, nc, ZERO, t, m, ws.zg, st);
            launch_zgemm('C', 'N', nc, 1, m, ONE, w.A0.as<double2>(), m, t, m, ZERO, v, nc, ws.zg, st);
            launch_znormalize(nc, v, &fl->pw[0], st);
        }
        MDP_HIP(hipMemcpyAsync(v, hv.data(), nc * sizeof(double2), hipMemcpyHostToDevice, st));
        launch_znormalize(nc, v, &fl->pw[1], st);
        for (int it = 0; it < 12; ++it) {
            // v <- R^{-1} R^{-*} v with R^{-*} = Linv_{p-1} ... Linv_0 (Linv_0 applied first)
            const double2* src = v;
            double2* bufs[2] = {y, z};
            int tt = 0;
            for (int p = 0; p < passes; ++p) {
                launch_zgemm('N', 'N', nc, 1, nc, ONE, w.Linv[p].as<double2>(), nc, src, nc, ZERO, bufs[tt], nc,
                             ws.zg, st);
                src = bufs[tt];
                tt ^= 1;
            }
            apply_rinv(passes, src, v, false);
            launch_znormalize(nc, v, &fl->pw[1], st);
        }
        MDP_HIP(hipMemcpyAsync(&hf, fl, sizeof(Flags), hipMemcpyDeviceToHost, st));
        MDP_HIP(hipStreamSynchronize(st));
        res.cond = std::sqrt(hf.pw[0] * hf.pw[1]);
    }
    return res;
}


// ---------------------------------------------------------------------------
// Block-sparse interface least squares (default path).
//
// Qbar is kept as one dense block per subdomain (its rows touch only that
// subdomain's unknown blocks).  R is the Cholesky factor of the Gram matrix
// Qbar^* Qbar = sum_i scatter(A_i^* A_i) -- the same R as in Qbar = Q R -- and
// the solution is c = R^{-1} R^{-*} Qbar^* Fbar = R^{-1} Q^* Fbar, followed by
// iterative refinement with the same factor (corrected semi-normal equations,
// Bjorck): each step r = Fbar - Qbar c, c += R^{-1} R^{-*} Qbar^* r.  When the
// columns are equilibrated and cond(Qbar) is moderate the corrected solution is
// as accurate as a Householder least-squares solution; the caller falls back to
// the dense Cholesky-QR passes when the Cholesky breaks down or the refinement
// does not contract.
namespace {

struct PackedFlags {
    int info;
    int badcol;
    double r2, f2, x2, dx2;
    double pw[2];
};

}  // namespace

// ---------------------------------------------------------------------------
// Multifrontal route (many subdomains).  The Gram matrix sum_i A_i^* A_i couples
// two unknowns only when one subdomain touches both, so with the unknowns of
// each half of the subdomains eliminated before those of the interfaces between
// the halves (nested dissection over the subdomain layout) the Cholesky factor
// keeps the block structure of the tree: each node holds the dense partial
// factorisation of its front (its eliminated columns and the columns it shares
// with subdomains outside it), and passes the Schur complement on the shared
// columns to its parent.
MFHost mf_plan(const PackedHost& h) {
    MFHost t;
    const int ns = h.n_sub, nc = h.nc;
    if ((int)h.cx.size() != ns || (int)h.cy.size() != ns) throw Error(MDP_ERR_ARG, "subdomain centres missing");
    // subdomains touching each column (at most two)
    std::vector<std::array<int, 2>> touch(nc, std::array<int, 2>{-1, -1});
    std::vector<std::vector<int>> subcols(ns);
    for (int pc = 0; pc < h.total_pc; ++pc) {
        const int g = h.pc_gcol[pc], s = h.pc_sub[pc];
        std::array<int, 2>& tt = touch[g];
        if (tt[0] < 0 || tt[0] == s) tt[0] = s;
        else if (tt[1] < 0 || tt[1] == s) tt[1] = s;
        else throw Error(MDP_ERR_ARG, "an interface unknown touches more than two subdomains");
        subcols[s].push_back(g);
    }
    for (auto& v : subcols) {
        std::sort(v.begin(), v.end());
        if (std::adjacent_find(v.begin(), v.end()) != v.end())
            throw Error(MDP_ERR_ARG, "a subdomain holds one unknown twice");
    }
    // the tree: halves along the longer extent of the centres, one subdomain per leaf
    std::vector<int> order(ns), parent, depth, leaf_of(ns, -1);
    for (int i = 0; i < ns; ++i) order[i] = i;
    std::vector<MFHost::Node>& nodes = t.nodes;
    std::function<int(int, int, int)> build = [&](int lo, int hi, int dep) -> int {
        const int v = (int)nodes.size();
        nodes.emplace_back();
        parent.push_back(-1);
        depth.push_back(dep);
        if (hi - lo == 1) {
            nodes[v].sub = order[lo];
            leaf_of[order[lo]] = v;
            return v;
        }
        double x0 = std::numeric_limits<double>::infinity(), x1 = -x0, y0 = x0, y1 = -x0;
        for (int i = lo; i < hi; ++i) {
            x0 = std::min(x0, h.cx[order[i]]); x1 = std::max(x1, h.cx[order[i]]);
            y0 = std::min(y0, h.cy[order[i]]); y1 = std::max(y1, h.cy[order[i]]);
        }
        const bool byx = (x1 - x0) >= (y1 - y0);
        std::stable_sort(order.begin() + lo, order.begin() + hi, [&](int a, int b) {
            return byx ? std::make_pair(h.cx[a], h.cy[a]) < std::make_pair(h.cx[b], h.cy[b])
                       : std::make_pair(h.cy[a], h.cx[a]) < std::make_pair(h.cy[b], h.cx[b]);
        });
        const int mid = lo + (hi - lo) / 2;
        const int k0 = build(lo, mid, dep + 1);
        const int k1 = build(mid, hi, dep + 1);
        parent[k0] = parent[k1] = v;
        nodes[v].kid[0] = k0;
        nodes[v].kid[1] = k1;
        nodes[v].height = 1 + std::max(nodes[k0].height, nodes[k1].height);
        return v;
    };
    build(0, ns, 0);
    const int nn = (int)nodes.size();
    auto lca = [&](int a, int b) {
        while (depth[a] > depth[b]) a = parent[a];
        while (depth[b] > depth[a]) b = parent[b];
        while (a != b) { a = parent[a]; b = parent[b]; }
        return a;
    };
    std::vector<std::vector<int>> elim(nn), bnd(nn);
    for (int g = 0; g < nc; ++g) {
        if (touch[g][0] < 0) throw Error(MDP_ERR_ARG, "an unknown touches no subdomain");
        const int v = touch[g][1] < 0 ? leaf_of[touch[g][0]] : lca(leaf_of[touch[g][0]], leaf_of[touch[g][1]]);
        elim[v].push_back(g);
    }
    // boundary columns, children before parents (nodes were created parents first)
    std::vector<int> posg(nc, -1), pgl(nc, -1);
    for (int v = nn - 1; v >= 0; --v) {
        MFHost::Node& nd = nodes[v];
        std::vector<int> cand;
        if (nd.sub >= 0) {
            cand = subcols[nd.sub];
        } else {
            const std::vector<int>&a = bnd[nd.kid[0]], &b = bnd[nd.kid[1]];
            std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(cand));
        }
        std::set_difference(cand.begin(), cand.end(), elim[v].begin(), elim[v].end(), std::back_inserter(bnd[v]));
        if (cand.size() != bnd[v].size() + elim[v].size()) throw Error(MDP_ERR_ARG, "inconsistent elimination tree");
        nd.e = (int)elim[v].size();
        nd.b = (int)bnd[v].size();
        nd.idx = elim[v];
        nd.idx.insert(nd.idx.end(), bnd[v].begin(), bnd[v].end());
        const int f = nd.e + nd.b;
        for (int a = 0; a < f; ++a) posg[nd.idx[a]] = a;
        if (nd.sub >= 0) {
            const int s = nd.sub;
            for (int p = 0; p < h.s[s]; ++p) pgl[h.pc_gcol[h.pc_start[s] + p]] = p;
            nd.spos.resize(f);
            for (int a = 0; a < f; ++a) nd.spos[a] = pgl[nd.idx[a]];
            for (int p = 0; p < h.s[s]; ++p) pgl[h.pc_gcol[h.pc_start[s] + p]] = -1;
        } else {
            for (int c = 0; c < 2; ++c) {
                const std::vector<int>& kb = bnd[nd.kid[c]];
                nd.kpos[c].resize(kb.size());
                nd.inv[c].assign(f, -1);
                for (size_t r = 0; r < kb.size(); ++r) {
                    const int a = posg[kb[r]];
                    if (a < 0) throw Error(MDP_ERR_ARG, "inconsistent elimination tree");
                    nd.kpos[c][r] = a;
                    nd.inv[c][a] = (int)r;
                }
            }
        }
        for (int a = 0; a < f; ++a) posg[nd.idx[a]] = -1;
        if (nd.height >= (int)t.by_height.size()) t.by_height.resize(nd.height + 1);
        t.by_height[nd.height].push_back(v);
        t.max_f = std::max(t.max_f, f);
        t.max_e = std::max(t.max_e, nd.e);
        t.lds_fwd = std::max(t.lds_fwd, nd.e);   // the substitutions stage e or b values in LDS
        t.lds_bwd = std::max(t.lds_bwd, nd.b);
    }
    if (nodes[0].b != 0) throw Error(MDP_ERR_ARG, "inconsistent elimination tree");
    // factor arena: every front G (f x f), then per height the L, Z, W (f x e each) of its nodes
    // (cleared together before the height's steps), then the solve vectors z (e) and cw (b)
    size_t off = 0;
    auto take = [&](size_t n) { const size_t o = off; off += (n + 15) / 16 * 16; return o; };
    for (MFHost::Node& nd : nodes) nd.G = take((size_t)(nd.e + nd.b) * (nd.e + nd.b));
    for (const auto& hv : t.by_height) {
        int me = 0, mb = 0;
        for (int v : hv) { me = std::max(me, nodes[v].e); mb = std::max(mb, nodes[v].b); }
        t.h_max_e.push_back(me);
        t.h_max_b.push_back(mb);
        t.lzw.push_back(off);
        for (int v : hv) {
            MFHost::Node& nd = nodes[v];
            const size_t fe = (size_t)(nd.e + nd.b) * nd.e;
            nd.L = take(fe);
            nd.Z = take(fe);
            nd.W = take(fe);
        }
    }
    t.lzw.push_back(off);
    for (MFHost::Node& nd : nodes) {
        nd.z = take(nd.e);
        nd.cw = take(nd.b);
    }
    // batched steps: panel s of every front of a height with more than 64 s eliminated columns
    for (size_t hh = 0; hh < t.by_height.size(); ++hh) {
        int max_e = 0;
        for (int v : t.by_height[hh]) max_e = std::max(max_e, nodes[v].e);
        for (int kb = 0; kb < max_e; kb += 64) {
            MFHost::Step sp{(int)hh, (int)t.entry_node.size(), 0, 0, 0, 0, 0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int v : t.by_height[hh]) {
                const MFHost::Node& nd = nodes[v];
                if (nd.e <= kb) continue;
                const int f = nd.e + nd.b, w = std::min(64, nd.e - kb), rest = f - kb - w;
                const int np = (rest + 31) / 32, nz = (kb + 31) / 32;
                t.entry_node.push_back(v);
                t.entry_kb.push_back(kb);
                ++sp.count;
                sp.max_roles = std::max(sp.max_roles, np + nz);
                sp.max_tiles64 = std::max(sp.max_tiles64, chol_update_tiles(f, kb, w, 64));
                sp.max_tiles32 = std::max(sp.max_tiles32, chol_update_tiles(f, kb, w, 32));
                sp.tiles64 += chol_update_tiles(f, kb, w, 64);
                const double W_ = w, R_ = rest, K_ = kb;
                sp.diag_flops += 8.0 / 3.0 * W_ * W_ * W_;
                sp.diag_bytes += 16.0 * 2.0 * W_ * W_;
                sp.panel_flops += 8.0 * R_ * W_ * W_ + 8.0 * K_ * W_ * W_;
                sp.panel_bytes += 16.0 * (W_ * W_ + R_ * W_ + 2.0 * K_ * W_);
                sp.update_flops += 4.0 * R_ * R_ * W_ + 8.0 * R_ * (K_ + W_) * W_;
                sp.update_bytes += 16.0 * (R_ * R_ + 2.0 * R_ * W_ + 2.0 * R_ * (K_ + W_));
            }
            t.steps.push_back(sp);
        }
    }
    t.arena = off;
    return t;
}

PackedTables ls_packed_tables(Workspace& ws, const PackedHost& h, HostBlob& blob) {
    PackedWork& w = ws.pk;
    const int nc = h.nc, n_sub = h.n_sub;
    long mtot = 0, ptot = 0;
    for (int i = 0; i < n_sub; ++i) { mtot += h.m[i]; ptot += (long)h.m[i] * h.s[i]; }
    grow(w.Ap, (size_t)ptot * sizeof(double2));
    LSWork& lw = ws.ls;
    if (h.multifrontal) {
        // the factor arena
        grow(w.mf, std::max<size_t>(h.mf.arena, 1) * sizeof(double2));
    } else {
        const size_t nn = (size_t)nc * nc;
        grow(lw.G, nn * sizeof(double2));
        grow(lw.L, nn * sizeof(double2));
        grow(lw.Linv[0], nn * sizeof(double2));
        grow(lw.T, nn * sizeof(double2));
    }
    grow(lw.vec, (size_t)(6 * nc + 2 * mtot) * sizeof(double2));
    grow(lw.norms, 2 * (size_t)nc * sizeof(double));
    grow(lw.flags, 64);
    grow(lw.rp, std::max<size_t>((size_t)h.total_pc * packed_slabs(h.max_m), 1) * sizeof(double2));
    PackedTables t{};
    t.Q = blob.put(h.Q);
    t.m = blob.put(h.m);
    t.s = blob.put(h.s);
    t.off = blob.put(h.off);
    t.roff = blob.put(h.roff);
    t.sub = blob.put(h.pc_sub);
    t.p = blob.put(h.pc_p);
    t.gcol = blob.put(h.pc_gcol);
    t.start = blob.put(h.pc_start);
    t.cols = blob.put(h.pc_cols);
    t.coef = blob.put(h.pc_coef);
    {
        std::vector<int> gs(nc + 1, 0), gl(h.total_pc);
        for (int pc = 0; pc < h.total_pc; ++pc) ++gs[h.pc_gcol[pc] + 1];
        for (int g = 0; g < nc; ++g) gs[g + 1] += gs[g];
        std::vector<int> fill(gs.begin(), gs.end() - 1);
        for (int pc = 0; pc < h.total_pc; ++pc) gl[fill[h.pc_gcol[pc]]++] = pc;
        t.gc_start = blob.put(gs);
        t.gc_list = blob.put(gl);
    }
    // all subdomains' A_i^* A_i in one split-K launch (reduced and scattered in a second)
    int max_m = 0, tiles = 0;
    for (int i = 0; i < n_sub; ++i) {
        max_m = std::max(max_m, h.m[i]);
        tiles += ((h.s[i] + kGramTile - 1) / kGramTile) * ((h.s[i] + kGramTile - 1) / kGramTile);
    }
    const int nsplit = std::max(1, std::min(std::min(2048 / std::max(tiles, 1), std::max(1, max_m / 128)), 64));
    std::vector<ZBatch> zb(n_sub);
    double2* Ap = w.Ap.as<double2>();
    long poff = 0;
    for (int i = 0; i < n_sub; ++i) {
        int kchunk = (h.m[i] + nsplit - 1) / nsplit;
        kchunk = std::max(16, (kchunk + 15) / 16 * 16);
        zb[i] = ZBatch{Ap + h.off[i], h.s[i], h.m[i], kchunk, h.pc_start[i], poff};
        poff += (long)nsplit * h.s[i] * h.s[i];
    }
    grow(ws.zg, (size_t)std::max(poff, 1L) * sizeof(double2));
    t.zb = blob.put(zb);
    t.nsplit = nsplit;
    if (h.multifrontal) {
        const MFHost& mf = h.mf;
        std::vector<MFNodeDev> nd(mf.nodes.size());
        for (size_t v = 0; v < mf.nodes.size(); ++v) {
            const MFHost::Node& a = mf.nodes[v];
            MFNodeDev& o = nd[v];
            o.e = a.e;
            o.b = a.b;
            o.f = a.e + a.b;
            o.leaf = a.sub >= 0;
            o.idx = (long)blob.put(a.idx);
            o.G = (long)a.G; o.L = (long)a.L; o.Z = (long)a.Z; o.W = (long)a.W;
            o.z = (long)a.z; o.cw = (long)a.cw;
            o.kid0 = a.kid[0];
            o.kid1 = a.kid[1];
            if (o.leaf) {
                const ZBatch& z = zb[a.sub];
                o.n = z.n;
                o.nsplit = nsplit;
                o.pstride = (long)z.n * z.n;
                o.poff = z.poff;
                o.spos = (long)blob.put(a.spos);
            } else {
                o.inv0 = (long)blob.put(a.inv[0]);
                o.inv1 = (long)blob.put(a.inv[1]);
                o.kpos0 = (long)blob.put(a.kpos[0]);
                o.kpos1 = (long)blob.put(a.kpos[1]);
            }
        }
        t.mf_nodes = blob.put(nd);
        std::vector<int> lists;
        t.mf_list_off.clear();
        for (const auto& hv : mf.by_height) {
            t.mf_list_off.push_back(lists.size());
            lists.insert(lists.end(), hv.begin(), hv.end());
        }
        t.mf_list_off.push_back(lists.size());
        t.mf_lists = blob.put(lists);
        double2* arena = w.mf.as<double2>();
        std::vector<CholBatchEntry> ent(mf.entry_node.size());
        for (size_t q = 0; q < ent.size(); ++q) {
            const MFHost::Node& a = mf.nodes[mf.entry_node[q]];
            const int f = a.e + a.b, kb = mf.entry_kb[q], wd = std::min(64, a.e - kb), rest = f - kb - wd;
            const int np = (rest + 31) / 32;
            ent[q] = CholBatchEntry{arena + a.G, arena + a.L, arena + a.Z, arena + a.W, f, kb, wd, np, (kb + 31) / 32};
        }
        t.mf_steps = blob.put(ent);
    }
    return t;
}

LSResult ls_solve_packed(Workspace& ws, const PackedHost& h, const char* image, const PackedTables& tb,
                         const double2* F, double2* x_out, bool want_cond, hipStream_t st, bool* fallback,
                         bool reuse) {
    LSResult res{};
    *fallback = false;
    PackedWork& w = ws.pk;
    const int nc = h.nc, n_sub = h.n_sub, npc = h.total_pc;
    long mtot = 0;
    for (int i = 0; i < n_sub; ++i) mtot += h.m[i];
    LSWork& lw = ws.ls;
    const size_t nn = (size_t)nc * nc;
    auto at = [&](size_t off) { return image + off; };
    PackedDevice d{reinterpret_cast<const double2* const*>(at(tb.Q)), reinterpret_cast<const int*>(at(tb.m)),
                   reinterpret_cast<const long*>(at(tb.off)), reinterpret_cast<const int*>(at(tb.s)),
                   reinterpret_cast<const int*>(at(tb.sub)), reinterpret_cast<const int*>(at(tb.p)),
                   reinterpret_cast<const int*>(at(tb.gcol)), reinterpret_cast<const int4*>(at(tb.cols)),
                   reinterpret_cast<const double2*>(at(tb.coef)), reinterpret_cast<const long*>(at(tb.roff)),
                   reinterpret_cast<const int*>(at(tb.start)), reinterpret_cast<const int*>(at(tb.gc_start)),
                   reinterpret_cast<const int*>(at(tb.gc_list))};
    double2* Ap = w.Ap.as<double2>();
    double* norms2 = lw.norms.as<double>();
    double* norms = norms2 + nc;
    double2* y = lw.vec.as<double2>();
    double2* t = y + nc;
    double2* x = x_out;   // the solution is refined in place
    double2* dx = t + 2 * nc;
    double2* v1 = dx + nc;
    double2* v2 = v1 + nc;
    double2* r = v2 + nc;
    PackedFlags* fl = lw.flags.as<PackedFlags>();
    const bool mfr = h.multifrontal;
    double2* G = mfr ? nullptr : lw.G.as<double2>();
    double2* L = lw.L.as<double2>();
    double2* Linv = mfr ? nullptr : lw.Linv[0].as<double2>();
    const MFNodeDev* mf_nodes = mfr ? reinterpret_cast<const MFNodeDev*>(at(tb.mf_nodes)) : nullptr;
    const int* mf_lists = mfr ? reinterpret_cast<const int*>(at(tb.mf_lists)) : nullptr;
    double2* arena = mfr ? w.mf.as<double2>() : nullptr;

    MDP_HIP(hipMemsetAsync(fl, 0, sizeof(PackedFlags), st));
    double chol_flops = 0.0;
    if (!reuse) {
        // packed blocks, equilibrated columns (norms from Q, then one assembling pass)
        MDP_HIP(hipMemsetAsync(norms2, 0, nc * sizeof(double), st));
        launch_packed_colnorm2(d, npc, norms2, st);
        launch_finalize_norms(nc, norms2, norms, &fl->badcol, st);
        launch_assemble_packed(d, npc, h.max_m, norms, Ap, st);
        // Gram matrix (multifrontal: the per-subdomain blocks stay apart)
        if (!mfr) MDP_HIP(hipMemsetAsync(G, 0, nn * sizeof(double2), st));
        {
            int max_m = 0;
            double gram_flops = 0.0, gram_bytes = 0.0;
            for (int i = 0; i < n_sub; ++i) {
                max_m = std::max(max_m, h.m[i]);
                gram_flops += 4.0 * h.m[i] * (double)h.s[i] * (h.s[i] + 1);   // lower half of A_i^* A_i
                gram_bytes += 16.0 * h.m[i] * (double)h.s[i];
            }
            ws.prof.run("gram", st, gram_flops, gram_bytes, [&] {
                launch_gram_batched(reinterpret_cast<const ZBatch*>(at(tb.zb)), n_sub, h.max_s, max_m, tb.nsplit,
                                    ws.zg.as<double2>(), d.pc_gcol, G, nc, st);
            });
        }
        if (!mfr) {
            chol_flops = cholesky_and_inverse(G, L, Linv, lw.T.as<double2>(), &fl->info, nc, 0.0, st, &ws.prof,
                                              h.steps.empty() ? nullptr : &h.steps);
        } else {
            // children before parents: assemble every front of one height, then factor the first e columns
            // of all its fronts together, one batched panel and one batched update launch per 64 columns
            // (the panel rows below the eliminated block are L21, the trailing update leaves
            // F22 - L21 L21^* in G(e:, e:))
            const MFHost& mf = h.mf;
            const CholBatchEntry* ent = reinterpret_cast<const CholBatchEntry*>(image + tb.mf_steps);
            size_t si = 0;
            for (size_t hh = 0; hh < mf.by_height.size(); ++hh) {
                const std::vector<int>& lv = mf.by_height[hh];
                int mxf = 0;
                double abytes = 0.0;
                for (int v : lv) {
                    const int f = mf.nodes[v].e + mf.nodes[v].b;
                    mxf = std::max(mxf, f);
                    abytes += 32.0 * f * f;
                }
                if (mf.lzw[hh + 1] > mf.lzw[hh])
                    MDP_HIP(hipMemsetAsync(arena + mf.lzw[hh], 0, (mf.lzw[hh + 1] - mf.lzw[hh]) * sizeof(double2), st));
                ws.prof.run("mf_assemble", st, 0.0, abytes, [&] {
                    launch_mf_assemble(mf_nodes, mf_lists + tb.mf_list_off[hh], (int)lv.size(), mxf, image,
                                       ws.zg.as<double2>(), arena, st);
                });
                for (; si < mf.steps.size() && mf.steps[si].height == (int)hh; ++si) {
                    const MFHost::Step& sp = mf.steps[si];
                    ws.prof.run("chol_diag", st, sp.diag_flops, sp.diag_bytes, [&] {
                        launch_chol_diag_batched(ent + sp.entry0, sp.count, &fl->info, st);
                    });
                    if (sp.max_roles > 0)
                        ws.prof.run("chol_panel", st, sp.panel_flops, sp.panel_bytes, [&] {
                            launch_chol_slabs_batched(ent + sp.entry0, sp.count, sp.max_roles, st);
                        });
                    ws.prof.run("chol_update", st, sp.update_flops, sp.update_bytes, [&] {
                        launch_chol_update_batched(ent + sp.entry0, sp.count, sp.max_tiles64, sp.tiles64,
                                                   sp.max_tiles32, st);
                    });
                    chol_flops += sp.diag_flops + sp.panel_flops + sp.update_flops;
                }
            }
        }
    }
    // G^{-1} y (multifrontal): forward through the tree, children first, then back from the root
    auto mf_solve = [&](const double2* yv, double2* out) {
        const MFHost& mf = h.mf;
        const int H = (int)mf.by_height.size();
        ws.prof.run("mf_solve", st, 0.0, 0.0, [&] {
            for (int hh = 0; hh < H; ++hh)
                launch_mf_solve(mf_nodes, mf_lists + tb.mf_list_off[hh], (int)mf.by_height[hh].size(), mf.h_max_e[hh],
                                mf.h_max_b[hh], true, image, arena, yv, nullptr, st);
            for (int hh = H - 1; hh >= 0; --hh)
                launch_mf_solve(mf_nodes, mf_lists + tb.mf_list_off[hh], (int)mf.by_height[hh].size(), mf.h_max_e[hh],
                                mf.h_max_b[hh], false, image, arena, nullptr, out, st);
        });
    };
    // algorithmic flops: Gram (lower half), factor + inverse, and per normal solve (A^* v plus two
    // triangular products) or residual (A x): 8 flops per complex multiply-add
    double packed_cmacs = 0.0, gram_cmacs = 0.0;
    for (int i = 0; i < n_sub; ++i) {
        packed_cmacs += (double)h.m[i] * h.s[i];
        gram_cmacs += 0.5 * (double)h.m[i] * h.s[i] * (h.s[i] + 1);
    }
    double tri_cmacs = (double)nc * nc;   // two triangular products with Linv (dense)
    if (mfr) {
        tri_cmacs = 0.0;
        for (const MFHost::Node& nd : h.mf.nodes) tri_cmacs += (double)nd.e * nd.e + 2.0 * nd.b * nd.e;
    }
    const double solve_flops = 8.0 * (packed_cmacs + tri_cmacs), resid_flops = 8.0 * packed_cmacs;
    int n_solves = 0, n_resid = 0;
    // c = R^{-1} R^{-*} Qbar^* F, R^{-1} = Linv^*, R^{-*} = Linv
    // (every product below overwrites its output and sums in a fixed order, so the
    // sequence needs no clearing launches and repeats bit for bit)
    auto apply_inverse = [&](double2* out) {   // out = G^{-1} y
        if (mfr) {
            mf_solve(y, out);
            return;
        }
        launch_trmv_lower('N', nc, Linv, nc, y, t, st);
        launch_trmv_lower('C', nc, Linv, nc, t, out, st);
    };
    auto normal_solve = [&](const double2* rhs_rows, double2* out) {
        ++n_solves;
        launch_packed_ahx_set(d, nc, Ap, rhs_rows, y, st);
        apply_inverse(out);
    };
    // r = F - Qbar x (stacked rows); norms: ||r||^2, ||F||^2 into r2, f2; clr: accumulators to zero
    auto residual = [&](double* norms, double* clr) {
        ++n_resid;
        launch_packed_axpy(d, n_sub, h.max_m, Ap, x, MONE, F, r, norms, clr, st);
    };
    normal_solve(F, x);
    // refinement steps; the last correction's norm and the solution's norm are
    // measured so the host can decide on convergence (each step contracts the error
    // by about cond(Qbar)^2 u).  The last step's residual launch clears x2 and dx2
    // (adjacent), its update accumulates them and clears r2 and f2 (adjacent) for
    // the residual norms that follow.
    // A refinement step's residual and its product A^* r come from one pass over the packed matrix.
    auto refine = [&](int steps) {
        for (int it = 0; it < steps; ++it) {
            const bool last = it == steps - 1;
            ++n_resid;
            ++n_solves;
            launch_packed_resid_ahx(d, n_sub, h.max_m, h.max_s, nc, Ap, x, F, lw.rp.as<double2>(), y,
                                    last ? &fl->x2 : nullptr, st);
            apply_inverse(dx);
            launch_zaxpy_norms(nc, dx, x, last ? &fl->x2 : nullptr, last ? &fl->r2 : nullptr, st);
        }
    };
    PackedFlags hf{};
    PackedFlags* hpin = static_cast<PackedFlags*>(lw.hflags.get(sizeof(PackedFlags)));
    const bool verbose = std::getenv("MDP_VERBOSE") != nullptr;
    auto read_flags = [&]() {
        MDP_HIP(hipMemcpyAsync(hpin, fl, sizeof(PackedFlags), hipMemcpyDeviceToHost, st));
        MDP_HIP(hipStreamSynchronize(st));
        hf = *hpin;
        if (verbose)
            std::fprintf(stderr, "mdp: least squares after %d normal solves: |dx|/|x| %.3e, residual %.3e\n", n_solves,
                         std::sqrt(hf.dx2 / (hf.x2 > 0 ? hf.x2 : 1.0)), std::sqrt(hf.r2 / (hf.f2 > 0 ? hf.f2 : 1.0)));
        if (hf.badcol & 2) throw Error(MDP_ERR_NONFINITE, "non-finite entry in the interface matrix");
        if (hf.badcol & 1) throw Error(MDP_ERR_SINGULAR, "zero column in the interface matrix");
    };
    auto converged = [&]() { return !hf.info && hf.dx2 <= 1e-22 * hf.x2; };
    // the residual norms of the refined solution go to the host with the convergence data
    auto residual_norms = [&]() { residual(&fl->r2, nullptr); };
    refine(2);
    residual_norms();
    read_flags();
    if (!hf.info && !converged()) {
        // slower contraction (larger cond): continue while the corrections shrink
        double prev = hf.dx2;
        for (int round = 0; round < 3 && !converged(); ++round) {
            refine(2);
            residual_norms();
            read_flags();
            if (!(hf.dx2 < 0.25 * prev)) break;   // not contracting: hand over
            prev = hf.dx2;
        }
    }
    // the last correction must be negligible; otherwise the Gram matrix is too ill-conditioned
    if (!converged()) {
        if (std::getenv("MDP_VERBOSE"))
            std::fprintf(stderr, "mdp: semi-normal least squares handed over (pivot failure %d, |dx|/|x| %.3e)\n",
                         hf.info, std::sqrt(hf.dx2 / (hf.x2 > 0 ? hf.x2 : 1.0)));
        *fallback = true;
        return res;
    }
    res.passes = 1;
    res.rel_residual = std::sqrt(hf.r2) / (hf.f2 > 0 ? std::sqrt(hf.f2) : 1.0);
    res.flops = (reuse ? 0.0 : 8.0 * gram_cmacs) + chol_flops + n_solves * solve_flops + n_resid * resid_flops;
    launch_scale_cols(x, 1, nc, 1, norms, 1, st);
    if (want_cond) {
        // cond(Qbar_eq)^2 = lambda_max(G) lambda_max(G^{-1}); G v = L (L^* v), G^{-1} v = Linv^* (Linv v)
        std::vector<double2> hv(nc);
        for (int i = 0; i < nc; ++i) hv[i] = make_double2(1.0 + 0.001 * (i % 7), 0.37 * ((i * 13) % 5));
        for (int which = 0; which < 2; ++which) {
            MDP_HIP(hipMemcpyAsync(v1, hv.data(), nc * sizeof(double2), hipMemcpyHostToDevice, st));
            launch_znormalize(nc, v1, &fl->pw[which], st);
            for (int it = 0; it < 16; ++it) {
                if (mfr) {
                    if (which == 0) {   // G v = A^* (A v)
                        MDP_HIP(hipMemsetAsync(r, 0, mtot * sizeof(double2), st));
                        launch_packed_ax(d, n_sub, h.max_m, h.max_s, Ap, v1, ONE, r, st);
                        MDP_HIP(hipMemsetAsync(v1, 0, nc * sizeof(double2), st));
                        launch_packed_ahx(d, npc, Ap, r, ONE, v1, st);
                    } else {
                        MDP_HIP(hipMemcpyAsync(v2, v1, nc * sizeof(double2), hipMemcpyDeviceToDevice, st));
                        mf_solve(v2, v1);
                    }
                } else if (which == 0) {
                    launch_zgemm('C', 'N', nc, 1, nc, ONE, L, nc, v1, nc, ZERO, v2, nc, ws.zg, st);
                    launch_zgemm('N', 'N', nc, 1, nc, ONE, L, nc, v2, nc, ZERO, v1, nc, ws.zg, st);
                } else {
                    launch_zgemm('N', 'N', nc, 1, nc, ONE, Linv, nc, v1, nc, ZERO, v2, nc, ws.zg, st);
                    launch_zgemm('C', 'N', nc, 1, nc, ONE, Linv, nc, v2, nc, ZERO, v1, nc, ws.zg, st);
                }
                launch_znormalize(nc, v1, &fl->pw[which], st);
            }
        }
        MDP_HIP(hipMemcpyAsync(hpin, fl, sizeof(PackedFlags), hipMemcpyDeviceToHost, st));
        MDP_HIP(hipStreamSynchronize(st));
        hf = *hpin;
        res.cond = std::sqrt(hf.pw[0] * hf.pw[1]);
    }
    return res;
}

// G^{-1} v with the factor of the last ls_solve_packed on these workspaces (the Gram
// matrix of the column-equilibrated packed matrix; out may not alias v).
void ls_packed_factor_solve(Workspace& ws, const PackedHost& h, const char* image, const PackedTables& tb,
                            const double2* v, double2* out, hipStream_t st) {
    const int nc = h.nc;
    if (h.multifrontal) {
        const MFHost& mf = h.mf;
        const MFNodeDev* nodes = reinterpret_cast<const MFNodeDev*>(image + tb.mf_nodes);
        const int* lists = reinterpret_cast<const int*>(image + tb.mf_lists);
        double2* arena = ws.pk.mf.as<double2>();
        const int H = (int)mf.by_height.size();
        for (int hh = 0; hh < H; ++hh)
            launch_mf_solve(nodes, lists + tb.mf_list_off[hh], (int)mf.by_height[hh].size(), mf.h_max_e[hh],
                            mf.h_max_b[hh], true, image, arena, v, nullptr, st);
        for (int hh = H - 1; hh >= 0; --hh)
            launch_mf_solve(nodes, lists + tb.mf_list_off[hh], (int)mf.by_height[hh].size(), mf.h_max_e[hh],
                            mf.h_max_b[hh], false, image, arena, nullptr, out, st);
        return;
    }
    LSWork& lw = ws.ls;
    double2* t = lw.vec.as<double2>() + nc;   // the normal solve's own temporary
    const double2* Linv = lw.Linv[0].as<double2>();
    launch_trmv_lower('N', nc, Linv, nc, v, t, st);
    launch_trmv_lower('C', nc, Linv, nc, t, out, st);
}

}  // namespace mdp
