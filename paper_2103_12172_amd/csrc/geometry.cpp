// Host geometry of one subdomain: auxiliary grid, grid sets, gamma, side map
// and the equation-based extension matrix.
//
// Paper Sec. 3.2.2 (grid sets), Sec. 3.2.3 (extension, eqs. general_extension
// and cartesian_extension with f = 0), Sec. 3.2.4 (Chebyshev basis per side,
// eq. Psi_def).
#include <algorithm>
#include <cmath>

#include "mdp_internal.h"

namespace mdp {

Fold Fold::make(int n) {
    Fold f;
    f.n = n;
    f.p = n / 2;
    auto up = [](int v, int a) { return (v + a - 1) / a * a; };
    f.P1 = up(f.p, 64);
    f.P2 = up(std::max(f.p - 1, 1), 64);
    f.W = f.P1 + f.P2;
    return f;
}

// The auxiliary domain is the square of side 1.1*max(lx, ly) centred on the
// rectangle; n cells per direction.  M+ holds the nodes of M0 (not on the
// auxiliary boundary) inside the closed rectangle; since the rectangle is
// axis-aligned this is an index box.  gamma = N+ intersect N- is the two-node
// ring around the boundary of that box: the box grown by one node minus the
// box shrunk by one node.
Geometry make_geometry(double x0, double y0, double lx, double ly, int n) {
    if (!(lx > 0) || !(ly > 0) || !std::isfinite(x0) || !std::isfinite(y0) || !std::isfinite(lx) ||
        !std::isfinite(ly))
        throw Error(MDP_ERR_ARG, "subdomain rectangle must be finite with positive sides");
    if (n < 8 || (n & 1)) throw Error(MDP_ERR_ARG, "n must be even and >= 8");
    Geometry g;
    g.x0 = x0; g.y0 = y0; g.lx = lx; g.ly = ly; g.n = n;
    g.L = 1.1 * std::max(lx, ly);
    g.h = g.L / n;
    g.xa = (x0 + 0.5 * lx) - 0.5 * g.L;
    g.ya = (y0 + 0.5 * ly) - 0.5 * g.L;
    auto box = [&](double a, double lo, double len, int& ilo, int& ihi) {
        ilo = n; ihi = -1;
        for (int i = 1; i <= n - 1; ++i) {
            double v = a + i * g.h;
            if (v >= lo && v <= lo + len) { ilo = std::min(ilo, i); ihi = std::max(ihi, i); }
        }
    };
    box(g.xa, x0, lx, g.m_lo, g.m_hi);
    box(g.ya, y0, ly, g.q_lo, g.q_hi);
    if (g.m_hi < g.m_lo || g.q_hi < g.q_lo)
        throw Error(MDP_ERR_ARG, "the subdomain contains no interior grid node; increase n");
    if (g.m_lo < 2 || g.q_lo < 2 || g.m_hi > n - 2 || g.q_hi > n - 2)
        throw Error(MDP_ERR_ARG, "gamma would touch the auxiliary boundary; increase n");

    const double xr = x0 + lx, yt = y0 + ly, tol = 1e-9 * g.h;
    for (int m = g.m_lo - 1; m <= g.m_hi + 1; ++m) {
        for (int q = g.q_lo - 1; q <= g.q_hi + 1; ++q) {
            bool inner = (m > g.m_lo && m < g.m_hi && q > g.q_lo && q < g.q_hi);
            if (inner) continue;
            double x = g.xa + m * g.h, y = g.ya + q * g.h;
            double rb = y0 - y, rt = y - yt, rl = x0 - x, rr = x - xr;
            double vb = std::max(rl, rr), hb = std::max(rb, rt);
            int s;
            double r;
            if (vb >= hb - tol) { s = (rl >= rr) ? 2 : 3; r = (s == 2) ? rl : rr; }
            else { s = (rb >= rt) ? 0 : 1; r = (s == 0) ? rb : rt; }
            g.gm.push_back(m);
            g.gq.push_back(q);
            g.gmq.push_back(m);
            g.gmq.push_back(q);
            g.side.push_back(s);
            g.rho.push_back(r);
            bool horiz = (s == 0 || s == 1);
            g.t.push_back(horiz ? 2.0 * (x - x0) / lx - 1.0 : 2.0 * (y - y0) / ly - 1.0);
            g.slen.push_back(horiz ? lx : ly);
        }
    }
    g.n_gamma = (int)g.gm.size();
    return g;
}

}  // namespace mdp
