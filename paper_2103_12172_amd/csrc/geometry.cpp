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

// E(i, col) for gamma node i on side s, at signed distance rho, side parameter t:
//   Dirichlet column (xi0 = psi, xi1 = 0):
//     psi + rho^2/2 (-psi'' - k^2 psi) + rho^4/24 (psi'''' + 2 k^2 psi'' + k^4 psi)
//   Neumann column (xi0 = 0, xi1 = psi):
//     rho psi + rho^3/6 (-psi'' - k^2 psi)
// with psi = T_j(t) and tangential derivatives psi^(p) = (2/side length)^p T_j^(p)(t).
// T_j^(p) from the three-term recurrence differentiated p times:
//   T_{j+1}^(p) = 2 t T_j^(p) + 2 p T_j^(p-1) - T_{j-1}^(p).
std::vector<double> extension_matrix(const Geometry& g, double k, int m_star) {
    const int ng = g.n_gamma;
    std::vector<double> E((size_t)ng * 8 * m_star, 0.0);
    std::vector<double> T(5 * (size_t)m_star);
    const double k2 = k * k, k4 = k2 * k2;
    for (int i = 0; i < ng; ++i) {
        const double t = g.t[i];
        for (int p = 0; p <= 4; ++p) {
            double* Tp = &T[(size_t)p * m_star];
            const double* Tq = p ? &T[(size_t)(p - 1) * m_star] : nullptr;
            if (m_star > 0) Tp[0] = (p == 0) ? 1.0 : 0.0;
            if (m_star > 1) Tp[1] = (p == 0) ? t : (p == 1 ? 1.0 : 0.0);
            for (int j = 1; j + 1 < m_star; ++j) {
                double v = 2.0 * t * Tp[j] - Tp[j - 1];
                if (p) v += 2.0 * p * Tq[j];
                Tp[j + 1] = v;
            }
        }
        const double sc = 2.0 / g.slen[i], sc2 = sc * sc, sc4 = sc2 * sc2;
        const double r = g.rho[i], r2 = r * r, r3 = r2 * r, r4 = r2 * r2;
        const int s = g.side[i];
        for (int j = 0; j < m_star; ++j) {
            double p0 = T[j], p2 = sc2 * T[2 * (size_t)m_star + j], p4 = sc4 * T[4 * (size_t)m_star + j];
            double dcol = p0 + 0.5 * r2 * (-p2 - k2 * p0) + (r4 / 24.0) * (p4 + 2.0 * k2 * p2 + k4 * p0);
            double ncol = r * p0 + (r3 / 6.0) * (-p2 - k2 * p0);
            E[(size_t)(s * m_star + j) * ng + i] = dcol;
            E[(size_t)(4 * m_star + s * m_star + j) * ng + i] = ncol;
        }
    }
    return E;
}

}  // namespace mdp
