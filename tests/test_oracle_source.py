"""Pins of the oracle's source-term pieces (paper Sec. 3.2.1-3.2.5 with f != 0).

Each check is fixed by the mathematics or by the paper's printed errors, not by
the oracle's own formulas: the scheme's consistency with its right-hand side
B^(h) f (4th order), the fifth-order accuracy of the extension with its
inhomogeneous part, the discrete BEP with a source (exact up to rounding), and
the convergence of the whole solve on manufactured solutions and on the
inhomogeneous column of Table uniform_2.
"""
import json
import math
import os

import numpy as np

from paper_2103_12172_amd import workloads as wl
from oracle import grid as ogrid, projector, scheme, solve, source as osrc
from oracle.extension import extend_data

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def test_scheme_with_source_is_fourth_order():
    """L^(h) u - B^(h) f for u = exp(i(ax+by)), f = (k^2-a^2-b^2) u falls 16x per halving
    (dropping the 1/12 Laplacian of f would leave second order)."""
    k, a, b = 10.0, 6.0, 5.0
    u_fn, _, f_fn, _ = wl.manufactured_plane_wave(k, a, b)
    errs = []
    for n in (32, 64, 128, 256):
        h = 1.0 / n
        x = np.arange(n + 1) * h
        X, Y = np.meshgrid(x, x, indexing="ij")
        r = scheme.apply_L(u_fn(X, Y), h, k) - osrc.apply_B(f_fn(X, Y))
        errs.append(np.abs(r[1:-1, 1:-1]).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(14.0 < q < 18.5 for q in ratios), ratios


def test_extension_with_source_fifth_order():
    """|Ex(u, du/dn) - u| on gamma for a solution of Delta u + k^2 u = f falls ~32x per
    halving once Ex^(I) f is included (eqs. general_extension, cart_ext_2-4)."""
    k = 13.0
    u_fn, g_fn, f_fn, jet = wl.sin4_solution(k)
    errs, errs_h = [], []
    for n in (64, 128, 256):
        g = ogrid.APGrid(0.1, -0.2, 0.8, 0.7, n)
        x, y, nx, ny = osrc.foot_points(g)
        pi = math.pi
        # tangential derivatives of xi0 = u and xi1 = du/dn along the side, in closed form:
        # horizontal sides vary x, vertical sides vary y
        def dx(p, xx, yy):
            # d^p/dx^p sin^4(pi x) via sin^4 = (3 - 4 cos 2 pi x + cos 4 pi x)/8
            terms = [(3.0 / 8, 0.0), (-0.5, 2.0), (1.0 / 8, 4.0)]
            out = 0.0
            for amp, w in terms:
                if w == 0.0:
                    out = out + (amp if p == 0 else 0.0)
                else:
                    out = out + amp * (w * pi) ** p * np.cos(w * pi * xx + p * pi / 2)
            return out
        def dy(p, yy):
            return pi**p * np.sin(pi * yy + p * pi / 2)
        horiz = (g.side == 0) | (g.side == 1)
        a0 = np.where(horiz, dx(0, x, y) * dy(0, y), dx(0, x, y) * dy(0, y))
        a2 = np.where(horiz, dx(2, x, y) * dy(0, y), dx(0, x, y) * dy(2, y))
        a4 = np.where(horiz, dx(4, x, y) * dy(0, y), dx(0, x, y) * dy(4, y))
        # normal derivative and its second tangential derivative
        un = np.where(horiz, ny * dx(0, x, y) * dy(1, y), nx * dx(1, x, y) * dy(0, y))
        un2 = np.where(horiz, ny * dx(2, x, y) * dy(1, y), nx * dx(1, x, y) * dy(2, y))
        hom = extend_data(g, k, (a0, a2, a4), (un, un2))
        inh = osrc.extension_inhomogeneous(g, k, osrc.source_jet(g, jet))
        X = g.xs[g.gamma_m]
        Y = g.ys[g.gamma_q]
        exact = u_fn(X, Y)
        errs.append(np.abs(hom + inh - exact).max())
        errs_h.append(np.abs(hom - exact).max())
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    # at least fifth order (a wrong rho^3 term leaves third, a dropped k^2 f fourth order)
    assert all(q > 26.0 for q in ratios), ratios
    # without the inhomogeneous part the extension is only second order in h
    assert errs_h[-1] > 50 * errs[-1]


def test_bep_with_source_exact():
    """xi = trace of u with L^(h) u = B^(h) f on M+ satisfies P_gamma xi + Tr G B f = xi
    (eq. discrete_BEP with g = B f) to rounding; u from the AP with an arbitrary right-hand
    side outside M+."""
    g = ogrid.APGrid(0.0, 0.0, 1.0, 0.6, 32)
    k = 7.0
    rng = np.random.default_rng(3)
    fg = rng.standard_normal((33, 33)) + 1j * rng.standard_normal((33, 33))
    solver = scheme.make_solver(g.n, g.h, k)
    Bf = osrc.apply_B(fg)
    rhs = np.where(g.Mplus, Bf, 0.0) + np.where(g.Mminus, rng.standard_normal((33, 33)), 0.0)
    u = solver.solve(rhs)
    xi = u[g.gamma_m, g.gamma_q]
    gp = np.where(g.Mplus, Bf, 0.0)
    lhs = projector.projection(g, k, xi, solver) + solver.solve(gp)[g.gamma_m, g.gamma_q]
    assert np.abs(lhs - xi).max() < 1e-10 * np.abs(xi).max()
    # and the one-solve form of F agrees with its definition (I - P) Ex^(I) f - Tr G B f
    jv = tuple(rng.standard_normal(g.n_gamma) + 1j * rng.standard_normal(g.n_gamma) for _ in range(3))
    xi_i = osrc.extension_inhomogeneous(g, k, jv)
    F_def = xi_i - projector.projection(g, k, xi_i, solver) - solver.solve(gp)[g.gamma_m, g.gamma_q]
    F = osrc.system_rhs(g, k, fg, jv, solver)
    assert np.abs(F - F_def).max() < 1e-10 * np.abs(F_def).max()


def test_source_solve_fourth_order_manufactured():
    """End-to-end DD solve with a source: error vs exp(i(ax+by)) falls ~16x per halving."""
    errs = [solve.dd_solve(wl.config_source_plane(n=n))["info"]["error_max_Mplus"] for n in (32, 64, 128)]
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(14.0 < q < 18.5 for q in ratios), (errs, ratios)


def test_paper_inhomogeneous_column_reproduced():
    """sin^4(pi x) sin(pi y) on the two squares of Table uniform_2: same order of magnitude
    as the printed errors at n = 64, 128 and rate 4.0 +- 0.2."""
    gold = json.load(open(GOLDEN))["uniform_2_sin4"]
    ref = dict(zip(gold["n"], gold["error"]))
    errs = {n: solve.dd_solve(wl.config_paper_sin4(n=n))["info"]["error_max_Mplus"] for n in (64, 128)}
    for n in (64, 128):
        assert 0.1 < errs[n] / ref[n] < 10.0, (n, errs[n], ref[n])
    rate = math.log2(errs[64] / errs[128])
    assert abs(rate - 4.0) < 0.2, rate
