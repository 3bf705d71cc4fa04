"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks one part of the oracle against something other than the
oracle itself: closed forms, invariants of the difference potentials, brute
force on tiny grids, independent library routines, or the numbers the paper
prints.  No GPU is needed.
"""
import json
import math
import os

import numpy as np
import numpy.polynomial.chebyshev as npcheb
import pytest

from paper_2103_12172_amd import workloads as wl
from oracle import extension, grid as ogrid, interface, projector, scheme, solve

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


# ------------------------------------------------------------------ stencil
def test_stencil_consistency_constant_and_plane_wave():
    """Sum of the 9 weights is k^2 (L^(h) of a constant); the truncation error on
    a plane wave with xi^2 + eta^2 = k^2 falls ~16x per halving of h (4th order)."""
    k = 13.0
    for h in (0.05, 0.01):
        c0, ce, cc = scheme.stencil_coefficients(h, k)
        assert abs(c0 + 4 * ce + 4 * cc - k**2) < 1e-9 * (1 / h**2)
    errs = []
    for n in (32, 64, 128, 256):
        h = 1.0 / n
        x = np.arange(n + 1) * h
        X, Y = np.meshgrid(x, x, indexing="ij")
        u = np.exp(1j * k * (X * math.cos(0.3) + Y * math.sin(0.3)))
        r = scheme.apply_L(u, h, k)[1:-1, 1:-1]
        errs.append(np.abs(r).max())
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(14.0 < q < 18.0 for q in ratios), ratios


def test_stencil_separable_form():
    """Weights equal (dx2+dy2)/h^2 + dx2 dy2/(6h^2) + (k^2/12)(dx2+dy2) + k^2 term by term."""
    h, k = 0.037, 7.5
    c0, ce, cc = scheme.stencil_coefficients(h, k)
    # on a delta function: dx2+dy2 gives centre -4, edges 1; dx2 dy2 gives centre 4, edges -2, corners 1
    assert np.isclose(c0, -4 / h**2 + 4 / (6 * h**2) - 4 * k**2 / 12 + k**2)
    assert np.isclose(ce, 1 / h**2 - 2 / (6 * h**2) + k**2 / 12)
    assert np.isclose(cc, 1 / (6 * h**2))


# ------------------------------------------------------------------ AP solvers
@pytest.mark.parametrize("n,k", [(12, 10.0), (16, 31.0), (20, 3.0)])
def test_ap_solvers_agree_with_brute_force(n, k):
    h = 1.1 / n
    g = wl.random_rhs((4, n + 1, n + 1), seed=n)
    u_dense = scheme.solve_dense(g, n, h, k)
    u_band = scheme.BandedAP(n, h, k).solve(g)
    u_sep = scheme.SeparableAP(n, h, k).solve(g)
    s = np.abs(u_dense).max()
    assert np.abs(u_band - u_dense).max() / s < 1e-12
    assert np.abs(u_sep - u_dense).max() / s < 1e-12
    # the solution satisfies the assembled system, including the end rows
    A = scheme.assemble(n, h, k)
    b, _ = scheme._rhs_vector(g, n)
    x = u_band.reshape(4, n + 1, n + 1)[:, :, 1:n].reshape(4, -1).T
    assert np.abs(A @ x - b).max() / np.abs(b).max() < 1e-12


def test_ap_banded_vs_separable_medium():
    n, k = 96, 40.0
    h = 0.55 / n
    g = wl.random_rhs((3, n + 1, n + 1), seed=5)
    u1 = scheme.BandedAP(n, h, k).solve(g)
    u2 = scheme.SeparableAP(n, h, k).solve(g)
    assert np.abs(u1 - u2).max() / np.abs(u1).max() < 1e-11


def test_ap_banded_vs_separable_n256():
    """O1 (banded LU with partial pivoting of the assembled AP) and O2 (explicit
    sine sums + one tridiagonal solve per mode) at the cross-point size n = 256,
    k = 50, h = 0.55/256, where every larger oracle reference (O2) is anchored:
    both are backward stable (||A u - g|| / (||A|| ||u||) below 1e-14, max norms)
    and they agree to the AP's conditioning.  kappa(A) = max_j ||T_j|| / min_j
    sigma_min(T_j) over the per-mode tridiagonal blocks (the scaled sine transform
    is orthogonal), 2.7e5 here, so two backward-stable solves may differ by a few
    u kappa = 3e-11: the bound 5e-11 (measured 9.7e-12)."""
    n, k = 256, 50.0
    h = 0.55 / n
    g = wl.random_rhs((2, n + 1, n + 1), seed=256)
    u1 = scheme.BandedAP(n, h, k).solve(g)
    u2 = scheme.SeparableAP(n, h, k).solve(g)
    A = scheme.assemble(n, h, k)
    b = np.zeros((2, n + 1, n - 1), dtype=complex)
    b[:, 1:n, :] = g[:, 1:n, 1:n]
    b = b.reshape(2, -1).T
    anorm = abs(A).max()
    for u in (u1, u2):
        x = u[..., 1:n].reshape(2, -1).T
        assert np.abs(A @ x - b).max() / (anorm * np.abs(x).max()) < 1e-14
    sep = scheme.SeparableAP(n, h, k)
    smax, smin = 0.0, np.inf
    for j in range(n - 1):
        ab = sep.ab[j]
        T = np.diag(ab[1]) + np.diag(ab[0, 1:], 1) + np.diag(ab[2, :-1], -1)
        sv = np.linalg.svd(T, compute_uv=False)
        smax, smin = max(smax, sv[0]), min(smin, sv[-1])
    kappa = smax / smin
    assert 1e5 < kappa < 1e6
    assert np.abs(u1 - u2).max() / np.abs(u1).max() < 5e-11


def test_sine_matrix_is_scaled_involution_and_matches_dst1():
    """S S = (n/2) I; S agrees with the type-I discrete sine transform of scipy."""
    import scipy.fft
    for n in (8, 33, 128):
        S = scheme.sine_matrix(n)
        assert np.abs(S @ S - (n / 2) * np.eye(n - 1)).max() < 1e-11 * n
        v = wl.random_rhs(n - 1, seed=n, complex_=False)
        assert np.allclose(v @ S, scipy.fft.dst(v, type=1) / 2.0, atol=1e-12 * n)


def test_end_rows_are_fourth_order():
    """The assembled x-end rows applied to samples of a Helmholtz solution
    approximate (u_x +- i k u) at the half node with an error falling ~16x per
    halving (the reading of the garbled Sommerfeld-type rows)."""
    k, th = 9.0, 0.7
    xi, eta = k * math.cos(th), k * math.sin(th)
    errs = {"left": [], "right": []}
    for n in (32, 64, 128, 256):
        h = 1.0 / n
        A = scheme.assemble(n, h, k).tocsr()
        xs = np.arange(n + 1) * h
        X, Y = np.meshgrid(xs, xs, indexing="ij")
        u = np.exp(1j * (xi * X + eta * Y))
        uvec = u[:, 1:n].reshape(-1)
        for end, mo, xh, sgn in (("left", 0, 0.5 * h, -1.0), ("right", n, (n - 0.5) * h, 1.0)):
            qs = np.arange(2, n - 1)
            rows = scheme.unknown_index(n, mo, qs)
            val = A[rows] @ uvec
            exact = (1j * xi + sgn * 1j * k) * np.exp(1j * (xi * xh + eta * xs[qs]))
            errs[end].append(np.abs(val - exact).max())
    for end in errs:
        e = errs[end]
        ratios = [e[i] / e[i + 1] for i in range(len(e) - 1)]
        assert all(13.0 < q < 19.0 for q in ratios), (end, ratios)


# ------------------------------------------------------------------ grid sets
def test_grid_sets_paper_base_square():
    g = ogrid.APGrid(-1.0, -1.0, 2.0, 2.0, 64)
    assert g.cx == g.cy == 59
    assert g.n_gamma == 4 * (59 + 59) == 472
    # gamma is the two-node ring around the boundary of the M+ rectangle
    mm, qq = np.nonzero(g.Mplus)
    assert (mm.max() - mm.min() + 1) * (qq.max() - qq.min() + 1) == g.Mplus.sum()
    ring = np.zeros_like(g.Mplus)
    ring[mm.min() - 1:mm.max() + 2, qq.min() - 1:qq.max() + 2] = True
    ring[mm.min() + 1:mm.max(), qq.min() + 1:qq.max()] = False
    assert np.array_equal(ring, g.gamma_mask)
    assert not (g.Mplus & ~g.M0).any()


@pytest.mark.parametrize("args,expect", [((0.0, 0.0, 0.5, 1.0, 64), 4 * (29 + 59)),
                                         ((0.0, 0.0, 0.5, 0.5, 256), 1864),
                                         ((0.0, 0.0, 0.25, 1.0, 1024), 4656)])
def test_gamma_counts_of_workload_grids(args, expect):
    g = ogrid.APGrid(*args)
    assert g.n_gamma == 4 * (g.cx + g.cy) == expect
    # no node lies on the continuous boundary (margins never an integer number of cells)
    x0, y0, lx, ly, n = args
    for v, lo, hi in ((g.xs, x0, x0 + lx), (g.ys, y0, y0 + ly)):
        assert np.min(np.abs(np.concatenate([v - lo, v - hi]))) > 1e-6 * g.h


# ------------------------------------------------------------------ projection invariants
def _small_problem(n=24, k=11.0):
    g = ogrid.APGrid(0.0, 0.0, 1.0, 1.0, n)
    return g, k, scheme.BandedAP(n, g.h, k)


def test_projection_is_idempotent():
    g, k, solver = _small_problem()
    P = projector.projection_matrix(g, k, solver)
    assert np.abs(P @ P - P).max() / np.abs(P).max() < 1e-11


def test_projection_fixes_traces_of_homogeneous_solutions():
    """BEP (eq. discrete_BEP_homo): P xi = xi iff xi is the trace of a solution of
    L^(h) u = 0 on M+; traces of AP solutions driven from M- qualify."""
    g, k, solver = _small_problem()
    src = wl.random_rhs((3, g.n + 1, g.n + 1), seed=3)
    src[:, ~g.Mminus] = 0.0
    u = solver.solve(src)
    xi = u[:, g.gamma_m, g.gamma_q]
    Pxi = projector.projection(g, k, xi, solver)
    assert np.abs(Pxi - xi).max() / np.abs(xi).max() < 1e-11
    # reconstruction (eq. potential_solution_homo) recovers u on N+
    up = projector.potential(g, k, xi, solver)
    assert np.abs((up - u)[:, g.Nplus]).max() / np.abs(u).max() < 1e-11


def test_projection_annihilates_traces_of_interior_sources():
    """BEP with g supported in M+: P xi + Tr G g = xi for xi = Tr G g, so P xi = 0."""
    g, k, solver = _small_problem()
    src = wl.random_rhs((3, g.n + 1, g.n + 1), seed=4)
    src[:, ~g.Mplus] = 0.0
    xi = solver.solve(src)[:, g.gamma_m, g.gamma_q]
    Pxi = projector.projection(g, k, xi, solver)
    assert np.abs(Pxi).max() / np.abs(xi).max() < 1e-11


def test_projector_columns_equal_projection_minus_identity():
    """Q = (P_gamma - I) E column by column (eq. Q_construction)."""
    g, k, solver = _small_problem()
    P = projector.projection_matrix(g, k, solver)
    E = extension.extension_matrix(g, k, 6)
    Q = projector.build_projector(g, k, 6, solver)
    ref = (P - np.eye(g.n_gamma)) @ E
    assert np.abs(Q - ref).max() / np.abs(ref).max() < 1e-11


# ------------------------------------------------------------------ Chebyshev + extension
def test_chebyshev_values_and_derivatives():
    t = np.linspace(-1.0, 1.0, 23)
    M = 12
    D = extension.chebyshev_derivatives(t, M, 4)
    for j in range(M):
        c = np.zeros(M)
        c[j] = 1.0
        for p in range(5):
            ref = npcheb.chebval(t, npcheb.chebder(c, p)) if p else npcheb.chebval(t, c)
            assert np.allclose(D[p, :, j], ref, atol=1e-9 * (j + 1) ** (2 * p + 1))
    th = np.linspace(0.1, 3.0, 7)
    D = extension.chebyshev_derivatives(np.cos(th), M, 0)[0]
    assert np.allclose(D, np.cos(np.outer(th, np.arange(M))), atol=1e-13)
    D1 = extension.chebyshev_derivatives(np.array([1.0]), M, 2)
    j = np.arange(M)
    assert np.allclose(D1[1, 0], j**2)
    assert np.allclose(D1[2, 0], j**2 * (j**2 - 1) / 3.0)


def test_chebyshev_interpolation_is_exact_below_degree_M():
    M = 10
    t = extension.chebyshev_points(M)
    rng = np.random.default_rng(0)
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    vals = npcheb.chebval(t, c)
    assert np.allclose(extension.chebyshev_coefficients(vals), c, atol=1e-13)


def _plane_wave_side_data(g, k, th):
    """Exact Dirichlet data and its tangential derivatives at the foot point of each gamma node."""
    c, s = math.cos(th), math.sin(th)
    x = g.xs[g.gamma_m]
    y = g.ys[g.gamma_q]
    side = g.side
    fx = np.where(side == 2, g.x0, np.where(side == 3, g.x0 + g.lx, x))
    fy = np.where(side == 0, g.y0, np.where(side == 1, g.y0 + g.ly, y))
    u0 = np.exp(1j * k * (c * fx + s * fy))
    horiz = (side == 0) | (side == 1)
    kt = np.where(horiz, k * c, k * s)                 # tangential wavenumber
    nrm = np.select([side == 0, side == 1, side == 2], [-s, s, -c], c)
    kn = k * nrm                                       # outward normal wavenumber
    xi0 = (u0, -(kt**2) * u0, kt**4 * u0)
    xi1 = (1j * kn * u0, -(kt**2) * 1j * kn * u0)
    return xi0, xi1, np.exp(1j * k * (c * x + s * y))


def test_extension_is_fifth_order_on_gamma():
    """Ex (u, du/dn) approximates u at the gamma nodes to O(h^5) (Sec. 3.2.3).

    For a plane wave the equation-based normal derivatives are exact, so at a
    node at signed distance rho the extension is the degree-4 Taylor polynomial
    of exp(i k_n rho) times the foot value: the error must equal the series
    remainder, |k_n rho|^5/120 to leading order, node by node.  (Ratios of the
    maximum error between grids are not a clean 32 because the largest |rho|/h
    depends on where the boundary falls between grid lines.)"""
    k, th = 13.0, 0.4
    for n in (64, 128, 256):
        g = ogrid.APGrid(-1.0, -1.0, 2.0, 2.0, n)
        xi0, xi1, exact = _plane_wave_side_data(g, k, th)
        v = extension.extend_data(g, k, xi0, xi1)
        kn = np.abs(xi1[0] / (1j * xi0[0]))
        x = kn * np.abs(g.rho)
        lead = x**5 / 120.0
        err = np.abs(v - exact)
        assert np.all(err <= lead * (1.0 + x) + 1e-13)
        sel = x > 0.02
        assert np.all(err[sel] >= lead[sel] * (1.0 - x[sel]) - 1e-13)


def test_extension_matrix_matches_direct_extension_for_polynomial_data():
    """E c (basis columns) equals the extension of the data the coefficients represent."""
    k, M, n = 6.0, 8, 40
    g = ogrid.APGrid(0.0, 0.0, 1.0, 0.5, n)
    E = extension.extension_matrix(g, k, M)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(8 * M)
    # data per side: xi0 = sum_j c[side*M+j] T_j(t), xi1 = sum_j c[4M+side*M+j] T_j(t)
    D = extension.chebyshev_derivatives(g.t, M, 4)
    sc = 2.0 / g.side_len
    a = [np.zeros(g.n_gamma) for _ in range(3)]
    b = [np.zeros(g.n_gamma) for _ in range(2)]
    for i in range(g.n_gamma):
        s = g.side[i]
        c0 = c[s * M:(s + 1) * M]
        c1 = c[4 * M + s * M:4 * M + (s + 1) * M]
        a[0][i], a[1][i], a[2][i] = D[0, i] @ c0, sc[i] ** 2 * D[2, i] @ c0, sc[i] ** 4 * D[4, i] @ c0
        b[0][i], b[1][i] = D[0, i] @ c1, sc[i] ** 2 * D[2, i] @ c1
    v = extension.extend_data(g, k, a, b)
    assert np.allclose(E @ c, v, atol=1e-11 * np.abs(v).max())


# ------------------------------------------------------------------ least squares + elimination
def test_householder_least_squares_matches_lapack():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((90, 30)) + 1j * rng.standard_normal((90, 30))
    A[:, 3] *= 1e-4                          # bad column scaling
    b = rng.standard_normal(90) + 1j * rng.standard_normal(90)
    x, R, res = interface.householder_qr_solve(A, b)
    xr = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.abs(x - xr).max() / np.abs(xr).max() < 1e-10
    assert np.allclose(R.conj().T @ R, A.conj().T @ A, rtol=0, atol=1e-10 * np.abs(A.conj().T @ A).max())
    assert np.isclose(res, np.linalg.norm(A @ xr - b))


def test_elimination_reproduces_block_system_with_constraints():
    """Qbar x - Fbar equals the stacked block-diagonal residual [Q^(i) c^(i)] of the
    expanded coefficients, and the expanded coefficients satisfy every boundary
    (eq. BC_coefficients) and interface (eq. transmission_coefficients) equation."""
    M = 3
    def bc(ix, iy, s):
        return [(1.0, 0.0), (0.0, 1.0), (1.0, 1.0), (2.0, -0.5)][(ix + 2 * iy + s) % 4]
    subs, sides = wl.grid_topology(3, 2, 0.0, 0.0, 1.0, 1.0, [1.0] * 6, 16, bc)
    rng = np.random.default_rng(2)
    Qs = [rng.standard_normal((11 + i, 8 * M)) + 1j * rng.standard_normal((11 + i, 8 * M)) for i in range(6)]
    d = [[(rng.standard_normal(M) + 1j * rng.standard_normal(M)) if sides[i][s].kind == wl.BOUNDARY else None
          for s in range(4)] for i in range(6)]
    Qbar, Fbar, blocks = interface.assemble(Qs, sides, d, M)
    assert Qbar.shape[1] == 4 * 6 * M
    x = rng.standard_normal(Qbar.shape[1]) + 1j * rng.standard_normal(Qbar.shape[1])
    c = interface.expand(x, sides, d, M, blocks)
    stacked = np.concatenate([Qs[i] @ c[i] for i in range(6)])
    assert np.allclose(Qbar @ x - Fbar, stacked, atol=1e-11)
    for i in range(6):
        for s in range(4):
            sd = sides[i][s]
            c0 = c[i][s * M:(s + 1) * M]
            c1 = c[i][4 * M + s * M:4 * M + (s + 1) * M]
            if sd.kind == wl.BOUNDARY:
                assert np.allclose(sd.alpha * c0 + sd.beta * c1, d[i][s])
            else:
                j, t = sd.nbr, sd.nbr_side
                assert np.allclose(c0, c[j][t * M:(t + 1) * M])
                assert np.allclose(c1, -c[j][4 * M + t * M:4 * M + (t + 1) * M])


# ------------------------------------------------------------------ exact solutions
def test_piecewise_plane_wave_amplitudes():
    k1, k2 = 5.0, 40.0
    a, b = wl.piecewise_amplitudes([0.0], [k1, k2])
    assert np.isclose(b[0], (k1 - k2) / (k1 + k2)) and np.isclose(a[1], 2 * k1 / (k1 + k2))
    # the printed closed form R = k2/(2k1) - 1/2 violates the derivative condition
    R_printed, T_printed = k2 / (2 * k1) - 0.5, k2 / (2 * k1) + 0.5
    assert abs(k1 * (1 - R_printed) - k2 * T_printed) > 1.0
    edges, ks = [0.25, 0.5, 0.75], [20.0, 200.0, 20.0, 200.0]
    u, grad, a, b = wl.piecewise_plane_wave(edges, ks)
    for xe in edges:
        for f in (lambda x: u(x, 0.0), lambda x: grad(x, 0.0)[0]):
            lo, hi = f(np.nextafter(xe, -1)), f(xe)
            assert abs(lo - hi) < 1e-9 * max(1.0, abs(hi))
    assert a[0] == 1.0 and b[-1] == 0.0


# ------------------------------------------------------------------ end to end
def test_fourth_order_convergence_two_rectangles():
    errs = [solve.dd_solve(wl.config_two_rect(n=n))["info"]["error_max_Mplus"] for n in (32, 64, 128)]
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(12.0 < q < 21.0 for q in ratios), (errs, ratios)
    assert errs[1] < 1e-4


def test_paper_printed_errors_reproduced():
    """Errors of the paper's base case and two-subdomain jump case at n = 64, 128
    match the printed tables (same order of magnitude, rate 4.0 +- 0.2)."""
    gold = json.load(open(GOLDEN))
    for key, make in (("base_case", wl.config_paper_base), ("piecewise_2_k5_k13", wl.config_paper_jump),
                      ("uniform_2_plane_wave", wl.config_paper_two)):
        ref = dict(zip(gold[key]["n"], gold[key]["error"]))
        errs = {n: solve.dd_solve(make(n=n))["info"]["error_max_Mplus"] for n in (64, 128)}
        for n in (64, 128):
            assert 0.33 < errs[n] / ref[n] < 3.0, (key, n, errs[n], ref[n])
        rate = math.log2(errs[64] / errs[128])
        assert abs(rate - 4.0) < 0.2, (key, rate)
