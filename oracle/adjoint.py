"""Receiver misfit of a DD solve and its derivatives.  Test infrastructure only.

For receivers r at nodes (m_r, q_r) of subdomain i_r's auxiliary grid (nodes
of M+, where the reconstructed u of eq. potential_solution_homo is the
solution), the functional Phi = Re sum_r conj(ubar_r) u_r and the misfit
J = sum_r |u_r - u_obs_r|^2 (its gradient is that of Phi with
ubar = 2 (u - u_obs)) depend on every subdomain's k^2 and on the boundary
data's Chebyshev coefficients d.  This module computes the derivatives of Phi
in FORWARD mode, one direction at a time, by differentiating each step of the
solve of Sec. 3.5 as written (no adjoint solves):

  * the discrete AP operator A(k^2) (eqs. FD_scheme, discrete_AP, with the
    end-row reading of scheme.py): interior weights (centre, edge, corner)
    have derivatives (2/3, 1/12, 0); the end rows D/h + d2(D)/(24h) +
    (k^2 h/24) D +- i k [A + d2(A)/8 + (k^2 h^2/8) A] have derivative
    (h/24) D +- i [(1 + k^2 h^2/8)/(2k) + k h^2/8] A +- (i/(2k)) d2(A)/8;
  * the extension E(k^2) (eq. general_extension with eqs. cart_ext_0-4):
    Dirichlet column psi + rho^2/2 (-psi'' - k^2 psi) + rho^4/24 (psi'''' +
    2k^2 psi'' + k^4 psi) has derivative -rho^2/2 psi + rho^4/24 (2 psi'' +
    2 k^2 psi); Neumann column rho psi + rho^3/6 (-psi'' - k^2 psi) has
    derivative -rho^3/6 psi;
  * Q's columns -Tr G (L w|M+) (eq. Q_construction): d(A^{-1}) = -A^{-1} dA A^{-1};
  * the reduced system (Sec. 3.3.3) is linear in Q and d; the least-squares
    solution x = (Qbar^* Qbar)^{-1} Qbar^* Fbar has
    dx = (Qbar^* Qbar)^{-1} [Qbar^* (dFbar - dQbar x) + dQbar^* (Fbar - Qbar x)];
  * the reconstruction u = w - A^{-1}(L w|M+), w = E c on gamma
    (eqs. Potential_def, potential_solution_homo).

Complex data d: the returned derivative is dPhi/d(Re d) + i dPhi/d(Im d).
Sizes: dense and sparse direct solves, small grids only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu

from paper_2103_12172_amd import workloads as wl

from .extension import chebyshev_derivatives, extension_matrix
from .grid import APGrid
from .interface import assemble as assemble_reduced, expand
from .scheme import assemble, end_row_weights, stencil_coefficients, unknown_index
from .solve import boundary_coefficients


def _stencil(w, c0, ce, cc):
    """The 9-node operator with weights (c0, ce, cc) at the interior nodes of w[..., m, q]."""
    out = np.zeros_like(w)
    C = w[..., 1:-1, 1:-1]
    E = w[..., 2:, 1:-1] + w[..., :-2, 1:-1] + w[..., 1:-1, 2:] + w[..., 1:-1, :-2]
    K = w[..., 2:, 2:] + w[..., :-2, 2:] + w[..., 2:, :-2] + w[..., :-2, :-2]
    out[..., 1:-1, 1:-1] = c0 * C + ce * E + cc * K
    return out


def assemble_dk2(n: int, h: float, k: float) -> sp.csr_matrix:
    """d A / d(k^2) on the unknowns of scheme.assemble (same ordering)."""
    N = (n + 1) * (n - 1)
    rows, cols, vals = [], [], []

    def put(r, m, q, v):
        if 1 <= q <= n - 1:
            rows.append(r)
            cols.append(unknown_index(n, m, q))
            vals.append(v)

    for m in range(1, n):
        for q in range(1, n):
            r = unknown_index(n, m, q)
            put(r, m, q, 2.0 / 3.0)
            for dm, dq in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                put(r, m + dm, q + dq, 1.0 / 12.0)
    _, _, wA, wA2 = end_row_weights(h, k)
    dA_mid = (wA - 2.0 * wA2) / (2.0 * k) + k * h * h / 8.0   # d/dk^2 of k (wA - 2 wA2)
    dA_side = wA2 / (2.0 * k)                                 # d/dk^2 of k wA2
    for end, (mo, mi, sgn) in (("left", (0, 1, -1.0)), ("right", (n, n - 1, +1.0))):
        for q in range(1, n):
            r = unknown_index(n, mo, q)
            dwd = h / 24.0
            if end == "right":
                put(r, n, q, dwd)
                put(r, n - 1, q, -dwd)
            else:
                put(r, 1, q, dwd)
                put(r, 0, q, -dwd)
            for dq, aw in ((0, dA_mid), (1, dA_side), (-1, dA_side)):
                v = sgn * 1j * aw * 0.5
                put(r, mo, q + dq, v)
                put(r, mi, q + dq, v)
    return sp.csr_matrix((np.asarray(vals, dtype=complex), (rows, cols)), shape=(N, N))


def extension_dk2(grid, k: float, m_star: int) -> np.ndarray:
    """d E / d(k^2) (real |gamma| x 8M*, the column layout of extension_matrix)."""
    ng = grid.n_gamma
    dE = np.zeros((ng, 8 * m_star))
    D = chebyshev_derivatives(grid.t, m_star, 4)
    scale = 2.0 / grid.side_len
    psi0 = D[0]
    psi2 = D[2] * (scale**2)[:, None]
    rho = grid.rho[:, None]
    dir_col = -rho**2 / 2.0 * psi0 + rho**4 / 24.0 * (2.0 * psi2 + 2.0 * k**2 * psi0)
    neu_col = -rho**3 / 6.0 * psi0
    for i in range(ng):
        s = grid.side[i]
        dE[i, s * m_star:(s + 1) * m_star] = dir_col[i]
        dE[i, 4 * m_star + s * m_star:4 * m_star + (s + 1) * m_star] = neu_col[i]
    return dE


def _vec(g, n):
    """Grid [..., m, q] -> unknown vector(s) over m = 0..n, q = 1..n-1 (last axis)."""
    g = np.asarray(g)
    return g[..., :, 1:n].reshape(g.shape[:-2] + ((n + 1) * (n - 1),))


def _grid(v, n):
    v = np.asarray(v)
    out = np.zeros(v.shape[:-1] + (n + 1, n + 1), dtype=complex)
    out[..., :, 1:n] = v.reshape(v.shape[:-1] + (n + 1, n - 1))
    return out


class _Sub:
    """One subdomain's operators at its k."""

    def __init__(self, sd, m_star):
        self.sd = sd
        self.grid = APGrid(sd.x0, sd.y0, sd.lx, sd.ly, sd.n)
        g = self.grid
        self.n, self.h, self.k = sd.n, g.h, sd.k
        self.A = assemble(sd.n, g.h, sd.k).tocsc()
        self.lu = splu(self.A)
        self.E = extension_matrix(g, sd.k, m_star)
        self.coef = stencil_coefficients(g.h, sd.k)

    def solve(self, rhs_grid):
        """A^{-1} of a right-hand side given on every unknown row (end rows included)."""
        n = self.n
        v = _vec(rhs_grid, n)
        if v.ndim == 1:
            return _grid(self.lu.solve(v), n)
        return _grid(self.lu.solve(v.T).T, n)

    def scatter(self, xi):
        g = self.grid
        xi = np.asarray(xi)
        w = np.zeros(xi.shape[:-1] + (self.n + 1, self.n + 1), dtype=complex)
        w[..., g.gamma_m, g.gamma_q] = xi
        return w

    def rl(self, w, coef=None):
        """L w restricted to M+ (coef: other stencil weights, e.g. their k^2-derivatives)."""
        c0, ce, cc = coef or self.coef
        out = _stencil(w, c0, ce, cc)
        out[..., ~self.grid.Mplus] = 0.0
        return out


def forward(w: wl.Workload, m_star=None, d=None):
    """The DD solve of Sec. 3.5 (f = 0) with its intermediate quantities (d: boundary
    coefficients d[i][s]; default: those of the workload's data)."""
    m_star = m_star or w.m_star
    subs = [_Sub(sd, m_star) for sd in w.subdomains]
    Qs, V = [], []
    for S in subs:
        W = S.scatter(S.E.T)                    # (8M*, n+1, n+1) densities on gamma
        v = S.solve(S.rl(W))                    # A^{-1} (L w_j |M+)
        V.append(v)
        Qs.append(-v[:, S.grid.gamma_m, S.grid.gamma_q].T)
    d = boundary_coefficients(w, m_star) if d is None else d
    Qbar, Fbar, blocks = assemble_reduced(Qs, w.sides, d, m_star)
    x = np.linalg.lstsq(Qbar, Fbar, rcond=None)[0]
    c = expand(x, w.sides, d, m_star, blocks)
    us = []
    for S, ci in zip(subs, c):
        wi = S.scatter(S.E @ ci)
        us.append(wi - S.solve(S.rl(wi)))
    return {"subs": subs, "Q": Qs, "V": V, "d": d, "Qbar": Qbar, "Fbar": Fbar, "blocks": blocks, "x": x, "c": c,
            "u": us, "m_star": m_star}


def receiver_values(st, rcv):
    """u at receivers rcv = [(i, m, q), ...]."""
    return np.array([st["u"][i][m, q] for (i, m, q) in rcv])


def _phi_derivative(st, rcv, ubar, du):
    """d Phi for per-subdomain grid derivatives du."""
    return float(np.real(sum(np.conj(ub) * du[i][m, q] for ub, (i, m, q) in zip(ubar, rcv))))


def _ls_derivative(st, dQbar, dFbar):
    Qb, x = st["Qbar"], st["x"]
    r = st["Fbar"] - Qb @ x
    rhs = Qb.conj().T @ (dFbar - dQbar @ x) + dQbar.conj().T @ r
    return np.linalg.solve(Qb.conj().T @ Qb, rhs)


def _reconstruction_derivative(st, dc, i_k=None, dA=None, dE=None, dcoef=None):
    """du per subdomain from coefficient derivatives dc (and, for subdomain i_k, its k^2)."""
    out = []
    for l, S in enumerate(st["subs"]):
        xi = S.E @ dc[l]
        if l == i_k:
            xi = xi + dE @ st["c"][l]
        dw = S.scatter(xi)
        rhs = S.rl(dw)
        if l == i_k:
            wl_ = S.scatter(S.E @ st["c"][l])
            vu = S.solve(S.rl(wl_))
            rhs = rhs + S.rl(wl_, dcoef) - _grid(dA @ _vec(vu, S.n), S.n)
        out.append(dw - S.solve(rhs))
    return out


def gradient(w: wl.Workload, rcv, ubar, st=None):
    """(dPhi/dk_i^2 for every subdomain, dPhi/dd per boundary side (complex, None for interfaces))."""
    st = st or forward(w)
    m_star = st["m_star"]
    subs = st["subs"]
    N = len(subs)
    zeros_d = [[np.zeros(m_star, dtype=complex) if w.sides[i][s].kind == wl.BOUNDARY else None
                for s in range(4)] for i in range(N)]
    g_k = np.zeros(N)
    for i, S in enumerate(subs):
        dA = assemble_dk2(S.n, S.h, S.k)
        dE = extension_dk2(S.grid, S.k, m_star)
        dcoef = (2.0 / 3.0, 1.0 / 12.0, 0.0)
        Wd = S.scatter(S.E.T)
        dW = S.scatter(dE.T)
        hrhs = S.rl(Wd, dcoef) + S.rl(dW)
        hrhs = hrhs - _grid((dA @ _vec(st["V"][i], S.n).T).T, S.n)
        dQi = -S.solve(hrhs)[:, S.grid.gamma_m, S.grid.gamma_q].T
        dQs = [np.zeros_like(Q) for Q in st["Q"]]
        dQs[i] = dQi
        dQbar, dFbar, _ = assemble_reduced(dQs, w.sides, st["d"], m_star)
        dx = _ls_derivative(st, dQbar, dFbar)
        dc = expand(dx, w.sides, zeros_d, m_star, st["blocks"])
        du = _reconstruction_derivative(st, dc, i, dA, dE, dcoef)
        g_k[i] = _phi_derivative(st, rcv, ubar, du)
    g_d = [[None] * 4 for _ in range(N)]
    zQ = [np.zeros_like(Q) for Q in st["Q"]]
    for i in range(N):
        for s in range(4):
            if w.sides[i][s].kind != wl.BOUNDARY:
                continue
            gs = np.zeros(m_star, dtype=complex)
            for j in range(m_star):
                parts = []
                for unit in (1.0, 1j):
                    dd = [[None if v is None else np.zeros(m_star, dtype=complex) for v in row] for row in zeros_d]
                    dd[i][s][j] = unit
                    _, dFbar, _ = assemble_reduced(st["Q"], w.sides, dd, m_star)
                    dQbar = assemble_reduced(zQ, w.sides, zeros_d, m_star)[0]
                    dx = _ls_derivative(st, dQbar, dFbar)
                    dc = expand(dx, w.sides, dd, m_star, st["blocks"])
                    parts.append(_phi_derivative(st, rcv, ubar, _reconstruction_derivative(st, dc)))
                gs[j] = parts[0] + 1j * parts[1]
            g_d[i][s] = gs
    return g_k, g_d


def snap_receivers(w: wl.Workload, points, subs_of_points):
    """Each point to the nearest M+ node of its subdomain's auxiliary grid: [(i, m, q), ...]."""
    out = []
    for (x, y), i in zip(points, subs_of_points):
        sd = w.subdomains[i]
        g = APGrid(sd.x0, sd.y0, sd.lx, sd.ly, sd.n)
        X, Y = np.meshgrid(g.xs, g.ys, indexing="ij")
        dist = (X - x) ** 2 + (Y - y) ** 2
        dist[~g.Mplus] = np.inf
        m, q = np.unravel_index(int(np.argmin(dist)), dist.shape)
        out.append((int(i), int(m), int(q)))
    return out
