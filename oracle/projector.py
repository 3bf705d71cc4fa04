"""Difference potential, projection and the per-subdomain matrix Q.  Test infrastructure only.

Follows paper Sec. 3.2.2 and 3.2.5:
  * difference potential with density xi on gamma (eq. Potential_def):
        P_{N+} xi = w - G^(h)(L^(h) w restricted to M+),  w = xi on gamma, 0 elsewhere;
  * projection P_gamma xi = (P_{N+} xi) restricted to gamma (eq. def_Pgamma);
  * Q = [(P_gamma - I) Ex Psi_1, ..., (P_gamma - I) Ex Psi_{8M*}] (eq. Q_construction),
    one application of G^(h) per column.  Since w equals xi on gamma,
    (P_gamma - I) xi = -Tr_gamma G^(h)(L^(h) w |_{M+}).
"""
from __future__ import annotations

import numpy as np

from .extension import extension_matrix
from .scheme import apply_L, make_solver


def density_rhs(grid, k: float, xi: np.ndarray) -> np.ndarray:
    """g = L^(h) w |_{M+} for densities xi[..., |gamma|] (one grid per leading index)."""
    n = grid.n
    xi = np.asarray(xi)
    w = np.zeros(xi.shape[:-1] + (n + 1, n + 1), dtype=xi.dtype)
    w[..., grid.gamma_m, grid.gamma_q] = xi
    g = apply_L(w, grid.h, k)
    g[..., ~grid.Mplus] = 0.0
    return w, g


def potential(grid, k: float, xi: np.ndarray, solver=None) -> np.ndarray:
    """P_{N+} xi on the full auxiliary grid (meaningful on N+)."""
    solver = solver or make_solver(grid.n, grid.h, k)
    w, g = density_rhs(grid, k, xi)
    return w - solver.solve(g)


def projection(grid, k: float, xi: np.ndarray, solver=None) -> np.ndarray:
    u = potential(grid, k, xi, solver)
    return u[..., grid.gamma_m, grid.gamma_q]


def projection_matrix(grid, k: float, solver=None) -> np.ndarray:
    """Explicit |gamma| x |gamma| P_gamma (small grids only)."""
    solver = solver or make_solver(grid.n, grid.h, k)
    eye = np.eye(grid.n_gamma)
    return projection(grid, k, eye, solver).T


def build_projector(grid, k: float, m_star: int, solver=None, cols=None, chunk: int = 64) -> np.ndarray:
    """Q (|gamma| x 8M*, or the listed columns), one AP solve per column."""
    solver = solver or make_solver(grid.n, grid.h, k)
    E = extension_matrix(grid, k, m_star)
    cols = np.arange(8 * m_star) if cols is None else np.asarray(cols)
    Q = np.zeros((grid.n_gamma, cols.size), dtype=complex)
    for s in range(0, cols.size, chunk):
        cc = cols[s:s + chunk]
        _, g = density_rhs(grid, k, E[:, cc].T)
        u = solver.solve(g)
        Q[:, s:s + cc.size] = -u[:, grid.gamma_m, grid.gamma_q].T
    return Q
