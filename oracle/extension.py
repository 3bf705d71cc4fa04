"""Boundary basis and equation-based extension (paper Sec. 3.2.3-3.2.4).  Test infrastructure only.

Readings:
  * psi_j(t) = T_{j-1}(t), j = 1..M*, Chebyshev polynomials of the first kind
    in the side parameter t (Chebyshev basis via Chebfun, Sec. 4; orthogonal,
    Sec. 3.3.1).  Derivatives in the physical tangential coordinate carry the
    factor (2/side length)^p.
  * The extension keeps the Taylor terms through rho^4 (eq. general_extension)
    with the normal derivatives of eqs. cart_ext_0-4 for f = 0:
        v = xi0 + rho xi1 + rho^2/2 (-xi0'' - k^2 xi0)
              + rho^3/6 (-xi1'' - k^2 xi1) + rho^4/24 (xi0'''' + 2k^2 xi0'' + k^4 xi0)
    (the third and fourth normal derivatives follow from differentiating the
    Helmholtz equation; they hold for every side because the Laplacian is
    invariant under the reflections that map one side onto another).
  * Column order of E (and of Q, eq. Q_construction): all Dirichlet pairs
    Psi^(0) first, then all Neumann pairs Psi^(1); inside each, side-major
    (bottom, top, left, right), then j = 1..M*:
        col = kind*4M* + side*M* + (j-1).
  * Coefficients of given side data phi: interpolation at the M* first-kind
    Chebyshev points t_i = cos(pi (i + 1/2)/M*) by discrete orthogonality
    (exact for polynomials of degree < M*).
"""
from __future__ import annotations

import numpy as np


def chebyshev_derivatives(t: np.ndarray, m_star: int, pmax: int = 4) -> np.ndarray:
    """D[p, i, j] = d^p/dt^p T_j(t_i), p = 0..pmax, j = 0..m_star-1.

    Recurrence T_{j+1} = 2 t T_j - T_{j-1}, differentiated p times:
    T_{j+1}^(p) = 2 t T_j^(p) + 2 p T_j^(p-1) - T_{j-1}^(p).
    """
    t = np.asarray(t, dtype=float)
    D = np.zeros((pmax + 1, t.size, m_star))
    for p in range(pmax + 1):
        if m_star > 0:
            D[p, :, 0] = 1.0 if p == 0 else 0.0
        if m_star > 1:
            D[p, :, 1] = t if p == 0 else (1.0 if p == 1 else 0.0)
        for j in range(1, m_star - 1):
            D[p, :, j + 1] = 2.0 * t * D[p, :, j] - D[p, :, j - 1]
            if p > 0:
                D[p, :, j + 1] += 2.0 * p * D[p - 1, :, j]
    return D


def extension_matrix(grid, k: float, m_star: int) -> np.ndarray:
    """E = Ex^(H) Psi: real |gamma| x 8M* matrix (row i nonzero only in its side's columns)."""
    ng = grid.n_gamma
    E = np.zeros((ng, 8 * m_star))
    D = chebyshev_derivatives(grid.t, m_star, 4)
    scale = 2.0 / grid.side_len
    psi0 = D[0]
    psi2 = D[2] * (scale**2)[:, None]
    psi4 = D[4] * (scale**4)[:, None]
    rho = grid.rho[:, None]
    dir_col = psi0 + rho**2 / 2.0 * (-psi2 - k**2 * psi0) + rho**4 / 24.0 * (psi4 + 2.0 * k**2 * psi2 + k**4 * psi0)
    neu_col = rho * psi0 + rho**3 / 6.0 * (-psi2 - k**2 * psi0)
    for i in range(ng):
        s = grid.side[i]
        E[i, s * m_star:(s + 1) * m_star] = dir_col[i]
        E[i, 4 * m_star + s * m_star:4 * m_star + (s + 1) * m_star] = neu_col[i]
    return E


def extend_data(grid, k: float, xi0_derivs, xi1_derivs) -> np.ndarray:
    """Ex^(H)(xi0, xi1) for data given by tangential derivatives at each gamma node.

    xi0_derivs = (xi0, xi0'', xi0''''), xi1_derivs = (xi1, xi1'') evaluated at the
    foot point of each node on its side (physical tangential derivatives).
    """
    a0, a2, a4 = xi0_derivs
    b0, b2 = xi1_derivs
    r = grid.rho
    return (a0 + r * b0 + r**2 / 2.0 * (-a2 - k**2 * a0) + r**3 / 6.0 * (-b2 - k**2 * b0)
            + r**4 / 24.0 * (a4 + 2.0 * k**2 * a2 + k**4 * a0))


def chebyshev_points(m_star: int) -> np.ndarray:
    i = np.arange(m_star)
    return np.cos(np.pi * (i + 0.5) / m_star)


def chebyshev_coefficients(samples: np.ndarray) -> np.ndarray:
    """Coefficients d_j (j = 0..M*-1) of the interpolant through samples at chebyshev_points."""
    samples = np.asarray(samples)
    M = samples.shape[-1]
    t = chebyshev_points(M)
    T = chebyshev_derivatives(t, M, 0)[0]          # T[i, j] = T_j(t_i)
    w = np.full(M, 2.0 / M)
    w[0] = 1.0 / M
    return (samples @ T) * w
