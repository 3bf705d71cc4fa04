"""Compact fourth-order scheme and the discrete auxiliary problem.  Test infrastructure only.

Follows paper Sec. 3.1 (eq. FD_scheme) and Sec. 3.2.1 (eqs. auxiliary_problem,
discrete_AP):

  * interior rows (1 <= m, q <= n-1): the 9-node left-hand side of
    eq. FD_scheme, i.e.
      (1/h^2)(E - 4u) + (1/(6h^2))(C + 4u - 2E) + (k^2/12)(E + 8u)
    with E the sum of the four edge neighbours and C of the four corners;
  * y-boundary rows: u(m,0) = u(m,n) = 0 (eq. AP_bounds_top_bottom), so the
    unknowns are u(m,q), m = 0..n, q = 1..n-1;
  * x-boundary rows: the Sommerfeld-type conditions u_x + i k u = 0 at the
    right end and u_x - i k u = 0 at the left end (eq. auxiliary_problem),
    discretised to fourth order at the half node between the last two
    x-nodes.  The printed discretisation (eqs. AP_bounds_right/left) is
    garbled (its i k bracket carries a difference quotient where the value at
    the half node belongs, and the weights of the tangential second
    differences do not match a Taylor expansion).  Reading used here, with
    D_q = u(n,q) - u(n-1,q), A_q = (u(n,q) + u(n-1,q))/2 and the y second
    difference d2 (Dirichlet-zero ends):
        D/h + d2(D)/(24 h) + (k^2 h/24) D + i k [A + d2(A)/8 + (k^2 h^2/8) A] = 0
    on the right; on the left D = u(1,q) - u(0,q), A = (u(1,q) + u(0,q))/2 and
    the sign of the i k term is minus.  (From the Taylor expansions
    D/h = u_x + h^2 u_xxx/24 and A = u + h^2 u_xx/8 at the half node with
    u_xx = -u_yy - k^2 u.)  The right-hand side of these rows is zero; the
    right-hand side g of the interior rows is given on m, q = 1..n-1.

Solvers of the assembled system, all returning u on the full (n+1)x(n+1) grid
(with the y-boundary zeros):
  * solve_dense  -- brute-force dense LU (numpy), tiny grids only;
  * BandedAP     -- LAPACK banded LU with partial pivoting (gbtrf / gbtrs);
  * SeparableAP  -- explicit sine sums in y plus one LAPACK tridiagonal solve
                    (with pivoting) per sine mode in x; same system, faster.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.linalg import lapack, solve_banded


def stencil_coefficients(h: float, k: float):
    """(centre, edge, corner) weights of the 9-node operator of eq. FD_scheme."""
    centre = -4.0 / h**2 + 4.0 / (6.0 * h**2) + 8.0 * k**2 / 12.0
    edge = 1.0 / h**2 - 2.0 / (6.0 * h**2) + k**2 / 12.0
    corner = 1.0 / (6.0 * h**2)
    return centre, edge, corner


def apply_L(w: np.ndarray, h: float, k: float) -> np.ndarray:
    """L^(h) w at the interior nodes of a grid function w[..., m, q]; zero on the ring."""
    c0, ce, cc = stencil_coefficients(h, k)
    out = np.zeros_like(w)
    C = w[..., 1:-1, 1:-1]
    E = w[..., 2:, 1:-1] + w[..., :-2, 1:-1] + w[..., 1:-1, 2:] + w[..., 1:-1, :-2]
    K = w[..., 2:, 2:] + w[..., :-2, 2:] + w[..., 2:, :-2] + w[..., :-2, :-2]
    out[..., 1:-1, 1:-1] = c0 * C + ce * E + cc * K
    return out


def end_row_weights(h: float, k: float):
    """Weights of the x-end rows: (wD, wD2, wA, wA2) so that a row reads
    wD*D + wD2*d2(D) + i k (wA*A + wA2*d2(A)) with the sign of i k set per end."""
    return 1.0 / h + k**2 * h / 24.0, 1.0 / (24.0 * h), 1.0 + k**2 * h**2 / 8.0, 1.0 / 8.0


def unknown_index(n: int, m, q):
    return m * (n - 1) + (q - 1)


def assemble(n: int, h: float, k: float) -> sp.csr_matrix:
    """Sparse matrix of the discrete AP on the unknowns u(m,q), m=0..n, q=1..n-1."""
    N = (n + 1) * (n - 1)
    rows, cols, vals = [], [], []
    c0, ce, cc = stencil_coefficients(h, k)

    def put(r, m, q, v):
        if 1 <= q <= n - 1:  # q = 0, n are the Dirichlet zeros
            rows.append(r)
            cols.append(unknown_index(n, m, q))
            vals.append(v)

    for m in range(1, n):
        for q in range(1, n):
            r = unknown_index(n, m, q)
            put(r, m, q, c0)
            for dm, dq in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                put(r, m + dm, q + dq, ce)
            for dm, dq in ((1, 1), (-1, 1), (1, -1), (-1, -1)):
                put(r, m + dm, q + dq, cc)
    wD, wD2, wA, wA2 = end_row_weights(h, k)
    for end, (mo, mi, sgn) in (("left", (0, 1, -1.0)), ("right", (n, n - 1, +1.0))):
        # D = u(outer) - u(inner) oriented outward: right: u(n)-u(n-1); left: u(1)-u(0)
        for q in range(1, n):
            r = unknown_index(n, mo, q)
            # contributions of D_q' and A_q' for q' = q-1, q, q+1 (d2 = f(q+1) - 2f(q) + f(q-1))
            for dq, dw in ((0, wD - 2.0 * wD2), (1, wD2), (-1, wD2)):
                if end == "right":
                    put(r, n, q + dq, dw)
                    put(r, n - 1, q + dq, -dw)
                else:
                    put(r, 1, q + dq, dw)
                    put(r, 0, q + dq, -dw)
            for dq, aw in ((0, wA - 2.0 * wA2), (1, wA2), (-1, wA2)):
                v = sgn * 1j * k * aw * 0.5
                put(r, mo, q + dq, v)
                put(r, mi, q + dq, v)
    return sp.csr_matrix((np.asarray(vals, dtype=complex), (rows, cols)), shape=(N, N))


def _rhs_vector(g: np.ndarray, n: int) -> np.ndarray:
    """Stack the interior-node right-hand side g[..., m, q] into unknown order
    (zero on the x-end rows).  Returns (N, R)."""
    g = np.asarray(g)
    batch = g.shape[:-2]
    R = int(np.prod(batch)) if batch else 1
    gg = g.reshape(R, n + 1, n + 1)
    b = np.zeros((R, n + 1, n - 1), dtype=complex)
    b[:, 1:n, :] = gg[:, 1:n, 1:n]
    return b.reshape(R, -1).T, batch


def _to_grid(x: np.ndarray, n: int, batch) -> np.ndarray:
    R = x.shape[1]
    u = np.zeros((R, n + 1, n + 1), dtype=complex)
    u[:, :, 1:n] = x.T.reshape(R, n + 1, n - 1)
    return u.reshape(tuple(batch) + (n + 1, n + 1))


def solve_dense(g: np.ndarray, n: int, h: float, k: float) -> np.ndarray:
    A = assemble(n, h, k).toarray()
    b, batch = _rhs_vector(g, n)
    return _to_grid(np.linalg.solve(A, b), n, batch)


class BandedAP:
    """G^(h) by LAPACK banded LU with partial pivoting of the assembled AP."""

    def __init__(self, n: int, h: float, k: float):
        self.n, self.h, self.k = n, h, k
        A = assemble(n, h, k).tocoo()
        N = A.shape[0]
        kl = ku = n  # unknowns are x-major with y fastest: couplings reach +-n
        ab = np.zeros((2 * kl + ku + 1, N), dtype=complex)
        # LAPACK band layout for gbtrf: A[i, j] -> ab[kl + ku + i - j, j]
        ab[kl + ku + A.row - A.col, A.col] = A.data
        lu, piv, info = lapack.zgbtrf(ab, kl, ku)
        if info != 0:
            raise np.linalg.LinAlgError("banded LU failed (info=%d)" % info)
        self.lu, self.piv, self.kl, self.ku = lu, piv, kl, ku

    def solve(self, g: np.ndarray) -> np.ndarray:
        b, batch = _rhs_vector(g, self.n)
        x, info = lapack.zgbtrs(self.lu, self.kl, self.ku, b, self.piv)
        if info != 0:
            raise np.linalg.LinAlgError("banded solve failed (info=%d)" % info)
        return _to_grid(x, self.n, batch)


def sine_matrix(n: int) -> np.ndarray:
    """S[q-1, j-1] = sin(pi j q / n), q, j = 1..n-1, argument reduced exactly mod 2n."""
    j = np.arange(1, n)
    jq = np.outer(j, j) % (2 * n)
    return np.sin(np.pi * jq / n)


class SeparableAP:
    """G^(h) by the sine transform in y (Dirichlet ends) and one tridiagonal solve
    in x per sine mode (LAPACK gtsv with partial pivoting through solve_banded).

    With u(m,q) = sum_j U(m,j) sin(pi j q/n) the second difference in y acts on
    mode j as multiplication by 2cos(pi j/n) - 2, so every row of the assembled
    system decouples into one tridiagonal system per j.  The forward transform
    is U = (2/n) sum_q g(q) sin(pi j q/n), the inverse of the synthesis above.
    """

    def __init__(self, n: int, h: float, k: float):
        self.n, self.h, self.k = n, h, k
        self.S = sine_matrix(n)
        c0, ce, cc = stencil_coefficients(h, k)
        cosj = np.cos(np.pi * np.arange(1, n) / n)
        off = ce + 2.0 * cc * cosj            # weight of U(m-1, j) and U(m+1, j)
        dia = c0 + 2.0 * ce * cosj            # weight of U(m, j)
        wD, wD2, wA, wA2 = end_row_weights(h, k)
        d2 = 2.0 * cosj - 2.0
        cD = wD + wD2 * d2                    # D coefficient per mode
        cA = 1j * k * (wA + wA2 * d2) * 0.5   # coefficient of each of the two A nodes (times sign)
        # banded storage (1,1): ab[0, 1:] super, ab[1, :] diag, ab[2, :-1] sub
        ab = np.zeros((n - 1, 3, n + 1), dtype=complex)
        ab[:, 1, 1:n] = dia[:, None]
        ab[:, 0, 2:n + 1] = off[:, None]      # super-diagonal of rows 1..n-1
        ab[:, 2, 0:n - 1] = off[:, None]      # sub-diagonal of rows 1..n-1
        # left row m = 0: cD*(U1 - U0) - cA*(U1 + U0) = 0
        ab[:, 1, 0] = -cD - cA
        ab[:, 0, 1] = cD - cA
        # right row m = n: cD*(Un - U(n-1)) + cA*(Un + U(n-1)) = 0
        ab[:, 1, n] = cD + cA
        ab[:, 2, n - 1] = -cD + cA
        self.ab = ab

    def forward(self, g: np.ndarray) -> np.ndarray:
        """(2/n) sine transform in q of g[..., m, q] over q = 1..n-1 -> [..., m, j-1]."""
        n = self.n
        return (2.0 / n) * (g[..., 1:n] @ self.S)

    def inverse(self, U: np.ndarray) -> np.ndarray:
        n = self.n
        u = np.zeros(U.shape[:-1] + (n + 1,), dtype=complex)
        u[..., 1:n] = U @ self.S
        return u

    def solve(self, g: np.ndarray) -> np.ndarray:
        n = self.n
        g = np.asarray(g)
        batch = g.shape[:-2]
        R = int(np.prod(batch)) if batch else 1
        gg = np.zeros((R, n + 1, n + 1), dtype=g.dtype)
        gg[:, 1:n, 1:n] = g.reshape(R, n + 1, n + 1)[:, 1:n, 1:n]
        G = self.forward(gg)                  # (R, n+1, n-1); rows m = 0, n are zero
        U = np.empty(G.shape, dtype=complex)
        for jj in range(n - 1):
            rhs = G[:, :, jj].T               # (n+1, R)
            U[:, :, jj] = solve_banded((1, 1), self.ab[jj], rhs).T
        return self.inverse(U).reshape(tuple(batch) + (n + 1, n + 1))


def make_solver(n: int, h: float, k: float, kind: str = "auto"):
    if kind == "auto":
        kind = "banded" if n <= 128 else "separable"
    if kind == "banded":
        return BandedAP(n, h, k)
    if kind == "separable":
        return SeparableAP(n, h, k)
    raise ValueError(kind)
