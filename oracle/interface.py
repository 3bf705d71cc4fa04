"""Coupling of the subdomains and the least-squares solve.  Test infrastructure only.

Follows paper Sec. 3.3-3.5:
  * the per-subdomain systems Q^(i) c^(i) = F^(i) (F^(i) from the source term,
    eq. linear_system_equations; zero for f = 0) are stacked
    block-diagonally (eqs. 2_block_system, N_block_system);
  * boundary conditions alpha c^(0) + beta c^(1) = d on every boundary side
    (eq. BC_coefficients) and interface conditions c^(0)_a = c^(0)_b,
    c^(1)_a = -c^(1)_b (eq. transmission_coefficients) are resolved by
    substitution and elimination (Sec. 3.3.3): Dirichlet and Neumann sides move
    the known block times its columns to the right-hand side; Robin sides use
    c^(1) = d/beta - (alpha/beta) c^(0) (eq. BCs_rewritten); interface blocks
    add (Dirichlet) or subtract (Neumann) the two subdomains' columns;
  * the reduced system Qbar c = Fbar (sum |gamma_i| x 4 N M*) is solved in the
    least-squares sense by a Householder QR factorisation and
    c = R^{-1} Q^* Fbar (Sec. 3.5, steps 2b-2c).

Readings: the Neumann coefficient c^(1) is the outward normal derivative on
every side; the interface unknowns are owned by the lexicographically first
(subdomain, side) of the pair; no row scaling is applied between subdomains.
Unknown blocks are numbered by first appearance over subdomains i = 0..N-1 and
sides s = 0..3; a Robin or Neumann side's unknown is its Dirichlet block, a
Dirichlet side's is its Neumann block, an interface owns a Dirichlet block
followed by a Neumann block.
"""
from __future__ import annotations

import numpy as np

BOUNDARY, INTERFACE = 0, 1


def _cols(m_star, s, kind):
    base = kind * 4 * m_star + s * m_star
    return slice(base, base + m_star)


def plan_unknowns(sides, m_star):
    """Unknown blocks as (type, [(i, s, kind, coefficient), ...]) column contributions."""
    blocks = []
    for i, ss in enumerate(sides):
        for s, side in enumerate(ss):
            if side.kind == BOUNDARY:
                a, b = side.alpha, side.beta
                if a == 0.0 and b == 0.0:
                    raise ValueError("boundary side with alpha = beta = 0")
                if b == 0.0:
                    blocks.append(("dirichlet", [(i, s, 1, 1.0)]))
                elif a == 0.0:
                    blocks.append(("neumann", [(i, s, 0, 1.0)]))
                else:
                    blocks.append(("robin", [(i, s, 0, 1.0), (i, s, 1, -a / b)]))
            else:
                j, t = side.nbr, side.nbr_side
                other = sides[j][t]
                if other.kind != INTERFACE or other.nbr != i or other.nbr_side != s:
                    raise ValueError("inconsistent interface (%d,%d)-(%d,%d)" % (i, s, j, t))
                if (i, s) < (j, t):
                    blocks.append(("interface", [(i, s, 0, 1.0), (j, t, 0, 1.0)]))
                    blocks.append(("interface", [(i, s, 1, 1.0), (j, t, 1, -1.0)]))
    return blocks


def assemble(Qs, sides, d, m_star, F_src=None):
    """Reduced system (Qbar, Fbar) from per-subdomain Q matrices, boundary coefficients d[i][s]
    and the per-subdomain right-hand sides F_src[i] of the source term (None: f = 0)."""
    N = len(sides)
    rows = [Q.shape[0] for Q in Qs]
    off = np.concatenate([[0], np.cumsum(rows)])
    blocks = plan_unknowns(sides, m_star)
    Qbar = np.zeros((off[-1], len(blocks) * m_star), dtype=complex)
    Fbar = np.zeros(off[-1], dtype=complex)
    if F_src is not None:
        for i in range(N):
            if F_src[i] is not None:
                Fbar[off[i]:off[i + 1]] += F_src[i]
    for b, (_, contrib) in enumerate(blocks):
        for (i, s, kind, coef) in contrib:
            Qbar[off[i]:off[i + 1], b * m_star:(b + 1) * m_star] += coef * Qs[i][:, _cols(m_star, s, kind)]
    for i in range(N):
        for s, side in enumerate(sides[i]):
            if side.kind != BOUNDARY:
                continue
            a, bb = side.alpha, side.beta
            di = np.asarray(d[i][s], dtype=complex)
            Qi = Qs[i]
            if bb == 0.0:
                Fbar[off[i]:off[i + 1]] -= Qi[:, _cols(m_star, s, 0)] @ (di / a)
            else:
                Fbar[off[i]:off[i + 1]] -= Qi[:, _cols(m_star, s, 1)] @ (di / bb)
    return Qbar, Fbar, blocks


def expand(x, sides, d, m_star, blocks):
    """Full coefficient vectors c^(i) (8M* each, column order of Q) from the unknowns x."""
    N = len(sides)
    c = [np.zeros(8 * m_star, dtype=complex) for _ in range(N)]
    for b, (btype, contrib) in enumerate(blocks):
        xb = x[b * m_star:(b + 1) * m_star]
        if btype == "robin":            # only the Dirichlet block is unknown; the Neumann one follows below
            i, s, _, _ = contrib[0]
            c[i][_cols(m_star, s, 0)] = xb
        else:
            for (i, s, kind, coef) in contrib:
                c[i][_cols(m_star, s, kind)] = coef * xb
    for i in range(N):
        for s, side in enumerate(sides[i]):
            if side.kind != BOUNDARY:
                continue
            a, bb = side.alpha, side.beta
            di = np.asarray(d[i][s], dtype=complex)
            if bb == 0.0:
                c[i][_cols(m_star, s, 0)] = di / a
            elif a == 0.0:
                c[i][_cols(m_star, s, 1)] = di / bb
            else:
                c[i][_cols(m_star, s, 1)] = di / bb - (a / bb) * c[i][_cols(m_star, s, 0)]
    return c


def householder_qr_solve(A, b):
    """Least squares min ||A x - b||_2 by Householder QR (complex), x = R^{-1} (Q^* b)[:n].

    Returns (x, R, residual norm).  Reflector for column kk: v = x - alpha e1 with
    alpha = -exp(i arg x_0) ||x||, H = I - 2 v v^* / (v^* v).
    """
    A = np.array(A, dtype=complex, copy=True)
    y = np.array(b, dtype=complex, copy=True)
    m, n = A.shape
    if m < n:
        raise ValueError("least squares needs rows >= columns")
    for kk in range(n):
        x = A[kk:, kk]
        nx = np.sqrt(np.vdot(x, x).real)
        if nx == 0.0:
            continue
        x0 = x[0]
        phase = x0 / abs(x0) if x0 != 0 else 1.0
        alpha = -phase * nx
        v = x.copy()
        v[0] -= alpha
        v /= np.sqrt(np.vdot(v, v).real)
        A[kk:, kk:] -= 2.0 * np.outer(v, v.conj() @ A[kk:, kk:])
        y[kk:] -= 2.0 * v * np.vdot(v, y[kk:])
    R = np.triu(A[:n, :n])
    x = np.zeros(n, dtype=complex)
    for i in range(n - 1, -1, -1):                  # back substitution R x = (Q^* b)[:n]
        x[i] = (y[i] - R[i, i + 1:] @ x[i + 1:]) / R[i, i]
    res = float(np.linalg.norm(y[n:]))
    return x, R, res


def solve_interface(Qs, sides, d, m_star, F_src=None):
    Qbar, Fbar, blocks = assemble(Qs, sides, d, m_star, F_src)
    x, R, res = householder_qr_solve(Qbar, Fbar)
    c = expand(x, sides, d, m_star, blocks)
    info = {"rows": Qbar.shape[0], "cols": Qbar.shape[1], "residual": res,
            "rel_residual": res / max(np.linalg.norm(Fbar), 1e-300)}
    return c, x, info, (Qbar, Fbar, R)
