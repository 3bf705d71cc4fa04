"""Auxiliary grid and grid sets (paper Sec. 3.2.1-3.2.2).  Test infrastructure only.

Readings:
  * n is the number of cells per direction of the auxiliary square; nodes are
    numbered 0..n in x (index m) and y (index q); h is the side over n
    (Sec. 4: "n cells uniformly spaced in each direction", uniform h of
    eq. FD_scheme).
  * The auxiliary domain of a rectangle [x0,x0+lx]x[y0,y0+ly] is the square of
    side 1.1*max(lx, ly) centred on it (the paper uses side 2.2 around a square
    of side 2, Sec. 4, and allows any auxiliary domain, Sec. 3.2.1).
  * M0 = nodes not on the auxiliary boundary (1 <= m, q <= n-1);
    M+ = nodes of M0 inside the closed rectangle; M- = M0 \\ M+;
    N+- = nodes needed by the 3x3 stencil at M+- (the 3x3 dilation);
    gamma = N+ intersect N- (Sec. 3.2.2).
  * gamma is listed in the order of increasing (m, q) lexicographically.
  * Side of a gamma node: the side whose outward signed distance rho is the
    largest (rho > 0 outside); a vertical side (left/right) wins ties within
    1e-9 h.  rho of the chosen side is the distance used by the Taylor
    extension and the tangential coordinate is not clamped to the side.
"""
from __future__ import annotations

import numpy as np

BOTTOM, TOP, LEFT, RIGHT = 0, 1, 2, 3


class APGrid:
    def __init__(self, x0: float, y0: float, lx: float, ly: float, n: int):
        if n < 8:
            raise ValueError("n must be >= 8")
        self.x0, self.y0, self.lx, self.ly, self.n = float(x0), float(y0), float(lx), float(ly), int(n)
        L = 1.1 * max(lx, ly)
        self.L = L
        self.h = L / n
        cx, cy = x0 + 0.5 * lx, y0 + 0.5 * ly
        self.xa = cx - 0.5 * L
        self.ya = cy - 0.5 * L
        m = np.arange(n + 1)
        self.xs = self.xa + m * self.h
        self.ys = self.ya + m * self.h

        # M+ : nodes of M0 inside the closed rectangle
        inx = (self.xs >= x0) & (self.xs <= x0 + lx)
        iny = (self.ys >= y0) & (self.ys <= y0 + ly)
        inx[0] = inx[n] = False
        iny[0] = iny[n] = False
        mp = np.zeros((n + 1, n + 1), dtype=bool)      # indexed [m, q]
        mp[np.ix_(inx, iny)] = True
        m0 = np.zeros_like(mp)
        m0[1:n, 1:n] = True
        mm = m0 & ~mp
        self.Mplus, self.Mminus, self.M0 = mp, mm, m0
        self.Nplus = self._dilate(mp)
        self.Nminus = self._dilate(mm)
        self.gamma_mask = self.Nplus & self.Nminus
        gm, gq = np.nonzero(self.gamma_mask)            # lexicographic in (m, q)
        self.gamma_m, self.gamma_q = gm, gq
        self.n_gamma = gm.size
        # counts of M+ nodes along x and y
        self.cx = int(inx.sum())
        self.cy = int(iny.sum())
        self._side_map()

    @staticmethod
    def _dilate(mask: np.ndarray) -> np.ndarray:
        out = mask.copy()
        n1 = mask.shape[0]
        for dm in (-1, 0, 1):
            for dq in (-1, 0, 1):
                sh = np.zeros_like(mask)
                ms = slice(max(dm, 0), n1 + min(dm, 0))
                md = slice(max(-dm, 0), n1 + min(-dm, 0))
                qs = slice(max(dq, 0), n1 + min(dq, 0))
                qd = slice(max(-dq, 0), n1 + min(-dq, 0))
                sh[md, qd] = mask[ms, qs]
                out |= sh
        return out

    def _side_map(self):
        x = self.xs[self.gamma_m]
        y = self.ys[self.gamma_q]
        rho = np.stack([self.y0 - y,                    # bottom
                        y - (self.y0 + self.ly),        # top
                        self.x0 - x,                    # left
                        x - (self.x0 + self.lx)], 1)    # right
        tol = 1e-9 * self.h
        side = np.empty(self.n_gamma, dtype=np.int64)
        for i in range(self.n_gamma):
            r = rho[i]
            vbest = max(r[LEFT], r[RIGHT])
            hbest = max(r[BOTTOM], r[TOP])
            if vbest >= hbest - tol:
                side[i] = LEFT if r[LEFT] >= r[RIGHT] else RIGHT
            else:
                side[i] = BOTTOM if r[BOTTOM] >= r[TOP] else TOP
        self.side = side
        self.rho = rho[np.arange(self.n_gamma), side]
        # tangential parameter t in [-1, 1] (+O(h) beyond the corners), increasing
        # with global x on horizontal sides and with global y on vertical sides
        horiz = (side == BOTTOM) | (side == TOP)
        self.t = np.where(horiz, 2.0 * (x - self.x0) / self.lx - 1.0, 2.0 * (y - self.y0) / self.ly - 1.0)
        self.side_len = np.where(horiz, self.lx, self.ly)

    def gamma_index_map(self) -> np.ndarray:
        """(n+1)x(n+1) int array: position of each node in the gamma list, -1 elsewhere."""
        g = -np.ones((self.n + 1, self.n + 1), dtype=np.int64)
        g[self.gamma_m, self.gamma_q] = np.arange(self.n_gamma)
        return g
