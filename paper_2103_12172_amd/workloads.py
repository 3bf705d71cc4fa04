"""Seeded synthetic workloads for the MDP domain-decomposition hot path.

This module only *describes* problems: subdomain rectangles, wavenumbers,
grid sizes, boundary-condition kinds, the exact test solutions and their
boundary samples.  It holds none of the method's arithmetic (no stencil, no
auxiliary-problem solve, no extension, no Chebyshev expansion, no least
squares), so both the CPU oracle and the GPU path can draw their inputs from
here without sharing any of the computation they are compared on.

Geometry conventions (paper Sec. 3.3-3.4):
  * a subdomain is an axis-aligned rectangle [x0, x0+lx] x [y0, y0+ly] with a
    constant wavenumber k (Sec. 3.1 assumes k constant on every subdomain);
  * its four sides are numbered 0 = bottom (y = y0), 1 = top (y = y0+ly),
    2 = left (x = x0), 3 = right (x = x0+lx);
  * a side is either an outer boundary carrying alpha*u + beta*du/dn = phi
    (eq. helmholtz_robin, outward normal n) or an interface shared with one
    side of a neighbouring subdomain (Sec. 3.3.2);
  * the auxiliary grid has n cells per direction.

Test solutions of the homogeneous equation (f = 0):
  * plane wave exp(i k (x cos(theta) + y sin(theta)));
  * the piecewise plane wave of Appendix A: in strip i,
    a_i exp(i k_i x) + b_i exp(-i k_i x), amplitudes fixed by continuity of u
    and u_x at every interface with a_1 = 1 (incident wave) and b_N = 0 (no
    reflection from the right end).  The closed form for two strips printed in
    the appendix (eq. R_T_solved) does not satisfy its own derivative
    condition; the amplitudes here come from solving the appendix's linear
    system directly, which for two strips gives R = (k1-k2)/(k1+k2) and
    T = 2 k1/(k1+k2).

Problems with a source f (eq. helmholtz, Delta u + k^2 u = f):
  * a manufactured plane wave exp(i (a x + b y)) with a^2 + b^2 != k^2, so that
    f = (k^2 - a^2 - b^2) u;
  * sin^4(pi x) sin(pi y) (a test solution of Table uniform_2), f = Delta u + k^2 u
    in closed form;
  * the compactly supported bump of eq. source_bump with homogeneous boundary
    data (no exact solution; grid self-convergence).  Reading: the printed
    support x^2 + y^2 < 1/2 does not match the singular point of the exponent,
    r^2 = 1/4; the support used is r^2 < 1/4 (the function and all its
    derivatives vanish there, so f is smooth).
A source is described by f(x, y) (sampled on the auxiliary grids) and its jet
at boundary points with outward normal (nx, ny): (f, df/dn, d2f/dn2 - d2f/dtau2),
the terms of the equation-based extension that involve f (eqs. cart_ext_2-4).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Tuple

import numpy as np

BOTTOM, TOP, LEFT, RIGHT = 0, 1, 2, 3
SIDE_NAMES = ("bottom", "top", "left", "right")
BOUNDARY, INTERFACE = 0, 1


@dataclass
class Subdomain:
    x0: float
    y0: float
    lx: float
    ly: float
    k: float
    n: int


@dataclass
class Side:
    kind: int                 # BOUNDARY or INTERFACE
    alpha: float = 0.0        # boundary: alpha*u + beta*du/dn = phi
    beta: float = 0.0
    nbr: int = -1             # interface: neighbour subdomain index
    nbr_side: int = -1        # interface: neighbour's side index


@dataclass
class Workload:
    name: str
    subdomains: List[Subdomain]
    sides: List[List[Side]]   # sides[i][s]
    m_star: int
    exact: Callable           # exact(x, y) -> complex ndarray
    exact_grad: Callable      # exact_grad(x, y) -> (u_x, u_y) complex ndarrays
    precision: str = "c128"   # compute precision of the AP solves: c128 | c64 | c64r
    notes: str = ""
    extra: dict = field(default_factory=dict)
    source: Optional[Callable] = None      # f(x, y) -> complex ndarray (None: f = 0)
    source_jet: Optional[Callable] = None  # (x, y, nx, ny) -> (f, df/dn, d2f/dn2 - d2f/dtau2)
    has_exact: bool = True                  # exact() is the solution (False: boundary data only)


# ----------------------------------------------------------------- solutions
def plane_wave(k: float, theta: float):
    c, s = math.cos(theta), math.sin(theta)

    def u(x, y):
        return np.exp(1j * k * (np.asarray(x) * c + np.asarray(y) * s))

    def grad(x, y):
        v = u(x, y)
        return 1j * k * c * v, 1j * k * s * v

    return u, grad


def manufactured_plane_wave(k: float, a: float, b: float):
    """u = exp(i (a x + b y)) and its source f = (k^2 - a^2 - b^2) u with the jet of f."""
    amp = k * k - a * a - b * b

    def u(x, y):
        return np.exp(1j * (a * np.asarray(x) + b * np.asarray(y)))

    def grad(x, y):
        v = u(x, y)
        return 1j * a * v, 1j * b * v

    def f(x, y):
        return amp * u(x, y)

    def jet(x, y, nx, ny):
        v = f(x, y)
        dn = a * nx + b * ny            # derivative along the normal: i dn
        dt = -a * ny + b * nx           # along the tangent (-ny, nx)
        return v, 1j * dn * v, (-dn * dn + dt * dt) * v

    return u, grad, f, jet


def sin4_solution(k: float):
    """u = sin^4(pi x) sin(pi y), f = Delta u + k^2 u = sin(pi y) P(x) with
    P = 3 pi^2/2 (1 - cos 4 pi x) + (k^2 - 5 pi^2)/8 (3 - 4 cos 2 pi x + cos 4 pi x)."""
    pi = math.pi
    c1 = 1.5 * pi * pi
    c2 = (k * k - 5.0 * pi * pi) / 8.0

    def u(x, y):
        return (np.sin(pi * np.asarray(x)) ** 4 * np.sin(pi * np.asarray(y))).astype(complex)

    def grad(x, y):
        x, y = np.asarray(x), np.asarray(y)
        sx = np.sin(pi * x)
        return ((4.0 * pi * sx ** 3 * np.cos(pi * x) * np.sin(pi * y)).astype(complex),
                (pi * sx ** 4 * np.cos(pi * y)).astype(complex))

    def P(x, d=0):
        c2x, c4x = np.cos(2 * pi * x), np.cos(4 * pi * x)
        s2x, s4x = np.sin(2 * pi * x), np.sin(4 * pi * x)
        if d == 0:
            return c1 * (1.0 - c4x) + c2 * (3.0 - 4.0 * c2x + c4x)
        if d == 1:
            return c1 * 4 * pi * s4x + c2 * (8 * pi * s2x - 4 * pi * s4x)
        return c1 * 16 * pi * pi * c4x + c2 * (16 * pi * pi * c2x - 16 * pi * pi * c4x)

    def f(x, y):
        x, y = np.asarray(x), np.asarray(y)
        return (np.sin(pi * y) * P(x)).astype(complex)

    def jet(x, y, nx, ny):
        x, y = np.asarray(x, dtype=float), np.asarray(y, dtype=float)
        sy, cy = np.sin(pi * y), np.cos(pi * y)
        fx, fy = sy * P(x, 1), pi * cy * P(x)
        fxx, fyy, fxy = sy * P(x, 2), -pi * pi * sy * P(x), pi * cy * P(x, 1)
        tx, ty = -ny, nx
        fn = nx * fx + ny * fy
        fnn = nx * nx * fxx + 2 * nx * ny * fxy + ny * ny * fyy
        ftt = tx * tx * fxx + 2 * tx * ty * fxy + ty * ty * fyy
        return f(x, y), fn.astype(complex), (fnn - ftt).astype(complex)

    return u, grad, f, jet


def bump_source(x0: float = 0.0, y0: float = 0.0):
    """f = exp(-1/(1/4 - r^2)) for r^2 = (x-x0)^2 + (y-y0)^2 < 1/4, else 0 (eq. source_bump,
    support read as r^2 < 1/4), with its jet: f_x = f * dE/dx for the exponent E = -1/(1/4 - r^2)."""

    def f(x, y):
        x, y = np.asarray(x, dtype=float), np.asarray(y, dtype=float)
        r2 = (x - x0) ** 2 + (y - y0) ** 2
        out = np.zeros(np.broadcast(x, y).shape, dtype=complex)
        inside = r2 < 0.25
        d = 0.25 - r2[inside] if np.ndim(r2) else 0.25 - r2
        if np.ndim(r2):
            out[inside] = np.exp(-1.0 / d)
            return out
        return complex(np.exp(-1.0 / d)) if inside else 0j

    def jet(x, y, nx, ny):
        x, y = np.asarray(x, dtype=float), np.asarray(y, dtype=float)
        X, Y = x - x0, y - y0
        r2 = X * X + Y * Y
        inside = r2 < 0.25
        d = np.where(inside, 0.25 - r2, 1.0)
        e = np.where(inside, np.exp(-1.0 / d), 0.0)
        # E = -1/d, dE/dx = -2X/d^2, d2E/dx2 = -2/d^2 - 8X^2/d^3, d2E/dxdy = -8XY/d^3
        Ex, Ey = -2 * X / d ** 2, -2 * Y / d ** 2
        Exx = -2 / d ** 2 - 8 * X * X / d ** 3
        Eyy = -2 / d ** 2 - 8 * Y * Y / d ** 3
        Exy = -8 * X * Y / d ** 3
        fx, fy = e * Ex, e * Ey
        fxx, fyy, fxy = e * (Exx + Ex * Ex), e * (Eyy + Ey * Ey), e * (Exy + Ex * Ey)
        tx, ty = -ny, nx
        fn = nx * fx + ny * fy
        fnn = nx * nx * fxx + 2 * nx * ny * fxy + ny * ny * fyy
        ftt = tx * tx * fxx + 2 * tx * ty * fxy + ty * ty * fyy
        return e.astype(complex), fn.astype(complex), (fnn - ftt).astype(complex)

    return f, jet


def piecewise_amplitudes(interfaces: List[float], ks: List[float]) -> Tuple[np.ndarray, np.ndarray]:
    """Amplitudes (a_i, b_i) of a_i e^{i k_i x} + b_i e^{-i k_i x} on N strips.

    Unknowns: b_1, a_2, b_2, ..., a_{N-1}, b_{N-1}, a_N (2N-2 of them) with
    a_1 = 1 and b_N = 0; equations: continuity of u and of u_x at the N-1
    interfaces x_1 < ... < x_{N-1} (Appendix A, four-strip system and its
    N-strip generalisation).
    """
    N = len(ks)
    assert len(interfaces) == N - 1
    if N == 1:
        return np.array([1.0 + 0j]), np.array([0.0 + 0j])
    nunk = 2 * N - 2

    def col(i, which):  # which 0 -> a_i, 1 -> b_i ; returns unknown index or None
        if i == 0 and which == 0:
            return None
        if i == N - 1 and which == 1:
            return None
        return 2 * i - 1 + which  # b_1 -> 0, a_2 -> 1, b_2 -> 2, ...

    A = np.zeros((nunk, nunk), dtype=complex)
    rhs = np.zeros(nunk, dtype=complex)
    for j, xj in enumerate(interfaces):
        left, right = j, j + 1
        for row, deriv in ((2 * j, False), (2 * j + 1, True)):
            for strip, sgn in ((left, 1.0), (right, -1.0)):
                k = ks[strip]
                for which, e in ((0, np.exp(1j * k * xj)), (1, np.exp(-1j * k * xj))):
                    coef = sgn * e
                    if deriv:
                        coef *= (1j * k) if which == 0 else (-1j * k)
                    c = col(strip, which)
                    if c is None:
                        if strip == 0 and which == 0:
                            rhs[row] -= coef  # a_1 = 1 known
                    else:
                        A[row, c] += coef
    sol = np.linalg.solve(A, rhs)
    a = np.zeros(N, dtype=complex)
    b = np.zeros(N, dtype=complex)
    a[0] = 1.0
    for i in range(N):
        for which in (0, 1):
            c = col(i, which)
            if c is not None:
                (a if which == 0 else b)[i] = sol[c]
    return a, b


def piecewise_plane_wave(interfaces: List[float], ks: List[float]):
    a, b = piecewise_amplitudes(interfaces, ks)
    edges = np.asarray(interfaces, dtype=float)
    kk = np.asarray(ks, dtype=float)

    def strip_of(x):
        return np.searchsorted(edges, np.asarray(x, dtype=float), side="right")

    def u(x, y):
        x = np.asarray(x, dtype=float)
        i = strip_of(x)
        return a[i] * np.exp(1j * kk[i] * x) + b[i] * np.exp(-1j * kk[i] * x) + 0 * np.asarray(y)

    def grad(x, y):
        x = np.asarray(x, dtype=float)
        i = strip_of(x)
        ux = 1j * kk[i] * (a[i] * np.exp(1j * kk[i] * x) - b[i] * np.exp(-1j * kk[i] * x))
        return ux + 0 * np.asarray(y), 0 * ux + 0 * np.asarray(y)

    return u, grad, a, b


# ----------------------------------------------------------------- topology
def grid_topology(nx: int, ny: int, x0: float, y0: float, lx: float, ly: float,
                  ks: List[float], n: List[int] | int,
                  bc: Callable[[int, int, int], Tuple[float, float]]):
    """nx*ny rectangles of size lx*ly, row-major from (x0, y0) (index = iy*nx + ix).

    bc(ix, iy, side) -> (alpha, beta) for the sides on the outer boundary.
    """
    subs, sides = [], []
    for iy in range(ny):
        for ix in range(nx):
            i = iy * nx + ix
            nn = n[i] if isinstance(n, (list, tuple, np.ndarray)) else n
            subs.append(Subdomain(x0 + ix * lx, y0 + iy * ly, lx, ly, float(ks[i]), int(nn)))
            ss = []
            for s in range(4):
                nb = {BOTTOM: (ix, iy - 1, TOP), TOP: (ix, iy + 1, BOTTOM),
                      LEFT: (ix - 1, iy, RIGHT), RIGHT: (ix + 1, iy, LEFT)}[s]
                jx, jy, js = nb
                if 0 <= jx < nx and 0 <= jy < ny:
                    ss.append(Side(INTERFACE, nbr=jy * nx + jx, nbr_side=js))
                else:
                    a, b = bc(ix, iy, s)
                    ss.append(Side(BOUNDARY, alpha=a, beta=b))
            sides.append(ss)
    return subs, sides


def side_points(sd: Subdomain, s: int, t: np.ndarray):
    """Physical points on side s at affine parameter t in [-1, 1].

    The parameter increases with global x on horizontal sides and with global
    y on vertical sides, so the two subdomains sharing an interface agree on it.
    """
    t = np.asarray(t, dtype=float)
    if s in (BOTTOM, TOP):
        x = sd.x0 + 0.5 * (t + 1.0) * sd.lx
        y = np.full_like(x, sd.y0 if s == BOTTOM else sd.y0 + sd.ly)
    else:
        y = sd.y0 + 0.5 * (t + 1.0) * sd.ly
        x = np.full_like(y, sd.x0 if s == LEFT else sd.x0 + sd.lx)
    return x, y


def outward_normal(s: int) -> Tuple[float, float]:
    return {BOTTOM: (0.0, -1.0), TOP: (0.0, 1.0), LEFT: (-1.0, 0.0), RIGHT: (1.0, 0.0)}[s]


def boundary_samples(w: Workload, i: int, s: int, t: np.ndarray) -> np.ndarray:
    """phi = alpha*u + beta*du/dn of the exact solution at side parameters t."""
    sd = w.subdomains[i]
    side = w.sides[i][s]
    assert side.kind == BOUNDARY
    x, y = side_points(sd, s, t)
    ux, uy = w.exact_grad(x, y)
    nx, ny = outward_normal(s)
    return side.alpha * w.exact(x, y) + side.beta * (nx * ux + ny * uy)


# ----------------------------------------------------------------- workloads
def config_two_rect(n: int = 64, k: float = 10.0, m_star: int = 16, precision: str = "c128") -> Workload:
    """Unit square as 2x1 rectangles [0,.5]x[0,1] and [.5,1]x[0,1]; Dirichlet
    data of the plane wave at angle pi/6 on the six outer sides."""
    subs, sides = grid_topology(2, 1, 0.0, 0.0, 0.5, 1.0, [k, k], n, lambda ix, iy, s: (1.0, 0.0))
    u, g = plane_wave(k, math.pi / 6)
    return Workload("two_rect_k10_n%d" % n, subs, sides, m_star, u, g, precision,
                    notes="2x1 rectangles, k=%g, n=%d, M*=%d, Dirichlet, plane wave pi/6" % (k, n, m_star))


def config_cross_point(n: int = 256, k: float = 50.0, m_star: int = 32, seed: int = 2,
                       precision: str = "c64r") -> Workload:
    """Unit square as 2x2 squares of side 0.5 (one interior cross-point);
    Dirichlet on the x = 0 and x = 1 sides, Neumann on y = 0 and y = 1; plane
    wave at a seed-drawn angle theta = 2*pi*U[0,1)."""
    rng = np.random.default_rng(seed)
    theta = 2.0 * math.pi * float(rng.random())

    def bc(ix, iy, s):
        return (1.0, 0.0) if s in (LEFT, RIGHT) else (0.0, 1.0)

    subs, sides = grid_topology(2, 2, 0.0, 0.0, 0.5, 0.5, [k] * 4, n, bc)
    u, g = plane_wave(k, theta)
    w = Workload("cross_point_k50_n%d" % n, subs, sides, m_star, u, g, precision,
                 notes="2x2 squares, k=%g, n=%d, M*=%d, mixed Dirichlet/Neumann, theta=%.6f (seed %d)"
                 % (k, n, m_star, theta, seed))
    w.extra["theta"] = theta
    return w


def config_transmission(n: int = 1024, ks=(20.0, 200.0, 20.0, 200.0), m_star: int = 64,
                        precision: str = "c64r") -> Workload:
    """Unit square as 4 vertical strips [i/4,(i+1)/4]x[0,1] with alternating
    wavenumbers; exact piecewise plane wave; Dirichlet data on the outer sides."""
    N = len(ks)
    subs, sides = grid_topology(N, 1, 0.0, 0.0, 1.0 / N, 1.0, list(ks), n, lambda ix, iy, s: (1.0, 0.0))
    u, g, a, b = piecewise_plane_wave([(i + 1) / N for i in range(N - 1)], list(ks))
    w = Workload("transmission_%dstrips_n%d" % (N, n), subs, sides, m_star, u, g, precision,
                 notes="%d strips, k=%s, n=%d, M*=%d, Dirichlet, piecewise plane wave" % (N, list(ks), n, m_star))
    w.extra["a"], w.extra["b"] = a, b
    return w


def config_paper_base(n: int = 64, k: float = 13.0, m_star: int = 40) -> Workload:
    """Single square of side 2 centred at the origin, Robin alpha = beta = 1,
    plane wave exp(i k (x+y)/sqrt 2) (the single-subdomain base case of Sec. 4.1)."""
    subs, sides = grid_topology(1, 1, -1.0, -1.0, 2.0, 2.0, [k], n, lambda ix, iy, s: (1.0, 1.0))
    u, g = plane_wave(k, math.pi / 4)
    return Workload("paper_base_n%d" % n, subs, sides, m_star, u, g, "c128")


def config_paper_two(n: int = 64, k: float = 13.0, m_star: int = 40) -> Workload:
    """Two squares of side 2: the first centred at the origin, the second to its
    right (interface at x = 1); Robin alpha = beta = 1; plane wave at pi/4."""
    subs, sides = grid_topology(2, 1, -1.0, -1.0, 2.0, 2.0, [k, k], n, lambda ix, iy, s: (1.0, 1.0))
    u, g = plane_wave(k, math.pi / 4)
    return Workload("paper_two_n%d" % n, subs, sides, m_star, u, g, "c128")


def config_paper_jump(n: int = 64, k1: float = 5.0, k2: float = 13.0, m_star: int = 40) -> Workload:
    """Two squares of side 2 (interface at x = 1) with k1 | k2, incident wave
    e^{i k1 x}, Dirichlet data (the two-subdomain transmission case of Sec. 4.2)."""
    subs, sides = grid_topology(2, 1, -1.0, -1.0, 2.0, 2.0, [k1, k2], n, lambda ix, iy, s: (1.0, 0.0))
    u, g, a, b = piecewise_plane_wave([1.0], [k1, k2])
    return Workload("paper_jump_%g_%g_n%d" % (k1, k2, n), subs, sides, m_star, u, g, "c128")


def config_paper_sin4(n: int = 64, k: float = 13.0, m_star: int = 40) -> Workload:
    """Two squares of side 2 (interface at x = 1), Robin alpha = beta = 1, the
    inhomogeneous test solution sin^4(pi x) sin(pi y) of Table uniform_2."""
    subs, sides = grid_topology(2, 1, -1.0, -1.0, 2.0, 2.0, [k, k], n, lambda ix, iy, s: (1.0, 1.0))
    u, g, f, jet = sin4_solution(k)
    return Workload("paper_sin4_n%d" % n, subs, sides, m_star, u, g, "c128", source=f, source_jet=jet,
                    notes="2 squares of side 2, k=%g, n=%d, M*=%d, Robin 1/1, u = sin^4(pi x) sin(pi y)"
                    % (k, n, m_star))


def config_source_plane(n: int = 64, k: float = 10.0, m_star: int = 16, a: float = 6.0, b: float = 5.0) -> Workload:
    """The 2x1 rectangles of two_rect with the manufactured wave exp(i(a x + b y)),
    a^2 + b^2 != k^2, and its source; Dirichlet data."""
    subs, sides = grid_topology(2, 1, 0.0, 0.0, 0.5, 1.0, [k, k], n, lambda ix, iy, s: (1.0, 0.0))
    u, g, f, jet = manufactured_plane_wave(k, a, b)
    return Workload("source_plane_n%d" % n, subs, sides, m_star, u, g, "c128", source=f, source_jet=jet,
                    notes="2x1 rectangles, k=%g, n=%d, M*=%d, Dirichlet, u = exp(i(%gx+%gy)) with its source"
                    % (k, n, m_star, a, b))


def config_bump(n: int = 256, k: float = 50.0, m_star: int = 32) -> Workload:
    """2x2 squares of side 0.5 (the cross-point layout) with the bump source
    centred at the cross-point (0.5, 0.5) and homogeneous Dirichlet data; no
    exact solution (exact = 0 only gives the zero boundary data)."""
    subs, sides = grid_topology(2, 2, 0.0, 0.0, 0.5, 0.5, [k] * 4, n, lambda ix, iy, s: (1.0, 0.0))
    f, jet = bump_source(0.5, 0.5)

    def zero(x, y):
        return np.zeros(np.broadcast(np.asarray(x), np.asarray(y)).shape, dtype=complex)

    def zero_grad(x, y):
        z = zero(x, y)
        return z, z

    return Workload("bump_n%d" % n, subs, sides, m_star, zero, zero_grad, "c128", source=f, source_jet=jet,
                    has_exact=False,
                    notes="2x2 squares, k=%g, n=%d, M*=%d, Dirichlet 0, bump source at the cross-point"
                    % (k, n, m_star))


def config_uneven(nx: int = 16, ny: int = 16, n_choices=(128, 256, 384, 512), k_range=(20.0, 80.0),
                  m_star: int = 32, seed: int = 4, k_data: float = 50.0, theta: float = math.pi / 6) -> Workload:
    """Unit square as nx x ny equal squares with uneven AP grids and wavenumbers:
    every subdomain's n drawn uniformly from n_choices, then every k uniformly
    from k_range (one generator, all n first); Dirichlet data of the plane wave
    exp(i k_data (x cos theta + y sin theta)) on the outer sides.  The plane wave
    solves none of the subdomain equations, so there is no exact solution."""
    rng = np.random.default_rng(seed)
    N = nx * ny
    ns = [int(v) for v in rng.choice(np.asarray(n_choices), size=N)]
    ks = [float(v) for v in rng.uniform(k_range[0], k_range[1], size=N)]
    subs, sides = grid_topology(nx, ny, 0.0, 0.0, 1.0 / nx, 1.0 / ny, ks, ns, lambda ix, iy, s: (1.0, 0.0))
    u, g = plane_wave(k_data, theta)
    w = Workload("uneven_%dx%d" % (nx, ny), subs, sides, m_star, u, g, "c128", has_exact=False,
                 notes="%dx%d squares, n in %s, k in U[%g,%g] (seed %d), M*=%d, Dirichlet data of the plane "
                 "wave k=%g at theta=%.4f" % (nx, ny, list(n_choices), k_range[0], k_range[1], seed, m_star,
                                               k_data, theta))
    w.extra["ns"], w.extra["ks"] = ns, ks
    return w


def config_uneven_small(seed: int = 4) -> Workload:
    """The uneven layout at a size the oracle solves in seconds: 3x3 squares,
    n in {32, 48, 64}, k in U[5, 15], M* = 8, plane wave k = 10."""
    return config_uneven(3, 3, (32, 48, 64), (5.0, 15.0), 8, seed, 10.0)


def config_adjoint(nx: int = 4, ny: int = 4, n: int = 512, k2_range=(400.0, 3600.0), m_star: int = 32,
                   seed: int = 5, k_data: float = 40.0, theta: float = math.pi / 6, bc=None) -> Workload:
    """Unit square as nx x ny equal squares with piecewise-constant k^2 drawn
    uniformly from k2_range (numpy default_rng(seed)); data of the plane wave
    exp(i k_data (x cos theta + y sin theta)) on the outer sides (Dirichlet, or
    bc(ix, iy, side) -> (alpha, beta)).  No exact solution."""
    rng = np.random.default_rng(seed)
    k2 = rng.uniform(k2_range[0], k2_range[1], size=nx * ny)
    ks = [float(math.sqrt(v)) for v in k2]
    subs, sides = grid_topology(nx, ny, 0.0, 0.0, 1.0 / nx, 1.0 / ny, ks, n, bc or (lambda ix, iy, s: (1.0, 0.0)))
    u, g = plane_wave(k_data, theta)
    w = Workload("adjoint_%dx%d_n%d" % (nx, ny, n), subs, sides, m_star, u, g, "c128", has_exact=False,
                 notes="%dx%d squares, n=%d, k^2 in U[%g,%g] (seed %d), M*=%d, plane-wave data k=%g"
                 % (nx, ny, n, k2_range[0], k2_range[1], seed, m_star, k_data))
    w.extra["k2"] = [float(v) for v in k2]
    return w


def config_adjoint_small(seed: int = 5) -> Workload:
    """The adjoint layout at a size the oracle differentiates in seconds: 2x2
    squares, n = 24, k^2 in U[100, 400], M* = 5, plane-wave data k = 12;
    Dirichlet on x = 0, Neumann on y = 0, Robin (1, 1/2) on x = 1 and y = 1."""
    def bc(ix, iy, s):
        return {LEFT: (1.0, 0.0), BOTTOM: (0.0, 1.0), RIGHT: (1.0, 0.5), TOP: (1.0, 0.5)}[s]
    return config_adjoint(2, 2, 24, (100.0, 400.0), 5, seed, 12.0, bc=bc)


def receiver_points(w: Workload, count: int, seed: int):
    """count points uniform over the bounding box of the subdomains (seeded) and
    the subdomain holding each (the first in order whose closed rectangle does)."""
    rng = np.random.default_rng(seed)
    x0 = min(sd.x0 for sd in w.subdomains)
    x1 = max(sd.x0 + sd.lx for sd in w.subdomains)
    y0 = min(sd.y0 for sd in w.subdomains)
    y1 = max(sd.y0 + sd.ly for sd in w.subdomains)
    pts = np.column_stack([rng.uniform(x0, x1, size=count), rng.uniform(y0, y1, size=count)])
    owner = []
    for x, y in pts:
        for i, sd in enumerate(w.subdomains):
            if sd.x0 <= x <= sd.x0 + sd.lx and sd.y0 <= y <= sd.y0 + sd.ly:
                owner.append(i)
                break
    return pts, owner


WORKLOADS = {
    "two_rect": config_two_rect,
    "cross_point": config_cross_point,
    "transmission": config_transmission,
    "bump": config_bump,
    "uneven": config_uneven,
}


def random_rhs(shape, seed: int, complex_: bool = True) -> np.ndarray:
    """Seeded standard-normal test data (real or complex)."""
    rng = np.random.default_rng(seed)
    if complex_:
        return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return rng.standard_normal(shape)
