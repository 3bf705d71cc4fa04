"""End-to-end MDP domain-decomposition solve (paper Sec. 3.5).  Test infrastructure only.

Step 1: per subdomain, the auxiliary problem, grid sets and Q (cached per
distinct rectangle size, n, k and M*, Sec. 3.5: Q is computed once per distinct
wavenumber and reused).  Step 2: the reduced least-squares system.  Step 3: per
subdomain, xi_gamma = Ex (sum of c times basis pairs) and u = P_{N+} xi_gamma
(eq. potential_solution_homo, f = 0).  With a source f (Sec. 3.5 step 1c): the
per-subdomain right-hand sides F^(i) join the reduced system, Ex^(I) f joins
xi_gamma and u = P_{N+} xi_gamma + G B f (eq. potential_solution).  The error is
the maximum over M+ of all subdomains (Sec. 4).
"""
from __future__ import annotations

import numpy as np

from paper_2103_12172_amd import workloads as wl

from .extension import chebyshev_coefficients, chebyshev_points, extension_matrix
from .grid import APGrid
from .interface import solve_interface
from .projector import build_projector, potential
from .scheme import make_solver
from . import source as osrc


def boundary_coefficients(w, m_star):
    t = chebyshev_points(m_star)
    d = []
    for i in range(len(w.subdomains)):
        di = []
        for s in range(4):
            if w.sides[i][s].kind == wl.BOUNDARY:
                di.append(chebyshev_coefficients(wl.boundary_samples(w, i, s, t)))
            else:
                di.append(None)
        d.append(di)
    return d


def dd_solve(w, solver_kind: str = "auto", cache=None):
    m_star = w.m_star
    cache = {} if cache is None else cache
    grids, Qs, solvers, Es = [], [], [], []
    for sd in w.subdomains:
        grid = APGrid(sd.x0, sd.y0, sd.lx, sd.ly, sd.n)
        key = (sd.lx, sd.ly, sd.n, sd.k, m_star)
        if key not in cache:
            solver = make_solver(sd.n, grid.h, sd.k, solver_kind)
            cache[key] = (solver, build_projector(grid, sd.k, m_star, solver), extension_matrix(grid, sd.k, m_star))
        solver, Q, E = cache[key]
        grids.append(grid)
        Qs.append(Q)
        solvers.append(solver)
        Es.append(E)
    d = boundary_coefficients(w, m_star)
    F_src, fgs, xis_i = None, None, None
    if w.source is not None:
        F_src, fgs, xis_i = [], [], []
        for i, sd in enumerate(w.subdomains):
            fg = osrc.source_grid(grids[i], w.source)
            jv = osrc.source_jet(grids[i], w.source_jet)
            fgs.append(fg)
            xis_i.append(osrc.extension_inhomogeneous(grids[i], sd.k, jv))
            F_src.append(osrc.system_rhs(grids[i], sd.k, fg, jv, solvers[i]))
    c, x, info, _ = solve_interface(Qs, w.sides, d, m_star, F_src)
    us, err = [], 0.0
    for i, sd in enumerate(w.subdomains):
        grid = grids[i]
        xi = Es[i] @ c[i]
        if w.source is None:
            u = potential(grid, sd.k, xi, solvers[i])
        else:
            u = osrc.potential_with_source(grid, sd.k, xi + xis_i[i], fgs[i], solvers[i])
        us.append(u)
        X, Y = np.meshgrid(grid.xs, grid.ys, indexing="ij")
        ex = w.exact(X, Y)
        err = max(err, float(np.max(np.abs(u - ex)[grid.Mplus])))
    info["error_max_Mplus"] = err
    return {"u": us, "c": c, "x": x, "grids": grids, "Q": Qs, "d": d, "info": info, "F_src": F_src}
