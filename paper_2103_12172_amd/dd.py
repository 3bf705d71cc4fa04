"""The three algorithm steps of the paper (Sec. 3.5) chained through the C-ABI.

Argument marshalling only: boundary data are sampled from the workload at the
library's Chebyshev points, turned into coefficients by the library, and the
projector build, interface least squares and reconstruction all run in
libmdp on the GPU.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

from . import mdp
from . import workloads as wl


@dataclass
class DDResult:
    u: object            # torch complex128, all subdomain grids concatenated
    c: object            # torch complex128, 8M* coefficients per subdomain
    rel_residual: float
    cond: Optional[float]
    offsets: List[int]   # start of each subdomain's grid in u
    projectors: List[object]


def subdomain_structs(w: wl.Workload) -> List[mdp.Subdomain]:
    return [mdp.Subdomain(sd.x0, sd.y0, sd.lx, sd.ly, sd.k, sd.n) for sd in w.subdomains]


def side_structs(w: wl.Workload, m_star: int):
    t = mdp.mdp_cheb_points(m_star)
    sides, ds = [], []
    for i in range(len(w.subdomains)):
        for s in range(4):
            sd = w.sides[i][s]
            st = mdp.Side()
            st.kind = sd.kind
            st.alpha, st.beta = sd.alpha, sd.beta
            st.nbr, st.nbr_side = sd.nbr, sd.nbr_side
            sides.append(st)
            ds.append(mdp.mdp_cheb_coeffs(wl.boundary_samples(w, i, s, t)) if sd.kind == wl.BOUNDARY else None)
    return sides, ds


def build_projectors(ctx, w: wl.Workload, precision, stream=None) -> List[object]:
    out = []
    for s in subdomain_structs(w):
        out.append(mdp.mdp_build_projector(ctx, s, w.m_star, precision, stream))
    return out


def dd_solve(ctx, w: wl.Workload, precision=None, stream=None, projectors=None, sides=None,
             want_cond: bool = True) -> DDResult:
    import torch
    precision = precision or w.precision
    subs = subdomain_structs(w)
    projectors = projectors or build_projectors(ctx, w, precision, stream)
    if sides is None:
        sides = side_structs(w, w.m_star)
    dev = "cuda:%d" % ctx.device
    N = len(subs)
    c = torch.empty(N * 8 * w.m_star, dtype=torch.complex128, device=dev)
    rel, cond = mdp.mdp_solve_interface(ctx, subs, projectors, sides[0], sides[1], w.m_star, c, stream, want_cond)
    offs = [0]
    for sd in w.subdomains:
        offs.append(offs[-1] + (sd.n + 1) ** 2)
    u = torch.empty(offs[-1], dtype=torch.complex128, device=dev)
    mdp.mdp_reconstruct(ctx, projectors, c, u, stream)
    return DDResult(u, c, rel, cond, offs, projectors)
