"""The three algorithm steps of the paper (Sec. 3.5) chained through the C-ABI.

Argument marshalling only: boundary data are sampled from the workload at the
library's Chebyshev points, turned into coefficients by the library, and the
projector build, interface least squares and reconstruction all run in
libmdp on the GPU.  A workload with a source f is sampled on each auxiliary
grid (for B^(h) f) and, with its normal derivatives, at the foot points of
gamma (for Ex^(I) f) that the library reports.
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
    sources: Optional[list] = None   # device (f, jet) per subdomain, kept alive with the result


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
    return (mdp.Side * len(sides))(*sides), ds


def build_projectors(ctx, w: wl.Workload, precision, stream=None) -> List[object]:
    return mdp.mdp_build_projectors(ctx, subdomain_structs(w), w.m_star, precision, stream)


def source_tensors(ctx, w: wl.Workload, projectors) -> Optional[list]:
    """Per subdomain (f on its auxiliary grid, jet of f at the foot points of gamma) as device tensors."""
    import torch
    if w.source is None:
        return None
    dev = "cuda:%d" % ctx.device
    out = []
    for s, P in zip(subdomain_structs(w), projectors):
        xa, ya, h = mdp.mdp_ap_grid(s)
        nodes = np.arange(s.n + 1)
        X, Y = np.meshgrid(xa + nodes * h, ya + nodes * h, indexing="ij")
        f = np.ascontiguousarray(np.asarray(w.source(X, Y), dtype=np.complex128).reshape(-1))
        xy, side = mdp.mdp_projector_gamma_feet(P, s)
        normals = np.array([wl.outward_normal(int(v)) for v in side]).reshape(-1, 2)
        jet = np.concatenate([np.asarray(v, dtype=np.complex128).reshape(-1)
                              for v in w.source_jet(xy[:, 0], xy[:, 1], normals[:, 0], normals[:, 1])])
        out.append((torch.from_numpy(f).to(dev), torch.from_numpy(jet).to(dev)))
    return out


def dd_solve(ctx, w: wl.Workload, precision=None, stream=None, projectors=None, sides=None,
             want_cond: bool = True, sources=None) -> DDResult:
    import torch
    precision = precision or w.precision
    subs = subdomain_structs(w)
    projectors = projectors or build_projectors(ctx, w, precision, stream)
    if sides is None:
        sides = side_structs(w, w.m_star)
    if sources is None and w.source is not None:
        sources = source_tensors(ctx, w, projectors)
    dev = "cuda:%d" % ctx.device
    N = len(subs)
    c = torch.empty(N * 8 * w.m_star, dtype=torch.complex128, device=dev)
    # the grids' layout and buffer before the interface solve, which returns only once its
    # convergence test has reached the host (the reconstruction is queued right after it)
    offs = [0]
    for sd in w.subdomains:
        offs.append(offs[-1] + (sd.n + 1) ** 2)
    u = torch.empty(offs[-1], dtype=torch.complex128, device=dev)
    rel, cond = mdp.mdp_solve_interface(ctx, subs, projectors, sides[0], sides[1], w.m_star, c, stream, want_cond,
                                        sources)
    mdp.mdp_reconstruct(ctx, projectors, c, u, stream, sources)
    return DDResult(u, c, rel, cond, offs, projectors, sources)
