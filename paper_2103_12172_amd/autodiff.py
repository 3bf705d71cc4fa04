"""The DD solve's values at receivers as a differentiable torch function.

`ReceiverValues.apply(k2, d, problem)` runs the three steps of Sec. 3.5 through
the C-ABI (projectors for k = sqrt(k2), the interface least squares, the
reconstruction) and returns u at the receivers; its backward calls
`mdp_dd_gradient`, the library's reverse pass, which solves the interface
system again instead of keeping anything from the forward call.  Argument
marshalling only: every step runs in libmdp.

  k2  real float64 tensor [n_sub], the subdomains' k^2;
  d   complex128 tensor [n_sub, 4, M*], the Chebyshev coefficients of the
      boundary data of each side (entries of interface sides are ignored and
      get zero gradient).
Torch's convention for a real loss L of complex u: u.grad = dL/d(Re u) +
i dL/d(Im u); the library's functional Phi = Re sum conj(ubar) u with
ubar = u.grad then has dPhi/dk2 = dL/dk2 and dPhi/dd = d.grad.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence, Tuple

import numpy as np
import torch

from . import mdp
from . import workloads as wl


@dataclass
class Problem:
    ctx: object
    w: wl.Workload               # layout: rectangles, n, side kinds and (alpha, beta); its k and data are replaced
    rcv_sub: np.ndarray          # receiver subdomain
    rcv_node: np.ndarray         # receiver node m*(n+1)+q of that subdomain's auxiliary grid
    stream: object = None


def snap_receivers(w: wl.Workload, points, owners) -> Tuple[np.ndarray, np.ndarray, List[Tuple[int, int, int]]]:
    """Nearest M+ node (node of the auxiliary grid strictly inside the open rectangle) of each
    point's subdomain, with the grid origin and step the library reports."""
    subs, nodes, mq = [], [], []
    for (x, y), i in zip(points, owners):
        sd = w.subdomains[i]
        xa, ya, h = mdp.mdp_ap_grid(mdp.Subdomain(sd.x0, sd.y0, sd.lx, sd.ly, sd.k, sd.n))
        def axis(v, a0, lo, hi):
            first = math.floor((lo - a0) / h) + 1
            last = math.ceil((hi - a0) / h) - 1
            return int(min(max(round((v - a0) / h), first), last))
        m = axis(x, xa, sd.x0, sd.x0 + sd.lx)
        q = axis(y, ya, sd.y0, sd.y0 + sd.ly)
        subs.append(int(i))
        nodes.append(m * (sd.n + 1) + q)
        mq.append((int(i), m, q))
    return np.asarray(subs, dtype=np.int32), np.asarray(nodes, dtype=np.int32), mq


def _structs(problem: Problem, k2: np.ndarray, d: np.ndarray):
    w = problem.w
    subs = [mdp.Subdomain(sd.x0, sd.y0, sd.lx, sd.ly, float(math.sqrt(k2[i])), sd.n)
            for i, sd in enumerate(w.subdomains)]
    sides, ds = [], []
    for i in range(len(w.subdomains)):
        for s in range(4):
            sd = w.sides[i][s]
            st = mdp.Side()
            st.kind = sd.kind
            st.alpha, st.beta = sd.alpha, sd.beta
            st.nbr, st.nbr_side = sd.nbr, sd.nbr_side
            sides.append(st)
            ds.append(np.ascontiguousarray(d[i, s]) if sd.kind == wl.BOUNDARY else None)
    return subs, sides, ds


class ReceiverValues(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k2, d, problem: Problem):
        k2h = k2.detach().cpu().numpy().astype(np.float64)
        dh = d.detach().cpu().numpy().astype(np.complex128)
        subs, sides, ds = _structs(problem, k2h, dh)
        c_ = problem.ctx
        M = problem.w.m_star
        projectors = mdp.mdp_build_projectors(c_, subs, M, "c128", problem.stream)
        dev = "cuda:%d" % c_.device
        c = torch.empty(len(subs) * 8 * M, dtype=torch.complex128, device=dev)
        mdp.mdp_solve_interface(c_, subs, projectors, sides, ds, M, c, problem.stream, want_cond=False)
        offs = np.concatenate([[0], np.cumsum([(s.n + 1) ** 2 for s in subs])])
        u = torch.empty(int(offs[-1]), dtype=torch.complex128, device=dev)
        mdp.mdp_reconstruct(c_, projectors, c, u, problem.stream)
        idx = torch.as_tensor(offs[problem.rcv_sub] + problem.rcv_node, dtype=torch.long, device=dev)
        ctx.problem = problem
        ctx.saved = (k2h, dh)
        ctx.devices = (k2.device, d.device)
        return u[idx]

    @staticmethod
    def backward(ctx, grad_u):
        problem = ctx.problem
        k2h, dh = ctx.saved
        subs, sides, ds = _structs(problem, k2h, dh)
        M = problem.w.m_star
        projectors = mdp.mdp_build_projectors(problem.ctx, subs, M, "c128", problem.stream)   # cached
        ubar = grad_u.detach().to(torch.complex128).cpu().numpy()
        gk, gd = mdp.mdp_dd_gradient(problem.ctx, subs, projectors, sides, ds, M, problem.rcv_sub, problem.rcv_node,
                                     ubar, problem.stream)
        dk, dd = ctx.devices
        return (torch.as_tensor(gk, dtype=torch.float64).to(dk), torch.as_tensor(gd, dtype=torch.complex128).to(dd),
                None)
