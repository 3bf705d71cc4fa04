"""GPU reverse-mode gradient of a receiver functional of the DD solve
(`mdp_dd_gradient`, `autodiff.ReceiverValues`) against the oracle's
forward-mode derivatives (oracle/adjoint.py, itself pinned by finite
differences) and against finite differences of the GPU forward solve.

Phi = Re sum_r conj(ubar_r) u_r on a 2x2 layout with Dirichlet, Neumann and
Robin sides (n = 24, M* = 5, k^2 in U[100, 400]).  The gradient goes through
(Qbar^* Qbar)^{-1} once without refinement, so its rounding error scales with
cond(Qbar)^2 u: tolerance 1e-12 cond^2 (at least 1e-8), relative to the largest
component.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adjoint as adj
from paper_2103_12172_amd import autodiff, dd, mdp
from paper_2103_12172_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mdp.mdp_create(0)
    yield c
    c.close()


def _problem(ctx, w, n_rcv, seed):
    pts, own = wl.receiver_points(w, n_rcv, seed)
    rs, rn, mq = autodiff.snap_receivers(w, pts, own)
    return autodiff.Problem(ctx, w, rs, rn), mq, pts, own


def _inputs(w):
    k2 = torch.tensor([sd.k ** 2 for sd in w.subdomains], dtype=torch.float64)
    sides, ds = dd.side_structs(w, w.m_star)
    d = np.zeros((len(w.subdomains), 4, w.m_star), dtype=np.complex128)
    for i in range(len(w.subdomains)):
        for s in range(4):
            if ds[4 * i + s] is not None:
                d[i, s] = ds[4 * i + s]
    return k2, torch.tensor(d)


def test_gradient_matches_oracle(ctx):
    w = wl.config_adjoint_small()
    prob, mq, pts, own = _problem(ctx, w, 6, 7)
    assert mq == adj.snap_receivers(w, pts, own)   # both sides pick the same receiver nodes
    rng = np.random.default_rng(3)
    ubar = rng.standard_normal(len(mq)) + 1j * rng.standard_normal(len(mq))
    k2, d = _inputs(w)
    k2.requires_grad_(True)
    d.requires_grad_(True)
    u = autodiff.ReceiverValues.apply(k2, d, prob)
    phi = (torch.conj(torch.as_tensor(ubar, device=u.device)) * u).real.sum()
    phi.backward()
    st = adj.forward(w)
    uref = adj.receiver_values(st, mq)
    gk_ref, gd_ref = adj.gradient(w, mq, ubar, st)
    uerr = float(np.abs(u.detach().cpu().numpy() - uref).max() / np.abs(uref).max())
    gk = k2.grad.numpy()
    kerr = float(np.abs(gk - gk_ref).max() / np.abs(gk_ref).max())
    gd = d.grad.numpy()
    derr, dmax = 0.0, 0.0
    for i in range(len(w.subdomains)):
        for s in range(4):
            if gd_ref[i][s] is None:
                assert np.all(gd[i, s] == 0)
                continue
            derr = max(derr, float(np.abs(gd[i, s] - gd_ref[i][s]).max()))
            dmax = max(dmax, float(np.abs(gd_ref[i][s]).max()))
    derr /= dmax
    cond = np.linalg.cond(st["Qbar"])
    tol = max(1e-8, 1e-12 * cond ** 2)
    print("receivers u err %.3e; grad k^2 rel err %.3e; grad d rel err %.3e; cond %.3e (tol %.1e)"
          % (uerr, kerr, derr, cond, tol))
    assert uerr < 1e-9
    assert kerr < tol and derr < tol


def test_gradient_matches_gpu_differences(ctx):
    """A 3x3 layout at n = 64: central differences of the GPU forward along each k^2 and one
    boundary coefficient."""
    w = wl.config_adjoint(3, 3, 64, (200.0, 900.0), 8, 9, 20.0)
    prob, mq, _, _ = _problem(ctx, w, 12, 11)
    rng = np.random.default_rng(5)
    ubar = torch.as_tensor(rng.standard_normal(len(mq)) + 1j * rng.standard_normal(len(mq)))
    k2, d = _inputs(w)
    k2.requires_grad_(True)
    d.requires_grad_(True)
    u = autodiff.ReceiverValues.apply(k2, d, prob)
    (torch.conj(ubar.to(u.device)) * u).real.sum().backward()

    def phi(kk, dd_):
        with torch.no_grad():
            v = autodiff.ReceiverValues.apply(kk, dd_, prob)
        return float((torch.conj(ubar.to(v.device)) * v).real.sum())

    worst = 0.0
    for i in range(len(w.subdomains)):
        k2i = float(k2.detach()[i])
        vals = []
        for dl in (1e-4 * k2i, 0.5e-4 * k2i):
            e = torch.zeros_like(k2)
            e[i] = dl
            vals.append((phi(k2.detach() + e, d.detach()) - phi(k2.detach() - e, d.detach())) / (2 * dl))
        fd = (4 * vals[1] - vals[0]) / 3
        worst = max(worst, abs(fd - float(k2.grad[i])) / max(abs(fd), 1e-30))
    i, s, j = 0, 0, 2   # a Dirichlet side of the corner subdomain; Phi is affine in d
    e = torch.zeros_like(d)
    e[i, s, j] = 0.1
    fre = (phi(k2.detach(), d.detach() + e) - phi(k2.detach(), d.detach() - e)) / 0.2
    fim = (phi(k2.detach(), d.detach() + 1j * e) - phi(k2.detach(), d.detach() - 1j * e)) / 0.2
    g = complex(d.grad[i, s, j])
    derr = abs(complex(fre, fim) - g) / abs(g)
    print("k^2 gradients vs GPU differences: worst rel err %.3e; data gradient %.3e" % (worst, derr))
    assert worst < 1e-5 and derr < 1e-7
