"""GPU parity at the full sizes of the transmission, adjoint and uneven layouts,
through the C-ABI.

* Transmission (four strips, k = 20 | 200 | 20 | 200, n = 1024, M* = 64): the
  coefficients c and the solution on N+ (a seeded sample of 4096 nodes per strip
  plus every gamma node) against the oracle's solution stored in
  tests/golden/transmission_n1024_ref.npz (written by make_transmission_ref.py,
  which calls only oracle/: separable AP solves per column, its own Householder
  least squares, its reconstruction).  Tolerance 1e-10 * max(1, cond/100) for
  complex128 and 1e-8 * max(1, cond/100) for refined complex64, cond the 2-norm
  condition number of the column-equilibrated reduced matrix as the oracle
  computes it.
* Adjoint layout (4x4 squares, n = 512, k^2 in U[400, 3600], 64 receivers): the
  reverse-mode gradient against central differences of the GPU forward solve
  along four k^2 (Richardson-extrapolated) and three boundary coefficients
  (exact for any step: the receiver values are affine in the data).
* Uneven 16x16 layout: for one subdomain of every n in {128, 256, 384, 512},
  sampled columns of Q against the oracle's column-by-column AP solves.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import grid as ogrid, projector as oprojector, scheme
from paper_2103_12172_amd import autodiff, dd, mdp
from paper_2103_12172_amd import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "transmission_n1024_ref.npz")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mdp.mdp_create(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", ["c128", "c64r"])
def test_transmission_full_size_matches_oracle(ctx, prec):
    ref = np.load(GOLDEN)
    w = wl.config_transmission(n=1024)
    print("case transmission n=1024 prec=%s" % prec, flush=True)
    mdp.mdp_cache_clear(ctx)
    res = dd.dd_solve(ctx, w, prec)
    torch.cuda.synchronize()
    cond = float(ref["cond_equilibrated"])
    c = res.c.cpu().numpy()
    cref = ref["c"]
    cerr = float(np.abs(c - cref).max() / np.abs(cref).max())
    u = res.u.cpu().numpy()
    uerr = 0.0
    for i in range(len(w.subdomains)):
        ui = u[res.offsets[i]:res.offsets[i + 1]][ref["idx%d" % i]]
        uref = ref["u%d" % i]
        uerr = max(uerr, float(np.abs(ui - uref).max() / np.abs(uref).max()))
    base = 1e-10 if prec == "c128" else 1e-8
    tol = base * max(1.0, cond / 100.0)
    print("transmission n=1024 %s: c rel err %.3e, u rel err %.3e (sampled N+), cond %.3e (gpu estimate %.3e), "
          "residual %.3e (oracle %.3e), tol %.1e" % (prec, cerr, uerr, cond, res.cond or 0.0, res.rel_residual,
                                                     float(ref["rel_residual"]), tol))
    mdp.mdp_cache_clear(ctx)
    assert cerr < tol and uerr < tol
    assert abs(res.rel_residual - float(ref["rel_residual"])) < 1e-6 * max(1.0, cond / 100.0)


def test_adjoint_full_size_gradient_vs_differences(ctx):
    w = wl.config_adjoint()
    print("case adjoint 4x4 n=512", flush=True)
    pts, own = wl.receiver_points(w, 64, 5)
    rs, rn, mq = autodiff.snap_receivers(w, pts, own)
    prob = autodiff.Problem(ctx, w, rs, rn)
    rng = np.random.default_rng(13)
    ubar = torch.as_tensor(rng.standard_normal(len(mq)) + 1j * rng.standard_normal(len(mq)))
    k2 = torch.tensor([sd.k ** 2 for sd in w.subdomains], dtype=torch.float64)
    _, ds = dd.side_structs(w, w.m_star)
    d = np.zeros((len(w.subdomains), 4, w.m_star), dtype=np.complex128)
    for i in range(len(w.subdomains)):
        for s in range(4):
            if ds[4 * i + s] is not None:
                d[i, s] = ds[4 * i + s]
    d = torch.tensor(d)
    k2.requires_grad_(True)
    d.requires_grad_(True)
    mdp.mdp_cache_clear(ctx)
    u = autodiff.ReceiverValues.apply(k2, d, prob)
    (torch.conj(ubar.to(u.device)) * u).real.sum().backward()

    def phi(kk, dd_):
        with torch.no_grad():
            v = autodiff.ReceiverValues.apply(kk, dd_, prob)
        return float((torch.conj(ubar.to(v.device)) * v).real.sum())

    k0, d0 = k2.detach(), d.detach()
    worst_k = 0.0
    for i in (0, 5, 10, 15):   # a corner, two interior and the opposite corner subdomain
        k2i = float(k0[i])
        vals = []
        for dl in (1e-4 * k2i, 0.5e-4 * k2i):
            e = torch.zeros_like(k0)
            e[i] = dl
            vals.append((phi(k0 + e, d0) - phi(k0 - e, d0)) / (2 * dl))
        fd = (4 * vals[1] - vals[0]) / 3
        err = abs(fd - float(k2.grad[i])) / max(abs(fd), 1e-30)
        print("  dPhi/dk2[%d]: adjoint %.6e, differences %.6e, rel err %.3e" % (i, float(k2.grad[i]), fd, err))
        worst_k = max(worst_k, err)
    worst_d = 0.0
    for (i, s, j) in ((0, 0, 0), (3, 3, 7), (12, 1, 31)):   # Dirichlet coefficients of outer sides
        assert w.sides[i][s].kind == wl.BOUNDARY
        e = torch.zeros_like(d0)
        e[i, s, j] = 0.1
        fre = (phi(k0, d0 + e) - phi(k0, d0 - e)) / 0.2
        fim = (phi(k0, d0 + 1j * e) - phi(k0, d0 - 1j * e)) / 0.2
        g = complex(d.grad[i, s, j])
        err = abs(complex(fre, fim) - g) / abs(complex(fre, fim))
        print("  dPhi/dd[%d,%d,%d]: adjoint %s, differences %s, rel err %.3e" % (i, s, j, g, complex(fre, fim), err))
        worst_d = max(worst_d, err)
    print("adjoint 4x4 n=512: worst k^2 rel err %.3e, worst data rel err %.3e" % (worst_k, worst_d))
    mdp.mdp_cache_clear(ctx)
    assert worst_k < 1e-6 and worst_d < 1e-8


def test_uneven_full_size_projector_per_n(ctx):
    w = wl.config_uneven()
    cols = np.array([0, 17, 40, 95, 130, 200, 255])
    mdp.mdp_cache_clear(ctx)
    for n in (128, 256, 384, 512):
        i = next(j for j, sd in enumerate(w.subdomains) if sd.n == n)
        sd = w.subdomains[i]
        print("case uneven subdomain %d n=%d k=%.3f" % (i, n, sd.k), flush=True)
        P = mdp.mdp_build_projector(ctx, mdp.Subdomain(sd.x0, sd.y0, sd.lx, sd.ly, sd.k, sd.n), w.m_star, "c128")
        g = ogrid.APGrid(sd.x0, sd.y0, sd.lx, sd.ly, sd.n)
        Qref = oprojector.build_projector(g, sd.k, w.m_star, scheme.make_solver(sd.n, g.h, sd.k, "separable"),
                                          cols=cols)
        ng, mq, _ = P.info()
        assert ng == g.n_gamma and np.array_equal(mq[:, 0], g.gamma_m) and np.array_equal(mq[:, 1], g.gamma_q)
        Q = P.q_tensor().cpu().numpy()[:, cols]
        colerr = np.linalg.norm(Q - Qref, axis=0) / np.linalg.norm(Qref, axis=0)
        print("  max column rel err %.3e" % colerr.max())
        P.release()
        assert colerr.max() < 1e-10
    mdp.mdp_cache_clear(ctx)
