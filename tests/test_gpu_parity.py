"""GPU parity of the HIP path (through the C-ABI) against the CPU oracle.

Tolerances (relative, max-norm over the compared array unless stated):
  * complex128 AP solves and projector columns: 1e-10;
  * complex64 + one FP64-residual refinement: 1e-8 (AP solves), 1e-8 (Q);
  * plain complex64: 5e-4 (FP32 rounding amplified by the AP's conditioning);
  * interface coefficients c: 1e-10 * max(1, cond/100) in FP64 form, with cond
    the condition estimate the library reports for the equilibrated system.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import grid as ogrid, interface as ointerface, projector as oprojector, scheme, solve as osolve
from paper_2103_12172_amd import dd, mdp
from paper_2103_12172_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-10, "c64r": 1e-8, "c64": 5e-4}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mdp.mdp_create(0)
    yield c
    c.close()


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _ap_gpu(ctx, g, n, h, k, prec):
    gt = torch.from_numpy(np.ascontiguousarray(g).reshape(-1)).to("cuda:0")
    ut = torch.empty_like(gt)
    mdp.mdp_ap_solve(ctx, n, h, k, prec, gt, ut)
    torch.cuda.synchronize()
    return ut.cpu().numpy().reshape(g.shape)


@pytest.mark.parametrize("n,k,L", [(64, 10.0, 1.1), (96, 31.0, 0.55), (256, 50.0, 0.55)])
@pytest.mark.parametrize("prec", ["c128", "c64r", "c64"])
def test_ap_solve_matches_oracle(ctx, n, k, L, prec):
    h = L / n
    print("case ap_solve n=%d k=%g prec=%s" % (n, k, prec), flush=True)
    g = wl.random_rhs((3, n + 1, n + 1), seed=n + int(k))
    ref = (scheme.BandedAP if n <= 128 else scheme.SeparableAP)(n, h, k).solve(g)
    u = _ap_gpu(ctx, g, n, h, k, prec)
    err = rel(u, ref)
    print("  rel err %.3e" % err)
    assert err < TOL[prec]
    # boundary values of the solution are exactly zero (Dirichlet ends)
    assert np.all(u[:, :, 0] == 0) and np.all(u[:, :, n] == 0)


def test_ap_solve_batch_ragged_and_empty(ctx):
    n, k, h = 64, 7.0, 1.1 / 64
    g = wl.random_rhs((5, n + 1, n + 1), seed=3)
    ref = scheme.BandedAP(n, h, k).solve(g)
    assert rel(_ap_gpu(ctx, g, n, h, k, "c128"), ref) < 1e-10
    empty = torch.empty(0, dtype=torch.complex128, device="cuda:0")
    mdp.mdp_ap_solve(ctx, n, h, k, "c128", empty, empty)


def _q_oracle(w, i, m_star, cols=None, kind="auto"):
    sd = w.subdomains[i]
    g = ogrid.APGrid(sd.x0, sd.y0, sd.lx, sd.ly, sd.n)
    solver = scheme.make_solver(sd.n, g.h, sd.k, kind)
    return g, oprojector.build_projector(g, sd.k, m_star, solver, cols=cols)


def _check_gamma(P, g):
    ng, mq, _ = P.info()
    assert ng == g.n_gamma
    assert np.array_equal(mq[:, 0], g.gamma_m) and np.array_equal(mq[:, 1], g.gamma_q)


@pytest.mark.parametrize("prec", ["c128", "c64r"])
def test_projector_two_rect_matches_oracle(ctx, prec):
    w = wl.config_two_rect(n=64)
    sd = w.subdomains[0]
    P = mdp.mdp_build_projector(ctx, mdp.Subdomain(sd.x0, sd.y0, sd.lx, sd.ly, sd.k, sd.n), w.m_star, prec)
    g, Qref = _q_oracle(w, 0, w.m_star)
    _check_gamma(P, g)
    Q = P.q_tensor().cpu().numpy()
    colerr = np.linalg.norm(Q - Qref, axis=0) / np.linalg.norm(Qref, axis=0)
    print("projector two_rect %s: max column rel err %.3e" % (prec, colerr.max()))
    assert colerr.max() < TOL[prec]


@pytest.mark.parametrize("prec", ["c128", "c64r"])
def test_projector_cross_point_matches_oracle(ctx, prec):
    w = wl.config_cross_point(n=256)
    sd = w.subdomains[0]
    P = mdp.mdp_build_projector(ctx, mdp.Subdomain(sd.x0, sd.y0, sd.lx, sd.ly, sd.k, sd.n), w.m_star, prec)
    cols = np.array([0, 5, 31, 32, 77, 128, 160, 255])
    g, Qref = _q_oracle(w, 0, w.m_star, cols=cols, kind="separable")
    _check_gamma(P, g)
    Q = P.q_tensor().cpu().numpy()[:, cols]
    colerr = np.linalg.norm(Q - Qref, axis=0) / np.linalg.norm(Qref, axis=0)
    print("projector cross_point %s: max column rel err %.3e" % (prec, colerr.max()))
    assert colerr.max() < TOL[prec]


@pytest.mark.parametrize("geom", [(0.0, 0.0, 0.3, 0.7, 25.0, 128, 8), (0.1, 0.2, 0.5, 0.5, 50.0, 256, 32),
                                  (0.0, 0.0, 1.0, 0.45, 12.0, 96, 12)])
def test_projector_fused_route_matches_dense_and_oracle(ctx, geom):
    """The support-in / gamma-out route (default for complex128) against the
    dense route (full AP solve per column) and against oracle columns."""
    x0, y0, lx, ly, k, n, m_star = geom
    sd = mdp.Subdomain(x0, y0, lx, ly, k, n)
    mdp.mdp_cache_clear(ctx)
    P = mdp.mdp_build_projector(ctx, sd, m_star, "c128")
    Qf = P.q_tensor().cpu().numpy()
    mdp.mdp_set_projector_path(ctx, "dense")
    mdp.mdp_cache_clear(ctx)
    try:
        Pd = mdp.mdp_build_projector(ctx, sd, m_star, "c128")
        Qd = Pd.q_tensor().cpu().numpy()
    finally:
        mdp.mdp_set_projector_path(ctx, "auto")
        mdp.mdp_cache_clear(ctx)
    g = ogrid.APGrid(x0, y0, lx, ly, n)
    _check_gamma(P, g)
    cols = np.unique(np.array([0, 1, m_star, 3 * m_star - 1, 4 * m_star, 8 * m_star - 1]))
    solver = scheme.make_solver(n, g.h, k, "separable" if n > 128 else "auto")
    Qref = oprojector.build_projector(g, k, m_star, solver, cols=cols)
    e_dense = np.linalg.norm(Qf - Qd, axis=0) / np.linalg.norm(Qd, axis=0)
    e_orc = np.linalg.norm(Qf[:, cols] - Qref, axis=0) / np.linalg.norm(Qref, axis=0)
    print("fused vs dense %.3e, fused vs oracle %.3e" % (e_dense.max(), e_orc.max()))
    assert e_dense.max() < 1e-10 and e_orc.max() < 1e-10


def test_projector_cache_and_release(ctx):
    sd = mdp.Subdomain(0.0, 0.0, 0.5, 1.0, 10.0, 64)
    P1 = mdp.mdp_build_projector(ctx, sd, 16, "c128")
    sd2 = mdp.Subdomain(0.5, 0.0, 0.5, 1.0, 10.0, 64)   # translated copy: same Q
    P2 = mdp.mdp_build_projector(ctx, sd2, 16, "c128")
    assert P1.handle.value == P2.handle.value
    P1.release()
    P2.release()


def _dd_compare(ctx, w, prec, tol_scale=1.0):
    res = dd.dd_solve(ctx, w, prec)
    torch.cuda.synchronize()
    ores = osolve.dd_solve(w)
    c = res.c.cpu().numpy()
    cref = np.concatenate(ores["c"])
    cond = res.cond or 1.0
    cerr = rel(c, cref)
    u = res.u.cpu().numpy()
    uerr, exact_err_gpu = 0.0, 0.0
    for i, sd in enumerate(w.subdomains):
        ui = u[res.offsets[i]:res.offsets[i + 1]].reshape(sd.n + 1, sd.n + 1)
        g = ores["grids"][i]
        uref = ores["u"][i]
        uerr = max(uerr, float(np.abs(ui - uref)[g.Nplus].max() / np.abs(uref[g.Nplus]).max()))
        X, Y = np.meshgrid(g.xs, g.ys, indexing="ij")
        exact_err_gpu = max(exact_err_gpu, float(np.abs(ui - w.exact(X, Y))[g.Mplus].max()))
    print("%s %s: c rel err %.3e, u rel err %.3e, cond %.3e, residual %.3e, error vs exact gpu %.3e oracle %.3e"
          % (w.name, prec, cerr, uerr, cond, res.rel_residual, exact_err_gpu, ores["info"]["error_max_Mplus"]))
    return cerr, uerr, cond, exact_err_gpu, ores["info"]["error_max_Mplus"]


def test_dd_two_rect_c128(ctx):
    w = wl.config_two_rect(n=64)
    cerr, uerr, cond, e_gpu, e_ref = _dd_compare(ctx, w, "c128")
    tol = 1e-10 * max(1.0, cond / 100.0)
    assert cerr < tol and uerr < tol
    assert abs(e_gpu - e_ref) <= 1e-3 * e_ref


@pytest.mark.parametrize("prec", ["c128", "c64r"])
def test_dd_cross_point(ctx, prec):
    w = wl.config_cross_point(n=256)
    cerr, uerr, cond, e_gpu, e_ref = _dd_compare(ctx, w, prec)
    tol = (1e-10 if prec == "c128" else 1e-8) * max(1.0, cond / 100.0)
    assert cerr < tol and uerr < tol
    assert e_gpu < 2 * e_ref


def test_projector_transmission_full_size(ctx):
    """Projector of a k = 200 strip at the full size of the transmission workload
    (n = 1024, M* = 64: 512 columns in one launch), sampled columns vs the oracle."""
    w = wl.config_transmission(n=1024)
    sd = w.subdomains[1]
    P = mdp.mdp_build_projector(ctx, mdp.Subdomain(sd.x0, sd.y0, sd.lx, sd.ly, sd.k, sd.n), w.m_star, "c128")
    cols = np.array([0, 63, 64, 200, 300, 511])
    g, Qref = _q_oracle(w, 1, w.m_star, cols=cols, kind="separable")
    _check_gamma(P, g)
    Q = P.q_tensor().cpu().numpy()[:, cols]
    colerr = np.linalg.norm(Q - Qref, axis=0) / np.linalg.norm(Qref, axis=0)
    print("projector transmission n=1024 k=200: max column rel err %.3e" % colerr.max())
    assert colerr.max() < 1e-10


def test_dd_transmission_reduced_matches_oracle(ctx):
    """Four strips with a 4x wavenumber jump at a size the oracle finishes in
    seconds (n = 256, k = 10 | 40, M* = 32)."""
    w = wl.config_transmission(n=256, ks=(10.0, 40.0, 10.0, 40.0), m_star=32)
    cerr, uerr, cond, e_gpu, e_ref = _dd_compare(ctx, w, "c128")
    tol = 1e-10 * max(1.0, cond / 100.0)
    assert cerr < tol and uerr < tol
    assert abs(e_gpu - e_ref) <= 1e-3 * e_ref


def test_dd_transmission_full_size_fourth_order(ctx):
    """The transmission workload (k = 20 | 200, M* = 64) at n = 512 and at its full
    size n = 1024: the error vs the exact piecewise plane wave on M+ falls by ~16
    per halving (4th order) and the interface residual stays small."""
    errs = []
    for n in (512, 1024):
        w = wl.config_transmission(n=n)
        res = dd.dd_solve(ctx, w, "c128")
        torch.cuda.synchronize()
        u = res.u.cpu().numpy()
        err = 0.0
        for i, sd in enumerate(w.subdomains):
            g = ogrid.APGrid(sd.x0, sd.y0, sd.lx, sd.ly, sd.n)
            ui = u[res.offsets[i]:res.offsets[i + 1]].reshape(sd.n + 1, sd.n + 1)
            X, Y = np.meshgrid(g.xs, g.ys, indexing="ij")
            err = max(err, float(np.abs(ui - w.exact(X, Y))[g.Mplus].max()))
        print("transmission n=%d: error vs exact %.3e, cond %.3e, residual %.3e" % (n, err, res.cond, res.rel_residual))
        assert res.rel_residual < 1e-5
        errs.append(err)
        mdp.mdp_cache_clear(ctx)
    assert 12.0 < errs[0] / errs[1] < 20.0
    assert errs[1] < 2e-3


def test_interface_least_squares_on_gpu_projectors(ctx):
    """The device assembly + least squares against the oracle's elimination and
    Householder QR applied to the same (GPU-built) Q matrices."""
    w = wl.config_cross_point(n=128, m_star=16)
    projs = dd.build_projectors(ctx, w, "c128")
    sides, ds = dd.side_structs(w, w.m_star)
    c = torch.empty(len(w.subdomains) * 8 * w.m_star, dtype=torch.complex128, device="cuda:0")
    subs = dd.subdomain_structs(w)
    relres, cond = mdp.mdp_solve_interface(ctx, subs, projs, sides, ds, w.m_star, c)
    Qs = [p.q_tensor().cpu().numpy() for p in projs]
    d = [[ds[4 * i + s] for s in range(4)] for i in range(len(w.subdomains))]
    cref, _, info, _ = ointerface.solve_interface(Qs, w.sides, d, w.m_star)
    err = rel(c.cpu().numpy(), np.concatenate(cref))
    print("interface LS: rel err %.3e cond %.3e residual gpu %.3e oracle %.3e" % (err, cond, relres, info["rel_residual"]))
    assert err < 1e-10 * max(1.0, cond / 100.0)
    assert abs(relres - info["rel_residual"]) <= 1e-6 * max(info["rel_residual"], 1e-12) + 1e-13


def test_error_paths(ctx):
    with pytest.raises(mdp.MdpError) as e:
        mdp.mdp_build_projector(ctx, mdp.Subdomain(0, 0, 1, 1, 10.0, 63), 8, "c128")
    assert e.value.code == mdp.MDP_ERR_ARG
    with pytest.raises(mdp.MdpError) as e:
        mdp.mdp_build_projector(ctx, mdp.Subdomain(0, 0, 1, 1, float("nan"), 64), 8, "c128")
    assert e.value.code == mdp.MDP_ERR_NONFINITE
    with pytest.raises(mdp.MdpError) as e:
        mdp.mdp_build_projector(ctx, mdp.Subdomain(0, 0, 1, 1, 10.0, 64), 0, "c128")
    assert e.value.code == mdp.MDP_ERR_ARG
    with pytest.raises(mdp.MdpError) as e:
        mdp.mdp_build_projector(ctx, mdp.Subdomain(0, 0, 1, 1, 10.0, 64), 4, 7)
    assert e.value.code == mdp.MDP_ERR_ARG
    with pytest.raises(mdp.MdpError) as e:   # gamma would touch the auxiliary boundary
        mdp.mdp_build_projector(ctx, mdp.Subdomain(0, 0, 1, 1, 10.0, 8), 4, "c128")
    assert e.value.code == mdp.MDP_ERR_ARG


def test_dd_ill_conditioned_falls_back_to_cholesky_qr(ctx):
    """The paper's base case with M* = 40 on the coarsest grid has cond ~1e8 after
    column equilibration: the semi-normal path must hand over to the Cholesky-QR
    passes, which still reproduce the oracle's (Householder) accuracy vs the exact
    solution and its residual."""
    w = wl.config_paper_base(n=64)
    res = dd.dd_solve(ctx, w, "c128")
    torch.cuda.synchronize()
    ores = osolve.dd_solve(w)
    sd = w.subdomains[0]
    g = ores["grids"][0]
    u = res.u.cpu().numpy().reshape(sd.n + 1, sd.n + 1)
    X, Y = np.meshgrid(g.xs, g.ys, indexing="ij")
    e_gpu = float(np.abs(u - w.exact(X, Y))[g.Mplus].max())
    e_ref = ores["info"]["error_max_Mplus"]
    print("paper base n=64: cond %.3e, error vs exact gpu %.4e oracle %.4e, residual gpu %.3e oracle %.3e"
          % (res.cond, e_gpu, e_ref, res.rel_residual, ores["info"]["rel_residual"]))
    assert res.cond > 1e6
    assert abs(e_gpu - e_ref) < 0.02 * e_ref
    assert res.rel_residual < 1.05 * ores["info"]["rel_residual"] + 1e-14
