"""The fused support-in / gamma-out projector build (MDP_PATH_AUTO) in both
precisions and every sweep schedule, through the C-ABI.

* Every schedule (1, 2, 4 mode columns per lane) gives the same Q as the
  default one up to the order of the synthesis sums: 1e-12 relative per column
  in complex128, 1e-5 in complex64 (FP32 sums of a few hundred terms).
* The complex64 fused build against the oracle (separable AP solves column by
  column in FP64): the FP32 sweep's rounding, amplified by the AP's
  conditioning, stays below 2e-4 relative per column (the plain complex64
  tolerance of the AP solves is 5e-4); measured values are printed.
* The geometries cover rectangles, wavefronts whose 64-column blocks have
  different parities (n = 96 and 128: W = 128, one block of each parity; n = 320:
  W = 384 with the parity boundary at column 192), and a last wavefront that is
  only partly inside the fold (n = 320 with 4 columns per lane: 256 columns per
  wavefront).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import grid as ogrid, projector as oprojector, scheme
from paper_2103_12172_amd import mdp

pytestmark = pytest.mark.gpu

GEOMS = [(0.0, 0.0, 0.3, 0.7, 25.0, 128, 8), (0.1, 0.2, 0.5, 0.5, 50.0, 256, 32),
         (0.0, 0.0, 1.0, 0.45, 12.0, 96, 12), (0.0, 0.0, 0.5, 0.5, 30.0, 320, 16)]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mdp.mdp_create(0)
    yield c
    mdp.mdp_set_fused_schedule(c, 0)
    mdp.mdp_set_autotune(c, False)
    c.close()


def _q(ctx, sd, m_star, prec, cols_per_lane):
    mdp.mdp_set_fused_schedule(ctx, cols_per_lane)
    mdp.mdp_cache_clear(ctx)
    try:
        P = mdp.mdp_build_projector(ctx, sd, m_star, prec)
        Q = P.q_tensor().cpu().numpy()
        used = mdp.mdp_fused_schedule_used(ctx)
        P.release()
    finally:
        mdp.mdp_set_fused_schedule(ctx, 0)
        mdp.mdp_cache_clear(ctx)
    return Q, used


@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_schedules_agree(ctx, geom, prec):
    x0, y0, lx, ly, k, n, m_star = geom
    print("case schedules n=%d prec=%s" % (n, prec), flush=True)
    sd = mdp.Subdomain(x0, y0, lx, ly, k, n)
    Q0, used0 = _q(ctx, sd, m_star, prec, 0)
    assert used0 in (1, 2)
    tol = 1e-12 if prec == "c128" else 1e-5
    for L in (1, 2, 4):
        QL, used = _q(ctx, sd, m_star, prec, L)
        assert used == L
        err = float((np.linalg.norm(QL - Q0, axis=0) / np.linalg.norm(Q0, axis=0)).max())
        print("  %d columns per lane vs default (%d): max column rel diff %.3e" % (L, used0, err))
        assert err < tol


@pytest.mark.parametrize("geom", GEOMS)
def test_c64_fused_matches_oracle(ctx, geom):
    x0, y0, lx, ly, k, n, m_star = geom
    print("case c64 fused n=%d" % n, flush=True)
    sd = mdp.Subdomain(x0, y0, lx, ly, k, n)
    Q, _ = _q(ctx, sd, m_star, "c64", 0)
    g = ogrid.APGrid(x0, y0, lx, ly, n)
    cols = np.unique(np.array([0, 1, m_star, 3 * m_star - 1, 4 * m_star, 8 * m_star - 1]))
    Qref = oprojector.build_projector(g, k, m_star, scheme.make_solver(n, g.h, k, "separable"), cols=cols)
    err = float((np.linalg.norm(Q[:, cols] - Qref, axis=0) / np.linalg.norm(Qref, axis=0)).max())
    print("  complex64 fused vs oracle: max column rel err %.3e" % err)
    assert err < 2e-4


def test_autotuned_schedule_agrees(ctx):
    x0, y0, lx, ly, k, n, m_star = GEOMS[1]
    sd = mdp.Subdomain(x0, y0, lx, ly, k, n)
    Q0, _ = _q(ctx, sd, m_star, "c128", 0)
    mdp.mdp_set_autotune(ctx, True)
    try:
        for _ in range(2):   # the first build tunes, the second uses the stored choice
            Qt, used = _q(ctx, sd, m_star, "c128", 0)
    finally:
        mdp.mdp_set_autotune(ctx, False)
    err = float((np.linalg.norm(Qt - Q0, axis=0) / np.linalg.norm(Q0, axis=0)).max())
    print("autotuned schedule %d vs default: max column rel diff %.3e" % (used, err))
    assert used in (1, 2, 4)
    assert err < 1e-12
