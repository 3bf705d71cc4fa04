"""The allocation-free AP solve (mdp_ap_solve_noalloc: batch buffers in the library's
static device scratch array) against mdp_ap_solve (context workspaces) through the
C-ABI, on two calls in a row, the second with a smaller batch, in every precision;
and its errors: no plan yet, and a grid whose one right-hand side needs more than
the array holds.  complex128 must agree to 1e-12 relative (the same kernels; only
the chunking of the batch and the GEMM tile shape may differ), refined complex64
to 1e-10 and plain complex64 to 1e-5 (FP32 rounding of the same operations)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2103_12172_amd import mdp
from paper_2103_12172_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64r": 1e-10, "c64": 1e-5}


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mdp.mdp_create(0)
    yield c
    c.close()


def _solve(ctx, fn, g, n, h, k, prec):
    gt = torch.from_numpy(np.ascontiguousarray(g).reshape(-1)).to("cuda:0")
    ut = torch.full_like(gt, complex(float("nan"), float("nan")))   # every output element must be written
    fn(ctx, n, h, k, prec, gt, ut)
    torch.cuda.synchronize()
    return ut.cpu().numpy().reshape(g.shape)


@pytest.mark.parametrize("prec", ["c128", "c64r", "c64"])
def test_noalloc_matches_workspace_solve(ctx, prec):
    n, k = 256, 50.0
    h = 0.55 / n
    empty = torch.empty(0, dtype=torch.complex128, device="cuda:0")
    mdp.mdp_ap_solve(ctx, n, h, k, prec, empty, empty)   # creates the plan
    for batch, seed in ((70, 1), (5, 2)):   # 70 right-hand sides: more than one chunk of the 64 MiB array
        print("case noalloc n=%d prec=%s batch=%d" % (n, prec, batch), flush=True)
        g = wl.random_rhs((batch, n + 1, n + 1), seed=seed)
        ref = _solve(ctx, mdp.mdp_ap_solve, g, n, h, k, prec)
        got = _solve(ctx, mdp.mdp_ap_solve_noalloc, g, n, h, k, prec)
        assert np.all(np.isfinite(got))
        err = float(np.abs(got - ref).max() / np.abs(ref).max())
        print("  no-alloc vs workspace solve: rel diff %.3e" % err)
        assert err < TOL[prec]


def test_noalloc_errors(ctx):
    n, k = 128, 20.0
    h = 0.55 / n
    g = torch.zeros((n + 1) * (n + 1), dtype=torch.complex128, device="cuda:0")
    u = torch.empty_like(g)
    with pytest.raises(mdp.MdpError) as e:   # no plan for (n, h, k) yet
        mdp.mdp_ap_solve_noalloc(ctx, n, h, k + 1.0, "c128", g, u)
    assert e.value.code == mdp.MDP_ERR_ARG
    n2 = 2048
    h2 = 1.1 / n2
    empty = torch.empty(0, dtype=torch.complex128, device="cuda:0")
    mdp.mdp_ap_solve(ctx, n2, h2, k, "c128", empty, empty)
    g2 = torch.zeros((n2 + 1) * (n2 + 1), dtype=torch.complex128, device="cuda:0")
    u2 = torch.empty_like(g2)
    with pytest.raises(mdp.MdpError) as e:   # 32 (n+1) W bytes > 64 MiB
        mdp.mdp_ap_solve_noalloc(ctx, n2, h2, k, "c128", g2, u2)
    assert e.value.code == mdp.MDP_ERR_ARG
    assert "scratch" in str(e.value)
