"""The C-ABI library without a GPU: it loads, exports every function that
include/mdp.h declares, and its host-only helpers work.  mdp_create reports
MDP_ERR_NODEVICE when no HIP device is visible (nothing is computed here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2103_12172_amd import mdp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mdp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mdp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_three_steps():
    names = _declared()
    for f in ("mdp_build_projector", "mdp_solve_interface", "mdp_reconstruct"):
        assert f in names


def test_library_exports_every_declared_function():
    lib = mdp.load()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(mdp.EXPORTED) == _declared()


def test_host_helpers():
    assert mdp.version().startswith("mdp-gfx950")
    m = 9
    t = mdp.mdp_cheb_points(m)
    assert np.allclose(t, np.cos(np.pi * (np.arange(m) + 0.5) / m))
    # interpolation of a polynomial of degree < M* is exact: phi = T_3 + 2i T_0
    phi = np.cos(3 * np.arccos(t)) + 2j
    d = mdp.mdp_cheb_coeffs(phi)
    ref = np.zeros(m, complex)
    ref[0], ref[3] = 2j, 1.0
    assert np.abs(d - ref).max() < 1e-13


def test_argument_errors_without_device():
    lib = mdp.load()
    assert lib.mdp_cheb_points(0, None) == mdp.MDP_ERR_ARG
    assert lib.mdp_set_projector_path(None, 0) == mdp.MDP_ERR_ARG
    assert lib.mdp_cache_clear(None) == mdp.MDP_ERR_ARG
    assert lib.mdp_set_interface_path(None, 0) == mdp.MDP_ERR_ARG
    assert lib.mdp_set_autotune(None, 1) == mdp.MDP_ERR_ARG
    assert lib.mdp_build_projectors(None, 1, None, 8, 0, None, None) == mdp.MDP_ERR_ARG
    assert lib.mdp_dd_gradient(None, 1, None, None, None, 8, 0, None, None, None, None, None, None) == mdp.MDP_ERR_ARG


def test_create_without_device_fails_loudly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = mdp.load()
    h = ctypes.c_void_p()
    rc = lib.mdp_create(ctypes.byref(h), 0)
    assert rc == mdp.MDP_ERR_NODEVICE
    assert b"device" in lib.mdp_last_error(None)


def test_ap_grid_helper_follows_the_documented_grid():
    """mdp_ap_grid (host): the square of side 1.1 max(lx, ly) centred on the rectangle,
    n cells; odd n is rejected."""
    sub = mdp.Subdomain(0.25, -1.0, 0.5, 2.0, 10.0, 64)
    xa, ya, h = mdp.mdp_ap_grid(sub)
    L = 1.1 * 2.0
    assert abs(h - L / 64) < 1e-15
    assert abs(xa - (0.5 - L / 2)) < 1e-14 and abs(ya - (0.0 - L / 2)) < 1e-14
    with pytest.raises(mdp.MdpError):
        mdp.mdp_ap_grid(mdp.Subdomain(0.0, 0.0, 1.0, 1.0, 10.0, 63))


def test_side_marshalling_array_and_list_agree():
    """make_sides: the one-move copy of a ctypes Side array and the per-side path for a list give
    the same structs, and each boundary side's d pointer addresses its own coefficients."""
    from paper_2103_12172_amd import dd, workloads as wl
    w = wl.config_cross_point(n=128, m_star=16)
    sides, ds = dd.side_structs(w, w.m_star)
    a1, keep1 = mdp.make_sides(sides, ds)
    a2, keep2 = mdp.make_sides([sides[i] for i in range(len(sides))], ds)
    assert ctypes.sizeof(a1) == ctypes.sizeof(a2)
    nb = 0
    for i in range(len(sides)):
        for f in ("kind", "alpha", "beta", "nbr", "nbr_side"):
            assert getattr(a1[i], f) == getattr(a2[i], f) == getattr(sides[i], f)
        if ds[i] is None:
            assert not a1[i].d and not a2[i].d
            continue
        nb += 1
        for a in (a1, a2):
            got = np.array([complex(a[i].d[j].re, a[i].d[j].im) for j in range(w.m_star)])
            assert np.array_equal(got, np.asarray(ds[i], dtype=np.complex128))
    assert nb > 0
    with pytest.raises(ValueError):
        mdp.make_sides(sides, ds[:-1])
