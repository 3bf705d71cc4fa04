"""Pins of the oracle's derivatives of a receiver functional (oracle/adjoint.py)
against finite differences of the oracle's own forward solve.

* d A / d(k^2): central differences of the assembled AP matrix (interior rows
  are linear in k^2, the end rows smooth in k): agreement to 1e-9.
* d E / d(k^2): E is a polynomial of degree 2 in k^2, so a central difference
  is exact up to rounding.
* d Phi / d(k_i^2) for every subdomain of a 2x2 layout with Dirichlet, Neumann
  and Robin sides: central differences with Richardson extrapolation, 1e-7.
  A dropped end-row derivative, extension derivative or d(A^{-1}) term moves
  these by far more.
* d Phi / d d: u is affine in the boundary data, so central differences are
  exact up to rounding: 1e-9 for Dirichlet, Neumann and Robin sides.
"""
import copy
import math

import numpy as np
import pytest

from oracle import adjoint as adj
from oracle.extension import extension_matrix
from oracle.grid import APGrid
from oracle.scheme import assemble
from paper_2103_12172_amd import workloads as wl


@pytest.fixture(scope="module")
def setup():
    w = wl.config_adjoint_small()
    pts, own = wl.receiver_points(w, 6, 7)
    rcv = adj.snap_receivers(w, pts, own)
    rng = np.random.default_rng(3)
    ubar = rng.standard_normal(len(rcv)) + 1j * rng.standard_normal(len(rcv))
    st = adj.forward(w)
    gk, gd = adj.gradient(w, rcv, ubar, st)
    return w, rcv, ubar, st, gk, gd


def _phi(w, rcv, ubar, d=None):
    s = adj.forward(w, d=d)
    return float(np.real(np.vdot(ubar, adj.receiver_values(s, rcv))))


def test_operator_derivative_matches_differences():
    w = wl.config_adjoint_small()
    sd = w.subdomains[0]
    g = APGrid(sd.x0, sd.y0, sd.lx, sd.ly, sd.n)
    k2 = sd.k ** 2
    dl = 1e-2
    fd = (assemble(sd.n, g.h, math.sqrt(k2 + dl)) - assemble(sd.n, g.h, math.sqrt(k2 - dl))) / (2 * dl)
    dA = adj.assemble_dk2(sd.n, g.h, sd.k)
    assert abs(fd - dA).max() < 1e-9 * abs(dA).max()
    fdE = (extension_matrix(g, math.sqrt(k2 + 1.0), w.m_star) - extension_matrix(g, math.sqrt(k2 - 1.0), w.m_star)) / 2
    dE = adj.extension_dk2(g, sd.k, w.m_star)
    assert abs(fdE - dE).max() < 1e-11 * abs(dE).max()


def test_receivers_on_mplus(setup):
    w, rcv, _, st, _, _ = setup
    for (i, m, q) in rcv:
        assert st["subs"][i].grid.Mplus[m, q]


def test_k2_gradient_matches_differences(setup):
    w, rcv, ubar, _, gk, _ = setup
    for i in range(len(w.subdomains)):
        k2 = w.subdomains[i].k ** 2
        vals = []
        for dl in (1e-4 * k2, 0.5e-4 * k2):
            ph = []
            for sgn in (1, -1):
                ww = copy.deepcopy(w)
                ww.subdomains[i].k = math.sqrt(k2 + sgn * dl)
                ph.append(_phi(ww, rcv, ubar))
            vals.append((ph[0] - ph[1]) / (2 * dl))
        rich = (4 * vals[1] - vals[0]) / 3
        assert abs(rich - gk[i]) < 1e-7 * abs(gk[i]), (i, gk[i], rich)


def test_data_gradient_matches_differences(setup):
    w, rcv, ubar, st, _, gd = setup
    kinds = set()
    for i in range(len(w.subdomains)):
        for s in range(4):
            if gd[i][s] is None:
                continue
            kinds.add((w.sides[i][s].alpha != 0.0, w.sides[i][s].beta != 0.0))
            for j in (0, 2, 4):
                parts = []
                for unit in (1.0, 1j):
                    ph = []
                    for sgn in (1, -1):
                        dd = copy.deepcopy(st["d"])
                        dd[i][s] = dd[i][s].copy()
                        dd[i][s][j] += sgn * 0.1 * unit
                        ph.append(_phi(w, rcv, ubar, dd))
                    parts.append((ph[0] - ph[1]) / 0.2)
                fd = parts[0] + 1j * parts[1]
                assert abs(fd - gd[i][s][j]) < 1e-9 * max(abs(gd[i][s][j]), 1e-3), (i, s, j)
    assert kinds == {(True, False), (False, True), (True, True)}   # Dirichlet, Neumann and Robin sides
