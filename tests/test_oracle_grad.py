"""Pins of the oracle's band-energy gradient.

E = sum_n occ_n x_n^H H x_n is linear in V(q) and in Delta_H, so central
finite differences are exact up to rounding at any step, and the gradient
satisfies Euler-type identities: sum_q V_q dE/dV_q is the potential part of
E, sum_q dE/dV_q is x^H M x, and sum_a <Delta_H^a, dE/dDelta_H^a> is the
non-local part of E.
"""

import numpy as np
import pytest

from oracle import grad
from oracle.paw import PAWOperator
from workloads import make_system


@pytest.fixture(scope="module")
def setup():
    s = make_system("tiny")
    op = PAWOperator(s)
    X = s.trial(5)
    occ = np.array([2.0, 2.0, 1.5, 1.0, 0.25])
    return s, op, X, occ


def test_fd_veff_exact(setup):
    s, op, X, occ = setup
    g = grad.grad_veff(op, X, occ)
    E = abs(grad.band_energy(op, X, occ))
    rng = np.random.default_rng(2)
    for h in (1e-5, 1e-2):
        floor = 50 * np.finfo(float).eps * E / h          # rounding floor of the difference
        idx = rng.choice(g.size, 8, replace=False)
        for i in idx:
            d = np.zeros(g.size)
            d[i] = h
            Ep = grad.band_energy(PAWOperator(s.with_veff(s.veff_q + d.reshape(g.shape))), X, occ)
            Em = grad.band_energy(PAWOperator(s.with_veff(s.veff_q - d.reshape(g.shape))), X, occ)
            fd = (Ep - Em) / (2 * h)
            assert abs(fd - g.ravel()[i]) < floor + 1e-10 * abs(g.ravel()[i])


def test_fd_dH_exact(setup):
    s, op, X, occ = setup
    g = grad.grad_dH(op, X, occ)
    E = abs(grad.band_energy(op, X, occ))
    rng = np.random.default_rng(3)
    for i in rng.choice(g.size, 8, replace=False):
        h = 1e-3
        floor = 50 * np.finfo(float).eps * E / h
        d = np.zeros(g.size)
        d[i] = h
        Ep = grad.band_energy(PAWOperator(s.with_dH(s.dH + d)), X, occ)
        Em = grad.band_energy(PAWOperator(s.with_dH(s.dH - d)), X, occ)
        assert abs((Ep - Em) / (2 * h) - g[i]) < floor + 1e-10 * abs(g[i])


def test_gradient_identities(setup):
    s, op, X, occ = setup
    gV = grad.grad_veff(op, X, occ)
    gD = grad.grad_dH(op, X, occ)
    assert np.all(gV >= 0)                                 # |u|^2 W >= 0
    E = grad.band_energy(op, X, occ)
    op0 = PAWOperator(s.with_veff(np.zeros_like(s.veff_q)))
    E_V = E - grad.band_energy(op0, X, occ)               # potential part
    assert abs(np.sum(s.veff_q * gV) - E_V) < 1e-10 * abs(E)
    MX = op.loc.apply_M(X)
    assert abs(gV.sum() - np.einsum("in,in,n->", X, MX, occ)) < 1e-10 * abs(gV.sum())
    opnl = PAWOperator(s.with_dH(np.zeros_like(s.dH)))
    E_nl = E - grad.band_energy(opnl, X, occ)
    assert abs(np.dot(s.dH, gD) - E_nl) < 1e-10 * abs(E)


def test_grad_veff_cell_subset(setup):
    """The per-cell form used on sampled cells of large meshes equals the rows
    of the full gradient."""
    s, op, X, occ = setup
    full = grad.grad_veff(op, X, occ)
    cells = [0, 7, 33, 63]
    np.testing.assert_array_equal(grad.grad_veff(op, X, occ, cells=cells), full[cells])
