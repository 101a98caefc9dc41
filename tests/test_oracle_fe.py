"""Pins of the oracle's finite-element layer against textbook facts.

Every check compares the oracle with something it does not compute itself:
closed-form GLL nodes, polynomial exactness of quadrature, brute-force node
coordinates, the tensor-sum structure of the periodic Laplacian, the
continuum free-electron spectrum, and closed-form integrals.
"""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fe
from oracle.paw import PAWOperator
from workloads.configs import custom_system


# -- reference element ------------------------------------------------------

def test_gll_closed_forms():
    x4, _ = fe.gll_nodes_weights(4)
    np.testing.assert_allclose(x4, [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], atol=1e-15)
    x6, _ = fe.gll_nodes_weights(6)
    r = np.sqrt(5 / 3)
    a = np.sqrt(5 / 11 + 2 / 11 * r)
    b = np.sqrt(5 / 11 - 2 / 11 * r)
    np.testing.assert_allclose(x6, [-1, -a, -b, 0, b, a, 1], atol=1e-15)
    _, w2 = fe.gll_nodes_weights(2)          # Simpson
    np.testing.assert_allclose(w2, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)


@pytest.mark.parametrize("p", range(1, 9))
def test_gll_exactness(p):
    x, w = fe.gll_nodes_weights(p)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(0, 2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13, (p, k)
    # degree 2p is NOT integrated exactly (GLL with p+1 points)
    assert abs(np.dot(w, x ** (2 * p)) - 2.0 / (2 * p + 1)) > 1e-6


@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_exactness(n):
    x, w = fe.gauss_nodes_weights(n)
    for k in range(0, 2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13


@pytest.mark.parametrize("p", [2, 4, 6])
def test_lagrange_identities(p):
    xi, _ = fe.gll_nodes_weights(p)
    np.testing.assert_allclose(fe.lagrange_values(xi, xi), np.eye(p + 1), atol=1e-14)
    t = np.linspace(-1, 1, 23)
    L = fe.lagrange_values(xi, t)
    D = fe.lagrange_derivs(xi, t)
    np.testing.assert_allclose(L.sum(1), 1.0, atol=1e-13)
    np.testing.assert_allclose(D.sum(1), 0.0, atol=1e-11)
    np.testing.assert_allclose(L @ xi ** 2, t ** 2, atol=1e-13)
    np.testing.assert_allclose(D @ xi, 1.0, atol=1e-11)
    if p >= 3:                                     # x^3 lies in the space
        np.testing.assert_allclose(D @ xi ** 3, 3 * t ** 2, atol=1e-10)


# -- mesh, DOF map, colouring --------------------------------------------------

@pytest.mark.parametrize("ncell", [(2, 2, 2), (3, 2, 4), (5, 3, 2)])
def test_dofmap_matches_coordinates(ncell):
    box = (3.0, 2.5, 4.0)
    m = fe.Mesh(ncell, box, 3)
    cd = m.cell_dofs()
    X = m.node_coords().reshape(-1, 3)
    Xw = np.mod(X + 1e-9, m.box) - 1e-9                     # wrap into the box
    key = np.round(Xw / (m.h / m.p) * 1e3).astype(np.int64)  # exact grid positions
    key = np.where(np.isclose(Xw, m.box[None, :]), 0, key)
    kk = key[:, 0] + 10 ** 6 * (key[:, 1] + 10 ** 6 * key[:, 2])
    dof = cd.ravel()
    # same DOF <=> same physical point (mod box)
    order = np.argsort(dof, kind="stable")
    for s in np.split(order, np.flatnonzero(np.diff(dof[order])) + 1):
        assert len(set(kk[s])) == 1
    assert len(np.unique(dof)) == m.M == len(np.unique(kk))
    # multiplicity of each DOF = product over axes of (2 if on a cell face else 1)
    a, b, c = m.local_abc()
    mult_loc = np.where((a == 0) | (a == m.p), 2, 1) * np.where((b == 0) | (b == m.p), 2, 1) \
        * np.where((c == 0) | (c == m.p), 2, 1)
    counts = np.bincount(dof, minlength=m.M)
    assert np.all(counts[cd] == mult_loc[None, :])


@pytest.mark.parametrize("ncell", [(2, 2, 2), (4, 4, 4), (3, 5, 2), (5, 5, 5), (7, 2, 3)])
def test_colouring_brute_force(ncell):
    m = fe.Mesh(ncell, (1.0, 1.0, 1.0), 2)
    cd = m.cell_dofs()
    col = m.cell_colour()
    assert col.max() < m.ncolours()
    for c in range(m.ncolours()):
        cells = np.flatnonzero(col == c)
        allnodes = cd[cells].ravel()
        assert len(np.unique(allnodes)) == allnodes.size, f"colour {c} shares nodes"


def test_mesh_rejects_single_cell():
    with pytest.raises(ValueError):
        fe.Mesh((1, 2, 2), (1, 1, 1), 2)


# -- local operators -----------------------------------------------------------

def _free_system(ncell, L, p, nq, veff=None):
    s = custom_system(ncell, (L, L, L), p, nq)
    if veff is not None:
        s = s.with_veff(veff)
    return s


def test_kinetic_nullspace_and_volume():
    s = _free_system((3, 2, 2), 5.0, 4, 6)
    op = PAWOperator(s)
    K = op.loc.assemble_K()
    M = op.loc.assemble_M()
    one = np.ones(op.mesh.M)
    assert np.abs(K @ one).max() < 1e-12
    vol = 125.0
    assert abs(one @ (M @ one) - vol) < 1e-10
    assert abs(op.MD.sum() - vol) < 1e-10
    assert np.all(op.MD > 0)


def test_element_tensor_structure():
    """K^e and M^e equal their 1-D Kronecker forms (catches 3-D index errors)."""
    m = fe.Mesh((2, 2, 2), (2.0, 3.0, 4.0), 3)
    cq = fe.CellQuadrature(m, 5)
    eta, w = fe.gauss_nodes_weights(5)
    L1 = fe.lagrange_values(m.xi, eta)
    D1 = fe.lagrange_derivs(m.xi, eta)
    M1 = L1.T @ (w[:, None] * L1)
    K1 = D1.T @ (w[:, None] * D1)
    hx, hy, hz = m.h
    detJ = hx * hy * hz / 8
    Mk = detJ * np.kron(M1, np.kron(M1, M1))
    Kk = 0.5 * detJ * ((2 / hx) ** 2 * np.kron(M1, np.kron(M1, K1))
                       + (2 / hy) ** 2 * np.kron(M1, np.kron(K1, M1))
                       + (2 / hz) ** 2 * np.kron(K1, np.kron(M1, M1)))
    np.testing.assert_allclose(fe.element_mass(cq), Mk, atol=1e-14)
    np.testing.assert_allclose(fe.element_kinetic(cq), Kk, atol=1e-13)


def _periodic_1d(n, L, p, nq):
    """1-D periodic stiffness/mass (independent 1-D assembly)."""
    xi, _ = fe.gll_nodes_weights(p)
    eta, w = fe.gauss_nodes_weights(nq)
    Lv = fe.lagrange_values(xi, eta)
    Dv = fe.lagrange_derivs(xi, eta)
    h = L / n
    Kloc = (2 / h) * Dv.T @ (w[:, None] * Dv)
    Mloc = (h / 2) * Lv.T @ (w[:, None] * Lv)
    G = n * p
    K = np.zeros((G, G))
    M = np.zeros((G, G))
    for i in range(n):
        idx = (i * p + np.arange(p + 1)) % G
        K[np.ix_(idx, idx)] += Kloc
        M[np.ix_(idx, idx)] += Mloc
    return K, M


def test_free_electron_tensor_sum():
    """V = 0, no atoms: 3-D eigenvalues are sums of 1-D periodic ones."""
    n, L, p, nq = 3, 6.0, 4, 6
    op = PAWOperator(_free_system((n, n, n), L, p, nq))
    lam3 = sla.eigh(op.H_dense(), op.S_dense(), eigvals_only=True)
    K1, M1 = _periodic_1d(n, L, p, nq)
    mu = sla.eigh(K1, M1, eigvals_only=True)
    sums = np.sort((0.5 * (mu[:, None, None] + mu[None, :, None] + mu[None, None, :])).ravel())
    np.testing.assert_allclose(lam3, sums, rtol=1e-10, atol=1e-11)


def test_free_electron_continuum_limit():
    """Lowest modes converge to 1/2 |2 pi n / L|^2 at the spectral rate.

    On a cubic mesh the x, y, z copies of a mode are exactly degenerate; the
    cos/sin pair of each direction splits slightly (the FE space is not
    translation invariant below the cell size) and the split vanishes with h.
    """
    L, p, nq = 6.0, 4, 6
    exact = 0.5 * (2 * np.pi / L) ** 2
    errs = []
    for n in (2, 3, 4):
        op = PAWOperator(_free_system((n, n, n), L, p, nq))
        lam = sla.eigh(op.H_dense(), op.S_dense(), eigvals_only=True, subset_by_index=[0, 26])
        assert abs(lam[0]) < 1e-10                   # constant mode
        np.testing.assert_allclose(lam[1:4], lam[1], rtol=1e-10)   # cubic symmetry
        np.testing.assert_allclose(lam[4:7], lam[4], rtol=1e-10)
        assert lam[7] > 1.9 * exact                  # next shell at ~2x
        errs.append(np.abs(lam[1:7] - exact).max())
        assert np.all(lam[1:7] >= exact - 1e-12)     # variational (conforming FE)
    assert errs[0] > errs[1] > errs[2] > 0
    # rate h^(2p) = h^8: ratio of errors between h = 2 and h = 1.5
    rate = np.log(errs[1] / errs[2]) / np.log(4 / 3)
    assert 2 * p - 1.0 < rate < 2 * p + 1.5, rate
    assert errs[2] / exact < 1e-4


def test_constant_potential_shifts_spectrum():
    n, L, p, nq = 2, 4.0, 3, 5
    s0 = _free_system((n, n, n), L, p, nq)
    v0 = -0.37
    s1 = s0.with_veff(np.full_like(s0.veff_q, v0))
    l0 = sla.eigh(PAWOperator(s0).H_dense(), PAWOperator(s0).S_dense(), eigvals_only=True)
    op1 = PAWOperator(s1)
    l1 = sla.eigh(op1.H_dense(), op1.S_dense(), eigvals_only=True)
    np.testing.assert_allclose(l1, l0 + v0, atol=1e-11)


def test_potential_term_closed_form_integral():
    """1^T V s = int f(x) s(x) dx with f = x-coordinate, s = q(x)q(y)q(z).

    q(t) = u (h - u) / h^2, u = t mod h: continuous, periodic, quadratic per
    cell, so its nodal interpolant is exact for p >= 2 and the Gauss rule
    integrates x * q(x) exactly.  Closed form: (h^2 n^2 / 12) (n h / 6)^2.
    """
    n, L, p, nq = 3, 4.5, 3, 4
    s0 = _free_system((n, n, n), L, p, nq)
    op0 = PAWOperator(s0)
    pts = op0.cq.all_points(op0.mesh)                  # (E, nq^3, 3)
    s1 = s0.with_veff(pts[:, :, 0])
    op1 = PAWOperator(s1)
    h = L / n
    X = op0.mesh.node_coords().reshape(-1, 3)
    dof = op0.cell_dofs.ravel()
    u = np.mod(X, h)
    u = np.where(np.isclose(u, h), 0.0, u)
    qv = (u * (h - u) / h ** 2).prod(axis=1)
    svec = np.zeros(op0.mesh.M)
    svec[dof] = qv
    one = np.ones(op0.mesh.M)
    val = one @ (op1.apply_H(svec) - op0.apply_H(svec))
    exact = (h * h * n * n / 12.0) * (n * h / 6.0) ** 2
    assert abs(val - exact) < 1e-12 * max(1.0, abs(exact))
