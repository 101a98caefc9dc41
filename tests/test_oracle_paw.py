"""Pins of the oracle's PAW layer: projector integrals in closed form,
brute-force supports, Hermiticity / definiteness, and the Woodbury identity
that the approximate inverse overlap satisfies exactly for one atom.
"""

import numpy as np
import pytest
import scipy.linalg as sla
from scipy import integrate

from oracle.paw import PAWOperator, projector_value
from workloads import make_system
from workloads.configs import custom_system

# int over the unit sphere of S_lm(u)^2 for the unnormalized real solid harmonics
ANG = {(0, 0): 4 * np.pi, (1, -1): 4 * np.pi / 3, (1, 0): 4 * np.pi / 3, (1, 1): 4 * np.pi / 3,
       (2, -2): 4 * np.pi / 15, (2, -1): 4 * np.pi / 15, (2, 0): 16 * np.pi / 5,
       (2, 1): 4 * np.pi / 15, (2, 2): 16 * np.pi / 15}


def _radial(sig, rc):
    return lambda r: np.exp(-r * r / (2 * sig * sig)) * (1 - r * r / (rc * rc)) ** 2


@pytest.fixture(scope="module")
def one_atom():
    # one atom well inside a 3x3x3 mesh of 2-bohr cells, 18 channels, r_c = 2
    s = custom_system((3, 3, 3), (6.0, 6.0, 6.0), 6, 8, pos=[(3.1, 2.9, 3.05)], rcut=2.0,
                      channels="spd18", wells=[(1.0, 2.0, 3.0)], s_H=0.9, s_S=0.45)
    return PAWOperator(s)


@pytest.fixture(scope="module")
def one_atom_fine():
    # same atom on 1-bohr cells: Gauss error of the projector integrals ~1e-6
    s = custom_system((6, 6, 6), (6.0, 6.0, 6.0), 3, 8, pos=[(3.1, 2.9, 3.05)], rcut=2.0,
                      channels="spd18", wells=[(1.0, 2.0, 3.0)], s_H=0.9, s_S=0.45)
    return PAWOperator(s)


@pytest.fixture(scope="module")
def tiny():
    return PAWOperator(make_system("tiny"))


def test_projector_integrals_closed_form(one_atom_fine):
    """C^a^H 1 = int p_alpha (partition of unity), and <p|p> by radial integrals."""
    op = one_atom_fine
    s = op.system
    rc = float(s.rcut[0])
    ch = list(zip(s.proj_l[:18], s.proj_m[:18], s.proj_sigma[:18]))
    ints = np.real(op.CH @ np.ones(op.mesh.M))
    for t, (l, m, sg) in enumerate(ch):
        if l == 0:
            ref = 4 * np.pi * integrate.quad(lambda r: r * r * _radial(sg, rc)(r), 0, rc,
                                             epsabs=1e-14, epsrel=1e-13)[0]
            assert abs(ints[t] - ref) < 1e-5 * ref, (t, ints[t], ref)
        else:                                   # odd / non-spherical: zero by symmetry
            assert abs(ints[t]) < 1e-5 * abs(ints[0])
    G = op.Gpp[0]
    for t, (l, m, sg) in enumerate(ch):
        for u, (l2, m2, sg2) in enumerate(ch):
            if (l, m) != (l2, m2):
                assert abs(G[t, u]) < 1e-5 * np.sqrt(abs(G[t, t] * G[u, u])) + 1e-12
                continue
            g1, g2 = _radial(sg, rc), _radial(sg2, rc)
            ref = ANG[(l, m)] * integrate.quad(lambda r: r ** (2 * l + 2) * g1(r) * g2(r), 0, rc,
                                               epsabs=1e-15, epsrel=1e-13)[0]
            assert abs(G[t, u] - ref) < 1e-5 * ref, (t, u, G[t, u], ref)


def test_exact_g_approaches_projector_overlap(one_atom, one_atom_fine):
    """C^H M_D^{-1} C tends to <p|p> under refinement (the cheaper Delta_Sinv)."""
    e_coarse = np.linalg.norm(one_atom.G[0] - one_atom.Gpp[0]) / np.linalg.norm(one_atom.Gpp[0])
    e_fine = np.linalg.norm(one_atom_fine.G[0] - one_atom_fine.Gpp[0]) \
        / np.linalg.norm(one_atom_fine.Gpp[0])
    assert e_coarse < 0.02 and e_fine < 0.02


def test_support_brute_force(tiny):
    op = tiny
    s = op.system
    pts = op.cq.all_points(op.mesh)                     # (E, nq^3, 3)
    shifts = np.array([(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)]) \
        * op.mesh.box
    for a in range(op.natoms):
        d = pts[:, :, None, :] - s.pos[a] + shifts[None, None, :, :]
        inside = ((d * d).sum(-1) < s.rcut[a] ** 2).any(axis=(1, 2))
        np.testing.assert_array_equal(np.flatnonzero(inside), op.supp_cells[a])
        nodes = np.unique(op.cell_dofs[np.flatnonzero(inside)])
        np.testing.assert_array_equal(nodes, op.supp_nodes[a])
        # C^a vanishes outside the support nodes
        rows = np.unique(op.C[:, op.poff[a]:op.poff[a + 1]].nonzero()[0])
        assert np.all(np.isin(rows, op.supp_nodes[a]))


def test_hermitian_and_spd(tiny):
    H, S = tiny.H_dense(), tiny.S_dense()
    assert np.abs(H - H.T).max() < 1e-13 * np.abs(H).max()
    assert np.abs(S - S.T).max() < 1e-15 * 1e3
    assert np.linalg.eigvalsh(S)[0] > 0
    # the PAW term really changes S (non-local overlap is not negligible)
    Mloc = tiny.loc.assemble_M().toarray()
    assert np.abs(S - Mloc).max() > 1e-3


def test_complex_k_hermitian():
    s = custom_system((2, 3, 2), (4.0, 5.0, 4.0), 3, 5, pos=[(1.0, 2.0, 2.5)], rcut=1.2,
                      wells=[(2.0, 2.0, 2.0)], kpoint=(0.3, -0.2, 0.5), is_complex=True)
    op = PAWOperator(s)
    H, S = op.H_dense(), op.S_dense()
    assert np.iscomplexobj(H) and np.abs(H.imag).max() > 1e-3
    assert np.abs(H - H.conj().T).max() < 1e-13 * np.abs(H).max()
    assert np.abs(S - S.conj().T).max() < 1e-14
    assert np.linalg.eigvalsh(S)[0] > 0


def test_kterm_equals_bloch_shift():
    """Free electrons at k: eigenvalues are those at k=0 of |G + k|^2 / 2, so the
    lowest one is 1/2 |k|^2 to discretization accuracy and the FE k-term is a
    unitary-equivalent shift of the periodic problem."""
    L = 4.0
    k = np.array([0.2, -0.1, 0.15])
    s = custom_system((3, 3, 3), (L, L, L), 5, 7, kpoint=k, is_complex=True)
    op = PAWOperator(s)
    lam = sla.eigh(op.H_dense(), op.S_dense(), eigvals_only=True)
    assert abs(lam[0] - 0.5 * k @ k) < 1e-6
    # the next level is 1/2 |k - G|^2 for the reciprocal vector G closest to k
    Gs = [np.array(v) * 2 * np.pi / L for v in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                                              (0, 0, 1), (0, 0, -1)]]
    nxt = min(0.5 * np.sum((k + G) ** 2) for G in Gs)
    assert abs(lam[1] - nxt) < 1e-4 * nxt


def test_woodbury_one_atom(one_atom):
    """For one atom with G = C^H M_D^{-1} C, Sinv_hat inverts M_D + C Ds C^H exactly."""
    op = one_atom
    rng = np.random.default_rng(3)
    x = rng.standard_normal((op.mesh.M, 3))
    Sx = op.MD[:, None] * x + op.C @ (op.DS @ (op.CH @ x))
    np.testing.assert_allclose(op.apply_Sinv(Sx), x, atol=1e-12 * np.abs(x).max())


def test_sinv_two_atoms_is_approximate(tiny):
    """With shared support nodes, the per-atom Woodbury is only approximate."""
    op = tiny
    shared = np.intersect1d(op.supp_nodes[0], op.supp_nodes[1])
    x = np.random.default_rng(4).standard_normal(op.mesh.M)
    Sx = op.MD * x + op.C @ (op.DS @ (op.CH @ x))
    err = np.linalg.norm(op.apply_Sinv(Sx) - x) / np.linalg.norm(x)
    if len(shared):
        assert 1e-12 < err < 0.5
    else:
        assert err < 1e-12


def test_kterm_is_symmetric_bloch_form():
    """The k-dependent local operator of eq. "PAW Hamiltonian", -1/2 lap - i k.grad + 1/2|k|^2,
    is 1/2 (-i grad + k)^2, whose Galerkin matrix is the symmetric form
    1/2 sum_q W (grad N_I + i k N_I)^* . (grad N_J + i k N_J).  Element by element it
    differs from the oracle's K + 1/2|k|^2 M - i N_I (k.grad N_J) by i/2 k.grad(N_I N_J),
    which integrates to zero over the periodic mesh (the Gauss rule is exact for it),
    so the assembled matrices agree to rounding.  A flipped k-term sign fails this."""
    k = np.array([0.37, -0.21, 0.13])
    s = custom_system((3, 2, 3), (4.5, 3.2, 3.9), 3, 5, kpoint=k, is_complex=True)
    op = PAWOperator(s)
    cq = op.cq
    Z = (cq.dN + 1j * k[:, None, None] * cq.N[None]).astype(np.complex128)   # (3, nq^3, nloc)
    Ae = 0.5 * sum(Z[d].conj().T @ (cq.W[:, None] * Z[d]) for d in range(3))
    sym = op.loc._assemble(lambda e: Ae).toarray()
    ref = op.loc._assemble(lambda e: op.loc.Ke + op.loc.KTe).toarray()
    assert np.abs(ref.imag).max() > 1e-2                 # the k term is really there
    assert np.abs(sym - ref).max() < 1e-12 * np.abs(ref).max()
    # element-wise the two forms differ (only the assembly removes the difference)
    assert np.abs(Ae - (op.loc.Ke + op.loc.KTe)).max() > 1e-3


def _lowest_bloch(L, nc, p, k, nev=8):
    R = (0.45 * L, 0.55 * L, 0.5 * L)
    s = custom_system((nc,) * 3, (L,) * 3, p, p + 2, pos=[R], rcut=1.8, channels="spd8",
                      wells=[R], s_H=2.0, s_S=1.0, kpoint=k, is_complex=True)
    op = PAWOperator(s)
    return sla.eigh(op.H_dense(), op.S_dense(), eigvals_only=True, subset_by_index=[0, nev - 1])


def test_bloch_gauge_k_plus_reciprocal_vector():
    """k and k + G (G a reciprocal lattice vector) describe the same Bloch states
    (u_{k+G} = e^{-iG.x} u_k), so with an atom present the lowest eigenvalues agree up to
    the discretization error, which shrinks under p-refinement.  The k-term of the local
    operator and the phase e^{-ik.x} of C^a (eq. "FEM Cmatrix") must carry consistent
    signs for this: flipping either one leaves a k-dependent mismatch of ~3e-2 Ha here
    that does not shrink (measured on modified copies of the oracle)."""
    L = 5.0
    k = np.array([0.3, -0.2, 0.15])
    G = np.array([2.0 * np.pi / L, 0.0, 0.0])
    diffs = []
    for p in (4, 5):
        diffs.append(np.abs(_lowest_bloch(L, 3, p, k) - _lowest_bloch(L, 3, p, k + G)).max())
    assert diffs[1] < 2e-3, diffs
    assert diffs[1] < 0.2 * diffs[0], diffs
