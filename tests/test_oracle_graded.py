"""Pins of the oracle on graded (two-level) meshes and of the GGA term of
eq. "FEM Ham entries" (FE discretization section; figure "Finite-element
meshes employed in PAW-FE").

Each pin is fixed by mathematics rather than by the oracle itself:
  - the volume (1^T M 1 and the sum of M_D) on any mesh;
  - the kinetic energy of a cosine mode along each axis (a closed form, to
    the discretization error);
  - the GGA matrix of a constant field vanishes after periodic assembly
    (integration by parts, exact under the Gauss rule);
  - for a continuous periodic field that is linear inside each cell, the
    assembled GGA matrix equals minus the potential matrix of its divergence
    exactly (both integrands are polynomials the Gauss rule integrates);
  - the projector integrals 1^T C^a against an independent tensor Gauss
    quadrature of the projector;
  - the lowest generalized eigenvalues on a graded mesh against a finer
    uniform mesh (discretization error);
  - dE/dV on a graded mesh by exact differences (E is linear in V);
  - a graded mesh whose boundaries are the uniform ones reproduces the
    uniform operator.
"""

import dataclasses

import numpy as np
import pytest

from oracle import grad
from oracle.fe import CellQuadrature, LocalOperator, Mesh, element_potential, lumped_mass
from oracle.paw import PAWOperator, projector_value
from workloads.configs import custom_system, make_system, two_level_grid, with_two_level_gga


def _graded_mesh(p=3):
    xg = (np.array([0.0, 1.0, 3.0, 4.0, 6.5]), np.array([0.0, 2.0, 3.0, 5.0]), np.array([0.0, 1.5, 2.5, 5.0]))
    return Mesh((4, 3, 3), (6.5, 5.0, 5.0), p, xgrid=xg)


def test_two_level_grid_shape():
    s = make_system("tiny")
    xg = two_level_grid(s.ncell, s.box, s.pos, 1.5)
    for d in range(3):
        b = xg[d]
        assert b[0] == 0.0 and b[-1] == s.box[d] and len(b) == s.ncell[d] + 1
        h = np.diff(b)
        assert np.all(h > 0)
        ratios = set(np.round(h / h.min(), 12))
        assert ratios <= {1.0, 2.0}


@pytest.mark.parametrize("p", [2, 4])
def test_graded_volume(p):
    m = _graded_mesh(p)
    vol = float(np.prod(m.box))
    loc = LocalOperator(m, p + 2, np.zeros((m.E, (p + 2) ** 3)))
    one = np.ones(m.M)
    assert abs(one @ loc.apply_M(one) - vol) < 1e-12 * vol
    assert abs(lumped_mass(m).sum() - vol) < 1e-12 * vol


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_graded_kinetic_cosine(axis):
    """u = cos(2 pi x_d / L_d): 1/2 int |grad u|^2 = (2 pi / L_d)^2 V / 4."""
    m = _graded_mesh(5)
    loc = LocalOperator(m, 7, np.zeros((m.E, 7 ** 3)))
    X = np.zeros((m.M, 3))
    for e, cd in enumerate(m.cell_dofs()):
        X[cd] = m.node_coords()[e]
    u = np.cos(2 * np.pi * X[:, axis] / m.box[axis])
    K = loc.assemble_K()
    got = u @ (K @ u)
    want = (2 * np.pi / m.box[axis]) ** 2 * np.prod(m.box) / 4.0
    assert abs(got - want) < 2e-3 * want
    # and its L2 norm: int u^2 = V / 2
    assert np.isclose(u @ (loc.assemble_M() @ u), np.prod(m.box) / 2.0, rtol=2e-3)


@pytest.mark.parametrize("graded", [False, True])
def test_gga_constant_field_assembles_to_zero(graded):
    m = _graded_mesh(3) if graded else Mesh((3, 3, 4), (5.0, 5.0, 6.0), 3)
    nq3 = 5 ** 3
    vg = np.zeros((m.E, 3, nq3))
    vg[:, 0], vg[:, 1], vg[:, 2] = 0.7, -0.3, 1.1
    loc = LocalOperator(m, 5, np.zeros((m.E, nq3)), vgga_q=vg)
    G = loc.assemble_GGA()
    scale = max(abs(loc.cell_H(e)).max() for e in range(m.E))
    assert abs(G).max() < 1e-12 * scale
    # a single cell's contribution is not zero (the cancellation is global)
    from oracle.fe import element_gga
    assert abs(element_gga(loc.cell_cq(0), vg[0])).max() > 1e-2


@pytest.mark.parametrize("p", [2, 3, 5])
def test_gga_piecewise_linear_field_equals_minus_divergence(p):
    """V_d depends on x_d only, continuous, periodic and linear in each cell:
    sum_e int V . grad(N_I N_J) = - sum_e int (div V) N_I N_J exactly."""
    m = _graded_mesh(p)
    nq = p + 2
    rng = np.random.default_rng(11)
    knots = [np.append(v, v[0]) for v in (rng.standard_normal(n) for n in m.ncell)]
    cq0 = CellQuadrature(m, nq)
    eta = cq0.eta
    q = np.arange(nq ** 3)
    qi = (q % nq, (q // nq) % nq, q // (nq * nq))
    vg = np.zeros((m.E, 3, nq ** 3))
    div = np.zeros((m.E, nq ** 3))
    for e in range(m.E):
        ijk = m.cell_ijk(e)
        h = m.cell_h(e)
        for d in range(3):
            v0, v1 = knots[d][ijk[d]], knots[d][ijk[d] + 1]
            t = 0.5 * (eta[qi[d]] + 1.0)
            vg[e, d] = v0 + (v1 - v0) * t
            div[e] += (v1 - v0) / h[d]
    loc = LocalOperator(m, nq, np.zeros((m.E, nq ** 3)), vgga_q=vg)
    G = loc.assemble_GGA().toarray()
    Md = loc._assemble(lambda e: element_potential(loc.cell_cq(e), div[e])).toarray()
    assert np.abs(G + Md).max() < 1e-12 * np.abs(Md).max()
    assert np.abs(G - G.T).max() < 1e-13 * np.abs(G).max()


def test_graded_projector_integrals():
    """1^T C^a = int p_alpha (the FE basis sums to one) against a tensor
    Gauss rule of 48 points per axis over the cut-off box."""
    s = custom_system((4, 3, 3), (6.5, 5.0, 5.0), 4, 6, pos=[(3.1, 2.4, 2.6)], rcut=1.5, channels="spd8",
                      wells=[(1.0, 1.0, 1.0)])
    s = dataclasses.replace(s, xgrid=_graded_mesh(4).bounds)
    op = PAWOperator(s)
    got = np.asarray(op.C.sum(axis=0)).ravel()
    x, w = np.polynomial.legendre.leggauss(48)
    R, rc = s.pos[0], float(s.rcut[0])
    # split each axis at the atom so the kink of the cut-off stays at interval ends
    pts, wts = [], []
    for lo, hi in ((-rc, 0.0), (0.0, rc)):
        pts.append(lo + (x + 1) * 0.5 * (hi - lo))
        wts.append(w * 0.5 * (hi - lo))
    t, tw = np.concatenate(pts), np.concatenate(wts)
    D = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
    W = np.einsum("i,j,k->ijk", tw, tw, tw).ravel()
    want = []
    for c in range(int(s.nproj[0])):
        want.append(W @ projector_value(int(s.proj_l[c]), int(s.proj_m[c]), float(s.proj_sigma[c]), rc, D))
    want = np.array(want)
    assert np.abs(got - want).max() < 2e-3 * np.abs(want).max()
    assert abs(got[0] - want[0]) < 1e-3 * abs(want[0])


def test_graded_eigenvalues_against_uniform_refined():
    """Lowest eigenvalues of H x = lambda S x on a 3^3 two-level mesh of
    degree 4 against the same box in 3^3 uniform cells of degree 6 (the
    discretization error of both is below 3e-5 Ha here)."""
    def system(p):
        return custom_system((3, 3, 3), (6.0, 6.0, 6.0), p, p + 2, pos=[(3.3, 2.9, 3.1)], rcut=1.4,
                             channels="spd8", wells=[(3.0, 3.0, 3.0)], s_H=0.5, s_S=0.4, seed=5)
    g = with_two_level_gga(system(4), r_fine=1.0, gga=False)
    assert all(len(set(np.round(np.diff(b), 12))) == 2 for b in g.xgrid)
    lg = PAWOperator(g).dense_eigs(4)[0]
    lf = PAWOperator(system(6)).dense_eigs(4)[0]
    assert np.abs(lg - lf).max() < 1e-4


def test_graded_gga_grad_veff_exact_differences():
    base = make_system("tiny")
    s = with_two_level_gga(base, r_fine=1.5)
    op = PAWOperator(s)
    X = s.trial(3)
    occ = np.array([1.0, 0.5, 2.0])
    gV = grad.grad_veff(op, X, occ)
    rng = np.random.default_rng(3)
    for _ in range(4):
        e, q = int(rng.integers(op.mesh.E)), int(rng.integers(gV.shape[1]))
        v = s.veff_q.copy()
        v[e, q] += 1.0
        op2 = PAWOperator(dataclasses.replace(s, veff_q=v))
        diff = grad.band_energy(op2, X, occ) - grad.band_energy(op, X, occ)
        assert abs(diff - gV[e, q]) < 1e-9 * max(1.0, abs(gV[e, q]))


def test_graded_with_uniform_bounds_is_uniform():
    s = make_system("tiny")
    h = np.asarray(s.box) / np.asarray(s.ncell)
    xg = tuple(np.arange(n + 1) * h[d] for d, n in enumerate(s.ncell))
    a, b = PAWOperator(s), PAWOperator(dataclasses.replace(s, xgrid=xg))
    assert b.mesh.graded
    X = s.trial(4)
    for f in ("apply_H", "apply_S", "apply_Sinv"):
        ya, yb = getattr(a, f)(X), getattr(b, f)(X)
        assert np.abs(ya - yb).max() < 1e-12 * np.abs(ya).max()
    assert np.abs((a.C - b.C).toarray()).max() < 1e-14


def test_gga_term_enters_H_and_is_hermitian():
    s = with_two_level_gga(make_system("tiny"), r_fine=1.5)
    op = PAWOperator(s)
    plain = PAWOperator(dataclasses.replace(s, vgga_q=None))
    H, H0 = op.H_sparse(), plain.H_sparse()
    G = op.loc.assemble_GGA()
    assert abs((H - H0 - G)).max() < 1e-13 * abs(H).max()
    assert abs(G).max() > 1e-3
    assert abs(H - H.T).max() < 1e-12 * abs(H).max()
