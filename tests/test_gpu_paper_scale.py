"""GPU parity at the paper scale (20^3 cells, p = 6, 1,728,000 DOFs, 128 atoms
x 18 projectors), in the launch configuration the bench times (256-column
blocks).  The oracle computes the sampled columns only (columns are
independent in every apply and in the filter), so it finishes in seconds.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SAMPLE = [0, 1, 77, 128, 200, 255]       # columns of a 256-column block checked against the oracle


@pytest.fixture(scope="module")
def paper():
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads import make_system
    s = make_system("paper")
    op = Operator(s)
    ref = PAWOperator(s)
    X = s.trial(256)
    return s, ref, op, X


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _rel(a, b):
    fro = np.linalg.norm(a - b) / np.linalg.norm(b)
    col = np.max(np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0))
    return fro, col


def test_dofmap_paper(paper):
    s, ref, op, X = paper
    cd, col, sco, sc, sno, sn = op.dofmap()
    np.testing.assert_array_equal(col, ref.mesh.cell_colour())
    co, cells, no, nodes = ref.support_lists()
    np.testing.assert_array_equal(sc, cells)
    np.testing.assert_array_equal(sn, nodes)
    np.testing.assert_array_equal(cd[::97], ref.mesh.cell_dofs()[::97])


@pytest.mark.parametrize("which", ["H", "S", "Sinv"])
def test_apply_fp64_paper_block(paper, which):
    s, ref, op, X = paper
    Y = getattr(op, "apply_" + which)(_dev(X)).cpu().numpy()[:, SAMPLE]
    Yr = getattr(ref, "apply_" + which)(X[:, SAMPLE])
    fro, col = _rel(Y, Yr)
    assert fro < 1e-10 and col < 1e-10, (fro, col)


@pytest.mark.parametrize("which", ["H", "Sinv"])
def test_apply_fp32_paper_block(paper, which):
    s, ref, op, X = paper
    Y = getattr(op, "apply_" + which)(_dev(X).float(), prec=1).cpu().numpy()[:, SAMPLE]
    Yr = getattr(ref, "apply_" + which)(X[:, SAMPLE].astype(np.float32).astype(np.float64))
    fro, col = _rel(Y, Yr)
    assert fro < 2e-5 and col < 5e-5, (fro, col)


def test_filter_fp64_paper_block(paper):
    """Algorithm 2 (degree 3) on a 256-column block: sampled columns vs the oracle."""
    from oracle import chfsi
    s, ref, op, X = paper
    lam = np.linspace(-0.9, 0.4, 256)
    b0, bW, bU = -1.0, 0.5, 320.0
    got = op.cheb_filter(_dev(X), torch.from_numpy(lam), 3, b0, bW, bU, block=256).cpu().numpy()
    want, _ = chfsi.rchfsi_block(ref.apply_H, ref.apply_S, ref.apply_Sinv, X[:, SAMPLE], lam[SAMPLE], 3,
                                 b0, bW, bU)
    fro, col = _rel(got[:, SAMPLE], want)
    assert fro < 1e-9 and col < 1e-9, (fro, col)


def test_filter_mixed_paper_block(paper):
    """FP32 recurrence vs the FP64 oracle (degree 3): FP32-level agreement."""
    from oracle import chfsi
    s, ref, op, X = paper
    lam = np.linspace(-0.9, 0.4, 256)
    b0, bW, bU = -1.0, 0.5, 320.0
    got = op.cheb_filter(_dev(X), torch.from_numpy(lam), 3, b0, bW, bU, block=256, prec=1).cpu().numpy()
    want, _ = chfsi.rchfsi_block(ref.apply_H, ref.apply_S, ref.apply_Sinv, X[:, SAMPLE], lam[SAMPLE], 3,
                                 b0, bW, bU)
    fro, col = _rel(got[:, SAMPLE], want)
    assert fro < 1e-4 and col < 1e-4, (fro, col)


def test_rayleigh_ritz_paper(paper):
    from oracle import chfsi
    s, ref, op, X = paper
    Xs = X[:, :24]
    _, lam_ref, res_ref = chfsi.rayleigh_ritz(ref, Xs)
    lam, res = op.rayleigh_ritz(_dev(Xs))
    lam = lam.cpu().numpy()
    assert np.abs(lam - lam_ref).max() < 1e-10 * max(1.0, np.abs(lam_ref).max())
    np.testing.assert_allclose(res.cpu().numpy(), res_ref, rtol=1e-7)


def _colmax_rel(got, want):
    """Largest element-wise deviation of each column relative to that
    column's largest entry (no dilution by the column norm)."""
    return float(np.max(np.abs(got - want).max(axis=0) / np.abs(want).max(axis=0)))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_filter_paper_block_degree30_elementwise(paper, prec):
    """The bench's polynomial degree (30) on a 256-column block with Ritz-like
    bounds; two sampled columns against the oracle's Algorithm 2, element by
    element (FP64 1e-9, mixed 1e-4 of the column's largest entry)."""
    from oracle import chfsi
    s, ref, op, X = paper
    lam = np.linspace(1.5, 9.0, 256)
    b0, bW, bU = 1.4, 9.0, 346.0
    cols = [0, 201]
    got = op.cheb_filter(_dev(X), torch.from_numpy(lam), 30, b0, bW, bU, block=256,
                         prec=0 if prec == "fp64" else 1).cpu().numpy()[:, cols]
    want, _ = chfsi.rchfsi_block(ref.apply_H, ref.apply_S, ref.apply_Sinv, X[:, cols], lam[cols], 30,
                                 b0, bW, bU)
    err = _colmax_rel(got, want)
    assert err < (1e-9 if prec == "fp64" else 1e-4), err


@pytest.mark.parametrize("which", ["H", "Sinv"])
def test_apply_fp64_paper_block_elementwise(paper, which):
    s, ref, op, X = paper
    Y = getattr(op, "apply_" + which)(_dev(X)).cpu().numpy()[:, SAMPLE]
    Yr = getattr(ref, "apply_" + which)(X[:, SAMPLE])
    assert _colmax_rel(Y, Yr) < 1e-12
