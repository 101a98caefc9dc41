"""Edge cases through the C ABI against the oracle: the most projectors an
atom may carry (32, and 27: the padded lanes of the 32-wide kernels), an
operator without atoms (H = K + V, S = M, Sinv_hat = M_D^{-1}), and calls
on zero columns (no work, outputs untouched)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _system(channels, natoms=2, p=3):
    from workloads.configs import custom_system
    n = (3, 3, 3)
    box = tuple(1.7 * v for v in n)
    rng = np.random.Generator(np.random.PCG64(500 + natoms))
    pos = rng.uniform(0.0, 1.0, size=(natoms, 3)) * np.asarray(box)
    return custom_system(n, box, p, p + 2, pos=pos, rcut=1.4, channels=channels,
                         wells=rng.uniform(0.0, 1.0, size=(2, 3)) * np.asarray(box),
                         s_H=0.5, s_S=0.2, seed=600 + natoms, nstates=9)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _check_applies_and_filter(s):
    from oracle import chfsi
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    ref = PAWOperator(s)
    op = Operator(s)
    X = s.trial(9)
    Xd = _dev(X)
    for which in ("H", "S", "Sinv"):
        got = getattr(op, "apply_" + which)(Xd).cpu().numpy()
        assert _rel(got, getattr(ref, "apply_" + which)(X)) < 1e-10, which
    got32 = op.apply_H(Xd.float(), prec=1).cpu().numpy()
    assert _rel(got32, ref.apply_H(X.astype(np.float32).astype(np.float64))) < 2e-5
    Psi, lam, _ = chfsi.rayleigh_ritz(ref, X)
    bU = 1.02 * max(chfsi.lanczos_bounds(ref, k=20)[1], float(lam[-1])) + 1.0
    b0, bW = float(lam[0]) - 0.1, float(lam[-1])
    want = chfsi.rchfsi_filter(ref, Psi, lam, 6, b0, bW, bU, block=4)
    got = op.cheb_filter(_dev(Psi), torch.from_numpy(lam), 6, b0, bW, bU, block=4).cpu().numpy()
    assert _rel(got, want) < 1e-9
    lam_d, _ = op.rayleigh_ritz(_dev(X))
    assert np.abs(lam_d.cpu().numpy() - lam).max() < 1e-10 * max(1.0, np.abs(lam).max())


@pytest.mark.parametrize("channels", ["max32", "spd27"])
def test_most_projectors_per_atom(channels):
    s = _system(channels)
    assert int(s.nproj[0]) == (32 if channels == "max32" else 27)
    _check_applies_and_filter(s)


def test_operator_without_atoms():
    s = _system("spd8", natoms=0)
    assert len(s.pos) == 0
    _check_applies_and_filter(s)


def test_zero_columns_leave_outputs_untouched():
    from paper_2604_26037_amd import Operator
    s = _system("spd8")
    op = Operator(s)
    X = _dev(s.trial(4))
    Y = torch.full_like(X, 7.0)
    lib = __import__("paper_2604_26037_amd.pawfe", fromlist=["load"]).load()
    for fn in (lib.pawfe_apply_H, lib.pawfe_apply_S, lib.pawfe_apply_Sinv):
        assert fn(op._h, X.data_ptr(), 4, Y.data_ptr(), 4, 0, 0, None) == 0
    assert lib.pawfe_apply_local(op._h, 0, X.data_ptr(), 4, Y.data_ptr(), 4, 0, 1.0, 0, None) == 0
    torch.cuda.synchronize()
    assert bool((Y == 7.0).all())


def test_more_columns_than_one_chunk():
    """Applies over 600 columns (the entry points work in chunks of 512) and
    Rayleigh-Ritz over 300 (projections in blocks of 256), both with a ragged
    last piece, against the oracle."""
    from oracle import chfsi
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads import make_system
    s = make_system("tiny")
    ref = PAWOperator(s)
    op = Operator(s)
    X = s.trial(600)
    Xd = _dev(X)
    for which in ("H", "S", "Sinv"):
        got = getattr(op, "apply_" + which)(Xd).cpu().numpy()
        assert _rel(got, getattr(ref, "apply_" + which)(X)) < 1e-10, which
    X3 = np.ascontiguousarray(X[:, :300])
    _, lam_o, res_o = chfsi.rayleigh_ritz(ref, X3)
    X3d = _dev(X3)
    lam, res = op.rayleigh_ritz(X3d)
    lam, res = lam.cpu().numpy(), res.cpu().numpy()
    assert np.abs(lam - lam_o).max() < 1e-9 * max(1.0, np.abs(lam_o).max())
    np.testing.assert_allclose(res, res_o, rtol=1e-6, atol=1e-9 * np.abs(res_o).max())


@pytest.mark.parametrize("cplx", [False, True])
def test_rayleigh_ritz_singular_overlap_is_refused(cplx):
    """A zero column makes the projected overlap S^p singular (an exactly
    zero pivot of its Cholesky factor): Rayleigh-Ritz reports ENOTSPD instead
    of returning a rotation."""
    from paper_2604_26037_amd import Operator
    from paper_2604_26037_amd.pawfe import PAWFE_ENOTSPD, PawfeError
    from workloads.configs import custom_system
    n = (3, 3, 3)
    box = tuple(1.7 * v for v in n)
    rng = np.random.Generator(np.random.PCG64(77))
    extra = dict(kpoint=(0.2, -0.1, 0.3), is_complex=True) if cplx else {}
    s = custom_system(n, box, 3, 5, pos=rng.uniform(0.0, 1.0, size=(2, 3)) * np.asarray(box), rcut=1.4,
                      channels="spd8", wells=rng.uniform(0.0, 1.0, size=(2, 3)) * np.asarray(box),
                      s_H=0.5, s_S=0.2, seed=78, nstates=6, **extra)
    op = Operator(s)
    X = s.trial(6)
    X[:, 3] = 0.0
    with pytest.raises(PawfeError) as e:
        op.rayleigh_ritz(_dev(X))
    assert e.value.code == PAWFE_ENOTSPD
    # the operator still serves a well-posed block afterwards
    lam, _ = op.rayleigh_ritz(_dev(s.trial(6)))
    assert bool(torch.isfinite(lam).all())
