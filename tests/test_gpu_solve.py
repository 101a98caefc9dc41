"""The ChFSI outer loop on the GPU (pawfe_chfsi_solve): filter + FP64
Rayleigh-Ritz until the wanted residual norms meet the tolerance.  Against
the oracle's loop with the same b_U (same number of passes, same Ritz
values), and, with the device's own Lanczos bound, in mixed precision and
for a complex operator, against the dense eigenvalues through the
residual bound |theta_i - lambda_i| <= ||r_i||_2 / sqrt(lambda_min(S))."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NW, TOL = 8, 2e-3


@pytest.fixture(scope="module")
def tiny():
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads import make_system
    s = make_system("tiny")
    ref = PAWOperator(s)
    lam, _ = ref.dense_eigs(s.nstates)
    S = ref.S_dense()
    smin = float(np.linalg.eigvalsh(0.5 * (S + S.conj().T))[0])
    return s, ref, Operator(s), lam, smin


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def test_solve_fp64_matches_oracle_loop(tiny):
    from oracle import chfsi
    s, ref, op, lam, smin = tiny
    X = s.trial()
    t0, t1, beta = chfsi.lanczos_bounds(ref, k=20)
    bU = t1 + abs(beta)                                 # above every Ritz value
    _, th_o, res_o, it_o = chfsi.chfsi_solve(ref, X, s.cheb_degree, bU, TOL, 30, nwanted=NW)
    assert it_o >= 1
    Xd = _dev(X)
    th, res, it = op.chfsi_solve(Xd, s.cheb_degree, TOL, 30, nwanted=NW, bU=bU)
    th, res = th.cpu().numpy(), res.cpu().numpy()
    assert it == it_o
    assert np.max(np.abs(th - th_o)) < 1e-9 * max(1.0, np.abs(th_o).max())
    np.testing.assert_allclose(res, res_o, rtol=1e-6, atol=1e-12)
    assert np.max(res[:NW]) <= TOL


@pytest.mark.parametrize("prec", [0, 1])
def test_solve_lanczos_bound_converges(tiny, prec):
    s, ref, op, lam, smin = tiny
    Xd = _dev(s.trial())
    th, res, it = op.chfsi_solve(Xd, s.cheb_degree, TOL, 40, nwanted=NW, prec=prec, block=5)
    th, res = th.cpu().numpy(), res.cpu().numpy()
    assert 1 <= it < 40
    assert np.max(res[:NW]) <= TOL
    assert np.all(np.abs(th[:NW] - lam[:NW]) <= res[:NW] / np.sqrt(smin) * (1 + 1e-6))


def test_solve_complex_operator():
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads.configs import custom_system
    n = (3, 3, 3)
    box = tuple(1.7 * v for v in n)
    rng = np.random.Generator(np.random.PCG64(77))
    pos = rng.uniform(0.0, 1.0, size=(2, 3)) * np.asarray(box)
    s = custom_system(n, box, 3, 5, pos=pos, rcut=1.2, channels="spd8", wells=pos, s_H=0.5, s_S=0.4,
                      seed=78, nstates=10, kpoint=(0.2, -0.1, 0.3), is_complex=True)
    ref = PAWOperator(s)
    lam, _ = ref.dense_eigs(10)
    S = ref.S_dense()
    smin = float(np.linalg.eigvalsh(0.5 * (S + S.conj().T))[0])
    op = Operator(s)
    th, res, it = op.chfsi_solve(_dev(s.trial(10)), 12, 1e-4, 60, nwanted=5)
    th, res = th.cpu().numpy(), res.cpu().numpy()
    assert np.max(res[:5]) <= 1e-4
    assert np.all(np.abs(th[:5] - lam[:5]) <= res[:5] / np.sqrt(smin) * (1 + 1e-6))
