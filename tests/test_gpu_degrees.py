"""Parity of every compiled element degree (p = 2..6 with n_q = p + 2) against
the oracle, on small periodic meshes with ragged column counts: H, S and
Sinv_hat applies in FP64 (and H in FP32), and a short filter in FP64 and in
mixed precision."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _system(p):
    from workloads.configs import custom_system
    n = (2, 3, 2) if p >= 5 else (3, 2, 3)
    box = tuple(1.6 * v for v in n)
    rng = np.random.Generator(np.random.PCG64(100 + p))
    pos = rng.uniform(0.0, 1.0, size=(2, 3)) * np.asarray(box)
    wells = rng.uniform(0.0, 1.0, size=(2, 3)) * np.asarray(box)
    return custom_system(n, box, p, p + 2, pos=pos, rcut=1.2, channels="spd8", wells=wells,
                         s_H=0.5, s_S=0.4, seed=200 + p, nstates=13)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
def test_degree_applies_and_filter(p):
    from oracle import chfsi
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    s = _system(p)
    ref = PAWOperator(s)
    op = Operator(s)
    X = s.trial(13)
    Xd = torch.from_numpy(X).to("cuda:0")
    for which in ("H", "S", "Sinv"):
        got = getattr(op, "apply_" + which)(Xd).cpu().numpy()
        assert _rel(got, getattr(ref, "apply_" + which)(X)) < 1e-10, which
    got32 = op.apply_H(Xd.float(), prec=1).cpu().numpy()
    assert _rel(got32, ref.apply_H(X.astype(np.float32).astype(np.float64))) < 2e-5
    Psi, lam, _ = chfsi.rayleigh_ritz(ref, X)
    bU = 1.02 * max(chfsi.lanczos_bounds(ref, k=20)[1], float(lam[-1])) + 1.0
    b0, bW = float(lam[0]), float(lam[-1])
    want = chfsi.rchfsi_filter(ref, Psi, lam, 7, b0, bW, bU, block=5)
    got = op.cheb_filter(torch.from_numpy(Psi).to("cuda:0"), torch.from_numpy(lam), 7, b0, bW, bU,
                         block=5).cpu().numpy()
    assert _rel(got, want) < 1e-9
    # mixed precision (FP32 recurrence, FP64 residual correction), element-wise per column
    got32 = op.cheb_filter(torch.from_numpy(Psi).to("cuda:0"), torch.from_numpy(lam), 7, b0, bW, bU,
                           block=5, prec=1).cpu().numpy()
    assert float(np.max(np.abs(got32 - want).max(axis=0) / np.abs(want).max(axis=0))) < 1e-4
