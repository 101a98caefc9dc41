"""Parity on a mesh whose cells' node-row offsets exceed the packed per-lane
field of the cell kernel (p + Gx (p + Gy p) >= 2^18), so every cell takes the
kernel's general (wrapping) node path: 100 x 100 x 2 cells of degree 3
(540,000 DOFs), a few columns, against the oracle."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_apply_general_node_path():
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads.configs import custom_system
    n, p = (100, 100, 2), 3
    assert p + n[0] * p * (p + n[1] * p * p) >= 1 << 18
    box = tuple(1.2 * v for v in n)
    pos = np.array([[30.0, 40.0, 1.0], [90.5, 100.2, 1.7]])
    s = custom_system(n, box, p, p + 2, pos=pos, rcut=1.0, channels="spd8", wells=pos, s_H=0.5, s_S=0.4,
                      seed=31, nstates=3)
    op = Operator(s)
    ref = PAWOperator(s)
    X = s.trial(3)
    Xd = torch.from_numpy(X).to("cuda:0")
    for which in ("H", "S"):
        got = getattr(op, "apply_" + which)(Xd).cpu().numpy()
        want = getattr(ref, "apply_" + which)(X)
        assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-10, which
    got32 = op.apply_H(Xd.float(), prec=1).cpu().numpy()
    want32 = ref.apply_H(X.astype(np.float32).astype(np.float64))
    assert np.linalg.norm(got32 - want32) / np.linalg.norm(want32) < 2e-5
