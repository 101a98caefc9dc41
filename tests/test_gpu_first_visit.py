"""The builder's first-visit bits of the colour-ordered assembly, which the
filter's fused step uses to apply the node part of a step exactly once per
DOF, against a brute force over the oracle's DOF map and colouring: for every
DOF the cells holding it, the lowest colour among them, and the position
class of the node in each of them.  Integer data: compared bit-exactly, on
meshes with even and odd cell counts (two and three colours per axis, two
cells per axis) and on a graded mesh."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")   # the HIP runtime the library shares with PyTorch


def _expected(mesh, p):
    cd = mesh.cell_dofs()                 # [E][np^3]
    col = mesh.cell_colour()              # [E]
    E, nl = cd.shape
    mincol = np.full(mesh.M, np.iinfo(np.int32).max, dtype=np.int64)
    np.minimum.at(mincol, cd.ravel(), np.repeat(col, nl))
    l = np.arange(nl)
    a, b, c = l % (p + 1), (l // (p + 1)) % (p + 1), l // ((p + 1) ** 2)
    cls1 = lambda x: np.where(x == 0, 0, np.where(x == p, 2, 1))
    cls = cls1(a) + 3 * cls1(b) + 9 * cls1(c)
    first = col[:, None] == mincol[cd]    # [E][nl]: this cell makes the node's first visit
    # every node of one class in one cell must agree (the bits are per class)
    masks = np.zeros(E, dtype=np.uint32)
    for k in range(27):
        sel = cls == k
        f = first[:, sel]
        assert np.all(f == f[:, :1]), f"class {k} not uniform"
        masks |= (f[:, 0].astype(np.uint32) << np.uint32(k))
    # exactly one first visit per DOF
    cnt = np.zeros(mesh.M, dtype=np.int64)
    np.add.at(cnt, cd[first], 1)
    assert np.all(cnt == 1)
    return masks


@pytest.mark.parametrize("n,p", [((3, 2, 4), 3), ((2, 3, 2), 5), ((5, 4, 3), 2), ((4, 4, 4), 6)])
def test_first_visit_bit_exact(n, p):
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads.configs import custom_system
    box = tuple(1.6 * v for v in n)
    s = custom_system(n, box, p, p + 2, pos=[(1.0, 1.2, 1.4)], rcut=0.9, channels="spd8",
                      wells=[(1.5, 1.0, 2.0)], seed=90 + p, nstates=4)
    ref, op = PAWOperator(s), Operator(s)
    np.testing.assert_array_equal(op.first_visit(), _expected(ref.mesh, p))


def test_first_visit_graded():
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads import make_system
    from workloads.configs import with_two_level_gga
    s = with_two_level_gga(make_system("tiny"), r_fine=1.5)
    ref, op = PAWOperator(s), Operator(s)
    np.testing.assert_array_equal(op.first_visit(), _expected(ref.mesh, s.degree))
