"""BF16 halo pack / unpack (pawfe_halo_pack_bf16, pawfe_halo_unpack_bf16)
against the oracle's definitions: bit-exact BF16 bits on both shared planes of
a slab, bit-exact FP32 accumulation, planes that wrap around the periodic
mesh, ragged column counts, complex operators, and the paper-scale plane
(20 x 20 cells of degree 6: 14,400 nodes per plane, 256 columns)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _check(op_h, ref, Y, kz0, kz1):
    from oracle import halo
    Yd = torch.from_numpy(Y).to("cuda:0")
    buf = op_h.halo_pack_bf16(Yd, kz0, kz1)
    torch.cuda.synchronize()
    Yr = Y.view(np.float32).reshape(Y.shape[0], -1) if Y.dtype == np.complex64 else Y
    want = halo.pack(ref, Yr, kz0, kz1)
    got = buf.cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(got, want)
    Z = np.random.default_rng(kz0 + 7).standard_normal(Yr.shape).astype(np.float32)
    Zd = torch.from_numpy(Z.view(np.complex64) if Y.dtype == np.complex64 else Z).to("cuda:0")
    op_h.halo_unpack_bf16(buf, Zd, kz0, kz1)
    torch.cuda.synchronize()
    gotZ = Zd.cpu().numpy()
    gotZ = gotZ.view(np.float32).reshape(Z.shape) if Y.dtype == np.complex64 else gotZ
    np.testing.assert_array_equal(gotZ, halo.unpack_add(ref, want, Z, kz0, kz1))


@pytest.mark.parametrize("kz", [(0, 2), (1, 3), (2, 4), (0, 3)])
@pytest.mark.parametrize("ncols", [1, 6, 13])
def test_halo_small(kz, ncols):
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads.configs import custom_system
    s = custom_system((3, 2, 4), (3.0, 2.0, 4.0), 3, 5)
    ref, op = PAWOperator(s), Operator(s)
    rng = np.random.default_rng(ncols)
    Y = (rng.standard_normal((op.ndof, ncols)) * 10.0 ** rng.integers(-20, 20, (op.ndof, ncols))).astype(np.float32)
    _check(op, ref, Y, *kz)


def test_halo_rejects_whole_mesh_slab():
    """A slab of all nz layers would share one plane with itself: rejected."""
    from paper_2604_26037_amd import Operator
    from paper_2604_26037_amd.pawfe import PawfeError
    from workloads.configs import custom_system
    op = Operator(custom_system((2, 2, 3), (2.0, 2.0, 3.0), 2, 4))
    Y = torch.zeros((op.ndof, 3), dtype=torch.float32, device="cuda:0")
    with pytest.raises(PawfeError):
        op.halo_pack_bf16(Y, 0, 3)


def test_halo_complex_operator():
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads.configs import custom_system
    s = custom_system((2, 3, 3), (2.0, 3.0, 3.0), 2, 4, kpoint=(0.2, 0.1, -0.3), is_complex=True)
    ref, op = PAWOperator(s), Operator(s)
    rng = np.random.default_rng(5)
    Y = (rng.standard_normal((op.ndof, 5)) + 1j * rng.standard_normal((op.ndof, 5))).astype(np.complex64)
    _check(op, ref, Y, 1, 2)


def test_halo_paper_plane():
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads import make_system
    from oracle import halo
    s = make_system("paper")
    op = Operator(s)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(3)
    Y = torch.randn((op.ndof, 256), generator=g, dtype=torch.float32, device="cuda:0")
    buf = op.halo_pack_bf16(Y, 5, 10)
    torch.cuda.synchronize()
    p, G = s.degree, s.ncell[0] * s.degree
    rows0 = np.arange(G * G) + 5 * p * G * G
    rows1 = np.arange(G * G) + 10 * p * G * G
    Yh = Y.cpu().numpy()
    got = buf.cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(got[0], halo.to_bf16_bits(Yh[rows0]))
    np.testing.assert_array_equal(got[1], halo.to_bf16_bits(Yh[rows1]))
