"""Parity of the filter's fused local step against the oracle.

pawfe_cheb_step_local is the part of one step of Algorithm 2 (step 4) that
the filter's cell kernel carries:
    RX <- (-a c RY - zeta zeta' RX) + a Y Lambda_Y + a H_loc M_D^{-1} RY
with H_loc = K + V (+ the GGA term) the cell part of H (operator-action
subsection) and M_D the lumped GLL mass of eq. "Delta Sinv".  The oracle
side is the same formula written with the oracle's cell operator and lumped
mass, element by element, at every compiled degree, real and complex
operators, FP64 and FP32, ragged column counts, graded two-level meshes and
the GGA term, and at the paper's size (uniform and two-level GGA meshes) on
sampled columns in the launch configuration of the bench (256 columns)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _want(ref, RY, RX, Y, lam, a, ac, zz):
    return (-ac * RY - zz * RX) + a * Y * lam[None, :] + a * ref.loc.apply_H(ref.MDinv[:, None] * RY)


def _colmax_rel(got, want):
    return float(np.max(np.abs(got - want).max(axis=0) / np.abs(want).max(axis=0)))


def _real_cols(Z):
    """complex [M][n] -> real [M][2n] with (re, im) pairs, or a copy of real data"""
    Z = np.ascontiguousarray(Z)
    return Z.view(np.float64) if np.iscomplexobj(Z) else Z.copy()


def _case(ref, op, nc, cplx, prec, seed):
    rng = np.random.default_rng(seed)
    M = ref.mesh.M
    def draw():
        x = rng.standard_normal((M, nc))
        if cplx:
            x = x + 1j * rng.standard_normal((M, nc))
        return x
    RY, RX, Y = draw(), draw(), draw()
    lam = rng.uniform(-1.0, 3.0, nc)
    a, ac, zz = 0.37, -0.81, 0.42
    if prec == 1:   # FP32 data: both sides start from the rounded values
        RY = RY.astype(np.complex64 if cplx else np.float32).astype(RY.dtype)
        RX = RX.astype(np.complex64 if cplx else np.float32).astype(RX.dtype)
    want = _want(ref, RY, RX, Y, lam, a, ac, zz)
    dt = torch.float64 if prec == 0 else torch.float32
    RYd = _dev(_real_cols(RY)).to(dt)
    RXd = _dev(_real_cols(RX)).to(dt)
    lamr = np.repeat(lam, 2) if cplx else lam
    op.cheb_step_local(RYd, RXd, _dev(_real_cols(Y)), _dev(lamr), a, ac, zz, prec=prec)
    got = RXd.double().cpu().numpy()
    if cplx:
        got = got.view(np.complex128)
    return got, want


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
def test_step_local_every_degree(p, cplx):
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads.configs import custom_system
    n = (2, 3, 2) if p >= 5 else (3, 2, 3)
    box = tuple(1.6 * v for v in n)
    rng = np.random.Generator(np.random.PCG64(300 + p))
    pos = rng.uniform(0.0, 1.0, size=(2, 3)) * np.asarray(box)
    wells = rng.uniform(0.0, 1.0, size=(2, 3)) * np.asarray(box)
    kw = dict(kpoint=(0.3, -0.2, 0.45), is_complex=True) if cplx else {}
    s = custom_system(n, box, p, p + 2, pos=pos, rcut=1.2, channels="spd8", wells=wells, s_H=0.5, s_S=0.4,
                      seed=400 + p, nstates=9, **kw)
    ref, op = PAWOperator(s), Operator(s)
    nc = 7 if cplx else 13
    got, want = _case(ref, op, nc, cplx, 0, 10 + p)
    assert _colmax_rel(got, want) < 1e-12
    got, want = _case(ref, op, nc, cplx, 1, 20 + p)
    assert _colmax_rel(got, want) < 2e-5


@pytest.mark.parametrize("name", ["graded", "gga", "graded_gga"])
@pytest.mark.parametrize("p", [3, 6])
def test_step_local_general(p, name):
    """Graded two-level meshes and the GGA term: per-cell geometry, and the
    face factors of the lumped mass where neighbouring cells differ."""
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads.configs import custom_system, with_two_level_gga
    n = (3, 2, 4) if p < 5 else (2, 3, 2)
    box = tuple(1.6 * v for v in n)
    s = custom_system(n, box, p, p + 2, pos=[(1.0, 1.2, 1.4)], rcut=0.9, channels="spd8",
                      wells=[(1.5, 1.0, 2.0)], s_H=0.5, s_S=0.4, seed=70 + p, nstates=9)
    s = with_two_level_gga(s, r_fine=0.8, graded=name != "gga", gga=name != "graded")
    ref, op = PAWOperator(s), Operator(s)
    got, want = _case(ref, op, 11, False, 0, 30 + p)
    assert _colmax_rel(got, want) < 1e-12
    got, want = _case(ref, op, 11, False, 1, 40 + p)
    assert _colmax_rel(got, want) < 2e-5


@pytest.mark.parametrize("mesh", ["uniform", "graded_gga"])
def test_step_local_paper_sampled(mesh):
    """The paper's operator (20^3 cells of degree 6, 1,728,000 DOFs), and the
    same operator on the bench's two-level mesh with the GGA term, 256
    columns as in a filter block; columns 0, 77 and 255 against the oracle
    (the step is column by column)."""
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads import make_system
    from workloads.configs import with_two_level_gga
    s = make_system("paper")
    if mesh == "graded_gga":
        s = with_two_level_gga(s, r_fine=1.0)
    ref, op = PAWOperator(s), Operator(s)
    M, nc = ref.mesh.M, 256
    rng = np.random.default_rng(5)
    RY, RX, Y = (rng.standard_normal((M, nc)) for _ in range(3))
    lam = rng.uniform(-1.0, 3.0, nc)
    a, ac, zz = 0.37, -0.81, 0.42
    cols = [0, 77, 255]
    got = {}
    for prec in (0, 1):
        dt = torch.float64 if prec == 0 else torch.float32
        RYd, RXd = _dev(RY).to(dt), _dev(RX).to(dt)
        op.cheb_step_local(RYd, RXd, _dev(Y), _dev(lam), a, ac, zz, prec=prec)
        got[prec] = RXd.double().cpu().numpy()[:, cols]
        del RYd, RXd
    # one oracle call over both precisions' inputs (the step is column by
    # column): the FP64 columns, then the same columns rounded to FP32
    r32 = lambda z: z.astype(np.float32).astype(np.float64)
    ry, rx = RY[:, cols], RX[:, cols]
    want = _want(ref, np.hstack([ry, r32(ry)]), np.hstack([rx, r32(rx)]), np.hstack([Y[:, cols]] * 2),
                 np.concatenate([lam[cols]] * 2), a, ac, zz)
    k = len(cols)
    assert _colmax_rel(got[0], want[:, :k]) < 1e-12
    assert _colmax_rel(got[1], want[:, k:]) < 2e-5


def test_step_local_refusals():
    import dataclasses
    from paper_2604_26037_amd import BF16X3, Operator, PawfeError
    from workloads import make_system
    from workloads.configs import with_two_level_gga
    s = make_system("tiny")
    op = Operator(s)
    M = op.ndof
    z = torch.zeros((M, 4), dtype=torch.float32, device="cuda:0")
    y = torch.zeros((M, 4), dtype=torch.float64, device="cuda:0")
    lam = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    with pytest.raises(PawfeError):
        op.cheb_step_local(z, z.clone(), y, lam, 1.0, 1.0, 1.0, prec=BF16X3)
    g = Operator(with_two_level_gga(s, r_fine=1.5))
    with pytest.raises(PawfeError):
        g.cheb_step_local(z, z.clone(), y, lam, 1.0, 1.0, 1.0, prec=BF16X3)
    c = Operator(dataclasses.replace(s, kpoint=np.array([0.1, 0.0, 0.2]), is_complex=True))
    z3 = torch.zeros((M, 3), dtype=torch.float32, device="cuda:0")
    with pytest.raises(PawfeError):   # odd number of real columns on a complex operator
        c.cheb_step_local(z3, z3.clone(), y[:, :3], lam[:3], 1.0, 1.0, 1.0, prec=1)
