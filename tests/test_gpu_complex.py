"""GPU parity for complex (k-point) operators against the oracle built from
the same complex system: the Bloch Hamiltonian's 1/2 |k|^2 M and -i k.grad
local terms, the phased projectors, the complex G^{ab} and Delta_Sinv, through
every entry point that takes complex columns (applies, filter, Rayleigh-Ritz,
Lanczos bounds, the batched filter).  Columns are complex128 (complex64 for
the FP32 applies), stored as interleaved (re, im)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

K = (0.31, -0.22, 0.47)


def _system(p, k=K, nst=6, seed=0, sinv="exact_g"):
    from workloads.configs import custom_system
    n = (3, 3, 3) if p <= 4 else (2, 3, 2)
    box = tuple(1.7 * v for v in n)
    rng = np.random.Generator(np.random.PCG64(300 + p + seed))
    # positions outside the box too: the Bloch phase uses the given position
    pos = rng.uniform(0.0, 1.0, size=(3, 3)) * np.asarray(box) + np.array([[0, 0, 0], [5.1, 0, 0], [0, -3.4, 0]])
    wells = rng.uniform(0.0, 1.0, size=(3, 3)) * np.asarray(box)
    return custom_system(n, box, p, p + 2, pos=pos, rcut=1.2, channels="spd8", wells=wells, s_H=0.5, s_S=0.4,
                         seed=400 + p + seed, nstates=nst, kpoint=k, is_complex=True)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("sinv", ["exact_g", "pp"])
def test_complex_applies(p, sinv):
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    s = _system(p)
    ref = PAWOperator(s, sinv_mode=sinv)
    op = Operator(s, sinv_mode=sinv)
    assert op.complex and ref.complex
    X = s.trial(7)
    assert np.iscomplexobj(X)
    Xd = _dev(X)
    for which in ("H", "S", "Sinv"):
        got = getattr(op, "apply_" + which)(Xd).cpu().numpy()
        assert _rel(got, getattr(ref, "apply_" + which)(X)) < 1e-10, which
    X32 = X.astype(np.complex64)
    got32 = op.apply_H(_dev(X32), prec=1).cpu().numpy()
    assert _rel(got32, ref.apply_H(X32.astype(np.complex128))) < 2e-5


def test_complex_k_zero_matches_real_operator():
    """is_complex with k = 0: the complex operator acts on re and im parts as
    the real operator does."""
    from paper_2604_26037_amd import Operator
    sc = _system(4, k=(0.0, 0.0, 0.0))
    opc = Operator(sc)
    import dataclasses
    sr = dataclasses.replace(sc, is_complex=False)
    opr = Operator(sr)
    X = sc.trial(5)
    got = opc.apply_H(_dev(X)).cpu().numpy()
    re = opr.apply_H(_dev(np.ascontiguousarray(X.real))).cpu().numpy()
    im = opr.apply_H(_dev(np.ascontiguousarray(X.imag))).cpu().numpy()
    assert _rel(got, re + 1j * im) < 1e-12


@pytest.mark.parametrize("p", [3, 5])
def test_complex_filter_and_rr(p):
    from oracle import chfsi
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    s = _system(p, nst=10)
    ref = PAWOperator(s)
    op = Operator(s)
    X = s.trial(10)
    Psi, lam, res = chfsi.rayleigh_ritz(ref, X)
    # Rayleigh-Ritz on the GPU from the same start
    Xd = _dev(X)
    lam_d, res_d = op.rayleigh_ritz(Xd)
    assert np.abs(lam_d.cpu().numpy() - lam).max() < 1e-10 * max(1.0, np.abs(lam).max())
    np.testing.assert_allclose(res_d.cpu().numpy(), res, rtol=1e-7)
    # the rotated columns span the same eigenvectors (up to a phase per column)
    P = Xd.cpu().numpy()
    ov = np.abs(np.einsum('ij,ij->j', Psi.conj(), ref.apply_S(P)))
    np.testing.assert_allclose(ov, 1.0, atol=1e-8)
    # Algorithm 2, FP64, two blocks
    bU = 1.02 * max(chfsi.lanczos_bounds(ref, k=25)[1], float(lam[-1])) + 1.0
    b0, bW = float(lam[0]) - 0.1, float(lam[-1])
    want = chfsi.rchfsi_filter(ref, Psi, lam, 6, b0, bW, bU, block=6)
    got = op.cheb_filter(_dev(Psi), torch.from_numpy(lam), 6, b0, bW, bU, block=6).cpu().numpy()
    assert _rel(got, want) < 1e-9
    # mixed precision: FP32 recurrence, FP64 residual correction
    got32 = op.cheb_filter(_dev(Psi), torch.from_numpy(lam), 6, b0, bW, bU, block=6, prec=1).cpu().numpy()
    assert _rel(got32, want) < 1e-4


def test_complex_mixed_rotation():
    """Mixed-precision subspace rotation of a complex operator: the FP64 part
    is the complex diagonal of Q; vectors against the oracle's up to a unit
    phase per column."""
    from oracle import chfsi
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    s = _system(3, nst=10)
    ref = PAWOperator(s)
    op = Operator(s)
    X = s.trial(10)
    P_o, lam_o, res_o = chfsi.rayleigh_ritz(ref, X, mixed_sr=True)
    Xd = _dev(X)
    lam, res = op.rayleigh_ritz(Xd, sr_prec=1)
    lam, res, P = lam.cpu().numpy(), res.cpu().numpy(), Xd.cpu().numpy()
    assert np.abs(lam - lam_o).max() < 1e-10 * max(1.0, np.abs(lam_o).max())
    ph = np.einsum("ij,ij->j", P.conj(), P_o)
    ph = ph / np.abs(ph)
    assert np.abs(P * ph[None, :] - P_o).max() <= 1e-5 * np.abs(P_o).max()
    np.testing.assert_allclose(res, res_o, rtol=1e-3, atol=1e-6 * np.abs(res_o).max())


def test_complex_band_energy_gradient():
    """E = sum occ x^H H x, dE/dV(q) and dE/dDelta_H of a complex operator
    against the oracle's (the real part of the Hermitian projector form)."""
    from oracle import grad
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    s = _system(3, nst=6)
    ref = PAWOperator(s)
    op = Operator(s)
    X = s.trial(6)
    occ = np.linspace(2.0, 0.5, 6)
    E, dV, dD = op.band_energy_grad(_dev(X), occ=torch.from_numpy(occ))
    assert abs(float(E.cpu()[0]) - grad.band_energy(ref, X, occ)) < 1e-10 * abs(grad.band_energy(ref, X, occ))
    assert _rel(dV.cpu().numpy().ravel(), grad.grad_veff(ref, X, occ).ravel()) < 1e-10
    assert _rel(dD.cpu().numpy(), grad.grad_dH(ref, X, occ)) < 1e-10


def test_complex_lanczos_bounds():
    from oracle import chfsi
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    s = _system(3)
    ref = PAWOperator(s)
    op = Operator(s)
    tmin, tmax, beta = op.lanczos_bounds(k=25)
    mu_max = chfsi.lanczos_bounds(ref, k=60)[1]
    assert tmax <= mu_max * (1 + 1e-8)
    assert tmax + beta >= mu_max * (1 - 1e-6)


def test_complex_batch_matches_standalone():
    from oracle import chfsi
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator, Batch
    jobs, want = [], []
    for i, (p, k) in enumerate([(3, K), (4, (0.1, 0.0, -0.3)), (3, (0.0, 0.5, 0.0))]):
        s = _system(p, k=k, nst=8, seed=i)
        ref = PAWOperator(s)
        op = Operator(s)
        Psi, lam, _ = chfsi.rayleigh_ritz(ref, s.trial(8))
        bU = 1.02 * max(chfsi.lanczos_bounds(ref, k=20)[1], float(lam[-1])) + 1.0
        b0, bW = float(lam[0]) - 0.1, float(lam[-1])
        X = _dev(Psi)
        out = torch.empty_like(X)
        jobs.append(dict(op=op, X=X, out=out, lam=torch.from_numpy(lam).to("cuda:0"), degree=5, b0=b0, bW=bW,
                         bU=bU))
        want.append(op.cheb_filter(X, torch.from_numpy(lam), 5, b0, bW, bU).cpu().numpy())
    b = Batch(jobs, nstreams=2)
    b.run()
    torch.cuda.synchronize()
    for j, w in zip(jobs, want):
        assert _rel(j["out"].cpu().numpy(), w) < 1e-12
    b.close()
    # one graph per job
    for j in jobs:
        j["out"].zero_()
    b = Batch(jobs, nstreams=2, max_graph_launches=1)
    assert b.ngraphs == len(jobs)
    b.run()
    torch.cuda.synchronize()
    for j, w in zip(jobs, want):
        assert _rel(j["out"].cpu().numpy(), w) < 1e-12
    b.close()
