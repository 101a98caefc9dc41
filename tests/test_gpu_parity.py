"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Inputs are the seeded synthetic systems of workloads/; expected values come
from oracle/ on the same arrays.  Tolerances (relative, Frobenius norm over
the block and worst single column): FP64 operator applies <= 1e-10, FP64
filter output <= 1e-9, FP64 Ritz values <= 1e-10 Ha, mixed-precision Ritz
values after the FP64 Rayleigh-Ritz <= 1e-6 Ha, gradient <= 1e-10.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def systems():
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads import make_system
    out = {}
    for name in ("tiny", "mid"):
        s = make_system(name)
        out[name] = (s, PAWOperator(s), Operator(s))
    return out


def _rel(a, b):
    """(Frobenius relative error, worst column relative error)."""
    fro = np.linalg.norm(a - b) / np.linalg.norm(b)
    col = np.max(np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(b, axis=0), 1e-300))
    return fro, col


def _to(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(_dev())


@pytest.mark.parametrize("name", ["tiny", "mid"])
def test_dofmap_bit_exact(systems, name):
    s, ref, op = systems[name]
    cd, col, sco, sc, sno, sn = op.dofmap()
    np.testing.assert_array_equal(cd, ref.mesh.cell_dofs())
    np.testing.assert_array_equal(col, ref.mesh.cell_colour())
    co, cells, no, nodes = ref.support_lists()
    np.testing.assert_array_equal(sco, co)
    np.testing.assert_array_equal(sc, cells)
    np.testing.assert_array_equal(sno, no)
    np.testing.assert_array_equal(sn, nodes)


@pytest.mark.parametrize("name,ncols", [("tiny", 16), ("tiny", 5), ("mid", 70), ("mid", 1)])
@pytest.mark.parametrize("which", ["H", "S", "Sinv"])
def test_apply_fp64(systems, name, ncols, which):
    s, ref, op = systems[name]
    X = s.trial(ncols)
    Y = getattr(op, "apply_" + which)(_to(X)).cpu().numpy()
    Yr = getattr(ref, "apply_" + which)(X)
    fro, col = _rel(Y, Yr)
    assert fro < 1e-10 and col < 1e-10, (fro, col)


@pytest.mark.parametrize("which", ["H", "S", "Sinv"])
def test_apply_fp32(systems, which):
    s, ref, op = systems["mid"]
    X = s.trial(33)
    Y = getattr(op, "apply_" + which)(_to(X).float(), prec=1).cpu().numpy()
    Yr = getattr(ref, "apply_" + which)(X.astype(np.float32).astype(np.float64))
    fro, col = _rel(Y, Yr)
    assert fro < 2e-5 and col < 5e-5, (fro, col)


def test_apply_ld_and_strided_columns(systems):
    s, ref, op = systems["mid"]
    X = s.trial(24)
    big = torch.zeros((X.shape[0], 40), dtype=torch.float64, device=_dev())
    big[:, 3:27] = _to(X)
    out = torch.full((X.shape[0], 50), 7.0, dtype=torch.float64, device=_dev())
    op.apply_H(big[:, 3:27], out=out[:, 10:34])
    Yr = ref.apply_H(X)
    fro, _ = _rel(out[:, 10:34].cpu().numpy(), Yr)
    assert fro < 1e-10
    o = out.cpu().numpy()
    assert np.all(o[:, :10] == 7.0) and np.all(o[:, 34:] == 7.0)     # untouched columns


def _bounds(ref_lam, bU):
    return float(ref_lam[0]), float(ref_lam[-1]), bU


@pytest.mark.parametrize("name,N,block,m", [("tiny", 16, 16, 20), ("tiny", 16, 5, 7), ("mid", 70, 40, 12)])
def test_cheb_filter_fp64(systems, name, N, block, m):
    from oracle import chfsi
    s, ref, op = systems[name]
    X = s.trial(N)
    Psi, lam, _ = chfsi.rayleigh_ritz(ref, X)
    bU = 1.02 * chfsi.lanczos_bounds(ref, k=25)[1] + 1.0
    b0, bW = float(lam[0]), float(lam[-1])
    ref_out = chfsi.rchfsi_filter(ref, Psi, lam, m, b0, bW, bU, block=block)
    got = op.cheb_filter(_to(Psi), torch.from_numpy(lam), m, b0, bW, bU, block=block).cpu().numpy()
    fro, col = _rel(got, ref_out)
    assert fro < 1e-9 and col < 1e-9, (fro, col)


def test_cheb_filter_in_place(systems):
    from oracle import chfsi
    s, ref, op = systems["tiny"]
    X = s.trial(16)
    Psi, lam, _ = chfsi.rayleigh_ritz(ref, X)
    b0, bW, bU = float(lam[0]), float(lam[-1]), 150.0
    Pd = _to(Psi)
    out = op.cheb_filter(Pd, torch.from_numpy(lam), 9, b0, bW, bU, block=6)
    Pd2 = _to(Psi)
    op.cheb_filter(Pd2, torch.from_numpy(lam), 9, b0, bW, bU, block=6, out=Pd2)
    assert torch.equal(out, Pd2)


def test_rayleigh_ritz_fp64(systems):
    from oracle import chfsi
    s, ref, op = systems["tiny"]
    X = s.trial(16)
    _, lam_ref, res_ref = chfsi.rayleigh_ritz(ref, X)
    Xd = _to(X)
    lam, res = op.rayleigh_ritz(Xd)
    lam, res = lam.cpu().numpy(), res.cpu().numpy()
    assert np.abs(lam - lam_ref).max() < 1e-10 * max(1.0, np.abs(lam_ref).max())
    np.testing.assert_allclose(res, res_ref, rtol=1e-8, atol=1e-10)
    Psi = Xd.cpu().numpy()
    np.testing.assert_allclose(Psi.T @ ref.apply_S(Psi), np.eye(16), atol=1e-10)


@pytest.mark.parametrize("name,n", [("tiny", 16), ("mid", 40)])
def test_rayleigh_ritz_mixed_rotation(systems, name, n):
    """Mixed-precision subspace rotation (FP64 diagonal of Q, FP32 off-diagonal
    GEMM) against the oracle's: the same Ritz values as FP64, the rotated
    vectors within the FP32 rounding of the off-diagonal part (up to the sign
    of each eigenvector), the residual norms of the rotated vectors."""
    from oracle import chfsi
    s, ref, op = systems[name]
    X = s.trial(n)
    P_o, lam_o, res_o = chfsi.rayleigh_ritz(ref, X, mixed_sr=True)
    Xd = _to(X)
    lam, res = op.rayleigh_ritz(Xd, sr_prec=1)
    lam, res, P = lam.cpu().numpy(), res.cpu().numpy(), Xd.cpu().numpy()
    assert np.abs(lam - lam_o).max() < 1e-10 * max(1.0, np.abs(lam_o).max())
    sg = np.sign(np.einsum("ij,ij->j", P, P_o))
    assert np.abs(P * sg[None, :] - P_o).max() <= 1e-5 * np.abs(P_o).max()
    np.testing.assert_allclose(res, res_o, rtol=1e-3, atol=1e-6 * np.abs(res_o).max())
    # not the FP64 rotation: the off-diagonal part was rounded
    Xe = _to(X)
    op.rayleigh_ritz(Xe)
    assert np.abs(Xe.cpu().numpy() * sg[None, :] - P * sg[None, :]).max() > 0


def test_mixed_rotation_degenerate_states():
    """The mixed-precision rotation near convergence on a spectrum with
    degenerate levels (free electrons in a cube: levels of multiplicity 1, 6,
    12, 8), where Q is not close to the identity inside each degenerate
    cluster.  The change of every residual norm against the FP64 rotation is
    bounded by the FP32 rounding of the off-diagonal product:
    | ||r_i^32|| - ||r_i^64|| | <= ||H - lambda_i S||_2 ||E_i||_2 with
    |E_i| <= gamma_{N+2}(u32) |X| |Q_off|[:, i]."""
    from oracle import chfsi
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads.configs import custom_system
    s = custom_system((3, 3, 3), (6.0, 6.0, 6.0), 4, 6, nstates=20)
    ref, op = PAWOperator(s), Operator(s)
    H, S = ref.H_dense(), ref.S_dense()
    evS = np.linalg.eigvalsh(S)
    X = _to(s.trial(20))
    lam, res = op.rayleigh_ritz(X)
    lam_all = ref.dense_eigs()[0]
    bU = 1.01 * float(lam_all[-1])
    for it in range(7):
        lh = lam.cpu().numpy()
        op.cheb_filter(X, lam, 12, float(lh[0]), float(lh[-1]), bU, out=X)
        if it < 6:
            lam, res = op.rayleigh_ritz(X)
    Xh = X.cpu().numpy()                                  # filtered, not yet rotated
    X64, X32 = _to(Xh), _to(Xh)
    lam64, res64 = op.rayleigh_ritz(X64)
    lam32, res32 = op.rayleigh_ritz(X32, sr_prec=1)
    lam64, res64, res32 = lam64.cpu().numpy(), res64.cpu().numpy(), res32.cpu().numpy()
    P64 = X64.cpu().numpy()
    G = Xh.T @ (S @ Xh)
    Q = np.linalg.solve(G, Xh.T @ (S @ P64))              # P64 = X Q
    Qoff = Q - np.diag(np.diag(Q))
    assert np.abs(Qoff).max() > 1e-3                      # the off-diagonal product is not trivial
    u32 = 2.0 ** -24
    gam = (20 + 2) * u32 / (1 - (20 + 2) * u32)
    Ebound = gam * np.linalg.norm(np.abs(Xh) @ np.abs(Qoff), axis=0)
    normS = float(evS[-1])
    normH = float(np.abs(np.linalg.eigvalsh(H)).max())
    bound = (normH + np.abs(lam64) * normS) * Ebound
    diff = np.abs(res32 - res64)
    assert np.all(diff <= bound), (diff / bound).max()
    print(f"[mixed-rotation] max |Q_off| {np.abs(Qoff).max():.2f}, residual change "
          f"{diff.max():.2e} (bound {bound.min():.2e}..{bound.max():.2e}), FP64 residuals {res64.max():.2e}")


def test_chfsi_iterations_fp64_vs_oracle_and_dense(systems):
    """Config 'tiny': RR of the start, then 3 x (filter degree 20 + RR), all on the GPU."""
    from oracle import chfsi
    s, ref, op = systems["tiny"]
    lam_dense = ref.dense_eigs(nev=16)[0]
    bU = 1.02 * chfsi.lanczos_bounds(ref, k=25)[1] + 1.0
    X = s.trial()
    _, lam_o, hist = chfsi.chfsi_iterations(ref, X, s.iterations, s.cheb_degree, bU)
    Xd = _to(X)
    lam, _ = op.rayleigh_ritz(Xd)
    for _ in range(s.iterations):
        l = lam.cpu().numpy()
        Xd = op.cheb_filter(Xd, lam, s.cheb_degree, float(l[0]), float(l[-1]), bU, out=Xd)
        lam, res = op.rayleigh_ritz(Xd)
    lam = lam.cpu().numpy()
    assert np.abs(lam - lam_o).max() < 1e-9
    assert np.all(lam >= lam_dense - 1e-10)            # Courant-Fischer vs the dense GHEP


def test_mixed_precision_eigenvalues(systems):
    """FP32 recurrence + FP64 RR reaches the FP64 Ritz values within 1e-6 Ha."""
    from oracle import chfsi
    s, ref, op = systems["mid"]
    bU = 1.02 * chfsi.lanczos_bounds(ref, k=25)[1] + 1.0
    X = s.trial(40)
    X64 = _to(X)
    lam, _ = op.rayleigh_ritz(X64)
    X32 = X64.clone()
    l32 = lam.clone()
    l64 = lam.clone()
    nw = int(np.ceil(40 / 1.2))
    for it in range(3):
        a = l64.cpu().numpy()
        X64 = op.cheb_filter(X64, l64, 12, float(a[0]), float(a[-1]), bU, out=X64)
        l64, _ = op.rayleigh_ritz(X64)
        b = l32.cpu().numpy()
        X32 = op.cheb_filter(X32, l32, 12, float(b[0]), float(b[-1]), bU, prec=1, out=X32)
        l32, _ = op.rayleigh_ritz(X32)
        err = np.abs(l32.cpu().numpy()[:nw] - l64.cpu().numpy()[:nw]).max()
        assert err < 1e-6, (it, err)


def test_band_energy_gradient(systems):
    from oracle import grad
    s, ref, op = systems["mid"]
    X = s.trial(12)
    occ = np.linspace(2.0, 0.5, 12)
    E, dV, dD = op.band_energy_grad(_to(X), torch.from_numpy(occ))
    assert abs(E.item() - grad.band_energy(ref, X, occ)) < 1e-10 * abs(E.item())
    gV = grad.grad_veff(ref, X, occ)
    fro, _ = _rel(dV.cpu().numpy().reshape(gV.shape), gV)
    assert fro < 1e-10
    gD = grad.grad_dH(ref, X, occ)
    assert np.linalg.norm(dD.cpu().numpy() - gD) < 1e-10 * np.linalg.norm(gD)


def test_band_energy_autograd_fd(systems):
    """torch.autograd through the hand-written adjoint vs central differences."""
    from paper_2604_26037_amd import band_energy_function
    s, ref, op = systems["tiny"]
    BE = band_energy_function()
    X = _to(s.trial(4))
    V = torch.from_numpy(s.veff_q.copy()).requires_grad_(True)
    D = torch.from_numpy(s.dH.copy()).requires_grad_(True)
    E = BE.apply(X, V, D, op)
    E.backward()
    rng = np.random.default_rng(0)
    for _ in range(4):
        i = int(rng.integers(V.numel()))
        h = 1e-2
        Vp = s.veff_q.copy().ravel(); Vp[i] += h
        Vm = s.veff_q.copy().ravel(); Vm[i] -= h
        op.set_veff(Vp)
        Ep = op.band_energy_grad(X, want_dV=False, want_dH=False)[0].item()
        op.set_veff(Vm)
        Em = op.band_energy_grad(X, want_dV=False, want_dH=False)[0].item()
        fd = (Ep - Em) / (2 * h)
        assert abs(fd - V.grad.view(-1)[i].item()) < 1e-9 * max(1.0, abs(fd)) + 1e-12 * abs(Ep) / h
    op.set_veff(s.veff_q)
    op.set_dH(s.dH)


def test_band_energy_autograd_dX(systems):
    """The X gradient of the band energy (2 H X diag(occ)) through torch.autograd
    against central differences along a random direction (E is quadratic in X,
    so the central difference is exact up to rounding)."""
    from paper_2604_26037_amd import band_energy_function
    s, ref, op = systems["tiny"]
    BE = band_energy_function()
    X0 = _to(s.trial(4))
    occ = torch.tensor([2.0, 1.5, 1.0, 0.5], dtype=torch.float64, device=X0.device)
    V = torch.from_numpy(s.veff_q.copy())
    D = torch.from_numpy(s.dH.copy())
    X = X0.clone().requires_grad_(True)
    BE.apply(X, V, D, op, occ).backward()
    dirn = _to(np.random.default_rng(5).standard_normal(X0.shape))
    h = 1e-3
    Ep = op.band_energy_grad(X0 + h * dirn, occ, want_dV=False, want_dH=False)[0].item()
    Em = op.band_energy_grad(X0 - h * dirn, occ, want_dV=False, want_dH=False)[0].item()
    fd = (Ep - Em) / (2 * h)
    an = float((X.grad * dirn).sum())
    assert abs(fd - an) < 1e-9 * abs(an), (fd, an)


def test_lanczos_bounds(systems):
    from oracle import chfsi
    s, ref, op = systems["tiny"]
    tmin, tmax, beta = op.lanczos_bounds(k=25)
    mu_max = chfsi.lanczos_bounds(ref, k=60)[1]
    assert tmax <= mu_max * (1 + 1e-8)
    assert tmax + beta >= mu_max * (1 - 1e-6)


def test_repeat_bit_identical(systems):
    """Colour-ordered assembly, fixed-order reductions: repeat runs are bit-identical."""
    s, ref, op = systems["mid"]
    Xd = _to(s.trial(70))
    a = op.apply_H(Xd)
    b = op.apply_H(Xd)
    assert torch.equal(a, b)
