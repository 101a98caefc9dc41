"""The differentiation workload at its own size: the paper operator (20^3
cells, p = 6, 128 atoms x 18 projectors) with 512 states taken as the Ritz
vectors after one FP64 Rayleigh-Ritz of random columns.  The hand-written
adjoint (pawfe_band_energy_grad) gives dE/dV at all 4,096,000 quadrature
points and dE/dDelta_H for 128 x 18 x 18 entries.

Checks: central finite differences of E (through the library) at 32 seeded
quadrature points and 32 seeded Delta_H entries, at h = 1e-2 and h = 1e-5.  E
is linear in V and in Delta_H, so the difference is exact up to the rounding
of E; the bound is that rounding (n u sum |x_i (H x)_i| over all entries,
n = 64) divided by 2h, plus 1e-8 relative.  And the oracle's gradient on 24
sampled cells (dE/dV) and on every atom (dE/dDelta_H), to 1e-10 relative.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NST = 512


@pytest.fixture(scope="module")
def grad_paper():
    from paper_2604_26037_amd import Operator
    from workloads import make_system
    s = make_system("paper")
    op = Operator(s)
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(26037 + 3000)
    X = torch.randn((op.ndof, NST), generator=g, dtype=torch.float64, device=dev)
    op.rayleigh_ritz(X)                       # X <- S-orthonormal Ritz vectors
    torch.cuda.synchronize()
    E, dV, dD = op.band_energy_grad(X)
    HX = op.apply_H(X)
    absum = float((X.abs() * HX.abs()).sum())
    del HX
    print(f"[grad-paper] E = {E.item():.6f}, sum|x Hx| = {absum:.3e}", flush=True)
    return s, op, X, E.item(), dV.cpu().numpy(), dD.cpu().numpy(), absum


def _E(op, X):
    return op.band_energy_grad(X, want_dV=False, want_dH=False)[0].item()


@pytest.mark.parametrize("h", [1e-2, 1e-5])
def test_fd_veff_paper(grad_paper, h):
    s, op, X, E, dV, dD, absum = grad_paper
    u = np.finfo(np.float64).eps / 2
    floor = 64 * u * absum / (2 * h)
    rng = np.random.default_rng(26037 + 31)
    idx = rng.choice(dV.size, 32, replace=False)
    V0 = np.ascontiguousarray(s.veff_q).ravel()
    worst = 0.0
    try:
        for i in idx:
            Vp = V0.copy(); Vp[i] += h
            op.set_veff(Vp)
            Ep = _E(op, X)
            Vm = V0.copy(); Vm[i] -= h
            op.set_veff(Vm)
            Em = _E(op, X)
            fd = (Ep - Em) / (2 * h)
            g = float(dV.ravel()[i])
            worst = max(worst, abs(fd - g) / (floor + 1e-8 * abs(g)))
            assert abs(fd - g) <= floor + 1e-8 * abs(g), (i, fd, g, floor)
    finally:
        op.set_veff(V0)
    print(f"[grad-paper] V: h={h:g} worst |fd-g| / bound = {worst:.3f}", flush=True)


@pytest.mark.parametrize("h", [1e-2, 1e-5])
def test_fd_dH_paper(grad_paper, h):
    s, op, X, E, dV, dD, absum = grad_paper
    u = np.finfo(np.float64).eps / 2
    floor = 64 * u * absum / (2 * h)
    rng = np.random.default_rng(26037 + 32)
    idx = rng.choice(dD.size, 32, replace=False)
    D0 = np.ascontiguousarray(s.dH).copy()
    worst = 0.0
    try:
        for i in idx:
            Dp = D0.copy(); Dp[i] += h
            op.set_dH(Dp)
            Ep = _E(op, X)
            Dm = D0.copy(); Dm[i] -= h
            op.set_dH(Dm)
            Em = _E(op, X)
            fd = (Ep - Em) / (2 * h)
            g = float(dD[i])
            worst = max(worst, abs(fd - g) / (floor + 1e-8 * abs(g)))
            assert abs(fd - g) <= floor + 1e-8 * abs(g), (i, fd, g, floor)
    finally:
        op.set_dH(D0)
    print(f"[grad-paper] dH: h={h:g} worst |fd-g| / bound = {worst:.3f}", flush=True)


def test_grad_vs_oracle_paper(grad_paper):
    from oracle import grad
    from oracle.paw import PAWOperator
    s, op, X, E, dV, dD, absum = grad_paper
    ref = PAWOperator(s)
    Xh = X.cpu().numpy()
    cells = np.random.default_rng(26037 + 33).choice(ref.mesh.E, 24, replace=False)
    gV = grad.grad_veff(ref, Xh, cells=cells)
    got = dV.reshape(ref.mesh.E, -1)[cells]
    assert np.linalg.norm(got - gV) <= 1e-10 * np.linalg.norm(gV)
    gD = grad.grad_dH(ref, Xh)
    assert np.linalg.norm(dD - gD) <= 1e-10 * np.linalg.norm(gD)
