"""Pins of the oracle's filter and Rayleigh-Ritz.

* The scalar recurrences reproduce T_m from its closed form (cos / cosh).
* With the exact S^{-1}, Algorithm 2 and the standard ChFSI recurrence both
  equal C_m(H~) Psi computed through a dense generalized eigendecomposition
  (the equivalence stated after eq. "RChFSI final"), for any Lambda_in.
* Exact eigenpairs give a zero residual and Psi_f = Psi C_m(Lambda~).
* With the approximate Sinv_hat, Algorithm 2's error is O(eps) in the
  quality of the input, while the standard recurrence with Sinv_hat is O(1).
* Rayleigh-Ritz obeys Courant-Fischer, S-orthonormality and the residual
  bound; the Lanczos estimate brackets the top of the spectrum.
"""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import chfsi
from oracle.paw import PAWOperator
from workloads import make_system


@pytest.fixture(scope="module")
def tiny():
    op = PAWOperator(make_system("tiny"))
    H, S = op.H_dense(), op.S_dense()
    H = 0.5 * (H + H.T)
    S = 0.5 * (S + S.T)
    lam, V = sla.eigh(H, S)
    return op, H, S, lam, V


def _bounds(lam, nwanted):
    return float(lam[0]), float(lam[nwanted + 4]), float(lam[-1]) * 1.01


@pytest.mark.parametrize("m", [2, 3, 7, 20, 31])
def test_lambda_recurrence_closed_form(m):
    b0, bW, bU = -1.3, 0.4, 57.0
    lam = np.array([-1.3, -1.0, 0.0, 0.39, 0.41, 3.0, 30.0, 56.9])
    ident = lambda X: X                                   # noqa: E731
    zero = lambda X: 0 * X                                # noqa: E731
    X = np.eye(len(lam))
    # H = diag(lam), S = I, Sinv = I: residual zero, Psi_f = X diag(Lambda_Y)
    _, LY = chfsi.rchfsi_block(lambda V: lam[:, None] * V, ident, ident, X, lam, m, b0, bW, bU)
    e, c, _ = chfsi.cheb_scalars(b0, bW, bU)
    ref = chfsi.cheb_T(m, (lam - c) / e) / chfsi.cheb_T(m, np.array([(b0 - c) / e]))[0]
    np.testing.assert_allclose(LY, ref, rtol=1e-12, atol=1e-14)
    assert zero(1.0) == 0


def test_zeta_closed_form():
    b0, bW, bU = -0.7, 0.9, 12.0
    e, c, _ = chfsi.cheb_scalars(b0, bW, bU)
    a0 = (b0 - c) / e
    z = chfsi.zeta_sequence(25, b0, bW, bU)
    t = np.arange(0, 26)
    T = chfsi.cheb_T(1, np.array([a0]))  # noqa: F841
    Ts = np.array([chfsi.cheb_T(int(k), np.array([a0]))[0] for k in t])
    np.testing.assert_allclose(z, Ts[:-1] / Ts[1:], rtol=1e-13)


def test_cheb_T_closed_form_matches_recurrence():
    x = np.array([-3.0, -1.2, -1.0, -0.3, 0.0, 0.7, 1.0, 1.5, 4.0])
    T0, T1 = np.ones_like(x), x.copy()
    for m in range(2, 15):
        T0, T1 = T1, 2 * x * T1 - T0
        np.testing.assert_allclose(chfsi.cheb_T(m, x), T1, rtol=1e-12, atol=1e-12)


def test_rchfsi_exact_inverse_equals_spectral_filter(tiny):
    """Algorithm 2 with S^{-1} equals T_m(H~)Psi/T_m(a0~) for ANY Lambda_in."""
    op, H, S, lam, V = tiny
    N = 6
    b0, bW, bU = _bounds(lam, N)
    X = np.random.default_rng(0).standard_normal((op.mesh.M, N))
    lam_in = np.random.default_rng(1).uniform(b0, bU, N)         # arbitrary estimates
    Sinv = lambda Z: sla.cho_solve(sla.cho_factor(S), Z)          # noqa: E731
    m = 9
    out, _ = chfsi.rchfsi_block(lambda Z: H @ Z, lambda Z: S @ Z, Sinv, X, lam_in, m, b0, bW, bU)
    ref = chfsi.cheb_filter_spectral(H, S, X, m, b0, bW, bU, eig=(lam, V))
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-9 * np.abs(ref).max())
    std = chfsi.chfsi_filter(lambda Z: H @ Z, Sinv, X, m, b0, bW, bU)
    np.testing.assert_allclose(std, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_exact_eigenpairs(tiny):
    """Exact pairs: residual Y = 0 and Psi_f = Psi diag(C_m(lambda~)), any Sinv."""
    op, H, S, lam, V = tiny
    N = 5
    b0, bW, bU = _bounds(lam, N)
    X = V[:, :N]
    out, LY = chfsi.rchfsi_block(op.apply_H, op.apply_S, op.apply_Sinv, X, lam[:N], 12, b0, bW, bU)
    Y = op.apply_H(X) - op.apply_S(X) * lam[None, :N]
    assert np.abs(Y).max() < 1e-10
    np.testing.assert_allclose(out, X * LY[None, :], atol=1e-9 * np.abs(X).max())
    e, c, _ = chfsi.cheb_scalars(b0, bW, bU)
    ref = chfsi.cheb_T(12, (lam[:N] - c) / e) / chfsi.cheb_T(12, np.array([(b0 - c) / e]))[0]
    np.testing.assert_allclose(LY, ref, rtol=1e-11)


def test_residual_form_tolerates_inexact_inverse(tiny):
    """Error of Algorithm 2 with Sinv_hat vanishes linearly with the input
    error eps; the standard recurrence with Sinv_hat keeps an eps-independent
    error floor (it filters with the wrong operator).  This is the paper's
    argument for the residual form."""
    op, H, S, lam, V = tiny
    N = 6
    b0, bW, bU = _bounds(lam, N)
    m = 10
    noise = np.random.default_rng(5).standard_normal((op.mesh.M, N))
    err_r, err_s = [], []
    for eps in (1e-6, 1e-8):
        X = V[:, :N] + eps * noise
        ref = chfsi.cheb_filter_spectral(H, S, X, m, b0, bW, bU, eig=(lam, V))
        got, _ = chfsi.rchfsi_block(op.apply_H, op.apply_S, op.apply_Sinv, X, lam[:N], m,
                                    b0, bW, bU)
        std = chfsi.chfsi_filter(op.apply_H, op.apply_Sinv, X, m, b0, bW, bU)
        err_r.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        err_s.append(np.linalg.norm(std - ref) / np.linalg.norm(ref))
    assert 30 < err_r[0] / err_r[1] < 300               # linear in eps
    assert 0.5 < err_s[0] / err_s[1] < 2.0              # floor, independent of eps
    assert err_s[1] > 100 * err_r[1]


def test_block_invariance(tiny):
    op, H, S, lam, V = tiny
    N = 10
    b0, bW, bU = _bounds(lam, N)
    X = np.random.default_rng(7).standard_normal((op.mesh.M, N))
    lam_in = lam[:N] + 0.01
    a = chfsi.rchfsi_filter(op, X, lam_in, 6, b0, bW, bU, block=N)
    b = chfsi.rchfsi_filter(op, X, lam_in, 6, b0, bW, bU, block=3)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * np.abs(a).max())


def test_rayleigh_ritz_properties(tiny):
    op, H, S, lam, V = tiny
    N = 8
    rng = np.random.default_rng(11)
    X = V[:, :N] + 0.05 * rng.standard_normal((op.mesh.M, N))
    Psi, theta, res = chfsi.rayleigh_ritz(op, X)
    # S-orthonormal Ritz vectors
    np.testing.assert_allclose(Psi.T @ (S @ Psi), np.eye(N), atol=1e-11)
    # Courant-Fischer: Ritz values bound the eigenvalues from above
    assert np.all(theta >= lam[:N] - 1e-12)
    # residual bound: some eigenvalue within ||S^{-1/2} r|| of each Ritz value
    Lc = np.linalg.cholesky(S)
    R = H @ Psi - (S @ Psi) * theta[None, :]
    np.testing.assert_allclose(np.linalg.norm(R, axis=0), res, rtol=1e-10)
    bnd = np.linalg.norm(sla.solve_triangular(Lc, R, lower=True), axis=0)
    for i in range(N):
        assert np.min(np.abs(lam - theta[i])) <= bnd[i] * (1 + 1e-10) + 1e-14
    # a subspace containing exact eigenvectors returns their eigenvalues
    _, th2, res2 = chfsi.rayleigh_ritz(op, V[:, :N] @ rng.standard_normal((N, N)))
    np.testing.assert_allclose(th2, lam[:N], atol=1e-11)
    assert res2.max() < 1e-9


def test_lanczos_brackets_top_of_spectrum(tiny):
    op, H, S, lam, V = tiny
    Sinv = op.Sinv_dense()
    mu = np.sort(np.linalg.eigvals(H @ Sinv).real)
    tmin, tmax, beta = chfsi.lanczos_bounds(op, k=20)
    assert tmax <= mu[-1] * (1 + 1e-10)
    assert tmax + abs(beta) >= mu[-1]
    assert tmin >= mu[0] - 1e-10


def test_chfsi_iterations_converge(tiny):
    """Three filter + RR iterations from random vectors approach the dense eigenvalues."""
    op, H, S, lam, V = tiny
    s = op.system
    X = s.trial()
    bU = float(lam[-1]) * 1.01
    Psi, th, hist = chfsi.chfsi_iterations(op, X, s.iterations, s.cheb_degree, bU)
    errs = [np.abs(h[0][:12] - lam[:12]).max() for h in hist]
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:]))     # monotone, fast
    assert np.all(th >= lam[:len(th)] - 1e-12)
    assert errs[-1] < 0.05


def test_chfsi_solve_residual_bound(tiny):
    """The convergence loop stops at the first Rayleigh-Ritz whose wanted
    residuals are <= tol, and each converged Ritz value then lies within the
    residual bound of the dense eigenvalue of the same index:
    |theta_i - lambda_i| <= ||r_i||_2 / sqrt(lambda_min(S)) (S-orthonormal
    Ritz vectors, residual measured in the S^{-1} norm)."""
    op, H, S, lam, V = tiny
    s = op.system
    X = s.trial()
    bU = float(lam[-1]) * 1.01
    nw, tol = 8, 2e-3
    Psi, th, res, it = chfsi.chfsi_solve(op, X, s.cheb_degree, bU, tol, 30, nwanted=nw)
    assert 1 <= it < 30
    assert np.max(res[:nw]) <= tol
    smin = float(np.linalg.eigvalsh(0.5 * (S + S.conj().T))[0])
    assert np.all(np.abs(th[:nw] - lam[:nw]) <= res[:nw] / np.sqrt(smin) * (1 + 1e-9))
    # one pass fewer does not meet the tolerance
    _, th1, res1, it1 = chfsi.chfsi_solve(op, X, s.cheb_degree, bU, tol, it - 1, nwanted=nw)
    assert it1 == it - 1 and np.max(res1[:nw]) > tol


def test_mixed_rotation_pins(tiny):
    """Mixed-precision subspace rotation: exact for a diagonal Q; otherwise
    within the FP32 rounding bound of the off-diagonal product, elementwise
    |Psi_mixed - X Q| <= 2 (N + 2) u32 |X| |Q_off| (u32 = 2^-24); the Ritz
    values do not depend on it."""
    op, H, S, lam, V = tiny
    s = op.system
    rng = np.random.Generator(np.random.PCG64(11))
    X = s.trial()
    N = X.shape[1]
    Dq = np.diag(rng.uniform(0.5, 2.0, N))
    np.testing.assert_array_equal(chfsi.mixed_rotation(X, Dq), X * np.diag(Dq)[None, :])
    Q = Dq + 1e-2 * rng.standard_normal((N, N))
    Qoff = Q - np.diag(np.diag(Q))
    err = np.abs(chfsi.mixed_rotation(X, Q) - X @ Q)
    bound = 2 * (N + 2) * 2.0 ** -24 * (np.abs(X) @ np.abs(Qoff))
    assert np.all(err <= bound + 1e-300)
    assert err.max() > 0                                   # FP32 did round
    P1, l1, r1 = chfsi.rayleigh_ritz(op, X)
    P2, l2, r2 = chfsi.rayleigh_ritz(op, X, mixed_sr=True)
    np.testing.assert_array_equal(l1, l2)
    assert np.abs(P2 - P1).max() <= 1e-5 * np.abs(P1).max()
    np.testing.assert_allclose(r2, r1, rtol=1e-3, atol=1e-5 * np.abs(r1).max())
