"""Chebyshev filtering and Rayleigh-Ritz in the oracle (TEST INFRASTRUCTURE).

* ``rchfsi_filter`` takes Algorithm 2 (residual-based Chebyshev filtered
  subspace) step by step, blockwise over the columns, with the same
  polynomial (e, c, zeta) for every block.
* ``chfsi_filter`` is the standard scaled three-term recurrence of eq.
  "ChFSI recurrance2" (X_{theta+1} from S^{-1}H X_theta), with any inverse.
* ``cheb_T`` evaluates T_m from its closed form (cos / cosh), used to pin the
  recurrences.
* ``rayleigh_ritz`` is Algorithm 1 steps 4-6: H^p = X^H H X, S^p = X^H S X,
  the projected generalized eigenproblem, and the rotation X Q, followed by
  the residual norms ||H psi_i - lambda_i S psi_i||_2 of the residual check.
* ``lanczos_bounds`` is a k-step Lanczos on H Sinv_hat in the Sinv_hat inner
  product, giving the upper bound b_U = theta_max + |beta_k|.
* ``chfsi_solve`` repeats filter + Rayleigh-Ritz until the wanted residual
  norms meet a tolerance (the residual check of Algorithm 1).
* ``mixed_rotation`` is the mixed-precision subspace rotation of the
  Rayleigh-Ritz subsection (FP64 diagonal of Q, FP32 off-diagonal product).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def cheb_scalars(b0, bW, bU):
    """Step 1 of Algorithm 2: e, c and zeta_1."""
    e = (bU - bW) / 2.0
    c = (bU + bW) / 2.0
    zeta1 = e / (b0 - c)
    return e, c, zeta1


def cheb_T(m, x):
    """T_m(x) from its closed form: cos(m arccos x) on [-1,1], cosh outside."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inner = np.abs(x) <= 1.0
    out[inner] = np.cos(m * np.arccos(x[inner]))
    hi = x > 1.0
    out[hi] = np.cosh(m * np.arccosh(x[hi]))
    lo = x < -1.0
    out[lo] = (-1.0) ** m * np.cosh(m * np.arccosh(-x[lo]))
    return out


def zeta_sequence(m, b0, bW, bU):
    """zeta_1..zeta_m by the recurrence zeta_{t+1} = 1/(2/zeta_1 - zeta_t)."""
    e, c, z1 = cheb_scalars(b0, bW, bU)
    z = [z1]
    for _ in range(2, m + 1):
        z.append(1.0 / (2.0 / z1 - z[-1]))
    return np.array(z)


def rchfsi_block(apply_H, apply_S, apply_Sinv, X, lam, m, b0, bW, bU):
    """Algorithm 2 on one block of columns.  Returns (Psi_f, Lambda_Y)."""
    if m < 2:
        raise ValueError("Chebyshev degree must be >= 2")
    lam = np.asarray(lam, dtype=np.float64)
    # step 1
    e = (bU - bW) / 2.0
    c = (bU + bW) / 2.0
    zeta = e / (b0 - c)
    zeta1 = zeta
    gamma = 2.0 / zeta1
    # step 2: residual of the input pairs
    Y = apply_H(X) - apply_S(X) * lam[None, :]
    # step 3
    RX = np.zeros_like(Y)
    RY = (zeta1 / e) * Y
    LX = np.ones_like(lam)
    LY = (zeta1 / e) * (lam - c)
    # step 4
    for _theta in range(2, m + 1):
        znew = 1.0 / (gamma - zeta)
        a = 2.0 * znew / e
        RX = (a * apply_H(apply_Sinv(RY)) - a * c * RY - zeta * znew * RX
              + a * Y * LY[None, :])
        LX = a * LY * lam - a * c * LY - zeta * znew * LX
        RX, RY = RY, RX
        LX, LY = LY, LX
        zeta = znew
    # step 5
    return apply_Sinv(RY) + X * LY[None, :], LY


def rchfsi_filter(op, X, lam, m, b0, bW, bU, block=None, apply_Sinv=None):
    """Algorithm 2 applied blockwise (uncoupled blocks, one polynomial)."""
    N = X.shape[1]
    B = N if block is None else int(block)
    sinv = op.apply_Sinv if apply_Sinv is None else apply_Sinv
    out = np.empty_like(X)
    for j0 in range(0, N, B):
        j1 = min(N, j0 + B)
        out[:, j0:j1], _ = rchfsi_block(op.apply_H, op.apply_S, sinv, X[:, j0:j1],
                                        lam[j0:j1], m, b0, bW, bU)
    return out


def chfsi_filter(apply_H, apply_Sinv, X, m, b0, bW, bU):
    """Standard scaled ChFSI (eq. ChFSI recurrance2): C_m(H_tilde) X."""
    e, c, zeta1 = cheb_scalars(b0, bW, bU)
    A = lambda V: apply_Sinv(apply_H(V))                     # noqa: E731
    X0 = X
    X1 = (zeta1 / e) * (A(X) - c * X)
    zeta = zeta1
    for _theta in range(1, m):
        znew = 1.0 / (2.0 / zeta1 - zeta)
        X2 = (2.0 * znew / e) * A(X1) - (2.0 * znew * c / e) * X1 - zeta * znew * X0
        X0, X1 = X1, X2
        zeta = znew
    return X1


def cheb_filter_spectral(H, S, X, m, b0, bW, bU, eig=None):
    """C_m(H_tilde) X through the dense generalized eigendecomposition of (H, S).

    S^{-1} H = V diag(lambda) V^H S with V^H S V = I, hence
    C_m(H_tilde) X = V diag(T_m(l~)/T_m(a~0)) V^H S X, T_m by its closed form.
    """
    e, c, _ = cheb_scalars(b0, bW, bU)
    lam, V = eig if eig is not None else sla.eigh(0.5 * (H + H.conj().T), 0.5 * (S + S.conj().T))
    f = cheb_T(m, (lam - c) / e) / cheb_T(m, np.array([(b0 - c) / e]))[0]
    return V @ (f[:, None] * (V.conj().T @ (S @ X)))


def rayleigh_ritz(op, X, mixed_sr=False):
    """Algorithm 1 steps 4-6 plus the residual norms (FP64).

    Returns (Psi, lambda ascending, resnorm) with Psi^H S Psi = I.
    mixed_sr: the subspace rotation in mixed precision (the paper's RR-SR
    strategy): Psi = X diag(Q) in FP64 plus X Q_off with Q_off = Q with a
    zero diagonal, X and Q_off rounded to FP32 and the product formed in
    FP32; the residual norms are then those of the rotated Psi.
    """
    HX = op.apply_H(X)
    SX = op.apply_S(X)
    Hp = X.conj().T @ HX
    Sp = X.conj().T @ SX
    Hp = 0.5 * (Hp + Hp.conj().T)
    Sp = 0.5 * (Sp + Sp.conj().T)
    lam, Q = sla.eigh(Hp, Sp)
    if not mixed_sr:
        Psi = X @ Q
        R = HX @ Q - (SX @ Q) * lam[None, :]
        return Psi, lam, np.linalg.norm(R, axis=0)
    Psi = mixed_rotation(X, Q)
    return Psi, lam, residual_norms(op, Psi, lam)


def mixed_rotation(X, Q):
    """X Q as X diag(Q) (FP64) + fl32(fl32(X) fl32(Q_off)), Q_off = Q - diag(Q)."""
    d = np.diag(Q)
    Qoff = Q - np.diag(d)
    out = np.result_type(X.dtype, Q.dtype)
    f32 = np.complex64 if np.iscomplexobj(np.zeros(0, out)) else np.float32
    off = (X.astype(f32) @ Qoff.astype(f32)).astype(out)
    return X * d[None, :] + off


def residual_norms(op, Psi, lam):
    """||H psi_i - lambda_i S psi_i||_2 per column."""
    R = op.apply_H(Psi) - op.apply_S(Psi) * np.asarray(lam)[None, :]
    return np.linalg.norm(R, axis=0)


def lanczos_bounds(op, k=20, seed=1234):
    """k-step Lanczos on A = H Sinv_hat, self-adjoint in <x, y> = x^H Sinv_hat y.

    Returns (theta_min, theta_max, beta_k); b_U = theta_max + |beta_k|.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(op.mesh.M).astype(op.dtype)
    z = op.apply_Sinv(v)
    nrm = np.sqrt(np.real(np.vdot(v, z)))
    v, z = v / nrm, z / nrm
    v_prev = np.zeros_like(v)
    beta_prev = 0.0
    alphas, betas = [], []
    for _ in range(k):
        w = op.apply_H(z)
        alpha = np.real(np.vdot(z, w))
        w = w - alpha * v - beta_prev * v_prev
        u = op.apply_Sinv(w)
        beta = np.sqrt(max(np.real(np.vdot(w, u)), 0.0))
        alphas.append(alpha)
        betas.append(beta)
        if beta == 0.0:
            break
        v_prev, v, z = v, w / beta, u / beta
        beta_prev = beta
    T = np.diag(alphas) + np.diag(betas[:-1], 1) + np.diag(betas[:-1], -1)
    th = np.linalg.eigvalsh(T)
    return float(th[0]), float(th[-1]), float(betas[-1])


def chfsi_iterations(op, X, niter, m, bU, block=None, apply_Sinv=None, filt=None):
    """Algorithm 1 with explicit b_U: RR of the start, then niter x (filter + RR).

    b_0 and b_W are the lowest and highest current Ritz values.  Returns the
    list of (lambda, resnorm) after each RR (the first entry is the start).
    """
    Psi, lam, res = rayleigh_ritz(op, X)
    hist = [(lam, res)]
    for _ in range(niter):
        b0, bW = float(lam[0]), float(lam[-1])
        if filt is None:
            Xf = rchfsi_filter(op, Psi, lam, m, b0, bW, bU, block=block, apply_Sinv=apply_Sinv)
        else:
            Xf = filt(Psi, lam, m, b0, bW, bU)
        Psi, lam, res = rayleigh_ritz(op, Xf)
        hist.append((lam, res))
    return Psi, lam, hist


def chfsi_solve(op, X, m, bU, tol, max_iter, nwanted=None, block=None):
    """Algorithm 1 run to convergence: Rayleigh-Ritz of the start, then
    filter + Rayleigh-Ritz until the residual norms of the lowest nwanted
    Ritz pairs (all when None) are <= tol, or max_iter filter passes have
    run (the convergence test on the residual norms of the algorithm's
    last step).  b_0 and b_W are the lowest and highest current Ritz values,
    b_U is given.  Returns (Psi, lambda, resnorm, iterations)."""
    Psi, lam, res = rayleigh_ritz(op, X)
    nw = len(lam) if nwanted is None else int(nwanted)
    it = 0
    while np.max(res[:nw]) > tol and it < max_iter:
        b0, bW = float(lam[0]), float(lam[-1])
        Xf = rchfsi_filter(op, Psi, lam, m, b0, bW, bU, block=block)
        Psi, lam, res = rayleigh_ritz(op, Xf)
        it += 1
    return Psi, lam, res, it
