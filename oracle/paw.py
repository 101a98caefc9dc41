"""PAW layer of the oracle (TEST INFRASTRUCTURE, plain FP64).

Follows eq. "FE nonlocal contribution" (H_nloc = sum_a C^a Delta_H^a C^a^H,
S_nloc = sum_a C^a Delta_S^a C^a^H), eq. "FEM Cmatrix" for the projector
matrix C^a (cell quadrature, sum over periodic images, Bloch phase
exp(-i k.(x - L_r))), eqs. "Sinvapprox" / "Delta Sinv" for the approximate
inverse overlap Sinv_hat, and the cheaper <p|p> variant described right after
them.

Synthetic projector channels (the paper's come from PAW datasets, which are
not available):  p_{l m sigma}(d) = S_lm(d) exp(-|d|^2 / (2 sigma^2))
(1 - |d|^2/r_c^2)^2 for |d| < r_c, else 0, with S_lm the unnormalized real
solid harmonics 1 | y, z, x | xy, yz, 3z^2 - r^2, xz, x^2 - y^2.

Support of atom a: the cells having at least one Gauss point strictly inside
r_c of some periodic image of R^a.  The oracle finds these by enumerating
every (cell, image) pair whose box can reach the sphere and testing each
quadrature point, so it needs no minimum-image shortcut.

Delta_Sinv^a is evaluated as Delta_S^a (I + G^a Delta_S^a)^{-1}, which equals
(Delta_S^{a,-1} + G^a)^{-1} whenever Delta_S^a is invertible and needs no
inverse of Delta_S.  G^a = C^a^H M_D^{-1} C^a ("exact_g") or the projector
overlap <p_alpha|p_beta> by Gauss quadrature ("pp").
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .fe import Mesh, CellQuadrature, LocalOperator, lumped_mass


def solid_harmonic(l, m, d):
    """Unnormalized real solid harmonic S_lm at displacements d[..., 3]."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    if l == 0:
        return np.ones_like(x)
    if l == 1:
        return {-1: y, 0: z, 1: x}[m]
    if l == 2:
        r2 = x * x + y * y + z * z
        return {-2: x * y, -1: y * z, 0: 3.0 * z * z - r2, 1: x * z, 2: x * x - y * y}[m]
    raise ValueError("l > 2 not supported")


def projector_value(l, m, sigma, rc, d):
    """p(d) = S_lm(d) exp(-|d|^2/(2 sigma^2)) (1 - |d|^2/r_c^2)^2 inside r_c, 0 outside."""
    r2 = (d * d).sum(axis=-1)
    inside = r2 < rc * rc
    g = np.exp(-r2 / (2.0 * sigma * sigma)) * (1.0 - r2 / (rc * rc)) ** 2
    return np.where(inside, solid_harmonic(l, m, d) * g, 0.0)


def _axis_images(bounds, L, lo, hi):
    """(cell i, shift s) along one axis whose interval [b_i, b_{i+1}] + s L
    meets [lo, hi]."""
    out = []
    for s in range(int(np.floor(lo / L)) - 1, int(np.floor(hi / L)) + 2):
        for i in range(len(bounds) - 1):
            if bounds[i] + s * L <= hi and bounds[i + 1] + s * L >= lo:
                out.append((i, s))
    return out


def cell_image_pairs(mesh: Mesh, R, rc):
    """All (cell e, image shift vector s*L) whose cell box can reach the sphere.

    Uniform mesh: unwrapped cell index iu in [floor((R-rc)/h), floor((R+rc)/h)]
    per axis; the actual cell is iu mod n and the point x of that cell sits at
    x + s*L with s = floor(iu / n) in the unwrapped frame.  Graded mesh: per
    axis every (cell, shift) whose shifted interval meets [R-rc, R+rc].
    """
    R = np.asarray(R, dtype=np.float64)
    nx, ny, nz = mesh.ncell
    out = []
    if mesh.graded:
        ax = [_axis_images(mesh.bounds[d], mesh.box[d], R[d] - rc, R[d] + rc) for d in range(3)]
        for k, sk in ax[2]:
            for j, sj in ax[1]:
                for i, si in ax[0]:
                    out.append((i + nx * (j + ny * k), np.array([si, sj, sk]) * mesh.box))
        return out
    lo = np.floor((R - rc) / mesh.h).astype(int)
    hi = np.floor((R + rc) / mesh.h).astype(int)
    for ku in range(lo[2], hi[2] + 1):
        for ju in range(lo[1], hi[1] + 1):
            for iu in range(lo[0], hi[0] + 1):
                i, j, k = iu % nx, ju % ny, ku % nz
                shift = np.array([(iu - i) // nx, (ju - j) // ny, (ku - k) // nz]) * mesh.box
                out.append((i + nx * (j + ny * k), shift))
    return out


class PAWOperator:
    """H = H_loc + sum_a C^a Dh^a C^a^H,  S = M + sum_a C^a Ds^a C^a^H, Sinv_hat."""

    def __init__(self, system, sinv_mode="exact_g"):
        s = system
        self.system = s
        self.mesh = Mesh(s.ncell, s.box, s.degree, getattr(s, "xgrid", None))
        k = np.asarray(s.kpoint, dtype=np.float64)
        self.kpoint = k if np.any(k) else None
        self.complex = bool(s.is_complex) or self.kpoint is not None
        self.dtype = np.complex128 if self.complex else np.float64
        self.loc = LocalOperator(self.mesh, s.nq, s.veff_q, self.kpoint, getattr(s, "vgga_q", None))
        self.cq = self.loc.cq
        self.MD = lumped_mass(self.mesh)
        self.MDinv = 1.0 / self.MD
        self.natoms = len(s.pos)
        self.nproj = [int(n) for n in s.nproj]
        self.poff = np.concatenate([[0], np.cumsum(self.nproj)]).astype(int)
        self.dH = s.dH_blocks()
        self.dS = s.dS_blocks()
        self.cell_dofs = self.loc.cell_dofs
        self._build_projectors()
        self.sinv_mode = sinv_mode
        self._build_sinv()

    # -- eq. FEM Cmatrix ------------------------------------------------------
    def _build_projectors(self):
        s, mesh = self.system, self.mesh
        rows, cols, vals = [], [], []
        self.supp_cells, self.supp_nodes = [], []
        self.Gpp = []
        for a in range(self.natoms):
            R, rc = s.pos[a], float(s.rcut[a])
            p0, npj = self.poff[a], self.nproj[a]
            chans = [(int(s.proj_l[p0 + t]), int(s.proj_m[p0 + t]), float(s.proj_sigma[p0 + t]))
                     for t in range(npj)]
            Cloc = {}     # cell -> (nloc, npj) contribution
            Gpp = np.zeros((npj, npj))
            for e, shift in cell_image_pairs(mesh, R, rc):
                cq = self.loc.cell_cq(e)
                xq = cq.points(mesh, e) + shift            # unwrapped positions
                d = xq - R
                if not np.any((d * d).sum(axis=1) < rc * rc):
                    continue
                P = np.stack([projector_value(l, m, sg, rc, d) for (l, m, sg) in chans], axis=1)
                if self.complex:
                    ph = np.exp(-1j * (xq @ (self.kpoint if self.kpoint is not None else np.zeros(3))))
                    Pw = P * ph[:, None]
                else:
                    Pw = P
                contrib = cq.N.T @ (cq.W[:, None] * Pw)    # (nloc, npj)
                Cloc[e] = Cloc.get(e, 0) + contrib
                Gpp += P.T @ (cq.W[:, None] * P)
            cells = np.array(sorted(Cloc), dtype=np.int64)
            self.supp_cells.append(cells)
            self.supp_nodes.append(np.unique(self.cell_dofs[cells].ravel()).astype(np.int64))
            self.Gpp.append(Gpp)
            for e in cells:
                cd = self.cell_dofs[e]
                for t in range(npj):
                    rows.append(cd)
                    cols.append(np.full(len(cd), p0 + t))
                    vals.append(Cloc[e][:, t])
        ntot = int(self.poff[-1])
        if ntot:
            C = sp.csr_matrix((np.concatenate(vals).astype(self.dtype),
                               (np.concatenate(rows), np.concatenate(cols))),
                              shape=(self.mesh.M, ntot))
        else:
            C = sp.csr_matrix((self.mesh.M, 0), dtype=self.dtype)
        C.sum_duplicates()
        self.C = C
        self.CH = C.conj().T.tocsr()

    def C_atom(self, a):
        """Dense rows of C^a on atom a's support nodes, shape (n_supp, npj)."""
        p0, p1 = self.poff[a], self.poff[a + 1]
        return self.C[self.supp_nodes[a]][:, p0:p1].toarray()

    def _blockdiag(self, blocks):
        if not blocks:
            return sp.csr_matrix((0, 0))
        return sp.block_diag(blocks, format="csr")

    # -- eqs. Sinvapprox / Delta Sinv ----------------------------------------
    def _build_sinv(self):
        self.G = []
        self.dSinv = []
        for a in range(self.natoms):
            if self.sinv_mode == "exact_g":
                Ca = self.C_atom(a)
                Ga = Ca.conj().T @ (self.MDinv[self.supp_nodes[a]][:, None] * Ca)
            elif self.sinv_mode == "pp":
                Ga = self.Gpp[a]
            else:
                raise ValueError(self.sinv_mode)
            self.G.append(Ga)
            n = self.nproj[a]
            self.dSinv.append(self.dS[a] @ np.linalg.inv(np.eye(n) + Ga @ self.dS[a]))
        self.DH = self._blockdiag(self.dH)
        self.DS = self._blockdiag(self.dS)
        self.DSinv = self._blockdiag(self.dSinv)

    # -- operator applies -----------------------------------------------------
    def _nl(self, D, X):
        if self.C.shape[1] == 0:
            return np.zeros_like(X)
        return self.C @ (D @ (self.CH @ X))

    def _as2d(self, X):
        return X if X.ndim == 2 else X[:, None]

    def apply_H(self, X):
        """H X = H_loc X + sum_a C^a Dh^a C^a^H X."""
        X2 = self._as2d(X)
        Y = self.loc.apply_H(X2) + self._nl(self.DH, X2)
        return Y if X.ndim == 2 else Y[:, 0]

    def apply_S(self, X):
        """S X = M X + sum_a C^a Ds^a C^a^H X."""
        X2 = self._as2d(X)
        Y = self.loc.apply_M(X2) + self._nl(self.DS, X2)
        return Y if X.ndim == 2 else Y[:, 0]

    def apply_Sinv(self, X):
        """Sinv_hat X = M_D^{-1} X - sum_a M_D^{-1} C^a Dsinv^a C^a^H M_D^{-1} X."""
        X2 = self._as2d(X)
        Z = self.MDinv[:, None] * X2
        Y = Z - self.MDinv[:, None] * self._nl(self.DSinv, Z)
        return Y if X.ndim == 2 else Y[:, 0]

    # -- dense / sparse matrices (small meshes) -------------------------------
    def H_sparse(self):
        return (self.loc.assemble_H() + self.C @ self.DH @ self.CH).tocsr()

    def S_sparse(self):
        return (self.loc.assemble_M() + self.C @ self.DS @ self.CH).tocsr()

    def H_dense(self):
        return self.H_sparse().toarray()

    def S_dense(self):
        return self.S_sparse().toarray()

    def Sinv_dense(self):
        return self.apply_Sinv(np.eye(self.mesh.M, dtype=self.dtype))

    def dense_eigs(self, nev=None):
        """All (or the lowest nev) eigenpairs of H x = lambda S x, dense."""
        H, S = self.H_dense(), self.S_dense()
        H = 0.5 * (H + H.conj().T)
        S = 0.5 * (S + S.conj().T)
        if nev is None:
            return sla.eigh(H, S)
        return sla.eigh(H, S, subset_by_index=[0, nev - 1])

    # -- integer outputs ------------------------------------------------------
    def support_lists(self):
        """(cell offsets, cells, node offsets, nodes), atom after atom, sorted."""
        co = np.concatenate([[0], np.cumsum([len(c) for c in self.supp_cells])]).astype(np.int64)
        no = np.concatenate([[0], np.cumsum([len(n) for n in self.supp_nodes])]).astype(np.int64)
        cells = np.concatenate(self.supp_cells) if self.supp_cells else np.zeros(0, np.int64)
        nodes = np.concatenate(self.supp_nodes) if self.supp_nodes else np.zeros(0, np.int64)
        return co, cells, no, nodes
