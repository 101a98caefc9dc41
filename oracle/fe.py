"""Finite-element layer of the oracle (TEST INFRASTRUCTURE, plain FP64).

Follows the paper's FE discretization section: C^0 Lagrange basis of degree p
on Gauss-Lobatto-Legendre (GLL) nodes, tensor product n_p^3 = (p+1)^3 per
hexahedral cell; cell integrals by Gauss-Legendre quadrature with the affine
Jacobian (eq. "Quadrature Integration"); cell Hamiltonian and overlap entries
(eq. "FEM Ham entries", with the GGA term when a V_GGA field is given;
eq. "FEM S_loc entries"); GLL-lumped diagonal mass M_D used inside the
approximate inverse overlap (approximation (i) after eq. "Delta Sinv").

Meshes are periodic tensor products of axis-aligned cells: uniform, or
graded with per-axis cell boundaries (the two-level meshes of the figure
"Finite-element meshes employed in PAW-FE", read as fine cells along the
atoms' coordinates and cells of twice the size elsewhere, so every cell is
a box with its own diagonal Jacobian and no hanging nodes arise).

Everything is computed from its definition: basis values by the Lagrange
product formula, element matrices by summing over all 3-D quadrature points
(no sum factorization), global matrices by scipy.sparse assembly.

Conventions (not fixed by the paper; chosen here):
  cell e = i + nx*(j + ny*k), origin (i*hx, j*hy, k*hz) (uniform) or
    (bx[i], by[j], bz[k]) with the per-axis boundaries b (graded)
  local node l = a + np*(b + np*c), (a, b, c) in [0, p]^3, a along x
  periodic DOF I = gx + Gx*(gy + Gy*gz), gx = (i*p + a) mod (nx*p)
  quadrature point q = qx + nq*(qy + nq*qz)
  1-D colour col(i, n) = 2 if (n odd and i == n-1) else i mod 2;
  cell colour = col_x + cx*(col_y + cy*col_z), c_d = 2 (n_d even) or 3
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import legendre as npleg


# ---------------------------------------------------------------------------
# Reference element (FE discretization section: GLL nodal points)
# ---------------------------------------------------------------------------

def gll_nodes_weights(p):
    """GLL nodes and weights on [-1, 1] for degree p (p+1 points).

    Nodes: -1, the roots of P_p'(x), +1.  Weights 2 / (p (p+1) P_p(x_a)^2).
    """
    Pp = npleg.Legendre.basis(p)
    inner = np.sort(np.real(Pp.deriv().roots())) if p > 1 else np.zeros(0)
    x = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (p * (p + 1) * Pp(x) ** 2)
    return x, w


def gauss_nodes_weights(n):
    """n-point Gauss-Legendre rule on [-1, 1] (eq. Quadrature Integration)."""
    x, w = npleg.leggauss(n)
    return x, w


def lagrange_values(nodes, x):
    """L[q, a] = l_a(x_q), the Lagrange polynomial through ``nodes``, by the product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    L = np.ones((len(x), n))
    for a in range(n):
        for j in range(n):
            if j != a:
                L[:, a] *= (x - nodes[j]) / (nodes[a] - nodes[j])
    return L


def lagrange_derivs(nodes, x):
    """D[q, a] = l_a'(x_q): derivative of the product formula by the product rule."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    D = np.zeros((len(x), n))
    for a in range(n):
        for m in range(n):
            if m == a:
                continue
            term = np.full(len(x), 1.0 / (nodes[a] - nodes[m]))
            for j in range(n):
                if j != a and j != m:
                    term *= (x - nodes[j]) / (nodes[a] - nodes[j])
            D[:, a] += term
    return D


# ---------------------------------------------------------------------------
# Mesh, DOF map and colouring
# ---------------------------------------------------------------------------

class Mesh:
    """Periodic orthorhombic hexahedral mesh with degree-p spectral elements.

    ``xgrid`` (optional): three arrays of cell boundaries, n_d + 1 each,
    strictly increasing from 0 to box[d]; without it the cells are uniform
    (h = box / ncell).
    """

    def __init__(self, ncell, box, degree, xgrid=None):
        self.ncell = tuple(int(n) for n in ncell)
        if min(self.ncell) < 2:
            raise ValueError("each direction needs at least 2 cells (periodic)")
        self.box = np.asarray(box, dtype=np.float64)
        self.p = int(degree)
        self.np1 = self.p + 1
        self.h = self.box / np.asarray(self.ncell)
        self.E = int(np.prod(self.ncell))
        self.G = tuple(n * self.p for n in self.ncell)
        self.M = int(np.prod(self.G))
        self.xi, self.rho = gll_nodes_weights(self.p)
        self.graded = xgrid is not None
        if self.graded:
            self.bounds = [np.asarray(xgrid[d], dtype=np.float64) for d in range(3)]
            for d in range(3):
                b = self.bounds[d]
                if (b.shape != (self.ncell[d] + 1,) or b[0] != 0.0 or b[-1] != self.box[d]
                        or np.any(np.diff(b) <= 0.0)):
                    raise ValueError("xgrid[d] must rise strictly from 0 to box[d] in ncell[d] steps")
        else:
            self.bounds = [np.arange(self.ncell[d] + 1) * self.h[d] for d in range(3)]

    def cell_ijk(self, e):
        nx, ny, _ = self.ncell
        return e % nx, (e // nx) % ny, e // (nx * ny)

    def cell_h(self, e):
        """Edge lengths (hx, hy, hz) of cell e."""
        if not self.graded:
            return self.h.copy()
        i, j, k = self.cell_ijk(e)
        b = self.bounds
        return np.array([b[0][i + 1] - b[0][i], b[1][j + 1] - b[1][j], b[2][k + 1] - b[2][k]])

    def cell_origin(self, e):
        i, j, k = self.cell_ijk(e)
        return np.array([self.bounds[0][i], self.bounds[1][j], self.bounds[2][k]])

    def local_abc(self):
        n = self.np1
        l = np.arange(n ** 3)
        return l % n, (l // n) % n, l // (n * n)

    def cell_dofs(self):
        """cell_dofs[e, l] (int32) per the periodic lexicographic rule."""
        nx, ny, nz = self.ncell
        Gx, Gy, Gz = self.G
        p = self.p
        a, b, c = self.local_abc()
        out = np.empty((self.E, self.np1 ** 3), dtype=np.int64)
        for e in range(self.E):
            i, j, k = self.cell_ijk(e)
            gx = (i * p + a) % Gx
            gy = (j * p + b) % Gy
            gz = (k * p + c) % Gz
            out[e] = gx + Gx * (gy + Gy * gz)
        return out.astype(np.int32)

    def node_coords(self):
        """Physical coordinates (E, n_p^3, 3) of every cell-local node (unwrapped)."""
        a, b, c = self.local_abc()
        out = np.empty((self.E, self.np1 ** 3, 3))
        for e in range(self.E):
            i, j, k = self.cell_ijk(e)
            if not self.graded:
                out[e, :, 0] = (i + 0.5 * (self.xi[a] + 1.0)) * self.h[0]
                out[e, :, 1] = (j + 0.5 * (self.xi[b] + 1.0)) * self.h[1]
                out[e, :, 2] = (k + 0.5 * (self.xi[c] + 1.0)) * self.h[2]
            else:
                o, h = self.cell_origin(e), self.cell_h(e)
                for d, t in enumerate((a, b, c)):
                    out[e, :, d] = o[d] + 0.5 * (self.xi[t] + 1.0) * h[d]
        return out

    @staticmethod
    def _colour1d(i, n):
        return 2 if (n % 2 == 1 and i == n - 1) else i % 2

    def cell_colour(self):
        nx, ny, nz = self.ncell
        cx = 2 if nx % 2 == 0 else 3
        cy = 2 if ny % 2 == 0 else 3
        out = np.empty(self.E, dtype=np.int32)
        for e in range(self.E):
            i, j, k = self.cell_ijk(e)
            out[e] = (self._colour1d(i, nx) + cx * (self._colour1d(j, ny)
                      + cy * self._colour1d(k, nz)))
        return out

    def ncolours(self):
        return int(np.prod([2 if n % 2 == 0 else 3 for n in self.ncell]))

    def scatter_matrix(self):
        """P^T as a sparse (M, E*n_p^3) 0/1 matrix: global = P^T @ cellwise."""
        cd = self.cell_dofs().ravel().astype(np.int64)
        n = cd.size
        return sp.csr_matrix((np.ones(n), (cd, np.arange(n))), shape=(self.M, n))


# ---------------------------------------------------------------------------
# Quadrature data of one (affine, axis-aligned) cell
# ---------------------------------------------------------------------------

class CellQuadrature:
    """Basis values and gradients at the n_q^3 Gauss points of a cell of size h.

    N[q, l] = l_a(eta_qx) l_b(eta_qy) l_c(eta_qz);
    dN[d, q, l] = physical derivative along d (J^{-1} = diag(2/h));
    W[q] = w_qx w_qy w_qz det J, det J = hx hy hz / 8.
    h defaults to the uniform cell size of the mesh.
    """

    def __init__(self, mesh: Mesh, nq, h=None):
        self.nq = int(nq)
        eta, w = gauss_nodes_weights(self.nq)
        self.eta, self.w = eta, w
        L = lagrange_values(mesh.xi, eta)     # (nq, np)
        dL = lagrange_derivs(mesh.xi, eta)
        a, b, c = mesh.local_abc()
        q = np.arange(self.nq ** 3)
        qx, qy, qz = q % self.nq, (q // self.nq) % self.nq, q // (self.nq * self.nq)
        h = mesh.h if h is None else np.asarray(h, dtype=np.float64)
        self.h = h
        nloc = mesh.np1 ** 3
        N = np.empty((len(q), nloc))
        dN = np.empty((3, len(q), nloc))
        for l in range(nloc):
            lx, ly, lz = L[qx, a[l]], L[qy, b[l]], L[qz, c[l]]
            N[:, l] = lx * ly * lz
            dN[0, :, l] = (2.0 / h[0]) * dL[qx, a[l]] * ly * lz
            dN[1, :, l] = (2.0 / h[1]) * lx * dL[qy, b[l]] * lz
            dN[2, :, l] = (2.0 / h[2]) * lx * ly * dL[qz, c[l]]
        self.N, self.dN = N, dN
        self.detJ = float(h[0] * h[1] * h[2] / 8.0)
        self.W = w[qx] * w[qy] * w[qz] * self.detJ
        self.qoff = np.stack([(eta[qx] + 1.0) * 0.5 * h[0],
                              (eta[qy] + 1.0) * 0.5 * h[1],
                              (eta[qz] + 1.0) * 0.5 * h[2]], axis=1)

    def points(self, mesh: Mesh, e):
        """Gauss points of cell e (this quadrature must be the one of e's size)."""
        if not mesh.graded:
            i, j, k = mesh.cell_ijk(e)
            return self.qoff + np.array([i * mesh.h[0], j * mesh.h[1], k * mesh.h[2]])
        return self.qoff + mesh.cell_origin(e)

    def all_points(self, mesh: Mesh):
        return np.stack([self.points(mesh, e) for e in range(mesh.E)])


def cell_quadratures(mesh: Mesh, nq):
    """One CellQuadrature per cell (shared between cells of equal size)."""
    cache, out = {}, []
    for e in range(mesh.E):
        h = mesh.cell_h(e)
        key = tuple(h)
        if key not in cache:
            cache[key] = CellQuadrature(mesh, nq, h)
        out.append(cache[key])
    return out


# ---------------------------------------------------------------------------
# Element matrices (eq. FEM Ham entries / FEM S_loc entries)
# ---------------------------------------------------------------------------

def element_kinetic(cq: CellQuadrature):
    """K^e_IJ = 1/2 sum_q W_q grad N_I . grad N_J."""
    K = np.zeros((cq.N.shape[1],) * 2)
    for d in range(3):
        K += cq.dN[d].T @ (cq.W[:, None] * cq.dN[d])
    return 0.5 * K


def element_mass(cq: CellQuadrature):
    """M^e_IJ = sum_q W_q N_I N_J (consistent mass, Gauss rule)."""
    return cq.N.T @ (cq.W[:, None] * cq.N)


def element_potential(cq: CellQuadrature, vq_e):
    """V^e_IJ = sum_q W_q V(x_q) N_I N_J."""
    return cq.N.T @ ((cq.W * vq_e)[:, None] * cq.N)


def element_gga(cq: CellQuadrature, vgga_e):
    """Sum_q W_q V_GGA(x_q) . (grad N_I N_J + N_I grad N_J), vgga_e[d, q]
    (the GGA term of eq. "FEM Ham entries")."""
    A = sum(cq.dN[d].T @ ((cq.W * vgga_e[d])[:, None] * cq.N) for d in range(3))
    return A + A.T


def element_kterm(cq: CellQuadrature, k):
    """1/2 |k|^2 M^e_IJ - i sum_q W_q N_I (k . grad N_J)  (complex).

    The Galerkin matrix of the k terms of eq. "PAW Hamiltonian" acting on the
    periodic part u of psi = e^{ik.x} u.  Eq. "FEM Ham entries" prints this term
    with the gradient on N_I, which assembles to the opposite sign; the form here
    is the one consistent with the e^{-ik.x} phase of C^a (eq. "FEM Cmatrix"),
    pinned by the symmetric-form identity and the k -> k+G gauge check.
    """
    k = np.asarray(k, dtype=np.float64)
    G = sum(k[d] * (cq.N.T @ (cq.W[:, None] * cq.dN[d])) for d in range(3))
    return 0.5 * float(k @ k) * element_mass(cq) - 1j * G


def lumped_mass(mesh: Mesh):
    """M_D[I] = sum_{e containing I} det J_e rho_a rho_b rho_c (GLL quadrature mass)."""
    a, b, c = mesh.local_abc()
    ref = mesh.rho[a] * mesh.rho[b] * mesh.rho[c]
    md = np.zeros(mesh.M)
    cd = mesh.cell_dofs()
    for e in range(mesh.E):
        detJ = float(np.prod(mesh.cell_h(e)) / 8.0)
        np.add.at(md, cd[e], detJ * ref)
    return md


# ---------------------------------------------------------------------------
# Local operators
# ---------------------------------------------------------------------------

class LocalOperator:
    """H_loc = sum_e P_e^T (K^e + V^e [+ GGA^e] [+ k terms]) P_e and
    M = sum_e P_e^T M^e P_e.

    Applies are element-batched dense products (no sum factorization); small
    meshes can also be assembled as scipy.sparse matrices.  On a graded mesh,
    or with a GGA field vgga_q[e, d, q], the element matrices are formed cell
    by cell.
    """

    def __init__(self, mesh: Mesh, nq, veff_q, kpoint=None, vgga_q=None):
        self.mesh = mesh
        self.cq = CellQuadrature(mesh, nq)
        self.veff_q = np.asarray(veff_q, dtype=np.float64).reshape(mesh.E, -1)
        assert self.veff_q.shape[1] == self.cq.nq ** 3
        self.vgga_q = None
        if vgga_q is not None:
            self.vgga_q = np.asarray(vgga_q, dtype=np.float64).reshape(mesh.E, 3, self.cq.nq ** 3)
        self.k = None if kpoint is None or not np.any(kpoint) else np.asarray(kpoint, float)
        self.Ke = element_kinetic(self.cq)
        self.Me = element_mass(self.cq)
        self.KTe = None if self.k is None else element_kterm(self.cq, self.k)
        self.cell_dofs = mesh.cell_dofs()
        self.PT = mesh.scatter_matrix()
        self.general = mesh.graded or self.vgga_q is not None
        self.cqs = cell_quadratures(mesh, nq) if mesh.graded else [self.cq] * mesh.E
        self._shape_mats = {}

    def cell_cq(self, e):
        return self.cqs[e]

    def _by_shape(self, e):
        """(K^e, M^e, k-term^e) of cell e's size."""
        cq = self.cqs[e]
        key = id(cq)
        if key not in self._shape_mats:
            self._shape_mats[key] = (element_kinetic(cq), element_mass(cq),
                                     None if self.k is None else element_kterm(cq, self.k))
        return self._shape_mats[key]

    def cell_H(self, e):
        """H^e of cell e: kinetic + potential [+ GGA] [+ k terms]."""
        cq = self.cqs[e]
        K, _, KT = self._by_shape(e)
        A = K + element_potential(cq, self.veff_q[e])
        if self.vgga_q is not None:
            A = A + element_gga(cq, self.vgga_q[e])
        return A if KT is None else A + KT

    def cell_M(self, e):
        return self._by_shape(e)[1]

    # -- cellwise pieces -----------------------------------------------------
    def _gather(self, X):
        return X[self.cell_dofs]                      # (E, nloc, ncol)

    def _scatter(self, Ye):
        E, nloc, ncol = Ye.shape
        return self.PT @ Ye.reshape(E * nloc, ncol)

    def apply_H(self, X):
        X2 = X if X.ndim == 2 else X[:, None]
        Xe = self._gather(X2)
        if self.general:
            Ye = np.stack([self.cell_H(e) @ Xe[e] for e in range(self.mesh.E)])
            Y = self._scatter(Ye)
            return Y if X.ndim == 2 else Y[:, 0]
        Ye = self.Ke @ Xe                              # (E, nloc, ncol)
        if self.KTe is not None:
            Ye = Ye + self.KTe @ Xe
        Uq = self.cq.N @ Xe                            # values at quadrature points
        Uq = Uq * (self.cq.W[None, :] * self.veff_q)[:, :, None]
        Ye = Ye + self.cq.N.T @ Uq
        Y = self._scatter(Ye)
        return Y if X.ndim == 2 else Y[:, 0]

    def apply_M(self, X):
        X2 = X if X.ndim == 2 else X[:, None]
        Xe = self._gather(X2)
        if self.mesh.graded:
            Ye = np.stack([self.cell_M(e) @ Xe[e] for e in range(self.mesh.E)])
        else:
            Ye = self.Me @ Xe
        Y = self._scatter(Ye)
        return Y if X.ndim == 2 else Y[:, 0]

    # -- assembled (small meshes) ---------------------------------------------
    def _assemble(self, elem):
        rows, cols, vals = [], [], []
        nloc = self.cell_dofs.shape[1]
        for e in range(self.mesh.E):
            A = elem(e)
            cd = self.cell_dofs[e]
            rows.append(np.repeat(cd, nloc))
            cols.append(np.tile(cd, nloc))
            vals.append(A.ravel())
        dtype = np.complex128 if any(np.iscomplexobj(v) for v in vals) else np.float64
        return sp.csr_matrix((np.concatenate(vals).astype(dtype),
                              (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.mesh.M, self.mesh.M))

    def assemble_H(self):
        if self.general:
            return self._assemble(self.cell_H)

        def elem(e):
            A = self.Ke + element_potential(self.cq, self.veff_q[e])
            return A if self.KTe is None else A + self.KTe
        return self._assemble(elem)

    def assemble_K(self):
        return self._assemble(lambda e: self._by_shape(e)[0])

    def assemble_M(self):
        return self._assemble(self.cell_M)

    def assemble_GGA(self):
        """The GGA term alone, assembled (zero matrix without a GGA field)."""
        if self.vgga_q is None:
            return sp.csr_matrix((self.mesh.M, self.mesh.M))
        return self._assemble(lambda e: element_gga(self.cqs[e], self.vgga_q[e]))
