"""Band energy and its gradient in the oracle (TEST INFRASTRUCTURE, FP64).

E = sum_n occ_n x_n^H H x_n with H the FE-PAW Hamiltonian.  E is linear in the
potential at quadrature points and in Delta_H, so

  dE/dV[e, q]     = W_{e,q} sum_n occ_n |u_n(x_{e,q})|^2,
                    u_n(x_{e,q}) = sum_l N_l(x_q) X[dof(e, l), n]
                    (the density-like contraction of the FE governing
                    equations: sum over states of |psi|^2 at the points),
  dE/dDh^a[al,be] = sum_n occ_n conj(P_{al n}) P_{be n},  P = C^a^H X
                    (the contraction U^H U that defines D^a in the same
                    equations),

with Delta_H treated as a full matrix of independent entries.
"""

from __future__ import annotations

import numpy as np


def band_energy(op, X, occ=None):
    occ = np.ones(X.shape[1]) if occ is None else np.asarray(occ, dtype=np.float64)
    HX = op.apply_H(X)
    return float(np.real(np.einsum("in,in,n->", X.conj(), HX, occ)))


def grad_veff(op, X, occ=None, cells=None):
    """dE/dV at every quadrature point, shape (E, nq^3); with ``cells`` only at
    the points of those cells, shape (len(cells), nq^3)."""
    occ = np.ones(X.shape[1]) if occ is None else np.asarray(occ, dtype=np.float64)
    cells = np.arange(op.mesh.E) if cells is None else np.asarray(cells)
    cd = op.cell_dofs[cells]
    Xe = X[cd]                                             # (ncells, nloc, ncol)
    U = op.cq.N @ Xe                                       # (ncells, nq^3, ncol); N is size-free
    dens = np.einsum("eqn,eqn,n->eq", U.conj(), U, occ).real
    W = np.stack([op.loc.cell_cq(e).W for e in cells])     # per-cell det J on graded meshes
    return W * dens


def grad_dH(op, X, occ=None):
    """dE/dDelta_H, packed like the input (nproj_a^2 per atom, row-major)."""
    occ = np.ones(X.shape[1]) if occ is None else np.asarray(occ, dtype=np.float64)
    P = op.CH @ X                                          # (sum npj, ncol)
    out = []
    for a in range(op.natoms):
        Pa = P[op.poff[a]:op.poff[a + 1]]
        G = (Pa.conj() * occ[None, :]) @ Pa.T
        out.append(np.real(G).ravel())
    return np.concatenate(out) if out else np.zeros(0)
