// Host-side operator builder of libpawfe.
//
// Builds, once per operator (the paper puts this setup below 1 % of an SCF
// step), everything the device kernels read:
//  * GLL nodes/weights and Gauss-Legendre nodes/weights by Newton iteration
//    on the Legendre three-term recurrence (FE discretization section);
//  * Lagrange values/derivatives at the Gauss points by the barycentric
//    formula, the 1-D reference stiffness K1 = D^T W D and mass M1 = B^T W B;
//  * the cell colouring (cells of one colour share no DOF);
//  * per-atom supports and the projector matrix C^a on the support nodes,
//    eq. "FEM Cmatrix" evaluated by sum factorization over the Gauss
//    points, with the minimum periodic image (requires r_c < L/2);
//  * the lumped GLL mass M_D (approximation (i) of eq. "Delta Sinv"),
//    G^{ab} = C^a^T M_D^{-1} C^b for atoms sharing support nodes, and
//    Delta_Sinv^a = Delta_S^a (I + G^a Delta_S^a)^{-1}.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <numeric>

#include "internal.h"

namespace pawfe {

namespace {

// Legendre P_n(x) and P_n'(x), P_n''(x) by the three-term recurrence.
void legendre(int n, double x, double& P, double& dP, double& d2P) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { P = 1.0; dP = 0.0; d2P = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  P = p1;
  // derivatives from (1-x^2) P' = n (P_{n-1} - x P_n)
  double den = 1.0 - x * x;
  dP = n * (p0 - x * p1) / den;
  d2P = (2.0 * x * dP - n * (n + 1.0) * P) / den;
}

bool finite_all(const double* v, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// Barycentric Lagrange values and derivatives of the basis through `nodes` at x.
void lagrange_at(const std::vector<double>& nodes, double x, double* val, double* der) {
  const int n = (int)nodes.size();
  std::vector<double> lam(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k)
      if (k != j) lam[j] /= (nodes[j] - nodes[k]);
  int hit = -1;
  for (int j = 0; j < n; ++j)
    if (std::fabs(x - nodes[j]) < 1e-15) hit = j;
  if (hit >= 0) {
    for (int j = 0; j < n; ++j) val[j] = (j == hit) ? 1.0 : 0.0;
    double s = 0.0;
    for (int k = 0; k < n; ++k)
      if (k != hit) s += 1.0 / (nodes[hit] - nodes[k]);
    for (int j = 0; j < n; ++j)
      der[j] = (j == hit) ? s : (lam[j] / lam[hit]) / (nodes[hit] - nodes[j]);
    return;
  }
  double den = 0.0;
  for (int k = 0; k < n; ++k) den += lam[k] / (x - nodes[k]);
  for (int j = 0; j < n; ++j) val[j] = (lam[j] / (x - nodes[j])) / den;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int k = 0; k < n; ++k)
      if (k != j) s += 1.0 / (x - nodes[k]);
    der[j] = val[j] * s;
  }
}

double solid_harmonic(int l, int m, double x, double y, double z) {
  if (l == 0) return 1.0;
  if (l == 1) return m == -1 ? y : (m == 0 ? z : x);
  switch (m) {
    case -2: return x * y;
    case -1: return y * z;
    case 0: return 3.0 * z * z - (x * x + y * y + z * z);
    case 1: return x * z;
    default: return x * x - y * y;
  }
}

// Solve Z (I + G S) = S for Z (n x n, row-major) by Gaussian elimination with
// partial pivoting on the transposed system.  Returns false if singular.
bool dsinv_block(int n, const double* G, const double* S, double* Z) {
  std::vector<double> A(n * n), R(n * n);
  // A = (I + G S)^T, R = S^T
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double gs = (i == j) ? 1.0 : 0.0;
      for (int k = 0; k < n; ++k) gs += G[i * n + k] * S[k * n + j];
      A[j * n + i] = gs;
      R[j * n + i] = S[i * n + j];
    }
  double scale = 0.0;
  for (double v : A) scale = std::max(scale, std::fabs(v));
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (std::fabs(A[piv * n + c]) <= 1e-13 * scale) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[c * n + k], A[piv * n + k]);
        std::swap(R[c * n + k], R[piv * n + k]);
      }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c] / A[c * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        A[r * n + k] -= f * A[c * n + k];
        R[r * n + k] -= f * R[c * n + k];
      }
    }
  }
  // Z^T = A^{-1} R  ->  Z[i][j] = (A^{-1}R)[j][i]
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) Z[i * n + j] = R[j * n + i] / A[j * n + j];
  return true;
}

// Complex version: Z (I + G S) = S with G = Gr + i Gi and S real; Z = Zr + i Zi.
bool dsinv_block_c(int n, const double* Gr, const double* Gi, const double* S, double* Zr, double* Zi) {
  typedef std::complex<double> C;
  std::vector<C> A(n * n), R(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      C gs = (i == j) ? C(1.0, 0.0) : C(0.0, 0.0);
      for (int k = 0; k < n; ++k) gs += C(Gr[i * n + k], Gi[i * n + k]) * S[k * n + j];
      A[j * n + i] = gs;
      R[j * n + i] = C(S[i * n + j], 0.0);
    }
  double scale = 0.0;
  for (const C& v : A) scale = std::max(scale, std::abs(v));
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::abs(A[r * n + c]) > std::abs(A[piv * n + c])) piv = r;
    if (std::abs(A[piv * n + c]) <= 1e-13 * scale) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[c * n + k], A[piv * n + k]);
        std::swap(R[c * n + k], R[piv * n + k]);
      }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const C f = A[r * n + c] / A[c * n + c];
      if (f == C(0.0, 0.0)) continue;
      for (int k = 0; k < n; ++k) {
        A[r * n + k] -= f * A[c * n + k];
        R[r * n + k] -= f * R[c * n + k];
      }
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      const C z = R[j * n + i] / A[j * n + j];
      Zr[i * n + j] = z.real();
      Zi[i * n + j] = z.imag();
    }
  return true;
}

}  // namespace

void gll_rule(int p, std::vector<double>& x, std::vector<double>& w) {
  x.assign(p + 1, 0.0);
  w.assign(p + 1, 0.0);
  const double pi = 3.14159265358979323846;
  for (int j = 0; j <= p; ++j) {
    double xj = -std::cos(pi * j / p);
    if (j > 0 && j < p) {
      for (int it = 0; it < 100; ++it) {
        double P, dP, d2P;
        legendre(p, xj, P, dP, d2P);
        double dx = dP / d2P;
        xj -= dx;
        if (std::fabs(dx) < 1e-16) break;
      }
    }
    x[j] = xj;
  }
  x[0] = -1.0;
  x[p] = 1.0;
  for (int j = 0; j <= p; ++j) {
    // P_p at +-1 is (+-1)^p; inside use the recurrence value
    double P = 1.0, p0 = 1.0, p1 = x[j];
    for (int k = 2; k <= p; ++k) {
      double pk = ((2.0 * k - 1.0) * x[j] * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = pk;
    }
    P = (p == 0) ? 1.0 : p1;
    w[j] = 2.0 / (p * (p + 1.0) * P * P);
  }
}

void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double xi = -std::cos(pi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP, d2P;
      legendre(n, xi, P, dP, d2P);
      double dx = P / dP;
      xi -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double P, dP, d2P;
    legendre(n, xi, P, dP, d2P);
    x[i] = xi;
    w[i] = 2.0 / ((1.0 - xi * xi) * dP * dP);
  }
}

pawfe_status build_host(const pawfe_op_desc* d, pawfe_op* op) {
  if (!d) return fail(PAWFE_EINVAL, "desc is NULL");
  for (int k = 0; k < 3; ++k) {
    if (d->ncell[k] < 2) return fail(PAWFE_EINVAL, "each ncell must be >= 2 (periodic mesh)");
    // the cell kernel packs a cell's coordinates into 10 bits each
    if (d->ncell[k] > 1024) return fail(PAWFE_EINVAL, "each ncell must be <= 1024");
    if (!(d->box[k] > 0.0) || !std::isfinite(d->box[k])) return fail(PAWFE_EINVAL, "box lengths must be positive");
  }
  const int p = d->degree, nq = d->nq1d;
  const bool ok_pair = (p == 2 && nq == 4) || (p == 3 && nq == 5) || (p == 4 && nq == 6) ||
                       (p == 5 && nq == 7) || (p == 6 && nq == 8);
  if (!ok_pair) return fail(PAWFE_EUNSUPPORTED, "supported (degree, nq): (2,4) (3,5) (4,6) (5,7) (6,8)");
  if (d->is_complex != 0 && d->is_complex != 1) return fail(PAWFE_EINVAL, "is_complex must be 0 or 1");
  if (!d->is_complex && (d->kpoint[0] != 0.0 || d->kpoint[1] != 0.0 || d->kpoint[2] != 0.0))
    return fail(PAWFE_EINVAL, "non-zero kpoint requires is_complex");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(d->kpoint[k])) return fail(PAWFE_ENONFINITE, "kpoint has NaN/Inf");
  if (d->sinv_mode != PAWFE_SINV_EXACT_G && d->sinv_mode != PAWFE_SINV_PP)
    return fail(PAWFE_EINVAL, "unknown sinv_mode");
  if (d->natoms < 0) return fail(PAWFE_EINVAL, "natoms < 0");
  if (!d->veff_q) return fail(PAWFE_EINVAL, "veff_q is NULL");

  for (int k = 0; k < 3; ++k) {
    op->n[k] = d->ncell[k];
    op->L[k] = d->box[k];
    op->h[k] = d->box[k] / d->ncell[k];
  }
  // cell boundaries: given (graded mesh) or i h (uniform)
  op->graded = d->xgrid != nullptr;
  {
    const double* xg = d->xgrid;
    for (int k = 0; k < 3; ++k) {
      op->bnd[k].assign(op->n[k] + 1, 0.0);
      for (int i = 0; i <= op->n[k]; ++i) op->bnd[k][i] = op->graded ? *xg++ : i * op->h[k];
      if (!op->graded) continue;
      const std::vector<double>& b = op->bnd[k];
      if (b[0] != 0.0 || b[op->n[k]] != op->L[k])
        return fail(PAWFE_EINVAL, "xgrid: each axis must start at 0 and end at the box length");
      for (int i = 0; i < op->n[k]; ++i)
        if (!std::isfinite(b[i + 1]) || !(b[i + 1] > b[i]))
          return fail(PAWFE_EINVAL, "xgrid: cell boundaries must increase strictly");
    }
  }
  op->p = p;
  op->np = p + 1;
  op->nq = nq;
  op->nloc = op->np * op->np * op->np;
  op->nq3 = nq * nq * nq;
  op->E = op->n[0] * op->n[1] * op->n[2];
  op->M = (int64_t)op->E * p * p * p;
  op->detJ = op->h[0] * op->h[1] * op->h[2] / 8.0;
  op->sinv_mode = d->sinv_mode;
  op->cplx = d->is_complex != 0;
  for (int k = 0; k < 3; ++k) op->kpt[k] = op->cplx ? d->kpoint[k] : 0.0;
  const int np = op->np, E = op->E;
  const int64_t nquad = (int64_t)E * op->nq3;
  if (!finite_all(d->veff_q, nquad)) return fail(PAWFE_ENONFINITE, "veff_q has NaN/Inf");
  op->gga = d->vgga_q != nullptr;
  if (op->gga) {
    if (!finite_all(d->vgga_q, 3 * nquad)) return fail(PAWFE_ENONFINITE, "vgga_q has NaN/Inf");
    op->vgga.assign(d->vgga_q, d->vgga_q + 3 * nquad);
  }
  op->general = op->graded || op->gga;
  if (op->general && op->cplx)
    return fail(PAWFE_EUNSUPPORTED, "graded meshes and the GGA term are built for real (Gamma-point) operators");
  // edge length of cell i along axis k, and per-cell det J (graded meshes)
  auto cell_h = [op](int k, int i) { return op->graded ? op->bnd[k][i + 1] - op->bnd[k][i] : op->h[k]; };
  op->cell_detJ.clear();
  if (op->graded) {
    op->cell_detJ.resize(E);
    for (int e = 0; e < E; ++e) {
      const int i = e % op->n[0], j = (e / op->n[0]) % op->n[1], k = e / (op->n[0] * op->n[1]);
      op->cell_detJ[e] = cell_h(0, i) * cell_h(1, j) * cell_h(2, k) / 8.0;
    }
  }

  // reference element
  gll_rule(p, op->gll_x, op->gll_w);
  gauss_rule(nq, op->gauss_x, op->gauss_w);
  op->B.assign(nq * np, 0.0);
  op->D.assign(nq * np, 0.0);
  for (int q = 0; q < nq; ++q)
    lagrange_at(op->gll_x, op->gauss_x[q], &op->B[q * np], &op->D[q * np]);
  op->K1.assign(np * np, 0.0);
  op->M1.assign(np * np, 0.0);
  op->G1.assign(np * np, 0.0);
  for (int a = 0; a < np; ++a)
    for (int b = 0; b < np; ++b) {
      double k = 0.0, m = 0.0, g = 0.0;
      for (int q = 0; q < nq; ++q) {
        k += op->gauss_w[q] * op->D[q * np + a] * op->D[q * np + b];
        m += op->gauss_w[q] * op->B[q * np + a] * op->B[q * np + b];
        g += op->gauss_w[q] * op->B[q * np + a] * op->D[q * np + b];
      }
      op->K1[a * np + b] = k;
      op->M1[a * np + b] = m;
      op->G1[a * np + b] = g;
    }
  op->W3.assign(op->nq3, 0.0);
  for (int qz = 0; qz < nq; ++qz)
    for (int qy = 0; qy < nq; ++qy)
      for (int qx = 0; qx < nq; ++qx)
        op->W3[qx + nq * (qy + nq * qz)] =
            op->gauss_w[qx] * op->gauss_w[qy] * op->gauss_w[qz] * op->detJ;
  op->veff.assign(d->veff_q, d->veff_q + nquad);

  // DOF helper
  const int Gx = op->n[0] * p, Gy = op->n[1] * p, Gz = op->n[2] * p;
  auto dof = [&](int e, int l) -> int64_t {
    int i = e % op->n[0], j = (e / op->n[0]) % op->n[1], k = e / (op->n[0] * op->n[1]);
    int a = l % np, b = (l / np) % np, c = l / (np * np);
    int64_t gx = (i * p + a) % Gx, gy = (j * p + b) % Gy, gz = (k * p + c) % Gz;
    return gx + (int64_t)Gx * (gy + (int64_t)Gy * gz);
  };

  // lumped GLL mass
  op->MD.assign(op->M, 0.0);
  for (int e = 0; e < E; ++e) {
    const double dJ = op->graded ? op->cell_detJ[e] : op->detJ;
    for (int l = 0; l < op->nloc; ++l) {
      int a = l % np, b = (l / np) % np, c = l / (np * np);
      op->MD[dof(e, l)] += dJ * op->gll_w[a] * op->gll_w[b] * op->gll_w[c];
    }
  }

  // colouring: 1-D colour i mod 2, the last cell of an odd direction gets 2
  auto col1 = [](int i, int n) { return (n % 2 == 1 && i == n - 1) ? 2 : i % 2; };
  const int cx = op->n[0] % 2 ? 3 : 2, cy = op->n[1] % 2 ? 3 : 2, cz = op->n[2] % 2 ? 3 : 2;
  op->ncolour = cx * cy * cz;
  op->cell_colour.assign(E, 0);
  for (int e = 0; e < E; ++e) {
    int i = e % op->n[0], j = (e / op->n[0]) % op->n[1], k = e / (op->n[0] * op->n[1]);
    op->cell_colour[e] = col1(i, op->n[0]) + cx * (col1(j, op->n[1]) + cy * col1(k, op->n[2]));
  }
  op->colour_off.assign(op->ncolour + 1, 0);
  for (int e = 0; e < E; ++e) op->colour_off[op->cell_colour[e] + 1]++;
  for (int c = 0; c < op->ncolour; ++c) op->colour_off[c + 1] += op->colour_off[c];
  op->cells_by_colour.assign(E, 0);
  {
    std::vector<int32_t> fill(op->colour_off.begin(), op->colour_off.end() - 1);
    for (int e = 0; e < E; ++e) op->cells_by_colour[fill[op->cell_colour[e]]++] = e;
  }
  // First visit of each DOF in the colour-ordered assembly (colours run in
  // ascending order): the cell of the lowest colour among the cells sharing
  // the DOF.  A local node's position class per axis is 0 (low face), 1
  // (inside) or 2 (high face); the cells sharing it are this cell and its
  // neighbours across the faces the node lies on.  Bit ca + 3 cb + 9 cc of
  // cell_own[e] is set when cell e makes the first visit of its nodes of
  // class (ca, cb, cc).
  op->cell_own.assign(E, 0);
  for (int e = 0; e < E; ++e) {
    const int ijk[3] = {e % op->n[0], (e / op->n[0]) % op->n[1], e / (op->n[0] * op->n[1])};
    for (int cls = 0; cls < 27; ++cls) {
      const int cl[3] = {cls % 3, (cls / 3) % 3, cls / 9};
      int nb[3][2], nn[3];
      for (int d = 0; d < 3; ++d) {
        nb[d][0] = ijk[d];
        nn[d] = 1;
        if (cl[d] != 1) nb[d][nn[d]++] = (ijk[d] + (cl[d] == 0 ? op->n[d] - 1 : 1)) % op->n[d];
      }
      bool first = true;
      for (int z = 0; z < nn[2]; ++z)
        for (int y = 0; y < nn[1]; ++y)
          for (int x = 0; x < nn[0]; ++x) {
            const int e2 = nb[0][x] + op->n[0] * (nb[1][y] + op->n[1] * nb[2][z]);
            if (e2 == e) continue;
            if (op->cell_colour[e2] == op->cell_colour[e])
              return fail(PAWFE_EINVAL, "internal: cells sharing a DOF have one colour");
            if (op->cell_colour[e2] < op->cell_colour[e]) first = false;
          }
      if (first) op->cell_own[e] |= 1u << cls;
    }
  }

  // ---- atoms ----------------------------------------------------------------
  const int na = d->natoms;
  op->natoms = na;
  op->nproj.assign(na, 0);
  op->poff.assign(na + 1, 0);
  op->poff2.assign(na + 1, 0);
  for (int a = 0; a < na; ++a) {
    int npj = d->nproj[a];
    if (npj < 1 || npj > kNpjMax) return fail(PAWFE_EINVAL, "nproj must be in 1..32");
    op->nproj[a] = npj;
    op->poff[a + 1] = op->poff[a] + npj;
    op->poff2[a + 1] = op->poff2[a] + npj * npj;
  }
  op->npj_total = op->poff[na];
  op->npj2_total = op->poff2[na];
  op->npj_max = 0;
  for (int a = 0; a < na; ++a) op->npj_max = std::max(op->npj_max, op->nproj[a]);
  if (na > 0) {
    if (!d->pos || !d->rcut || !d->nproj || !d->proj_l || !d->proj_m || !d->proj_sigma || !d->dH || !d->dS)
      return fail(PAWFE_EINVAL, "atom arrays must not be NULL when natoms > 0");
    if (!finite_all(d->pos, 3 * (int64_t)na) || !finite_all(d->dH, op->npj2_total) ||
        !finite_all(d->dS, op->npj2_total) || !finite_all(d->proj_sigma, op->npj_total))
      return fail(PAWFE_ENONFINITE, "atom data has NaN/Inf");
    const double Lmin = std::min(op->L[0], std::min(op->L[1], op->L[2]));
    for (int a = 0; a < na; ++a)
      if (!(d->rcut[a] > 0.0) || !(d->rcut[a] < 0.5 * Lmin))
        return fail(PAWFE_EINVAL, "rcut must satisfy 0 < r_c < min(L)/2");
    for (int t = 0; t < op->npj_total; ++t) {
      int l = d->proj_l[t], m = d->proj_m[t];
      if (l < 0 || l > 2 || m < -l || m > l) return fail(PAWFE_EINVAL, "projector (l, m) out of range (l <= 2)");
      if (!(d->proj_sigma[t] > 0.0)) return fail(PAWFE_EINVAL, "proj_sigma must be positive");
    }
  }
  op->dH.assign(d->dH ? d->dH : nullptr, d->dH ? d->dH + op->npj2_total : nullptr);
  op->dS.assign(d->dS ? d->dS : nullptr, d->dS ? d->dS + op->npj2_total : nullptr);

  // supports and C^a (sum-factorized Gauss quadrature of W_q N_l(x_q) p(d_q))
  op->supp_cell_off.assign(na + 1, 0);
  op->supp_node_off.assign(na + 1, 0);
  op->supp_cells.clear();
  op->supp_nodes.clear();
  op->Cvals.clear();
  op->atom_coff.assign(na, 0);
  std::vector<std::vector<double>> Gpp(na);
  std::vector<int32_t> rowmap(op->M, -1);
  const int nq3 = op->nq3;
  std::vector<double> xq(nq), F(nq3), T1(nq * nq * np), T2(nq * np * np), Cl(op->nloc);
  for (int a = 0; a < na; ++a) {
    const int npj = op->nproj[a];
    const double rc = d->rcut[a], rc2 = rc * rc;
    double R[3];
    for (int k = 0; k < 3; ++k) R[k] = d->pos[3 * a + k] - op->L[k] * std::floor(d->pos[3 * a + k] / op->L[k]);
    // candidate cells: index window around R, wrapped, de-duplicated
    std::vector<int> cand[3];
    for (int k = 0; k < 3; ++k) {
      std::vector<int> v;
      if (!op->graded) {
        int lo = (int)std::floor((R[k] - rc) / op->h[k]), hi = (int)std::floor((R[k] + rc) / op->h[k]);
        for (int i = lo; i <= hi; ++i) v.push_back(((i % op->n[k]) + op->n[k]) % op->n[k]);
      } else {   // cells whose interval, or a periodic image of it, meets [R - rc, R + rc]
        for (int sh = -1; sh <= 1; ++sh)
          for (int i = 0; i < op->n[k]; ++i)
            if (op->bnd[k][i] + sh * op->L[k] <= R[k] + rc && op->bnd[k][i + 1] + sh * op->L[k] >= R[k] - rc)
              v.push_back(i);
      }
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
      cand[k] = v;
    }
    std::vector<int> cells;
    std::vector<std::vector<double>> Ppts;    // per support cell: [nq3][npj] W p
    std::vector<std::vector<double>> Pth;     // per support cell: [nq3] Bloch phase k.x (complex)
    Gpp[a].assign(npj * npj, 0.0);
    for (int k : cand[2])
      for (int j : cand[1])
        for (int i : cand[0]) {
          int e = i + op->n[0] * (j + op->n[1] * k);
          std::vector<double> P((size_t)nq3 * npj, 0.0), TH(op->cplx ? nq3 : 0, 0.0);
          bool inside_any = false;
          const int ijk[3] = {i, j, k};
          for (int qz = 0; qz < nq; ++qz)
            for (int qy = 0; qy < nq; ++qy)
              for (int qx = 0; qx < nq; ++qx) {
                double x[3] = {(i + 0.5 * (op->gauss_x[qx] + 1.0)) * op->h[0],
                               (j + 0.5 * (op->gauss_x[qy] + 1.0)) * op->h[1],
                               (k + 0.5 * (op->gauss_x[qz] + 1.0)) * op->h[2]};
                if (op->graded) {
                  const int qq[3] = {qx, qy, qz};
                  for (int t = 0; t < 3; ++t)
                    x[t] = op->bnd[t][ijk[t]] + 0.5 * (op->gauss_x[qq[t]] + 1.0) * cell_h(t, ijk[t]);
                }
                double dd[3];
                for (int t = 0; t < 3; ++t) {
                  dd[t] = x[t] - R[t];
                  dd[t] -= op->L[t] * std::nearbyint(dd[t] / op->L[t]);
                }
                double r2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
                if (!(r2 < rc2)) continue;
                inside_any = true;
                int q = qx + nq * (qy + nq * qz);
                // phase at the point's image next to the atom (the given, unwrapped
                // atom position plus the minimum-image displacement)
                if (op->cplx)
                  for (int t = 0; t < 3; ++t) TH[q] += op->kpt[t] * (d->pos[3 * a + t] + dd[t]);
                for (int t = 0; t < npj; ++t) {
                  int g = op->poff[a] + t;
                  double sg = d->proj_sigma[g];
                  double u = 1.0 - r2 / rc2;
                  double val = solid_harmonic(d->proj_l[g], d->proj_m[g], dd[0], dd[1], dd[2]) *
                               std::exp(-r2 / (2.0 * sg * sg)) * u * u;
                  P[(size_t)q * npj + t] = val;
                }
              }
          if (!inside_any) continue;
          cells.push_back(e);
          // <p|p> by the same quadrature
          const double wsc = op->graded ? op->cell_detJ[e] / op->detJ : 1.0;
          for (int q = 0; q < nq3; ++q)
            for (int s = 0; s < npj; ++s) {
              double ps = P[(size_t)q * npj + s];
              if (ps == 0.0) continue;
              for (int t = 0; t < npj; ++t) Gpp[a][s * npj + t] += wsc * op->W3[q] * ps * P[(size_t)q * npj + t];
            }
          Ppts.push_back(std::move(P));
          Pth.push_back(std::move(TH));
        }
    // sort support cells (and their point data) by cell index
    std::vector<int> order(cells.size());
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int x, int y) { return cells[x] < cells[y]; });
    std::vector<int64_t> nodes;
    for (int idx : order) {
      op->supp_cells.push_back(cells[idx]);
      for (int l = 0; l < op->nloc; ++l) nodes.push_back(dof(cells[idx], l));
    }
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
    op->supp_cell_off[a + 1] = op->supp_cells.size();
    op->supp_node_off[a + 1] = op->supp_node_off[a] + (int64_t)nodes.size();
    for (size_t r = 0; r < nodes.size(); ++r) rowmap[nodes[r]] = (int32_t)r;
    op->atom_coff[a] = (int32_t)op->Cvals.size();
    op->Cvals.resize(op->Cvals.size() + nodes.size() * npj, 0.0);
    if (op->cplx) op->Cvals_im.resize(op->Cvals.size(), 0.0);
    double* Ca = &op->Cvals[op->atom_coff[a]];
    double* Ca_im = op->cplx ? &op->Cvals_im[op->atom_coff[a]] : nullptr;
    for (int idx : order) {
      const int e = cells[idx];
      const std::vector<double>& P = Ppts[idx];
      const double wsc = op->graded ? op->cell_detJ[e] / op->detJ : 1.0;
      // C = N^T W (p e^{-i k.x}): real part, then (complex) imaginary part
      for (int part = 0; part < (op->cplx ? 2 : 1); ++part)
      for (int t = 0; t < npj; ++t) {
        for (int q = 0; q < nq3; ++q) {
          const double wp = wsc * op->W3[q] * P[(size_t)q * npj + t];
          F[q] = !op->cplx ? wp : (part == 0 ? wp * std::cos(Pth[idx][q]) : -wp * std::sin(Pth[idx][q]));
        }
        // x: F[qz][qy][qx] -> T1[qz][qy][a]
        for (int qz = 0; qz < nq; ++qz)
          for (int qy = 0; qy < nq; ++qy)
            for (int aa = 0; aa < np; ++aa) {
              double s = 0.0;
              for (int qx = 0; qx < nq; ++qx) s += op->B[qx * np + aa] * F[qx + nq * (qy + nq * qz)];
              T1[aa + np * (qy + nq * qz)] = s;
            }
        // y: -> T2[qz][b][a]
        for (int qz = 0; qz < nq; ++qz)
          for (int bb = 0; bb < np; ++bb)
            for (int aa = 0; aa < np; ++aa) {
              double s = 0.0;
              for (int qy = 0; qy < nq; ++qy) s += op->B[qy * np + bb] * T1[aa + np * (qy + nq * qz)];
              T2[aa + np * (bb + np * qz)] = s;
            }
        // z: -> Cl[c][b][a]
        for (int cc = 0; cc < np; ++cc)
          for (int bb = 0; bb < np; ++bb)
            for (int aa = 0; aa < np; ++aa) {
              double s = 0.0;
              for (int qz = 0; qz < nq; ++qz) s += op->B[qz * np + cc] * T2[aa + np * (bb + np * qz)];
              Cl[aa + np * (bb + np * cc)] = s;
            }
        double* dst = part == 0 ? Ca : Ca_im;
        for (int l = 0; l < op->nloc; ++l) dst[(size_t)rowmap[dof(e, l)] * npj + t] += Cl[l];
      }
    }
    for (int64_t nd : nodes) {
      op->supp_nodes.push_back(nd);
      rowmap[nd] = -1;
    }
  }

  // node-major support rows: every DOF in some support, with its (atom, C row) entries
  std::vector<std::pair<int64_t, std::pair<int, int>>> ent;   // (dof, (atom, row)), sorted
  for (int a = 0; a < na; ++a)
    for (int64_t r = op->supp_node_off[a]; r < op->supp_node_off[a + 1]; ++r)
      ent.push_back({op->supp_nodes[r], {a, (int)(r - op->supp_node_off[a])}});
  std::sort(ent.begin(), ent.end());
  op->nent = (int64_t)ent.size();
  op->node2srow.assign(op->M, -1);
  op->srow_ptr.assign(1, 0);
  op->srow_atom.clear();
  op->srow_coff.clear();
  for (size_t x = 0; x < ent.size(); ++x) {
    if (x > 0 && ent[x].first != ent[x - 1].first) op->srow_ptr.push_back((int32_t)x);
    if (x == 0 || ent[x].first != ent[x - 1].first) op->node2srow[ent[x].first] = (int32_t)op->srow_ptr.size() - 1;
    const int a = ent[x].second.first;
    op->srow_atom.push_back(a);
    op->srow_coff.push_back(op->atom_coff[a] + ent[x].second.second * op->nproj[a]);
  }
  if (!ent.empty()) op->srow_ptr.push_back((int32_t)ent.size());
  op->nsrow = (int64_t)op->srow_ptr.size() - 1;

  // G^{ab} = C^a^H M_D^{-1} C^b over shared support nodes (imaginary part in
  // Gab_im for complex operators)
  std::map<std::pair<int, int>, std::vector<double>> Gab, Gab_im;
  {
    size_t s0 = 0;
    while (s0 < ent.size()) {
      size_t s1 = s0;
      while (s1 < ent.size() && ent[s1].first == ent[s0].first) ++s1;
      const double minv = 1.0 / op->MD[ent[s0].first];
      for (size_t x = s0; x < s1; ++x)
        for (size_t y = s0; y < s1; ++y) {
          int a = ent[x].second.first, b = ent[y].second.first;
          int na_ = op->nproj[a], nb_ = op->nproj[b];
          auto& G = Gab[{a, b}];
          if (G.empty()) G.assign(na_ * nb_, 0.0);
          const size_t oa = op->atom_coff[a] + (size_t)ent[x].second.second * na_;
          const size_t ob = op->atom_coff[b] + (size_t)ent[y].second.second * nb_;
          const double* ca = &op->Cvals[oa];
          const double* cb = &op->Cvals[ob];
          if (!op->cplx) {
            for (int s = 0; s < na_; ++s)
              for (int t = 0; t < nb_; ++t) G[s * nb_ + t] += ca[s] * minv * cb[t];
          } else {
            auto& Gi = Gab_im[{a, b}];
            if (Gi.empty()) Gi.assign(na_ * nb_, 0.0);
            const double* cai = &op->Cvals_im[oa];
            const double* cbi = &op->Cvals_im[ob];
            for (int s = 0; s < na_; ++s)
              for (int t = 0; t < nb_; ++t) {   // conj(ca) cb
                G[s * nb_ + t] += minv * (ca[s] * cb[t] + cai[s] * cbi[t]);
                Gi[s * nb_ + t] += minv * (ca[s] * cbi[t] - cai[s] * cb[t]);
              }
          }
        }
      s0 = s1;
    }
  }
  op->gp_ptr.assign(na + 1, 0);
  op->gp_b.clear();
  op->gp_off.clear();
  op->Gvals.clear();
  for (auto& kv : Gab) op->gp_ptr[kv.first.first + 1]++;
  for (int a = 0; a < na; ++a) op->gp_ptr[a + 1] += op->gp_ptr[a];
  op->Gvals_im.clear();
  for (auto& kv : Gab) {   // std::map iterates (a, b) in order
    op->gp_b.push_back(kv.first.second);
    op->gp_off.push_back((int32_t)op->Gvals.size());
    op->Gvals.insert(op->Gvals.end(), kv.second.begin(), kv.second.end());
    if (op->cplx) {
      const std::vector<double>& gi = Gab_im[kv.first];
      op->Gvals_im.insert(op->Gvals_im.end(), gi.begin(), gi.end());
    }
  }

  // Delta_Sinv^a = Delta_S^a (I + G^a Delta_S^a)^{-1} (complex for complex
  // operators with the exact G^a)
  op->dSinv.assign(op->npj2_total, 0.0);
  const bool csinv = op->cplx && op->sinv_mode != PAWFE_SINV_PP;
  op->dSinv_im.assign(csinv ? op->npj2_total : 0, 0.0);
  for (int a = 0; a < na; ++a) {
    const int npj = op->nproj[a];
    std::vector<double> Ga(npj * npj, 0.0), Gai(npj * npj, 0.0);
    if (op->sinv_mode == PAWFE_SINV_PP) {
      Ga = Gpp[a];
    } else {
      auto it = Gab.find({a, a});
      if (it != Gab.end()) Ga = it->second;
      if (csinv) {
        auto jt = Gab_im.find({a, a});
        if (jt != Gab_im.end()) Gai = jt->second;
      }
    }
    const bool ok = csinv ? dsinv_block_c(npj, Ga.data(), Gai.data(), &op->dS[op->poff2[a]],
                                          &op->dSinv[op->poff2[a]], &op->dSinv_im[op->poff2[a]])
                          : dsinv_block(npj, Ga.data(), &op->dS[op->poff2[a]], &op->dSinv[op->poff2[a]]);
    if (!ok) return fail(PAWFE_ENOTSPD, "I + G^a Delta_S^a is singular for atom " + std::to_string(a));
  }

  // reduction work items: chunks of at most kItemRows support rows per atom
  const int kItemRows = 128;
  op->item_atom.clear();
  op->item_row0.clear();
  op->item_row1.clear();
  op->item_poff.clear();
  op->item_ptr.assign(na + 1, 0);
  int64_t prow = 0;
  for (int a = 0; a < na; ++a) {
    const int64_t nrow = op->supp_node_off[a + 1] - op->supp_node_off[a];
    for (int64_t r0 = 0; r0 < nrow; r0 += kItemRows) {
      op->item_atom.push_back(a);
      op->item_row0.push_back((int32_t)r0);
      op->item_row1.push_back((int32_t)std::min<int64_t>(nrow, r0 + kItemRows));
      op->item_poff.push_back((int32_t)prow);
      prow += op->nproj[a];
    }
    op->item_ptr[a + 1] = (int32_t)op->item_atom.size();
  }
  op->nitems = (int)op->item_atom.size();
  op->item_rows_total = prow;

  // greedy colouring of the atom overlap graph (atoms sharing a support node)
  std::vector<std::vector<int>> nbr(na);
  for (int64_t sr = 0; sr < op->nsrow; ++sr)
    for (int32_t k = op->srow_ptr[sr]; k < op->srow_ptr[sr + 1]; ++k)
      for (int32_t k2 = k + 1; k2 < op->srow_ptr[sr + 1]; ++k2) {
        nbr[op->srow_atom[k]].push_back(op->srow_atom[k2]);
        nbr[op->srow_atom[k2]].push_back(op->srow_atom[k]);
      }
  std::vector<int> acol(na, -1);
  int ncol = 0;
  for (int a = 0; a < na; ++a) {
    std::vector<char> used(ncol + 1, 0);
    for (int b : nbr[a])
      if (acol[b] >= 0) used[acol[b]] = 1;
    int c = 0;
    while (used[c]) ++c;
    acol[a] = c;
    ncol = std::max(ncol, c + 1);
  }
  op->natom_colours = ncol;
  const int kFixRows = 16;   // rows per add-back work item
  op->fix_atom.clear();
  op->fix_row0.clear();
  op->fix_row1.clear();
  op->fix_colour_off.assign(1, 0);
  for (int c = 0; c < ncol; ++c) {
    for (int a = 0; a < na; ++a) {
      if (acol[a] != c) continue;
      const int64_t nrow = op->supp_node_off[a + 1] - op->supp_node_off[a];
      for (int64_t r0 = 0; r0 < nrow; r0 += kFixRows) {
        op->fix_atom.push_back(a);
        op->fix_row0.push_back((int32_t)r0);
        op->fix_row1.push_back((int32_t)std::min<int64_t>(nrow, r0 + kFixRows));
      }
    }
    op->fix_colour_off.push_back((int32_t)op->fix_atom.size());
  }
  op->atom_noff.assign(na + 1, 0);
  for (int a = 0; a <= na; ++a) op->atom_noff[a] = (int32_t)op->supp_node_off[a];
  op->atom_nodes.assign(op->supp_nodes.begin(), op->supp_nodes.end());
  return PAWFE_OK;
}

}  // namespace pawfe
