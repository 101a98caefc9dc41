// Cell-level entry of the FE operators and the band-energy density.
//
// launch_cell sets up the arguments of the cell operator (kinetic + V(q)W_q,
// the residual variant with -lambda_n M, or the mass; the cell-level product
// of the operator-action subsection) and runs, one launch per cell colour,
// the vector-ALU kernel (cell_valu.h: kernels_cell_valu.hip for operators
// whose cells share one size, with the imaginary k term of complex
// operators in the same launch; kernels_cell_gen_*.hip for graded meshes and
// the GGA term) or, for bf16x3, the matrix-core kernel of
// kernels_cell_mfma.hip.
//
// k_cell_density is the adjoint contraction of the potential term: the
// band-energy density W_q sum_n occ_n |u_n(x_q)|^2 at the Gauss points of
// every cell (the dE/dV of the governing equations), with the columns
// interpolated to the points by the same three 1-D sweeps as the V term.

#include "kernels.h"

namespace pawfe {

// Band-energy density: dE/dV[e][q] = W_q sum_n occ_n |u_n(x_q)|^2 for one
// cell per workgroup, looping over all column tiles so every output is
// written once (no cell-local state kept across cell batches).
template <int NP, int NQ, int CB>
__global__ void __launch_bounds__(256) k_cell_density(DensArgs A, const Tab1D<double>* __restrict__ tabp) {
  const Tab1D<double>& tab = *tabp;
  constexpr int NL = NP * NP * NP;
  constexpr int NLG = 256 / CB;
  constexpr int NQ3 = NQ * NQ * NQ;
  __shared__ double U[NL * CB];
  __shared__ double Q1[NP * NP * NQ * CB];
  __shared__ double Q2[NP * NQ * NQ * CB];
  __shared__ double acc[NQ3];
  const int tid = threadIdx.x, col = tid % CB, lg = tid / CB;
  const int e = blockIdx.x;
  const int ci = e % A.n0, cj = (e / A.n0) % A.n1, ck = e / (A.n0 * A.n1);
  const int p = NP - 1;
  const int Gx = A.n0 * p, Gy = A.n1 * p, Gz = A.n2 * p;
  auto dof = [&](int a, int b, int c) -> int64_t {
    int gx = ci * p + a; gx = gx >= Gx ? gx - Gx : gx;
    int gy = cj * p + b; gy = gy >= Gy ? gy - Gy : gy;
    int gz = ck * p + c; gz = gz >= Gz ? gz - Gz : gz;
    return (int64_t)gx + (int64_t)Gx * ((int64_t)gy + (int64_t)Gy * gz);
  };
  for (int q = tid; q < NQ3; q += 256) acc[q] = 0.0;
  for (int n0 = 0; n0 < A.ncols; n0 += CB) {
    const int n = n0 + col;
    const bool valid = n < A.ncols;
    __syncthreads();
    for (int l = lg; l < NL; l += NLG) {
      const int a = l % NP, b = (l / NP) % NP, c = l / (NP * NP);
      U[l * CB + col] = valid ? A.X[dof(a, b, c) * A.ldx + n] : 0.0;
    }
    __syncthreads();
    for (int ln = lg; ln < NP * NP; ln += NLG) {
      const int b = ln % NP, c = ln / NP;
      double u[NP];
#pragma unroll
      for (int a = 0; a < NP; ++a) u[a] = U[((c * NP + b) * NP + a) * CB + col];
#pragma unroll
      for (int qa = 0; qa < NQ; ++qa) {
        double s = 0;
#pragma unroll
        for (int a = 0; a < NP; ++a) s += tab.B[qa * NP + a] * u[a];
        Q1[((c * NP + b) * NQ + qa) * CB + col] = s;
      }
    }
    __syncthreads();
    for (int ln = lg; ln < NP * NQ; ln += NLG) {
      const int qa = ln % NQ, c = ln / NQ;
      double v[NP];
#pragma unroll
      for (int b = 0; b < NP; ++b) v[b] = Q1[((c * NP + b) * NQ + qa) * CB + col];
#pragma unroll
      for (int qb = 0; qb < NQ; ++qb) {
        double s = 0;
#pragma unroll
        for (int b = 0; b < NP; ++b) s += tab.B[qb * NP + b] * v[b];
        Q2[((c * NQ + qb) * NQ + qa) * CB + col] = s;
      }
    }
    __syncthreads();
    const double w = (valid && A.occ) ? A.occ[n] : (valid ? 1.0 : 0.0);
    for (int ln = lg; ln < NQ * NQ; ln += NLG) {
      const int qa = ln % NQ, qb = ln / NQ;
      double v[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) v[c] = Q2[((c * NQ + qb) * NQ + qa) * CB + col];
#pragma unroll
      for (int qc = 0; qc < NQ; ++qc) {
        double s = 0;
#pragma unroll
        for (int c = 0; c < NP; ++c) s += tab.B[qc * NP + c] * v[c];
        // reduce w |u|^2 over the CB columns of this line (lanes col..)
        double val = w * s * s;
#pragma unroll
        for (int off = CB / 2; off > 0; off >>= 1) val += __shfl_xor(val, off, CB);
        if (col == 0) acc[(qc * NQ + qb) * NQ + qa] += val;
      }
    }
  }
  __syncthreads();
  const double cs = A.cscale ? A.cscale[e] : 1.0;
  for (int q = tid; q < NQ3; q += 256) A.out[(int64_t)e * NQ3 + q] = A.W3[q] * cs * acc[q];
}

template <typename T>
pawfe_status launch_cell(const pawfe_op* op, int mode, const T* X, int64_t ldx, T* Y, int64_t ldy,
                         int ncols, const double* lam, double alpha, hipStream_t s, bool bf3) {
  if (ncols <= 0) return PAWFE_OK;
  if (bf3 && sizeof(T) != 4) return fail(PAWFE_EINVAL, "bf16x3 needs FP32 data");
  CellArgs<T> a{};
  a.bf3 = bf3 ? 1 : 0;
  a.X = X;
  a.ldx = ldx;
  a.Y = Y;
  a.ldy = ldy;
  a.ncols = ncols;
  a.Vw = std::is_same<T, double>::value ? (const T*)op->d.Vw : (const T*)op->d.Vw_f;
  a.W3 = std::is_same<T, double>::value ? (const T*)op->d.W3 : (const T*)op->d.W3_f;
  a.lam = lam;
  a.alpha = (T)alpha;
  a.n0 = op->n[0];
  a.n1 = op->n[1];
  a.n2 = op->n[2];
  if (op->general) {   // graded mesh / GGA term: every local term on the vector-ALU variants
    if (bf3) return fail(PAWFE_EUNSUPPORTED, "bf16x3 is not built for graded meshes or the GGA term");
    return launch_cell_gen<T>(op, mode, a, s);
  }
  pawfe_status st = PAWFE_OK;
  bool done = false;
  // K + V, the residual K + V - lambda M and the mass term in FP32 or FP64:
  // vector-ALU kernel (the matrix-core kernel keeps bf16x3)
  if ((mode == kModeH || mode == kModeHRes || mode == kModeMass) && !bf3) st = launch_cell_valu(op, mode, a, s, &done);
  if (st == PAWFE_OK && !done) st = launch_cell_mfma<T>(op, mode, a, s);
  if (done) return st;   // the vector-ALU variants include the imaginary k term
  // complex operators on the matrix cores: the imaginary local term, on the
  // (re, im) column pairs, as a second launch
  if (st != PAWFE_OK || !op->cplx || (mode != kModeH && mode != kModeHRes)) return st;
  return launch_cell_mfma<T>(op, kModeImg, a, s);
}

template pawfe_status launch_cell<double>(const pawfe_op*, int, const double*, int64_t, double*, int64_t,
                                          int, const double*, double, hipStream_t, bool);
template pawfe_status launch_cell<float>(const pawfe_op*, int, const float*, int64_t, float*, int64_t,
                                         int, const double*, double, hipStream_t, bool);

pawfe_status launch_density(const pawfe_op* op, const double* X, int64_t ldx, int ncols,
                            const double* occ, double* out, hipStream_t s) {
  DensArgs a{};
  a.X = X;
  a.ldx = ldx;
  a.ncols = ncols;
  a.occ = occ;
  a.out = out;
  a.W3 = op->d.W3;
  a.cscale = op->d.cscale;
  a.n0 = op->n[0];
  a.n1 = op->n[1];
  a.n2 = op->n[2];
  const Tab1D<double>* tab = op->d.tab64;
  const dim3 grid(op->E), block(256);
  switch (op->p) {
    case 2: hipLaunchKernelGGL((k_cell_density<3, 4, 8>), grid, block, 0, s, a, tab); break;
    case 3: hipLaunchKernelGGL((k_cell_density<4, 5, 8>), grid, block, 0, s, a, tab); break;
    case 4: hipLaunchKernelGGL((k_cell_density<5, 6, 8>), grid, block, 0, s, a, tab); break;
    case 5: hipLaunchKernelGGL((k_cell_density<6, 7, 8>), grid, block, 0, s, a, tab); break;
    case 6: hipLaunchKernelGGL((k_cell_density<7, 8, 8>), grid, block, 0, s, a, tab); break;
    default: return fail(PAWFE_EUNSUPPORTED, "degree not compiled");
  }
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

}  // namespace pawfe
