// Local (cell) part of the FE operators on gfx950.
//
// One workgroup handles one hexahedral cell and CB columns of the block
// (the cell-level product of the operator-action subsection, "extraction ->
// local action -> assembly").  The cell matrices of the paper are never
// formed: on the uniform periodic mesh every cell shares the 1-D tables, so
//   kinetic  K^e = fx Mz(x)My(x)Kx + fy Mz(x)Ky(x)Mx + fz Kz(x)My(x)Mx
//            (eq. "FEM Ham entries", gradient term; 7 one-dimensional
//            contractions),
//   V term   B^T diag(V(q) W_q) B with B = Bz(x)By(x)Bx the Lagrange values
//            at the Gauss points (3 contractions to the points, pointwise
//            scale, 3 back),
//   mass     detJ Mz(x)My(x)Mx (eq. "FEM S_loc entries").
// Lane <-> column: gathers and scatters read/write CB contiguous columns of
// a DOF row (node-major layout).  The cell's data lives in LDS between
// contraction passes; each thread owns whole 1-D lines of a pass.
// The scatter is a plain read-modify-write: the host launches one colour
// at a time and cells of one colour share no DOF, so no atomics are needed
// and the result is deterministic.

#include <cstdlib>
#include <string>

#include "kernels.h"

namespace pawfe {

template <typename T, int NP, int NQ, int CB, int MODE>
__global__ void __launch_bounds__(256) k_cell(CellArgs<T> A, const Tab1D<T>* __restrict__ tabp) {
  const Tab1D<T>& tab = *tabp;
  constexpr int NL = NP * NP * NP;
  constexpr int NLG = 256 / CB;
  constexpr int SZ_U = NL * CB;
  constexpr int SZ_Q1 = NP * NP * NQ * CB;
  constexpr int SZ_Q2 = NP * NQ * NQ * CB;
  __shared__ T smem[SZ_U + SZ_Q1 + SZ_Q2];
  T* U = smem;
  T* Q1 = smem + SZ_U;
  T* Q2 = Q1 + SZ_Q1;

  const int tid = threadIdx.x;
  const int col = tid % CB, lg = tid / CB;
  const int n = blockIdx.y * CB + col;
  const bool valid = n < A.ncols;
  const int e = A.cells[blockIdx.x];
  const int ci = e % A.n0, cj = (e / A.n0) % A.n1, ck = e / (A.n0 * A.n1);
  const int p = NP - 1;
  const int Gx = A.n0 * p, Gy = A.n1 * p, Gz = A.n2 * p;
  auto dof = [&](int a, int b, int c) -> int64_t {
    int gx = ci * p + a; gx = gx >= Gx ? gx - Gx : gx;
    int gy = cj * p + b; gy = gy >= Gy ? gy - Gy : gy;
    int gz = ck * p + c; gz = gz >= Gz ? gz - Gz : gz;
    return (int64_t)gx + (int64_t)Gx * ((int64_t)gy + (int64_t)Gy * gz);
  };

  // extraction (gather) of the cell's CB-column slab
  for (int l = lg; l < NL; l += NLG) {
    const int a = l % NP, b = (l / NP) % NP, c = l / (NP * NP);
    U[l * CB + col] = valid ? A.X[dof(a, b, c) * A.ldx + n] : T(0);
  }
  __syncthreads();

  if constexpr (MODE == kModeMass) {
    // z: Q1 = Mz U
    for (int ln = lg; ln < NP * NP; ln += NLG) {
      const int a = ln % NP, b = ln / NP;
      T u[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) u[c] = U[((c * NP + b) * NP + a) * CB + col];
#pragma unroll
      for (int c2 = 0; c2 < NP; ++c2) {
        T s = 0;
#pragma unroll
        for (int c = 0; c < NP; ++c) s += tab.M1[c2 * NP + c] * u[c];
        Q1[((c2 * NP + b) * NP + a) * CB + col] = s;
      }
    }
    __syncthreads();
    // y: in place, Q1 = My Q1
    for (int ln = lg; ln < NP * NP; ln += NLG) {
      const int a = ln % NP, c = ln / NP;
      T v[NP];
#pragma unroll
      for (int b = 0; b < NP; ++b) v[b] = Q1[((c * NP + b) * NP + a) * CB + col];
#pragma unroll
      for (int b2 = 0; b2 < NP; ++b2) {
        T s = 0;
#pragma unroll
        for (int b = 0; b < NP; ++b) s += tab.M1[b2 * NP + b] * v[b];
        Q1[((c * NP + b2) * NP + a) * CB + col] = s;
      }
    }
    __syncthreads();
    // x + assembly
    for (int ln = lg; ln < NP * NP; ln += NLG) {
      const int b = ln % NP, c = ln / NP;
      T w[NP];
#pragma unroll
      for (int a = 0; a < NP; ++a) w[a] = Q1[((c * NP + b) * NP + a) * CB + col];
#pragma unroll
      for (int a2 = 0; a2 < NP; ++a2) {
        T s = 0;
#pragma unroll
        for (int a = 0; a < NP; ++a) s += tab.M1[a2 * NP + a] * w[a];
        if (valid) {
          T* y = A.Y + dof(a2, b, c) * A.ldy + n;
          *y = *y + A.alpha * tab.detJ * s;
        }
      }
    }
    return;
  } else {
    // ---- V term: to the Gauss points ----
    // x: Q1[c][b][qa] = sum_a B[qa][a] U[c][b][a]
    for (int ln = lg; ln < NP * NP; ln += NLG) {
      const int b = ln % NP, c = ln / NP;
      T u[NP];
#pragma unroll
      for (int a = 0; a < NP; ++a) u[a] = U[((c * NP + b) * NP + a) * CB + col];
#pragma unroll
      for (int qa = 0; qa < NQ; ++qa) {
        T s = 0;
#pragma unroll
        for (int a = 0; a < NP; ++a) s += tab.B[qa * NP + a] * u[a];
        Q1[((c * NP + b) * NQ + qa) * CB + col] = s;
      }
    }
    __syncthreads();
    // y: Q2[c][qb][qa] = sum_b B[qb][b] Q1[c][b][qa]
    for (int ln = lg; ln < NP * NQ; ln += NLG) {
      const int qa = ln % NQ, c = ln / NQ;
      T v[NP];
#pragma unroll
      for (int b = 0; b < NP; ++b) v[b] = Q1[((c * NP + b) * NQ + qa) * CB + col];
#pragma unroll
      for (int qb = 0; qb < NQ; ++qb) {
        T s = 0;
#pragma unroll
        for (int b = 0; b < NP; ++b) s += tab.B[qb * NP + b] * v[b];
        Q2[((c * NQ + qb) * NQ + qa) * CB + col] = s;
      }
    }
    __syncthreads();
    // z, pointwise V(q) W_q (minus lambda_n W_q for the residual), z back; in place
    {
      const T lam = (MODE == kModeHRes && valid) ? (T)A.lam[n] : T(0);
      const T* Vw = A.Vw + (int64_t)e * (NQ * NQ * NQ);
      for (int ln = lg; ln < NQ * NQ; ln += NLG) {
        const int qa = ln % NQ, qb = ln / NQ;
        T w[NP], z[NQ];
#pragma unroll
        for (int c = 0; c < NP; ++c) w[c] = Q2[((c * NQ + qb) * NQ + qa) * CB + col];
#pragma unroll
        for (int qc = 0; qc < NQ; ++qc) {
          T s = 0;
#pragma unroll
          for (int c = 0; c < NP; ++c) s += tab.B[qc * NP + c] * w[c];
          const int q = (qc * NQ + qb) * NQ + qa;
          T vq = Vw[q];
          if constexpr (MODE == kModeHRes) vq -= lam * A.W3[q];
          z[qc] = s * vq;
        }
#pragma unroll
        for (int c = 0; c < NP; ++c) {
          T s = 0;
#pragma unroll
          for (int qc = 0; qc < NQ; ++qc) s += tab.B[qc * NP + c] * z[qc];
          Q2[((c * NQ + qb) * NQ + qa) * CB + col] = s;
        }
      }
    }
    __syncthreads();
    // y back: Q1[c][b][qa] = sum_qb B[qb][b] Q2[c][qb][qa]
    for (int ln = lg; ln < NP * NQ; ln += NLG) {
      const int qa = ln % NQ, c = ln / NQ;
      T v[NQ];
#pragma unroll
      for (int qb = 0; qb < NQ; ++qb) v[qb] = Q2[((c * NQ + qb) * NQ + qa) * CB + col];
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        T s = 0;
#pragma unroll
        for (int qb = 0; qb < NQ; ++qb) s += tab.B[qb * NP + b] * v[qb];
        Q1[((c * NP + b) * NQ + qa) * CB + col] = s;
      }
    }
    __syncthreads();
    // ---- kinetic ----
    // z: t1 = Mz U -> Q2 (as an NL buffer), t4 = Kz U -> U (in place)
    for (int ln = lg; ln < NP * NP; ln += NLG) {
      const int a = ln % NP, b = ln / NP;
      T u[NP];
#pragma unroll
      for (int c = 0; c < NP; ++c) u[c] = U[((c * NP + b) * NP + a) * CB + col];
#pragma unroll
      for (int c2 = 0; c2 < NP; ++c2) {
        T s1 = 0, s4 = 0;
#pragma unroll
        for (int c = 0; c < NP; ++c) {
          s1 += tab.M1[c2 * NP + c] * u[c];
          s4 += tab.K1[c2 * NP + c] * u[c];
        }
        Q2[((c2 * NP + b) * NP + a) * CB + col] = s1;
        U[((c2 * NP + b) * NP + a) * CB + col] = s4;
      }
    }
    __syncthreads();
    // y: t2 = My t1 (Q2, in place), s = fy Ky t1 + fz My t4 (U, in place)
    for (int ln = lg; ln < NP * NP; ln += NLG) {
      const int a = ln % NP, c = ln / NP;
      T v1[NP], v4[NP];
#pragma unroll
      for (int b = 0; b < NP; ++b) {
        v1[b] = Q2[((c * NP + b) * NP + a) * CB + col];
        v4[b] = U[((c * NP + b) * NP + a) * CB + col];
      }
#pragma unroll
      for (int b2 = 0; b2 < NP; ++b2) {
        T t2 = 0, sk = 0, sm = 0;
#pragma unroll
        for (int b = 0; b < NP; ++b) {
          t2 += tab.M1[b2 * NP + b] * v1[b];
          sk += tab.K1[b2 * NP + b] * v1[b];
          sm += tab.M1[b2 * NP + b] * v4[b];
        }
        Q2[((c * NP + b2) * NP + a) * CB + col] = t2;
        U[((c * NP + b2) * NP + a) * CB + col] = tab.f[1] * sk + tab.f[2] * sm;
      }
    }
    __syncthreads();
    // x: out = B^T Q1 (V term back) + fx Kx t2 + Mx s; assembly
    for (int ln = lg; ln < NP * NP; ln += NLG) {
      const int b = ln % NP, c = ln / NP;
      T g[NQ], t2[NP], s[NP];
#pragma unroll
      for (int qa = 0; qa < NQ; ++qa) g[qa] = Q1[((c * NP + b) * NQ + qa) * CB + col];
#pragma unroll
      for (int a = 0; a < NP; ++a) {
        t2[a] = Q2[((c * NP + b) * NP + a) * CB + col];
        s[a] = U[((c * NP + b) * NP + a) * CB + col];
      }
#pragma unroll
      for (int a2 = 0; a2 < NP; ++a2) {
        T ov = 0, ok = 0, om = 0;
#pragma unroll
        for (int qa = 0; qa < NQ; ++qa) ov += tab.B[qa * NP + a2] * g[qa];
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          ok += tab.K1[a2 * NP + a] * t2[a];
          om += tab.M1[a2 * NP + a] * s[a];
        }
        if (valid) {
          T* y = A.Y + dof(a2, b, c) * A.ldy + n;
          *y = *y + A.alpha * (ov + tab.f[0] * ok + om);
        }
      }
    }
  }
}

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
  for (int q = tid; q < NQ3; q += 256) A.out[(int64_t)e * NQ3 + q] = A.W3[q] * acc[q];
}

namespace {

template <typename T>
constexpr int cb_of() { return sizeof(T) == 8 ? 8 : 16; }

template <typename T>
const Tab1D<T>* dev_tab(const pawfe_op* op) {
  if constexpr (std::is_same<T, double>::value) return op->d.tab64; else return op->d.tab32;
}


template <typename T, int NP, int NQ, int CB>
pawfe_status run_cell(const pawfe_op* op, int mode, CellArgs<T> a, hipStream_t s) {
  const Tab1D<T>* tab = dev_tab<T>(op);
  const dim3 block(256);
  for (int c = 0; c < op->ncolour; ++c) {
    const int c0 = op->colour_off[c], c1 = op->colour_off[c + 1];
    if (c1 == c0) continue;
    CellArgs<T> ac = a;
    ac.cells = op->d.cells_by_colour + c0;
    const dim3 grid(c1 - c0, (a.ncols + CB - 1) / CB);
    if (mode == kModeH)
      hipLaunchKernelGGL((k_cell<T, NP, NQ, CB, kModeH>), grid, block, 0, s, ac, tab);
    else if (mode == kModeHRes)
      hipLaunchKernelGGL((k_cell<T, NP, NQ, CB, kModeHRes>), grid, block, 0, s, ac, tab);
    else
      hipLaunchKernelGGL((k_cell<T, NP, NQ, CB, kModeMass>), grid, block, 0, s, ac, tab);
  }
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

}  // namespace

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
  static const bool use_valu = [] {
    const char* v = std::getenv("PAWFE_CELL_KERNEL");
    return v && std::string(v) == "valu";
  }();
  if (!use_valu || bf3) return launch_cell_mfma<T>(op, mode, a, s);
  constexpr int CB = cb_of<T>();
  switch (op->p) {
    case 2: return run_cell<T, 3, 4, CB>(op, mode, a, s);
    case 3: return run_cell<T, 4, 5, CB>(op, mode, a, s);
    case 4: return run_cell<T, 5, 6, CB>(op, mode, a, s);
    case 5: return run_cell<T, 6, 7, CB>(op, mode, a, s);
    case 6: return run_cell<T, 7, 8, CB>(op, mode, a, s);
    default: return fail(PAWFE_EUNSUPPORTED, "degree not compiled");
  }
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
