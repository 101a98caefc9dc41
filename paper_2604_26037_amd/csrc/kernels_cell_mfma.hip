// Local (cell) part of the FE operators on the gfx950 matrix cores.
//
// Every 1-D contraction of the sum-factorized cell operator (kinetic
// fx Mz My Kx + fy Mz Ky Mx + fz Kz My Mx, the potential term
// B^T diag(V(q) W_q) B, the mass detJ Mz My Mx; eqs. "FEM Ham entries" and
// "FEM S_loc entries") is a small GEMM  Out[r][o] = sum_k In[r][k] Cf[o][k]
// with r = (line, column) pairs, k the input index along the axis and o the
// output index (several 1-D matrices stacked along o or k).  It runs as
// v_mfma_{f32,f64}_16x16x4: A (16 r x 4 k) is read from LDS, B (4 k x 16 o)
// is the 1-D table, held in registers for the whole pass (one value per
// lane per k-step), D (16 r x 16 o) is written back to LDS.
//
// LDS holds three slabs of 8x8x8 padded slots per column (slot
// (z*8 + y)*8 + x), so every pass can run in place: a wave owns whole lines
// and reads all of a tile's inputs before writing its outputs.
//
// Order of the passes (U = gathered cell values, slab A):
//   P1 x: [Bx; Kx; Mx] U  -> slab B (V path), slab C (Kx U), slab A (Mx U)
//   P2 y: By     (slab B)        P3 z: Bz, times V(q) W_q (slab B)
//   P4 z: Bz^T   (slab B)        P5 y: By^T (slab B)
//   P6 y: [fx My | fy Ky ; 0 | My] on (C, A) -> C = P, A = Q
//   P7 z: [Mz | fz Kz] on (C, A) -> C = kinetic result
//   P8 x: Bx^T (slab B), added into C; then the colour-ordered assembly.
// The grid is remapped so that consecutive logical blocks (all column tiles
// of one cell, then the next cells) land on the same XCD and share its L2.

#include "kernels.h"

namespace pawfe {

namespace {

template <typename T>
struct Mma;
template <>
struct Mma<float> {
  typedef float V4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V4 op(float a, float b, V4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mma<double> {
  typedef double V4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V4 op(double a, double b, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

constexpr int kSlots = 512;   // 8 x 8 x 8 padded slots per column

__device__ __forceinline__ int slot(int x, int y, int z) { return (z * 8 + y) * 8 + x; }

// slot of (line, k) for a contraction along `ax`; the line enumerates the two
// other axes with the lower axis fastest (extent e0 of that lower axis).
template <int AX>
__device__ __forceinline__ int line_slot(int line, int e0, int k) {
  const int u = line % e0, v = line / e0;
  if constexpr (AX == 0) return slot(k, u, v);
  else if constexpr (AX == 1) return slot(u, k, v);
  else return slot(u, v, k);
}

}  // namespace

// One MFMA contraction pass.  Coefficient callback cf(o, k) gives the stacked
// matrix; inputs k < K0 come from `in0`, K0 <= k < K0 + K1 from `in1`;
// outputs o < O0 go to `out0`, then the next O1 to `out1`, the next O2 to
// `out2` (each indexed from 0).  post(line, o, col, value, old) returns the
// value to store (pointwise V(q) W_q, or an accumulation in the last pass).
template <typename T, int AX, int CB, int K0, int K1, int O0, int O1, int O2, int NLINES, int E0, class CF,
          class POST>
__device__ __forceinline__ void mfma_pass(const T* in0, const T* in1, T* out0, T* out1, T* out2, CF cf,
                                          POST post) {
  using M = Mma<T>;
  constexpr int KT = K0 + K1, NKS = (KT + 3) / 4;
  constexpr int OT = O0 + O1 + O2, NOB = (OT + 15) / 16;
  constexpr int LPT = 16 / CB;                      // lines per tile
  constexpr int NTILES = (NLINES + LPT - 1) / LPT;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane & 15, kr = lane >> 4;
  T bco[NOB][NKS];
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int o = ob * 16 + r, k = ks * 4 + kr;
      bco[ob][ks] = (o < OT && k < KT) ? cf(o, k) : T(0);
    }
  for (int t = wave; t < NTILES; t += 4) {
    const int line_a = t * LPT + r / CB, col_a = r % CB;
    T av[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int k = ks * 4 + kr;
      T v = T(0);
      if (line_a < NLINES) {
        if (k < K0) v = in0[line_slot<AX>(line_a, E0, k) * CB + col_a];
        else if (k < KT) v = in1[line_slot<AX>(line_a, E0, k - K0) * CB + col_a];
      }
      av[ks] = v;
    }
    typename M::V4 acc[NOB];
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) {
      acc[ob] = typename M::V4{T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) acc[ob] = M::op(av[ks], bco[ob][ks], acc[ob]);
    }
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int rr = kr * 4 + j;
        const int line = t * LPT + rr / CB, col = rr % CB;
        const int o = ob * 16 + r;
        if (line < NLINES && o < OT) {
          T* dst = o < O0 ? out0 : (o < O0 + O1 ? out1 : out2);
          const int oo = o < O0 ? o : (o < O0 + O1 ? o - O0 : o - O0 - O1);
          const int s = line_slot<AX>(line, E0, oo) * CB + col;
          dst[s] = post(line, o, col, acc[ob][j], dst[s]);
        }
      }
  }
}

template <typename T, int NP, int NQ, int CB, int MODE>
__global__ void __launch_bounds__(256) k_cell_mfma(CellArgs<T> A, const Tab1D<T>* __restrict__ tabp,
                                                   int ncoltiles, int nblocks) {
  constexpr int NL = NP * NP * NP;
  __shared__ T smem[3 * kSlots * CB];
  T* SA = smem;
  T* SB = smem + kSlots * CB;
  T* SC = smem + 2 * kSlots * CB;
  const Tab1D<T>& tab = *tabp;

  // XCD-aware remap: hardware dispatches block w to XCD w % 8
  const int w = blockIdx.x;
  const int per = nblocks / 8, rem = nblocks % 8;
  const int xcd = w % 8, idx = w / 8;
  const int logical = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + idx;
  const int ct = logical % ncoltiles;
  const int e = A.cells[logical / ncoltiles];
  const int n0 = ct * CB;

  const int ci = e % A.n0, cj = (e / A.n0) % A.n1, ck = e / (A.n0 * A.n1);
  const int p = NP - 1;
  const int Gx = A.n0 * p, Gy = A.n1 * p, Gz = A.n2 * p;
  auto dof = [&](int a, int b, int c) -> int64_t {
    int gx = ci * p + a; gx = gx >= Gx ? gx - Gx : gx;
    int gy = cj * p + b; gy = gy >= Gy ? gy - Gy : gy;
    int gz = ck * p + c; gz = gz >= Gz ? gz - Gz : gz;
    return (int64_t)gx + (int64_t)Gx * ((int64_t)gy + (int64_t)Gy * gz);
  };

  // extraction: gather the cell's CB columns into slab A
  for (int i = threadIdx.x; i < NL * CB; i += 256) {
    const int l = i / CB, col = i % CB;
    const int a = l % NP, b = (l / NP) % NP, c = l / (NP * NP);
    const int n = n0 + col;
    SA[slot(a, b, c) * CB + col] = n < A.ncols ? A.X[dof(a, b, c) * A.ldx + n] : T(0);
  }
  __syncthreads();

  auto store = [](int, int, int, T v, T) { return v; };
  T* OUT;
  if constexpr (MODE == kModeMass) {
    // x: Mx U -> C;  y: My C -> C;  z: detJ Mz C -> C
    mfma_pass<T, 0, CB, NP, 0, NP, 0, 0, NP * NP, NP>(
        SA, SA, SC, SC, SC, [&](int o, int k) { return tab.M1[o * NP + k]; }, store);
    __syncthreads();
    mfma_pass<T, 1, CB, NP, 0, NP, 0, 0, NP * NP, NP>(
        SC, SC, SC, SC, SC, [&](int o, int k) { return tab.M1[o * NP + k]; }, store);
    __syncthreads();
    mfma_pass<T, 2, CB, NP, 0, NP, 0, 0, NP * NP, NP>(
        SC, SC, SC, SC, SC, [&](int o, int k) { return tab.detJ * tab.M1[o * NP + k]; }, store);
    __syncthreads();
    OUT = SC;
  } else {
    // P1 x: [Bx; Kx; Mx] U -> B, C, A(in place)
    mfma_pass<T, 0, CB, NP, 0, NQ, NP, NP, NP * NP, NP>(
        SA, SA, SB, SC, SA,
        [&](int o, int k) {
          return o < NQ ? tab.B[o * NP + k] : (o < NQ + NP ? tab.K1[(o - NQ) * NP + k] : tab.M1[(o - NQ - NP) * NP + k]);
        },
        store);
    __syncthreads();
    // P2 y: By on slab B; lines (x in NQ, z in NP)
    mfma_pass<T, 1, CB, NP, 0, NQ, 0, 0, NQ * NP, NQ>(
        SB, SB, SB, SB, SB, [&](int o, int k) { return tab.B[o * NP + k]; }, store);
    __syncthreads();
    // P3 z: Bz, then V(q) W_q (minus lambda_n W_q); lines (x in NQ, y in NQ)
    {
      const T* Vw = A.Vw + (int64_t)e * (NQ * NQ * NQ);
      auto vpost = [&](int line, int o, int col, T v, T) {
        const int qa = line % NQ, qb = line / NQ;
        const int q = (o * NQ + qb) * NQ + qa;
        T s = Vw[q];
        if constexpr (MODE == kModeHRes) {
          const int n = n0 + col;
          s -= (n < A.ncols ? (T)A.lam[n] : T(0)) * A.W3[q];
        }
        return v * s;
      };
      mfma_pass<T, 2, CB, NP, 0, NQ, 0, 0, NQ * NQ, NQ>(
          SB, SB, SB, SB, SB, [&](int o, int k) { return tab.B[o * NP + k]; }, vpost);
    }
    __syncthreads();
    // P4 z: Bz^T
    mfma_pass<T, 2, CB, NQ, 0, NP, 0, 0, NQ * NQ, NQ>(
        SB, SB, SB, SB, SB, [&](int o, int k) { return tab.B[k * NP + o]; }, store);
    __syncthreads();
    // P5 y: By^T; lines (x in NQ, z in NP)
    mfma_pass<T, 1, CB, NQ, 0, NP, 0, 0, NQ * NP, NQ>(
        SB, SB, SB, SB, SB, [&](int o, int k) { return tab.B[k * NP + o]; }, store);
    __syncthreads();
    // P6 y: P = fx My C + fy Ky A -> C ; Q = My A -> A
    mfma_pass<T, 1, CB, NP, NP, NP, NP, 0, NP * NP, NP>(
        SC, SA, SC, SA, SA,
        [&](int o, int k) {
          if (o < NP) return k < NP ? tab.f[0] * tab.M1[o * NP + k] : tab.f[1] * tab.K1[o * NP + (k - NP)];
          return k < NP ? T(0) : tab.M1[(o - NP) * NP + (k - NP)];
        },
        store);
    __syncthreads();
    // P7 z: kinetic = Mz P + fz Kz Q -> C
    mfma_pass<T, 2, CB, NP, NP, NP, 0, 0, NP * NP, NP>(
        SC, SA, SC, SC, SC,
        [&](int o, int k) { return k < NP ? tab.M1[o * NP + k] : tab.f[2] * tab.K1[o * NP + (k - NP)]; },
        store);
    __syncthreads();
    // P8 x: Bx^T on slab B, accumulated into C
    mfma_pass<T, 0, CB, NQ, 0, NP, 0, 0, NP * NP, NP>(
        SB, SB, SC, SC, SC, [&](int o, int k) { return tab.B[k * NP + o]; },
        [](int, int, int, T v, T old) { return old + v; });
    __syncthreads();
    OUT = SC;
  }

  // assembly: colour-ordered read-modify-write, CB contiguous columns per DOF
  for (int i = threadIdx.x; i < NL * CB; i += 256) {
    const int l = i / CB, col = i % CB;
    const int a = l % NP, b = (l / NP) % NP, c = l / (NP * NP);
    const int n = n0 + col;
    if (n < A.ncols) {
      T* y = A.Y + dof(a, b, c) * A.ldy + n;
      *y = *y + A.alpha * OUT[slot(a, b, c) * CB + col];
    }
  }
}

namespace {

template <typename T>
const Tab1D<T>* dev_tab_m(const pawfe_op* op) {
  if constexpr (std::is_same<T, double>::value) return op->d.tab64; else return op->d.tab32;
}

template <typename T, int NP, int NQ, int CB>
pawfe_status run_cell_mfma(const pawfe_op* op, int mode, CellArgs<T> a, hipStream_t s) {
  const Tab1D<T>* tab = dev_tab_m<T>(op);
  const int ncoltiles = (a.ncols + CB - 1) / CB;
  for (int c = 0; c < op->ncolour; ++c) {
    const int c0 = op->colour_off[c], c1 = op->colour_off[c + 1];
    if (c1 == c0) continue;
    CellArgs<T> ac = a;
    ac.cells = op->d.cells_by_colour + c0;
    const int nblocks = (c1 - c0) * ncoltiles;
    const dim3 grid(nblocks), block(256);
    if (mode == kModeH)
      hipLaunchKernelGGL((k_cell_mfma<T, NP, NQ, CB, kModeH>), grid, block, 0, s, ac, tab, ncoltiles, nblocks);
    else if (mode == kModeHRes)
      hipLaunchKernelGGL((k_cell_mfma<T, NP, NQ, CB, kModeHRes>), grid, block, 0, s, ac, tab, ncoltiles, nblocks);
    else
      hipLaunchKernelGGL((k_cell_mfma<T, NP, NQ, CB, kModeMass>), grid, block, 0, s, ac, tab, ncoltiles, nblocks);
  }
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

}  // namespace

template <typename T>
pawfe_status launch_cell_mfma(const pawfe_op* op, int mode, const CellArgs<T>& a, hipStream_t s) {
  constexpr int CB = 8;
  switch (op->p) {
    case 2: return run_cell_mfma<T, 3, 4, CB>(op, mode, a, s);
    case 3: return run_cell_mfma<T, 4, 5, CB>(op, mode, a, s);
    case 4: return run_cell_mfma<T, 5, 6, CB>(op, mode, a, s);
    case 5: return run_cell_mfma<T, 6, 7, CB>(op, mode, a, s);
    case 6: return run_cell_mfma<T, 7, 8, CB>(op, mode, a, s);
    default: return fail(PAWFE_EUNSUPPORTED, "degree not compiled");
  }
}

template pawfe_status launch_cell_mfma<double>(const pawfe_op*, int, const CellArgs<double>&, hipStream_t);
template pawfe_status launch_cell_mfma<float>(const pawfe_op*, int, const CellArgs<float>&, hipStream_t);

}  // namespace pawfe
