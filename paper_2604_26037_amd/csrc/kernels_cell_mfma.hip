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
// LDS holds three slabs of 8x8x8 slots per column (slot (z*8 + y)*8 + x),
// zero-initialized.  Every pass walks all 64 padded lines of the slab with
// linear addressing and unconditional stores: rows and outputs beyond the
// true extents only ever meet zero coefficients, so they stay finite and
// never reach a true slot.  Each wave owns whole lines and reads all of a
// tile's inputs before writing its outputs, so the passes run in place.
//
// Passes (U = gathered cell values, slab A):
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

// Operand layouts (checked on gfx950): A[i][k] in lane i + 16k, B[k][j] in
// lane j + 16k; the 16x16 result D[i][j] sits in lane j + 16*g, element e,
// with i = 4g + e for f32 and i = g + 4e for f64.
template <typename T>
struct Mma;
template <>
struct Mma<float> {
  typedef float V4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V4 op(float a, float b, V4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int e) { return 4 * g + e; }
};
template <>
struct Mma<double> {
  typedef double V4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V4 op(double a, double b, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int e) { return g + 4 * e; }
};

constexpr int kSlots = 512;   // 8 x 8 x 8 padded slots per column

__device__ __forceinline__ int slot(int x, int y, int z) { return (z * 8 + y) * 8 + x; }

// Slot of padded line L at index 0 for a contraction along AX.  The line
// enumerates the other two axes (u, v) = (L % 8, L / 8), lower axis first.
template <int AX>
__device__ __forceinline__ int line_base(int L) {
  if constexpr (AX == 0) return L * 8;                         // (y, z)
  else if constexpr (AX == 1) return (L >> 3) * 64 + (L & 7);  // (x, z)
  else return L;                                               // (x, y)
}
template <int AX>
constexpr int kstride() { return AX == 0 ? 1 : (AX == 1 ? 8 : 64); }

}  // namespace

// One MFMA contraction pass over the 64 padded lines.
//   inputs:  NIN buffers; input k in [8b, 8b + 8) comes from in[b]
//   outputs: NG groups of 8; output o in [8g, 8g + 8) goes to out[g]
//   cf(o, k): stacked coefficient (0 outside the true extents)
//   post(L, o, col, value, old): the value stored
template <typename T, int AX, int CB, int NIN, int NG, class CF, class POST>
__device__ __forceinline__ void mfma_pass(T* const* in, T* const* out, CF cf, POST post) {
  using M = Mma<T>;
  constexpr int NKS = 2 * NIN;                 // k-steps of 4
  constexpr int NOB = (NG + 1) / 2;            // 16-wide output blocks
  constexpr int LPT = 16 / CB;                 // lines per tile
  constexpr int NT = 64 / LPT;                 // tiles per pass
  constexpr int KS = kstride<AX>() * CB;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane & 15, kr = lane >> 4;
  T bco[NOB][NKS];
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) bco[ob][ks] = cf(ob * 16 + r, ks * 4 + kr);
  const int la = r / CB, ca = r % CB;
#pragma unroll
  for (int it = 0; it < NT / 4; ++it) {
    const int t = wave + 4 * it;
    const int abase = line_base<AX>(t * LPT + la) * CB + ca;
    T av[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int k = ks * 4 + kr;            // from buffer ks / 2, index k % 8
      av[ks] = in[ks / 2][abase + (k & 7) * KS];
    }
    typename M::V4 acc[NOB];
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) {
      acc[ob] = typename M::V4{T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) acc[ob] = M::op(av[ks], bco[ob][ks], acc[ob]);
    }
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) {
      const int o = ob * 16 + r;
      if (2 * ob + 1 < NG || r < 8) {
        T* dst = out[o >> 3];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int rr = M::row(kr, e);
          const int L2 = t * LPT + rr / CB, c2 = rr % CB;
          const int s = line_base<AX>(L2) * CB + c2 + (o & 7) * KS;
          dst[s] = post(L2, o, c2, acc[ob][e], dst[s]);
        }
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

  // zero the padded slabs, then extraction (gather) of the cell's columns
  for (int i = threadIdx.x; i < 3 * kSlots * CB; i += 256) smem[i] = T(0);
  __syncthreads();
  for (int i = threadIdx.x; i < NL * CB; i += 256) {
    const int l = i / CB, col = i % CB;
    const int a = l % NP, b = (l / NP) % NP, c = l / (NP * NP);
    const int n = n0 + col;
    SA[slot(a, b, c) * CB + col] = n < A.ncols ? A.X[dof(a, b, c) * A.ldx + n] : T(0);
  }
  __syncthreads();

  auto store = [](int, int, int, T v, T) { return v; };
  // padded 1-D tables: zero outside the true extents
  auto Bm = [&](int q, int a) { return (q < NQ && a < NP) ? tab.B[q * NP + a] : T(0); };
  auto Km = [&](int a, int b) { return (a < NP && b < NP) ? tab.K1[a * NP + b] : T(0); };
  auto Mm = [&](int a, int b) { return (a < NP && b < NP) ? tab.M1[a * NP + b] : T(0); };
  T* OUT;
  if constexpr (MODE == kModeMass) {
    T* inA[1] = {SA};
    T* inC[1] = {SC};
    T* oC[1] = {SC};
    mfma_pass<T, 0, CB, 1, 1>(inA, oC, [&](int o, int k) { return Mm(o, k); }, store);
    __syncthreads();
    mfma_pass<T, 1, CB, 1, 1>(inC, oC, [&](int o, int k) { return Mm(o, k); }, store);
    __syncthreads();
    mfma_pass<T, 2, CB, 1, 1>(inC, oC, [&](int o, int k) { return tab.detJ * Mm(o, k); }, store);
    __syncthreads();
    OUT = SC;
  } else {
    T* inA[1] = {SA};
    T* inB[1] = {SB};
    T* inCA[2] = {SC, SA};
    T* oB[1] = {SB};
    T* oC[1] = {SC};
    T* oBCA[3] = {SB, SC, SA};
    T* oCA[2] = {SC, SA};
    // P1 x: [Bx; Kx; Mx] U
    mfma_pass<T, 0, CB, 1, 3>(
        inA, oBCA,
        [&](int o, int k) { return o < 8 ? Bm(o, k) : (o < 16 ? Km(o - 8, k) : Mm(o - 16, k)); }, store);
    __syncthreads();
    // P2 y: By
    mfma_pass<T, 1, CB, 1, 1>(inB, oB, [&](int o, int k) { return Bm(o, k); }, store);
    __syncthreads();
    // P3 z: Bz, then V(q) W_q (minus lambda_n W_q); lines are (qa, qb)
    {
      const T* Vw = A.Vw + (int64_t)e * (NQ * NQ * NQ);
      auto vpost = [&](int L, int o, int col, T v, T) {
        const int qa = L & 7, qb = L >> 3;
        if (qa >= NQ || qb >= NQ || o >= NQ) return T(0);
        const int q = (o * NQ + qb) * NQ + qa;
        T s = Vw[q];
        if constexpr (MODE == kModeHRes) {
          const int n = n0 + col;
          s -= (n < A.ncols ? (T)A.lam[n] : T(0)) * A.W3[q];
        }
        return v * s;
      };
      mfma_pass<T, 2, CB, 1, 1>(inB, oB, [&](int o, int k) { return Bm(o, k); }, vpost);
    }
    __syncthreads();
    // P4 z: Bz^T;  P5 y: By^T
    mfma_pass<T, 2, CB, 1, 1>(inB, oB, [&](int o, int k) { return Bm(k, o); }, store);
    __syncthreads();
    mfma_pass<T, 1, CB, 1, 1>(inB, oB, [&](int o, int k) { return Bm(k, o); }, store);
    __syncthreads();
    // P6 y: P = fx My C + fy Ky A -> C ; Q = My A -> A
    mfma_pass<T, 1, CB, 2, 2>(
        inCA, oCA,
        [&](int o, int k) {
          if (o < 8) return k < 8 ? tab.f[0] * Mm(o, k) : tab.f[1] * Km(o, k - 8);
          return k < 8 ? T(0) : Mm(o - 8, k - 8);
        },
        store);
    __syncthreads();
    // P7 z: kinetic = Mz P + fz Kz Q -> C
    mfma_pass<T, 2, CB, 2, 1>(
        inCA, oC, [&](int o, int k) { return k < 8 ? Mm(o, k) : tab.f[2] * Km(o, k - 8); }, store);
    __syncthreads();
    // P8 x: Bx^T on slab B, accumulated into C
    mfma_pass<T, 0, CB, 1, 1>(inB, oC, [&](int o, int k) { return Bm(k, o); },
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
  constexpr int CB = sizeof(T) == 8 ? 4 : 8;
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
