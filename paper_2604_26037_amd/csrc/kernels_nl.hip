// Non-local PAW terms, node-wise recurrence kernels and column reductions,
// for gfx950.
//
// Non-local action (eq. "FE nonlocal contribution"): the projector
// coefficients c_a = C^a^T s X (s = 1 or M_D^{-1}) are a long-K skinny
// reduction over the support nodes of each atom (K <= 19^3 rows, M = nproj,
// N = columns): one workgroup per (atom, 256-row chunk, 64-column tile),
// lane <-> column so every row read is one coalesced 512-byte segment and the
// C^a row is wave-uniform (scalar loads).  Partial sums go to a workspace and
// a second kernel adds the chunks of each atom in a fixed order (no atomics,
// deterministic).  The atom-block products (Delta x c, G^{ab} corrections)
// are tiny and run one thread per (projector, column).  The add-back
// sum_a C^a q_a on the support rows is a separate pass per atom colour
// (k_nl_fixup) after the node-wise kernels that stream the rows.

#include <cstdint>
#include <initializer_list>
#include <type_traits>

#include "kernels.h"

namespace pawfe {

namespace {

constexpr int kRowsPerWaveGroup = 4;   // waves per 256-thread block in row-wise kernels

// One workgroup per (item, 256-column slab): wave w owns the 64 columns
// [64 w, 64 w + 64) of the slab and walks all rows of the item, so no
// cross-wave reduction is needed.  Rows are taken kUnroll at a time with all
// their loads issued before the FMAs (memory-level parallelism).
constexpr int kUnroll = 8;

// Complex operators (CPLX): the columns are (re, im) pairs of the complex
// columns and c = C^H x mixes them: c[n] = sum Cr x[n] + s' Ci x[n ^ 1],
// s' = +1 on real and -1 on imaginary columns; the partner value comes from
// the neighbouring lane.
template <typename T, int NPJ, bool SCALE, bool CPLX = false>
__global__ void __launch_bounds__(256) k_nl_reduce(const T* __restrict__ X, int64_t ldx, int ncols,
                                                   const T* __restrict__ Minv,
                                                   const T* __restrict__ Cv, DeviceTables d,
                                                   double* __restrict__ part, const T* __restrict__ Cvi = nullptr) {
  const int item = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = (blockIdx.y * kRowsPerWaveGroup + w) * 64 + lane;
  if ((blockIdx.y * kRowsPerWaveGroup + w) * 64 >= ncols) return;   // wave-uniform
  const bool valid = n < ncols;
  const int nc = valid ? n : 0;
  const int a = d.item_atom[item];
  const int npj = d.nproj[a];
  const int r0 = d.item_row0[item], r1 = d.item_row1[item];
  const int noff = d.atom_noff[a], coff = d.atom_coff[a];
  T acc[NPJ];
#pragma unroll
  for (int al = 0; al < NPJ; ++al) acc[al] = T(0);
  // every load is unconditional (indices clamped into range, padded entries
  // multiply zeros or land in accumulators that are never stored), so the
  // loads of a batch are all in flight together
  auto rows = [&](auto full) {
    constexpr bool FULL = decltype(full)::value;
    for (int rb = r0; rb < r1; rb += kUnroll) {
      // the node list is padded by kUnroll entries, so the batch of indices
      // is one contiguous read; rows past r1 are masked below
      int I[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) I[u] = d.atom_nodes[noff + rb + u];
      T x[kUnroll], m[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        x[u] = __builtin_nontemporal_load(X + (int64_t)I[u] * ldx + nc);
        if constexpr (SCALE) m[u] = Minv[I[u]];
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        if constexpr (SCALE) x[u] *= m[u];
        if (rb + u >= r1 || !valid) x[u] = T(0);
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int r = rb + u < r1 ? rb + u : r1 - 1;
        const T* cr = Cv + coff + (int64_t)r * npj;
#pragma unroll
        for (int al = 0; al < NPJ; ++al) acc[al] += cr[FULL ? al : (al < npj ? al : npj - 1)] * x[u];
        if constexpr (CPLX) {
          // the shuffle runs in every lane before the sign is chosen: a
          // lane-permute reads 0 from lanes that are switched off, so it
          // must not sit inside a branch on the column parity
          const T xs = __shfl_xor(x[u], 1);
          const T xp = (n & 1) ? -xs : xs;
          const T* ci = Cvi + coff + (int64_t)r * npj;
#pragma unroll
          for (int al = 0; al < NPJ; ++al) acc[al] += ci[FULL ? al : (al < npj ? al : npj - 1)] * xp;
        }
      }
    }
  };
  if (npj == NPJ) rows(std::true_type{}); else rows(std::false_type{});
  if (!valid) return;
  const int po = d.item_poff[item];
#pragma unroll
  for (int al = 0; al < NPJ; ++al)
    if (al < npj) part[(int64_t)(po + al) * ncols + n] = (double)acc[al];
}

// The same reduction on the matrix cores (real operators, FP32 data), as
// the long-K skinny product  c[alpha][n] = sum_r C[r][alpha] x[r][n]:
// projectors alpha on the M side (two 16-blocks), support rows r on K,
// columns n on N.  Each wave owns 64 columns (four 16-column blocks).
//   FP32:   v_mfma_f32_16x16x4f32, 4 rows per step; A[i][k] (lane i + 16k) =
//           C[r0 + k][16 b + i], B[k][j] (lane j + 16k) = x[r0 + k][n + j].
//   bf16x3: v_mfma_f32_16x16x16_bf16, 16 rows per step; lane (i, g) holds rows
//           r0 + 4g + e (e = 0..3) of its projector / column; both operands
//           split as hi = bf16(v), lo = bf16(v - hi), the product taken as
//           lo*hi + hi*lo + hi*hi with FP32 accumulation.
// D[i][j] sits in lane j + 16g, element e, i = 4g + e.
typedef float RF4 __attribute__((ext_vector_type(4)));
typedef short RB4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short nl_bf16(float x, float& back) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  back = __uint_as_float(u & 0xFFFF0000u);
  return (short)(u >> 16);
}

template <bool SCALE, bool BF3>
__global__ void __launch_bounds__(256) k_nl_reduce_mfma(const float* __restrict__ X, int64_t ldx, int ncols,
                                                        const float* __restrict__ Minv,
                                                        const float* __restrict__ Cv, DeviceTables d,
                                                        double* __restrict__ part) {
  const int item = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nbase = (blockIdx.y * kRowsPerWaveGroup + w) * 64;
  if (nbase >= ncols) return;   // wave-uniform
  const int a = d.item_atom[item];
  const int npj = d.nproj[a];
  const int r0 = d.item_row0[item], r1 = d.item_row1[item];
  const int noff = d.atom_noff[a], coff = d.atom_coff[a];
  const int i = lane & 15, g = lane >> 4;
  RF4 acc[2][4];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[b][cb] = RF4{0.f, 0.f, 0.f, 0.f};
  constexpr int RPS = BF3 ? 16 : 4;            // support rows per step
  constexpr int RPL = BF3 ? 4 : 1;             // of them per lane
  for (int rb = r0; rb < r1; rb += RPS) {
    float xv[4][RPL], cv[2][RPL];
#pragma unroll
    for (int e = 0; e < RPL; ++e) {
      const int r = rb + g * RPL + e;
      const bool rin = r < r1;
      const int rr = rin ? r : r1 - 1;
      const int I = d.atom_nodes[noff + rr];
      const float m = SCALE ? Minv[I] : 1.0f;
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int n = nbase + 16 * cb + i;
        const float v = X[(int64_t)I * ldx + (n < ncols ? n : 0)];
        xv[cb][e] = (rin && n < ncols) ? v * m : 0.0f;
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int al = 16 * b + i;
        const float c = Cv[coff + (int64_t)rr * npj + (al < npj ? al : 0)];
        cv[b][e] = al < npj ? c : 0.0f;
      }
    }
    if constexpr (!BF3) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
          acc[b][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(cv[b][0], xv[cb][0], acc[b][cb], 0, 0, 0);
    } else {
      RB4 chi[2], clo[2], xhi[4], xlo[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          float h, dummy;
          chi[b][e] = nl_bf16(cv[b][e], h);
          clo[b][e] = nl_bf16(cv[b][e] - h, dummy);
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          float h, dummy;
          xhi[cb][e] = nl_bf16(xv[cb][e], h);
          xlo[cb][e] = nl_bf16(xv[cb][e] - h, dummy);
        }
      }
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          acc[b][cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(clo[b], xhi[cb], acc[b][cb], 0, 0, 0);
          acc[b][cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(chi[b], xlo[cb], acc[b][cb], 0, 0, 0);
          acc[b][cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(chi[b], xhi[cb], acc[b][cb], 0, 0, 0);
        }
    }
  }
  const int po = d.item_poff[item];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int n = nbase + 16 * cb + i;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int al = 16 * b + 4 * g + e;
        if (al < npj && n < ncols) part[(int64_t)(po + al) * ncols + n] = (double)acc[b][cb][e];
      }
    }
}

__global__ void __launch_bounds__(256) k_nl_final(const double* __restrict__ part, int ncols,
                                                  const int32_t* __restrict__ proj_atom,
                                                  const int32_t* __restrict__ proj_alpha, DeviceTables d,
                                                  double* __restrict__ c) {
  const int g = blockIdx.x;
  const int n = blockIdx.y * 256 + threadIdx.x;
  if (n >= ncols) return;
  const int a = proj_atom[g], al = proj_alpha[g];
  const int i0 = d.item_ptr[a], i1 = d.item_ptr[a + 1];
  // the partials of all items are independent loads: eight in flight at a
  // time, summed in item order
  double s = 0.0;
  for (int it = i0; it < i1; it += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = it + u < i1 ? it + u : i1 - 1;
      v[u] = part[(int64_t)(d.item_poff[k] + al) * ncols + n];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (it + u < i1) s += v[u];
  }
  c[(int64_t)g * ncols + n] = s;
}

// D1i (complex D1 = D1 + i D1i; complex operators): the columns are (re, im)
// pairs, D1 c mixes them: + s D1i c[n ^ 1], s = -1 on real, +1 on imaginary
// columns.
__global__ void __launch_bounds__(256) k_atom_mul(const double* __restrict__ D1, const double* __restrict__ D2,
                                                  const double* __restrict__ lam, double f,
                                                  const double* __restrict__ in, double* __restrict__ out,
                                                  int ncols, const int32_t* __restrict__ proj_atom,
                                                  const int32_t* __restrict__ proj_alpha, DeviceTables d,
                                                  const double* __restrict__ D1i) {
  const int g = blockIdx.x;
  const int n = blockIdx.y * 256 + threadIdx.x;
  if (n >= ncols) return;
  const int a = proj_atom[g], s = proj_alpha[g];
  const int npj = d.nproj[a], po = d.poff[a];
  const double* r1 = D1 + d.poff2[a] + s * npj;
  double acc = 0.0, acc2 = 0.0;
  for (int t = 0; t < npj; ++t) acc += r1[t] * in[(int64_t)(po + t) * ncols + n];
  if (D1i) {
    const double* ri = D1i + d.poff2[a] + s * npj;
    double ai = 0.0;
    for (int t = 0; t < npj; ++t) ai += ri[t] * in[(int64_t)(po + t) * ncols + (n ^ 1)];
    acc += (n & 1) ? ai : -ai;
  }
  if (D2) {
    const double* r2 = D2 + d.poff2[a] + s * npj;
    for (int t = 0; t < npj; ++t) acc2 += r2[t] * in[(int64_t)(po + t) * ncols + n];
    acc -= lam[n] * acc2;
  }
  out[(int64_t)g * ncols + n] = f * acc;
}

__global__ void __launch_bounds__(256) k_atom_gcorr(const double* __restrict__ c, const double* __restrict__ dv,
                                                    double* __restrict__ out, int ncols,
                                                    const int32_t* __restrict__ proj_atom,
                                                    const int32_t* __restrict__ proj_alpha, DeviceTables d) {
  const int g = blockIdx.x;
  const int n = blockIdx.y * 256 + threadIdx.x;
  if (n >= ncols) return;
  const int a = proj_atom[g], s = proj_alpha[g];
  double acc = c[(int64_t)g * ncols + n];
  for (int k = d.gp_ptr[a]; k < d.gp_ptr[a + 1]; ++k) {
    const int b = d.gp_b[k], nb = d.nproj[b], pb = d.poff[b];
    const double* G = d.Gvals + d.gp_off[k] + s * nb;
#pragma unroll 6
    for (int u = 0; u < nb; ++u) acc -= G[u] * dv[(int64_t)(pb + u) * ncols + n];
    if (d.Gvals_im) {   // complex operators: (re, im) column pairs mix
      const double* Gi = d.Gvals_im + d.gp_off[k] + s * nb;
      double ai = 0.0;
      for (int u = 0; u < nb; ++u) ai += Gi[u] * dv[(int64_t)(pb + u) * ncols + (n ^ 1)];
      acc -= (n & 1) ? ai : -ai;
    }
  }
  out[(int64_t)g * ncols + n] = acc;
}

// Projector part of the fused Chebyshev step (per projector row g, column n;
// nw = -w, w the vector whose C w the step still owes R_X):
//   v  = nw_prev + d                  (the step's fix-up R_Y -= C v)
//   nw = -q + ac d + zz d_prev        (q already scaled by a)
// and, on row 0, lamX = a lamY lam_in - ac lamY - zz lamX.  nw_prev and
// d_prev may be null (zero: the first step); q null: v only, no nw, no lambda.
__global__ void __launch_bounds__(256) k_step_combine(int npj, int ncols, const double* __restrict__ q,
                                                      const double* __restrict__ dv,
                                                      const double* __restrict__ dprev,
                                                      const double* __restrict__ nwprev, double* __restrict__ v,
                                                      double* __restrict__ nw, double* __restrict__ lamX,
                                                      const double* __restrict__ lamY,
                                                      const double* __restrict__ lam_in, double a, double ac,
                                                      double zz) {
  const int g = blockIdx.x;
  const int n = blockIdx.y * 256 + threadIdx.x;
  if (n >= ncols) return;
  if (g < npj) {
    const int64_t i = (int64_t)g * ncols + n;
    const double d = dv[i];
    v[i] = (nwprev ? nwprev[i] : 0.0) + d;
    if (q) nw[i] = -q[i] + ac * d + (dprev ? zz * dprev[i] : 0.0);
  }
  if (g == 0 && q) lamX[n] = a * lamY[n] * lam_in[n] - ac * lamY[n] - zz * lamX[n];
}

// Row-wise kernels.  A 256-thread block is 4 waves; a wave takes R
// consecutive DOF rows at a time, so the row index and its projector entries
// are wave-uniform (scalar loads).  Each lane owns V consecutive columns:
// with V = 16 / sizeof(element) every access of the streamed blocks is one
// 16-byte load or store per lane.  All loads of the R rows are issued before
// the first store, which keeps enough bytes in flight per CU to cover the HBM
// latency.  The grid is persistent (a fixed multiple of 8 workgroups): work
// item = (group of 4 R rows, column tile); XCD x takes the x-th contiguous
// eighth of the items (block w runs on XCD w % 8) and its workgroups stride
// through it, so each XCD streams one slab of rows and the projector
// coefficients of the atoms in that slab stay in its L2.  The host takes
// V = 1 when a leading dimension, a base pointer or the column count does
// not allow 16-byte accesses.
constexpr int kRowsPerWave = 4;
constexpr int kPersistBlocks = 2048;

template <typename T, int V>
struct Lanes {
  T v[V];
};

// The row kernels touch each streamed element once per launch: their loads
// and stores carry the non-temporal hint, so the stream does not displace
// cached data (the projector tables, the other stream's working set).
template <int V, typename T>
__device__ __forceinline__ Lanes<T, V> vld(const T* p) {
  Lanes<T, V> r;
  if constexpr (V == 1) {
    r.v[0] = __builtin_nontemporal_load(p);
  } else {
    typedef T VT __attribute__((ext_vector_type(V)));
    const VT x = __builtin_nontemporal_load(reinterpret_cast<const VT*>(p));
#pragma unroll
    for (int i = 0; i < V; ++i) r.v[i] = x[i];
  }
  return r;
}

template <int V, typename T>
__device__ __forceinline__ void vst(T* p, const Lanes<T, V>& r) {
  if constexpr (V == 1) {
    __builtin_nontemporal_store(r.v[0], p);
  } else {
    typedef T VT __attribute__((ext_vector_type(V)));
    VT x;
#pragma unroll
    for (int i = 0; i < V; ++i) x[i] = r.v[i];
    __builtin_nontemporal_store(x, reinterpret_cast<VT*>(p));
  }
}

// Persistent loop; inside, I0 is the wave's first row and n its first
// column (both valid), the rows are I0 + [0, R) below M.  Row groups of 4 R
// rows are split into 8 contiguous ranges, one per XCD; the workgroups of an
// XCD stride through its range and sweep the column tiles of each group.
#define ROWS_BEGIN(V, R)                                                                         \
  const int lane_ = threadIdx.x & 63;                                                            \
  const int wv_ = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);                              \
  const int xcd_ = blockIdx.x & 7;                                                               \
  const int ngroups_ = (int)((M + kRowsPerWaveGroup * (R) - 1) / (kRowsPerWaveGroup * (R)));     \
  const int ge_ = (int)((int64_t)ngroups_ * (xcd_ + 1) / 8);                                     \
  for (int grp_ = (int)((int64_t)ngroups_ * xcd_ / 8) + (blockIdx.x >> 3); grp_ < ge_;           \
       grp_ += (gridDim.x >> 3)) {                                                               \
    const int64_t I0 = ((int64_t)grp_ * kRowsPerWaveGroup + wv_) * (R);                          \
    for (int ct_ = 0; ct_ < ncoltiles; ++ct_) {                                                  \
      const int n = (ct_ * 64 + lane_) * (V);                                                    \
      if (n < ncols && I0 < M) {
#define ROWS_END \
  }              \
  }              \
  }

// row I0 + r clamped into range (loads only; its result is not stored)
#define ROW_CLAMP(r) ((I0 + (r) < M) ? I0 + (r) : M - 1)

// Streaming parts of the node-wise operations (local terms only); the
// projector terms sum_a C^a v_a at the support nodes are added afterwards by
// k_nl_fixup, atom colour by atom colour.

template <typename T, int V, int R>
__global__ void __launch_bounds__(256) k_node_zero(int64_t M, int ncols, int ncoltiles, T* __restrict__ Y,
                                                   int64_t ldy) {
  ROWS_BEGIN(V, R)
  Lanes<T, V> z;
#pragma unroll
  for (int i = 0; i < V; ++i) z.v[i] = T(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (I0 + r >= M) break;
    vst<V>(Y + (I0 + r) * ldy + n, z);
  }
  ROWS_END
}

// Y = M_D^{-1} X
template <typename T, int V, int R>
__global__ void __launch_bounds__(256) k_node_sinv(int64_t M, int ncols, int ncoltiles,
                                                   const T* __restrict__ X, int64_t ldx, T* __restrict__ Y,
                                                   int64_t ldy, const T* __restrict__ Minv) {
  ROWS_BEGIN(V, R)
  Lanes<T, V> x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = vld<V>(X + ROW_CLAMP(r) * ldx + n);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t I = I0 + r;
    if (I >= M) break;
    const T m = Minv[I];
    Lanes<T, V> y;
#pragma unroll
    for (int i = 0; i < V; ++i) y.v[i] = m * x[r].v[i];
    vst<V>(Y + I * ldy + n, y);
  }
  ROWS_END
}

// T = M_D^{-1} R_Y;  R_X <- -a c R_Y - zeta zeta' R_X + a Y Lambda_Y
template <typename TR, int V, int R>
__global__ void __launch_bounds__(256) k_node_cheb(int64_t M, int ncols, int ncoltiles,
                                                   const TR* __restrict__ RY,
                                                   TR* __restrict__ RX, TR* __restrict__ Tb, int64_t ld,
                                                   const double* __restrict__ Y, int64_t ldy,
                                                   const double* __restrict__ lamY, double* __restrict__ lamX,
                                                   const double* __restrict__ lam_in, double a, double ac,
                                                   double zz, const TR* __restrict__ Minv) {
  ROWS_BEGIN(V, R)
  Lanes<TR, V> ry[R], rx[R];
  Lanes<double, V> y[R];
  TR m[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t I = ROW_CLAMP(r);
    ry[r] = vld<V>(RY + I * ld + n);
    rx[r] = vld<V>(RX + I * ld + n);
    y[r] = vld<V>(Y + I * ldy + n);
    m[r] = Minv[I];
  }
  double ly[V];
#pragma unroll
  for (int i = 0; i < V; ++i) ly[i] = a * lamY[n + i];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t I = I0 + r;
    if (I >= M) break;
    Lanes<TR, V> t, o;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      t.v[i] = m[r] * ry[r].v[i];
      // recurrence part in TR arithmetic, residual correction a Y lamY in FP64
      const TR part = (TR)(-ac) * ry[r].v[i] - (TR)zz * rx[r].v[i];
      o.v[i] = (TR)((double)part + y[r].v[i] * ly[i]);
    }
    vst<V>(Tb + I * ld + n, t);
    vst<V>(RX + I * ld + n, o);
    if (I == 0) {
#pragma unroll
      for (int i = 0; i < V; ++i)
        lamX[n + i] = a * lamY[n + i] * lam_in[n + i] - ac * lamY[n + i] - zz * lamX[n + i];
    }
  }
  ROWS_END
}

// Xout = M_D^{-1} R_Y + X Lambda_Y
template <typename TR, int V, int R>
__global__ void __launch_bounds__(256) k_node_finalize(int64_t M, int ncols, int ncoltiles,
                                                       const TR* __restrict__ RY, int64_t ld,
                                                       const double* __restrict__ X, int64_t ldx,
                                                       const double* __restrict__ lamY, double* __restrict__ Xo,
                                                       int64_t ldo, const TR* __restrict__ Minv) {
  ROWS_BEGIN(V, R)
  Lanes<TR, V> ry[R];
  Lanes<double, V> x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t I = ROW_CLAMP(r);
    ry[r] = vld<V>(RY + I * ld + n);
    x[r] = vld<V>(X + I * ldx + n);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t I = I0 + r;
    if (I >= M) break;
    const TR m = Minv[I];
    Lanes<double, V> o;
#pragma unroll
    for (int i = 0; i < V; ++i) o.v[i] = (double)(m * ry[r].v[i]) + x[r].v[i] * lamY[n + i];
    vst<V>(Xo + I * ldo + n, o);
  }
  ROWS_END
}

// Projector add-back on the support nodes, for the items of one atom colour
// (atoms of a colour share no node, so the read-modify-writes never meet):
//   out1[I] += s1 * w_I * sum_alpha C^a[I][alpha] v1_a[alpha][n]
//   out2[I] +=              sum_alpha C^a[I][alpha] v2_a[alpha][n]   (if out2)
// with w_I = M_D^{-1}[I] if minv, else 1.  One workgroup per (item, 256
// columns): thread <-> column, the atom's coefficient vectors for that column
// sit in registers, the item's rows (<= 64) are walked kFixUnroll at a time
// with all loads issued first.
constexpr int kFixUnroll = 8;

// CPLX (complex operators): (re, im) column pairs, C v mixes them:
// + s Ci v[n ^ 1], s = -1 on real and +1 on imaginary columns (partner value
// from the neighbouring lane).
template <typename TR, typename TO1, int NPJ, bool MINV, bool HAS2, bool CPLX = false>
__global__ void __launch_bounds__(256) k_nl_fixup(const int32_t* __restrict__ fatom,
                                                  const int32_t* __restrict__ frow0,
                                                  const int32_t* __restrict__ frow1, int ncols,
                                                  const double* __restrict__ v1, double s1,
                                                  TO1* __restrict__ out1, int64_t ld1,
                                                  const double* __restrict__ v2, TR* __restrict__ out2,
                                                  int64_t ld2, const TR* __restrict__ Minv,
                                                  const TR* __restrict__ Cv, DeviceTables d,
                                                  const TR* __restrict__ Cvi = nullptr) {
  const int n = blockIdx.y * 256 + threadIdx.x;
  if (n >= ncols) return;
  const int a = fatom[blockIdx.x];
  const int r0 = frow0[blockIdx.x], r1 = frow1[blockIdx.x];
  const int npj = d.nproj[a], po = d.poff[a];
  const int noff = d.atom_noff[a], coff = d.atom_coff[a];
  // All loads are unconditional (indices clamped into range), so they are in
  // flight together; an atom with exactly NPJ projectors takes the path with
  // plain indices (wide scalar loads of its C rows).
  auto body = [&](auto full) {
    constexpr bool FULL = decltype(full)::value;
    auto idx = [&](int al) { return FULL ? al : (al < npj ? al : npj - 1); };
    TR w1[NPJ], w2[NPJ], p1[CPLX ? NPJ : 1], p2[CPLX ? NPJ : 1];
#pragma unroll
    for (int al = 0; al < NPJ; ++al) {
      const double x1 = v1[(int64_t)(po + idx(al)) * ncols + n];
      w1[al] = (FULL || al < npj) ? (TR)(s1 * x1) : TR(0);
      if constexpr (HAS2) {
        const double x2 = v2[(int64_t)(po + idx(al)) * ncols + n];
        w2[al] = (FULL || al < npj) ? (TR)x2 : TR(0);
      }
    }
    if constexpr (CPLX) {
      const TR sg = (n & 1) ? TR(1) : TR(-1);
#pragma unroll
      for (int al = 0; al < NPJ; ++al) {
        p1[al] = sg * __shfl_xor(w1[al], 1);
        if constexpr (HAS2) p2[al] = sg * __shfl_xor(w2[al], 1);
      }
    }
    for (int rb = r0; rb < r1; rb += kFixUnroll) {
      int I[kFixUnroll];
      TO1 o1[kFixUnroll];
      TR o2[kFixUnroll], c1[kFixUnroll], c2[kFixUnroll];
#pragma unroll
      for (int u = 0; u < kFixUnroll; ++u) I[u] = d.atom_nodes[noff + rb + u];   // list padded
#pragma unroll
      for (int u = 0; u < kFixUnroll; ++u) {   // rows touched once: non-temporal
        o1[u] = __builtin_nontemporal_load(out1 + (int64_t)I[u] * ld1 + n);
        if constexpr (HAS2) o2[u] = __builtin_nontemporal_load(out2 + (int64_t)I[u] * ld2 + n);
      }
#pragma unroll
      for (int u = 0; u < kFixUnroll; ++u) {
        const int r = rb + u < r1 ? rb + u : r1 - 1;
        const TR* cr = Cv + coff + (int64_t)r * npj;
        c1[u] = c2[u] = TR(0);
#pragma unroll
        for (int al = 0; al < NPJ; ++al) {
          const TR cv = cr[idx(al)];
          c1[u] += cv * w1[al];
          if constexpr (HAS2) c2[u] += cv * w2[al];
        }
        if constexpr (CPLX) {
          const TR* ci = Cvi + coff + (int64_t)r * npj;
#pragma unroll
          for (int al = 0; al < NPJ; ++al) {
            const TR cv = ci[idx(al)];
            c1[u] += cv * p1[al];
            if constexpr (HAS2) c2[u] += cv * p2[al];
          }
        }
        if constexpr (MINV) c1[u] *= Minv[I[u]];
      }
#pragma unroll
      for (int u = 0; u < kFixUnroll; ++u) {
        if (rb + u >= r1) break;
        __builtin_nontemporal_store(o1[u] + (TO1)c1[u], out1 + (int64_t)I[u] * ld1 + n);
        if constexpr (HAS2) __builtin_nontemporal_store(o2[u] + c2[u], out2 + (int64_t)I[u] * ld2 + n);
      }
    }
  };
  if (npj == NPJ) body(std::true_type{}); else body(std::false_type{});
}



template <typename TR, int V, int R>
__global__ void __launch_bounds__(256) k_cheb_init(int64_t M, int ncols, int ncoltiles,
                                                   const double* __restrict__ Y,
                                                   int64_t ldy, TR* __restrict__ RY, TR* __restrict__ RX,
                                                   int64_t ld, double f, double c,
                                                   const double* __restrict__ lam_in, double* __restrict__ lamY,
                                                   double* __restrict__ lamX) {
  ROWS_BEGIN(V, R)
  Lanes<double, V> y[R];
#pragma unroll
  for (int r = 0; r < R; ++r) y[r] = vld<V>(Y + ROW_CLAMP(r) * ldy + n);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t I = I0 + r;
    if (I >= M) break;
    Lanes<TR, V> ry, z;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      ry.v[i] = (TR)(f * y[r].v[i]);
      z.v[i] = TR(0);
    }
    vst<V>(RY + I * ld + n, ry);
    vst<V>(RX + I * ld + n, z);
    if (I == 0) {
#pragma unroll
      for (int i = 0; i < V; ++i) {
        lamY[n + i] = f * (lam_in[n + i] - c);
        lamX[n + i] = 1.0;
      }
    }
  }
  ROWS_END
}

template <int V, int R>
__global__ void __launch_bounds__(256) k_copy_cols(int64_t M, int ncols, int ncoltiles,
                                                   const double* __restrict__ X, int64_t ldx,
                                                   double* __restrict__ Y, int64_t ldy) {
  ROWS_BEGIN(V, R)
  Lanes<double, V> x[R];
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = vld<V>(X + ROW_CLAMP(r) * ldx + n);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (I0 + r >= M) break;
    vst<V>(Y + (I0 + r) * ldy + n, x[r]);
  }
  ROWS_END
}

template <typename T>
__global__ void k_fill(T* __restrict__ Y, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Y[i] = v;
}

// partial[chunk][n] = sum_{i in chunk} A[i][n] B[i][n]
__global__ void __launch_bounds__(256) k_coldot(const double* __restrict__ A, int64_t lda,
                                                const double* __restrict__ B, int64_t ldb, int64_t nrows,
                                                int ncols, int64_t rows_per_chunk, double* __restrict__ partial) {
  __shared__ double red[kRowsPerWaveGroup][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = blockIdx.y * 64 + lane;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r1 = (r0 + rows_per_chunk < nrows) ? r0 + rows_per_chunk : nrows;
  double acc = 0.0;
  if (n < ncols)
    for (int64_t i = r0 + w; i < r1; i += kRowsPerWaveGroup) acc += A[i * lda + n] * B[i * ldb + n];
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0 && n < ncols)
    partial[(int64_t)blockIdx.x * ncols + n] = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

__global__ void __launch_bounds__(256) k_coldot_final(const double* __restrict__ partial, int nchunks, int ncols,
                                                      double* __restrict__ out, const double* __restrict__ w,
                                                      int sqrt_out, int scalar) {
  __shared__ double red[256];
  if (!scalar) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= ncols) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += partial[(int64_t)c * ncols + n];
    out[n] = sqrt_out ? sqrt(s) : s;
    return;
  }
  double s = 0.0;
  for (int n = threadIdx.x; n < ncols; n += 256) {
    double t = 0.0;
    for (int c = 0; c < nchunks; ++c) t += partial[(int64_t)c * ncols + n];
    s += (w ? w[n] : 1.0) * t;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] += red[0];
}

__global__ void k_grad_dh(const double* __restrict__ c, int ncols, const double* __restrict__ occ,
                          const int32_t* __restrict__ ent_atom, const int32_t* __restrict__ ent_s,
                          const int32_t* __restrict__ ent_t, int nent, DeviceTables d, double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nent) return;
  const int a = ent_atom[k], s = ent_s[k], t = ent_t[k];
  const int po = d.poff[a], npj = d.nproj[a];
  const double* ps = c + (int64_t)(po + s) * ncols;
  const double* pt = c + (int64_t)(po + t) * ncols;
  double acc = 0.0;
  for (int n = 0; n < ncols; ++n) acc += (occ ? occ[n] : 1.0) * ps[n] * pt[n];
  out[d.poff2[a] + s * npj + t] = acc;
}

struct RowGrid {
  int ncoltiles;
  dim3 grid;
};
// Persistent grid: the workgroups of kernel K that are resident at once
// (so none waits for a second round), a multiple of 8, capped by the work.
template <typename K>
inline int resident_blocks(K kernel) {
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
    ncu = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess || per_cu <= 0)
    per_cu = 1;
  return std::max(8, ncu * per_cu / 8 * 8);
}
template <auto K>
inline RowGrid row_grid(int64_t M, int ncols, int V, int R) {
  static const int resident = resident_blocks(K);
  RowGrid g;
  g.ncoltiles = (ncols + 64 * V - 1) / (64 * V);
  const int64_t ngroups = (M + kRowsPerWaveGroup * R - 1) / (kRowsPerWaveGroup * R);
  g.grid = dim3((unsigned)std::max<int64_t>(8, std::min<int64_t>(resident, (ngroups + 7) / 8 * 8)));
  return g;
}

// True when V columns per lane are allowed: ncols a multiple of V and every
// (base pointer, leading dimension) pair 16-byte aligned row by row.
struct Strided {
  const void* p;
  int64_t ld;
};
inline bool vec_ok(int V, int ncols, std::initializer_list<Strided> xs) {
  if (ncols % V) return false;
  for (const Strided& x : xs)
    if ((reinterpret_cast<uintptr_t>(x.p) & 15) || x.ld % V) return false;
  return true;
}

template <typename T>
const T* pick(const double* d64, const float* d32) {
  if constexpr (std::is_same<T, double>::value) return d64; else return d32;
}

}  // namespace

// ---------------------------------------------------------------------------

template <typename T>
pawfe_status launch_nl_reduce(const pawfe_op* op, const T* X, int64_t ldx, int ncols, bool scale_minv,
                              double* part, double* c, hipStream_t s, bool bf3) {
  if (op->natoms == 0 || ncols <= 0) return PAWFE_OK;
  const T* Cv = pick<T>(op->d.Cvals, op->d.Cvals_f);
  const T* Minv = pick<T>(op->d.Minv, op->d.Minv_f);
  const T* Cvi = pick<T>(op->d.Cvals_im, op->d.Cvals_im_f);
  const dim3 grid(op->nitems, (ncols + 255) / 256), block(256);
  if constexpr (std::is_same<T, float>::value) {
    if (!op->cplx) {   // real operators in FP32: the matrix-core reduction
      auto go = [&](auto scale, auto b3) {
        constexpr bool SC = decltype(scale)::value, B3 = decltype(b3)::value;
        hipLaunchKernelGGL((k_nl_reduce_mfma<SC, B3>), grid, block, 0, s, X, ldx, ncols, Minv, Cv, op->d, part);
      };
      if (scale_minv) {
        if (bf3) go(std::true_type{}, std::true_type{}); else go(std::true_type{}, std::false_type{});
      } else {
        if (bf3) go(std::false_type{}, std::true_type{}); else go(std::false_type{}, std::false_type{});
      }
      const dim3 g2(op->npj_total, (ncols + 255) / 256);
      hipLaunchKernelGGL(k_nl_final, g2, block, 0, s, part, ncols, op->d_proj_atom, op->d_proj_alpha, op->d, c);
      PAWFE_HIP(hipGetLastError());
      return PAWFE_OK;
    }
  }
  auto go = [&](auto scale, auto cplx) {
    constexpr bool SC = decltype(scale)::value, CX = decltype(cplx)::value;
    if (op->npj_max <= 8)
      hipLaunchKernelGGL((k_nl_reduce<T, 8, SC, CX>), grid, block, 0, s, X, ldx, ncols, Minv, Cv, op->d, part, Cvi);
    else if (op->npj_max <= 18)
      hipLaunchKernelGGL((k_nl_reduce<T, 18, SC, CX>), grid, block, 0, s, X, ldx, ncols, Minv, Cv, op->d, part, Cvi);
    else
      hipLaunchKernelGGL((k_nl_reduce<T, 32, SC, CX>), grid, block, 0, s, X, ldx, ncols, Minv, Cv, op->d, part, Cvi);
  };
  if (op->cplx) {
    if (scale_minv) go(std::true_type{}, std::true_type{}); else go(std::false_type{}, std::true_type{});
  } else {
    if (scale_minv) go(std::true_type{}, std::false_type{}); else go(std::false_type{}, std::false_type{});
  }
  const dim3 g2(op->npj_total, (ncols + 255) / 256);
  hipLaunchKernelGGL(k_nl_final, g2, block, 0, s, part, ncols, op->d_proj_atom, op->d_proj_alpha, op->d, c);
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}
template pawfe_status launch_nl_reduce<double>(const pawfe_op*, const double*, int64_t, int, bool, double*, double*,
                                               hipStream_t, bool);
template pawfe_status launch_nl_reduce<float>(const pawfe_op*, const float*, int64_t, int, bool, double*, double*,
                                              hipStream_t, bool);

pawfe_status launch_atom_mul(const pawfe_op* op, const double* D1, const double* D2, const double* lam, double f,
                             const double* in, double* out, int ncols, hipStream_t s, const double* D1i) {
  if (op->natoms == 0 || ncols <= 0) return PAWFE_OK;
  const dim3 grid(op->npj_total, (ncols + 255) / 256), block(256);
  hipLaunchKernelGGL(k_atom_mul, grid, block, 0, s, D1, D2, lam, f, in, out, ncols, op->d_proj_atom,
                     op->d_proj_alpha, op->d, D1i);
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

__global__ void k_dup_pairs(const double* __restrict__ in, double* __restrict__ out, int n) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < n) {
    const double v = in[j];
    out[2 * j] = v;
    out[2 * j + 1] = v;
  }
}

pawfe_status launch_dup_pairs(const double* in, double* out, int n, hipStream_t s) {
  if (n <= 0) return PAWFE_OK;
  hipLaunchKernelGGL(k_dup_pairs, dim3((n + 255) / 256), dim3(256), 0, s, in, out, n);
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

pawfe_status launch_step_combine(const pawfe_op* op, const double* q, const double* d, const double* dprev,
                                 const double* nwprev, double* v, double* nw, double* lamX, const double* lamY,
                                 const double* lam_in, double a, double ac, double zz, int ncols, hipStream_t s) {
  if (ncols <= 0) return PAWFE_OK;
  if (op->npj_total == 0 && !q) return PAWFE_OK;
  const dim3 grid(std::max(op->npj_total, 1), (ncols + 255) / 256), block(256);
  hipLaunchKernelGGL(k_step_combine, grid, block, 0, s, op->npj_total, ncols, q, d, dprev, nwprev, v, nw, lamX, lamY,
                     lam_in, a, ac, zz);
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

pawfe_status launch_atom_gcorr(const pawfe_op* op, const double* c, const double* dv, double* out, int ncols,
                               hipStream_t s) {
  if (op->natoms == 0 || ncols <= 0) return PAWFE_OK;
  const dim3 grid(op->npj_total, (ncols + 255) / 256), block(256);
  hipLaunchKernelGGL(k_atom_gcorr, grid, block, 0, s, c, dv, out, ncols, op->d_proj_atom, op->d_proj_alpha, op->d);
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

// out1 += s1 w C v1 (w = M_D^{-1} if MINV), out2 += C v2 (if HAS2), atom colour by colour
template <typename TR, typename TO1, bool MINV, bool HAS2>
pawfe_status nl_fixup(const pawfe_op* op, int ncols, const double* v1, double s1, TO1* out1, int64_t ld1,
                      const double* v2, TR* out2, int64_t ld2, hipStream_t s) {
  if (op->natoms == 0 || ncols <= 0) return PAWFE_OK;
  const TR* Cv = pick<TR>(op->d.Cvals, op->d.Cvals_f);
  const TR* Cvi = pick<TR>(op->d.Cvals_im, op->d.Cvals_im_f);
  const TR* Minv = pick<TR>(op->d.Minv, op->d.Minv_f);
  for (int c = 0; c < op->natom_colours; ++c) {
    const int i0 = op->fix_colour_off[c], i1 = op->fix_colour_off[c + 1];
    if (i1 == i0) continue;
    const dim3 grid(i1 - i0, (ncols + 255) / 256), block(256);
    const int32_t *fa = op->d.fix_atom + i0, *f0 = op->d.fix_row0 + i0, *f1 = op->d.fix_row1 + i0;
    auto go = [&](auto cplx) {
      constexpr bool CX = decltype(cplx)::value;
      if (op->npj_max <= 8)
        hipLaunchKernelGGL((k_nl_fixup<TR, TO1, 8, MINV, HAS2, CX>), grid, block, 0, s, fa, f0, f1, ncols, v1, s1,
                           out1, ld1, v2, out2, ld2, Minv, Cv, op->d, Cvi);
      else if (op->npj_max <= 18)
        hipLaunchKernelGGL((k_nl_fixup<TR, TO1, 18, MINV, HAS2, CX>), grid, block, 0, s, fa, f0, f1, ncols, v1, s1,
                           out1, ld1, v2, out2, ld2, Minv, Cv, op->d, Cvi);
      else
        hipLaunchKernelGGL((k_nl_fixup<TR, TO1, 32, MINV, HAS2, CX>), grid, block, 0, s, fa, f0, f1, ncols, v1, s1,
                           out1, ld1, v2, out2, ld2, Minv, Cv, op->d, Cvi);
    };
    if (op->cplx) go(std::true_type{}); else go(std::false_type{});
  }
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

template <typename T>
pawfe_status launch_node_nl_init(const pawfe_op* op, const double* q, int ncols, T* Y, int64_t ldy, hipStream_t s) {
  if (ncols <= 0) return PAWFE_OK;
  constexpr int V = 16 / sizeof(T);
  if (vec_ok(V, ncols, {{Y, ldy}})) {
    const RowGrid g = row_grid<k_node_zero<T, V, kRowsPerWave>>(op->M, ncols, V, kRowsPerWave);
    hipLaunchKernelGGL((k_node_zero<T, V, kRowsPerWave>), g.grid, dim3(256), 0, s, op->M, ncols, g.ncoltiles, Y, ldy);
  } else {
    const RowGrid g = row_grid<k_node_zero<T, 1, kRowsPerWave>>(op->M, ncols, 1, kRowsPerWave);
    hipLaunchKernelGGL((k_node_zero<T, 1, kRowsPerWave>), g.grid, dim3(256), 0, s, op->M, ncols, g.ncoltiles, Y, ldy);
  }
  PAWFE_HIP(hipGetLastError());
  return nl_fixup<T, T, false, false>(op, ncols, q, 1.0, Y, ldy, nullptr, (T*)nullptr, 0, s);
}
template pawfe_status launch_node_nl_init<double>(const pawfe_op*, const double*, int, double*, int64_t, hipStream_t);
template pawfe_status launch_node_nl_init<float>(const pawfe_op*, const double*, int, float*, int64_t, hipStream_t);

template <typename T>
pawfe_status launch_node_fixup(const pawfe_op* op, const double* v1, double s1, int ncols, T* out1, int64_t ld1,
                               hipStream_t s) {
  return nl_fixup<T, T, false, false>(op, ncols, v1, s1, out1, ld1, nullptr, (T*)nullptr, 0, s);
}
template pawfe_status launch_node_fixup<double>(const pawfe_op*, const double*, double, int, double*, int64_t,
                                                hipStream_t);
template pawfe_status launch_node_fixup<float>(const pawfe_op*, const double*, double, int, float*, int64_t,
                                               hipStream_t);

template <typename T>
pawfe_status launch_node_sinv(const pawfe_op* op, const T* X, int64_t ldx, const double* dv, int ncols, T* Y,
                              int64_t ldy, hipStream_t s) {
  if (ncols <= 0) return PAWFE_OK;
  constexpr int V = 16 / sizeof(T);
  const T* Minv = pick<T>(op->d.Minv, op->d.Minv_f);
  if (vec_ok(V, ncols, {{X, ldx}, {Y, ldy}})) {
    const RowGrid g = row_grid<k_node_sinv<T, V, kRowsPerWave>>(op->M, ncols, V, kRowsPerWave);
    hipLaunchKernelGGL((k_node_sinv<T, V, kRowsPerWave>), g.grid, dim3(256), 0, s, op->M, ncols, g.ncoltiles, X, ldx,
                       Y, ldy, Minv);
  } else {
    const RowGrid g = row_grid<k_node_sinv<T, 1, kRowsPerWave>>(op->M, ncols, 1, kRowsPerWave);
    hipLaunchKernelGGL((k_node_sinv<T, 1, kRowsPerWave>), g.grid, dim3(256), 0, s, op->M, ncols, g.ncoltiles, X, ldx,
                       Y, ldy, Minv);
  }
  PAWFE_HIP(hipGetLastError());
  return nl_fixup<T, T, true, false>(op, ncols, dv, -1.0, Y, ldy, nullptr, (T*)nullptr, 0, s);
}
template pawfe_status launch_node_sinv<double>(const pawfe_op*, const double*, int64_t, const double*, int, double*,
                                               int64_t, hipStream_t);
template pawfe_status launch_node_sinv<float>(const pawfe_op*, const float*, int64_t, const double*, int, float*,
                                              int64_t, hipStream_t);

template <typename TR>
pawfe_status launch_node_cheb(const pawfe_op* op, const TR* RY, TR* RX, TR* Tb, int64_t ld, const double* Y,
                              int64_t ldy, const double* dv, const double* qv, const double* lamY, double* lamX,
                              const double* lam_in, double a, double ac, double zz, int ncols, hipStream_t s) {
  if (ncols <= 0) return PAWFE_OK;
  constexpr int V = 16 / sizeof(TR);
  const TR* Minv = pick<TR>(op->d.Minv, op->d.Minv_f);
  if (vec_ok(V, ncols, {{RY, ld}, {RX, ld}, {Tb, ld}, {Y, ldy}})) {
    const RowGrid g = row_grid<k_node_cheb<TR, V, kRowsPerWave>>(op->M, ncols, V, kRowsPerWave);
    hipLaunchKernelGGL((k_node_cheb<TR, V, kRowsPerWave>), g.grid, dim3(256), 0, s, op->M, ncols, g.ncoltiles, RY,
                       RX, Tb, ld, Y, ldy, lamY, lamX, lam_in, a, ac, zz, Minv);
  } else {
    const RowGrid g = row_grid<k_node_cheb<TR, 1, kRowsPerWave>>(op->M, ncols, 1, kRowsPerWave);
    hipLaunchKernelGGL((k_node_cheb<TR, 1, kRowsPerWave>), g.grid, dim3(256), 0, s, op->M, ncols, g.ncoltiles, RY,
                       RX, Tb, ld, Y, ldy, lamY, lamX, lam_in, a, ac, zz, Minv);
  }
  PAWFE_HIP(hipGetLastError());
  // T -= M_D^{-1} C d ; R_X += C q  (q already scaled by a)
  return nl_fixup<TR, TR, true, true>(op, ncols, dv, -1.0, Tb, ld, qv, RX, ld, s);
}
template pawfe_status launch_node_cheb<double>(const pawfe_op*, const double*, double*, double*, int64_t,
                                               const double*, int64_t, const double*, const double*, const double*,
                                               double*, const double*, double, double, double, int, hipStream_t);
template pawfe_status launch_node_cheb<float>(const pawfe_op*, const float*, float*, float*, int64_t, const double*,
                                              int64_t, const double*, const double*, const double*, double*,
                                              const double*, double, double, double, int, hipStream_t);

template <typename TR>
pawfe_status launch_node_finalize(const pawfe_op* op, const TR* RY, int64_t ld, const double* dv, const double* X,
                                  int64_t ldx, const double* lamY, double* Xo, int64_t ldo, int ncols, hipStream_t s) {
  if (ncols <= 0) return PAWFE_OK;
  constexpr int V = 16 / sizeof(TR);
  const TR* Minv = pick<TR>(op->d.Minv, op->d.Minv_f);
  if (vec_ok(V, ncols, {{RY, ld}, {X, ldx}, {Xo, ldo}})) {
    const RowGrid g = row_grid<k_node_finalize<TR, V, kRowsPerWave>>(op->M, ncols, V, kRowsPerWave);
    hipLaunchKernelGGL((k_node_finalize<TR, V, kRowsPerWave>), g.grid, dim3(256), 0, s, op->M, ncols, g.ncoltiles,
                       RY, ld, X, ldx, lamY, Xo, ldo, Minv);
  } else {
    const RowGrid g = row_grid<k_node_finalize<TR, 1, kRowsPerWave>>(op->M, ncols, 1, kRowsPerWave);
    hipLaunchKernelGGL((k_node_finalize<TR, 1, kRowsPerWave>), g.grid, dim3(256), 0, s, op->M, ncols, g.ncoltiles,
                       RY, ld, X, ldx, lamY, Xo, ldo, Minv);
  }
  PAWFE_HIP(hipGetLastError());
  return nl_fixup<TR, double, true, false>(op, ncols, dv, -1.0, Xo, ldo, nullptr, (TR*)nullptr, 0, s);
}
template pawfe_status launch_node_finalize<double>(const pawfe_op*, const double*, int64_t, const double*,
                                                   const double*, int64_t, const double*, double*, int64_t, int,
                                                   hipStream_t);
template pawfe_status launch_node_finalize<float>(const pawfe_op*, const float*, int64_t, const double*, const double*,
                                                  int64_t, const double*, double*, int64_t, int, hipStream_t);

template <typename TR>
pawfe_status launch_cheb_init(const pawfe_op* op, const double* Y, int64_t ldy, TR* RY, TR* RX, int64_t ld, double f,
                              double c, const double* lam_in, double* lamY, double* lamX, int ncols, hipStream_t s) {
  if (ncols <= 0) return PAWFE_OK;
  constexpr int V = 16 / sizeof(TR);
  if (vec_ok(V, ncols, {{Y, ldy}, {RY, ld}, {RX, ld}})) {
    const RowGrid g = row_grid<k_cheb_init<TR, V, kRowsPerWave>>(op->M, ncols, V, kRowsPerWave);
    hipLaunchKernelGGL((k_cheb_init<TR, V, kRowsPerWave>), g.grid, dim3(256), 0, s, op->M, ncols, g.ncoltiles, Y, ldy,
                       RY, RX, ld, f, c, lam_in, lamY, lamX);
  } else {
    const RowGrid g = row_grid<k_cheb_init<TR, 1, kRowsPerWave>>(op->M, ncols, 1, kRowsPerWave);
    hipLaunchKernelGGL((k_cheb_init<TR, 1, kRowsPerWave>), g.grid, dim3(256), 0, s, op->M, ncols, g.ncoltiles, Y, ldy,
                       RY, RX, ld, f, c, lam_in, lamY, lamX);
  }
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}
template pawfe_status launch_cheb_init<double>(const pawfe_op*, const double*, int64_t, double*, double*, int64_t,
                                               double, double, const double*, double*, double*, int, hipStream_t);
template pawfe_status launch_cheb_init<float>(const pawfe_op*, const double*, int64_t, float*, float*, int64_t,
                                              double, double, const double*, double*, double*, int, hipStream_t);

pawfe_status launch_copy_cols(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t nrows, int ncols,
                              hipStream_t s) {
  if (ncols <= 0 || nrows <= 0) return PAWFE_OK;
  if (vec_ok(2, ncols, {{X, ldx}, {Y, ldy}})) {
    const RowGrid g = row_grid<k_copy_cols<2, kRowsPerWave>>(nrows, ncols, 2, kRowsPerWave);
    hipLaunchKernelGGL((k_copy_cols<2, kRowsPerWave>), g.grid, dim3(256), 0, s, nrows, ncols, g.ncoltiles, X, ldx, Y,
                       ldy);
  } else {
    const RowGrid g = row_grid<k_copy_cols<1, kRowsPerWave>>(nrows, ncols, 1, kRowsPerWave);
    hipLaunchKernelGGL((k_copy_cols<1, kRowsPerWave>), g.grid, dim3(256), 0, s, nrows, ncols, g.ncoltiles, X, ldx, Y,
                       ldy);
  }
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

template <typename T>
pawfe_status launch_fill(T* Y, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return PAWFE_OK;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, Y, n, v);
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}
template pawfe_status launch_fill<double>(double*, int64_t, double, hipStream_t);
template pawfe_status launch_fill<float>(float*, int64_t, float, hipStream_t);

pawfe_status launch_coldot(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t nrows, int ncols,
                           double* partial, double* out, const double* w, bool sqrt_out, bool scalar, hipStream_t s) {
  const int64_t rpc = 4096;
  const int nchunks = (int)((nrows + rpc - 1) / rpc);
  hipLaunchKernelGGL(k_coldot, dim3(nchunks, (ncols + 63) / 64), dim3(256), 0, s, A, lda, B, ldb, nrows, ncols, rpc,
                     partial);
  hipLaunchKernelGGL(k_coldot_final, dim3(scalar ? 1 : (ncols + 255) / 256), dim3(256), 0, s, partial, nchunks, ncols,
                     out, w, (int)sqrt_out, (int)scalar);
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

pawfe_status launch_grad_dh(const pawfe_op* op, const double* c, int ncols, const double* occ, double* out,
                            hipStream_t s) {
  if (op->natoms == 0) return PAWFE_OK;
  const int nent = op->npj2_total;
  hipLaunchKernelGGL(k_grad_dh, dim3((nent + 255) / 256), dim3(256), 0, s, c, ncols, occ, op->d_g2_atom, op->d_g2_s,
                     op->d_g2_t, nent, op->d, out);
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

}  // namespace pawfe
