// Local (cell) part of the FE operators on the gfx950 matrix cores.
//
// Built for the bf16x3 precision (FP32 data, every contraction as three
// bf16 products with FP32 accumulation on v_mfma_f32_16x16x16_bf16): K + V,
// the mass term and the imaginary k term.  FP32 and FP64 run on the
// vector-ALU kernel (cell_valu.h), which avoids the padding of the 7- and
// 8-wide contractions that the matrix-core tiles need; the FP32 / FP64 MFMA
// forms described below remain in the templates but are not instantiated.
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
// LDS holds three slabs of 8x8x8 slots of CB columns each, zero-initialized.
// Every pass walks the padded lines of the slab with unconditional stores:
// rows and outputs beyond the true extents only ever meet zero
// coefficients, so they stay finite and never reach a true slot.  Lines
// whose outer coordinate lies beyond its axis' extent hold zeros on input
// and output alike (the zero fill, then every pass that wrote them) and are
// skipped where a tile holds nothing else (FP32, two lines per tile).  Each wave
// owns whole lines and reads all of a tile's inputs before writing its
// outputs, so the passes run in place.
//
// Slab layout (XOR swizzle, a bijection on the slab): element (x, y, z, col)
// lives at ((z*8 + y)*8 + x')*CB + col', where x' and col' mix in bits of the
// other coordinates and of a per-slab key.  The masks are chosen (GF(2) rank
// conditions, one per contraction axis) so that the A-operand reads (16 rows
// x 4 k) hit distinct banks whether the LDS serves 32 or 64 lanes per cycle,
// and the 16-byte f32 result writes (one output per lane, two slabs told
// apart by the key) and the 8-byte f64 accesses hit distinct bank groups
// whether 8 or 16 lanes are served per cycle.  Without it the stride of the
// contracted axis (64 or 512 elements) put all outputs of a row in one bank.
// The two low column bits are never swizzled, so the four f32 results of a
// lane stay one aligned 16-byte chunk.
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

#include <algorithm>
#include <type_traits>

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

// bf16x3 split products (FP32 data on the bf16 matrix cores): x = hi + lo with
// hi = bf16(x), lo = bf16(x - hi) (round to nearest even; finite inputs), and
// a*b ~ lo_a hi_b + hi_a lo_b + hi_a hi_b accumulated in FP32 (the lo*lo
// term, ~2^-16 relative, is dropped).  v_mfma_f32_16x16x16_bf16 operand
// layout (checked on gfx950): A[i][k] in lane i + 16 (k/4), element k % 4;
// B[k][j] in lane j + 16 (k/4), element k % 4; D as for f32.
typedef short BfV4 __attribute__((ext_vector_type(4)));
typedef float F4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_rne(float x, float& back) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  back = __uint_as_float(u & 0xFFFF0000u);
  return (short)(u >> 16);
}

__device__ __forceinline__ void bf16_split(const float (&x)[4], BfV4& hi, BfV4& lo) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    float h, dummy;
    hi[v] = bf16_rne(x[v], h);
    lo[v] = bf16_rne(x[v] - h, dummy);
  }
}

__device__ __forceinline__ F4 mfma_bf3(const BfV4& ahi, const BfV4& alo, const BfV4& bhi, const BfV4& blo, F4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo, acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, acc, 0, 0, 0);
}

constexpr int kSlots = 512;   // 8 x 8 x 8 padded slots per column

__host__ __device__ constexpr int rev3(int v) { return ((v & 1) << 2) | (v & 2) | ((v >> 2) & 1); }

// LDS offset of element (x, y, z, col) of a slab with the given key.
template <typename T, int CB>
__host__ __device__ constexpr int phys(int x, int y, int z, int col, int key) {
  const int r = y ^ z;
  if constexpr (sizeof(T) == 4) {
    // x'0 = x0^y2^z2, x'1 = x1^y0^z0, x'2 = x2^y0^y1^z1, col'2 = c2^x2^y1^z1^key
    const int xs = x ^ ((r >> 2) & 1) ^ ((r & 1) << 1) ^ (((y ^ (y >> 1) ^ (z >> 1)) & 1) << 2);
    const int cs = col ^ ((((x >> 2) ^ (y >> 1) ^ (z >> 1)) & 1) << 2) ^ key;
    return ((z * 8 + y) * 8 + xs) * CB + cs;
  } else {
    return ((z * 8 + y) * 8 + (x ^ (r & 3))) * CB + (col ^ (((x ^ r) >> 2) & 1) ^ key);
  }
}
// key that tells apart two slabs written by one instruction (0 for the other)
template <typename T>
constexpr int kKeyC = sizeof(T) == 4 ? 4 : 2;

// Element at byte offset `b` of the LDS block.  Offsets are kept in bytes so
// that an access is the XOR alone (no scaling shift per access).
template <typename T>
__device__ __forceinline__ T& lds_at(T* smem, int b) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(smem) + b);
}

// A slab: its byte offset in the LDS block (a multiple of the slab size, so
// it never overlaps the bits of an address inside a slab) and its key.
struct Slab {
  int off;
  int key;
};

// Coordinates of index a along AX on padded line L; the line enumerates the
// other two axes (u, v) = (L % 8, L / 8), lower axis first.
template <int AX>
__host__ __device__ constexpr void line_coords(int L, int a, int& x, int& y, int& z) {
  const int u = L & 7, v = L >> 3;
  if constexpr (AX == 0) { x = a; y = u; z = v; }
  else if constexpr (AX == 1) { x = u; y = a; z = v; }
  else { x = u; y = v; z = a; }
}

// byte offset of (line L, index a, col) in a slab with the given key
template <typename T, int CB, int AX>
__host__ __device__ constexpr int line_addr(int L, int a, int col, int key) {
  int x = 0, y = 0, z = 0;
  line_coords<AX>(L, a, x, y, z);
  return phys<T, CB>(x, y, z, col, key) * (int)sizeof(T);
}

// Bits that the lane part of a read (RD) or result-write address can set;
// a constant part splits into the bits inside this mask (XORed) and those
// outside it (added through the instruction's offset field).
template <typename T, int CB, int AX, bool RD>
constexpr int lane_mask() {
  constexpr int LPT = 16 / CB;
  int m = 0;
  for (int w = 0; w < 4; ++w)
    for (int r = 0; r < 16; ++r)
      for (int kr = 0; kr < 4; ++kr)
        for (int key = 0; key < 2; ++key) {
          const int rl = sizeof(T) == 4 ? 4 * kr : kr;   // result row of element 0
          m |= RD ? line_addr<T, CB, AX>(LPT * w | (r / CB), kr, r % CB, 0)
                  : line_addr<T, CB, AX>(LPT * w | (rl / CB), r & 7, rl % CB, key * kKeyC<T>);
        }
  return m;
}

// Same for the A-operand reads of the bf16x3 variant: lane (row r, group g)
// reads axis index 4 (g & 1) + v of input buffer g >> 1 (buffer 0 when the
// pass has one input), v = 0..3 in the constant part.
template <int CB, int AX>
constexpr int lane_mask_bf3(int nin, int keyc) {
  constexpr int LPT = 16 / CB;
  int m = 0;
  for (int w = 0; w < 4; ++w)
    for (int r = 0; r < 16; ++r)
      for (int g = 0; g < 4; ++g) {
        const int key = (nin == 2 && (g >> 1)) ? 0 : keyc;
        m |= line_addr<float, CB, AX>(LPT * w | (r / CB), 4 * (g & 1), r % CB, key);
        m |= line_addr<float, CB, AX>(LPT * w | (r / CB), 4 * (g & 1), r % CB, 0);
      }
  return m;
}

}  // namespace

// One MFMA contraction pass over the 64 padded lines.
//   inputs:  NIN buffers; input k in [8b, 8b + 8) comes from in[b]
//   outputs: NG groups of 8; output o in [8g, 8g + 8) goes to out[g]
//   cf(o, k): stacked coefficient (0 outside the true extents)
//   pre(L, o): a value the store of (line L, output o) needs, read one tile
//     ahead with the A operands (NoPre: none)
//   post(L, o, col, value, old, pre value): the value stored
// Every address is built from disjoint bit fields (col, x', y, z, slab) and
// the swizzle is an XOR, so it splits as  lane part ^ constant part: the lane
// part (row, k or output index within a tile, wave) is computed once per
// pass, the constant part (tile, k-step, result element) folds at compile
// time, and each access costs one XOR.
struct NoPre {};

// element (row, column n) of a row-major block with a row stride of ldb
// bytes: the address is one 32 x 32 + 64-bit multiply-add
template <typename P>
__device__ __forceinline__ P* elem_ptr(P* base, uint32_t ldb, int n, int row) {
  using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<C*>(base + n) + (uint64_t)(uint32_t)row * ldb);
}

template <typename T, int AX, int CB, int NIN, int NG, bool BF3, int VEXT = 8, class CF, class POST, class PRE = NoPre>
__device__ __forceinline__ void mfma_pass(T* smem, const Slab* in, const Slab* out, CF cf, POST post,
                                          PRE pre = PRE()) {
  constexpr bool HAS_PRE = !std::is_same<PRE, NoPre>::value;
  using M = Mma<T>;
  constexpr int NKS = 2 * NIN;                 // k-steps of 4
  constexpr int NOB = (NG + 1) / 2;            // 16-wide output blocks
  constexpr int LPT = 16 / CB;                 // lines per tile
  constexpr int NT = 64 / LPT;                 // tiles per pass
  // With two lines per tile, iteration it covers exactly the lines whose
  // outer coordinate v (line / 8) is it.  Lines with v >= VEXT (the extent of
  // that axis in this pass's input and output) read only zeros and their
  // output slots already hold zeros, so those iterations are skipped.
  constexpr int NIT = (LPT == 2 && VEXT < NT / 4) ? VEXT : NT / 4;
  constexpr int MR = lane_mask<T, CB, AX, true>() | (sizeof(T) - 1);
  constexpr int MW = lane_mask<T, CB, AX, false>() | (sizeof(T) - 1);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 15, kr = lane >> 4;
  static_assert(!BF3 || sizeof(T) == 4, "bf16x3 runs on FP32 data");
  T bco[NOB][NKS];
  BfV4 bhi[NOB], blo[NOB];
  if constexpr (BF3) {
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) {
      float c[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) c[v] = (float)cf(ob * 16 + r, 4 * kr + v);
      bf16_split(c, bhi[ob], blo[ob]);
    }
  } else {
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) bco[ob][ks] = cf(ob * 16 + r, ks * 4 + kr);
  }
  // tile t = wave + 4 it covers lines LPT t + [0, LPT)
  const int lw = LPT * wave;
  const int rd_lane = line_addr<T, CB, AX>(lw | (r / CB), kr, r % CB, 0);
  const int rl = M::row(kr, 0);                // result row = rl | M::row(0, e)
  int wr_lane[NOB];
#pragma unroll
  for (int ob = 0; ob < NOB; ++ob) {
    const Slab s0 = out[2 * ob], s1 = out[(2 * ob + 1 < NG) ? 2 * ob + 1 : 2 * ob];
    const Slab b = r < 8 ? s0 : s1;
    wr_lane[ob] = b.off | line_addr<T, CB, AX>(lw | (rl / CB), r & 7, rl % CB, b.key);
  }
  // A operands of tile `it`.  FP32/FP64: k = 4 ks + kr, index k % 8 in
  // buffer ks / 2.  bf16x3: the lane's four k = 4 kr + v (v = 0..3), buffer
  // kr / 2 when there are two inputs (else buffer 0, duplicates that meet
  // zero coefficients), index 4 (kr & 1) + v.
  constexpr int NA = BF3 ? 4 : NKS;
  constexpr int MR3 = BF3 ? (lane_mask_bf3<CB, AX>(NIN, kKeyC<float>) | 3) : 0;
  int rd3_lane = 0;
  if constexpr (BF3) {
    const Slab b = in[(NIN == 2 && (kr >> 1)) ? NIN - 1 : 0];
    rd3_lane = b.off | line_addr<T, CB, AX>(lw | (r / CB), 4 * (kr & 1), r % CB, b.key);
  }
  auto load_a = [&](int it, T (&av)[NA]) {
    if constexpr (BF3) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = line_addr<T, CB, AX>(LPT * 4 * it, v, 0, 0);
        av[v] = lds_at(smem, (rd3_lane ^ (c & MR3)) + (c & ~MR3));
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        const Slab b = in[ks / 2];
        const int c = b.off | line_addr<T, CB, AX>(LPT * 4 * it, 4 * (ks & 1), 0, b.key);
        av[ks] = lds_at(smem, (rd_lane ^ (c & MR)) + (c & ~MR));
      }
    }
  };
  // the pre values of tile `it`, one per output block and result element
  // (f32: the four results of a lane lie on one line, one value serves them)
  auto load_pre = [&](int it, T (&pv)[NOB][4]) {
    if constexpr (HAS_PRE) {
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob) {
        if constexpr (sizeof(T) == 4) {
          const T v = pre(lw | (LPT * 4 * it) | (rl / CB), ob * 16 + r);
#pragma unroll
          for (int e = 0; e < 4; ++e) pv[ob][e] = v;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) pv[ob][e] = pre(lw | (LPT * 4 * it) | ((rl | M::row(0, e)) / CB), ob * 16 + r);
        }
      }
    }
  };
  // software pipeline: the next tile's operands are read before this tile's
  // results are written (in program order), so the LDS latency overlaps the
  // MFMAs instead of waiting behind the in-place stores
  T av[NA];
  T pv[NOB][4];
  load_a(0, av);
  load_pre(0, pv);
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int lc = LPT * 4 * it;
    T an[NA];
    T pvn[NOB][4];
    if (it + 1 < NIT) {
      load_a(it + 1, an);
      load_pre(it + 1, pvn);
    }
    typename M::V4 acc[NOB];
    if constexpr (BF3) {
      BfV4 ahi, alo;
      float a4[4] = {(float)av[0], (float)av[1], (float)av[2], (float)av[3]};
      bf16_split(a4, ahi, alo);
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob) {
        F4 z = {0.f, 0.f, 0.f, 0.f};
        const F4 d = mfma_bf3(ahi, alo, bhi[ob], blo[ob], z);
        acc[ob] = typename M::V4{(T)d[0], (T)d[1], (T)d[2], (T)d[3]};
      }
    } else {
#pragma unroll
      for (int ob = 0; ob < NOB; ++ob) {
        acc[ob] = typename M::V4{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) acc[ob] = M::op(av[ks], bco[ob][ks], acc[ob]);
      }
    }
#pragma unroll
    for (int ob = 0; ob < NOB; ++ob) {
      const int o = ob * 16 + r;
      if (2 * ob + 1 < NG || r < 8) {
        if constexpr (sizeof(T) == 4) {
          // f32: the four result rows of a lane are four consecutive columns
          // (the swizzle never touches the two low column bits): one 16-byte
          // access, 16-byte aligned.
          const int c = line_addr<T, CB, AX>(lc, 0, 0, 0);
          const int s = (wr_lane[ob] ^ (c & MW)) + (c & ~MW);
          typename M::V4* dp = reinterpret_cast<typename M::V4*>(&lds_at(smem, s));
          typename M::V4 v = *dp;
          const int L2 = lw | lc | (rl / CB);
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = post(L2, o, (rl % CB) | e, acc[ob][e], v[e], pv[ob][e]);
          *dp = v;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int re = M::row(0, e);
            const int c = line_addr<T, CB, AX>(lc | (re / CB), 0, re % CB, 0);
            const int s = (wr_lane[ob] ^ (c & MW)) + (c & ~MW);
            const int L2 = lw | lc | ((rl | re) / CB), c2 = (rl | re) % CB;
            T& d = lds_at(smem, s);
            d = post(L2, o, c2, acc[ob][e], d, pv[ob][e]);
          }
        }
      }
    }
    if (it + 1 < NIT) {
#pragma unroll
      for (int ks = 0; ks < NA; ++ks) av[ks] = an[ks];
      if constexpr (HAS_PRE) {
#pragma unroll
        for (int ob = 0; ob < NOB; ++ob)
#pragma unroll
          for (int e = 0; e < 4; ++e) pv[ob][e] = pvn[ob][e];
      }
    }
  }
}

// FP32, and the FP64 residual mode: registers held to three waves per
// SIMD (the LDS of three workgroups fits in a CU; the residual mode forms
// W_q from the 1-D weights instead of keeping a table of nq^3 of them).
template <typename T, int NP, int NQ, int CB, int MODE, bool BF3>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 || MODE == kModeHRes) ? 3 : 1)))
k_cell_mfma(CellArgs<T> A, const Tab1D<T>* __restrict__ tabp,
                                                   int ncoltiles, int nitems) {
  constexpr int NL = NP * NP * NP;
  constexpr int NQ3 = NQ * NQ * NQ;
  constexpr int NJ = (NL * CB + 255) / 256;   // gathered elements per thread and item
  constexpr int NV = (NQ3 + 255) / 256;       // V(q) W_q values per thread and item
  constexpr bool HAS_V = MODE == kModeH || MODE == kModeHRes;
  constexpr bool RES = MODE == kModeHRes;
  constexpr bool IMG = MODE == kModeImg;
  __shared__ T smem[3 * kSlots * CB];
  // V(q) W_q of the current cell; entry q at q + q / 64, so the 8 outputs
  // of a result write (stride 64) differ in bank
  constexpr int NQP = NQ3 + NQ3 / 64;
  __shared__ T vws[HAS_V ? NQP : 1];
  __shared__ T lams[RES ? CB : 1];            // lambda_n of the item's columns (residual mode)
  const Tab1D<T>& tab = *tabp;
  const int tid = threadIdx.x;
  const int col = tid % CB;                   // 256 is a multiple of CB
  // The 1-D tables and the scale factors f_x, f_y, f_z, detJ live in LDS,
  // so that no global load sits between the passes (a vector-memory wait
  // there would also wait for the next item's prefetch).  FP32: zero-padded
  // 8x8 blocks B[q][a], K1, M1 and a zero block (no bounds test on a read).
  // FP64 (no LDS to spare at three workgroups per CU): B unpadded, the
  // symmetric K1 and M1 as lower triangles, one zero.
  // In the imaginary-term mode the K slot holds G1 (not symmetric: FP64
  // keeps it unpacked) and the scale factors are g_d.
  constexpr bool PADT = sizeof(T) == 4;
  constexpr int NB = NQ * NP, NS = NP * (NP + 1) / 2, NKS = IMG ? NP * NP : NS;
  constexpr int tK = PADT ? 64 : NB, tM = PADT ? 128 : NB + NKS, tZ = PADT ? 192 : NB + NKS + NS;
  // (residual mode: the 1-D Gauss weights follow the scale factors, so that
  // W_q = w_qx w_qy w_qz detJ needs no table of its own)
  constexpr int tF = PADT ? 256 : tZ + 1, NCT = tF + 4 + (RES ? 8 : 0);
  const T* Kt = IMG ? tab.G1 : tab.K1;
  const T* ft = IMG ? tab.g : tab.f;
  __shared__ T ctab[NCT];
  for (int i = tid; i < NCT; i += 256) {
    T v = T(0);
    if (i >= tF) {
      const int k = i - tF;
      v = k < 3 ? ft[k] : (k == 3 ? tab.detJ : tab.w[(k - 4) & 7]);
    } else if constexpr (PADT) {
      const int blk = i >> 6, o = (i >> 3) & 7, k = i & 7;
      if (blk == 0) v = (o < NQ && k < NP) ? tab.B[o * NP + k] : T(0);
      else if (blk == 1) v = (o < NP && k < NP) ? Kt[o * NP + k] : T(0);
      else if (blk == 2) v = (o < NP && k < NP) ? tab.M1[o * NP + k] : T(0);
    } else {
      if (i < tK) {
        v = tab.B[i];
      } else if (IMG && i < tM) {
        v = Kt[i - tK];
      } else if (i < tZ) {
        int t = i < tM ? i - tK : i - tM, h = 0;   // packed (h, l), l <= h
        while ((h + 1) * (h + 2) / 2 <= t) ++h;
        v = (i < tM ? Kt : tab.M1)[h * NP + (t - h * (h + 1) / 2)];
      }
    }
    ctab[i] = v;
  }

  // local nodes gathered by this thread: local node l = tid / CB +
  // (256 / CB) j = (a, b, c).  pk[j] = (off << 14) | (byte offset of the
  // element in slab A), off = a + Gx (b + Gy c) the node's row offset from
  // the cell's first node when no index wraps.  Threads past the last node
  // (only in the last group) carry off 0 and a padding slot (7, 7, 7): they
  // load a valid row, stage a zero into padding and store nothing.  The
  // offset field holds 18 bits; larger meshes send every cell down the wrap
  // path, which recomputes (a, b, c).
  constexpr int kLast = (NL * CB) % 256 == 0 ? NJ : NJ - 1;   // groups before kLast are all real
  constexpr int kLdsBits = 14;
  static_assert(kSlots * CB * sizeof(T) <= (1u << kLdsBits), "slab A offsets must fit the field");
  const int p = NP - 1;
  const int Gx = A.n0 * p, Gy = A.n1 * p, Gz = A.n2 * p;
  const bool off_fits = (int64_t)p + (int64_t)Gx * (p + (int64_t)Gy * p) < (1 << (32 - kLdsBits));
  auto lnode = [&](int j) { return tid / CB + (256 / CB) * j; };
  auto lreal = [&](int j) { return j < kLast || lnode(j) < NL; };
  unsigned pk[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int l = lnode(j);
    const int a = l % NP, b = (l / NP) % NP, c = l / (NP * NP);
    pk[j] = l < NL ? ((off_fits ? (unsigned)(a + Gx * (b + Gy * c)) : 0u) << kLdsBits) |
                         (unsigned)(phys<T, CB>(a, b, c, col, 0) * (int)sizeof(T))
                   : (unsigned)(phys<T, CB>(7, 7, 7, col, 0) * (int)sizeof(T));
  }
  // global node of local node j in cell e (periodic wrap only for the last
  // cell along an axis; the cell index is wave-uniform, so is the branch)
  struct CellPos {
    int ci, cj, ck, e, base;
    bool inner;
  };
  auto cell_pos = [&](int packed) {
    CellPos c;
    c.ci = packed & 1023;
    c.cj = (packed >> 10) & 1023;
    c.ck = (packed >> 20) & 1023;
    c.e = c.ci + A.n0 * (c.cj + A.n1 * c.ck);
    c.base = c.ci * p + Gx * (c.cj * p + Gy * c.ck * p);
    c.inner = off_fits && c.ci + 1 < A.n0 && c.cj + 1 < A.n1 && c.ck + 1 < A.n2;
    return c;
  };
  auto node_inner = [&](const CellPos& cp, int j) -> int { return cp.base + (int)(pk[j] >> kLdsBits); };
  auto node_wrap = [&](const CellPos& cp, int j) -> int {
    const int l = lreal(j) ? lnode(j) : 0;
    const int a = l % NP, b = (l / NP) % NP, c = l / (NP * NP);
    int gx = cp.ci * p + a; gx = gx >= Gx ? gx - Gx : gx;
    int gy = cp.cj * p + b; gy = gy >= Gy ? gy - Gy : gy;
    int gz = cp.ck * p + c; gz = gz >= Gz ? gz - Gz : gz;
    return gx + Gx * (gy + Gy * gz);
  };
  // global nodes of the thread's local nodes (one wave-uniform branch)
  auto nodes_of = [&](const CellPos& cp, int (&node)[NJ]) {
    if (cp.inner) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) node[j] = node_inner(cp, j);
    } else {
#pragma unroll
      for (int j = 0; j < NJ; ++j) node[j] = node_wrap(cp, j);
    }
  };
  // row strides in bytes (below 4 GiB, checked on launch)
  const uint32_t ldxb = (uint32_t)(A.ldx * (int64_t)sizeof(T)), ldyb = (uint32_t)(A.ldy * (int64_t)sizeof(T));
  // rows of those nodes, column n: the loads are issued after the branch
  // joins, so no copy of a loaded value waits for its load
  auto gather = [&](const T* __restrict__ src, uint32_t ldb, const CellPos& cp, int n, T (&dst)[NJ]) {
    int node[NJ];
    nodes_of(cp, node);
#pragma unroll
    for (int j = 0; j < NJ; ++j) dst[j] = *elem_ptr(src, ldb, n, node[j]);
  };
  auto lds_a = [&](unsigned pkj) -> T& { return lds_at(smem, (int)(pkj & ((1u << kLdsBits) - 1))); };
  // same element in slab C: its key flips column bits, its base is 2 slabs on
  auto lds_c = [&](unsigned pkj) -> T& {
    return lds_at(smem, ((int)(pkj & ((1u << kLdsBits) - 1)) ^ (kKeyC<T> * (int)sizeof(T))) +
                            2 * kSlots * CB * (int)sizeof(T));
  };

  // items (cell of the colour, column tile), cell-major; the x-th eighth of
  // them goes to the workgroups on XCD x (block w runs on XCD w % 8).  The
  // cell list (packed cell coordinates) is read through the scalar cache (it
  // is not written here), so reading it never waits for the vector loads in
  // flight; (cell, tile) advance by a fixed step without divisions.
  typedef const __attribute__((address_space(4))) int* ConstIntP;
  const ConstIntP cells = (ConstIntP)A.cells;
  const int xcd = blockIdx.x & 7;
  const int i_end = (int)((int64_t)nitems * (xcd + 1) / 8);
  const int i_step = gridDim.x >> 3;
  int item = (int)((int64_t)nitems * xcd / 8) + (blockIdx.x >> 3);
  const int st_c = i_step / ncoltiles, st_t = i_step % ncoltiles;
  int cur_c = item / ncoltiles, cur_t = item % ncoltiles;
  auto advance = [&](int& c, int& t) {
    c += st_c;
    t += st_t;
    if (t >= ncoltiles) {
      t -= ncoltiles;
      ++c;
    }
  };

  // registers for the gathered values (and V W) of the next item
  T xr[NJ], vr[NV];
  int xn0 = 0;
  double xlam = 0.0;
  auto load_item = [&](int c, int t) {
    const CellPos cp = cell_pos(cells[c]);
    const int e = cp.e;
    xn0 = t * CB;
    const int n = xn0 + col;
    gather(A.X, ldxb, cp, n < A.ncols ? n : 0, xr);
    if constexpr (RES) xlam = A.lam[min(xn0 + col, A.ncols - 1)];
    if constexpr (HAS_V) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int q = tid + 256 * v;
        if (NQ3 % 256 == 0 || q < NQ3) vr[v] = A.Vw[(int64_t)e * NQ3 + q];
      }
    }
  };

  // value v, or +0 where `keep` is false, through a bit mask (a select the
  // compiler cannot turn into a branch around the wait for v's load)
  auto zero_unless = [](bool keep, T v) -> T {
    if constexpr (sizeof(T) == 4) return __uint_as_float(__float_as_uint(v) & (keep ? ~0u : 0u));
    else return __longlong_as_double(__double_as_longlong(v) & (keep ? ~0ll : 0ll));
  };
  // stage the loaded item: gathered values -> slab A (extraction), V W and
  // the columns' lambdas -> LDS.  Columns past the last one carry the values
  // of column 0 (a valid load): columns never mix in the passes and those
  // are never stored.  Threads past the last node stage a zero into padding.
  // It runs at the end of the previous item
  // (slab A and these tables are no longer read once the last pass has
  // started), where the loads it waits for are the most recent vector-memory
  // operations and have had a whole item to arrive.
  auto stage = [&]() {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      T v = xr[j];
      if constexpr (IMG) {   // s_n x[n ^ 1]: the partner column sits in the neighbouring lane
        const T w = __shfl_xor(v, 1);
        v = (col & 1) ? w : -w;
      }
      lds_a(pk[j]) = j < kLast ? v : zero_unless(lreal(j), v);
    }
    // (writes without branches, so that the wait for every load happens on
    // every path and nothing is left in doubt at the top of the loop)
    if constexpr (HAS_V) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (NQ3 % 256 == 0 || tid + 256 * v < NQ3) vws[tid + 256 * v + (tid + 256 * v) / 64] = vr[v];
    }
    // every thread of a column writes the same value
    if constexpr (RES) lams[col] = xn0 + col < A.ncols ? (T)xlam : T(0);
  };

  // the padded slots are zero once and stay zero: every pass only ever
  // writes zeros there (zero inputs, zero coefficients)
  for (int i = tid; i < 3 * kSlots * CB; i += 256) smem[i] = T(0);
  if (item < i_end) load_item(cur_c, cur_t);
  __syncthreads();
  if (item < i_end) stage();
  __syncthreads();

  auto store = [](int, int, int, T v, T, T) { return v; };
  // 1-D tables, zero outside the true extents
  auto sym = [](int a, int b) { const int h = a > b ? a : b, l = a > b ? b : a; return h * (h + 1) / 2 + l; };
  auto Bm = [&](int q, int a) -> T {
    if constexpr (PADT) return ctab[(q < 8 && a < 8) ? q * 8 + a : tZ];
    else return ctab[(q < NQ && a < NP) ? q * NP + a : tZ];
  };
  auto Km = [&](int a, int b) -> T {
    if constexpr (PADT) return ctab[(a < 8 && b < 8) ? tK + a * 8 + b : tZ];
    else if constexpr (IMG) return ctab[(a < NP && b < NP) ? tK + a * NP + b : tZ];
    else return ctab[(a < NP && b < NP) ? tK + sym(a, b) : tZ];
  };
  auto Mm = [&](int a, int b) -> T {
    if constexpr (PADT) return ctab[(a < 8 && b < 8) ? tM + a * 8 + b : tZ];
    else return ctab[(a < NP && b < NP) ? tM + sym(a, b) : tZ];
  };
  auto fsc = [&](int i) -> T { return ctab[tF + i]; };
  constexpr int KC = kKeyC<T>;
  constexpr int SLB = kSlots * CB * (int)sizeof(T);   // slab size in bytes
  const Slab sA{0, 0}, sB{SLB, 0}, sC{2 * SLB, KC};

  for (; item < i_end; item += i_step) {
    const int n0 = cur_t * CB;
    const int n = n0 + col;
    const bool valid = n < A.ncols;
    // output rows of this item (old values) and the next item's inputs are
    // fetched now and arrive while the passes run (the item itself is staged)
    const CellPos cp = cell_pos(cells[cur_c]);
    T yo[NJ];
    gather(A.Y, ldyb, cp, valid ? n : 0, yo);
    int nxt_c = cur_c, nxt_t = cur_t;
    advance(nxt_c, nxt_t);
    // (the last item loads itself again: unconditional loads, no join)
    const bool more = item + i_step < i_end;
    load_item(more ? nxt_c : cur_c, more ? nxt_t : cur_t);

    if constexpr (IMG) {
      // kinetic structure with G1: C = sum_d g_d (G1 along d, M1 along the others) U'
      const Slab inA[1] = {sA};
      const Slab inCA[2] = {sC, sA};
      const Slab oC[1] = {sC};
      const Slab oCA[2] = {sC, sA};
      mfma_pass<T, 0, CB, 1, 2, BF3, NP>(smem, inA, oCA,
                                         [&](int o, int k) { return o < 8 ? Km(o, k) : Mm(o - 8, k); }, store);
      __syncthreads();
      mfma_pass<T, 1, CB, 2, 2, BF3, NP>(
          smem, inCA, oCA,
          [&](int o, int k) {
            if (o < 8) return k < 8 ? fsc(0) * Mm(o, k) : fsc(1) * Km(o, k - 8);
            return k < 8 ? T(0) : Mm(o - 8, k - 8);
          },
          store);
      __syncthreads();
      mfma_pass<T, 2, CB, 2, 1, BF3, NP>(
          smem, inCA, oC, [&](int o, int k) { return k < 8 ? Mm(o, k) : fsc(2) * Km(o, k - 8); }, store);
      __syncthreads();
    } else if constexpr (MODE == kModeMass) {
      const Slab inA[1] = {sA};
      const Slab inC[1] = {sC};
      const Slab oC[1] = {sC};
      mfma_pass<T, 0, CB, 1, 1, BF3, NP>(smem, inA, oC, [&](int o, int k) { return Mm(o, k); }, store);
      __syncthreads();
      mfma_pass<T, 1, CB, 1, 1, BF3, NP>(smem, inC, oC, [&](int o, int k) { return Mm(o, k); }, store);
      __syncthreads();
      mfma_pass<T, 2, CB, 1, 1, BF3, NP>(smem, inC, oC, [&](int o, int k) { return fsc(3) * Mm(o, k); }, store);
      __syncthreads();
    } else {
      const Slab inA[1] = {sA};
      const Slab inB[1] = {sB};
      const Slab inCA[2] = {sC, sA};
      const Slab oB[1] = {sB};
      const Slab oC[1] = {sC};
      const Slab oBCA[3] = {sB, sC, sA};
      const Slab oCA[2] = {sC, sA};
      // P1 x: [Bx; Kx; Mx] U
      mfma_pass<T, 0, CB, 1, 3, BF3, NP>(
          smem, inA, oBCA,
          [&](int o, int k) { return o < 8 ? Bm(o, k) : (o < 16 ? Km(o - 8, k) : Mm(o - 16, k)); }, store);
      __syncthreads();
      // P2 y: By
      mfma_pass<T, 1, CB, 1, 1, BF3, NP>(smem, inB, oB, [&](int o, int k) { return Bm(o, k); }, store);
      __syncthreads();
      // P3 z: Bz, then V(q) W_q (minus lambda_n W_q); lines are (qa, qb)
      {
        // point index (clamped, so that a read never leaves the table) and
        // whether the point is real; the weight is read one tile ahead
        auto qidx = [](int L, int o) {
          if constexpr (NQ == 8) {
            // q = 64 o + L, stored at q + o: the lane part plus a constant
            // (o >= 8 lanes read in range and are discarded)
            return 65 * (o & 7) + L;
          } else {
            const int qa = L & 7, qb = L >> 3;
            const int q = ((o < NQ ? o : 0) * NQ + (qb < NQ ? qb : 0)) * NQ + (qa < NQ ? qa : 0);
            return q + q / 64;
          }
        };
        auto qin = [](int L, int o) { return (L & 7) < NQ && (L >> 3) < NQ && o < NQ; };
        auto vpre = [&](int L, int o) {
          const T w = vws[qidx(L, o)];   // unconditional read, then select
          return qin(L, o) ? w : T(0);
        };
        auto vpost = [&](int L, int o, int c, T v, T, T w) {
          if constexpr (RES) {
            // W_q of point (qa, qb, qc) = (L & 7, L >> 3, o), multiplied in the
            // order the host forms it (bit-identical weights)
            const T* wq = &ctab[tF + 4];
            const T wgt = wq[L & 7] * wq[L >> 3] * wq[o & 7] * fsc(3);
            return qin(L, o) ? v * (w - lams[c] * wgt) : T(0);
          }
          else return v * w;
        };
        mfma_pass<T, 2, CB, 1, 1, BF3, NQ>(smem, inB, oB, [&](int o, int k) { return Bm(o, k); }, vpost, vpre);
      }
      __syncthreads();
      // P4 z: Bz^T;  P5 y: By^T
      mfma_pass<T, 2, CB, 1, 1, BF3, NQ>(smem, inB, oB, [&](int o, int k) { return Bm(k, o); }, store);
      __syncthreads();
      mfma_pass<T, 1, CB, 1, 1, BF3, NP>(smem, inB, oB, [&](int o, int k) { return Bm(k, o); }, store);
      __syncthreads();
      // P6 y: P = fx My C + fy Ky A -> C ; Q = My A -> A
      mfma_pass<T, 1, CB, 2, 2, BF3, NP>(
          smem, inCA, oCA,
          [&](int o, int k) {
            if (o < 8) return k < 8 ? fsc(0) * Mm(o, k) : fsc(1) * Km(o, k - 8);
            return k < 8 ? T(0) : Mm(o - 8, k - 8);
          },
          store);
      __syncthreads();
      // P7 z: kinetic = Mz P + fz Kz Q -> C
      mfma_pass<T, 2, CB, 2, 1, BF3, NP>(
          smem, inCA, oC, [&](int o, int k) { return k < 8 ? Mm(o, k) : fsc(2) * Km(o, k - 8); }, store);
      __syncthreads();
      // P8 x: Bx^T on slab B, accumulated into C
      mfma_pass<T, 0, CB, 1, 1, BF3, NP>(smem, inB, oC, [&](int o, int k) { return Bm(k, o); },
                                [](int, int, int, T v, T old, T) { return old + v; });
      __syncthreads();
    }
    stage();

    // assembly: colour-ordered read-modify-write, CB contiguous columns per DOF
    if (valid) {
      int node[NJ];
      nodes_of(cp, node);
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        if (lreal(j)) *elem_ptr(A.Y, ldyb, n, node[j]) = yo[j] + A.alpha * lds_c(pk[j]);
    }
    __syncthreads();
    cur_c = nxt_c;
    cur_t = nxt_t;
  }
}

namespace {

template <typename T>
const Tab1D<T>* dev_tab_m(const pawfe_op* op) {
  if constexpr (std::is_same<T, double>::value) return op->d.tab64; else return op->d.tab32;
}

// persistent grid: as many 256-thread workgroups as are resident on the
// chip at once (LDS- and register-limited), a multiple of 8, never more than
// the items need
template <auto K>
int cell_grid(int nitems) {
  static const int resident = [] {
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
      ncu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, K, 256, 0) != hipSuccess || per_cu <= 0) per_cu = 1;
    return std::max(8, ncu * per_cu / 8 * 8);
  }();
  return std::max(8, std::min(resident, (nitems + 7) / 8 * 8));
}

// bf16x3 split products only (FP32 data): every other local term runs on the
// vector-ALU kernel
template <typename T, int NP, int NQ, int CB, int MODE>
void launch_mode(const CellArgs<T>& ac, const Tab1D<T>* tab, int ncoltiles, int nitems, hipStream_t s) {
  const dim3 grid(cell_grid<k_cell_mfma<T, NP, NQ, CB, MODE, true>>(nitems)), block(256);
  hipLaunchKernelGGL((k_cell_mfma<T, NP, NQ, CB, MODE, true>), grid, block, 0, s, ac, tab, ncoltiles, nitems);
}

template <typename T, int NP, int NQ, int CB>
pawfe_status run_cell_mfma(const pawfe_op* op, int mode, CellArgs<T> a, hipStream_t s) {
  const Tab1D<T>* tab = dev_tab_m<T>(op);
  const int ncoltiles = (a.ncols + CB - 1) / CB;
  for (int c = 0; c < op->ncolour; ++c) {
    const int c0 = op->colour_off[c], c1 = op->colour_off[c + 1];
    if (c1 == c0) continue;
    CellArgs<T> ac = a;
    ac.cells = op->d.cell_pack + c0;
    const int nitems = (c1 - c0) * ncoltiles;
    if (mode == kModeH)
      launch_mode<T, NP, NQ, CB, kModeH>(ac, tab, ncoltiles, nitems, s);
    else if (mode == kModeImg)
      launch_mode<T, NP, NQ, CB, kModeImg>(ac, tab, ncoltiles, nitems, s);
    else
      launch_mode<T, NP, NQ, CB, kModeMass>(ac, tab, ncoltiles, nitems, s);
  }
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

}  // namespace

template <typename T>
pawfe_status launch_cell_mfma(const pawfe_op* op, int mode, const CellArgs<T>& a, hipStream_t s) {
  constexpr int CB = sizeof(T) == 8 ? 4 : 8;
  if (sizeof(T) != 4 || !a.bf3 || mode == kModeHRes)
    return fail(PAWFE_EUNSUPPORTED, "the matrix-core cell kernel is built for bf16x3 (K + V, mass, imaginary term)");
  if (a.ldx < 0 || a.ldy < 0 || a.ldx * (int64_t)sizeof(T) >= (int64_t(1) << 32) ||
      a.ldy * (int64_t)sizeof(T) >= (int64_t(1) << 32))
    return fail(PAWFE_EINVAL, "row stride of 4 GiB or more");
  switch (op->p) {
    case 2: return run_cell_mfma<T, 3, 4, CB>(op, mode, a, s);
    case 3: return run_cell_mfma<T, 4, 5, CB>(op, mode, a, s);
    case 4: return run_cell_mfma<T, 5, 6, CB>(op, mode, a, s);
    case 5: return run_cell_mfma<T, 6, 7, CB>(op, mode, a, s);
    case 6: return run_cell_mfma<T, 7, 8, CB>(op, mode, a, s);
    default: return fail(PAWFE_EUNSUPPORTED, "degree not compiled");
  }
}

template <>
pawfe_status launch_cell_mfma<double>(const pawfe_op*, int, const CellArgs<double>&, hipStream_t) {
  return fail(PAWFE_EUNSUPPORTED, "the matrix-core cell kernel is built for bf16x3 (FP32 data) only");
}
template pawfe_status launch_cell_mfma<float>(const pawfe_op*, int, const CellArgs<float>&, hipStream_t);

}  // namespace pawfe
