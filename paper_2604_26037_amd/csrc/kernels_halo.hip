// BF16 halo of a z-slab decomposition (the paper's reduced-precision
// inter-processor communication: partial sums on the node planes shared with
// a neighbouring processor travel in BF16 and are cast back to FP32 and
// added on the receiving side).  One GPU's part: the pack kernel that turns
// the FP32 values of a slab's two shared node planes into BF16, and the
// unpack kernel that adds received BF16 planes into an FP32 block.
//
// Layout of the buffer: [2][Gx * Gy][ncols] BF16 bits, plane gz0 then gz1,
// nodes of a plane (gy, gx) row-major, columns contiguous.  Plane rows are
// contiguous blocks of Gx * Gy DOF rows in the node-major multivector, so
// both kernels are plain streaming copies: each thread moves four columns
// of one row (16 bytes of FP32, 8 bytes of BF16).

#include "kernels.h"

namespace pawfe {

namespace {

// round to nearest, ties to even; NaNs stay NaN (quiet bit set)
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (u >> 16) | 0x40u;
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

// t = thread of (row, 4-column group); rows of both planes, plane-major
__global__ void __launch_bounds__(256) k_halo_pack(const float* __restrict__ Y, int64_t ldy, int ncols,
                                                   int64_t plane0, int64_t plane1, int64_t prow,
                                                   uint16_t* __restrict__ buf) {
  const int ngrp = (ncols + 3) / 4;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= 2 * prow * ngrp) return;
  const int64_t r = t / ngrp;
  const int n0 = (int)(t - r * ngrp) * 4;
  const int64_t row = (r < prow ? plane0 : plane1) + (r < prow ? r : r - prow);
  const float* src = Y + row * ldy + n0;
  uint16_t* dst = buf + r * ncols + n0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (n0 + i < ncols) dst[i] = (uint16_t)bf16_bits(src[i]);
}

__global__ void __launch_bounds__(256) k_halo_unpack(const uint16_t* __restrict__ buf, int ncols, int64_t plane0,
                                                     int64_t plane1, int64_t prow, float* __restrict__ Y,
                                                     int64_t ldy) {
  const int ngrp = (ncols + 3) / 4;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= 2 * prow * ngrp) return;
  const int64_t r = t / ngrp;
  const int n0 = (int)(t - r * ngrp) * 4;
  const int64_t row = (r < prow ? plane0 : plane1) + (r < prow ? r : r - prow);
  float* dst = Y + row * ldy + n0;
  const uint16_t* src = buf + r * ncols + n0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (n0 + i < ncols) dst[i] = dst[i] + bf16_value(src[i]);
}

}  // namespace

pawfe_status launch_halo(const pawfe_op* op, bool pack, float* Y, int64_t ldy, int ncols, int kz0, int kz1,
                         uint16_t* buf, hipStream_t s) {
  const int64_t prow = (int64_t)op->n[0] * op->p * op->n[1] * op->p;
  const int64_t Gz = (int64_t)op->n[2] * op->p;
  const int64_t gz0 = ((int64_t)kz0 * op->p) % Gz, gz1 = ((int64_t)kz1 * op->p) % Gz;
  const int64_t nthr = 2 * prow * ((ncols + 3) / 4);
  if (nthr == 0) return PAWFE_OK;
  const dim3 grid((unsigned)((nthr + 255) / 256)), block(256);
  if (pack)
    hipLaunchKernelGGL(k_halo_pack, grid, block, 0, s, Y, ldy, ncols, gz0 * prow, gz1 * prow, prow, buf);
  else
    hipLaunchKernelGGL(k_halo_unpack, grid, block, 0, s, buf, ncols, gz0 * prow, gz1 * prow, prow, Y, ldy);
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

}  // namespace pawfe
