// C ABI of libpawfe: operator lifetime, applies, the residual-based
// Chebyshev filter (Algorithm 2), Rayleigh-Ritz (Algorithm 1, steps 4-6),
// the band-energy gradient and the Lanczos bound estimate.

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <new>
#include <vector>

#include "kernels.h"

namespace pawfe {

namespace {
thread_local std::string g_last_error;
}

pawfe_status fail(pawfe_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

namespace {

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

template <typename T>
pawfe_status up(pawfe_op* op, T** dptr, const T* src, size_t n, hipStream_t s) {
  const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(PAWFE_ENOMEM, "hipMalloc failed in operator upload");
  op->allocations.push_back(p);
  *dptr = static_cast<T*>(p);
  if (n) PAWFE_HIP(hipMemcpyAsync(p, src, n * sizeof(T), hipMemcpyHostToDevice, s));
  return PAWFE_OK;
}

template <typename T>
pawfe_status up(pawfe_op* op, T** dptr, const std::vector<T>& v, hipStream_t s) {
  return up(op, dptr, v.data(), v.size(), s);
}

std::vector<float> to_f32(const std::vector<double>& v) {
  return std::vector<float>(v.begin(), v.end());
}

#define CHECK(x)                            \
  do {                                      \
    pawfe_status st_ = (x);                 \
    if (st_ != PAWFE_OK) return st_;        \
  } while (0)

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Bump allocator over a caller workspace.
struct Carve {
  char* base;
  size_t off = 0, cap;
  Carve(void* p, size_t c) : base((char*)p), cap(c) {}
  template <typename T>
  T* take(size_t n) {
    T* r = (T*)(base + off);
    off += align256(n * sizeof(T));
    return r;
  }
  bool ok() const { return off <= cap; }
};

// Scratch of one apply over `ncols` columns: partial sums, c, d/q, t (each at
// least one row, as carve_nl takes them, also for an operator without atoms).
size_t nl_scratch_bytes(const pawfe_op* op, int64_t ncols) {
  return align256((size_t)std::max<int64_t>(op->item_rows_total, 1) * ncols * 8) +
         3 * align256((size_t)std::max(op->npj_total, 1) * ncols * 8) + 256;
}

pawfe_status ensure_scratch(pawfe_op* op, size_t bytes) {
  if (op->scratch_bytes >= bytes) return PAWFE_OK;
  if (op->scratch) {
    PAWFE_HIP(hipDeviceSynchronize());
    (void)hipFree(op->scratch);
    op->scratch = nullptr;
    op->scratch_bytes = 0;
  }
  if (hipMalloc(&op->scratch, bytes) != hipSuccess) return fail(PAWFE_ENOMEM, "scratch allocation failed");
  op->scratch_bytes = bytes;
  return PAWFE_OK;
}

struct NlBufs {
  double *part, *c, *d, *t;
};

NlBufs carve_nl(const pawfe_op* op, Carve& cv, int64_t ncols) {
  NlBufs b;
  b.part = cv.take<double>((size_t)std::max<int64_t>(op->item_rows_total, 1) * ncols);
  b.c = cv.take<double>((size_t)std::max(op->npj_total, 1) * ncols);
  b.d = cv.take<double>((size_t)std::max(op->npj_total, 1) * ncols);
  b.t = cv.take<double>((size_t)std::max(op->npj_total, 1) * ncols);
  return b;
}

// ---- building blocks (all enqueue on s) -------------------------------------

template <typename T>
pawfe_status do_apply(const pawfe_op* op, int which, const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols,
                      const NlBufs& b, hipStream_t s, bool bf3 = false) {
  if (which == 0 || which == 1) {   // H or S
    CHECK(launch_nl_reduce<T>(op, X, ldx, ncols, false, b.part, b.c, s, bf3));
    CHECK(launch_atom_mul(op, which == 0 ? op->d.dH : op->d.dS, nullptr, nullptr, 1.0, b.c, b.d, ncols, s));
    if (op->natoms)
      CHECK(launch_node_nl_init<T>(op, b.d, ncols, Y, ldy, s));
    else
      CHECK(launch_node_nl_init<T>(op, nullptr, ncols, Y, ldy, s));
    return launch_cell<T>(op, which == 0 ? kModeH : kModeMass, X, ldx, Y, ldy, ncols, nullptr, 1.0, s, bf3);
  }
  // Sinv_hat
  CHECK(launch_nl_reduce<T>(op, X, ldx, ncols, true, b.part, b.c, s, bf3));
  CHECK(launch_atom_mul(op, op->d.dSinv, nullptr, nullptr, 1.0, b.c, b.d, ncols, s, op->d.dSinv_im));
  return launch_node_sinv<T>(op, X, ldx, b.d, ncols, Y, ldy, s);
}

// Y = H X - S X diag(lam), FP64
pawfe_status do_residual(const pawfe_op* op, const double* X, int64_t ldx, const double* lam, double* Y, int64_t ldy,
                         int ncols, const NlBufs& b, hipStream_t s) {
  CHECK(launch_nl_reduce<double>(op, X, ldx, ncols, false, b.part, b.c, s));
  CHECK(launch_atom_mul(op, op->d.dH, op->d.dS, lam, 1.0, b.c, b.d, ncols, s));
  CHECK(launch_node_nl_init<double>(op, op->natoms ? b.d : nullptr, ncols, Y, ldy, s));
  return launch_cell<double>(op, kModeHRes, X, ldx, Y, ldy, ncols, lam, 1.0, s);
}

// PAWFE_BF16X3: FP32 data, the cell contractions as bf16x3 split products
// (everything else as PAWFE_FP32).
pawfe_status check_prec(int32_t prec, const pawfe_op* op) {
  if (prec != PAWFE_FP64 && prec != PAWFE_FP32 && prec != PAWFE_BF16X3) return fail(PAWFE_EINVAL, "unknown precision");
  if (prec == PAWFE_BF16X3 && op->general)
    return fail(PAWFE_EUNSUPPORTED, "bf16x3 is not built for graded meshes or the GGA term");
  return PAWFE_OK;
}

pawfe_status apply_entry(const pawfe_op* cop, int which, const void* X, int64_t ldx, void* Y, int64_t ldy,
                         int64_t nvec, int32_t prec, void* stream) {
  if (!cop) return fail(PAWFE_EINVAL, "op is NULL");
  if (nvec < 0) return fail(PAWFE_EINVAL, "nvec < 0");
  if (nvec == 0) return PAWFE_OK;
  if (!X || !Y) return fail(PAWFE_EINVAL, "X or Y is NULL");
  if (ldx < nvec || ldy < nvec) return fail(PAWFE_EINVAL, "leading dimension smaller than nvec");
  CHECK(check_prec(prec, cop));
  pawfe_op* op = const_cast<pawfe_op*>(cop);
  if (op->cplx) {   // complex columns as (re, im) pairs of real columns
    nvec *= 2;
    ldx *= 2;
    ldy *= 2;
  }
  const int64_t chunk = 512;
  const int64_t cmax = std::min<int64_t>(chunk, nvec);
  CHECK(ensure_scratch(op, nl_scratch_bytes(op, cmax)));
  Carve cv(op->scratch, op->scratch_bytes);
  NlBufs b = carve_nl(op, cv, cmax);
  if (!cv.ok()) return fail(PAWFE_EINVAL, "internal: apply scratch smaller than its carve");
  hipStream_t s = S(stream);
  for (int64_t j0 = 0; j0 < nvec; j0 += chunk) {
    const int nc = (int)std::min<int64_t>(chunk, nvec - j0);
    if (prec == PAWFE_FP64)
      CHECK(do_apply<double>(op, which, (const double*)X + j0, ldx, (double*)Y + j0, ldy, nc, b, s));
    else
      CHECK(do_apply<float>(op, which, (const float*)X + j0, ldx, (float*)Y + j0, ldy, nc, b, s,
                            prec == PAWFE_BF16X3));
  }
  return PAWFE_OK;
}

// ---- filter ------------------------------------------------------------------

// The filter step fused into the cell kernel (FP64 or FP32 recurrence, on
// uniform and graded meshes); bf16x3 keeps the node-wise step with an
// explicit T.
bool fused_step(const pawfe_op* op, int32_t prec) { return prec != PAWFE_BF16X3 && cell_step_available(op); }

// B: real columns of one block (two per complex column)
size_t filter_ws_bytes(const pawfe_op* op, int64_t B, int32_t prec) {
  const size_t tr = prec == PAWFE_FP64 ? 8 : 4;
  size_t b = align256((size_t)op->M * B * 8);            // Y
  if (fused_step(op, prec)) {
    b += 2 * align256((size_t)op->M * B * tr);                              // RX, RY
    b += 4 * align256((size_t)std::max(op->npj_total, 1) * B * 8);         // c', d_prev, nw (two)
  } else {
    b += 3 * align256((size_t)op->M * B * tr);          // RX, RY, T
  }
  b += nl_scratch_bytes(op, B);
  b += 2 * align256((size_t)B * 8);                      // lamX, lamY
  if (op->cplx) b += align256((size_t)B * 8);             // lambda per real column
  return b + 256;
}

template <typename TR>
pawfe_status filter_block(const pawfe_op* op, const double* X, int64_t ldx, const double* Rin, int64_t ldr,
                          double* Xo, int64_t ldo, int nc, int64_t B, const double* lam_in, int m, double b0,
                          double bW, double bU, Carve cv, hipStream_t s, bool bf3 = false) {
  double* Y = cv.take<double>((size_t)op->M * B);
  TR* RX = cv.take<TR>((size_t)op->M * B);
  TR* RY = cv.take<TR>((size_t)op->M * B);
  TR* Tb = cv.take<TR>((size_t)op->M * B);
  NlBufs nb = carve_nl(op, cv, B);
  double* lamX = cv.take<double>(B);
  double* lamY = cv.take<double>(B);
  if (!cv.ok()) return fail(PAWFE_EINVAL, "internal: filter workspace smaller than its carve");
  const int64_t ld = nc;   // block-local leading dimension
  // step 1 (Algorithm 2): polynomial scalars
  const double e = (bU - bW) / 2.0, c = (bU + bW) / 2.0;
  double zeta = e / (b0 - c);
  const double zeta1 = zeta, gamma = 2.0 / zeta1;
  // step 2: residual of the input pairs, FP64 (or the caller's)
  const double* Yr = Y;
  int64_t ldyr = ld;
  if (Rin) {
    Yr = Rin;
    ldyr = ldr;
  } else {
    CHECK(do_residual(op, X, ldx, lam_in, Y, ld, nc, nb, s));
  }
  // step 3
  CHECK(launch_cheb_init<TR>(op, Yr, ldyr, RY, RX, ld, zeta1 / e, c, lam_in, lamY, lamX, nc, s));
  // step 4
  for (int theta = 2; theta <= m; ++theta) {
    const double znew = 1.0 / (gamma - zeta);
    const double a = 2.0 * znew / e;
    // projector coefficients of Sinv_hat R_Y and of H's non-local term on T
    CHECK(launch_nl_reduce<TR>(op, RY, ld, nc, true, nb.part, nb.c, s, bf3));
    CHECK(launch_atom_mul(op, op->d.dSinv, nullptr, nullptr, 1.0, nb.c, nb.d, nc, s, op->d.dSinv_im));
    CHECK(launch_atom_gcorr(op, nb.c, nb.d, nb.t, nc, s));
    CHECK(launch_atom_mul(op, op->d.dH, nullptr, nullptr, a, nb.t, nb.c, nc, s));   // q = a Dh t (into c)
    // T = Sinv_hat R_Y; R_X <- -a c R_Y - zeta zeta' R_X + a C q + a Y Lambda_Y
    CHECK(launch_node_cheb<TR>(op, RY, RX, Tb, ld, Yr, ldyr, nb.d, nb.c, lamY, lamX, lam_in, a, a * c,
                               zeta * znew, nc, s));
    // R_X += a H_loc T
    CHECK(launch_cell<TR>(op, kModeH, Tb, ld, RX, ld, nc, nullptr, a, s, bf3));
    std::swap(RX, RY);
    std::swap(lamX, lamY);
    zeta = znew;
  }
  // step 5: Xout = Sinv_hat R_Y + X Lambda_Y
  CHECK(launch_nl_reduce<TR>(op, RY, ld, nc, true, nb.part, nb.c, s, bf3));
  CHECK(launch_atom_mul(op, op->d.dSinv, nullptr, nullptr, 1.0, nb.c, nb.d, nc, s, op->d.dSinv_im));
  return launch_node_finalize<TR>(op, RY, ld, nb.d, X, ldx, lamY, Xo, ldo, nc, s);
}

// The same filter with the step's node part fused into the cell kernel
// (FP64 or FP32 recurrence).  R_Y is kept as
// R~ = R - C w with w the projector vector whose C w the previous step still
// owes it (nw = -w is stored), and R_X as R' = R - C d of its own step:
//   c = C^T M_D^{-1} R = reduce(R~) - G nw_prev      (G = C^T M_D^{-1} C)
//   d = Delta_Sinv c,  t = c - G d,  q = a Delta_H t
//   R_Y <- R~ - C (nw_prev + d) = R - C d            (one add-back)
//   R_X <- -a c R_Y - zeta zeta' R_X + a Y Lambda_Y + a H_loc M_D^{-1} R_Y
//          (cell kernel; node part at the first visit of each DOF)
//   nw  = -q + a c d + zeta zeta' d_prev             (R_X is then R~ of the
//                                                      next step)
// which is Algorithm 2's step 4 with T = M_D^{-1}(R_Y - C d) never stored.
template <typename TR>
pawfe_status filter_block_fused(const pawfe_op* op, const double* X, int64_t ldx, const double* Rin, int64_t ldr,
                                double* Xo, int64_t ldo, int nc, int64_t B, const double* lam_in, int m, double b0,
                                double bW, double bU, Carve cv, hipStream_t s) {
  double* Y = cv.take<double>((size_t)op->M * B);
  TR* RX = cv.take<TR>((size_t)op->M * B);
  TR* RY = cv.take<TR>((size_t)op->M * B);
  NlBufs nb = carve_nl(op, cv, B);
  const size_t na = (size_t)std::max(op->npj_total, 1) * B;
  double* c2 = cv.take<double>(na);
  double* dprev = cv.take<double>(na);
  double* nwp = cv.take<double>(na);
  double* nwn = cv.take<double>(na);
  double* lamX = cv.take<double>(B);
  double* lamY = cv.take<double>(B);
  if (!cv.ok()) return fail(PAWFE_EINVAL, "internal: filter workspace smaller than its carve");
  const int64_t ld = nc;
  // step 1: polynomial scalars
  const double e = (bU - bW) / 2.0, c = (bU + bW) / 2.0;
  double zeta = e / (b0 - c);
  const double zeta1 = zeta, gamma = 2.0 / zeta1;
  // step 2: residual of the input pairs, FP64 (or the caller's)
  const double* Yr = Y;
  int64_t ldyr = ld;
  if (Rin) {
    Yr = Rin;
    ldyr = ldr;
  } else {
    CHECK(do_residual(op, X, ldx, lam_in, Y, ld, nc, nb, s));
  }
  // step 3
  CHECK(launch_cheb_init<TR>(op, Yr, ldyr, RY, RX, ld, zeta1 / e, c, lam_in, lamY, lamX, nc, s));
  // step 4
  double* dk = nb.d;
  bool first = true;
  for (int theta = 2; theta <= m; ++theta) {
    const double znew = 1.0 / (gamma - zeta);
    const double a = 2.0 * znew / e;
    const double zz = zeta * znew;
    CHECK(launch_nl_reduce<TR>(op, RY, ld, nc, true, nb.part, nb.c, s));
    const double* cc = nb.c;
    if (!first) {
      CHECK(launch_atom_gcorr(op, nb.c, nwp, c2, nc, s));
      cc = c2;
    }
    CHECK(launch_atom_mul(op, op->d.dSinv, nullptr, nullptr, 1.0, cc, dk, nc, s, op->d.dSinv_im));
    CHECK(launch_atom_gcorr(op, cc, dk, nb.t, nc, s));
    CHECK(launch_atom_mul(op, op->d.dH, nullptr, nullptr, a, nb.t, nb.c, nc, s));   // q = a Dh t (into c)
    CHECK(launch_step_combine(op, nb.c, dk, first ? nullptr : dprev, first ? nullptr : nwp, nb.t, nwn, lamX, lamY,
                              lam_in, a, a * c, zz, nc, s));
    CHECK(launch_node_fixup<TR>(op, nb.t, -1.0, nc, RY, ld, s));
    CHECK(launch_cell_step<TR>(op, RY, RX, ld, Yr, ldyr, lamY, a, a * c, zz, nc, s));
    std::swap(RX, RY);
    std::swap(lamX, lamY);
    std::swap(dk, dprev);
    std::swap(nwp, nwn);
    first = false;
    zeta = znew;
  }
  // step 5: Xout = Sinv_hat R + X Lambda_Y with R = R~ + C w
  CHECK(launch_nl_reduce<TR>(op, RY, ld, nc, true, nb.part, nb.c, s));
  const double* cc = nb.c;
  if (!first) {
    CHECK(launch_atom_gcorr(op, nb.c, nwp, c2, nc, s));
    cc = c2;
  }
  CHECK(launch_atom_mul(op, op->d.dSinv, nullptr, nullptr, 1.0, cc, dk, nc, s, op->d.dSinv_im));
  CHECK(launch_step_combine(op, nullptr, dk, nullptr, first ? nullptr : nwp, nb.t, nullptr, nullptr, nullptr, nullptr,
                            0.0, 0.0, 0.0, nc, s));   // v = nw + d
  return launch_node_finalize<TR>(op, RY, ld, nb.t, X, ldx, lamY, Xo, ldo, nc, s);
}

// ---- small host helpers -----------------------------------------------------

// eigenvalues of a small symmetric tridiagonal matrix by cyclic Jacobi on the dense form
std::vector<double> small_sym_eigvals(int n, std::vector<double> A) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double th = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = cs * akp - sn * akq;
          A[k * n + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = cs * apk - sn * aqk;
          A[q * n + k] = sn * apk + cs * aqk;
        }
      }
  }
  std::vector<double> ev(n);
  for (int i = 0; i < n; ++i) ev[i] = A[i * n + i];
  std::sort(ev.begin(), ev.end());
  return ev;
}

__global__ void k_lincomb(int64_t n, double* __restrict__ y, double a, const double* __restrict__ x, double b,
                          const double* __restrict__ z, double c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + (z ? b * z[i] : 0.0) + (c != 0.0 ? c * y[i] : 0.0);
}

__global__ void k_symmetrize(int N, double* __restrict__ A) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)N * N) return;
  const int i = (int)(idx / N), j = (int)(idx % N);
  if (j <= i) return;
  const double v = 0.5 * (A[(int64_t)i * N + j] + A[(int64_t)j * N + i]);
  A[(int64_t)i * N + j] = v;
  A[(int64_t)j * N + i] = v;
}

// column-major N x N symmetric matrix whose upper triangle holds the values:
// copy it into the lower triangle
__global__ void k_fill_lower(int N, double* __restrict__ A) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)N * N) return;
  const int i = (int)(idx % N), j = (int)(idx / N);
  if (i > j) A[idx] = A[(int64_t)i * N + j];
}

// Complex operators: the realified projection P (2N x 2N, row-major, real
// view of (re, im) column pairs) -> the N x N complex Hermitian matrix
// A_ij = x_i^H (A x)_j, column-major (i + j N), interleaved (re, im)
__global__ void k_form_herm(int N, const double* __restrict__ P, double* __restrict__ A) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)N * N) return;
  const int i = (int)(idx % N), j = (int)(idx / N);
  const int64_t n2 = 2 * (int64_t)N;
  const double rr = P[(2 * i) * n2 + 2 * j], ii = P[(2 * i + 1) * n2 + 2 * j + 1];
  const double ri = P[(2 * i) * n2 + 2 * j + 1], ir = P[(2 * i + 1) * n2 + 2 * j];
  A[2 * idx] = rr + ii;
  A[2 * idx + 1] = ri - ir;
}

// the complex N x N matrix Q (column-major, interleaved) -> its real 2N x 2N
// form R (column-major) acting on (re, im) column pairs: X_new = X R
__global__ void k_realify_rot(int N, const double* __restrict__ Q, double* __restrict__ R) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)N * N) return;
  const int i = (int)(idx % N), j = (int)(idx / N);
  const double qr = Q[2 * idx], qi = Q[2 * idx + 1];
  const int64_t n2 = 2 * (int64_t)N;
  R[(2 * i) + (2 * j) * n2] = qr;
  R[(2 * i + 1) + (2 * j) * n2] = -qi;
  R[(2 * i) + (2 * j + 1) * n2] = qi;
  R[(2 * i + 1) + (2 * j + 1) * n2] = qr;
}

// out[j] = sqrt(sq[2 j] + sq[2 j + 1])
__global__ void k_pair_norm(int N, const double* __restrict__ sq, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < N) out[j] = sqrt(sq[2 * j] + sq[2 * j + 1]);
}

// Mixed-precision subspace rotation, preparation: X32 = fl32(X) (row-major,
// ld N) and Q32 = fl32(Q) with the diagonal blocks (1x1, or the 2x2 blocks
// of a complex entry in the realified form) set to zero (column-major, ld N).
__global__ void k_sr_prep(int64_t M, int N, int bs, const double* __restrict__ X, int64_t ldx,
                          float* __restrict__ X32, const double* __restrict__ Q, float* __restrict__ Q32,
                          double* __restrict__ Qd) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nx = M * N;
  if (t < nx) {
    const int64_t i = t / N;
    const int j = (int)(t - i * N);
    X32[t] = (float)X[i * ldx + j];
  } else if (t < nx + (int64_t)N * N) {
    const int64_t u = t - nx;
    const int c = (int)(u / N), r = (int)(u - (int64_t)c * N);
    const bool diag = r / bs == c / bs;
    Q32[u] = diag ? 0.0f : (float)Q[u];
    if (diag) Qd[(int64_t)c * bs + r % bs] = Q[u];   // the diagonal blocks, compact
  }
}

// X <- X diag(Q) + Y32 (FP64), diag(Q) the diagonal blocks of Q, compact
// (entry (r, c) of the block of columns j0 .. j0 + bs at Qd[(j0 + c) bs + r],
// so neighbouring lanes read neighbouring entries); one thread per row and
// diagonal block, so the in-place update reads the block's inputs before it
// writes.
__global__ void k_sr_combine(int64_t M, int N, int bs, double* __restrict__ X, int64_t ldx,
                             const float* __restrict__ Y32, const double* __restrict__ Qd) {
  const int nb = N / bs;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * nb) return;
  const int64_t i = t / nb;
  const int j0 = (int)(t - i * nb) * bs;
  double x[2], o[2];
  for (int r = 0; r < bs; ++r) x[r] = X[i * ldx + j0 + r];
  for (int c = 0; c < bs; ++c) {
    double v = (double)Y32[i * N + j0 + c];
    for (int r = 0; r < bs; ++r) v += x[r] * Qd[(int64_t)(j0 + c) * bs + r];
    o[c] = v;
  }
  for (int c = 0; c < bs; ++c) X[i * ldx + j0 + c] = o[c];
}

// P[(i0 + i)*ldp + j0 + j] = sum_b part[b][j + i*nc], i < nrow (split-K
// partials of rows i0 .. i0 + nrow of a block column)
__global__ void k_part_reduce(const double* __restrict__ part, int nb, int nc, int nrow, double* __restrict__ P,
                              int64_t ldp, int64_t j0, int64_t i0) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nc * nrow) return;
  const int64_t pstride = (int64_t)nc * nrow;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) acc += part[b * pstride + idx];
  const int64_t i = idx / nc, j = idx % nc;
  P[(i0 + i) * ldp + j0 + j] = acc;
}

}  // namespace

// ---- upload / free ------------------------------------------------------------

pawfe_status upload_veff(pawfe_op* op, hipStream_t s) {
  // complex operators: the 1/2 |k|^2 M term of the Bloch Hamiltonian joins
  // the potential at the Gauss points (same quadrature)
  const double k2 = 0.5 * (op->kpt[0] * op->kpt[0] + op->kpt[1] * op->kpt[1] + op->kpt[2] * op->kpt[2]);
  std::vector<double> vw(op->veff.size());
  for (int e = 0; e < op->E; ++e) {
    const double wsc = op->graded ? op->cell_detJ[e] / op->detJ : 1.0;   // the cell's det J
    for (int q = 0; q < op->nq3; ++q)
      vw[(size_t)e * op->nq3 + q] = (op->veff[(size_t)e * op->nq3 + q] + k2) * (wsc * op->W3[q]);
  }
  std::vector<float> vwf(vw.begin(), vw.end());
  PAWFE_HIP(hipMemcpyAsync(op->d.Vw, vw.data(), vw.size() * 8, hipMemcpyHostToDevice, s));
  PAWFE_HIP(hipMemcpyAsync(op->d.Vw_f, vwf.data(), vwf.size() * 4, hipMemcpyHostToDevice, s));
  PAWFE_HIP(hipStreamSynchronize(s));
  return PAWFE_OK;
}

// per-cell geometry and the GGA table of general operators
pawfe_status upload_general(pawfe_op* op, hipStream_t s) {
  if (!op->general) return PAWFE_OK;
  DeviceTables& d = op->d;
  const int E = op->E, nq = op->nq, nq3 = op->nq3;
  std::vector<double> geo((size_t)E * 4), cs(E, 1.0);
  std::vector<double> hh((size_t)E * 3);
  for (int e = 0; e < E; ++e) {
    const int ijk[3] = {e % op->n[0], (e / op->n[0]) % op->n[1], e / (op->n[0] * op->n[1])};
    double h[3];
    for (int k = 0; k < 3; ++k) h[k] = op->graded ? op->bnd[k][ijk[k] + 1] - op->bnd[k][ijk[k]] : op->h[k];
    const double dJ = op->graded ? op->cell_detJ[e] : op->detJ;
    for (int k = 0; k < 3; ++k) {
      geo[(size_t)e * 4 + k] = 0.5 * dJ * (2.0 / h[k]) * (2.0 / h[k]);
      hh[(size_t)e * 3 + k] = h[k];
    }
    geo[(size_t)e * 4 + 3] = dJ;
    cs[e] = dJ / op->detJ;
  }
  CHECK(up(op, &d.geo, geo, s));
  std::vector<float> geof = to_f32(geo);
  CHECK(up(op, &d.geo_f, geof, s));
  // face factors of the fused filter step: along axis k the lumped mass of
  // a face node is w_0 (h_e + h_neighbour) / 2 per axis; the step kernel's
  // tables assume w_0 h_e (two cells of the cell's own size)
  if (!d.frho) {
    std::vector<double> fr((size_t)E * 6, 1.0);
    for (int e = 0; e < E; ++e) {
      const int ijk[3] = {e % op->n[0], (e / op->n[0]) % op->n[1], e / (op->n[0] * op->n[1])};
      for (int k = 0; k < 3; ++k) {
        auto hk = [&](int i) { return op->graded ? op->bnd[k][i + 1] - op->bnd[k][i] : op->h[k]; };
        const int n = op->n[k], i = ijk[k];
        const double h = hk(i), hlo = hk((i + n - 1) % n), hhi = hk((i + 1) % n);
        fr[(size_t)e * 6 + 2 * k] = 2.0 * h / (h + hlo);
        fr[(size_t)e * 6 + 2 * k + 1] = 2.0 * h / (h + hhi);
      }
    }
    CHECK(up(op, &d.frho, fr, s));
    std::vector<float> frf = to_f32(fr);
    CHECK(up(op, &d.frho_f, frf, s));
  }
  if (op->graded) CHECK(up(op, &d.cscale, cs, s));
  if (op->gga) {
    std::vector<double> vg((size_t)E * 3 * nq3);
    for (int e = 0; e < E; ++e) {
      const double dJ = op->graded ? op->cell_detJ[e] : op->detJ;
      for (int k = 0; k < 3; ++k)
        for (int qz = 0; qz < nq; ++qz)
          for (int qy = 0; qy < nq; ++qy)
            for (int qx = 0; qx < nq; ++qx) {
              const int q = qx + nq * (qy + nq * qz);
              const size_t i = ((size_t)e * 3 + k) * nq3 + q;
              const double w = op->gauss_w[qx] * op->gauss_w[qy] * op->gauss_w[qz] * dJ;
              vg[i] = w * (2.0 / hh[(size_t)e * 3 + k]) * op->vgga[i];
            }
    }
    if (d.vg) {   // replaced (pawfe_set_vgga): same size, overwrite in place
      PAWFE_HIP(hipMemcpyAsync(d.vg, vg.data(), vg.size() * 8, hipMemcpyHostToDevice, s));
      std::vector<float> vgf = to_f32(vg);
      PAWFE_HIP(hipMemcpyAsync(d.vg_f, vgf.data(), vgf.size() * 4, hipMemcpyHostToDevice, s));
      PAWFE_HIP(hipStreamSynchronize(s));
    } else {
      CHECK(up(op, &d.vg, vg, s));
      std::vector<float> vgf = to_f32(vg);
      CHECK(up(op, &d.vg_f, vgf, s));
    }
  }
  PAWFE_HIP(hipStreamSynchronize(s));   // the host vectors above are freed on return
  return PAWFE_OK;
}

pawfe_status upload(pawfe_op* op, hipStream_t s) {
  DeviceTables& d = op->d;
  const size_t nquad = (size_t)op->E * op->nq3;
  {
    void* p = nullptr;
    if (hipMalloc(&p, nquad * 8) != hipSuccess) return fail(PAWFE_ENOMEM, "Vw");
    op->allocations.push_back(p);
    d.Vw = (double*)p;
    if (hipMalloc(&p, nquad * 4) != hipSuccess) return fail(PAWFE_ENOMEM, "Vw_f");
    op->allocations.push_back(p);
    d.Vw_f = (float*)p;
  }
  {
    Tab1D<double> t64{};
    Tab1D<float> t32{};
    const int np = op->np, nq = op->nq;
    for (int i = 0; i < nq * np; ++i) t64.B[i] = op->B[i];
    for (int i = 0; i < np * np; ++i) {
      t64.K1[i] = op->K1[i];
      t64.M1[i] = op->M1[i];
    }
    for (int i = 0; i < np * np; ++i) t64.G1[i] = op->G1[i];
    for (int k = 0; k < 3; ++k) t64.f[k] = 0.5 * op->detJ * (2.0 / op->h[k]) * (2.0 / op->h[k]);
    for (int k = 0; k < 3; ++k) t64.g[k] = -op->kpt[k] * op->detJ * (2.0 / op->h[k]);
    t64.detJ = op->detJ;
    for (int q = 0; q < nq; ++q) t64.w[q] = op->gauss_w[q];
    for (int i = 0; i < kNqMax * kNpMax; ++i) t32.B[i] = (float)t64.B[i];
    for (int i = 0; i < kNpMax * kNpMax; ++i) {
      t32.K1[i] = (float)t64.K1[i];
      t32.M1[i] = (float)t64.M1[i];
      t32.G1[i] = (float)t64.G1[i];
    }
    for (int k = 0; k < 3; ++k) t32.f[k] = (float)t64.f[k];
    for (int k = 0; k < 3; ++k) t32.g[k] = (float)t64.g[k];
    t32.detJ = (float)t64.detJ;
    for (int q = 0; q < kNqMax; ++q) t32.w[q] = (float)t64.w[q];
    CHECK(up(op, &d.tab64, &t64, 1, s));
    CHECK(up(op, &d.tab32, &t32, 1, s));
  }
  CHECK(up(op, &d.W3, op->W3, s));
  std::vector<float> w3f = to_f32(op->W3);
  CHECK(up(op, &d.W3_f, w3f, s));
  std::vector<double> minv(op->M);
  for (int64_t i = 0; i < op->M; ++i) minv[i] = 1.0 / op->MD[i];
  CHECK(up(op, &d.Minv, minv, s));
  std::vector<float> minvf = to_f32(minv);
  CHECK(up(op, &d.Minv_f, minvf, s));
  CHECK(up(op, &d.cells_by_colour, op->cells_by_colour, s));
  if (op->n[0] > 1024 || op->n[1] > 1024 || op->n[2] > 1024) return fail(PAWFE_EINVAL, "more than 1024 cells along an axis");
  std::vector<int32_t> cpk(op->cells_by_colour.size());
  for (size_t t = 0; t < cpk.size(); ++t) {
    const int e = op->cells_by_colour[t];
    cpk[t] = (e % op->n[0]) | ((e / op->n[0]) % op->n[1]) << 10 | (e / (op->n[0] * op->n[1])) << 20;
  }
  CHECK(up(op, &d.cell_pack, cpk, s));
  CHECK(up(op, &d.cell_own, op->cell_own, s));
  CHECK(up(op, &d.node2srow, op->node2srow, s));
  CHECK(up(op, &d.srow_ptr, op->srow_ptr, s));
  CHECK(up(op, &d.srow_atom, op->srow_atom, s));
  CHECK(up(op, &d.srow_coff, op->srow_coff, s));
  CHECK(up(op, &d.Cvals, op->Cvals, s));
  std::vector<float> cf = to_f32(op->Cvals);
  CHECK(up(op, &d.Cvals_f, cf, s));
  std::vector<float> cfi;
  if (op->cplx) {
    CHECK(up(op, &d.Cvals_im, op->Cvals_im, s));
    cfi = to_f32(op->Cvals_im);
    CHECK(up(op, &d.Cvals_im_f, cfi, s));
    CHECK(up(op, &d.Gvals_im, op->Gvals_im, s));
    if (!op->dSinv_im.empty()) CHECK(up(op, &d.dSinv_im, op->dSinv_im, s));
  }
  std::vector<int32_t> an(op->atom_nodes.begin(), op->atom_nodes.end());
  {
    // padded so that batched reads of consecutive rows never leave the list
    std::vector<int32_t> an(op->atom_nodes);
    an.resize(an.size() + 16, an.empty() ? 0 : an.back());
    CHECK(up(op, &d.atom_nodes, an, s));
  }
  CHECK(up(op, &d.item_atom, op->item_atom, s));
  CHECK(up(op, &d.item_row0, op->item_row0, s));
  CHECK(up(op, &d.item_row1, op->item_row1, s));
  CHECK(up(op, &d.item_poff, op->item_poff, s));
  CHECK(up(op, &d.item_ptr, op->item_ptr, s));
  CHECK(up(op, &d.fix_atom, op->fix_atom, s));
  CHECK(up(op, &d.fix_row0, op->fix_row0, s));
  CHECK(up(op, &d.fix_row1, op->fix_row1, s));
  CHECK(up(op, &d.atom_noff, op->atom_noff, s));
  CHECK(up(op, &d.atom_coff, op->atom_coff, s));
  CHECK(up(op, &d.nproj, op->nproj, s));
  CHECK(up(op, &d.poff, op->poff, s));
  CHECK(up(op, &d.poff2, op->poff2, s));
  CHECK(up(op, &d.dH, op->dH, s));
  CHECK(up(op, &d.dS, op->dS, s));
  CHECK(up(op, &d.dSinv, op->dSinv, s));
  CHECK(up(op, &d.gp_ptr, op->gp_ptr, s));
  CHECK(up(op, &d.gp_b, op->gp_b, s));
  CHECK(up(op, &d.gp_off, op->gp_off, s));
  CHECK(up(op, &d.Gvals, op->Gvals, s));
  std::vector<int32_t> pa(op->npj_total), pal(op->npj_total), ga, gs, gt;
  for (int a = 0; a < op->natoms; ++a)
    for (int t = 0; t < op->nproj[a]; ++t) {
      pa[op->poff[a] + t] = a;
      pal[op->poff[a] + t] = t;
    }
  for (int a = 0; a < op->natoms; ++a)
    for (int i = 0; i < op->nproj[a]; ++i)
      for (int j = 0; j < op->nproj[a]; ++j) {
        ga.push_back(a);
        gs.push_back(i);
        gt.push_back(j);
      }
  CHECK(up(op, &op->d_proj_atom, pa, s));
  CHECK(up(op, &op->d_proj_alpha, pal, s));
  CHECK(up(op, &op->d_g2_atom, ga, s));
  CHECK(up(op, &op->d_g2_s, gs, s));
  CHECK(up(op, &op->d_g2_t, gt, s));
  CHECK(upload_general(op, s));
  return upload_veff(op, s);
}

void free_device(pawfe_op* op) {
  for (void* p : op->allocations) (void)hipFree(p);
  op->allocations.clear();
  if (op->scratch) (void)hipFree(op->scratch);
  op->scratch = nullptr;
  op->scratch_bytes = 0;
  if (op->blas) rocblas_destroy_handle((rocblas_handle)op->blas);
  op->blas = nullptr;
  for (hipEvent_t& e : op->fevent) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
}

// The filter's block streams (default priority): one set per device, shared
// by every operator, created on first use and kept until the process ends.
// A process has few hardware queues (four by default) and streams beyond
// them share queues, so a set of block streams per operator would leave the
// blocks of one operator's filter serialized on one queue once other
// operators had created theirs (measured: 12-19 % slower filter passes).
pawfe_status block_streams(int n, hipStream_t* out) {
  static std::mutex mu;
  static std::vector<std::array<hipStream_t, kMaxConcBlocks>> per_dev;
  int dev = 0;
  PAWFE_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  if ((int)per_dev.size() <= dev) per_dev.resize(dev + 1);
  for (int q = 0; q < n; ++q) {
    hipStream_t& st = per_dev[dev][q];
    if (!st) PAWFE_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    out[q] = st;
  }
  return PAWFE_OK;
}

}  // namespace pawfe

using namespace pawfe;

// ---- static scratch of the allocation-free apply ----------------------------

// Projector scratch of pawfe_apply_H_noalloc: one array per GPU, resident
// from the library's load on that GPU until the process ends.  Host code
// never uses the array's name as an address: each device's address comes
// from hipGetSymbolAddress, taken once per device with that device current.
// Every call on a GPU shares that GPU's array, so calls that overlap on one
// GPU race.  Nothing in it has to start at zero: each apply writes every
// partial sum and coefficient it reads.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace pawfe {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

pawfe_status static_scratch(void** out) {
  int dev = 0;
  PAWFE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PAWFE_EUNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    PAWFE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(PAWFE_EHIP, "hipGetSymbolAddress returned NULL for the static scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PAWFE_OK;
}
}  // namespace
}  // namespace pawfe

extern "C" {

const char* pawfe_last_error(void) { return g_last_error.c_str(); }

pawfe_status pawfe_build_operator(const pawfe_op_desc* desc, void* stream, pawfe_op** out) {
  if (!out) return fail(PAWFE_EINVAL, "out is NULL");
  *out = nullptr;
  pawfe_op* op = new (std::nothrow) pawfe_op();
  if (!op) return fail(PAWFE_ENOMEM, "host allocation failed");
  pawfe_status st;
  try {
    st = build_host(desc, op);
  } catch (const std::bad_alloc&) {
    st = fail(PAWFE_ENOMEM, "host allocation failed while building");
  } catch (...) {
    st = fail(PAWFE_EINVAL, "unexpected error while building");
  }
  if (st == PAWFE_OK) st = upload(op, S(stream));
  if (st == PAWFE_OK) {
    hipError_t e = hipStreamSynchronize(S(stream));
    if (e != hipSuccess) st = fail(PAWFE_EHIP, std::string("upload: ") + hipGetErrorString(e));
  }
  if (st != PAWFE_OK) {
    free_device(op);
    delete op;
    return st;
  }
  *out = op;
  g_last_error.clear();
  return PAWFE_OK;
}

pawfe_status pawfe_destroy_operator(pawfe_op* op) {
  if (!op) return PAWFE_OK;
  (void)hipDeviceSynchronize();
  free_device(op);
  delete op;
  return PAWFE_OK;
}

pawfe_status pawfe_query(const pawfe_op* op, int64_t* ndof, int64_t* nquad, int32_t* ncolour, int32_t* nproj_total,
                         int64_t* nsupp_cells, int64_t* nsupp_nodes) {
  if (!op) return fail(PAWFE_EINVAL, "op is NULL");
  if (ndof) *ndof = op->M;
  if (nquad) *nquad = (int64_t)op->E * op->nq3;
  if (ncolour) *ncolour = op->ncolour;
  if (nproj_total) *nproj_total = op->npj_total;
  if (nsupp_cells) *nsupp_cells = (int64_t)op->supp_cells.size();
  if (nsupp_nodes) *nsupp_nodes = (int64_t)op->supp_nodes.size();
  return PAWFE_OK;
}

pawfe_status pawfe_get_dofmap(const pawfe_op* op, int32_t* cell_dofs, int32_t* cell_colour, int64_t* supp_cell_off,
                              int64_t* supp_cells, int64_t* supp_node_off, int64_t* supp_nodes) {
  if (!op) return fail(PAWFE_EINVAL, "op is NULL");
  if (cell_dofs) {
    const int np = op->np, p = op->p;
    const int Gx = op->n[0] * p, Gy = op->n[1] * p, Gz = op->n[2] * p;
    for (int e = 0; e < op->E; ++e) {
      const int i = e % op->n[0], j = (e / op->n[0]) % op->n[1], k = e / (op->n[0] * op->n[1]);
      for (int l = 0; l < op->nloc; ++l) {
        const int a = l % np, b = (l / np) % np, c = l / (np * np);
        const int64_t gx = (i * p + a) % Gx, gy = (j * p + b) % Gy, gz = (k * p + c) % Gz;
        cell_dofs[(int64_t)e * op->nloc + l] = (int32_t)(gx + (int64_t)Gx * (gy + (int64_t)Gy * gz));
      }
    }
  }
  if (cell_colour) std::copy(op->cell_colour.begin(), op->cell_colour.end(), cell_colour);
  if (supp_cell_off) std::copy(op->supp_cell_off.begin(), op->supp_cell_off.end(), supp_cell_off);
  if (supp_cells) std::copy(op->supp_cells.begin(), op->supp_cells.end(), supp_cells);
  if (supp_node_off) std::copy(op->supp_node_off.begin(), op->supp_node_off.end(), supp_node_off);
  if (supp_nodes) std::copy(op->supp_nodes.begin(), op->supp_nodes.end(), supp_nodes);
  return PAWFE_OK;
}

pawfe_status pawfe_get_first_visit(const pawfe_op* op, uint32_t* first_visit) {
  if (!op || !first_visit) return fail(PAWFE_EINVAL, "op or first_visit is NULL");
  std::copy(op->cell_own.begin(), op->cell_own.end(), first_visit);
  return PAWFE_OK;
}

pawfe_status pawfe_set_veff(pawfe_op* op, const double* veff_q, void* stream) {
  if (!op || !veff_q) return fail(PAWFE_EINVAL, "op or veff_q is NULL");
  const size_t n = (size_t)op->E * op->nq3;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(veff_q[i])) return fail(PAWFE_ENONFINITE, "veff_q has NaN/Inf");
  op->veff.assign(veff_q, veff_q + n);
  return upload_veff(op, S(stream));
}

pawfe_status pawfe_set_vgga(pawfe_op* op, const double* vgga_q, void* stream) {
  if (!op || !vgga_q) return fail(PAWFE_EINVAL, "op or vgga_q is NULL");
  if (!op->gga) return fail(PAWFE_EINVAL, "the operator was built without a GGA field");
  const size_t n = (size_t)op->E * 3 * op->nq3;
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(vgga_q[i])) return fail(PAWFE_ENONFINITE, "vgga_q has NaN/Inf");
  op->vgga.assign(vgga_q, vgga_q + n);
  return upload_general(op, S(stream));
}

pawfe_status pawfe_set_dH(pawfe_op* op, const double* dH, void* stream) {
  if (!op || (!dH && op->npj2_total)) return fail(PAWFE_EINVAL, "op or dH is NULL");
  for (int i = 0; i < op->npj2_total; ++i)
    if (!std::isfinite(dH[i])) return fail(PAWFE_ENONFINITE, "dH has NaN/Inf");
  op->dH.assign(dH, dH + op->npj2_total);
  if (op->npj2_total)
    PAWFE_HIP(hipMemcpyAsync(op->d.dH, op->dH.data(), op->dH.size() * 8, hipMemcpyHostToDevice, S(stream)));
  PAWFE_HIP(hipStreamSynchronize(S(stream)));
  return PAWFE_OK;
}

pawfe_status pawfe_apply_H(const pawfe_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int64_t nvec,
                           int32_t prec, void* stream) {
  return apply_entry(op, 0, X, ldx, Y, ldy, nvec, prec, stream);
}

pawfe_status pawfe_apply_H_noalloc(const pawfe_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy,
                                   int64_t nvec, int32_t prec, void* stream) {
  if (!op) return fail(PAWFE_EINVAL, "op is NULL");
  if (nvec < 0) return fail(PAWFE_EINVAL, "nvec < 0");
  if (nvec == 0) return PAWFE_OK;
  if (!X || !Y) return fail(PAWFE_EINVAL, "X or Y is NULL");
  if (ldx < nvec || ldy < nvec) return fail(PAWFE_EINVAL, "leading dimension smaller than nvec");
  CHECK(check_prec(prec, op));
  const int64_t cf = op->cplx ? 2 : 1;   // complex columns as (re, im) pairs of real columns
  nvec *= cf;
  ldx *= cf;
  ldy *= cf;
  // column chunk: the widest (at most 512 real columns) whose projector
  // scratch fits the static array
  if (nl_scratch_bytes(op, cf) > kStaticScratchBytes)
    return fail(PAWFE_EINVAL, "the operator's projector scratch for one column exceeds the " +
                                  std::to_string(kStaticScratchBytes >> 20) + " MiB static scratch of this entry point");
  int64_t chunk = std::min<int64_t>(512, nvec);
  while (chunk > cf && nl_scratch_bytes(op, chunk) > kStaticScratchBytes) chunk -= cf;
  void* base = nullptr;
  CHECK(static_scratch(&base));
  Carve cv(base, kStaticScratchBytes);
  NlBufs b = carve_nl(op, cv, chunk);
  if (!cv.ok()) return fail(PAWFE_EINVAL, "internal: static scratch smaller than its carve");
  hipStream_t s = S(stream);
  for (int64_t j0 = 0; j0 < nvec; j0 += chunk) {
    const int nc = (int)std::min<int64_t>(chunk, nvec - j0);
    if (prec == PAWFE_FP64)
      CHECK(do_apply<double>(op, 0, (const double*)X + j0, ldx, (double*)Y + j0, ldy, nc, b, s));
    else
      CHECK(do_apply<float>(op, 0, (const float*)X + j0, ldx, (float*)Y + j0, ldy, nc, b, s,
                            prec == PAWFE_BF16X3));
  }
  return PAWFE_OK;
}

static pawfe_status halo_args(const pawfe_op* op, const void* Y, int64_t ldy, int64_t nvec, int32_t kz0,
                              int32_t kz1, const void* buf) {
  if (!op) return fail(PAWFE_EINVAL, "op is NULL");
  if (nvec < 0) return fail(PAWFE_EINVAL, "nvec < 0");
  if (nvec > 0 && (!Y || !buf)) return fail(PAWFE_EINVAL, "Y or buf is NULL");
  if (ldy < nvec) return fail(PAWFE_EINVAL, "leading dimension smaller than nvec");
  if (!(0 <= kz0 && kz0 < kz1 && kz1 <= op->n[2] && kz1 - kz0 < op->n[2]))
    return fail(PAWFE_EINVAL, "slab must satisfy 0 <= kz0 < kz1 <= nz and be thinner than the mesh");
  if (nvec * (op->cplx ? 2 : 1) > (int64_t)1 << 30) return fail(PAWFE_EINVAL, "nvec too large");
  return PAWFE_OK;
}

pawfe_status pawfe_halo_pack_bf16(const pawfe_op* op, const float* Y, int64_t ldy, int64_t nvec, int32_t kz0,
                                  int32_t kz1, uint16_t* buf, void* stream) {
  CHECK(halo_args(op, Y, ldy, nvec, kz0, kz1, buf));
  const int64_t cf = op->cplx ? 2 : 1;
  return launch_halo(op, true, const_cast<float*>(Y), ldy * cf, (int)(nvec * cf), kz0, kz1, buf, S(stream));
}

pawfe_status pawfe_halo_unpack_bf16(const pawfe_op* op, const uint16_t* buf, int64_t nvec, int32_t kz0, int32_t kz1,
                                    float* Y, int64_t ldy, void* stream) {
  CHECK(halo_args(op, Y, ldy, nvec, kz0, kz1, buf));
  const int64_t cf = op->cplx ? 2 : 1;
  return launch_halo(op, false, Y, ldy * cf, (int)(nvec * cf), kz0, kz1, const_cast<uint16_t*>(buf), S(stream));
}

pawfe_status pawfe_apply_S(const pawfe_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int64_t nvec,
                           int32_t prec, void* stream) {
  return apply_entry(op, 1, X, ldx, Y, ldy, nvec, prec, stream);
}

pawfe_status pawfe_apply_Sinv(const pawfe_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int64_t nvec,
                              int32_t prec, void* stream) {
  return apply_entry(op, 2, X, ldx, Y, ldy, nvec, prec, stream);
}

pawfe_status pawfe_apply_local(const pawfe_op* op, int32_t which, const void* X, int64_t ldx, void* Y,
                               int64_t ldy, int64_t nvec, double alpha, int32_t prec, void* stream) {
  if (!op) return fail(PAWFE_EINVAL, "op is NULL");
  if (which != 0 && which != 1) return fail(PAWFE_EINVAL, "which must be 0 (K + V) or 1 (M)");
  if (nvec < 0) return fail(PAWFE_EINVAL, "nvec < 0");
  if (nvec == 0) return PAWFE_OK;
  if (!X || !Y) return fail(PAWFE_EINVAL, "X or Y is NULL");
  if (ldx < nvec || ldy < nvec) return fail(PAWFE_EINVAL, "leading dimension smaller than nvec");
  CHECK(check_prec(prec, op));
  const int mode = which == 0 ? kModeH : kModeMass;
  if (nvec > (int64_t)1 << 29) return fail(PAWFE_EINVAL, "nvec too large");
  if (op->cplx) {   // complex columns as (re, im) pairs of real columns
    nvec *= 2;
    ldx *= 2;
    ldy *= 2;
  }
  if (prec == PAWFE_FP64)
    return launch_cell<double>(op, mode, (const double*)X, ldx, (double*)Y, ldy, (int)nvec, nullptr, alpha,
                               S(stream));
  return launch_cell<float>(op, mode, (const float*)X, ldx, (float*)Y, ldy, (int)nvec, nullptr, alpha, S(stream),
                            prec == PAWFE_BF16X3);
}

pawfe_status pawfe_cheb_step_local(const pawfe_op* op, const void* RY, void* RX, int64_t ld, const double* Y,
                                   int64_t ldy, const double* lamY, double a, double ac, double zz, int64_t nvec,
                                   int32_t prec, void* stream) {
  if (!op) return fail(PAWFE_EINVAL, "op is NULL");
  if (nvec < 0 || nvec > (int64_t)1 << 29) return fail(PAWFE_EINVAL, "nvec out of range");
  if (nvec == 0) return PAWFE_OK;
  if (!RY || !RX || !Y || !lamY) return fail(PAWFE_EINVAL, "NULL buffer");
  if (ld < nvec || ldy < nvec) return fail(PAWFE_EINVAL, "leading dimension smaller than nvec");
  if (op->cplx && (nvec & 1)) return fail(PAWFE_EINVAL, "complex operators take (re, im) column pairs");
  if (prec != PAWFE_FP64 && prec != PAWFE_FP32)
    return fail(PAWFE_EUNSUPPORTED, "the step kernel runs in FP64 or FP32");
  if (!cell_step_available(op))
    return fail(PAWFE_EUNSUPPORTED, "no step variant for this operator (graded mesh, GGA term or element)");
  if (prec == PAWFE_FP64)
    return launch_cell_step<double>(op, (const double*)RY, (double*)RX, ld, Y, ldy, lamY, a, ac, zz, (int)nvec,
                                    S(stream));
  return launch_cell_step<float>(op, (const float*)RY, (float*)RX, ld, Y, ldy, lamY, a, ac, zz, (int)nvec, S(stream));
}

pawfe_status pawfe_cheb_filter_workspace(const pawfe_op* op, int64_t nvec, int32_t block, int32_t prec,
                                         size_t* bytes) {
  if (!op || !bytes) return fail(PAWFE_EINVAL, "op or bytes is NULL");
  if (nvec < 1 || block < 1) return fail(PAWFE_EINVAL, "nvec and block must be >= 1");
  CHECK(check_prec(prec, op));
  const int64_t B = std::min<int64_t>(block, nvec);
  // room for two blocks in flight when there is more than one block
  *bytes = filter_ws_bytes(op, B * (op->cplx ? 2 : 1), prec) * (nvec > B ? 2 : 1);
  return PAWFE_OK;
}

// the filter; R (ldr) is the caller's FP64 residual H X - S X Lambda of
// the input columns, or NULL to form it (step 2 of Algorithm 2)
static pawfe_status cheb_filter_impl(const pawfe_op* op, const void* Xin, int64_t ldx, const double* R, int64_t ldr,
                                     void* Xout, int64_t ldo, int64_t nvec, int32_t block, const double* lambda_in,
                                     int32_t degree, double b0, double bW, double bU, int32_t prec, void* ws,
                                     size_t ws_bytes, void* stream) {
  if (!op) return fail(PAWFE_EINVAL, "op is NULL");
  if (!Xin || !Xout || !lambda_in || !ws) return fail(PAWFE_EINVAL, "NULL buffer");
  if (nvec < 1 || block < 1) return fail(PAWFE_EINVAL, "nvec and block must be >= 1");
  if (ldx < nvec || ldo < nvec) return fail(PAWFE_EINVAL, "leading dimension smaller than nvec");
  if (degree < 2) return fail(PAWFE_EINVAL, "Chebyshev degree must be >= 2");
  if (!(std::isfinite(b0) && std::isfinite(bW) && std::isfinite(bU)))
    return fail(PAWFE_ENONFINITE, "bounds must be finite");
  if (!(b0 < bW && bW < bU)) return fail(PAWFE_EINVAL, "bounds must satisfy b0 < bW < bU");
  CHECK(check_prec(prec, op));
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(PAWFE_EINVAL, "workspace must be 256-byte aligned");
  const int64_t cf = op->cplx ? 2 : 1;   // real columns per column
  const int64_t B = std::min<int64_t>(block, nvec);
  const size_t one = filter_ws_bytes(op, B * cf, prec);
  if (ws_bytes < one) return fail(PAWFE_EINVAL, "workspace too small");
  hipStream_t s = S(stream);
  // Blocks are uncoupled.  With room for several block states (and more
  // than one block), block b runs on internal stream b mod nconc, forked
  // from and joined back into `s`: one block's projector and node kernels
  // then overlap another's cell kernel.
  const int64_t nblocks = (nvec + B - 1) / B;
  const int nconc = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)kMaxConcBlocks, nblocks,
                                                                  (int64_t)(ws_bytes / one)}));
  pawfe_op* mop = const_cast<pawfe_op*>(op);
  hipStream_t bstream[kMaxConcBlocks] = {};
  if (nconc > 1) {
    CHECK(block_streams(nconc, bstream));
    for (int q = 0; q <= nconc; ++q)
      if (!mop->fevent[q]) PAWFE_HIP(hipEventCreateWithFlags(&mop->fevent[q], hipEventDisableTiming));
    PAWFE_HIP(hipEventRecord(mop->fevent[0], s));
    for (int q = 0; q < nconc; ++q) PAWFE_HIP(hipStreamWaitEvent(bstream[q], mop->fevent[0], 0));
  }
  for (int64_t j0 = 0, blk = 0; j0 < nvec; j0 += B, ++blk) {
    const int nc = (int)std::min<int64_t>(B, nvec - j0);
    const int k = nconc > 1 ? (int)(blk % nconc) : 0;
    hipStream_t sb = nconc > 1 ? bstream[k] : s;
    Carve cv((char*)ws + (size_t)k * one, one);
    const double* X = (const double*)Xin + j0 * cf;
    const double* Rb = R ? R + j0 * cf : nullptr;
    double* Xo = (double*)Xout + j0 * cf;
    const double* lam = lambda_in + j0;
    pawfe_status st = PAWFE_OK;
    if (op->cplx) {   // lambda per real column of the (re, im) pairs
      double* lam2 = cv.take<double>((size_t)B * cf);
      st = launch_dup_pairs(lambda_in + j0, lam2, nc, sb);
      lam = lam2;
    }
    if (st != PAWFE_OK) {
    } else if (fused_step(op, prec)) {
      st = prec == PAWFE_FP64
               ? filter_block_fused<double>(op, X, ldx * cf, Rb, ldr * cf, Xo, ldo * cf, (int)(nc * cf), B * cf, lam,
                                            degree, b0, bW, bU, cv, sb)
               : filter_block_fused<float>(op, X, ldx * cf, Rb, ldr * cf, Xo, ldo * cf, (int)(nc * cf), B * cf, lam,
                                           degree, b0, bW, bU, cv, sb);
    } else if (prec == PAWFE_FP64) {
      st = filter_block<double>(op, X, ldx * cf, Rb, ldr * cf, Xo, ldo * cf, (int)(nc * cf), B * cf, lam, degree, b0,
                                bW, bU, cv, sb);
    } else {
      st = filter_block<float>(op, X, ldx * cf, Rb, ldr * cf, Xo, ldo * cf, (int)(nc * cf), B * cf, lam, degree, b0,
                               bW, bU, cv, sb, prec == PAWFE_BF16X3);
    }
    if (st != PAWFE_OK) {
      if (nconc > 1)   // still join, so `s` never runs ahead of work already enqueued
        for (int q = 0; q < nconc; ++q) {
          (void)hipEventRecord(mop->fevent[1 + q], bstream[q]);
          (void)hipStreamWaitEvent(s, mop->fevent[1 + q], 0);
        }
      return st;
    }
  }
  if (nconc > 1)
    for (int q = 0; q < nconc; ++q) {
      PAWFE_HIP(hipEventRecord(mop->fevent[1 + q], bstream[q]));
      PAWFE_HIP(hipStreamWaitEvent(s, mop->fevent[1 + q], 0));
    }
  return PAWFE_OK;
}

pawfe_status pawfe_cheb_filter(const pawfe_op* op, const void* Xin, int64_t ldx, void* Xout, int64_t ldo,
                               int64_t nvec, int32_t block, const double* lambda_in, int32_t degree, double b0,
                               double bW, double bU, int32_t prec, void* ws, size_t ws_bytes, void* stream) {
  return cheb_filter_impl(op, Xin, ldx, nullptr, 0, Xout, ldo, nvec, block, lambda_in, degree, b0, bW, bU, prec, ws,
                          ws_bytes, stream);
}

pawfe_status pawfe_cheb_filter_res(const pawfe_op* op, const void* Xin, int64_t ldx, const void* R, int64_t ldr,
                                   void* Xout, int64_t ldo, int64_t nvec, int32_t block, const double* lambda_in,
                                   int32_t degree, double b0, double bW, double bU, int32_t prec, void* ws,
                                   size_t ws_bytes, void* stream) {
  if (!R) return fail(PAWFE_EINVAL, "R is NULL");
  if (ldr < nvec) return fail(PAWFE_EINVAL, "leading dimension of R smaller than nvec");
  if (R == Xout) return fail(PAWFE_EINVAL, "R must not be the output");
  return cheb_filter_impl(op, Xin, ldx, (const double*)R, ldr, Xout, ldo, nvec, block, lambda_in, degree, b0, bW, bU,
                          prec, ws, ws_bytes, stream);
}

// ---- Rayleigh-Ritz ------------------------------------------------------------

static size_t rr_ws_bytes(const pawfe_op* op, int64_t N) {
  N *= op->cplx ? 2 : 1;   // real columns
  const int64_t B = std::min<int64_t>(256, N);
  size_t b = align256((size_t)op->M * B * 8);             // HX block
  b += align256((size_t)op->M * N * 8);                    // rotated copy
  b += 2 * align256((size_t)N * N * 8);                    // Hp, Sp
  b += align256((size_t)64 * N * N * 8);                   // split-K partials
  b += align256((size_t)N * 8) + 256;                      // E work, info
  b += align256((size_t)((op->M + 4095) / 4096) * B * 8);  // norm partials
  b += nl_scratch_bytes(op, B);
  return b + 256;
}

pawfe_status pawfe_rayleigh_ritz_workspace(const pawfe_op* op, int64_t nvec, size_t* bytes) {
  if (!op || !bytes) return fail(PAWFE_EINVAL, "op or bytes is NULL");
  if (nvec < 1) return fail(PAWFE_EINVAL, "nvec must be >= 1");
  *bytes = rr_ws_bytes(op, nvec);
  return PAWFE_OK;
}

// Rayleigh-Ritz; R (ldr), when not NULL, receives the FP64 residual
// H x - lambda S x of the rotated columns (the blocks whose norms are taken)
static pawfe_status rayleigh_ritz_impl(const pawfe_op* cop, void* Xv, int64_t ldx, int64_t N, double* lambda,
                                       double* resnorm, double* R, int64_t ldr, int32_t sr_prec, void* ws,
                                       size_t ws_bytes, void* stream) {
  if (!cop) return fail(PAWFE_EINVAL, "op is NULL");
  if (!Xv || !lambda || !resnorm || !ws) return fail(PAWFE_EINVAL, "NULL buffer");
  if (N < 1 || ldx < N) return fail(PAWFE_EINVAL, "bad nvec / ldx");
  if (N > 65536) return fail(PAWFE_EUNSUPPORTED, "nvec too large for the dense projected problem");
  if (sr_prec != PAWFE_FP64 && sr_prec != PAWFE_FP32) return fail(PAWFE_EINVAL, "sr_prec must be FP64 or FP32");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(PAWFE_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < rr_ws_bytes(cop, N)) return fail(PAWFE_EINVAL, "workspace too small");
  pawfe_op* op = const_cast<pawfe_op*>(cop);
  hipStream_t s = S(stream);
  double* X = (double*)Xv;
  // complex operators: the (re, im) real view, Nc complex columns
  const int64_t Nc = N;
  if (op->cplx) {
    N *= 2;
    ldx *= 2;
    ldr *= 2;
  }
  const int64_t B = std::min<int64_t>(256, N);
  Carve cv(ws, ws_bytes);
  double* HXb = cv.take<double>((size_t)op->M * B);
  double* Xr = cv.take<double>((size_t)op->M * N);
  double* Hp = cv.take<double>((size_t)N * N);
  double* Sp = cv.take<double>((size_t)N * N);
  const size_t npart = (size_t)64 * N * N;
  double* part = cv.take<double>(npart);
  double* Ework = cv.take<double>(N);
  rocblas_int* info = cv.take<rocblas_int>(1);
  double* npart_buf = cv.take<double>((size_t)((op->M + 4095) / 4096) * B);
  NlBufs nb = carve_nl(op, cv, B);
  if (!cv.ok()) return fail(PAWFE_EINVAL, "internal: Rayleigh-Ritz workspace smaller than its carve");
  if (!op->blas) {
    rocblas_handle h;
    if (rocblas_create_handle(&h) != rocblas_status_success) return fail(PAWFE_EHIP, "rocblas_create_handle failed");
    op->blas = h;
  }
  rocblas_handle h = (rocblas_handle)op->blas;
  if (rocblas_set_stream(h, s) != rocblas_status_success) return fail(PAWFE_EHIP, "rocblas_set_stream failed");
  // projection: H^p = X^T H X, S^p = X^T S X, block column by block column.
  // Each block is a plain FP64 GEMM with K = ndof: rocBLAS on the matrix
  // cores, split over K into `nsk` strided-batched pieces (the output is only
  // N x nc, so K is where the parallelism is), then a fixed-order sum.
  // Row-major X [K][ldx] is the column-major matrix X^T, so the block
  // P[:, j0:j0+nc] (row-major) is the column-major product HXb^T-block
  // (nc x K) times X (K x N).
  // Real operators: only the rows i >= j0 of block column j0 (the lower
  // triangle in row-major order, which is the upper triangle the dense solver
  // reads in its column-major view) are formed, as the paper's projection
  // step evaluates one triangle; complex operators form the whole realified
  // matrices (the Hermitian fold reads both triangles) and symmetrize them.
  const int64_t K = op->M;
  const bool lower_only = !op->cplx;
  for (int which = 0; which < 2; ++which) {
    double* P = which == 0 ? Hp : Sp;
    for (int64_t j0 = 0; j0 < N; j0 += B) {
      const int nc = (int)std::min<int64_t>(B, N - j0);
      const int64_t i0 = lower_only ? j0 : 0, nrow = N - i0;
      CHECK(do_apply<double>(op, which, X + j0, ldx, HXb, nc, nc, nb, s));
      const int64_t pbytes = (int64_t)nc * nrow;
      int64_t nsk = std::min<int64_t>(32, std::max<int64_t>(1, (int64_t)(npart / (size_t)pbytes) - 1));
      nsk = std::max<int64_t>(1, std::min<int64_t>(nsk, K / 1024));
      const int64_t kc = K / nsk, krem = K - nsk * kc;
      const double one = 1.0, zero = 0.0;
      if (rocblas_dgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_transpose, nc, (rocblas_int)nrow,
                                        (rocblas_int)kc, &one, HXb, nc, kc * nc, X + i0, (rocblas_int)ldx, kc * ldx,
                                        &zero, part, nc, pbytes, (rocblas_int)nsk) != rocblas_status_success)
        return fail(PAWFE_EHIP, "rocblas_dgemm_strided_batched failed");
      int64_t nparts = nsk;
      if (krem > 0) {
        if (rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, nc, (rocblas_int)nrow,
                          (rocblas_int)krem, &one, HXb + nsk * kc * nc, nc, X + nsk * kc * ldx + i0,
                          (rocblas_int)ldx, &zero, part + nsk * pbytes, nc) != rocblas_status_success)
          return fail(PAWFE_EHIP, "rocblas_dgemm failed");
        ++nparts;
      }
      hipLaunchKernelGGL(k_part_reduce, dim3((unsigned)((pbytes + 255) / 256)), dim3(256), 0, s, part, (int)nparts,
                         nc, (int)nrow, P, (int64_t)N, j0, i0);
    }
    if (!lower_only)
      hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)((N * N + 255) / 256)), dim3(256), 0, s, (int)N, P);
  }
  PAWFE_HIP(hipGetLastError());
  // projected generalized eigenproblem H^p q = lambda S^p q (dense, FP64),
  // reduced to a standard one: S^p = U^H U (Cholesky), U^-H H^p U^-1 z =
  // lambda z, q = U^-1 z (so Q^H S^p Q = I).  The two-sided transform and the
  // back-transform are blocked triangular solves on the matrix cores.
  // Complex operators: the Hermitian N x N problem formed from the realified
  // projections (in the split-K buffer, free by now), solved complex, and its
  // eigenvectors turned into the real rotation of the (re, im) pairs (into Hp)
  double* lam2 = nullptr;
  double* Hc = part;
  double* Sc = part + 2 * Nc * Nc;
  const dim3 gq((unsigned)((Nc * Nc + 255) / 256));
  const rocblas_double_complex onez(1.0, 0.0);
  const double one = 1.0;
  auto read_info = [&](rocblas_int* v) -> pawfe_status {
    PAWFE_HIP(hipMemcpyAsync(v, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
    PAWFE_HIP(hipStreamSynchronize(s));
    return PAWFE_OK;
  };
  rocblas_status rs;
  if (!op->cplx) {
    hipLaunchKernelGGL(k_fill_lower, gq, dim3(256), 0, s, (int)N, Hp);
    PAWFE_HIP(hipGetLastError());
    rs = rocsolver_dpotrf(h, rocblas_fill_upper, (rocblas_int)N, Sp, (rocblas_int)N, info);
  } else {
    lam2 = part + 4 * Nc * Nc;
    hipLaunchKernelGGL(k_form_herm, gq, dim3(256), 0, s, (int)Nc, Hp, Hc);
    hipLaunchKernelGGL(k_form_herm, gq, dim3(256), 0, s, (int)Nc, Sp, Sc);
    PAWFE_HIP(hipGetLastError());
    rs = rocsolver_zpotrf(h, rocblas_fill_upper, (rocblas_int)Nc, (rocblas_double_complex*)Sc, (rocblas_int)Nc, info);
  }
  if (rs != rocblas_status_success) return fail(PAWFE_EHIP, "rocsolver Cholesky factorization failed");
  rocblas_int hinfo = 0;
  CHECK(read_info(&hinfo));
  if (hinfo > 0) return fail(PAWFE_ENOTSPD, "projected overlap S^p is not positive definite");
  const rocblas_int n = (rocblas_int)Nc;
  rocblas_status r1, r2, r3;
  if (!op->cplx) {
    r1 = rocblas_dtrsm(h, rocblas_side_left, rocblas_fill_upper, rocblas_operation_transpose,
                       rocblas_diagonal_non_unit, n, n, &one, Sp, n, Hp, n);
    r2 = rocblas_dtrsm(h, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none, rocblas_diagonal_non_unit,
                       n, n, &one, Sp, n, Hp, n);
    r3 = rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, Hp, n, lambda, Ework, info);
  } else {
    rocblas_double_complex* H = (rocblas_double_complex*)Hc;
    const rocblas_double_complex* U = (const rocblas_double_complex*)Sc;
    r1 = rocblas_ztrsm(h, rocblas_side_left, rocblas_fill_upper, rocblas_operation_conjugate_transpose,
                       rocblas_diagonal_non_unit, n, n, &onez, U, n, H, n);
    r2 = rocblas_ztrsm(h, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none, rocblas_diagonal_non_unit,
                       n, n, &onez, U, n, H, n);
    r3 = rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, n, H, n, lambda, Ework, info);
  }
  if (r1 != rocblas_status_success || r2 != rocblas_status_success)
    return fail(PAWFE_EHIP, "rocblas triangular solve (reduction) failed");
  if (r3 != rocblas_status_success) return fail(PAWFE_EHIP, "rocsolver eigensolver failed");
  CHECK(read_info(&hinfo));
  if (hinfo > 0) return fail(PAWFE_ENONFINITE, "projected eigensolver did not converge");
  if (!op->cplx) {
    r1 = rocblas_dtrsm(h, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none, rocblas_diagonal_non_unit,
                       n, n, &one, Sp, n, Hp, n);
  } else {
    r1 = rocblas_ztrsm(h, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none, rocblas_diagonal_non_unit,
                       n, n, &onez, (const rocblas_double_complex*)Sc, n, (rocblas_double_complex*)Hc, n);
  }
  if (r1 != rocblas_status_success) return fail(PAWFE_EHIP, "rocblas triangular solve (back-transform) failed");
  if (op->cplx) {
    hipLaunchKernelGGL(k_realify_rot, gq, dim3(256), 0, s, (int)Nc, Hc, Hp);
    PAWFE_HIP(hipGetLastError());
    CHECK(launch_dup_pairs(lambda, lam2, (int)Nc, s));
  }
  // rotation X <- X Q (Q column-major in Hp; real form for complex operators)
  if (sr_prec == PAWFE_FP32) {
    // mixed precision (the paper's RR-SR strategy): X diag(Q) in FP64 plus
    // fl32(X) fl32(Q_off) on the FP32 matrix cores; X32 and Y32 share the
    // rotated-copy buffer, Q32 the overlap buffer (free after the solve)
    const int bs = op->cplx ? 2 : 1;
    float* X32 = reinterpret_cast<float*>(Xr);
    float* Y32 = X32 + (size_t)K * N;
    float* Q32 = reinterpret_cast<float*>(Sp);
    // the compact diagonal blocks (N bs doubles) in the split-K buffer, past
    // the complex path's lam2 and squared norms (N^2 + 2 N doubles in)
    double* Qd = part + N * N + 2 * N;
    const int64_t nprep = K * N + N * N;
    hipLaunchKernelGGL(k_sr_prep, dim3((unsigned)((nprep + 255) / 256)), dim3(256), 0, s, K, (int)N, bs, X, ldx,
                       X32, Hp, Q32, Qd);
    const float onef = 1.0f, zerof = 0.0f;
    if (rocblas_sgemm(h, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)N, (rocblas_int)K,
                      (rocblas_int)N, &onef, Q32, (rocblas_int)N, X32, (rocblas_int)N, &zerof, Y32,
                      (rocblas_int)N) != rocblas_status_success)
      return fail(PAWFE_EHIP, "rocblas_sgemm (rotation) failed");
    const int64_t ncomb = K * (N / bs);
    hipLaunchKernelGGL(k_sr_combine, dim3((unsigned)((ncomb + 255) / 256)), dim3(256), 0, s, K, (int)N, bs, X, ldx,
                       Y32, Qd);
    PAWFE_HIP(hipGetLastError());
  } else {
    // Xr = X Q: column-major, Xr^T (N x K) = Q^T (N x N) X^T (N x K)
    const double one = 1.0, zero = 0.0;
    if (rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)N, (rocblas_int)K,
                      (rocblas_int)N, &one, Hp, (rocblas_int)N, X, (rocblas_int)ldx, &zero, Xr,
                      (rocblas_int)N) != rocblas_status_success)
      return fail(PAWFE_EHIP, "rocblas_dgemm (rotation) failed");
    CHECK(launch_copy_cols(Xr, N, X, ldx, op->M, (int)N, s));
  }
  // residual norms ||H x - lambda S x||_2 (complex: over both parts)
  double* sq = op->cplx ? lam2 + N : nullptr;
  for (int64_t j0 = 0; j0 < N; j0 += B) {
    const int nc = (int)std::min<int64_t>(B, N - j0);
    double* Rb = R ? R + j0 : HXb;
    const int64_t ldb = R ? ldr : nc;
    CHECK(do_residual(op, X + j0, ldx, (op->cplx ? lam2 : lambda) + j0, Rb, ldb, nc, nb, s));
    CHECK(launch_coldot(Rb, ldb, Rb, ldb, op->M, nc, npart_buf, (op->cplx ? sq : resnorm) + j0, nullptr,
                        !op->cplx, false, s));
  }
  if (op->cplx) {
    hipLaunchKernelGGL(k_pair_norm, dim3((unsigned)((Nc + 255) / 256)), dim3(256), 0, s, (int)Nc, sq, resnorm);
    PAWFE_HIP(hipGetLastError());
  }
  return PAWFE_OK;
}

pawfe_status pawfe_rayleigh_ritz(const pawfe_op* op, void* X, int64_t ldx, int64_t nvec, double* lambda,
                                 double* resnorm, int32_t sr_prec, void* ws, size_t ws_bytes, void* stream) {
  return rayleigh_ritz_impl(op, X, ldx, nvec, lambda, resnorm, nullptr, 0, sr_prec, ws, ws_bytes, stream);
}

pawfe_status pawfe_rayleigh_ritz_res(const pawfe_op* op, void* X, int64_t ldx, int64_t nvec, double* lambda,
                                     double* resnorm, void* R, int64_t ldr, int32_t sr_prec, void* ws,
                                     size_t ws_bytes, void* stream) {
  if (!R) return fail(PAWFE_EINVAL, "R is NULL");
  if (ldr < nvec) return fail(PAWFE_EINVAL, "leading dimension of R smaller than nvec");
  if (R == X) return fail(PAWFE_EINVAL, "R must not be X");
  return rayleigh_ritz_impl(op, X, ldx, nvec, lambda, resnorm, (double*)R, ldr, sr_prec, ws, ws_bytes, stream);
}

// ---- band energy gradient ----------------------------------------------------

pawfe_status pawfe_band_energy_grad(const pawfe_op* cop, const void* Xv, int64_t ldx, int64_t N, const double* occ,
                                    double* E, double* dE_dVq, double* dE_dDH, void* stream) {
  if (!cop) return fail(PAWFE_EINVAL, "op is NULL");
  if (!Xv || N < 1 || ldx < N) return fail(PAWFE_EINVAL, "bad X / nvec / ldx");
  pawfe_op* op = const_cast<pawfe_op*>(cop);
  hipStream_t s = S(stream);
  const double* X = (const double*)Xv;
  // complex operators: the (re, im) real view; x^H H x, |u|^2 and
  // Re(conj(P_a) P_b) are then the real formulas summed over both columns of
  // a pair, each with the pair's occupation
  const int64_t Nc = N;
  if (op->cplx) {
    N *= 2;
    ldx *= 2;
  }
  const int64_t B = std::min<int64_t>(256, N);
  const int64_t nchunks = (op->M + 4095) / 4096;
  size_t need = nl_scratch_bytes(op, std::max<int64_t>(N, B)) + align256((size_t)op->M * B * 8) +
                align256((size_t)nchunks * B * 8) + align256((size_t)N * 8) + 1024;
  CHECK(ensure_scratch(op, need));
  Carve cv(op->scratch, op->scratch_bytes);
  NlBufs nb = carve_nl(op, cv, std::max<int64_t>(N, B));
  double* HXb = cv.take<double>((size_t)op->M * B);
  double* pbuf = cv.take<double>((size_t)nchunks * B);
  double* occ2 = cv.take<double>((size_t)N);
  if (!cv.ok()) return fail(PAWFE_EINVAL, "internal: gradient scratch smaller than its carve");
  if (op->cplx && occ) {
    CHECK(launch_dup_pairs(occ, occ2, (int)Nc, s));
    occ = occ2;
  }
  if (E) {
    CHECK(launch_fill<double>(E, 1, 0.0, s));
    for (int64_t j0 = 0; j0 < N; j0 += B) {
      const int nc = (int)std::min<int64_t>(B, N - j0);
      CHECK(do_apply<double>(op, 0, X + j0, ldx, HXb, nc, nc, nb, s));
      CHECK(launch_coldot(X + j0, ldx, HXb, nc, op->M, nc, pbuf, E, occ ? occ + j0 : nullptr, false, true, s));
    }
  }
  if (dE_dVq) CHECK(launch_density(op, X, ldx, (int)N, occ, dE_dVq, s));
  if (dE_dDH && op->natoms) {
    CHECK(launch_nl_reduce<double>(op, X, ldx, (int)N, false, nb.part, nb.c, s));
    CHECK(launch_grad_dh(op, nb.c, (int)N, occ, dE_dDH, s));
  }
  return PAWFE_OK;
}

// ---- Lanczos bounds ------------------------------------------------------------

pawfe_status pawfe_lanczos_bounds(const pawfe_op* cop, int32_t k, uint64_t seed, double* theta_min,
                                  double* theta_max, double* beta_k, void* stream) {
  if (!cop) return fail(PAWFE_EINVAL, "op is NULL");
  if (k < 2 || k > 200) return fail(PAWFE_EINVAL, "k must be in 2..200");
  pawfe_op* op = const_cast<pawfe_op*>(cop);
  hipStream_t s = S(stream);
  // complex operators: vectors of M complex entries as (re, im) pairs; the
  // real inner product of that view is Re x^H y, the Hermitian form
  const int cf = op->cplx ? 2 : 1;
  const int64_t M = op->M * cf;
  const int64_t nchunks = (M + 4095) / 4096;
  size_t need = nl_scratch_bytes(op, cf) + 5 * align256((size_t)M * 8) + align256((size_t)nchunks * 8) + 1024;
  CHECK(ensure_scratch(op, need));
  Carve cv(op->scratch, op->scratch_bytes);
  NlBufs nb = carve_nl(op, cv, cf);
  double* v = cv.take<double>(M);
  double* vp = cv.take<double>(M);
  double* z = cv.take<double>(M);
  double* w = cv.take<double>(M);
  double* u = cv.take<double>(M);
  double* pbuf = cv.take<double>(nchunks);
  double* dot = cv.take<double>(2);
  if (!cv.ok()) return fail(PAWFE_EINVAL, "internal: Lanczos scratch smaller than its carve");
  // seeded start vector (splitmix64 -> uniform(-1, 1)), generated on the host
  std::vector<double> h(M);
  uint64_t st = seed;
  for (int64_t i = 0; i < M; ++i) {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t x = st;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    h[i] = 2.0 * ((x >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  }
  PAWFE_HIP(hipMemcpyAsync(v, h.data(), M * 8, hipMemcpyHostToDevice, s));
  const dim3 g((unsigned)((M + 255) / 256)), b(256);
  auto ddot = [&](const double* x, const double* y, double* res) -> pawfe_status {
    CHECK(launch_fill<double>(dot, 1, 0.0, s));
    CHECK(launch_coldot(x, 1, y, 1, M, 1, pbuf, dot, nullptr, false, true, s));
    PAWFE_HIP(hipMemcpyAsync(res, dot, 8, hipMemcpyDeviceToHost, s));
    PAWFE_HIP(hipStreamSynchronize(s));
    return PAWFE_OK;
  };
  CHECK(do_apply<double>(op, 2, v, cf, z, cf, cf, nb, s));
  double nrm2 = 0.0;
  CHECK(ddot(v, z, &nrm2));
  if (!(nrm2 > 0.0)) return fail(PAWFE_ENOTSPD, "Sinv_hat is not positive on the start vector");
  const double inv = 1.0 / std::sqrt(nrm2);
  hipLaunchKernelGGL(k_lincomb, g, b, 0, s, M, v, inv, v, 0.0, nullptr, 0.0);
  hipLaunchKernelGGL(k_lincomb, g, b, 0, s, M, z, inv, z, 0.0, nullptr, 0.0);
  CHECK(launch_fill<double>(vp, M, 0.0, s));
  std::vector<double> al, be;
  double beta_prev = 0.0;
  for (int it = 0; it < k; ++it) {
    CHECK(do_apply<double>(op, 0, z, cf, w, cf, cf, nb, s));
    double alpha = 0.0;
    CHECK(ddot(z, w, &alpha));
    // w = w - alpha v - beta_prev vp
    hipLaunchKernelGGL(k_lincomb, g, b, 0, s, M, w, -alpha, v, -beta_prev, vp, 1.0);
    CHECK(do_apply<double>(op, 2, w, cf, u, cf, cf, nb, s));
    double bb = 0.0;
    CHECK(ddot(w, u, &bb));
    const double beta = std::sqrt(std::max(bb, 0.0));
    al.push_back(alpha);
    be.push_back(beta);
    if (beta == 0.0) break;
    std::swap(vp, v);   // vp <- v
    hipLaunchKernelGGL(k_lincomb, g, b, 0, s, M, v, 1.0 / beta, w, 0.0, nullptr, 0.0);
    hipLaunchKernelGGL(k_lincomb, g, b, 0, s, M, z, 1.0 / beta, u, 0.0, nullptr, 0.0);
    beta_prev = beta;
  }
  const int n = (int)al.size();
  std::vector<double> T(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    T[i * n + i] = al[i];
    if (i + 1 < n) T[i * n + i + 1] = T[(i + 1) * n + i] = be[i];
  }
  std::vector<double> ev = small_sym_eigvals(n, T);
  if (theta_min) *theta_min = ev.front();
  if (theta_max) *theta_max = ev.back();
  if (beta_k) *beta_k = std::fabs(be.back());
  PAWFE_HIP(hipGetLastError());
  return PAWFE_OK;
}

// ---- ChFSI outer loop ----------------------------------------------------------

pawfe_status pawfe_chfsi_solve_workspace(const pawfe_op* op, int64_t nvec, int32_t block, int32_t prec,
                                         size_t* bytes) {
  if (!op || !bytes) return fail(PAWFE_EINVAL, "op or bytes is NULL");
  size_t f = 0, r = 0;
  CHECK(pawfe_cheb_filter_workspace(op, nvec, block, prec, &f));
  CHECK(pawfe_rayleigh_ritz_workspace(op, nvec, &r));
  // the filter and Rayleigh-Ritz never overlap; after their shared part, the
  // residual Rayleigh-Ritz hands to the next filter pass
  *bytes = align256(std::max(f, r)) + align256((size_t)op->M * nvec * (op->cplx ? 2 : 1) * 8);
  return PAWFE_OK;
}

pawfe_status pawfe_chfsi_solve(const pawfe_op* op, void* X, int64_t ldx, int64_t nvec, int64_t nwanted,
                               int32_t degree, int32_t block, int32_t prec, double bU, int32_t lanczos_k,
                               double tol, int32_t max_iter, double* lambda, double* resnorm, int32_t* iterations,
                               void* ws, size_t ws_bytes, void* stream) {
  if (!op) return fail(PAWFE_EINVAL, "op is NULL");
  if (!X || !lambda || !resnorm || !ws) return fail(PAWFE_EINVAL, "NULL buffer");
  if (nvec < 2 || ldx < nvec) return fail(PAWFE_EINVAL, "need nvec >= 2 and ldx >= nvec");
  if (nwanted < 0 || nwanted > nvec) return fail(PAWFE_EINVAL, "nwanted must be in 0..nvec");
  if (degree < 2 || block < 1 || max_iter < 0) return fail(PAWFE_EINVAL, "degree >= 2, block >= 1, max_iter >= 0");
  if (!(std::isfinite(tol) && tol > 0.0) || !std::isfinite(bU)) return fail(PAWFE_EINVAL, "tol must be > 0, bU finite");
  CHECK(check_prec(prec, op));
  size_t need = 0;
  CHECK(pawfe_chfsi_solve_workspace(op, nvec, block, prec, &need));
  if (ws_bytes < need) return fail(PAWFE_EINVAL, "workspace too small");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(PAWFE_EINVAL, "workspace must be 256-byte aligned");
  // shared part of the filter and Rayleigh-Ritz, then the residual R of the
  // Ritz pairs (written by each Rayleigh-Ritz, step 2 of the next filter)
  const size_t shared = need - align256((size_t)op->M * nvec * (op->cplx ? 2 : 1) * 8);
  void* R = (char*)ws + shared;
  const int64_t nw = nwanted > 0 ? nwanted : nvec;
  // step 1 of Algorithm 1: the upper bound of the spectrum (given, or Lanczos)
  if (!(bU > 0.0)) {
    double tmin = 0.0, tmax = 0.0, beta = 0.0;
    CHECK(pawfe_lanczos_bounds(op, lanczos_k, 1234, &tmin, &tmax, &beta, stream));
    bU = tmax + beta;
  }
  std::vector<double> lh(nvec), rh(nvec);
  auto fetch = [&]() -> pawfe_status {
    hipStream_t s = S(stream);
    PAWFE_HIP(hipMemcpyAsync(lh.data(), lambda, nvec * 8, hipMemcpyDeviceToHost, s));
    PAWFE_HIP(hipMemcpyAsync(rh.data(), resnorm, nvec * 8, hipMemcpyDeviceToHost, s));
    PAWFE_HIP(hipStreamSynchronize(s));
    return PAWFE_OK;
  };
  auto worst = [&]() { return *std::max_element(rh.begin(), rh.begin() + nw); };
  CHECK(pawfe_rayleigh_ritz_res(op, X, ldx, nvec, lambda, resnorm, R, nvec, PAWFE_FP64, ws, shared, stream));
  CHECK(fetch());
  int32_t it = 0;
  while (worst() > tol && it < max_iter) {
    // b_0, b_W: lowest and highest current Ritz values (lambda stays the
    // filter's eigenvalue estimate; the filter runs in place, from the
    // residual the last Rayleigh-Ritz left)
    CHECK(pawfe_cheb_filter_res(op, X, ldx, R, nvec, X, ldx, nvec, block, lambda, degree, lh.front(), lh.back(), bU,
                                prec, ws, shared, stream));
    CHECK(pawfe_rayleigh_ritz_res(op, X, ldx, nvec, lambda, resnorm, R, nvec, PAWFE_FP64, ws, shared, stream));
    CHECK(fetch());
    ++it;
  }
  if (iterations) *iterations = it;
  return PAWFE_OK;
}

}  // extern "C"
