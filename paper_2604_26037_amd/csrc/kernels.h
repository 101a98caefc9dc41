// Kernel launch interface shared by the translation units of libpawfe.
#pragma once

#include <type_traits>

#include "internal.h"

namespace pawfe {

enum { kModeH = 0, kModeHRes = 1, kModeMass = 2, kModeImg = 3 };

template <typename T>
struct CellArgs {
  const T* X;
  int64_t ldx;
  T* Y;
  int64_t ldy;
  int ncols;
  const int32_t* cells;   // the colour's cells as i | j << 10 | k << 20
  const T* Vw;
  const T* W3;
  const double* lam;   // per-column lambda (residual mode)
  T alpha;
  int n0, n1, n2;
  int bf3;             // FP32 data, contractions as bf16x3 split products
  // general operators (vector-ALU kernel variants)
  const T* geo;        // [E][4] per cell: fx, fy, fz (1/2 det J (2/h_d)^2) and det J
  const T* vg;         // [E][3][nq^3] W_q det J (2/h_d) V_GGA,d (GGA term), or null
  T detJ;              // det J of every cell (residual mode of the vector-ALU kernel)
  T gk[3];             // complex operators: -k_d det J (2/h_d) (imaginary k term)
  // Chebyshev step of the filter (vector-ALU step variants)
  const uint32_t* own;   // [E] first-visit bits per local position class
  const double* y64;     // residual block Y (FP64), row stride ldy64
  int64_t ldy64;
  const double* lamY;    // per-column Lambda_Y
  double sa, sac, szz;   // a, a c, zeta zeta'
  const T* frho;         // general step: [E][6] face factors (x lo, x hi, y lo, y hi, z lo, z hi)
};

struct DensArgs {
  const double* X;
  int64_t ldx;
  int ncols;
  const double* occ;
  double* out;
  const double* W3;
  const double* cscale;   // [E] det J_e / det J of graded meshes, or null
  int n0, n1, n2;
};

// Y += alpha * A_loc X over all cells (colour by colour).
//  mode kModeH:    A_loc = K + V
//  mode kModeHRes: A_loc = K + V - lambda_n M (per column n)
//  mode kModeMass: A_loc = M
//  mode kModeImg:  complex operators, the imaginary local term applied to
//                  the partner columns: Y[n] += alpha s_n (Hi X)[n ^ 1],
//                  Hi = sum_d g_d (G1 along d, M1 along the others),
//                  s_n = -1 on real and +1 on imaginary columns
//  bf3: (FP32 only) the cell contractions as bf16x3 split products on the
//  bf16 matrix cores, FP32 accumulation.
template <typename T>
pawfe_status launch_cell(const pawfe_op* op, int mode, const T* X, int64_t ldx, T* Y, int64_t ldy,
                         int ncols, const double* lam, double alpha, hipStream_t s, bool bf3 = false);

// bf16x3 split products on the matrix cores (kernels_cell_mfma.hip): K + V
// (kModeH), the mass term (kModeMass) and the imaginary k term (kModeImg) of
// FP32 data; any other request returns PAWFE_EUNSUPPORTED.
template <typename T>
pawfe_status launch_cell_mfma(const pawfe_op* op, int mode, const CellArgs<T>& a, hipStream_t s);

// K + V (kModeH) or K + V - lambda_n M (kModeHRes) on the vector ALUs
// (kernels_cell_valu.hip); *done is false when no variant is compiled for
// the mode, the operator's degree and Gauss rule.
template <typename T>
pawfe_status launch_cell_valu(const pawfe_op* op, int mode, const CellArgs<T>& a, hipStream_t s, bool* done);

// Every local term of a general operator (graded mesh and / or the GGA term)
// on the vector ALUs (kernels_cell_gen_f32.hip / _f64.hip): kModeH, kModeMass
// and kModeHRes (K + V [+ GGA] - lambda_n M).
template <typename T>
pawfe_status launch_cell_gen(const pawfe_op* op, int mode, const CellArgs<T>& a, hipStream_t s);

// Chebyshev step of the filter, local part, on the vector ALUs
// (kernels_cell_step.hip): R_X <- -a c R_Y' - zz R_X + a Y lamY + a H_loc
// M_D^{-1} R_Y' with the node part applied at the first visit of each DOF;
// R_Y' = R_Y - C d is formed by the caller, the projector terms of R_X are
// added after it.  cell_step_available: the operator has a step variant
// (nq = p + 2, degree 2-6; graded meshes and the GGA term on real operators).
bool cell_step_available(const pawfe_op* op);
template <typename T>
pawfe_status launch_cell_step(const pawfe_op* op, const T* RY, T* RX, int64_t ld, const double* Y, int64_t ldy,
                              const double* lamY, double a, double ac, double zz, int ncols, hipStream_t s);

// the same on general operators (kernels_cell_step_gen.hip; the arguments
// already carry the per-cell tables)
template <typename T>
pawfe_status launch_cell_step_gen(const pawfe_op* op, const CellArgs<T>& c, hipStream_t s);

// out[e][q] = W_q sum_n occ_n |u_n(x_{e,q})|^2
pawfe_status launch_density(const pawfe_op* op, const double* X, int64_t ldx, int ncols,
                            const double* occ, double* out, hipStream_t s);

// out[2 j] = out[2 j + 1] = in[j], j < n (a value per complex column -> one
// per real column of the (re, im) pairs)
pawfe_status launch_dup_pairs(const double* in, double* out, int n, hipStream_t s);

// ---- non-local / node-wise kernels (kernels_nl.hip) ----

// c[(poff_a + alpha) * ncols + n] = sum_{I in supp(a)} C^a[I][alpha] s_I X[I][n],
// s_I = M_D^{-1}[I] if scale_minv, else 1.  part: >= item_rows_total*ncols doubles.
// Real operators in FP32 run on the matrix cores (FP32, or bf16x3 split
// products when bf3); FP64 and complex operators on the vector ALUs.
template <typename T>
pawfe_status launch_nl_reduce(const pawfe_op* op, const T* X, int64_t ldx, int ncols, bool scale_minv,
                              double* part, double* c, hipStream_t s, bool bf3 = false);

// out = (D1 - lam_n D2) in  (per atom block; D2 may be NULL), scaled by f.
// D1i: imaginary part of D1 (complex operators, Delta_Sinv with the exact G);
// the columns are then (re, im) pairs of complex columns.
pawfe_status launch_atom_mul(const pawfe_op* op, const double* D1, const double* D2, const double* lam,
                             double f, const double* in, double* out, int ncols, hipStream_t s,
                             const double* D1i = nullptr);

// out_a = c_a - sum_b G^{ab} d_b
pawfe_status launch_atom_gcorr(const pawfe_op* op, const double* c, const double* d, double* out,
                               int ncols, hipStream_t s);

// Projector part of the fused Chebyshev step: v = nw_prev + d,
// nw = -q + ac d + zz d_prev, lamX = a lamY lam_in - ac lamY - zz lamX
// (nw_prev, d_prev null: zero; q null: v only)
pawfe_status launch_step_combine(const pawfe_op* op, const double* q, const double* d, const double* dprev,
                                 const double* nwprev, double* v, double* nw, double* lamX, const double* lamY,
                                 const double* lam_in, double a, double ac, double zz, int ncols, hipStream_t s);

// out1 += s1 C v1 on the support rows (atom colour by colour)
template <typename T>
pawfe_status launch_node_fixup(const pawfe_op* op, const double* v1, double s1, int ncols, T* out1, int64_t ld1,
                               hipStream_t s);

// Y[I][n] = sum_{a: I in supp(a)} C^a[I] . q_a[n]   (0 outside the supports)
template <typename T>
pawfe_status launch_node_nl_init(const pawfe_op* op, const double* q, int ncols, T* Y, int64_t ldy,
                                 hipStream_t s);

// Y = M_D^{-1} (X - sum_a C^a d_a)
template <typename T>
pawfe_status launch_node_sinv(const pawfe_op* op, const T* X, int64_t ldx, const double* d, int ncols,
                              T* Y, int64_t ldy, hipStream_t s);

// Chebyshev step, node part:  T = M_D^{-1}(RY - C d);
// RX = -ac RY - zz RX + C q + a Y lamY (q already scaled by a);
// lamX = a lamY lam_in - ac lamY - zz lamX (row 0 threads).
template <typename TR>
pawfe_status launch_node_cheb(const pawfe_op* op, const TR* RY, TR* RX, TR* Tb, int64_t ld,
                              const double* Y, int64_t ldy, const double* d, const double* q,
                              const double* lamY, double* lamX, const double* lam_in, double a,
                              double ac, double zz, int ncols, hipStream_t s);

// Xout = M_D^{-1}(RY - C d) + X lamY
template <typename TR>
pawfe_status launch_node_finalize(const pawfe_op* op, const TR* RY, int64_t ld, const double* d,
                                  const double* X, int64_t ldx, const double* lamY, double* Xout,
                                  int64_t ldo, int ncols, hipStream_t s);

// RY = f * Y (cast), RX = 0, lamY = f (lam_in - c), lamX = 1
template <typename TR>
pawfe_status launch_cheb_init(const pawfe_op* op, const double* Y, int64_t ldy, TR* RY, TR* RX,
                              int64_t ld, double f, double c, const double* lam_in, double* lamY,
                              double* lamX, int ncols, hipStream_t s);

// partial[chunk][n] = sum over rows of the chunk of  A[i][n] * B[i][n]  (B == A -> squares)
pawfe_status launch_coldot(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t nrows,
                           int ncols, double* partial, double* out, const double* w, bool sqrt_out,
                           bool accumulate_scalar, hipStream_t s);

// dE/dDelta_H^a = sum_n occ_n P P^T, P = c rows of atom a
pawfe_status launch_grad_dh(const pawfe_op* op, const double* c, int ncols, const double* occ,
                            double* out, hipStream_t s);

// BF16 halo of a z-slab [kz0, kz1) of cell layers: pack (Y -> buf) or
// unpack-add (Y += buf) on its two shared node planes (kernels_halo.hip)
pawfe_status launch_halo(const pawfe_op* op, bool pack, float* Y, int64_t ldy, int ncols, int kz0, int kz1,
                         uint16_t* buf, hipStream_t s);

// elementwise copies / fills
pawfe_status launch_copy_cols(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t nrows,
                              int ncols, hipStream_t s);
template <typename T>
pawfe_status launch_fill(T* Y, int64_t n, T v, hipStream_t s);

}  // namespace pawfe
