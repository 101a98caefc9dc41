// The Chebyshev step of the filter: the vector-ALU kernel of cell_valu.h in
// its step variants (cells of one size here; graded meshes and the GGA term
// in kernels_cell_step_gen.hip).
//
// One step of Algorithm 2 (R_Y the current block, R_X the previous one,
// T = M_D^{-1} R_Y' with R_Y' = R_Y - sum_a C^a d_a already formed in R_Y):
//   R_X <- -a c R_Y' - zeta zeta' R_X + a Y Lambda_Y + a H_loc T
// The cell kernel gathers R_Y', contracts it with 1-D tables whose columns
// carry the lumped-mass factors (so T is never stored), and adds a H_loc T
// into R_X colour by colour; the first visit of each DOF (the cell of the
// lowest colour sharing it) first replaces the old R_X value by the node
// part -a c R_Y' - zeta zeta' R_X + a Y Lambda_Y.  The projector terms of
// the step are added to R_X afterwards by the caller.

#include "cell_valu.h"

namespace pawfe {

bool cell_step_available(const pawfe_op* op) {
  return op->nq == op->p + 2 && op->p >= 2 && op->p <= 6 && op->d.cell_own != nullptr &&
         (!op->general || (op->d.frho != nullptr && !op->cplx));
}

template <typename T>
pawfe_status launch_cell_step(const pawfe_op* op, const T* RY, T* RX, int64_t ld, const double* Y, int64_t ldy,
                              const double* lamY, double a, double ac, double zz, int ncols, hipStream_t s) {
  if (ncols <= 0) return PAWFE_OK;
  if (!cell_step_available(op)) return fail(PAWFE_EUNSUPPORTED, "internal: no step variant for this operator");
  if (ld < ncols || ldy < ncols || ld * (int64_t)sizeof(T) >= (int64_t(1) << 32))
    return fail(PAWFE_EINVAL, "internal: step leading dimensions");
  CellArgs<T> c{};
  c.X = RY;
  c.ldx = ld;
  c.Y = RX;
  c.ldy = ld;
  c.ncols = ncols;
  c.Vw = std::is_same<T, double>::value ? (const T*)op->d.Vw : (const T*)op->d.Vw_f;
  c.W3 = std::is_same<T, double>::value ? (const T*)op->d.W3 : (const T*)op->d.W3_f;
  c.alpha = (T)(a / op->detJ);   // the scaled tables carry det J M_D^{-1}
  c.n0 = op->n[0];
  c.n1 = op->n[1];
  c.n2 = op->n[2];
  c.own = op->d.cell_own;
  c.y64 = Y;
  c.ldy64 = ldy;
  c.lamY = lamY;
  c.sa = a;
  c.sac = ac;
  c.szz = zz;
  if (op->general) {   // graded mesh / GGA term: per-cell geometry, det J_e applied in the kernel
    c.alpha = (T)a;
    c.geo = std::is_same<T, double>::value ? (const T*)op->d.geo : (const T*)op->d.geo_f;
    c.vg = std::is_same<T, double>::value ? (const T*)op->d.vg : (const T*)op->d.vg_f;
    c.frho = std::is_same<T, double>::value ? (const T*)op->d.frho : (const T*)op->d.frho_f;
    return launch_cell_step_gen<T>(op, c, s);
  }
  if (op->cplx) {
    switch (op->p) {
      case 2: return run_cell_valu<T, 3, 4, kValuStepC>(op, c, s);
      case 3: return run_cell_valu<T, 4, 5, kValuStepC>(op, c, s);
      case 4: return run_cell_valu<T, 5, 6, kValuStepC>(op, c, s);
      case 5: return run_cell_valu<T, 6, 7, kValuStepC>(op, c, s);
      default: return run_cell_valu<T, 7, 8, kValuStepC>(op, c, s);
    }
  }
  switch (op->p) {
    case 2: return run_cell_valu<T, 3, 4, kValuStep>(op, c, s);
    case 3: return run_cell_valu<T, 4, 5, kValuStep>(op, c, s);
    case 4: return run_cell_valu<T, 5, 6, kValuStep>(op, c, s);
    case 5: return run_cell_valu<T, 6, 7, kValuStep>(op, c, s);
    default: return run_cell_valu<T, 7, 8, kValuStep>(op, c, s);
  }
}

template pawfe_status launch_cell_step<float>(const pawfe_op*, const float*, float*, int64_t, const double*, int64_t,
                                              const double*, double, double, double, int, hipStream_t);
template pawfe_status launch_cell_step<double>(const pawfe_op*, const double*, double*, int64_t, const double*,
                                               int64_t, const double*, double, double, double, int, hipStream_t);

}  // namespace pawfe
