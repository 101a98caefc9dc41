// K + V (and the residual K + V - lambda M) on the vector ALUs for operators
// whose cells share one geometry
// (the kernel and its tables are in cell_valu.h).

#include "cell_valu.h"

namespace pawfe {

// K + V (mode kModeH), K + V - lambda_n M (mode kModeHRes) or det J M (mode
// kModeMass) on the vector ALUs, for complex operators with the imaginary k
// term on the (re, im) column pairs in the same launch; *done is false when the mode, degree or
// Gauss rule has no compiled variant (the caller then uses the matrix-core
// kernel)
template <typename T>
pawfe_status launch_cell_valu(const pawfe_op* op, int mode, const CellArgs<T>& a, hipStream_t s, bool* done) {
  *done = false;
  if (a.ldx < 0 || a.ldy < 0 || a.ldx * (int64_t)sizeof(T) >= (int64_t(1) << 32) ||
      a.ldy * (int64_t)sizeof(T) >= (int64_t(1) << 32))
    return fail(PAWFE_EINVAL, "row stride of 4 GiB or more");
  if (op->nq != op->p + 2 || (mode != kModeH && mode != kModeHRes && mode != kModeMass)) return PAWFE_OK;
  if (mode == kModeHRes && !a.lam) return fail(PAWFE_EINVAL, "residual mode needs lambda");
  *done = true;
  if (mode == kModeMass) {   // real, also for complex operators (both halves alike)
    switch (op->p) {
      case 2: return run_cell_valu<T, 3, 4, kValuMass>(op, a, s);
      case 3: return run_cell_valu<T, 4, 5, kValuMass>(op, a, s);
      case 4: return run_cell_valu<T, 5, 6, kValuMass>(op, a, s);
      case 5: return run_cell_valu<T, 6, 7, kValuMass>(op, a, s);
      case 6: return run_cell_valu<T, 7, 8, kValuMass>(op, a, s);
      default: *done = false; return PAWFE_OK;
    }
  }
  const bool res = mode == kModeHRes;
  if (op->cplx) {   // the imaginary k term joins the same passes
    switch (op->p) {
      case 2: return res ? run_cell_valu<T, 3, 4, kValuHResC>(op, a, s) : run_cell_valu<T, 3, 4, kValuHC>(op, a, s);
      case 3: return res ? run_cell_valu<T, 4, 5, kValuHResC>(op, a, s) : run_cell_valu<T, 4, 5, kValuHC>(op, a, s);
      case 4: return res ? run_cell_valu<T, 5, 6, kValuHResC>(op, a, s) : run_cell_valu<T, 5, 6, kValuHC>(op, a, s);
      case 5: return res ? run_cell_valu<T, 6, 7, kValuHResC>(op, a, s) : run_cell_valu<T, 6, 7, kValuHC>(op, a, s);
      case 6: return res ? run_cell_valu<T, 7, 8, kValuHResC>(op, a, s) : run_cell_valu<T, 7, 8, kValuHC>(op, a, s);
      default: *done = false; return PAWFE_OK;
    }
  }
  switch (op->p) {
    case 2: return res ? run_cell_valu<T, 3, 4, kValuHRes>(op, a, s) : run_cell_valu<T, 3, 4, kValuH>(op, a, s);
    case 3: return res ? run_cell_valu<T, 4, 5, kValuHRes>(op, a, s) : run_cell_valu<T, 4, 5, kValuH>(op, a, s);
    case 4: return res ? run_cell_valu<T, 5, 6, kValuHRes>(op, a, s) : run_cell_valu<T, 5, 6, kValuH>(op, a, s);
    case 5: return res ? run_cell_valu<T, 6, 7, kValuHRes>(op, a, s) : run_cell_valu<T, 6, 7, kValuH>(op, a, s);
    case 6: return res ? run_cell_valu<T, 7, 8, kValuHRes>(op, a, s) : run_cell_valu<T, 7, 8, kValuH>(op, a, s);
    default: *done = false; return PAWFE_OK;
  }
}

template pawfe_status launch_cell_valu<float>(const pawfe_op*, int, const CellArgs<float>&, hipStream_t, bool*);
template pawfe_status launch_cell_valu<double>(const pawfe_op*, int, const CellArgs<double>&, hipStream_t, bool*);

}  // namespace pawfe
