// The Chebyshev step of the filter on general operators (graded meshes,
// the GGA term): the vector-ALU kernel of cell_valu.h in its general step
// variants (per-cell geometry, face factors of the lumped mass).

#include "cell_valu.h"

namespace pawfe {

template <typename T>
pawfe_status launch_cell_step_gen(const pawfe_op* op, const CellArgs<T>& c, hipStream_t s) {
  if (op->gga) {
    switch (op->p) {
      case 2: return run_cell_valu<T, 3, 4, kValuGenStepG>(op, c, s);
      case 3: return run_cell_valu<T, 4, 5, kValuGenStepG>(op, c, s);
      case 4: return run_cell_valu<T, 5, 6, kValuGenStepG>(op, c, s);
      case 5: return run_cell_valu<T, 6, 7, kValuGenStepG>(op, c, s);
      default: return run_cell_valu<T, 7, 8, kValuGenStepG>(op, c, s);
    }
  }
  switch (op->p) {
    case 2: return run_cell_valu<T, 3, 4, kValuGenStep>(op, c, s);
    case 3: return run_cell_valu<T, 4, 5, kValuGenStep>(op, c, s);
    case 4: return run_cell_valu<T, 5, 6, kValuGenStep>(op, c, s);
    case 5: return run_cell_valu<T, 6, 7, kValuGenStep>(op, c, s);
    default: return run_cell_valu<T, 7, 8, kValuGenStep>(op, c, s);
  }
}

template pawfe_status launch_cell_step_gen<float>(const pawfe_op*, const CellArgs<float>&, hipStream_t);
template pawfe_status launch_cell_step_gen<double>(const pawfe_op*, const CellArgs<double>&, hipStream_t);

}  // namespace pawfe
