// Local terms of general operators (graded meshes, the GGA term) in FP64:
// the vector-ALU kernel variants of cell_valu.h with per-cell geometry.

#include "cell_valu.h"

namespace pawfe {

template <typename T>
pawfe_status launch_cell_gen(const pawfe_op* op, int mode, const CellArgs<T>& a, hipStream_t s) {
  return launch_cell_gen_impl<T>(op, mode, a, s);
}

template pawfe_status launch_cell_gen<double>(const pawfe_op*, int, const CellArgs<double>&, hipStream_t);

}  // namespace pawfe
