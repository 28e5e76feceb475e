// Kernel instantiations and launch table for the 480 x 480 grid.
#include "nlinv_kernels.h"

namespace nlv {
const GTable* table_g480() {
  static const GTable t = make_table<480>();
  return &t;
}
}  // namespace nlv
