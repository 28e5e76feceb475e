// Kernel instantiations and launch table for the 432 x 432 grid.
#include "nlinv_kernels.h"

namespace nlv {
const GTable* table_g432() {
  static const GTable t = make_table<432>();
  return &t;
}
}  // namespace nlv
