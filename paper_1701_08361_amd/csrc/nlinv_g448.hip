// Kernel instantiations and launch table for the 448 x 448 grid.
#include "nlinv_kernels.h"

namespace nlv {
const GTable* table_g448() {
  static const GTable t = make_table<448>();
  return &t;
}
}  // namespace nlv
