// Kernel instantiations and launch table for the 64 x 64 grid.
#include "nlinv_kernels.h"

namespace nlv {
const GTable* table_g64() {
  static const GTable t = make_table<64>();
  return &t;
}
}  // namespace nlv
