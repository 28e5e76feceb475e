// Kernel instantiations and launch table for the 256 x 256 grid.
#include "nlinv_kernels.h"

namespace nlv {
const GTable* table_g256() {
  static const GTable t = make_table<256>();
  return &t;
}
}  // namespace nlv
