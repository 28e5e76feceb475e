// Kernel instantiations and launch table for the 128 x 128 grid.
#include "nlinv_kernels.h"

namespace nlv {
const GTable* table_g128() {
  static const GTable t = make_table<128>();
  return &t;
}
}  // namespace nlv
