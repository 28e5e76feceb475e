// Kernel instantiations and launch table for the 512 x 512 grid.
#include "nlinv_kernels.h"

namespace nlv {
const GTable* table_g512() {
  static const GTable t = make_table<512>();
  return &t;
}
}  // namespace nlv
