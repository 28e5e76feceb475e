// Kernel instantiations and launch table for the 384 x 384 grid.
#include "nlinv_kernels.h"

namespace nlv {
const GTable* table_g384() {
  static const GTable t = make_table<384>();
  return &t;
}
}  // namespace nlv
