// Kernel instantiations and launch table for the 320 x 320 grid.
#include "nlinv_kernels.h"

namespace nlv {
const GTable* table_g320() {
  static const GTable t = make_table<320>();
  return &t;
}
}  // namespace nlv
