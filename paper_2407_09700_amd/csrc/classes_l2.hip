// Class kernels with bra angular momentum la = 2.
#include "jk_classes_impl.h"
namespace jk {
void register_classes_l2(ClassInfo *table) {
  register_bra<2, 0>(table);
  register_bra<2, 1>(table);
  register_bra<2, 2>(table);
}
}  // namespace jk
