// Class kernels with bra angular momentum la = 1.
#include "jk_classes_impl.h"
namespace jk {
void register_classes_l1(ClassInfo *table) {
  register_bra<1, 0>(table);
  register_bra<1, 1>(table);
}
}  // namespace jk
