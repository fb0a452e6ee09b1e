// Class kernels with bra angular momentum la = 4.
#include "jk_classes_impl.h"
namespace jk {
void register_classes_l4(ClassInfo *table) {
  register_bra<4, 0>(table);
  register_bra<4, 1>(table);
  register_bra<4, 2>(table);
  register_bra<4, 3>(table);
  register_bra<4, 4>(table);
}
}  // namespace jk
