// Class kernels with bra angular momentum la = 3.
#include "jk_classes_impl.h"
namespace jk {
void register_classes_l3(ClassInfo *table) {
  register_bra<3, 0>(table);
  register_bra<3, 1>(table);
  register_bra<3, 2>(table);
  register_bra<3, 3>(table);
}
}  // namespace jk
