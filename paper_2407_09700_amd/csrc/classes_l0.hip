// Class kernels with bra angular momentum la = 0.
#include "jk_classes_impl.h"
namespace jk {
void register_classes_l0(ClassInfo *table) {
  register_bra<0, 0>(table);
}
}  // namespace jk
