// Kernels of the bra class (la, lb) = (4, 4) and every ket class up to it.
#include "jk_classes_impl.h"
namespace jk {
void register_bra_44(ClassInfo *classes, BraInfo *bras) { register_bra<4, 4>(classes, bras); }
}  // namespace jk
