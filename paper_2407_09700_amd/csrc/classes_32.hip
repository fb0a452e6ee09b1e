// Kernels of the bra class (la, lb) = (3, 2) and every ket class up to it.
#include "jk_classes_impl.h"
namespace jk {
void register_bra_32(ClassInfo *classes, BraInfo *bras) { register_bra<3, 2>(classes, bras); }
}  // namespace jk
