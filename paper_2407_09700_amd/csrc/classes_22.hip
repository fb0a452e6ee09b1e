// Kernels of the bra class (la, lb) = (2, 2) and every ket class up to it.
#include "jk_classes_impl.h"
namespace jk {
void register_bra_22(ClassInfo *classes, BraInfo *bras) { register_bra<2, 2>(classes, bras); }
}  // namespace jk
