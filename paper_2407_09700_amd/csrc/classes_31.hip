// Kernels of the bra class (la, lb) = (3, 1) and every ket class up to it.
#include "jk_classes_impl.h"
namespace jk {
void register_bra_31(ClassInfo *classes, BraInfo *bras) { register_bra<3, 1>(classes, bras); }
}  // namespace jk
