// Kernels of the bra class (la, lb) = (2, 1) and every ket class up to it.
#include "jk_classes_impl.h"
namespace jk {
void register_bra_21(ClassInfo *classes, BraInfo *bras) { register_bra<2, 1>(classes, bras); }
}  // namespace jk
