// Kernels of the bra class (la, lb) = (1, 1) and every ket class up to it.
#include "jk_classes_impl.h"
namespace jk {
void register_bra_11(ClassInfo *classes, BraInfo *bras) { register_bra<1, 1>(classes, bras); }
}  // namespace jk
