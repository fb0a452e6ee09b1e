// Kernels of the bra class (la, lb) = (4, 1) and every ket class up to it.
#include "jk_classes_impl.h"
namespace jk {
void register_bra_41(ClassInfo *classes, BraInfo *bras) { register_bra<4, 1>(classes, bras); }
}  // namespace jk
