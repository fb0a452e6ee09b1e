// Gradient kernels of the quartet classes whose bra pair has an f shell (ket classes up to (ff)).
#include "jk_grad.h"

namespace jk {

template <int LA, int LB, int LC, int LD>
hipError_t launch_grad_f(const GradArgs &args, int grid, hipStream_t stream) {
  hipLaunchKernelGGL((k_grad<LA, LB, LC, LD>), dim3(grid), dim3(256), 0, stream, args);
  return hipGetLastError();
}

constexpr int gfc_la(int c) { int l = 0; while ((l + 1) * (l + 2) / 2 <= c) ++l; return l; }
constexpr int gfc_lb(int c) { return c - gfc_la(c) * (gfc_la(c) + 1) / 2; }

template <int CB, int CK>
void register_grad_f_pairs(grad_launch_fn *table) {
  if constexpr (CB <= pair_class(GRAD_LMAX, GRAD_LMAX)) {
    if constexpr (CK <= CB) {
      table[qclass_index(CB, CK)] = launch_grad_f<gfc_la(CB), gfc_lb(CB), gfc_la(CK), gfc_lb(CK)>;
      register_grad_f_pairs<CB, CK + 1>(table);
    } else {
      register_grad_f_pairs<CB + 1, 0>(table);
    }
  }
}

void register_grad_f(grad_launch_fn *table) { register_grad_f_pairs<pair_class(3, 0), 0>(table); }

}  // namespace jk
