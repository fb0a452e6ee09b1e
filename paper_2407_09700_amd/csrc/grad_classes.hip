// Gradient kernels of the quartet classes whose bra pair has momenta up to d (the classes with
// an f in the bra: grad_classes_f.hip).
#include "jk_grad.h"

namespace jk {

template <int LA, int LB, int LC, int LD>
hipError_t launch_grad(const GradArgs &args, int grid, hipStream_t stream) {
  hipLaunchKernelGGL((k_grad<LA, LB, LC, LD>), dim3(grid), dim3(256), 0, stream, args);
  return hipGetLastError();
}

constexpr int gpc_la(int c) { int l = 0; while ((l + 1) * (l + 2) / 2 <= c) ++l; return l; }
constexpr int gpc_lb(int c) { return c - gpc_la(c) * (gpc_la(c) + 1) / 2; }

template <int CB, int CK>
void register_grad_pairs(grad_launch_fn *table) {
  if constexpr (CB <= pair_class(2, 2)) {
    if constexpr (CK <= CB) {
      table[qclass_index(CB, CK)] = launch_grad<gpc_la(CB), gpc_lb(CB), gpc_la(CK), gpc_lb(CK)>;
      register_grad_pairs<CB, CK + 1>(table);
    } else {
      register_grad_pairs<CB + 1, 0>(table);
    }
  }
}

void register_grad(grad_launch_fn *table) {
  for (int q = 0; q < NQCLASS; ++q) table[q] = nullptr;
  register_grad_pairs<0, 0>(table);
  register_grad_f(table);
}

}  // namespace jk
