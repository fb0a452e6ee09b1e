// Instantiation helpers for the class translation units.
#pragma once
#include "jk_classes.h"
#include "jk_kernels.h"

namespace jk {

constexpr int SMALL_REG_LIMIT = 100;   // k_small when [e0|f0] accumulators + one root's 2D integrals fit

template <int LA, int LB, int LC, int LD>
constexpr bool use_team() { return SmallCfg<LA, LB, LC, LD>::REGS > SMALL_REG_LIMIT; }

template <int LA, int LB, int LC, int LD, int MODE>
hipError_t launch_class(const ClassArgs &args, int grid, hipStream_t stream) {
  if constexpr (use_team<LA, LB, LC, LD>()) {
    using C = TeamCfg<LA, LB, LC, LD>;
    hipLaunchKernelGGL((k_team<LA, LB, LC, LD, MODE>), dim3(grid), dim3(C::BLOCK), 0, stream, args);
  } else {
    hipLaunchKernelGGL((k_small<LA, LB, LC, LD, MODE>), dim3(grid), dim3(256), 0, stream, args);
  }
  return hipGetLastError();
}

template <int LA, int LB, int LC, int LD>
void register_one(ClassInfo *table) {
  static_assert(LA >= LB && LC >= LD && LA * (LA + 1) / 2 + LB >= LC * (LC + 1) / 2 + LD, "canonical class");
  ClassInfo &ci = table[qclass_index(pair_class(LA, LB), pair_class(LC, LD))];
  ci.la = LA; ci.lb = LB; ci.lc = LC; ci.ld = LD;
  if constexpr (use_team<LA, LB, LC, LD>()) {
    using C = TeamCfg<LA, LB, LC, LD>;
    ci.team = 1;
    ci.block = C::BLOCK;
    ci.per_block = C::QB;
    ci.scratch_per_wg = C::GLOBAL_BUF ? (long long)C::BUF : 0;
  } else {
    ci.team = 0;
    ci.block = 256;
    ci.per_block = 256;
    ci.scratch_per_wg = 0;
  }
  ci.launch[MODE_JK] = launch_class<LA, LB, LC, LD, MODE_JK>;
  ci.launch[MODE_SCHWARZ] = (LA == LC && LB == LD) ? launch_class<LA, LB, LC, LD, MODE_SCHWARZ> : nullptr;
  ci.launch[MODE_ERI] = launch_class<LA, LB, LC, LD, MODE_ERI>;
}

// all ket classes (lc, ld) <= (LA, LB) for one bra class
template <int LA, int LB>
void register_bra(ClassInfo *table) {
#define JK_REG_KET(LC, LD) \
  if constexpr (LC * (LC + 1) / 2 + LD <= LA * (LA + 1) / 2 + LB) register_one<LA, LB, LC, LD>(table);
  JK_REG_KET(0, 0) JK_REG_KET(1, 0) JK_REG_KET(1, 1) JK_REG_KET(2, 0) JK_REG_KET(2, 1) JK_REG_KET(2, 2)
  JK_REG_KET(3, 0) JK_REG_KET(3, 1) JK_REG_KET(3, 2) JK_REG_KET(3, 3)
  JK_REG_KET(4, 0) JK_REG_KET(4, 1) JK_REG_KET(4, 2) JK_REG_KET(4, 3) JK_REG_KET(4, 4)
#undef JK_REG_KET
}

}  // namespace jk
