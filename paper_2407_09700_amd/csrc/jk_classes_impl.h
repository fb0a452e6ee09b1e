// Instantiation helpers for the class translation units.
#pragma once
#include "jk_classes.h"
#include "jk_kernels.h"

namespace jk {

constexpr int DYN_LDS_MAX = 150 * 1024;   // dynamic LDS the J/K kernels may request (CU: 160 KB)

// The dynamic-LDS attribute of every J/K kernel is set once at registration (before any
// launch, so that no attribute call happens while a stream is being recorded into a graph).
template <class F>
void allow_dyn_lds(F *fn) {
  (void)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, DYN_LDS_MAX);
  (void)hipGetLastError();   // the attribute is a hint; do not leave its status for a launch check
}

template <int LA, int LB, int LC, int LD, int KL = 0, bool GL = false>
hipError_t launch_cls(const JKArgs &args, int grid, size_t lds, hipStream_t stream) {
  hipLaunchKernelGGL((k_cls<LA, LB, LC, LD, KL, GL>), dim3(grid), dim3(cls_threads<LA, LB, LC, LD, KL>()), lds, stream,
                     args);
  return hipGetLastError();
}

template <int LA, int LB, int LC, int LD, int MODE>
hipError_t launch_mode(const ModeArgs &args, int grid, hipStream_t stream) {
  constexpr int block = mode_block<LA, LB, LC, LD, MODE>();
  constexpr size_t lds = (size_t)mode_lds<LA, LB, LC, LD, MODE>();
  hipLaunchKernelGGL((k_mode<LA, LB, LC, LD, MODE>), dim3(grid), dim3(block), lds, stream, args);
  return hipGetLastError();
}

template <int LA, int LB, int TIER, bool F32 = false>
hipError_t launch_bra(const JKArgs &args, int grid, size_t lds, hipStream_t stream) {
  hipLaunchKernelGGL((k_bra<LA, LB, TIER, F32>), dim3(grid), dim3(256), lds, stream, args);
  return hipGetLastError();
}

template <int LA, int LB, int LC, int LD>
void register_one(ClassInfo *table) {
  ClassInfo &ci = table[qclass_index(pair_class(LA, LB), pair_class(LC, LD))];
  ci.la = LA; ci.lb = LB; ci.lc = LC; ci.ld = LD;
  if constexpr (use_team<LA, LB, LC, LD>()) {
    using C = TeamCfg<LA, LB, LC, LD>;   // k_mode (Schwarz / ERI tensor) always uses this body
    ci.team = 1;
    ci.block = C::BLOCK;
    ci.per_block = C::QB;
    // k_cls sends exchange to global memory: the one-stage body then also needs its
    // per-quartet exchange blocks in LDS
    ci.team_lds = team_lds_bytes<LA, LB, LC, LD>() +
                  (use_team2<LA, LB, LC, LD>() ? Team2Cfg<LA, LB, LC, LD>::QB * Team2Cfg<LA, LB, LC, LD>::KQ * 8 : 0);
    ci.scratch_per_wg = C::GLOBAL_BUF ? (long long)C::BUF : 0;
  } else {
    ci.team = 0;
    ci.block = 256;
    ci.per_block = 256;
    ci.team_lds = 0;
    ci.scratch_per_wg = 0;
  }
  ci.launch_cls = launch_cls<LA, LB, LC, LD>;
  allow_dyn_lds(k_cls<LA, LB, LC, LD>);
  if constexpr (!use_team<LA, LB, LC, LD>()) {
    ci.launch_clsl = launch_cls<LA, LB, LC, LD, 1>;
    ci.launch_clsa = launch_cls<LA, LB, LC, LD, 2>;
    ci.table_lds = (int)(root_table_doubles<SmallCfg<LA, LB, LC, LD>::N>() * sizeof(double));
    allow_dyn_lds(k_cls<LA, LB, LC, LD, 1>);
    allow_dyn_lds(k_cls<LA, LB, LC, LD, 2>);
    if constexpr (SmallCfg<LA, LB, LC, LD>::N <= JK_TABLE_LDS_NMAX) {
      ci.launch_clslg = launch_cls<LA, LB, LC, LD, 1, true>;
      ci.launch_clsag = launch_cls<LA, LB, LC, LD, 2, true>;
      allow_dyn_lds(k_cls<LA, LB, LC, LD, 1, true>);
      allow_dyn_lds(k_cls<LA, LB, LC, LD, 2, true>);
    } else {
      ci.launch_clslg = nullptr;
      ci.launch_clsag = nullptr;
    }
  } else {
    ci.launch_clsl = nullptr;
    ci.launch_clsa = nullptr;
    ci.table_lds = 0;
    ci.launch_clslg = nullptr;
    ci.launch_clsag = nullptr;
  }
  ci.launch_mode[MODE_JK] = nullptr;
  ci.launch_mode[MODE_SCHWARZ] = (LA == LC && LB == LD) ? launch_mode<LA, LB, LC, LD, MODE_SCHWARZ> : nullptr;
  ci.launch_mode[MODE_ERI] = launch_mode<LA, LB, LC, LD, MODE_ERI>;
  if constexpr (mode_lds<LA, LB, LC, LD, MODE_ERI>() > 0) allow_dyn_lds(k_mode<LA, LB, LC, LD, MODE_ERI>);
}

template <int LA, int LB, int P = 0>
void register_kets(ClassInfo *table) {
  if constexpr (P <= pair_class(LA, LB)) {
    register_one<LA, LB, pc_la(P), pc_lb(P)>(table);
    register_kets<LA, LB, P + 1>(table);
  }
}

template <int LA, int LB, int TIER>
void register_tier(BraInfo &b) {
  b.tier_mask[TIER] = tier_mask<LA, LB, TIER>();
  b.fusable[TIER] = bra_fusable<LA, LB, TIER>() && tier_mask<LA, LB, TIER>() != 0;
  b.pool_bytes[TIER] = bra_pool_bytes<LA, LB, TIER>();
  b.scratch_per_wg[TIER] = bra_scratch_doubles<LA, LB, TIER>();
  b.launch_bra32[TIER] = nullptr;
  if constexpr (bra_fusable<LA, LB, TIER>() && tier_mask<LA, LB, TIER>() != 0) {
    b.launch_bra[TIER] = launch_bra<LA, LB, TIER>;
    allow_dyn_lds(k_bra<LA, LB, TIER>);
    if constexpr (TIER < TEAM_TIER && JK_FP32_BODIES) {
      b.launch_bra32[TIER] = launch_bra<LA, LB, TIER, true>;
      allow_dyn_lds(k_bra<LA, LB, TIER, true>);
    }
  } else
    b.launch_bra[TIER] = nullptr;
}

template <int LA, int LB>
void register_bra(ClassInfo *classes, BraInfo *bras) {
  register_kets<LA, LB>(classes);
  BraInfo &b = bras[pair_class(LA, LB)];
  b.la = LA; b.lb = LB;
  register_tier<LA, LB, 0>(b);
  register_tier<LA, LB, 1>(b);
  register_tier<LA, LB, 2>(b);
  register_tier<LA, LB, 3>(b);
  static_assert(NTIERS == NTIER && TEAM_TIER == 3, "tier tables and kernels disagree");
}

}  // namespace jk
