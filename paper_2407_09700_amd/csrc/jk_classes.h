// Registry of the quartet classes and bra classes and their launchers.
#pragma once
#include "jk_common.h"

namespace jk {

struct JKArgs;
struct ModeArgs;

typedef hipError_t (*jk_launch_fn)(const JKArgs &args, int grid, size_t lds, hipStream_t stream);
typedef hipError_t (*mode_launch_fn)(const ModeArgs &args, int grid, hipStream_t stream);

struct ClassInfo {           // one quartet class (la lb | lc ld)
  int la, lb, lc, ld;
  int team;                  // 1: workgroup body, 0: lane-per-quartet body
  int block;                 // threads of k_cls / k_mode
  int per_block;             // quartets one k_mode workgroup consumes per pass
  int team_lds;              // bytes of team LDS (pool)
  long long scratch_per_wg;  // doubles of global team buffer per workgroup
  jk_launch_fn launch_cls;   // k_cls (exchange to global memory)
  jk_launch_fn launch_clsl;  // k_cls with compacted LDS exchange rows (lane bodies; null for team classes)
  jk_launch_fn launch_clsa;  // the same with only the rows of a in LDS
  jk_launch_fn launch_clslg; // the two above with the root table in LDS (lane bodies of few roots; else null)
  jk_launch_fn launch_clsag;
  int table_lds;             // bytes of that root table
  mode_launch_fn launch_mode[3];
};

constexpr int NTIERS = 4;    // register tiers of the fused kernels (NTIER)

struct BraInfo {             // one bra class (la lb), per register tier
  int la, lb;
  int tier_mask[NTIERS];     // ket classes of each tier (bit ck)
  int fusable[NTIERS];       // k_bra can run every ket class of the tier with 256 lanes
  int pool_bytes[NTIERS];    // team LDS of k_bra
  long long scratch_per_wg[NTIERS];  // doubles of global team buffer per workgroup
  jk_launch_fn launch_bra[NTIERS];   // k_bra (null if not fusable)
  jk_launch_fn launch_bra32[NTIERS]; // FP32-only k_bra of the lane tiers (null for the team tier)
};

#define JK_DECL_BRA(LA, LB) void register_bra_##LA##LB(ClassInfo *classes, BraInfo *bras);
JK_DECL_BRA(0, 0) JK_DECL_BRA(1, 0) JK_DECL_BRA(1, 1) JK_DECL_BRA(2, 0) JK_DECL_BRA(2, 1) JK_DECL_BRA(2, 2)
JK_DECL_BRA(3, 0) JK_DECL_BRA(3, 1) JK_DECL_BRA(3, 2) JK_DECL_BRA(3, 3)
JK_DECL_BRA(4, 0) JK_DECL_BRA(4, 1) JK_DECL_BRA(4, 2) JK_DECL_BRA(4, 3) JK_DECL_BRA(4, 4)
#undef JK_DECL_BRA

}  // namespace jk
