// Registry of the 120 quartet classes and their launchers.
#pragma once
#include "jk_common.h"

namespace jk {

typedef hipError_t (*class_launch_fn)(const ClassArgs &args, int grid, hipStream_t stream);

struct ClassInfo {
  int la, lb, lc, ld;
  int team;                  // 1: k_team, 0: k_small
  int block;                 // threads per workgroup
  int per_block;             // quartets one workgroup consumes per pass (lanes or QB)
  long long scratch_per_wg;  // doubles of global scratch per workgroup (team, largest classes)
  class_launch_fn launch[3]; // by mode
};

// filled by the class translation units (one per bra angular momentum la)
void register_classes_l0(ClassInfo *table);
void register_classes_l1(ClassInfo *table);
void register_classes_l2(ClassInfo *table);
void register_classes_l3(ClassInfo *table);
void register_classes_l4(ClassInfo *table);

}  // namespace jk
