// Argument blocks and launchers of the auxiliary kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "jk_common.h"

namespace jk {

struct ShellInfo {            // device pointers
  const int *l, *pure, *cart_off, *ao_off;
  const int *cart2shell, *ao2shell;
  const double *tsph;         // T2 | T3 | T4 row-major
  int toff[5];                // offset of T_l in tsph (l >= 2)
  int nshell, nc, nao;
};

struct ScreenArgs {           // device pointers
  const double *pairI;        // Schwarz factor per kept pair (sorted by class, then I descending)
  const int *pair_cls, *pair_sa, *pair_sb, *pair_npp;
  const int *cls_beg;         // [16] first pair of each pair class
  const double *Pblk;         // nshell x nshell block maxima of |D_cart|
  const double *gmax;         // global maximum
  unsigned long long *cap;    // [120] size of each class region (k_capacity)
  int *segoff;                // [npairs * 15] segment offset in the class region (k_capacity)
  int *segcnt;                // [npairs * 15] kept kets of the segment (k_screen)
  int *count;                 // [120] kept quartets per class (k_screen)
  unsigned long long *nprim;  // [120] primitive quartets of the kept quartets (k_screen)
  const long long *class_off; // [120] first entry of each class region in kets
  int *kets;
  double tau;
  int npairs, nshell;
};

struct FoldArgs {             // Coulomb pair buffer -> Cartesian Jt
  const int *pair_cls, *pair_ca, *pair_cb, *pair_la, *pair_lb;
  const int *cls_beg;
  const long long *jp_off;
  const double *Jpair;
  double *Jc;
  int npairs, nc;
};

hipError_t launch_dcart(const ShellInfo &S, const double *D, double *Dc, hipStream_t st);
hipError_t launch_blockmax(const ShellInfo &S, const double *Dc, double *Pblk, double *gmax, hipStream_t st);
hipError_t launch_capacity(const ScreenArgs &A, hipStream_t st);
hipError_t launch_screen(const ScreenArgs &A, hipStream_t st);
hipError_t launch_finalize(const ShellInfo &S, const double *Jc, const double *Kc, double *J, double *K,
                           hipStream_t st);
hipError_t launch_fold(const FoldArgs &F, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, long long n, unsigned long long v, hipStream_t st);
hipError_t launch_fill_i32(int *p, long long n, int v, hipStream_t st);

}  // namespace jk
