// Argument blocks and launchers of the auxiliary kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "jk_common.h"

namespace jk {

constexpr int MAX_BINS = 64;  // bins of one (pair class, molecule): distinct contraction lengths, merged above this

struct ShellInfo {            // device pointers; molecules are stored one after another
  const int *l, *pure;        // per shell (global shell index)
  const int *cart_off, *ao_off;   // per shell, inside its molecule
  const int *cart2shell;      // per concatenated Cartesian AO -> global shell
  const int *ao2shell;        // per concatenated final AO -> global shell
  const long long *mc_off;    // [nmol+1] first element of each molecule's nc_m x nc_m block
  const long long *mf_off;    // [nmol+1] prefix of the nao_m^2 block sizes (iteration order)
  const long long *mf_user;   // [nmol] first element of each molecule's block in the caller's D, J, K
  const long long *ps_off;    // [nmol+1] first element of each molecule's shell-pair block
  const int *cbase, *abase, *sbase;   // [nmol+1] first Cartesian AO / final AO / shell of each molecule
  const double *tsph;         // T2 | T3 | T4 row-major
  int toff[5];                // offset of T_l in tsph (l >= 2)
  int nmol;
  long long nc2_tot, nf2_tot, ns2_tot;
};

struct ScreenArgs {           // device pointers
  const double *pairI;        // Schwarz factor per kept pair (sorted by class, molecule, then I descending)
  const int *pair_cls, *pair_sa, *pair_sb, *pair_npp, *pair_mol;
  const int *bin_beg;         // [nbins+1] first pair of each bin (class, molecule, contraction length)
  const int *cm_bin;          // [15 * (nmol+1)] first bin of each (class, molecule)
  const double *Pblk;         // per molecule: nshell_m x nshell_m block maxima of |D_cart|
  double *pairP;              // per kept pair: its own block maximum (k_pairp, read by k_screen)
  const long long *ps_off;    // [nmol+1] first element of each molecule's block in Pblk
  const int *sbase;           // [nmol+1] first shell of each molecule
  const double *gmax;         // global maximum of |D_cart|
  double gfix, gscale;        // k_capacity's density bound: gfix if > 0, else gscale * (*gmax) (k_screen: *gmax)
  unsigned long long *cap;    // [120] size of each class region (k_capacity)
  int *segoff;                // [npairs * 15] segment offset in the class region (k_capacity)
  int *segcnt;                // [npairs * 15] kept FP64 kets of the segment (k_screen)
  int *segoff32, *segcnt32;   // [npairs * 15] FP32 part of the segment (mixed precision) or null
  int *count;                 // [120] kept quartets per class (k_screen)
  int *count32;               // [120] of those, evaluated in FP32
  unsigned long long *nprim;  // [240] primitive quartets of the kept quartets, then of the FP32 ones (k_screen)
  const long long *class_off; // [120] first entry of each class region in kets
  const long long *room;      // [120] entries available to each class region (k_class_room)
  int *kets;
  double tau;
  double fp32_cut;            // quartets with I_ab I_cd P below this go to FP32 (0: none) ...
  unsigned long long f32_classes[2];   // ... if their class (bit qc) has an FP32 body
  int npairs, nmol;
  int want;                   // outputs: bit 0 J (Coulomb blocks in the test), bit 1 K (exchange blocks)
};

struct FoldArgs {             // Coulomb pair buffer -> Cartesian Jt of each molecule
  const int *pair_cls, *pair_ca, *pair_cb, *pair_la, *pair_lb, *pair_mol;
  const int *cls_beg;
  const long long *jp_off;
  const long long *mc_off;
  const int *cbase;
  const double *Jpair;
  double *Jc;
  int npairs;
  const double *Dc;           // k_unfold: Cartesian densities in, pair-ordered blocks out
  double *Dpair;
};

// Dc: Cartesian densities, row-major per molecule; Dp (optional): the same values with the rows
// of each shell stored as a column-major panel (shell rows r0..r0+n: element (r0+i, c) at r0 nc + c n + i)
hipError_t launch_dcart(const ShellInfo &S, const double *D, double *Dc, double *Dp, hipStream_t st);
hipError_t launch_blockmax(const ShellInfo &S, const double *Dc, double *Pblk, double *gmax, hipStream_t st);
hipError_t launch_class_room(const unsigned long long *cap, const long long *capc, long long *room, int *overflow,
                             hipStream_t st);
hipError_t launch_capacity(const ScreenArgs &A, hipStream_t st);
hipError_t launch_screen(const ScreenArgs &A, hipStream_t st);
hipError_t launch_pairp(const ScreenArgs &A, hipStream_t st);
hipError_t launch_finalize(const ShellInfo &S, const double *Jc, const double *Kc, double *J, double *K,
                           hipStream_t st);
hipError_t launch_fold(const FoldArgs &F, hipStream_t st);
hipError_t launch_unfold(const FoldArgs &F, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, long long n, unsigned long long v, hipStream_t st);
hipError_t launch_fill_i32(int *p, long long n, int v, hipStream_t st);
hipError_t launch_units(const int *segcnt, const int *segcnt32, int bra_beg, int bra_end, int mask, int parts,
                        int slice, int2 *units, int units_cap, int *nunits, int *overflow, hipStream_t st);

}  // namespace jk
