// Kernels of the J/K build (templated on the angular momenta of the bra and ket classes).
//
// Digestion (paper section 3, the six updates of Algorithm 2 with the eight-fold symmetry
// factor s of a unique quartet):
//   Jt[a,b] += 2s (ab|cd) D[c,d]    Jt[c,d] += 2s (ab|cd) D[a,b]
//   Kt[a,c] += s (ab|cd) D[b,d]     Kt[b,d] += s (ab|cd) D[a,c]
//   Kt[a,d] += s (ab|cd) D[b,c]     Kt[b,c] += s (ab|cd) D[a,d]
// in the Cartesian components; J = Jt + Jt^T and K = Kt + Kt^T are formed afterwards.
//
// Work units are bra pairs: the screen leaves, for every bra pair and ket class, a segment
// of kept ket pairs. Coulomb updates go to a buffer indexed by shell pair (element-major per
// pair class, so lanes that hold consecutive kets write consecutive addresses); the bra
// pair's own J block is reduced over the whole unit before it is written. Exchange updates
// all land in the two rows of the bra shells, K[a,:] and K[b,:]:
//   k_bra<la,lb>        one workgroup per bra pair over every ket class; both rows live in
//                       LDS (LDS atomics) and are flushed once per unit with coalesced
//                       global atomics;
//   k_cls<la,lb,lc,ld>  one workgroup per (bra pair, ket class) with exchange updates sent
//                       straight to global memory (used when the rows do not fit in LDS).
// Device FP64 atomics cost one L2 request per 64-byte line touched by a wave instruction,
// so the layouts above keep every global atomic of a wave on few lines.
#pragma once
#include "jk_eri.h"

// FP32 lane bodies for the mixed-precision quartets (0: they run the FP64 bodies)
#ifndef JK_FP32_BODIES
#define JK_FP32_BODIES 1
#endif

namespace jk {

#ifndef JK_SMALL_REG_LIMIT
#define JK_SMALL_REG_LIMIT 200
#endif
constexpr int SMALL_REG_LIMIT = JK_SMALL_REG_LIMIT;   // lane per quartet when [e0|f0] accumulators + one root's 2D integrals fit
#ifndef JK_SMALL_OUT_LIMIT
#define JK_SMALL_OUT_LIMIT 200
#endif
constexpr int SMALL_OUT_LIMIT = JK_SMALL_OUT_LIMIT;   // ... and the contracted block + the bra Coulomb partials fit

template <int LA, int LB, int LC, int LD>
constexpr bool use_team() {
  using C = SmallCfg<LA, LB, LC, LD>;
  return C::REGS > SMALL_REG_LIMIT || C::NG + C::NA * C::NB > SMALL_OUT_LIMIT;
}

// Register tiers of the fused kernels: 0 light, 1 middle and 2 heavy lane bodies, 3 team
// bodies (TEAM_TIER). Each tier is its own launch so that the heaviest body does not set the
// occupancy of all: the compiler sizes a kernel's registers by its largest body.
constexpr int NTIER = 4, TEAM_TIER = 3;
#ifndef JK_TIER0_MAX
#define JK_TIER0_MAX 64
#endif
#ifndef JK_TIER1_MAX
#define JK_TIER1_MAX 150
#endif
template <int LA, int LB, int LC, int LD>
constexpr int tier_of() {
  using C = SmallCfg<LA, LB, LC, LD>;
  if (use_team<LA, LB, LC, LD>()) return TEAM_TIER;
  constexpr int big = C::REGS > C::NG + C::NA * C::NB ? C::REGS : C::NG + C::NA * C::NB;
  return big <= JK_TIER0_MAX ? 0 : (big <= JK_TIER1_MAX ? 1 : 2);
}

constexpr int pc_la(int c) { int l = 0; while ((l + 1) * (l + 2) / 2 <= c) ++l; return l; }
constexpr int pc_lb(int c) { return c - pc_la(c) * (pc_la(c) + 1) / 2; }

struct JKArgs {
  const Pair *pairs;
  const PrimPair *pp;
  const int *kets;              // segment storage (ket pair indices)
  const long long *class_off;   // [120] first entry of each class region in kets
  const int *segoff;            // [npairs * 15] segment offset inside the class region
  const int *segcnt;            // [npairs * 15] kept kets of the segment (FP64 part)
  const int *segoff32;          // [npairs * 15] start of the FP32 part of the segment (mixed precision) or null
  const int *segcnt32;          // [npairs * 15] kets of the FP32 part or null
  const double *Dp;             // Cartesian densities, one nc_m x nc_m block per molecule, each shell's
                                // rows stored as a column-major panel (the block of shells s, t:
                                // ncart(s) ncart(t) consecutive doubles at r0_s nc + c0_t ncart(s))
  double *Kc;                   // Cartesian exchange accumulators, row-major nc_m x nc_m per molecule
  const long long *mbase;       // [nmol] first element of each molecule's block in Dp / Kc
  const int *mnc;               // [nmol] Cartesian AO count of each molecule
  double *Jpair;                // Coulomb accumulator per shell pair
  const double *Dpair;          // density block D[c,d] of every kept pair, laid out as Jpair
  const long long *jp_off;      // [15] first element of each pair class in Jpair
  const int *cls_beg;           // [16] first pair of each pair class
  int nc_max;                   // largest nc_m (row length of the LDS exchange rows)
  int bra_beg, bra_end;         // bra pairs of the launched bra class
  int *next;                    // work counter of the launch
  const int2 *units;            // work units (bra pair, slice index) of the launch (k_units)
  const int *nunits;            // their number (entries beyond units_cap were not written)
  int units_cap;
  int slice;                    // kets per unit: a unit runs kets [j slice, (j+1) slice) of the bra's
                                // kets in the launch, counted over the ket classes in order, FP64
                                // part of each segment before its FP32 part
  int parts;                    // segment parts of the launch: 1 FP64, 2 FP32, 3 both (k_bra)
  double *scratch;              // global buffers of the largest team classes
  long long scratch_per_wg;
  int want;                     // outputs of the build: bit 0 J, bit 1 K (both: the full digestion)
  // compacted exchange rows of the per-class kernel (k_cls with KL): for the ket class (lc, ld)
  // a row holds the Cartesian columns of the molecule's shells of angular momentum lc, then
  // (lc != ld) those of momentum ld
  const int *lcol;              // per shell: first column of the shell inside its momentum's segment
  const int *lcols;             // per molecule (from cbase[m]): Cartesian columns ordered by momentum
  const int *lseg;              // [nmol * 6] start of each momentum's segment in lcols (l = 0..4, end)
  const int *cbase;             // [nmol + 1] first Cartesian AO of each molecule
  int kw;                       // LDS row length of the launch (largest over its molecules)
  int kwb;                      // k_cls with KL = 2: compacted columns of the rows of b held in LDS
};

__device__ __forceinline__ double *jp_elem(const JKArgs &A, int cls, int pair, int e) {
  const int beg = A.cls_beg[cls];
  return A.Jpair + A.jp_off[cls] + (long long)e * (A.cls_beg[cls + 1] - beg) + (pair - beg);
}

// element e of pair `pair`'s density block in the pair-ordered copy: the kets of a segment are
// mostly consecutive pairs, so the lanes of a wave read one element of their blocks coalesced
__device__ __forceinline__ double dp_elem(const JKArgs &A, int cls, int pair, int e) {
  const int beg = A.cls_beg[cls];
  return A.Dpair[A.jp_off[cls] + (long long)e * (A.cls_beg[cls + 1] - beg) + (pair - beg)];
}

// exchange update into row `r` of the unit: LDS rows (KLDS; r < NA+NB, row length kst, column
// kcol) or the global matrix Km (the molecule's exchange block, row grow, column gcol, row
// length nc).
template <bool KLDS>
__device__ __forceinline__ void k_update(double *Krow, double *Km, int kst, int nc, int r, int grow, int kcol, int gcol,
                                         double v) {
  if constexpr (KLDS)
    atomicAdd(&Krow[(size_t)r * kst + kcol], v);
  else
    atomic_add(&Km[(size_t)grow * nc + gcol], v);
}

// ------------------------------------------------------------------ lane-per-quartet body
// R: arithmetic type of the integral evaluation (double, or float for the FP32 quartets of
// mixed precision); the digestion always runs in double.
// KMAP: the LDS rows are the compacted rows of k_cls (row length kst, ket class columns from
// kdofs); otherwise full rows of the molecule's Cartesian columns (row length nc). KLB false:
// only the rows of a are full LDS rows; the rows of b keep their first A.kwb compacted columns
// in LDS (after the rows of a, row length A.kwb) and send the others to global memory.
template <int LA, int LB, int LC, int LD, bool KLDS, typename R = double, bool KMAP = false, bool KLB = true>
__device__ __forceinline__ void jk_small_body(const JKArgs &A, int bi, const int *kl, int cnt, double *Krow,
                                              double (&jab)[ncart(LA) * ncart(LB)], int rot, int kdofs = 0,
                                              int kst_map = 0, const double *table = nullptr) {
  using C = SmallCfg<LA, LB, LC, LD>;
  constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND;
  constexpr int ck = pair_class(LC, LD);
  const Pair bra = A.pairs[bi];
  const int nc = A.mnc[bra.mol];
  // density rows of a and of b from the shell panels: D[a, col] = Pa[col NA + a], so each block
  // D[a-shell, ket shell] the digestion reads is one contiguous run
  const double *Pa = A.Dp + A.mbase[bra.mol] + (size_t)bra.ca * nc;
  const double *Pb = A.Dp + A.mbase[bra.mol] + (size_t)bra.cb * nc;
  double *Km = A.Kc + A.mbase[bra.mol];
  double Dab[NA * NB];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) Dab[a * NB + b] = Pa[(size_t)(bra.cb + b) * NA + a];
  // ket k runs on lane (k + rot) mod blockDim: successive segments of a unit continue where the
  // previous one ended, so the waves of the workgroup share the unit's kets evenly
  for (int k = (int)((threadIdx.x + blockDim.x - rot) % blockDim.x); k < cnt; k += blockDim.x) {
    const int ki = kl[k];
    const Pair ket = A.pairs[ki];
    R g[C::NG];                 // FP32 integrals stay FP32 in registers; each use widens to double
    small_eri<LA, LB, LC, LD, R>(bra, ket, A.pp, g, table);
    const double s = sym_factor(bra, ket, bi, ki);
    const int oc = ket.ca, od = ket.cb;
    if (A.want & 1) {
      double Dcd[NC * ND];
#pragma unroll
      for (int cd = 0; cd < NC * ND; ++cd) Dcd[cd] = dp_elem(A, ck, ki, cd);
#pragma unroll
      for (int ab = 0; ab < NA * NB; ++ab) {
        double v = 0.0;
#pragma unroll
        for (int cd = 0; cd < NC * ND; ++cd) v = fma((double)g[ab * NC * ND + cd], Dcd[cd], v);
        jab[ab] = fma(2.0 * s, v, jab[ab]);
      }
#pragma unroll
      for (int cd = 0; cd < NC * ND; ++cd) {
        double v = 0.0;
#pragma unroll
        for (int ab = 0; ab < NA * NB; ++ab) v = fma((double)g[ab * NC * ND + cd], Dab[ab], v);
        atomic_add(jp_elem(A, ck, ki, cd), 2.0 * s * v);
      }
    }
    if (!(A.want & 2)) continue;
    const int kc = KMAP ? A.lcol[ket.sa] : oc, kd = KMAP ? kdofs + A.lcol[ket.sb] : od;
    const int kst = KMAP ? kst_map : nc;
    // exchange: rows a (K[a,c] with D[b,d], K[a,d] with D[b,c]), rows b (K[b,c] with D[a,d], K[b,d] with D[a,c])
#pragma unroll
    for (int a = 0; a < NA; ++a) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int d = 0; d < ND; ++d) v = fma((double)g[(a * NB + b) * NC * ND + c * ND + d], Pb[(size_t)(od + d) * NB + b], v);
        k_update<KLDS>(Krow, Km, kst, nc, a, bra.ca + a, kc + c, oc + c, s * v);
      }
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int c = 0; c < NC; ++c) v = fma((double)g[(a * NB + b) * NC * ND + c * ND + d], Pb[(size_t)(oc + c) * NB + b], v);
        k_update<KLDS>(Krow, Km, kst, nc, a, bra.ca + a, kd + d, od + d, s * v);
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double v = 0.0;
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int d = 0; d < ND; ++d) v = fma((double)g[(a * NB + b) * NC * ND + c * ND + d], Pa[(size_t)(od + d) * NA + a], v);
        if (KLDS && !KLB && kc + c < A.kwb)
          atomicAdd(&Krow[(size_t)NA * A.kw + b * A.kwb + kc + c], s * v);
        else
          k_update<KLDS && KLB>(Krow, Km, kst, nc, NA + b, bra.cb + b, kc + c, oc + c, s * v);
      }
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        double v = 0.0;
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int c = 0; c < NC; ++c) v = fma((double)g[(a * NB + b) * NC * ND + c * ND + d], Pa[(size_t)(oc + c) * NA + a], v);
        if (KLDS && !KLB && kd + d < A.kwb)
          atomicAdd(&Krow[(size_t)NA * A.kw + b * A.kwb + kd + d], s * v);
        else
          k_update<KLDS && KLB>(Krow, Km, kst, nc, NA + b, bra.cb + b, kd + d, od + d, s * v);
      }
    }
  }
}

// ------------------------------------------------------------------ density blocks of a batch
// The density blocks a batch's digestion reads, staged in LDS (independent loads, all in flight):
//   ds[0, NA NB) = D[a,b]; per quartet q from ds + NA NB + q DQ: D[c,d] | D[a,c] | D[a,d] |
//   D[b,c] | D[b,d]; then the symmetry factors s of the QB quartets.
template <int NA, int NB, int NC, int ND>
constexpr int stage_dq() { return NC * ND + (NA + NB) * (NC + ND); }
template <int NA, int NB, int NC, int ND>
constexpr int stage_doubles(int qb) { return NA * NB + qb * (stage_dq<NA, NB, NC, ND>() + 1); }

// Dp: the molecule's densities in shell panels (element (r0 + i, col) of the shell whose rows
// start at r0, with n rows, at r0 nc + col n + i), so each block below is one contiguous run.
template <int NA, int NB, int NC, int ND, int QB>
__device__ __forceinline__ void stage_density(const JKArgs &A, const Pair &bra, int bi, const double *Dp, int nc,
                                              const int *qi, double *ds) {
  constexpr int NAB = NA * NB, NCD = NC * ND, DQ = stage_dq<NA, NB, NC, ND>();
  const int oa = bra.ca, ob = bra.cb;
  for (int t = threadIdx.x; t < NAB + QB * (DQ + 1); t += blockDim.x) {
    if (t < NAB) {
      ds[t] = Dp[(size_t)oa * nc + (size_t)(ob + t % NB) * NA + t / NB];
      continue;
    }
    int u = t - NAB;
    if (u >= QB * DQ) {                      // symmetry factor of quartet u - QB DQ
      const int q = u - QB * DQ;
      if (qi[q * 8 + 6]) ds[t] = sym_factor(bra, A.pairs[qi[q * 8 + 1]], bi, qi[q * 8 + 1]);
      continue;
    }
    const int q = u / DQ;
    u %= DQ;
    if (!qi[q * 8 + 6]) continue;
    const Pair &ket = A.pairs[qi[q * 8 + 1]];
    const int oc = ket.ca, od = ket.cb;
    int r0, n, i, c;   // element (r0 + i, c) of the panel of the shell with rows r0 .. r0 + n
    if (u < NCD) {
      r0 = oc; n = NC; i = u / ND; c = od + u % ND;
    } else if ((u -= NCD) < NA * NC) {
      r0 = oa; n = NA; i = u / NC; c = oc + u % NC;
    } else if ((u -= NA * NC) < NA * ND) {
      r0 = oa; n = NA; i = u / ND; c = od + u % ND;
    } else if ((u -= NA * ND) < NB * NC) {
      r0 = ob; n = NB; i = u / NC; c = oc + u % NC;
    } else {
      u -= NB * NC;
      r0 = ob; n = NB; i = u / ND; c = od + u % ND;
    }
    ds[t] = Dp[(size_t)r0 * nc + (size_t)c * n + i];
  }
}

// Row sums of eight rows over the 64 lanes of a wave (p[r]: this lane's share of row r). Three
// exchange steps halve the rows each lane carries (lane bit 2, 1, 0 picks the half it keeps),
// three more add the eight lane groups: lane l returns the full sum of row l & 7. Ten shuffles
// for eight rows instead of six per row.
__device__ __forceinline__ double rows8_sum(const double (&p)[8], int lane) {
  const bool b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
  double q4[4], q2[2];
#pragma unroll
  for (int j = 0; j < 4; ++j) q4[j] = (b2 ? p[j + 4] : p[j]) + __shfl_xor(b2 ? p[j] : p[j + 4], 4);
#pragma unroll
  for (int j = 0; j < 2; ++j) q2[j] = (b1 ? q4[j + 2] : q4[j]) + __shfl_xor(b1 ? q4[j] : q4[j + 2], 2);
  double v = (b0 ? q2[1] : q2[0]) + __shfl_xor(b0 ? q2[0] : q2[1], 1);
  v += __shfl_xor(v, 8);
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// ------------------------------------------------------------------ workgroup body
// pool: TeamCfg::LDS_BYTES of LDS; jab_s: NA*NB doubles of LDS (bra Coulomb block).
template <int LA, int LB, int LC, int LD, bool KLDS>
__device__ __forceinline__ void jk_team_body(const JKArgs &A, int bi, const int *kl, int cnt, double *Krow,
                                             double *jab_s, double *pool) {
  using C = TeamCfg<LA, LB, LC, LD>;
  constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND, QB = C::QB;
  constexpr int ck = pair_class(LC, LD);
  double *sG = pool;
  double *co = pool + C::SG;                          // recurrence coefficients of a primitive window
  double *ds = pool;                                  // D blocks of the batch (after team_eri, same region)
  double *lbuf = pool + C::SGC;
  double *dg = lbuf + (C::GLOBAL_BUF ? 0 : C::BUF);   // QB x DG digestion accumulators
  double *geo = dg + QB * C::DG;
  int *qi = reinterpret_cast<int *>(geo + QB * 12);
  int *smax = qi + QB * 8;
  double *buf = C::GLOBAL_BUF ? A.scratch + (size_t)blockIdx.x * A.scratch_per_wg : lbuf;
  const Pair bra = A.pairs[bi];
  const int tid = threadIdx.x;
  const int nc = A.mnc[bra.mol];
  const double *Dpm = A.Dp + A.mbase[bra.mol];   // shell panels
  double *Km = A.Kc + A.mbase[bra.mol];
  const int oa = bra.ca, ob = bra.cb;
  constexpr int NCD = NC * ND, CH = (NCD + 63) / 64, DQ = C::DQ;
  constexpr int NAB = NA * NB, NG = NAB * NCD;
  for (int k0 = 0; k0 < cnt; k0 += QB) {
    if (tid < QB) {
      const int k = k0 + tid;
      const bool valid = k < cnt;
      const int ki = kl[valid ? k : k0];
      team_fill<LA, LB, LC, LD>(tid, bra, A.pairs[ki], bi, ki, valid, qi, geo);
    }
    __syncthreads();
    // Z_LDS: Y (the digestion forms Z block by block); ZS_LDS: Z in LDS after the staged densities
    const double *Z = team_eri<LA, LB, LC, LD, C::X_LDS, C::Z_LDS>(A.pp, sG, co, buf, qi, geo, smax,
                                                                  C::ZS_LDS ? ds + C::DSTG : nullptr);
    stage_density<NA, NB, NC, ND, QB>(A, bra, bi, Dpm, nc, qi, ds);
    for (int t = tid; t < QB * C::DG; t += blockDim.x) dg[t] = 0.0;
    double *pbc = ds + C::DSTG, *pbd = pbc + QB * NB * NCD;   // streamed digestion only
    for (int t = tid; t < C::PBD; t += blockDim.x) pbc[t] = 0.0;
    __syncthreads();
    const double *dab_s = ds, *sq = ds + NAB + QB * DQ;
    if constexpr (NCD < TEAM_STREAM_MIN) {
      // Small ket blocks: one task per output element, one loop per kind of output (no
      // divergence between kinds), integrals and densities read from LDS (or the buffer).
      const int nj = (A.want & 1) ? 1 : 0, nk = (A.want & 2) ? 1 : 0;
      for (int t = tid; t < nj * QB * NAB; t += blockDim.x) {     // J[a,b] += 2s sum_cd g D[c,d]
        const int q = t / NAB, r = t % NAB;
        if (!qi[q * 8 + 6]) continue;
        const double *gr = Z + (size_t)q * NG + r * NCD, *dcd = ds + NAB + q * DQ;
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < NCD; ++i) v = fma(gr[i], dcd[i], v);
        atomicAdd(&jab_s[r], 2.0 * sq[q] * v);
      }
      for (int t = tid; t < nj * QB * NCD; t += blockDim.x) {     // J[c,d] += 2s sum_ab g D[a,b]
        const int q = t / NCD, r = t % NCD;
        if (!qi[q * 8 + 6]) continue;
        const double *g = Z + (size_t)q * NG + r;
        double v = 0.0;
#pragma unroll 16
        for (int i = 0; i < NAB; ++i) v = fma(g[i * NCD], dab_s[i], v);
        atomic_add(jp_elem(A, ck, qi[q * 8 + 1], r), 2.0 * sq[q] * v);
      }
      for (int t = tid; t < nk * QB * NA * NC; t += blockDim.x) { // K[a,c] += s sum_bd g D[b,d]
        const int q = t / (NA * NC), a = (t / NC) % NA, c = t % NC;
        if (!qi[q * 8 + 6]) continue;
        const double *g = Z + (size_t)q * NG + a * NB * NCD + c * ND;
        const double *dbd = ds + NAB + q * DQ + NCD + NA * NC + NA * ND + NB * NC;
        double v = 0.0;
#pragma unroll
        for (int i = 0; i < NB * ND; ++i) v = fma(g[(i / ND) * NCD + i % ND], dbd[i], v);
        const int oc = A.pairs[qi[q * 8 + 1]].ca;
        k_update<KLDS>(Krow, Km, nc, nc, a, oa + a, oc + c, oc + c, sq[q] * v);
      }
      for (int t = tid; t < nk * QB * NA * ND; t += blockDim.x) { // K[a,d] += s sum_bc g D[b,c]
        const int q = t / (NA * ND), a = (t / ND) % NA, d = t % ND;
        if (!qi[q * 8 + 6]) continue;
        const double *g = Z + (size_t)q * NG + a * NB * NCD + d;
        const double *dbc = ds + NAB + q * DQ + NCD + NA * NC + NA * ND;
        double v = 0.0;
#pragma unroll 16
        for (int i = 0; i < NB * NC; ++i) v = fma(g[(i / NC) * NCD + (i % NC) * ND], dbc[i], v);
        const int od = A.pairs[qi[q * 8 + 1]].cb;
        k_update<KLDS>(Krow, Km, nc, nc, a, oa + a, od + d, od + d, sq[q] * v);
      }
      for (int t = tid; t < nk * QB * NB * NC; t += blockDim.x) { // K[b,c] += s sum_ad g D[a,d]
        const int q = t / (NB * NC), b = (t / NC) % NB, c = t % NC;
        if (!qi[q * 8 + 6]) continue;
        const double *g = Z + (size_t)q * NG + b * NCD + c * ND;
        const double *dad = ds + NAB + q * DQ + NCD + NA * NC;
        double v = 0.0;
#pragma unroll 16
        for (int i = 0; i < NA * ND; ++i) v = fma(g[(i / ND) * NB * NCD + i % ND], dad[i], v);
        const int oc = A.pairs[qi[q * 8 + 1]].ca;
        k_update<KLDS>(Krow, Km, nc, nc, NA + b, ob + b, oc + c, oc + c, sq[q] * v);
      }
      for (int t = tid; t < nk * QB * NB * ND; t += blockDim.x) { // K[b,d] += s sum_ac g D[a,c]
        const int q = t / (NB * ND), b = (t / ND) % NB, d = t % ND;
        if (!qi[q * 8 + 6]) continue;
        const double *g = Z + (size_t)q * NG + b * NCD + d;
        const double *dac = ds + NAB + q * DQ + NCD;
        double v = 0.0;
#pragma unroll 16
        for (int i = 0; i < NA * NC; ++i) v = fma(g[(i / NC) * NB * NCD + (i % NC) * ND], dac[i], v);
        const int od = A.pairs[qi[q * 8 + 1]].cb;
        k_update<KLDS>(Krow, Km, nc, nc, NA + b, ob + b, od + d, od + d, sq[q] * v);
      }
      __syncthreads();
      continue;
    }
    // Digestion, every integral read once: each wave streams rows (a, b) of the block (RB rows
    // loaded together: all NB rows of an a when they fit), its lanes run over (c, d). J[a,b] is
    // wave-reduced eight rows at a time; J[c,d], K[a,c] and K[a,d] collect in registers; K[b,c]
    // and K[b,d] in LDS per (b, cd), summed over d or c afterwards (no two lanes of a wave add
    // to the same address). The per-quartet sums are flushed below. Z_LDS: per quartet, the
    // ket transfer first writes the rows of NAZ components a into LDS, which the waves then read.
    const int lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
    const bool wj = A.want & 1, wk = A.want & 2;
    constexpr int RB = NB * CH <= 32 ? NB : 4;
    double *zb = ds + C::DSTG + C::PBD;    // Z_LDS: block of ket-transferred rows (free LDS)
    for (int q = 0; q < QB; ++q) {
      if (!qi[q * 8 + 6]) continue;
      const double s2 = 2.0 * sq[q];
      const double *Dcd = ds + NAB + q * DQ, *Dac = Dcd + NCD, *Dad = Dac + NA * NC, *Dbc = Dad + NA * ND,
                   *Dbd = Dbc + NB * NC;
      double *kac = dg + q * C::DG, *kad = kac + NA * NC;
      double *jcd = kad + NA * ND + NB * NC + NB * ND;
      double *pbcq = pbc + q * NB * NCD, *pbdq = pbd + q * NB * NCD;
      int cc[CH], dd[CH];
      bool on[CH];
      double dcd[CH], jcda[CH];
#pragma unroll
      for (int h = 0; h < CH; ++h) {
        const int cd = h * 64 + lane;
        on[h] = cd < NCD;
        cc[h] = on[h] ? cd / ND : 0;
        dd[h] = on[h] ? cd % ND : 0;
        dcd[h] = on[h] ? Dcd[cd] : 0.0;
        jcda[h] = 0.0;
      }
      for (int a0 = 0; a0 < NA; a0 += (C::Z_LDS ? C::NAZ : NA)) {
      const int a1 = C::Z_LDS ? min(a0 + C::NAZ, NA) : NA;
      const double *g;         // rows (a, b) of this block: g[((a - ga0) * NB + b) * NCD + cd]
      int ga0 = 0;
      if constexpr (C::Z_LDS) {
        team_ket_rows<LA, LB, LC, LD>(Z, geo, q, a0, a1 - a0, zb);
        __syncthreads();
        g = zb;
        ga0 = a0;
      } else {
        g = Z + (size_t)q * NG;
      }
      for (int a = a0 + wave; a < a1; a += nwave) {
        double dad[CH], dac[CH], kacs[CH], kads[CH];
#pragma unroll
        for (int h = 0; h < CH; ++h) {
          dad[h] = Dad[a * ND + dd[h]];
          dac[h] = Dac[a * NC + cc[h]];
          kacs[h] = 0.0;
          kads[h] = 0.0;
        }
        constexpr int NB8 = (NB + 7) / 8 * 8;
        double vr[NB8];
#pragma unroll
        for (int b = NB; b < NB8; ++b) vr[b] = 0.0;
#pragma unroll
        for (int b0 = 0; b0 < NB; b0 += RB) {
          double xs[RB][CH];
#pragma unroll
          for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int h = 0; h < CH; ++h)
              xs[i][h] = (b0 + i < NB && on[h]) ? g[(size_t)((a - ga0) * NB + b0 + i) * NCD + h * 64 + lane] : 0.0;
#pragma unroll
          for (int i = 0; i < RB; ++i) {
            const int b = b0 + i;
            if (b >= NB) break;
            const double dab = dab_s[a * NB + b];
            double vab = 0.0;
#pragma unroll
            for (int h = 0; h < CH; ++h) {
              if (!on[h]) continue;
              const double x = xs[i][h];
              if (wj) {
                vab = fma(x, dcd[h], vab);
                jcda[h] = fma(x, dab, jcda[h]);
              }
              if (wk) {
                kacs[h] = fma(x, Dbd[b * ND + dd[h]], kacs[h]);
                kads[h] = fma(x, Dbc[b * NC + cc[h]], kads[h]);
                atomicAdd(&pbcq[b * NCD + h * 64 + lane], x * dad[h]);
                atomicAdd(&pbdq[b * NCD + h * 64 + lane], x * dac[h]);
              }
            }
            vr[b] = vab;
          }
        }
#pragma unroll
        for (int b0 = 0; b0 < NB8; b0 += 8) {
          double p8[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) p8[i] = vr[b0 + i];
          const double v = rows8_sum(p8, lane);
          const int b = b0 + lane;
          if (lane < 8 && b < NB && v != 0.0) atomicAdd(&jab_s[a * NB + b], s2 * v);
        }
#pragma unroll
        for (int h = 0; h < CH; ++h)
          if (on[h]) {
            atomicAdd(&kac[a * NC + cc[h]], kacs[h]);
            atomicAdd(&kad[a * ND + dd[h]], kads[h]);
          }
      }
      if constexpr (C::Z_LDS) __syncthreads();   // the block is read before the next one is written
      }
#pragma unroll
      for (int h = 0; h < CH; ++h)
        if (on[h]) atomicAdd(&jcd[h * 64 + lane], jcda[h]);
    }
    __syncthreads();
    // K[b,c] = sum_d and K[b,d] = sum_c of the per-(b, cd) partials
    for (int t = tid; t < QB * NB * (NC + ND); t += blockDim.x) {
      const int q = t / (NB * (NC + ND)), r = t % (NB * (NC + ND));
      const double *pq = pbc + q * NB * NCD, *pdq = pbd + q * NB * NCD;
      double *kbc = dg + q * C::DG + NA * NC + NA * ND, *kbd = kbc + NB * NC;
      double v = 0.0;
      if (r < NB * NC) {
        const int b = r / NC, c = r % NC;
#pragma unroll
        for (int d = 0; d < ND; ++d) v += pq[b * NCD + c * ND + d];
        kbc[r] = v;
      } else {
        const int b = (r - NB * NC) / ND, d = (r - NB * NC) % ND;
#pragma unroll
        for (int c = 0; c < NC; ++c) v += pdq[b * NCD + c * ND + d];
        kbd[r - NB * NC] = v;
      }
    }
    __syncthreads();
    for (int t = tid; t < QB * C::DG; t += blockDim.x) {
      const int q = t / C::DG;
      int r = t % C::DG;
      const double v = dg[t];
      if (!qi[q * 8 + 6] || v == 0.0) continue;
      const int ki = qi[q * 8 + 1];
      const Pair &ket = A.pairs[ki];
      const double s = sq[q];
      const int oc = ket.ca, od = ket.cb;
      if (r < NA * NC) {                                // K[a,c] += s sum_bd g D[b,d]
        k_update<KLDS>(Krow, Km, nc, nc, r / NC, oa + r / NC, oc + r % NC, oc + r % NC, s * v);
        continue;
      }
      r -= NA * NC;
      if (r < NA * ND) {                                // K[a,d] += s sum_bc g D[b,c]
        k_update<KLDS>(Krow, Km, nc, nc, r / ND, oa + r / ND, od + r % ND, od + r % ND, s * v);
        continue;
      }
      r -= NA * ND;
      if (r < NB * NC) {                                // K[b,c] += s sum_ad g D[a,d]
        k_update<KLDS>(Krow, Km, nc, nc, NA + r / NC, ob + r / NC, oc + r % NC, oc + r % NC, s * v);
        continue;
      }
      r -= NB * NC;
      if (r < NB * ND) {                                // K[b,d] += s sum_ac g D[a,c]
        k_update<KLDS>(Krow, Km, nc, nc, NA + r / ND, ob + r / ND, od + r % ND, od + r % ND, s * v);
        continue;
      }
      r -= NB * ND;                                     // J[c,d] += 2s sum_ab g D[a,b]
      atomic_add(jp_elem(A, ck, ki, r), 2.0 * s * v);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ workgroup body, one LDS stage
// pool: Team2Cfg::LDS_BYTES of LDS. The bra Coulomb partials accumulate in jab (registers).
template <int LA, int LB, int LC, int LD, bool KLDS>
__device__ __forceinline__ void jk_team2_body(const JKArgs &A, int bi, const int *kl, int cnt, double *Krow,
                                              double *pool, double (&jab)[ncart(LA) * ncart(LB)]) {
  using C = Team2Cfg<LA, LB, LC, LD>;
  constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND, QB = C::QB;
  constexpr int ck = pair_class(LC, LD);
  double *sG = pool;
  double *Y = pool;                      // written after the primitive loop, over the 2D integrals
  double *co = pool + C::SGY;            // recurrence coefficients of a primitive window
  double *kq = co + C::CO;               // per-quartet exchange blocks (rows a|b, columns c|d), !KLDS only
  double *geo = kq + (KLDS ? 0 : QB * C::KQ);
  int *qi = reinterpret_cast<int *>(geo + QB * 12);
  int *smax = qi + QB * 8;
  const Pair bra = A.pairs[bi];
  const int tid = threadIdx.x;
  const int nc = A.mnc[bra.mol];
  // density rows of a and of b from the shell panels: D[a, col] = Pa[col NA + a]
  const double *Pa = A.Dp + A.mbase[bra.mol] + (size_t)bra.ca * nc;
  const double *Pb = A.Dp + A.mbase[bra.mol] + (size_t)bra.cb * nc;
  double *Km = A.Kc + A.mbase[bra.mol];
  const int oa = bra.ca, ob = bra.cb;
  for (int k0 = 0; k0 < cnt; k0 += QB) {
    if (tid < QB) {
      const int k = k0 + tid;
      const bool valid = k < cnt;
      const int ki = kl[valid ? k : k0];
      team_fill<LA, LB, LC, LD>(tid, bra, A.pairs[ki], bi, ki, valid, qi, geo);
    }
    if constexpr (!KLDS)
      for (int t = tid; t < QB * C::KQ; t += blockDim.x) kq[t] = 0.0;
    __syncthreads();
    team2_eri<LA, LB, LC, LD>(A.pp, sG, co, Y, qi, geo, smax);
    // exchange: into the LDS rows of the bra (KLDS), else into the quartet's LDS block, which
    // is flushed once per quartet below (one global atomic per element instead of one per
    // contributing lane)
    auto kadd = [&](int q, int r, int grow, int lc, int gcol, double v) {
      if constexpr (KLDS)
        k_update<true>(Krow, Km, nc, nc, r, grow, gcol, gcol, v);
      else
        atomicAdd(&kq[q * C::KQ + r * (NC + ND) + lc], v);
    };
    for (int t = tid; t < QB * NC * ND; t += blockDim.x) {
      const int q = t / (NC * ND), cd = t % (NC * ND);
      if (!qi[q * 8 + 6]) continue;
      const int ki = qi[q * 8 + 1];
      const Pair &ket = A.pairs[ki];
      const double s = sym_factor(bra, ket, bi, ki);
      double g[NA * NB];
      team2_ket<LA, LB, LC, LD>(Y, geo, q, cd, g);
      const int c = cd / ND, d = cd % ND;
      const int cc = ket.ca + c, dd = ket.cb + d;
      if (A.want & 1) {
        const double dcd = dp_elem(A, ck, ki, cd);
        double vj = 0.0;
#pragma unroll
        for (int ab = 0; ab < NA * NB; ++ab) {
          jab[ab] = fma(2.0 * s * dcd, g[ab], jab[ab]);
          vj = fma(g[ab], Pa[(size_t)(ob + ab % NB) * NA + ab / NB], vj);
        }
        atomic_add(jp_elem(A, ck, ki, cd), 2.0 * s * vj);
      }
      if (!(A.want & 2)) continue;
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        double kc = 0.0, kd = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          kc = fma(g[a * NB + b], Pb[(size_t)dd * NB + b], kc);
          kd = fma(g[a * NB + b], Pb[(size_t)cc * NB + b], kd);
        }
        kadd(q, a, oa + a, c, cc, s * kc);
        kadd(q, a, oa + a, NC + d, dd, s * kd);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        double kc = 0.0, kd = 0.0;
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          kc = fma(g[a * NB + b], Pa[(size_t)dd * NA + a], kc);
          kd = fma(g[a * NB + b], Pa[(size_t)cc * NA + a], kd);
        }
        kadd(q, NA + b, ob + b, c, cc, s * kc);
        kadd(q, NA + b, ob + b, NC + d, dd, s * kd);
      }
    }
    __syncthreads();
    if constexpr (!KLDS) {
      for (int t = tid; t < QB * C::KQ; t += blockDim.x) {
        const int q = t / C::KQ, r = (t % C::KQ) / (NC + ND), lc = t % (NC + ND);
        const double v = kq[t];
        if (!qi[q * 8 + 6] || v == 0.0) continue;
        const Pair &ket = A.pairs[qi[q * 8 + 1]];
        const int row = r < NA ? oa + r : ob + (r - NA);
        const int col = lc < NC ? ket.ca + lc : ket.cb + (lc - NC);
        atomic_add(&Km[(size_t)row * nc + col], v);
      }
      __syncthreads();
    }
  }
}

template <int LA, int LB, int LC, int LD>
constexpr bool use_team2() { return use_team<LA, LB, LC, LD>() && Team2Cfg<LA, LB, LC, LD>::OK; }

template <int LA, int LB, int LC, int LD>
constexpr int team_lds_bytes() {
  if constexpr (!use_team<LA, LB, LC, LD>()) return 0;
  else if constexpr (use_team2<LA, LB, LC, LD>()) return Team2Cfg<LA, LB, LC, LD>::LDS_BYTES;
  else return TeamCfg<LA, LB, LC, LD>::LDS_BYTES;
}

template <int LA, int LB, int LC, int LD>
constexpr int team_block() {
  if constexpr (use_team<LA, LB, LC, LD>() && !use_team2<LA, LB, LC, LD>()) return TeamCfg<LA, LB, LC, LD>::BLOCK;
  else return 256;
}

// R = float selects the FP32 lane body; the team bodies always evaluate in double.
template <int LA, int LB, int LC, int LD, bool KLDS, typename R = double>
__device__ __forceinline__ void jk_body(const JKArgs &A, int bi, const int *kl, int cnt, double *Krow, double *jab_s,
                                        double *pool, double (&jab)[ncart(LA) * ncart(LB)], int rot = 0) {
  if constexpr (use_team2<LA, LB, LC, LD>())
    jk_team2_body<LA, LB, LC, LD, KLDS>(A, bi, kl, cnt, Krow, pool, jab);
  else if constexpr (use_team<LA, LB, LC, LD>())
    jk_team_body<LA, LB, LC, LD, KLDS>(A, bi, kl, cnt, Krow, jab_s, pool);
  else
    jk_small_body<LA, LB, LC, LD, KLDS, R>(A, bi, kl, cnt, Krow, jab, rot);
}

// adds the per-lane bra Coulomb partials into jab_s (LDS), one wave-reduced value per wave
template <int NAB>
__device__ __forceinline__ void jab_reduce(double (&jab)[NAB], double *jab_s) {
#pragma unroll
  for (int e = 0; e < NAB; ++e) {
    double v = jab[e];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0 && v != 0.0) atomicAdd(&jab_s[e], v);
  }
}

template <int LA, int LB, int TIER, int P, typename R = double>
__device__ __forceinline__ void ket_dispatch(int ck, const JKArgs &A, int bi, const int *kl, int cnt, double *Krow,
                                             double *jab_s, double *pool, double (&jab)[ncart(LA) * ncart(LB)], int rot) {
  if constexpr (P <= pair_class(LA, LB)) {
    if constexpr (tier_of<LA, LB, pc_la(P), pc_lb(P)>() == TIER) {
      if (ck == P) {
        jk_body<LA, LB, pc_la(P), pc_lb(P), true, R>(A, bi, kl, cnt, Krow, jab_s, pool, jab, rot);
        return;
      }
    }
    ket_dispatch<LA, LB, TIER, P + 1, R>(ck, A, bi, kl, cnt, Krow, jab_s, pool, jab, rot);
  }
}

// Ket classes of a bra class that belong to a tier (bit P set for ket class P).
template <int LA, int LB, int TIER, int P = 0>
constexpr int tier_mask() {
  if constexpr (P > pair_class(LA, LB)) return 0;
  else return ((tier_of<LA, LB, pc_la(P), pc_lb(P)>() == TIER) ? (1 << P) : 0) | tier_mask<LA, LB, TIER, P + 1>();
}

// Largest team LDS over the ket classes of a tier (pool of k_bra), in bytes.
template <int LA, int LB, int TIER, int P = 0>
constexpr int bra_pool_bytes() {
  if constexpr (P > pair_class(LA, LB)) {
    return 0;
  } else {
    constexpr bool mine = tier_of<LA, LB, pc_la(P), pc_lb(P)>() == TIER;
    constexpr int here = mine ? team_lds_bytes<LA, LB, pc_la(P), pc_lb(P)>() : 0;
    constexpr int rest = bra_pool_bytes<LA, LB, TIER, P + 1>();
    return here > rest ? here : rest;
  }
}

// True when every team body of the tier runs with 256 lanes (k_bra's block).
template <int LA, int LB, int TIER, int P = 0>
constexpr bool bra_fusable() {
  if constexpr (P > pair_class(LA, LB)) {
    return true;
  } else {
    constexpr bool mine = tier_of<LA, LB, pc_la(P), pc_lb(P)>() == TIER;
    constexpr bool ok = !mine || team_block<LA, LB, pc_la(P), pc_lb(P)>() == 256;
    return ok && bra_fusable<LA, LB, TIER, P + 1>();
  }
}

// Largest global team buffer (doubles per workgroup) over the ket classes of a tier.
template <int LA, int LB, int TIER, int P = 0>
constexpr long long bra_scratch_doubles() {
  if constexpr (P > pair_class(LA, LB)) {
    return 0;
  } else {
    using C = TeamCfg<LA, LB, pc_la(P), pc_lb(P)>;
    constexpr bool mine = tier_of<LA, LB, pc_la(P), pc_lb(P)>() == TIER && use_team<LA, LB, pc_la(P), pc_lb(P)>() &&
                          !use_team2<LA, LB, pc_la(P), pc_lb(P)>();
    constexpr long long here = (mine && C::GLOBAL_BUF) ? C::BUF : 0;
    constexpr long long rest = bra_scratch_doubles<LA, LB, TIER, P + 1>();
    return here > rest ? here : rest;
  }
}

// ------------------------------------------------------------------ fused kernel: one bra pair, every ket class
// Dynamic LDS: Krow (NA+NB) x nc | jab_s NA*NB (padded to even) | team pool.
// F32: the FP32-only variant (lane tiers of mixed precision): it holds only the FP32 bodies,
// so its register budget, and hence its occupancy, is set by them alone.
template <int LA, int LB, int TIER, bool F32 = false>
__global__ __launch_bounds__(256) void k_bra(JKArgs A) {
  constexpr int NA = ncart(LA), NB = ncart(LB), cb = pair_class(LA, LB);
  extern __shared__ double smem[];
  __shared__ int s_unit;
  double *Krow = smem;
  double *jab_s = smem + (size_t)(NA + NB) * A.nc_max;
  double *pool = jab_s + ((NA * NB + 1) & ~1);
  const int nunits = min(*A.nunits, A.units_cap);
  const int tid = threadIdx.x;
  // the rows start at zero; the flush of each unit puts back the zeros it reads
  for (int t = tid; t < (NA + NB) * A.nc_max; t += blockDim.x) Krow[t] = 0.0;
  for (;;) {
    if (tid == 0) s_unit = atomicAdd(A.next, 1);
    for (int t = tid; t < NA * NB; t += blockDim.x) jab_s[t] = 0.0;
    __syncthreads();
    const int u = s_unit;
    if (u >= nunits) break;
    const int2 unit = A.units[u];
    const int bi = unit.x;
    const long long lo = (long long)unit.y * A.slice, hi = lo + A.slice;
    long long pos = 0;          // position of the current part in the bra's kets of this launch
    const int mol = A.pairs[bi].mol;
    const int nc = A.mnc[mol];
    double *Km = A.Kc + A.mbase[mol];
    double jab[NA * NB];
#pragma unroll
    for (int e = 0; e < NA * NB; ++e) jab[e] = 0.0;
    constexpr int mask = tier_mask<LA, LB, TIER>();
    for (int ck = 0; ck <= cb && pos < hi; ++ck) {
      if (!((mask >> ck) & 1)) continue;
      const size_t sg = (size_t)bi * NPAIRCLASS + ck;
      const int *cls_kets = A.kets + A.class_off[qclass_index(cb, ck)];
      for (int part = 0; part < 2; ++part) {   // FP64 part, then FP32 part of the segment
        if (!((A.parts >> part) & 1)) continue; // parts this launch runs
        const int n = part ? (A.segcnt32 ? A.segcnt32[sg] : 0) : A.segcnt[sg];
        const long long b0 = lo > pos ? lo : pos, b1 = hi < pos + n ? hi : pos + n;
        if (b1 > b0) {
          const int *kl = cls_kets + (part ? A.segoff32[sg] : A.segoff[sg]) + (b0 - pos);
          const int rot = (int)((b0 - lo) % blockDim.x);
          if constexpr (F32)
            ket_dispatch<LA, LB, TIER, 0, float>(ck, A, bi, kl, (int)(b1 - b0), Krow, jab_s, pool, jab, rot);
          else if constexpr (TIER == TEAM_TIER || !JK_FP32_BODIES)   // team bodies evaluate the FP32 part in double
            ket_dispatch<LA, LB, TIER, 0>(ck, A, bi, kl, (int)(b1 - b0), Krow, jab_s, pool, jab, rot);
          else if (part == 0)
            ket_dispatch<LA, LB, TIER, 0>(ck, A, bi, kl, (int)(b1 - b0), Krow, jab_s, pool, jab, rot);
          else
            ket_dispatch<LA, LB, TIER, 0, float>(ck, A, bi, kl, (int)(b1 - b0), Krow, jab_s, pool, jab, rot);
        }
        pos += n;
      }
    }
    jab_reduce<NA * NB>(jab, jab_s);
    __syncthreads();
    const Pair &bra = A.pairs[bi];
    for (int t = tid; t < (NA + NB) * nc; t += blockDim.x) {
      const double v = Krow[t];
      if (v != 0.0) {
        Krow[t] = 0.0;
        const int r = t / nc, col = t % nc;
        const int row = r < NA ? bra.ca + r : bra.cb + (r - NA);
        atomic_add(&Km[(size_t)row * nc + col], v);
      }
    }
    for (int t = tid; t < NA * NB; t += blockDim.x)
      if (jab_s[t] != 0.0) atomic_add(jp_elem(A, cb, bi, t), jab_s[t]);
    __syncthreads();
  }
}

// ------------------------------------------------------------------ per-class kernel (exchange to global memory)
template <int LA, int LB, int LC, int LD>
constexpr int cls_block() { return team_block<LA, LB, LC, LD>(); }

// Threads of a k_cls workgroup. With LDS exchange rows (KL != 0) one workgroup often fills most
// of a CU's LDS, so a light lane body (register tier 0 and total angular momentum at most 3:
// these fit 256 registers) carries JK_CLS_LDS_BLOCK threads (two waves per SIMD at 512) to
// keep more waves in flight than a 256-lane workgroup would. Heavier bodies keep 256 lanes:
// at two waves per SIMD they spill.
#ifndef JK_CLS_LDS_BLOCK
#define JK_CLS_LDS_BLOCK 512
#endif
// Root tables in LDS for the lane bodies of k_cls with LDS rows of up to this many roots
// (where they fit): the Boys grid for one and two roots (38.5 KB; 10 or 12 doubles per lookup
// from a different row per lane). The three-root block of the interpolation table (32.3 KB, 72
// doubles per lookup in runs of 24) measured slower from LDS than from the caches.
#ifndef JK_TABLE_LDS_NMAX
#define JK_TABLE_LDS_NMAX 2
#endif
template <int LA, int LB, int LC, int LD, int KL>
constexpr int cls_threads() {
  return KL != 0 && tier_of<LA, LB, LC, LD>() == 0 && LA + LB + LC + LD <= 3 ? JK_CLS_LDS_BLOCK
                                                                              : cls_block<LA, LB, LC, LD>();
}

// Waves per SIMD a per-class kernel is compiled for (0: the compiler's choice).
// - The (ps|ss) lane body with LDS rows takes 129 vector registers by default (three waves per
//   SIMD); held to 128 it runs four waves without spilling. (The other light bodies spill when
//   held to their next step, and run slower.)
// - Workgroup-body classes whose registers exceed 256 by a few accumulation registers (or, for
//   (gg|gd), (gp|dd), (gp|fd), (gp|ff), (fd|dp), by more) run one 256-lane workgroup per CU
//   although their LDS was sized for two; held to two waves per SIMD they spill a little and run
//   two. Listed by measurement: (gp|dp), (gp|gs), (gp|gp), (gp|fs), (gp|fp) and the (fd|**)
//   classes other than (fd|dp) ran slower that way and are left out.
template <int LA, int LB, int LC, int LD, int KL>
constexpr int cls_waves() {
  constexpr int k = ((LA * 5 + LB) * 5 + LC) * 5 + LD;
  constexpr int two[] = {
      ((3 * 5 + 1) * 5 + 1) * 5 + 1, ((3 * 5 + 1) * 5 + 2) * 5 + 0, ((3 * 5 + 1) * 5 + 2) * 5 + 1,
      ((3 * 5 + 1) * 5 + 2) * 5 + 2, ((3 * 5 + 1) * 5 + 3) * 5 + 0, ((3 * 5 + 1) * 5 + 3) * 5 + 1,
      ((3 * 5 + 3) * 5 + 3) * 5 + 2, ((4 * 5 + 1) * 5 + 2) * 5 + 2, ((4 * 5 + 2) * 5 + 3) * 5 + 2,
      ((4 * 5 + 3) * 5 + 3) * 5 + 2, ((4 * 5 + 4) * 5 + 2) * 5 + 2, ((4 * 5 + 4) * 5 + 3) * 5 + 1,
      ((4 * 5 + 4) * 5 + 3) * 5 + 2, ((4 * 5 + 4) * 5 + 4) * 5 + 1, ((4 * 5 + 4) * 5 + 4) * 5 + 2,
      ((2 * 5 + 0) * 5 + 2) * 5 + 0, ((4 * 5 + 1) * 5 + 3) * 5 + 2, ((4 * 5 + 1) * 5 + 3) * 5 + 3,
      ((3 * 5 + 2) * 5 + 2) * 5 + 1};
  if constexpr (KL == 0) {
    for (int t : two)
      if (t == k) return 2;
    return 0;
  } else {
    return LA == 1 && LB == 0 && LC == 0 && LD == 0 ? 4 : 0;
  }
}

// Dynamic LDS: jab_s NA*NB (padded to even) | team pool (team classes) or, with KL (lane
// bodies), the unit's exchange rows compacted to the columns of the ket class's momenta
// (KL = 1: rows K[a,:] and K[b,:], (NA+NB) x A.kw; KL = 2: rows K[a,:] only, NA x A.kw, the
// rows of b updated in global memory), flushed once per unit with one global atomic per
// nonzero element.
template <int LA, int LB, int LC, int LD, int KL = 0, bool GL = false>
__global__ __launch_bounds__((cls_threads<LA, LB, LC, LD, KL>()))
__attribute__((amdgpu_waves_per_eu(cls_waves<LA, LB, LC, LD, KL>() ? cls_waves<LA, LB, LC, LD, KL>() : 1)))
void k_cls(JKArgs A) {
  constexpr int NA = ncart(LA), NB = ncart(LB), cb = pair_class(LA, LB), ck = pair_class(LC, LD);
  static_assert(!KL || !use_team<LA, LB, LC, LD>(), "compacted LDS rows are for the lane bodies");
  static_assert(!GL || (KL && SmallCfg<LA, LB, LC, LD>::N <= JK_TABLE_LDS_NMAX), "LDS root tables: lane bodies");
  constexpr int RL = KL == 1 ? NA + NB : NA;    // full exchange rows held in LDS
  extern __shared__ double smem[];
  __shared__ int s_unit;
  double *jab_s = smem;
  double *pool = smem + ((NA * NB + 1) & ~1);
  double *Krow = pool;
  const int nunits = min(*A.nunits, A.units_cap);
  const int tid = threadIdx.x;
  if constexpr (KL != 0)   // the rows start at zero; each unit's flush puts back the zeros it reads
    for (int t = tid; t < RL * A.kw + (KL == 2 ? NB * A.kwb : 0); t += blockDim.x) Krow[t] = 0.0;
  // GL: the table the roots read (the Boys grid for one and two roots, else the N-root block of
  // the interpolation table) copied to LDS after the rows, so that its per-lane lookups (a
  // different row for nearly every lane) are LDS reads rather than vector-memory gathers
  // (visible after the loop's first barrier)
  const double *table = nullptr;
  if constexpr (GL) {
    constexpr int N = SmallCfg<LA, LB, LC, LD>::N;
    double *ts = Krow + RL * A.kw + (KL == 2 ? NB * A.kwb : 0);
    const double *src = root_table<N>();
    for (int t = tid; t < root_table_doubles<N>(); t += blockDim.x) ts[t] = src[t];
    table = ts;
  }
  for (;;) {
    if (tid == 0) s_unit = atomicAdd(A.next, 1);
    for (int t = tid; t < NA * NB; t += blockDim.x) jab_s[t] = 0.0;
    __syncthreads();
    const int u = s_unit;
    if (u >= nunits) break;
    const int2 unit = A.units[u];
    const int bi = unit.x;
    const size_t sg = (size_t)bi * NPAIRCLASS + ck;
    // this unit's kets: positions [lo, hi) of the segment's FP64 part [0, n64) followed by
    // its FP32 part [n64, n64 + n32)
    const long long n64 = A.segcnt[sg], n32 = A.segcnt32 ? A.segcnt32[sg] : 0;
    const long long lo = (long long)unit.y * A.slice, hi = lo + A.slice;
    const long long s64 = min(lo, n64), e64 = min(hi, n64);
    const long long s32 = max(lo, n64) - n64, e32 = max(min(hi, n64 + n32), n64) - n64;
    const int cnt = (int)(e64 - s64), cnt32 = (int)max(e32 - s32, 0ll);
    if (cnt + cnt32 > 0) {
      const int *cls_kets = A.kets + A.class_off[qclass_index(cb, ck)] + s64;   // + segoff: FP64 kets of the unit
      const int *cls_kets32 = A.kets + A.class_off[qclass_index(cb, ck)] + s32; // + segoff32: FP32 kets
      if constexpr (use_team<LA, LB, LC, LD>() && !use_team2<LA, LB, LC, LD>()) {
        for (int part = 0; part < 2; ++part) {   // FP32 part in double as well
          const int n = part ? cnt32 : cnt;
          if (n) jk_team_body<LA, LB, LC, LD, false>(A, bi, (part ? cls_kets32 + A.segoff32[sg] : cls_kets + A.segoff[sg]), n,
                                                     nullptr, jab_s, pool);
        }
      } else if constexpr (use_team2<LA, LB, LC, LD>()) {
        double jab[NA * NB];
#pragma unroll
        for (int e = 0; e < NA * NB; ++e) jab[e] = 0.0;
        for (int part = 0; part < 2; ++part) {
          const int n = part ? cnt32 : cnt;
          if (n) jk_body<LA, LB, LC, LD, false>(A, bi, (part ? cls_kets32 + A.segoff32[sg] : cls_kets + A.segoff[sg]), n, nullptr,
                                                jab_s, pool, jab);
        }
        jab_reduce<NA * NB>(jab, jab_s);
      } else if constexpr (KL != 0) {
        const Pair &bra = A.pairs[bi];
        const int m = bra.mol;
        const int *lseg = A.lseg + m * 6;
        const int ncl = lseg[LC + 1] - lseg[LC];
        const int kw = ncl + (LC != LD ? lseg[LD + 1] - lseg[LD] : 0);   // this molecule's row length
        const int kdofs = LC != LD ? ncl : 0;
        double jab[NA * NB];
#pragma unroll
        for (int e = 0; e < NA * NB; ++e) jab[e] = 0.0;
        if (cnt)
          jk_small_body<LA, LB, LC, LD, true, double, true, KL == 1>(A, bi, cls_kets + A.segoff[sg], cnt, Krow, jab, 0,
                                                                     kdofs, kw, table);
        if (cnt32)
          jk_small_body<LA, LB, LC, LD, true, float, true, KL == 1>(A, bi, cls_kets32 + A.segoff32[sg], cnt32, Krow,
                                                                    jab, 0, kdofs, kw, table);
        jab_reduce<NA * NB>(jab, jab_s);
        __syncthreads();
        const int nc = A.mnc[m];
        double *Km = A.Kc + A.mbase[m];
        const int *cols = A.lcols + A.cbase[m];
        for (int t = tid; t < RL * kw; t += blockDim.x) {
          const double v = Krow[t];
          if (v != 0.0) {
            Krow[t] = 0.0;
            const int r = t / kw, j = t % kw;
            const int col = cols[j < ncl ? lseg[LC] + j : lseg[LD] + (j - ncl)];
            const int row = r < NA ? bra.ca + r : bra.cb + (r - NA);
            atomic_add(&Km[(size_t)row * nc + col], v);
          }
        }
        if constexpr (KL == 2) {    // the LDS part of the rows of b (row length A.kwb)
          const int kwb = A.kwb < kw ? A.kwb : kw;
          double *Kb = Krow + (size_t)NA * A.kw;
          for (int t = tid; t < NB * kwb; t += blockDim.x) {
            const int r = t / kwb, j = t % kwb;
            const double v = Kb[r * A.kwb + j];
            if (v != 0.0) {
              Kb[r * A.kwb + j] = 0.0;
              const int col = cols[j < ncl ? lseg[LC] + j : lseg[LD] + (j - ncl)];
              atomic_add(&Km[(size_t)(bra.cb + r) * nc + col], v);
            }
          }
        }
      } else {
        double jab[NA * NB];
#pragma unroll
        for (int e = 0; e < NA * NB; ++e) jab[e] = 0.0;
        if (cnt) jk_body<LA, LB, LC, LD, false>(A, bi, cls_kets + A.segoff[sg], cnt, nullptr, jab_s, pool, jab);
        if (cnt32)
          jk_body<LA, LB, LC, LD, false, float>(A, bi, cls_kets32 + A.segoff32[sg], cnt32, nullptr, jab_s, pool, jab);
        jab_reduce<NA * NB>(jab, jab_s);
      }
      __syncthreads();
      for (int t = tid; t < NA * NB; t += blockDim.x)
        if (jab_s[t] != 0.0) atomic_add(jp_elem(A, cb, bi, t), jab_s[t]);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ Schwarz / ERI-tensor kernels (flat lists)
struct ModeArgs {
  const Pair *pairs;
  const PrimPair *pp;
  const int2 *quartets;
  int count;
  double *out;             // MODE_SCHWARZ: max |(ab|ab)| per pair (as bits); MODE_ERI: nc^4 tensor
  double *scratch;
  long long scratch_per_wg;
  int nc;
};

__device__ __forceinline__ void eri_store8(double *out, size_t nc, size_t i, size_t j, size_t k, size_t l, double v) {
  out[((i * nc + j) * nc + k) * nc + l] = v;
  out[((j * nc + i) * nc + k) * nc + l] = v;
  out[((i * nc + j) * nc + l) * nc + k] = v;
  out[((j * nc + i) * nc + l) * nc + k] = v;
  out[((k * nc + l) * nc + i) * nc + j] = v;
  out[((l * nc + k) * nc + i) * nc + j] = v;
  out[((k * nc + l) * nc + j) * nc + i] = v;
  out[((l * nc + k) * nc + j) * nc + i] = v;
}

// The ERI tensor of a one-stage class comes from the one-stage body (the body its J/K build
// runs), so that the tensor test checks that body element by element; its LDS is dynamic.
template <int LA, int LB, int LC, int LD, int MODE>
constexpr bool mode_team2() { return MODE == MODE_ERI && use_team2<LA, LB, LC, LD>(); }
template <int LA, int LB, int LC, int LD, int MODE>
constexpr int mode_lds() { return mode_team2<LA, LB, LC, LD, MODE>() ? Team2Cfg<LA, LB, LC, LD>::LDS_BYTES : 0; }

template <int LA, int LB, int LC, int LD, int MODE>
constexpr int mode_block() {
  return use_team<LA, LB, LC, LD>() && !mode_team2<LA, LB, LC, LD, MODE>() ? TeamCfg<LA, LB, LC, LD>::BLOCK : 256;
}

template <int LA, int LB, int LC, int LD, int MODE>
__global__ __launch_bounds__((mode_block<LA, LB, LC, LD, MODE>())) void k_mode(ModeArgs M) {
  constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
  if constexpr (mode_team2<LA, LB, LC, LD, MODE>()) {
    using C = Team2Cfg<LA, LB, LC, LD>;
    extern __shared__ double dyn[];
    double *sG = dyn;                    // 2D integrals, then Y (team2_eri)
    double *co = dyn + C::SGY;
    double *geo = co + C::CO;
    int *qi = reinterpret_cast<int *>(geo + C::QB * 12);
    int *smax = qi + C::QB * 8;
    const int nbatch = (M.count + C::QB - 1) / C::QB;
    for (int batch = blockIdx.x; batch < nbatch; batch += gridDim.x) {
      if (threadIdx.x < C::QB) {
        const int q = batch * C::QB + threadIdx.x;
        const bool valid = q < M.count;
        const int2 qd = M.quartets[valid ? q : batch * C::QB];
        team_fill<LA, LB, LC, LD>(threadIdx.x, M.pairs[qd.x], M.pairs[qd.y], qd.x, qd.y, valid, qi, geo);
      }
      __syncthreads();
      const double *Y = team2_eri<LA, LB, LC, LD>(M.pp, sG, co, sG, qi, geo, smax);
      for (int t = threadIdx.x; t < C::QB * NC * ND; t += blockDim.x) {
        const int q = t / (NC * ND), cd = t % (NC * ND);
        if (!qi[q * 8 + 6]) continue;
        double g[NA * NB];
        team2_ket<LA, LB, LC, LD>(Y, geo, q, cd, g);
        const Pair &bra = M.pairs[qi[q * 8]];
        const Pair &ket = M.pairs[qi[q * 8 + 1]];
        for (int ab = 0; ab < NA * NB; ++ab)
          eri_store8(M.out, M.nc, bra.ca + ab / NB, bra.cb + ab % NB, ket.ca + cd / ND, ket.cb + cd % ND, g[ab]);
      }
      __syncthreads();
    }
  } else if constexpr (use_team<LA, LB, LC, LD>()) {
    using C = TeamCfg<LA, LB, LC, LD>;
    __shared__ double sG[C::SG];
    __shared__ double sCo[C::CO];
    __shared__ double sBuf[C::GLOBAL_BUF ? 1 : C::BUF];
    __shared__ double geo[C::QB * 12];
    __shared__ int qi[C::QB * 8];
    __shared__ int smax;
    double *buf = C::GLOBAL_BUF ? M.scratch + (size_t)blockIdx.x * M.scratch_per_wg : sBuf;
    const int nbatch = (M.count + C::QB - 1) / C::QB;
    for (int batch = blockIdx.x; batch < nbatch; batch += gridDim.x) {
      if (threadIdx.x < C::QB) {
        const int q = batch * C::QB + threadIdx.x;
        const bool valid = q < M.count;
        const int2 qd = M.quartets[valid ? q : batch * C::QB];
        team_fill<LA, LB, LC, LD>(threadIdx.x, M.pairs[qd.x], M.pairs[qd.y], qd.x, qd.y, valid, qi, geo);
      }
      __syncthreads();
      const double *Z = team_eri<LA, LB, LC, LD>(M.pp, sG, sCo, buf, qi, geo, &smax);
      if constexpr (MODE == MODE_SCHWARZ && LA == LC && LB == LD) {
        for (int t = threadIdx.x; t < C::QB * NA * NB; t += blockDim.x) {
          const int q = t / (NA * NB), ab = t % (NA * NB);
          if (qi[q * 8 + 6]) atomic_max_nonneg(&M.out[qi[q * 8]], fabs(Z[((size_t)q * NA * NB + ab) * NC * ND + ab]));
        }
      } else if constexpr (MODE == MODE_ERI) {
        for (int t = threadIdx.x; t < C::QB * NA * NB * NC * ND; t += blockDim.x) {
          const int q = t / (NA * NB * NC * ND);
          if (!qi[q * 8 + 6]) continue;
          const int rem = t % (NA * NB * NC * ND);
          const int ab = rem / (NC * ND), cd = rem % (NC * ND);
          const Pair &bra = M.pairs[qi[q * 8]];
          const Pair &ket = M.pairs[qi[q * 8 + 1]];
          eri_store8(M.out, M.nc, bra.ca + ab / NB, bra.cb + ab % NB, ket.ca + cd / ND, ket.cb + cd % ND,
                     Z[(size_t)q * NA * NB * NC * ND + rem]);
        }
      }
      __syncthreads();
    }
  } else {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < M.count; q += gridDim.x * blockDim.x) {
      const int2 qd = M.quartets[q];
      const Pair bra = M.pairs[qd.x];
      const Pair ket = M.pairs[qd.y];
      double g[SmallCfg<LA, LB, LC, LD>::NG];
      small_eri<LA, LB, LC, LD>(bra, ket, M.pp, g);
      if constexpr (MODE == MODE_SCHWARZ && LA == LC && LB == LD) {
        double mx = 0.0;
#pragma unroll
        for (int ab = 0; ab < NA * NB; ++ab) mx = fmax(mx, fabs(g[ab * NC * ND + ab]));
        atomic_max_nonneg(&M.out[qd.x], mx);
      } else if constexpr (MODE == MODE_ERI) {
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
              for (int d = 0; d < ND; ++d)
                eri_store8(M.out, M.nc, bra.ca + a, bra.cb + b, ket.ca + c, ket.cb + d,
                           g[(a * NB + b) * NC * ND + c * ND + d]);
      }
    }
  }
}

}  // namespace jk
