// Contracted ERI blocks of one class, shared by every kernel of the build.
//
// Both bodies evaluate contracted shell quartets (ab|cd) of one class with la >= lb,
// lc >= ld, (la,lb) >= (lc,ld): the Rys product of paper section 2 is accumulated over
// primitive quartets at the [e0|f0] level (e = a + k on centre A, f = c + k' on centre C),
// then moved to (ab|cd) once per contracted quartet with the binomial transfer relation.
//
// small_eri: one lane per quartet, every intermediate in registers (the register-resident
//   design the paper uses for small classes, section 3, Algorithm 2).
// team_eri:  a workgroup per batch of QB quartets. For each chunk of primitive quartets the
//   lanes compute the 2D integrals of every (quartet, primitive quartet, root, direction)
//   into LDS; each lane then accumulates the [e0|f0] elements of one f component (and one
//   slice of e components) from LDS into registers. The transfer runs through a buffer in
//   LDS (or global memory for the largest classes) and leaves (ab|cd) in that buffer.
#pragma once
#include "jk_device.h"

// Accumulators per lane in the workgroup body (more: fewer lanes per quartet, smaller blocks,
// more registers per lane)
#ifndef JK_TEAM_EMAX
#define JK_TEAM_EMAX 48
#endif

// LDS budget (KB) and largest primitive chunk of the one-stage workgroup body
#ifndef JK_TEAM2_KB
#define JK_TEAM2_KB 64
#endif
#ifndef JK_TEAM2_VRR_PASSES
#define JK_TEAM2_VRR_PASSES 2   // passes of the block over the recurrence tasks of one chunk
#endif
#ifndef JK_TEAM2_NEMAX
#define JK_TEAM2_NEMAX 56     // largest [e0| component count of the one-stage body (0: not used)
#endif
#ifndef JK_TEAM2_PCMAX
#define JK_TEAM2_PCMAX 8
#endif
#ifndef JK_TEAM2_CO_KB
#define JK_TEAM2_CO_KB 24     // LDS (KB) of the one-stage body's coefficient window
#endif
// LDS per workgroup (bytes) under which two one-stage workgroups fit one CU (160 KB, less the
// bra Coulomb block and slack)
constexpr int TEAM2_PAIR_LDS = 78 * 1024;

// Rule for 1 and 2 roots in the lane bodies: 0 the interpolation table, 1 the closed form
// from erf/series Boys moments, 2 the closed form from Boys moments taken off a grid by Taylor
// series (fewest memory loads: 10 or 12 doubles per primitive quartet against 24 per root)
#ifndef JK_LOW_ROOTS
#define JK_LOW_ROOTS 2
#endif

namespace jk {

// Ket blocks of at least this many components use the streamed digestion in the workgroup body.
constexpr int TEAM_STREAM_MIN = 24;
// LDS per workgroup of the two-stage body that still fits twice per CU: the chunk of primitive
// quartets shrinks to stay under it, and the blocks X are kept in LDS under it
#ifndef JK_TEAM_XLDS_KB
#define JK_TEAM_XLDS_KB 78
#endif
constexpr int TEAM_XLDS_MAX = JK_TEAM_XLDS_KB * 1024;
#ifndef JK_TEAM_ZLDS
#define JK_TEAM_ZLDS 1
#endif

// ================================================================== lane per quartet
template <int LA, int LB, int LC, int LD>
struct SmallCfg {
  static constexpr int E = LA + LB, F = LC + LD, N = (E + F) / 2 + 1;
  static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
  static constexpr int NE = range_count(LA, E), NF = range_count(LC, F);
  static constexpr int REGS = NE * NF + 3 * (E + 1) * (F + 1);
  static constexpr int NG = NA * NB * NC * ND;
};

// R: type of the 2D integrals, their products and the transfer (double, or float for the
// FP32 quartets of mixed precision; roots, weights, the per-primitive scalars and the sum over
// primitive quartets and roots stay double).
// table: an LDS copy of root_table<N>() (the Boys grid of the one- and two-root rule, or the
// N-root block of the interpolation table), or null for the table itself.
template <int LA, int LB, int LC, int LD, typename R = double>
__device__ __forceinline__ void small_eri(const Pair &bra, const Pair &ket, const PrimPair *__restrict__ pp,
                                          R (&g)[SmallCfg<LA, LB, LC, LD>::NG], const double *table = nullptr) {
  using C = SmallCfg<LA, LB, LC, LD>;
  constexpr int E = C::E, F = C::F, N = C::N, NE = C::NE, NF = C::NF;
  constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND;
  constexpr int E0 = CT.start[LA], F0 = CT.start[LC];
  // the contraction over primitive quartets and roots is accumulated in double for both
  // types: an FP32 product is widened before it is added
  double acc[NE * NF];
#pragma unroll
  for (int i = 0; i < NE * NF; ++i) acc[i] = 0.0;
  const double *tab = table ? table : root_table<N>();

  // ket primitives outside: their loads differ from lane to lane, the bra's are the same for
  // every lane of the workgroup (one cache line per wave)
  for (int ik = 0; ik < ket.npp; ++ik) {
    const PrimPair pk = pp[ket.pp_off + ik];
    for (int ib = 0; ib < bra.npp; ++ib) {
      const PrimPair pb = pp[bra.pp_off + ib];
      const double hp = 0.5 * pb.ip;
      PrimQuartet Q;
      prim_quartet(pb, pk, bra.A, ket.A, Q);
      const double hq = 0.5 * pk.ip;
      auto root = [&](double un, double wn) {
        const double uq = un * Q.pq_inv;
        const R b00 = (R)(0.5 * uq);
        const R b10 = (R)(hp * (1.0 - uq * Q.q));
        const R b01 = (R)(hq * (1.0 - uq * Q.p));
        R Gx[E + 1][F + 1], Gy[E + 1][F + 1], Gz[E + 1][F + 1];
        vrr2d<E, F, R>(Gx, (R)1, (R)(Q.PA[0] - uq * Q.q * Q.PQ[0]), (R)(Q.QC[0] + uq * Q.p * Q.PQ[0]), b10, b01, b00);
        vrr2d<E, F, R>(Gy, (R)1, (R)(Q.PA[1] - uq * Q.q * Q.PQ[1]), (R)(Q.QC[1] + uq * Q.p * Q.PQ[1]), b10, b01, b00);
        vrr2d<E, F, R>(Gz, (R)(wn * Q.pref), (R)(Q.PA[2] - uq * Q.q * Q.PQ[2]), (R)(Q.QC[2] + uq * Q.p * Q.PQ[2]), b10,
                       b01, b00);
#pragma unroll
        for (int ie = 0; ie < NE; ++ie) {
#pragma unroll
          for (int jf = 0; jf < NF; ++jf) {
            const R gxy = Gx[CT.x[E0 + ie]][CT.x[F0 + jf]] * Gy[CT.y[E0 + ie]][CT.y[F0 + jf]];
            if constexpr (sizeof(R) == sizeof(double))
              acc[ie * NF + jf] = fma(gxy, Gz[CT.z[E0 + ie]][CT.z[F0 + jf]], acc[ie * NF + jf]);
            else
              acc[ie * NF + jf] += (double)(gxy * Gz[CT.z[E0 + ie]][CT.z[F0 + jf]]);
          }
        }
      };
      if constexpr (N <= 2 && JK_LOW_ROOTS != 0) {
        double u[N], w[N];
        if constexpr (JK_LOW_ROOTS == 1)
          rys_closed<N>(Q.T, u, w);
        else
          rys_low<N>(Q.T, u, w, tab);
#pragma unroll
        for (int n = 0; n < N; ++n) root(u[n], w[n]);
      } else {
#pragma unroll 1
        for (int n = 0; n < N; ++n) {
          double un, wn;
          rys_root1<N>(Q.T, n, un, wn, tab);
          root(un, wn);
        }
      }
    }
  }

  const R AB[3] = {(R)(bra.A[0] - bra.B[0]), (R)(bra.A[1] - bra.B[1]), (R)(bra.A[2] - bra.B[2])};
  const R CD[3] = {(R)(ket.A[0] - ket.B[0]), (R)(ket.A[1] - ket.B[1]), (R)(ket.A[2] - ket.B[2])};
  R abp[3][LB + 1], cdp[3][LD + 1];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    abp[d][0] = (R)1;
#pragma unroll
    for (int k = 1; k <= LB; ++k) abp[d][k] = abp[d][k - 1] * AB[d];
    cdp[d][0] = (R)1;
#pragma unroll
    for (int k = 1; k <= LD; ++k) cdp[d][k] = cdp[d][k - 1] * CD[d];
  }
  R hb[NA * NB * NF];
#pragma unroll
  for (int a = 0; a < NA; ++a) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      constexpr int A0 = CT.start[LA], B0 = CT.start[LB];
      const int ax = CT.x[A0 + a], ay = CT.y[A0 + a], az = CT.z[A0 + a];
      const int bx = CT.x[B0 + b], by = CT.y[B0 + b], bz = CT.z[B0 + b];
#pragma unroll
      for (int jf = 0; jf < NF; ++jf) hb[(a * NB + b) * NF + jf] = (R)0;
#pragma unroll
      for (int kx = 0; kx <= LB; ++kx) {
        if (kx > bx) continue;
#pragma unroll
        for (int ky = 0; ky <= LB; ++ky) {
          if (ky > by) continue;
#pragma unroll
          for (int kz = 0; kz <= LB; ++kz) {
            if (kz > bz) continue;
            const R cf = (R)(binom(bx, kx) * binom(by, ky) * binom(bz, kz)) * abp[0][bx - kx] *
                         abp[1][by - ky] * abp[2][bz - kz];
            const int ie = CT.idx[ax + kx][ay + ky][az + kz] - E0;
#pragma unroll
            for (int jf = 0; jf < NF; ++jf)
              hb[(a * NB + b) * NF + jf] = fma(cf, (R)acc[ie * NF + jf], hb[(a * NB + b) * NF + jf]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      constexpr int C0 = CT.start[LC], D0 = CT.start[LD];
      const int cx = CT.x[C0 + c], cy = CT.y[C0 + c], cz = CT.z[C0 + c];
      const int dx = CT.x[D0 + d], dy = CT.y[D0 + d], dz = CT.z[D0 + d];
#pragma unroll
      for (int ab = 0; ab < NA * NB; ++ab) g[ab * NC * ND + c * ND + d] = (R)0;
#pragma unroll
      for (int kx = 0; kx <= LD; ++kx) {
        if (kx > dx) continue;
#pragma unroll
        for (int ky = 0; ky <= LD; ++ky) {
          if (ky > dy) continue;
#pragma unroll
          for (int kz = 0; kz <= LD; ++kz) {
            if (kz > dz) continue;
            const R cf = (R)(binom(dx, kx) * binom(dy, ky) * binom(dz, kz)) * cdp[0][dx - kx] *
                         cdp[1][dy - ky] * cdp[2][dz - kz];
            const int jf = CT.idx[cx + kx][cy + ky][cz + kz] - F0;
#pragma unroll
            for (int ab = 0; ab < NA * NB; ++ab)
              g[ab * NC * ND + c * ND + d] = fma(cf, hb[ab * NF + jf], g[ab * NC * ND + c * ND + d]);
          }
        }
      }
    }
  }
}

// ================================================================== workgroup per batch
// The ten coefficients of one (quartet, primitive quartet, root) lie CO_STRIDE doubles apart:
// an odd stride, so that lanes reading consecutive sets fall on different LDS banks.
constexpr int CO_STRIDE = 11;
// Recurrence coefficients of the primitive quartets [w0, w0 + PW) of every quartet of a batch
// and every root, computed once per window (primitive pairs, Rys root and weight):
//   co[((q * PW + p) * N + n) * CO_STRIDE + k], k = b00, b10, b01, z weight x prefactor,
//   C00 (x, y, z), C00' (x, y, z).
template <int N, int QB, int PW>
__device__ __forceinline__ void prim_coefs(const PrimPair *__restrict__ pp, const int *qi, const double *geo, int w0,
                                           double *co) {
  for (int t = threadIdx.x; t < QB * PW * N; t += blockDim.x) {
    const int q = t / (PW * N), p = (t / N) % PW, n = t % N;
    const int pidx = w0 + p;
    const int nk = qi[q * 8 + 5];
    if (pidx >= qi[q * 8 + 3] * nk) continue;
    const PrimPair pb = pp[qi[q * 8 + 2] + pidx / nk];
    const PrimPair pk = pp[qi[q * 8 + 4] + pidx % nk];
    PrimQuartet Q;
    prim_quartet(pb, pk, &geo[q * 12], &geo[q * 12 + 6], Q);
    double u, w;
    rys_root1<N>(Q.T, n, u, w);
    const double uq = u * Q.pq_inv;
    double *c = co + (size_t)t * CO_STRIDE;
    c[0] = 0.5 * uq;
    c[1] = 0.5 * Q.ip * (1.0 - uq * Q.q);
    c[2] = 0.5 * Q.iq * (1.0 - uq * Q.p);
    c[3] = w * Q.pref;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      c[4 + d] = Q.PA[d] - uq * Q.q * Q.PQ[d];
      c[7 + d] = Q.QC[d] + uq * Q.p * Q.PQ[d];
    }
  }
}

// primitive quartets per coefficient window: a multiple of the chunk pc within `bytes` of LDS
constexpr int coef_window(int qb, int pc, int n, int bytes) {
  const int m = bytes / (qb * pc * n * CO_STRIDE * 8);
  return pc * (m < 1 ? 1 : m);
}

// Number of e slices per f component in the f-major product: the count (each slice at most
// emax accumulators) that keeps the largest share of a 256-lane block busy.
// Candidates whose accumulators and per-root 2D values (2 registers per double, plus ~48
// registers of other state) would not fit the register share of their block are skipped.
constexpr int team_slices(int ne, int nf, int emax, int e) {
  int best = (ne + emax - 1) / emax;
  double best_util = -1.0;
  for (int nep = 1; nep <= 8; ++nep) {
    const int eps = (ne + nep - 1) / nep;
    if (eps > emax) continue;
    const int fw = nep > 1 ? ((nf + 63) / 64) * 64 : nf;
    const int tpq = nep * fw;
    const int block = tpq > 256 ? ((tpq + 63) / 64) * 64 : 256;
    const int waves_per_simd = (block + 255) / 256;
    const int reg_cap = 512 / waves_per_simd > 256 && waves_per_simd > 1 ? 256 : 512 / waves_per_simd;
    if (2 * (eps + 3 * (e + 1)) + 48 > reg_cap) continue;
    const int qb = block / tpq;
    const double util = (double)(qb * nep * nf) / block;
    if (util > best_util + 1e-9) {
      best_util = util;
      best = nep;
    }
  }
  return best;
}

template <int LA, int LB, int LC, int LD>
struct TeamCfg {
  static constexpr int E = LA + LB, F = LC + LD, N = (E + F) / 2 + 1;
  static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
  static constexpr int NE = range_count(LA, E), NF = range_count(LC, F);
  static constexpr int GS1 = (E + 1) * (F + 1);          // one direction of one root
  // stride of one direction's table in LDS: odd, so that lanes writing or reading consecutive
  // tables fall on different LDS banks (an even stride such as 16 doubles puts 32 lanes on one bank)
  static constexpr int GT = GS1 | 1;
  static constexpr int GS = 3 * GT;
  static constexpr int EMAXACC = JK_TEAM_EMAX;           // accumulators per lane
  // Product roles. f-major: a lane owns one f component and a slice of EPS e components
  // (NEP slices per f, each slice wave-uniform). e-major (few f, many e): a lane owns one e
  // component and all NF f components, so that small ket classes keep the lanes busy.
  static constexpr bool EMAJOR = NF <= EMAXACC && NE > NF && NE <= 256;
  static constexpr int NEP = EMAJOR ? 1 : team_slices(NE, NF, EMAXACC, E);
  static constexpr int EPS = EMAJOR ? NF : (NE + NEP - 1) / NEP;   // accumulators per lane
  static constexpr int FW = EMAJOR ? 0 : (NEP > 1 ? ((NF + 63) / 64) * 64 : NF);
  static constexpr int TPQ = EMAJOR ? NE : NEP * FW;
  static constexpr int BLOCK = TPQ > 256 ? ((TPQ + 63) / 64) * 64 : 256;
  static constexpr int QB0 = BLOCK / TPQ;
  static constexpr int QBL = (40 * 1024) / (N * GS * 8);       // one primitive chunk of 2D integrals in 40 KB
  static constexpr int R1_ = (NE * NF > NA * NB * NC * ND) ? NE * NF : NA * NB * NC * ND;
  static constexpr int QBB = (48 * 1024) / ((R1_ + NA * NB * NF) * 8);   // transfer buffers in 48 KB of LDS
  static constexpr int QB1 = QB0 < QBL ? QB0 : QBL;
  // the transfer buffers limit QB only while they are meant to stay in LDS
  static constexpr bool BUF_LDS = QB1 * (R1_ + NA * NB * NF) * 8 <= 48 * 1024;
  static constexpr int QB2 = BUF_LDS ? QB1 : (QB1 < 4 ? QB1 : 4);
  static constexpr int QB = QB2 < 1 ? 1 : QB2;
  static constexpr int PC0 = (40 * 1024) / (QB * N * GS * 8);
  static constexpr int PC1 = BLOCK / (QB * N * 3);
  static constexpr int PC_MAX = (PC0 < PC1 ? PC0 : PC1) < 1 ? 1 : (PC0 < PC1 ? PC0 : PC1);
  static constexpr int XS = NE * NF, YS = NA * NB * NF, ZS = NA * NB * NC * ND;
  static constexpr int R1 = XS > ZS ? XS : ZS;
  static constexpr int BUF = QB * (R1 + YS);
  static constexpr bool GLOBAL_BUF = BUF * 8 > 48 * 1024;
  // LDS carved by team_eri: 2D integrals, (buffer), geometry; descriptors are ints
  // per-quartet digestion accumulators: K[a,c], K[a,d], K[b,c], K[b,d] and J[c,d]
  static constexpr int DG = NA * NC + NA * ND + NB * NC + NB * ND + NC * ND;
  // density blocks of the digestion: D[a,b], then per quartet D[c,d], D[a,c], D[a,d], D[b,c],
  // D[b,d] and the symmetry factor; they reuse the region of the 2D integrals and coefficients
  static constexpr int DQ = NC * ND + (NA + NB) * (NC + ND);
  static constexpr int DSTG = NA * NB + QB * (DQ + 1);
  // streamed digestion (ket blocks of TEAM_STREAM_MIN or more components): partial K[b,c] and
  // K[b,d] per (b, cd) after the density blocks
  static constexpr int PBD = NC * ND >= TEAM_STREAM_MIN ? 2 * QB * NB * NC * ND : 0;
  static constexpr int LDS_INTS = QB * 8 + 2;
  // primitive quartets per chunk: PC_MAX, or the largest of its halvings with which the
  // workgroup fits twice per CU (fewer quartets per synchronised chunk, more waves in flight)
  static constexpr int sgc_for(int pc) {
    const int sg = QB * pc * N * GS + QB * coef_window(QB, pc, N, 16 * 1024) * N * CO_STRIDE;
    return sg > DSTG + PBD ? sg : DSTG + PBD;
  }
  static constexpr int lds_for(int pc) {
    return (sgc_for(pc) + (GLOBAL_BUF ? 0 : BUF) + QB * DG + QB * 12) * 8 + LDS_INTS * 4;
  }
  static constexpr int pick_pc() {
    if (lds_for(PC_MAX) <= TEAM_XLDS_MAX) return PC_MAX;
    for (int pc = PC_MAX / 2; pc >= 1; pc /= 2)
      if (lds_for(pc) <= TEAM_XLDS_MAX) return pc;
    return PC_MAX;
  }
  static constexpr int PC = pick_pc();
  static constexpr int SG = QB * PC * N * GS;
  static constexpr int PW = coef_window(QB, PC, N, 16 * 1024);     // coefficient window (primitive quartets)
  static constexpr int CO = QB * PW * N * CO_STRIDE;
  static constexpr int SGC0 = SG + CO > DSTG + PBD ? SG + CO : DSTG + PBD;
  // global buffer: the blocks X go to the LDS region of the 2D integrals and coefficients (free
  // after the primitive loop; grown to hold them where the workgroup still fits twice per CU),
  // so only Y and Z pass through the buffer
  static constexpr int XSL = NE * (NF | 1);              // X in LDS: rows at an odd stride
  static constexpr int SGCX = SGC0 > QB * XSL ? SGC0 : QB * XSL;
  static constexpr bool X_LDS = GLOBAL_BUF && (SGCX + QB * DG + QB * 12) * 8 + LDS_INTS * 4 <= TEAM_XLDS_MAX;
  static constexpr int SGC1 = X_LDS ? SGCX : SGC0;
  // Z in LDS (global buffer, streamed digestion): during the digestion the region [DSTG + PBD,
  // SGC) is free; the ket transfer fills it with the rows (a, all b) of NAZ bra components a at a
  // time, which the streamed digestion then reads, so Z never passes through the global buffer.
  // NAZ is at least one component per wave; the region grows for it while the workgroup still
  // fits twice per CU.
  static constexpr int NWAVE = BLOCK / 64;
  static constexpr int NAZW = NA < NWAVE ? NA : NWAVE;
  static constexpr int ZNEED = DSTG + PBD + NAZW * NB * NC * ND;
  static constexpr int SGCZ = SGC1 > ZNEED ? SGC1 : ZNEED;
  static constexpr bool Z_LDS = JK_TEAM_ZLDS && GLOBAL_BUF && NC * ND >= TEAM_STREAM_MIN &&
                                (SGCZ + QB * DG + QB * 12) * 8 + LDS_INTS * 4 <= TEAM_XLDS_MAX;
  // small ket blocks (per-output digestion loops, each reading every integral): Z in LDS after
  // the staged densities, where the region (grown if need be) keeps as many workgroups per CU
  static constexpr int ZSNEED = DSTG + QB * ZS;
  static constexpr int SGCS = SGC1 > ZSNEED ? SGC1 : ZSNEED;
  static constexpr int lds_with(int sgc) { return (sgc + QB * DG + QB * 12) * 8 + LDS_INTS * 4; }
  static constexpr bool ZS_LDS = JK_TEAM_ZLDS && GLOBAL_BUF && NC * ND < TEAM_STREAM_MIN &&
                                 lds_with(SGCS) <= TEAM_XLDS_MAX &&   // and no fewer workgroups per CU
                                 (160 * 1024) / lds_with(SGCS) >= (160 * 1024) / lds_with(SGC1);
  static constexpr int SGC = Z_LDS ? SGCZ : (ZS_LDS ? SGCS : SGC1);
  static constexpr int NAZ0 = (SGC - DSTG - PBD) / (NB * NC * ND);
  static constexpr int NAZ = NAZ0 > NA ? NA : NAZ0;
  static constexpr int LDS_DOUBLES = SGC + (GLOBAL_BUF ? 0 : BUF) + QB * DG + QB * 12;
  static constexpr int LDS_BYTES = LDS_DOUBLES * 8 + LDS_INTS * 4;
};

// Batch descriptor in LDS, filled by the caller before team_eri:
//   qi[q*8 + 0..6] = bra pair, ket pair, bra pp_off, bra npp, ket pp_off, ket npp, valid
//   geo[q*12 + 0..11] = A, B (bra centres), C, D (ket centres)
template <int LA, int LB, int LC, int LD>
__device__ __forceinline__ void team_fill(int q, const Pair &b, const Pair &k, int bi, int ki, bool valid, int *qi,
                                          double *geo) {
  qi[q * 8 + 0] = bi; qi[q * 8 + 1] = ki;
  qi[q * 8 + 2] = b.pp_off; qi[q * 8 + 3] = valid ? b.npp : 0;
  qi[q * 8 + 4] = k.pp_off; qi[q * 8 + 5] = valid ? k.npp : 0;
  qi[q * 8 + 6] = valid;
  for (int d = 0; d < 3; ++d) {
    geo[q * 12 + d] = b.A[d]; geo[q * 12 + 3 + d] = b.B[d];
    geo[q * 12 + 6 + d] = k.A[d]; geo[q * 12 + 9 + d] = k.B[d];
  }
}

// Product of one e-slice for one lane: elements e in [P0*EPS, min(NE,(P0+1)*EPS)).
template <int LA, int LB, int LC, int LD, int P0>
__device__ __forceinline__ void team_product(const double *__restrict__ base, int xo, int yo, int zo,
                                             double (&acc)[TeamCfg<LA, LB, LC, LD>::EPS]) {
  using C = TeamCfg<LA, LB, LC, LD>;
  constexpr int E0 = CT.start[LA];
  constexpr int LO = P0 * C::EPS;
  constexpr int HI = (LO + C::EPS < C::NE) ? LO + C::EPS : C::NE;
  constexpr int EX = C::E;
  double gx[EX + 1], gy[EX + 1], gz[EX + 1];
#pragma unroll
  for (int e = 0; e <= EX; ++e) {
    gx[e] = base[xo + e * (C::F + 1)];
    gy[e] = base[yo + e * (C::F + 1)];
    gz[e] = base[zo + e * (C::F + 1)];
  }
#pragma unroll
  for (int i = LO; i < HI; ++i) acc[i - LO] = fma(gx[CT.x[E0 + i]] * gy[CT.y[E0 + i]], gz[CT.z[E0 + i]], acc[i - LO]);
}

template <int LA, int LB, int LC, int LD, int P0>
__device__ __forceinline__ void team_product_dispatch(int part, const double *base, int xo, int yo, int zo,
                                                      double (&acc)[TeamCfg<LA, LB, LC, LD>::EPS]) {
  if constexpr (P0 < TeamCfg<LA, LB, LC, LD>::NEP) {
    if (part == P0)
      team_product<LA, LB, LC, LD, P0>(base, xo, yo, zo, acc);
    else
      team_product_dispatch<LA, LB, LC, LD, P0 + 1>(part, base, xo, yo, zo, acc);
  }
}

// Computes (ab|cd) of the QB quartets described in qi/geo; on return Z[q*ZS + ab*NC*ND + cd]
// (Z = buf) holds the contracted Cartesian blocks. Every thread of the block must call it;
// it synchronises the block. sG: SG doubles of LDS; buf: BUF doubles (LDS or global).
// XL (TeamCfg::X_LDS, with sG the start of an LDS region of SGC doubles): the [e0|f0] blocks X
// go to that region, free after the primitive loop, instead of the global buffer.
// NOZ: return Y[(q*NA*NB + ab)*NF + f] after the bra transfer (the caller's team_ket_rows
// then forms Z block by block in LDS).
// zl: where the ket transfer writes Z (null: buf).
template <int LA, int LB, int LC, int LD, bool XL = false, bool NOZ = false>
__device__ __forceinline__ const double *team_eri(const PrimPair *__restrict__ pp, double *sG, double *co,
                                                  double *buf, const int *qi, const double *geo, int *smax,
                                                  double *zl = nullptr) {
  using C = TeamCfg<LA, LB, LC, LD>;
  constexpr int E = C::E, F = C::F, N = C::N, NE = C::NE, NF = C::NF;
  constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND;
  constexpr int QB = C::QB, PC = C::PC, GS = C::GS, GT = C::GT, BLOCK = C::BLOCK;
  constexpr int E0 = CT.start[LA], F0 = CT.start[LC];
  double *X = XL ? sG : buf;          // [QB][NE][XR]  (later Z: [QB][NA*NB][NC*ND], in buf)
  // row stride of X: odd in LDS, so that the lanes of the e-major product (one row each) store
  // to different banks (an even NF puts half the wave on one bank)
  constexpr int XR = XL ? (NF | 1) : NF;
  double *Y = buf + QB * C::R1;       // [QB][NA*NB][NF]
  const int tid = threadIdx.x;

  const int pq_ = tid / C::TPQ;
  const int pr = tid % C::TPQ;
  const int part = C::EMAJOR ? 0 : pr / (C::EMAJOR ? 1 : C::FW);
  const int pf = C::EMAJOR ? pr : pr % (C::EMAJOR ? 1 : C::FW);   // e-major: the lane's e component
  const bool prole = pq_ < QB && (C::EMAJOR || pf < NF);
  int xo = 0, yo = 0, zo = 0;
  if (prole) {
    if constexpr (C::EMAJOR) {                 // row e of each direction's table
      xo = CTD.x[E0 + pf] * (F + 1);
      yo = GT + CTD.y[E0 + pf] * (F + 1);
      zo = 2 * GT + CTD.z[E0 + pf] * (F + 1);
    } else {                                   // column f
      xo = CTD.x[F0 + pf];
      yo = GT + CTD.y[F0 + pf];
      zo = 2 * GT + CTD.z[F0 + pf];
    }
  }
  if (tid == 0) {
    int m = 0;
    for (int q = 0; q < QB; ++q) m = max(m, qi[q * 8 + 3] * qi[q * 8 + 5]);
    *smax = m;
  }
  __syncthreads();
  const int kmax = *smax;

  double acc[C::EPS];
#pragma unroll
  for (int i = 0; i < C::EPS; ++i) acc[i] = 0.0;

  constexpr int PW = C::PW;
  for (int w0 = 0; w0 < kmax; w0 += PW) {
  prim_coefs<N, QB, PW>(pp, qi, geo, w0, co);
  __syncthreads();
  const int wend = min(w0 + PW, kmax);
  for (int c0 = w0; c0 < wend; c0 += PC) {
    for (int t = tid; t < QB * PC * N * 3; t += BLOCK) {
      const int q = t / (PC * N * 3);
      const int rem = t % (PC * N * 3);
      const int pl = rem / (N * 3);
      const int n = (rem % (N * 3)) / 3;
      const int dir = rem % 3;
      const int pidx = c0 + pl;
      if (pidx < qi[q * 8 + 3] * qi[q * 8 + 5]) {
        const double *c = co + ((q * PW + (pidx - w0)) * N + n) * CO_STRIDE;
        double *dst = sG + ((q * PC + pl) * N + n) * GS + dir * GT;
        vrr2d_store<E, F>(dst, dir == 2 ? c[3] : 1.0, c[4 + dir], c[7 + dir], c[1], c[2], c[0]);
      }
    }
    __syncthreads();
    if (prole) {
      const int npl = min(PC, qi[pq_ * 8 + 3] * qi[pq_ * 8 + 5] - c0);
      for (int pl = 0; pl < npl; ++pl) {
#pragma unroll
        for (int n = 0; n < N; ++n) {
          const double *base = sG + ((pq_ * PC + pl) * N + n) * GS;
          if constexpr (C::EMAJOR) {
            double gx[F + 1], gy[F + 1], gz[F + 1];
#pragma unroll
            for (int f = 0; f <= F; ++f) {
              gx[f] = base[xo + f];
              gy[f] = base[yo + f];
              gz[f] = base[zo + f];
            }
#pragma unroll
            for (int j = 0; j < NF; ++j)
              acc[j] = fma(gx[CT.x[F0 + j]] * gy[CT.y[F0 + j]], gz[CT.z[F0 + j]], acc[j]);
          } else {
            team_product_dispatch<LA, LB, LC, LD, 0>(part, base, xo, yo, zo, acc);
          }
        }
      }
    }
    __syncthreads();
  }
  }

  if (prole) {
    if constexpr (C::EMAJOR) {
#pragma unroll
      for (int j = 0; j < NF; ++j) X[(pq_ * NE + pf) * XR + j] = acc[j];
    } else {
#pragma unroll
      for (int i = 0; i < C::EPS; ++i) {
        const int e = part * C::EPS + i;
        if (e < NE) X[(pq_ * NE + e) * XR + pf] = acc[i];
      }
    }
  }
  __syncthreads();
  // Bra transfer, one task per (quartet, a, f): the X[e][f] this a can reach (e = a + k,
  // |k| <= lb) are loaded together, then the NB outputs (a, b) are formed from registers.
  // Each lane runs TU tasks at once, their loads issued before any of them is used (the
  // buffer may be in global memory).
  constexpr int NKB = range_count(0, LB);       // components k with |k| <= lb
  constexpr int TUB = 3 * NKB <= 24 ? 3 : (2 * NKB <= 24 ? 2 : 1);
  for (int t0 = tid; t0 < QB * NA * NF; t0 += TUB * BLOCK) {
    double xv[TUB][NKB];
#pragma unroll
    for (int u = 0; u < TUB; ++u) {
      const int t = t0 + u * BLOCK;
      if (t >= QB * NA * NF) break;
      const int q = t / (NA * NF);
      const int rem = t % (NA * NF);
      const int a = rem / NF, f = rem % NF;
      const int ax = CTD.x[E0 + a], ay = CTD.y[E0 + a], az = CTD.z[E0 + a];
#pragma unroll
      for (int k = 0; k < NKB; ++k)
        xv[u][k] = X[(q * NE + cart_flat(ax + CT.x[k], ay + CT.y[k], az + CT.z[k]) - E0) * XR + f];
    }
#pragma unroll
    for (int u = 0; u < TUB; ++u) {
      const int t = t0 + u * BLOCK;
      if (t >= QB * NA * NF) break;
      const int q = t / (NA * NF);
      const int rem = t % (NA * NF);
      const int a = rem / NF, f = rem % NF;
      const double AB[3] = {geo[q * 12 + 0] - geo[q * 12 + 3], geo[q * 12 + 1] - geo[q * 12 + 4],
                            geo[q * 12 + 2] - geo[q * 12 + 5]};
      double pw[3][LB + 1];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        pw[d][0] = 1.0;
#pragma unroll
        for (int i = 1; i <= LB; ++i) pw[d][i] = pw[d][i - 1] * AB[d];
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        constexpr int B0 = CT.start[LB];
        const int bx = CT.x[B0 + b], by = CT.y[B0 + b], bz = CT.z[B0 + b];
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < NKB; ++k) {
          const int kx = CT.x[k], ky = CT.y[k], kz = CT.z[k];
          if (kx > bx || ky > by || kz > bz) continue;
          const double cf = (double)(binom(bx, kx) * binom(by, ky) * binom(bz, kz)) * pw[0][bx - kx] *
                            pw[1][by - ky] * pw[2][bz - kz];
          v = fma(cf, xv[u][k], v);
        }
        Y[(q * NA * NB + a * NB + b) * NF + f] = v;
      }
    }
  }
  __syncthreads();
  if constexpr (NOZ) return Y;
  // Ket transfer, one task per (quartet, ab, c): Y[ab][c + k] for |k| <= ld loaded together,
  // then the ND outputs (c, d); TU tasks per lane at once as above.
  constexpr int NKD = range_count(0, LD);
  constexpr int TUK = 3 * NKD <= 24 ? 3 : (2 * NKD <= 24 ? 2 : 1);
  double *Z = zl ? zl : buf;
  for (int t0 = tid; t0 < QB * NA * NB * NC; t0 += TUK * BLOCK) {
    double yv[TUK][NKD];
#pragma unroll
    for (int u = 0; u < TUK; ++u) {
      const int t = t0 + u * BLOCK;
      if (t >= QB * NA * NB * NC) break;
      const int q = t / (NA * NB * NC);
      const int rem = t % (NA * NB * NC);
      const int ab = rem / NC, c = rem % NC;
      const int cx = CTD.x[F0 + c], cy = CTD.y[F0 + c], cz = CTD.z[F0 + c];
#pragma unroll
      for (int k = 0; k < NKD; ++k)
        yv[u][k] = Y[(q * NA * NB + ab) * NF + cart_flat(cx + CT.x[k], cy + CT.y[k], cz + CT.z[k]) - F0];
    }
#pragma unroll
    for (int u = 0; u < TUK; ++u) {
      const int t = t0 + u * BLOCK;
      if (t >= QB * NA * NB * NC) break;
      const int q = t / (NA * NB * NC);
      const int rem = t % (NA * NB * NC);
      const int ab = rem / NC, c = rem % NC;
      const double CD[3] = {geo[q * 12 + 6] - geo[q * 12 + 9], geo[q * 12 + 7] - geo[q * 12 + 10],
                            geo[q * 12 + 8] - geo[q * 12 + 11]};
      double pw[3][LD + 1];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        pw[d][0] = 1.0;
#pragma unroll
        for (int i = 1; i <= LD; ++i) pw[d][i] = pw[d][i - 1] * CD[d];
      }
#pragma unroll
      for (int dd = 0; dd < ND; ++dd) {
        constexpr int D0 = CT.start[LD];
        const int dx = CT.x[D0 + dd], dy = CT.y[D0 + dd], dz = CT.z[D0 + dd];
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < NKD; ++k) {
          const int kx = CT.x[k], ky = CT.y[k], kz = CT.z[k];
          if (kx > dx || ky > dy || kz > dz) continue;
          const double cf = (double)(binom(dx, kx) * binom(dy, ky) * binom(dz, kz)) * pw[0][dx - kx] *
                            pw[1][dy - ky] * pw[2][dz - kz];
          v = fma(cf, yv[u][k], v);
        }
        Z[(q * NA * NB + ab) * NC * ND + c * ND + dd] = v;   // buf region 1: X was consumed above (or is in LDS)
      }
    }
  }
  __syncthreads();
  return Z;
}

// Ket transfer of the rows (a, b), a in [a0, a0 + na), every b, of quartet q: from Y (as
// team_eri<..., true> returns it) into zb[((a - a0) * NB + b) * NC * ND + c * ND + d]. Every
// thread of the block calls it; the caller synchronises before reading zb.
template <int LA, int LB, int LC, int LD>
__device__ __forceinline__ void team_ket_rows(const double *Y, const double *geo, int q, int a0, int na, double *zb) {
  using C = TeamCfg<LA, LB, LC, LD>;
  constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND, NF = C::NF;
  constexpr int F0 = CT.start[LC];
  constexpr int NKD = range_count(0, LD);
  constexpr int TUK = 3 * NKD <= 24 ? 3 : (2 * NKD <= 24 ? 2 : 1);
  const int ntask = na * NB * NC;
  const double CD[3] = {geo[q * 12 + 6] - geo[q * 12 + 9], geo[q * 12 + 7] - geo[q * 12 + 10],
                        geo[q * 12 + 8] - geo[q * 12 + 11]};
  double pw[3][LD + 1];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    pw[d][0] = 1.0;
#pragma unroll
    for (int i = 1; i <= LD; ++i) pw[d][i] = pw[d][i - 1] * CD[d];
  }
  const double *Yq = Y + ((size_t)q * NA + a0) * NB * NF;
  for (int t0 = threadIdx.x; t0 < ntask; t0 += TUK * blockDim.x) {
    double yv[TUK][NKD];
#pragma unroll
    for (int u = 0; u < TUK; ++u) {
      const int t = t0 + u * blockDim.x;
      if (t >= ntask) break;
      const int r = t / NC, c = t % NC;                 // r = (a - a0) * NB + b
      const int cx = CTD.x[F0 + c], cy = CTD.y[F0 + c], cz = CTD.z[F0 + c];
#pragma unroll
      for (int k = 0; k < NKD; ++k) yv[u][k] = Yq[(size_t)r * NF + cart_flat(cx + CT.x[k], cy + CT.y[k], cz + CT.z[k]) - F0];
    }
#pragma unroll
    for (int u = 0; u < TUK; ++u) {
      const int t = t0 + u * blockDim.x;
      if (t >= ntask) break;
      const int r = t / NC, c = t % NC;
#pragma unroll
      for (int dd = 0; dd < ND; ++dd) {
        constexpr int D0 = CT.start[LD];
        const int dx = CT.x[D0 + dd], dy = CT.y[D0 + dd], dz = CT.z[D0 + dd];
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < NKD; ++k) {
          const int kx = CT.x[k], ky = CT.y[k], kz = CT.z[k];
          if (kx > dx || ky > dy || kz > dz) continue;
          const double cf = (double)(binom(dx, kx) * binom(dy, ky) * binom(dz, kz)) * pw[0][dx - kx] *
                            pw[1][dy - ky] * pw[2][dz - kz];
          v = fma(cf, yv[u][k], v);
        }
        zb[(size_t)r * NC * ND + c * ND + dd] = v;
      }
    }
  }
}

}  // namespace jk

namespace jk {

// ================================================================== workgroup per batch, one LDS stage
// For classes whose e components fit in one lane (NE <= 56): lane (q, f) accumulates the
// [e0|f0] column of one f component for all e, applies the bra transfer in registers
// (compile-time indices) and stores (ab|f) in LDS; the ket transfer is then done per
// (quartet, cd) from LDS by the caller (team2_ket).
template <int LA, int LB, int LC, int LD>
struct Team2Cfg {
  static constexpr int E = LA + LB, F = LC + LD, N = (E + F) / 2 + 1;
  static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
  static constexpr int NE = range_count(LA, E), NF = range_count(LC, F);
  static constexpr int GS1 = (E + 1) * (F + 1);
  static constexpr int GT = GS1 | 1;
  static constexpr int GS = 3 * GT;
  static constexpr bool OK = NE <= JK_TEAM2_NEMAX && NF <= 256;
  static constexpr int YS = NA * NB * NF;
  static constexpr int YQ = YS | 1;                 // per-quartet stride of Y in LDS (odd: bank spread)
  static constexpr int QB0 = 256 / NF;
  // The 2D integrals of a primitive chunk and, once the primitive loop is done, the
  // bra-transferred Y share one LDS region of BUDGET doubles.
  static constexpr int BUDGET = JK_TEAM2_KB * 1024 / 8;
  static constexpr int QB1 = BUDGET / (YQ > N * GS ? YQ : N * GS);   // Y fits, and one primitive chunk
  static constexpr int QB = (QB0 < QB1 ? QB0 : QB1) < 1 ? 1 : (QB0 < QB1 ? QB0 : QB1);
  static constexpr int PCB = BUDGET / (QB * N * GS);
  static constexpr int PCT = JK_TEAM2_VRR_PASSES * 256 / (QB * N * 3);   // VRR items in so many passes of the block
  static constexpr int PC0 = PCB < PCT ? PCB : PCT;
  static constexpr int PC = PC0 < 1 ? 1 : (PC0 > JK_TEAM2_PCMAX ? JK_TEAM2_PCMAX : PC0);
  static constexpr int SG = QB * PC * N * GS;
  static constexpr int SGY = SG > QB * YQ ? SG : QB * YQ;       // the shared region
  static constexpr int KQ = (NA + NB) * (NC + ND);               // exchange block of one quartet
  static constexpr int LDS_INTS = QB * 8 + 2;
  // LDS of a workgroup whose exchange goes to global memory (per-quartet blocks) for a
  // coefficient window of pw primitive quartets
  static constexpr int bytes_for(int pw) { return (SGY + QB * pw * N * CO_STRIDE + QB * 12 + QB * KQ) * 8 + LDS_INTS * 4; }
  // Coefficient window (primitive quartets): JK_TEAM2_CO_KB of LDS, or half of it where that
  // lets two workgroups share a CU (fewer primitive quartets per window, more waves in flight)
  static constexpr int PW_FULL = coef_window(QB, PC, N, JK_TEAM2_CO_KB * 1024);
  static constexpr int PW_HALF = coef_window(QB, PC, N, JK_TEAM2_CO_KB * 512);
  static constexpr bool HALF_CO = bytes_for(PW_FULL) > TEAM2_PAIR_LDS && bytes_for(PW_HALF) <= TEAM2_PAIR_LDS;
  static constexpr int PW = HALF_CO ? PW_HALF : PW_FULL;
  static constexpr int CO = QB * PW * N * CO_STRIDE;
  static constexpr int LDS_DOUBLES = SGY + CO + QB * 12;         // + QB * KQ when K goes to global memory
  static constexpr int LDS_BYTES = LDS_DOUBLES * 8 + LDS_INTS * 4;
};

// Fills Y[q * YQ + ab * NF + f] = (ab|f0) of the QB quartets described in qi/geo (same layout as
// team_eri).
// Every thread of the block calls it; it synchronises the block. Returns Y.
template <int LA, int LB, int LC, int LD>
__device__ __forceinline__ const double *team2_eri(const PrimPair *__restrict__ pp, double *sG, double *co, double *Y,
                                                   const int *qi, const double *geo, int *smax) {
  using C = Team2Cfg<LA, LB, LC, LD>;
  constexpr int E = C::E, F = C::F, N = C::N, NE = C::NE, NF = C::NF;
  constexpr int NA = C::NA, NB = C::NB;
  constexpr int QB = C::QB, PC = C::PC, GS = C::GS, GT = C::GT;
  constexpr int E0 = CT.start[LA], F0 = CT.start[LC];
  const int tid = threadIdx.x;
  const int pq_ = tid / NF;
  const int pf = tid % NF;
  const bool prole = pq_ < QB;
  int xo = 0, yo = 0, zo = 0;
  if (prole) {
    xo = CTD.x[F0 + pf];
    yo = GT + CTD.y[F0 + pf];
    zo = 2 * GT + CTD.z[F0 + pf];
  }
  if (tid == 0) {
    int m = 0;
    for (int q = 0; q < QB; ++q) m = max(m, qi[q * 8 + 3] * qi[q * 8 + 5]);
    *smax = m;
  }
  __syncthreads();
  const int kmax = *smax;
  double acc[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) acc[i] = 0.0;
  constexpr int PW = C::PW;
  for (int w0 = 0; w0 < kmax; w0 += PW) {
  prim_coefs<N, QB, PW>(pp, qi, geo, w0, co);
  __syncthreads();
  const int wend = min(w0 + PW, kmax);
  for (int c0 = w0; c0 < wend; c0 += PC) {
    for (int t = tid; t < QB * PC * N * 3; t += blockDim.x) {
      const int q = t / (PC * N * 3);
      const int rem = t % (PC * N * 3);
      const int pl = rem / (N * 3);
      const int n = (rem % (N * 3)) / 3;
      const int dir = rem % 3;
      const int pidx = c0 + pl;
      if (pidx < qi[q * 8 + 3] * qi[q * 8 + 5]) {
        const double *c = co + ((q * PW + (pidx - w0)) * N + n) * CO_STRIDE;
        double *dst = sG + ((q * PC + pl) * N + n) * GS + dir * GT;
        vrr2d_store<E, F>(dst, dir == 2 ? c[3] : 1.0, c[4 + dir], c[7 + dir], c[1], c[2], c[0]);
      }
    }
    __syncthreads();
    if (prole) {
      const int npl = min(PC, qi[pq_ * 8 + 3] * qi[pq_ * 8 + 5] - c0);
      for (int pl = 0; pl < npl; ++pl) {
#pragma unroll
        for (int n = 0; n < N; ++n) {
          const double *base = sG + ((pq_ * PC + pl) * N + n) * GS;
          double gx[E + 1], gy[E + 1], gz[E + 1];
#pragma unroll
          for (int e = 0; e <= E; ++e) {
            gx[e] = base[xo + e * (F + 1)];
            gy[e] = base[yo + e * (F + 1)];
            gz[e] = base[zo + e * (F + 1)];
          }
#pragma unroll
          for (int i = 0; i < NE; ++i)
            acc[i] = fma(gx[CT.x[E0 + i]] * gy[CT.y[E0 + i]], gz[CT.z[E0 + i]], acc[i]);
        }
      }
    }
    __syncthreads();
  }
  }
  if (prole) {
    const double AB[3] = {geo[pq_ * 12 + 0] - geo[pq_ * 12 + 3], geo[pq_ * 12 + 1] - geo[pq_ * 12 + 4],
                          geo[pq_ * 12 + 2] - geo[pq_ * 12 + 5]};
    double abp[3][LB + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      abp[d][0] = 1.0;
#pragma unroll
      for (int k = 1; k <= LB; ++k) abp[d][k] = abp[d][k - 1] * AB[d];
    }
    constexpr int A0 = CT.start[LA], B0 = CT.start[LB];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int ax = CT.x[A0 + a], ay = CT.y[A0 + a], az = CT.z[A0 + a];
        const int bx = CT.x[B0 + b], by = CT.y[B0 + b], bz = CT.z[B0 + b];
        double v = 0.0;
#pragma unroll
        for (int kx = 0; kx <= LB; ++kx) {
          if (kx > bx) continue;
#pragma unroll
          for (int ky = 0; ky <= LB; ++ky) {
            if (ky > by) continue;
#pragma unroll
            for (int kz = 0; kz <= LB; ++kz) {
              if (kz > bz) continue;
              const double cf = (double)(binom(bx, kx) * binom(by, ky) * binom(bz, kz)) * abp[0][bx - kx] *
                                abp[1][by - ky] * abp[2][bz - kz];
              v = fma(cf, acc[CT.idx[ax + kx][ay + ky][az + kz] - E0], v);
            }
          }
        }
        Y[pq_ * C::YQ + (a * NB + b) * NF + pf] = v;
      }
    }
  }
  __syncthreads();
  return Y;
}

// (ab|cd) for one quartet q and one ket component pair cd, all ab, from Y (ket transfer).
template <int LA, int LB, int LC, int LD>
__device__ __forceinline__ void team2_ket(const double *Y, const double *geo, int q, int cd,
                                          double (&g)[ncart(LA) * ncart(LB)]) {
  using C = Team2Cfg<LA, LB, LC, LD>;
  constexpr int NA = C::NA, NB = C::NB, ND = C::ND, NF = C::NF;
  constexpr int F0 = CT.start[LC];
  const int c = cd / ND, d = cd % ND;
  const int cx = CTD.x[F0 + c], cy = CTD.y[F0 + c], cz = CTD.z[F0 + c];
  const int dx = CTD.x[CT.start[LD] + d], dy = CTD.y[CT.start[LD] + d], dz = CTD.z[CT.start[LD] + d];
  const double CDx = geo[q * 12 + 6] - geo[q * 12 + 9], CDy = geo[q * 12 + 7] - geo[q * 12 + 10],
               CDz = geo[q * 12 + 8] - geo[q * 12 + 11];
#pragma unroll
  for (int ab = 0; ab < NA * NB; ++ab) g[ab] = 0.0;
  const double *Yq = Y + (size_t)q * C::YQ;
  double px = 1.0;
  for (int kx = dx; kx >= 0; --kx) {
    double py = 1.0;
    for (int ky = dy; ky >= 0; --ky) {
      double pz = 1.0;
      for (int kz = dz; kz >= 0; --kz) {
        const double cf = (double)(binom(dx, kx) * binom(dy, ky) * binom(dz, kz)) * px * py * pz;
        const int jf = CTD.idx[cx + kx][cy + ky][cz + kz] - F0;
#pragma unroll
        for (int ab = 0; ab < NA * NB; ++ab) g[ab] = fma(cf, Yq[ab * NF + jf], g[ab]);
        pz *= CDz;
      }
      py *= CDy;
    }
    px *= CDx;
  }
}

}  // namespace jk
