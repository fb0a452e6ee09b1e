// Class kernels of the J/K build (templated on the angular momenta of the quartet).
//
// Both kernels evaluate contracted shell quartets (ab|cd) of one class with la >= lb,
// lc >= ld, (la,lb) >= (lc,ld), accumulate the primitive sum at the [e0|f0] level, move
// to (ab|cd) once per contracted quartet and then digest it with the density (paper
// section 3, the six updates of Algorithm 2 with the eight-fold symmetry factor s):
//   Jt[a,b] += 2s (ab|cd) D[c,d]    Jt[c,d] += 2s (ab|cd) D[a,b]
//   Kt[a,c] += s (ab|cd) D[b,d]     Kt[b,d] += s (ab|cd) D[a,c]
//   Kt[a,d] += s (ab|cd) D[b,c]     Kt[b,c] += s (ab|cd) D[a,d]
// in the Cartesian components; J = Jt + Jt^T and K = Kt + Kt^T are formed afterwards.
//
// k_small: one lane per contracted quartet, all intermediates in registers (the
//   paper's register-resident design for small classes, section 3, Algorithm 2).
// k_team:  a workgroup per batch of QB quartets; for each chunk of primitive quartets
//   the lanes compute the 2D integrals of every (primitive quartet, root, direction)
//   into LDS, then each lane accumulates the [e0|f0] elements of one f component (and
//   one slice of e components) from LDS into registers. Transfer to (ab|cd) and the
//   digestion run through a buffer in LDS (or global memory for the largest classes).
#pragma once
#include "jk_device.h"

namespace jk {

// ================================================================== k_small
template <int LA, int LB, int LC, int LD>
struct SmallCfg {
  static constexpr int E = LA + LB, F = LC + LD, N = (E + F) / 2 + 1;
  static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
  static constexpr int NE = range_count(LA, E), NF = range_count(LC, F);
  static constexpr int REGS = NE * NF + 3 * (E + 1) * (F + 1);
};

template <int LA, int LB, int LC, int LD, int MODE>
__global__ __launch_bounds__(256) void k_small(ClassArgs P) {
  using C = SmallCfg<LA, LB, LC, LD>;
  constexpr int E = C::E, F = C::F, N = C::N, NE = C::NE, NF = C::NF;
  constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND;
  constexpr int E0 = CT.start[LA], F0 = CT.start[LC];
  const int nq = *P.count;
  for (int qi = blockIdx.x * blockDim.x + threadIdx.x; qi < nq; qi += gridDim.x * blockDim.x) {
    const int2 qd = P.quartets[qi];
    const Pair bra = P.pairs[qd.x];
    const Pair ket = P.pairs[qd.y];
    double acc[NE * NF];
#pragma unroll
    for (int i = 0; i < NE * NF; ++i) acc[i] = 0.0;

    for (int ib = 0; ib < bra.npp; ++ib) {
      const PrimPair pb = P.pp[bra.pp_off + ib];
      const double hp = 0.5 / pb.p;
      for (int ik = 0; ik < ket.npp; ++ik) {
        const PrimPair pk = P.pp[ket.pp_off + ik];
        PrimQuartet Q;
        prim_quartet(pb, pk, bra.A, ket.A, Q);
        const double hq = 0.5 / pk.p;
        double u[N], w[N];
        rys_roots<N>(Q.T, u, w);
#pragma unroll
        for (int n = 0; n < N; ++n) {
          const double uq = u[n] * Q.pq_inv;
          const double b00 = 0.5 * uq;
          const double b10 = hp * (1.0 - uq * Q.q);
          const double b01 = hq * (1.0 - uq * Q.p);
          double Gx[E + 1][F + 1], Gy[E + 1][F + 1], Gz[E + 1][F + 1];
          vrr2d<E, F>(Gx, 1.0, Q.PA[0] - uq * Q.q * Q.PQ[0], Q.QC[0] + uq * Q.p * Q.PQ[0], b10, b01, b00);
          vrr2d<E, F>(Gy, 1.0, Q.PA[1] - uq * Q.q * Q.PQ[1], Q.QC[1] + uq * Q.p * Q.PQ[1], b10, b01, b00);
          vrr2d<E, F>(Gz, w[n] * Q.pref, Q.PA[2] - uq * Q.q * Q.PQ[2], Q.QC[2] + uq * Q.p * Q.PQ[2], b10, b01,
                      b00);
#pragma unroll
          for (int ie = 0; ie < NE; ++ie) {
#pragma unroll
            for (int jf = 0; jf < NF; ++jf) {
              acc[ie * NF + jf] = fma(Gx[CT.x[E0 + ie]][CT.x[F0 + jf]] * Gy[CT.y[E0 + ie]][CT.y[F0 + jf]],
                                      Gz[CT.z[E0 + ie]][CT.z[F0 + jf]], acc[ie * NF + jf]);
            }
          }
        }
      }
    }

    // transfer on the bra: hb[a][b][f]
    const double AB[3] = {bra.A[0] - bra.B[0], bra.A[1] - bra.B[1], bra.A[2] - bra.B[2]};
    const double CD[3] = {ket.A[0] - ket.B[0], ket.A[1] - ket.B[1], ket.A[2] - ket.B[2]};
    double abp[3][LB + 1], cdp[3][LD + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      abp[d][0] = 1.0;
#pragma unroll
      for (int k = 1; k <= LB; ++k) abp[d][k] = abp[d][k - 1] * AB[d];
      cdp[d][0] = 1.0;
#pragma unroll
      for (int k = 1; k <= LD; ++k) cdp[d][k] = cdp[d][k - 1] * CD[d];
    }
    double hb[NA * NB * NF];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        constexpr int A0 = CT.start[LA], B0 = CT.start[LB];
        const int ax = CT.x[A0 + a], ay = CT.y[A0 + a], az = CT.z[A0 + a];
        const int bx = CT.x[B0 + b], by = CT.y[B0 + b], bz = CT.z[B0 + b];
#pragma unroll
        for (int jf = 0; jf < NF; ++jf) hb[(a * NB + b) * NF + jf] = 0.0;
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
              const int ie = CT.idx[ax + kx][ay + ky][az + kz] - E0;
#pragma unroll
              for (int jf = 0; jf < NF; ++jf) hb[(a * NB + b) * NF + jf] = fma(cf, acc[ie * NF + jf], hb[(a * NB + b) * NF + jf]);
            }
          }
        }
      }
    }
    // transfer on the ket: g[ab][c][d]
    double g[NA * NB * NC * ND];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        constexpr int C0 = CT.start[LC], D0 = CT.start[LD];
        const int cx = CT.x[C0 + c], cy = CT.y[C0 + c], cz = CT.z[C0 + c];
        const int dx = CT.x[D0 + d], dy = CT.y[D0 + d], dz = CT.z[D0 + d];
#pragma unroll
        for (int ab = 0; ab < NA * NB; ++ab) g[ab * NC * ND + c * ND + d] = 0.0;
#pragma unroll
        for (int kx = 0; kx <= LD; ++kx) {
          if (kx > dx) continue;
#pragma unroll
          for (int ky = 0; ky <= LD; ++ky) {
            if (ky > dy) continue;
#pragma unroll
            for (int kz = 0; kz <= LD; ++kz) {
              if (kz > dz) continue;
              const double cf = (double)(binom(dx, kx) * binom(dy, ky) * binom(dz, kz)) * cdp[0][dx - kx] *
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

    if constexpr (MODE == MODE_JK) {
      const double s = sym_factor(bra, ket, qd.x, qd.y);
      const int oa = bra.ca, ob = bra.cb, oc = ket.ca, od = ket.cb;
      const int nc = P.nc;
      const double *Dm = P.Dc;
      double Dab[NA * NB], Dcd[NC * ND];
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) Dab[a * NB + b] = Dm[(size_t)(oa + a) * nc + ob + b];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int d = 0; d < ND; ++d) Dcd[c * ND + d] = Dm[(size_t)(oc + c) * nc + od + d];
      // Coulomb
#pragma unroll
      for (int ab = 0; ab < NA * NB; ++ab) {
        double v = 0.0;
#pragma unroll
        for (int cd = 0; cd < NC * ND; ++cd) v = fma(g[ab * NC * ND + cd], Dcd[cd], v);
        atomic_add(&P.Jc[(size_t)(oa + ab / NB) * nc + ob + ab % NB], 2.0 * s * v);
      }
#pragma unroll
      for (int cd = 0; cd < NC * ND; ++cd) {
        double v = 0.0;
#pragma unroll
        for (int ab = 0; ab < NA * NB; ++ab) v = fma(g[ab * NC * ND + cd], Dab[ab], v);
        atomic_add(&P.Jc[(size_t)(oc + cd / ND) * nc + od + cd % ND], 2.0 * s * v);
      }
      // exchange: K[a,c] += D[b,d], K[a,d] += D[b,c], K[b,c] += D[a,d], K[b,d] += D[a,c]
#pragma unroll
      for (int a = 0; a < NA; ++a) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          double v = 0.0;
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int d = 0; d < ND; ++d)
              v = fma(g[(a * NB + b) * NC * ND + c * ND + d], Dm[(size_t)(ob + b) * nc + od + d], v);
          atomic_add(&P.Kc[(size_t)(oa + a) * nc + oc + c], s * v);
        }
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          double v = 0.0;
#pragma unroll
          for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int c = 0; c < NC; ++c)
              v = fma(g[(a * NB + b) * NC * ND + c * ND + d], Dm[(size_t)(ob + b) * nc + oc + c], v);
          atomic_add(&P.Kc[(size_t)(oa + a) * nc + od + d], s * v);
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
            for (int d = 0; d < ND; ++d)
              v = fma(g[(a * NB + b) * NC * ND + c * ND + d], Dm[(size_t)(oa + a) * nc + od + d], v);
          atomic_add(&P.Kc[(size_t)(ob + b) * nc + oc + c], s * v);
        }
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          double v = 0.0;
#pragma unroll
          for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int c = 0; c < NC; ++c)
              v = fma(g[(a * NB + b) * NC * ND + c * ND + d], Dm[(size_t)(oa + a) * nc + oc + c], v);
          atomic_add(&P.Kc[(size_t)(ob + b) * nc + od + d], s * v);
        }
      }
    } else if constexpr (MODE == MODE_SCHWARZ) {
      if constexpr (LA == LC && LB == LD) {
        double mx = 0.0;
#pragma unroll
        for (int ab = 0; ab < NA * NB; ++ab) mx = fmax(mx, fabs(g[ab * NC * ND + ab]));
        atomic_max_nonneg(&P.out[qd.x], mx);
      }
    } else {  // MODE_ERI: all eight index images of the block
      const size_t nc = P.nc;
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int d = 0; d < ND; ++d) {
              const double v = g[(a * NB + b) * NC * ND + c * ND + d];
              const size_t i = bra.ca + a, j = bra.cb + b, k = ket.ca + c, l = ket.cb + d;
              P.out[((i * nc + j) * nc + k) * nc + l] = v;
              P.out[((j * nc + i) * nc + k) * nc + l] = v;
              P.out[((i * nc + j) * nc + l) * nc + k] = v;
              P.out[((j * nc + i) * nc + l) * nc + k] = v;
              P.out[((k * nc + l) * nc + i) * nc + j] = v;
              P.out[((l * nc + k) * nc + i) * nc + j] = v;
              P.out[((k * nc + l) * nc + j) * nc + i] = v;
              P.out[((l * nc + k) * nc + j) * nc + i] = v;
            }
    }
  }
}

// ================================================================== k_team
template <int LA, int LB, int LC, int LD>
struct TeamCfg {
  static constexpr int E = LA + LB, F = LC + LD, N = (E + F) / 2 + 1;
  static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
  static constexpr int NE = range_count(LA, E), NF = range_count(LC, F);
  static constexpr int GS1 = (E + 1) * (F + 1);          // one direction of one root
  static constexpr int GS = 3 * GS1;
  static constexpr int EMAXACC = 56;                     // accumulators per lane
  static constexpr int NEP = (NE + EMAXACC - 1) / EMAXACC;
  static constexpr int EPS = (NE + NEP - 1) / NEP;
  static constexpr int FW = NEP > 1 ? ((NF + 63) / 64) * 64 : NF;
  static constexpr int TPQ = NEP * FW;
  static constexpr int BLOCK = TPQ > 256 ? ((TPQ + 63) / 64) * 64 : 256;
  static constexpr int QB = BLOCK / TPQ;
  static constexpr int PC0 = (48 * 1024) / (QB * N * GS * 8);
  static constexpr int PC1 = BLOCK / (QB * N * 3);
  static constexpr int PC = (PC0 < PC1 ? PC0 : PC1) < 1 ? 1 : (PC0 < PC1 ? PC0 : PC1);
  static constexpr int XS = NE * NF, YS = NA * NB * NF, ZS = NA * NB * NC * ND;
  static constexpr int R1 = XS > ZS ? XS : ZS;
  static constexpr int BUF = QB * (R1 + YS);
  static constexpr bool GLOBAL_BUF = BUF * 8 > 56 * 1024;
  static constexpr int LDS_BUF = GLOBAL_BUF ? 1 : BUF;
};

// Product of one e-slice for one lane: elements e in [P0*EPS, min(NE,(P0+1)*EPS)).
template <int LA, int LB, int LC, int LD, int P0>
__device__ __forceinline__ void team_product(const double *__restrict__ base, int xo, int yo, int zo,
                                             double (&acc)[TeamCfg<LA, LB, LC, LD>::EPS]) {
  using C = TeamCfg<LA, LB, LC, LD>;
  constexpr int E0 = CT.start[LA];
  constexpr int LO = P0 * C::EPS;
  constexpr int HI = (LO + C::EPS < C::NE) ? LO + C::EPS : C::NE;
  constexpr int EX = C::E;   // largest component needed
  double gx[EX + 1], gy[EX + 1], gz[EX + 1];
#pragma unroll
  for (int e = 0; e <= EX; ++e) {
    gx[e] = base[xo + e * (C::F + 1)];
    gy[e] = base[yo + e * (C::F + 1)];
    gz[e] = base[zo + e * (C::F + 1)];
  }
#pragma unroll
  for (int i = LO; i < HI; ++i) {
    acc[i - LO] = fma(gx[CT.x[E0 + i]] * gy[CT.y[E0 + i]], gz[CT.z[E0 + i]], acc[i - LO]);
  }
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

template <int LA, int LB, int LC, int LD, int MODE>
__global__ __launch_bounds__((TeamCfg<LA, LB, LC, LD>::BLOCK)) void k_team(ClassArgs P) {
  using C = TeamCfg<LA, LB, LC, LD>;
  constexpr int E = C::E, F = C::F, N = C::N, NE = C::NE, NF = C::NF;
  constexpr int NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND;
  constexpr int QB = C::QB, PC = C::PC, GS = C::GS, GS1 = C::GS1, BLOCK = C::BLOCK;
  constexpr int E0 = CT.start[LA], F0 = CT.start[LC];

  __shared__ double sG[QB * PC * N * GS];
  __shared__ double sBuf[C::LDS_BUF];
  __shared__ int sQ[QB][8];           // bra idx, ket idx, bra pp_off, bra npp, ket pp_off, ket npp, valid
  __shared__ double sGeo[QB][12];     // A, B, C, D
  __shared__ int sKmax;

  double *buf = C::GLOBAL_BUF ? P.scratch + (size_t)blockIdx.x * P.scratch_per_wg : sBuf;
  double *X = buf;                    // [QB][NE][NF]  (later Z: [QB][NA*NB][NC*ND])
  double *Y = buf + QB * C::R1;       // [QB][NA*NB][NF]
  const int tid = threadIdx.x;
  const int nq = *P.count;
  const int nbatch = (nq + QB - 1) / QB;

  // product role of this lane
  const int pq_ = tid / C::TPQ;
  const int pr = tid % C::TPQ;
  const int part = pr / C::FW;
  const int pf = pr % C::FW;
  const bool prole = pq_ < QB && pf < NF;
  int xo = 0, yo = 0, zo = 0;
  if (prole) {
    xo = CTD.x[F0 + pf];
    yo = GS1 + CTD.y[F0 + pf];
    zo = 2 * GS1 + CTD.z[F0 + pf];
  }

  for (int batch = blockIdx.x; batch < nbatch; batch += gridDim.x) {
    if (tid < QB) {
      const int qi = batch * QB + tid;
      const bool valid = qi < nq;
      int2 qd = valid ? P.quartets[qi] : make_int2(0, 0);
      const Pair &b = P.pairs[qd.x];
      const Pair &k = P.pairs[qd.y];
      sQ[tid][0] = qd.x; sQ[tid][1] = qd.y;
      sQ[tid][2] = b.pp_off; sQ[tid][3] = valid ? b.npp : 0;
      sQ[tid][4] = k.pp_off; sQ[tid][5] = valid ? k.npp : 0;
      sQ[tid][6] = valid;
      for (int d = 0; d < 3; ++d) {
        sGeo[tid][d] = b.A[d]; sGeo[tid][3 + d] = b.B[d];
        sGeo[tid][6 + d] = k.A[d]; sGeo[tid][9 + d] = k.B[d];
      }
    }
    __syncthreads();
    if (tid == 0) {
      int m = 0;
      for (int q = 0; q < QB; ++q) m = max(m, sQ[q][3] * sQ[q][5]);
      sKmax = m;
    }
    __syncthreads();
    const int kmax = sKmax;

    double acc[C::EPS];
#pragma unroll
    for (int i = 0; i < C::EPS; ++i) acc[i] = 0.0;

    for (int c0 = 0; c0 < kmax; c0 += PC) {
      // 2D integrals of every (quartet, primitive quartet, root, direction) of the chunk
      for (int t = tid; t < QB * PC * N * 3; t += BLOCK) {
        const int q = t / (PC * N * 3);
        const int rem = t % (PC * N * 3);
        const int pl = rem / (N * 3);
        const int n = (rem % (N * 3)) / 3;
        const int dir = rem % 3;
        const int pidx = c0 + pl;
        const int nk = sQ[q][5];
        if (pidx < sQ[q][3] * nk) {
          const PrimPair pb = P.pp[sQ[q][2] + pidx / nk];
          const PrimPair pk = P.pp[sQ[q][4] + pidx % nk];
          PrimQuartet Q;
          prim_quartet(pb, pk, &sGeo[q][0], &sGeo[q][6], Q);
          double u, w;
          rys_root1<N>(Q.T, n, u, w);
          const double uq = u * Q.pq_inv;
          const double b00 = 0.5 * uq;
          const double b10 = 0.5 / Q.p * (1.0 - uq * Q.q);
          const double b01 = 0.5 / Q.q * (1.0 - uq * Q.p);
          const double pa = dir == 0 ? Q.PA[0] : (dir == 1 ? Q.PA[1] : Q.PA[2]);
          const double qc = dir == 0 ? Q.QC[0] : (dir == 1 ? Q.QC[1] : Q.QC[2]);
          const double pqd = dir == 0 ? Q.PQ[0] : (dir == 1 ? Q.PQ[1] : Q.PQ[2]);
          double G[E + 1][F + 1];
          vrr2d<E, F>(G, dir == 2 ? w * Q.pref : 1.0, pa - uq * Q.q * pqd, qc + uq * Q.p * pqd, b10, b01, b00);
          double *dst = sG + ((q * PC + pl) * N + n) * GS + dir * GS1;
#pragma unroll
          for (int e = 0; e <= E; ++e)
#pragma unroll
            for (int f = 0; f <= F; ++f) dst[e * (F + 1) + f] = G[e][f];
        }
      }
      __syncthreads();
      if (prole) {
        const int npl = min(PC, sQ[pq_][3] * sQ[pq_][5] - c0);
        for (int pl = 0; pl < npl; ++pl) {
#pragma unroll
          for (int n = 0; n < N; ++n) {
            const double *base = sG + ((pq_ * PC + pl) * N + n) * GS;
            team_product_dispatch<LA, LB, LC, LD, 0>(part, base, xo, yo, zo, acc);
          }
        }
      }
      __syncthreads();
    }

    // contracted [e0|f0] -> X
    if (prole) {
#pragma unroll
      for (int i = 0; i < C::EPS; ++i) {
        const int e = part * C::EPS + i;
        if (e < NE) X[(pq_ * NE + e) * NF + pf] = acc[i];
      }
    }
    __syncthreads();
    // transfer on the bra: Y[q][a*NB+b][f]
    for (int t = tid; t < QB * NA * NB * NF; t += BLOCK) {
      const int q = t / (NA * NB * NF);
      const int rem = t % (NA * NB * NF);
      const int ab = rem / NF, f = rem % NF;
      const int a = ab / NB, b = ab % NB;
      const int ax = CTD.x[E0 + a], ay = CTD.y[E0 + a], az = CTD.z[E0 + a];
      const int bx = CTD.x[CT.start[LB] + b], by = CTD.y[CT.start[LB] + b], bz = CTD.z[CT.start[LB] + b];
      const double ABx = sGeo[q][0] - sGeo[q][3], ABy = sGeo[q][1] - sGeo[q][4], ABz = sGeo[q][2] - sGeo[q][5];
      double v = 0.0;
      double px = 1.0;
      for (int kx = bx; kx >= 0; --kx) {
        double py = 1.0;
        for (int ky = by; ky >= 0; --ky) {
          double pz = 1.0;
          for (int kz = bz; kz >= 0; --kz) {
            const double cf = (double)(binom(bx, kx) * binom(by, ky) * binom(bz, kz)) * px * py * pz;
            const int ie = CTD.idx[ax + kx][ay + ky][az + kz] - E0;
            v = fma(cf, X[(q * NE + ie) * NF + f], v);
            pz *= ABz;
          }
          py *= ABy;
        }
        px *= ABx;
      }
      Y[(q * NA * NB + ab) * NF + f] = v;
    }
    __syncthreads();
    // transfer on the ket: Z[q][ab][c*ND+d] (overwrites X)
    double *Z = X;
    for (int t = tid; t < QB * NA * NB * NC * ND; t += BLOCK) {
      const int q = t / (NA * NB * NC * ND);
      const int rem = t % (NA * NB * NC * ND);
      const int ab = rem / (NC * ND), cd = rem % (NC * ND);
      const int c = cd / ND, d = cd % ND;
      const int cx = CTD.x[F0 + c], cy = CTD.y[F0 + c], cz = CTD.z[F0 + c];
      const int dx = CTD.x[CT.start[LD] + d], dy = CTD.y[CT.start[LD] + d], dz = CTD.z[CT.start[LD] + d];
      const double CDx = sGeo[q][6] - sGeo[q][9], CDy = sGeo[q][7] - sGeo[q][10], CDz = sGeo[q][8] - sGeo[q][11];
      double v = 0.0;
      double px = 1.0;
      for (int kx = dx; kx >= 0; --kx) {
        double py = 1.0;
        for (int ky = dy; ky >= 0; --ky) {
          double pz = 1.0;
          for (int kz = dz; kz >= 0; --kz) {
            const double cf = (double)(binom(dx, kx) * binom(dy, ky) * binom(dz, kz)) * px * py * pz;
            const int jf = CTD.idx[cx + kx][cy + ky][cz + kz] - F0;
            v = fma(cf, Y[(q * NA * NB + ab) * NF + jf], v);
            pz *= CDz;
          }
          py *= CDy;
        }
        px *= CDx;
      }
      // X (region 1) is read by other lanes of this pass only through Y, so Z may overwrite it
      Z[(q * NA * NB + ab) * NC * ND + cd] = v;
    }
    __syncthreads();

    if constexpr (MODE == MODE_JK) {
      constexpr int T1 = NA * NB, T2 = NC * ND, T3 = NA * NC, T4 = NA * ND, T5 = NB * NC, T6 = NB * ND;
      constexpr int TOT = T1 + T2 + T3 + T4 + T5 + T6;
      const int nc = P.nc;
      const double *Dm = P.Dc;
      for (int t = tid; t < QB * TOT; t += BLOCK) {
        const int q = t / TOT;
        int r = t % TOT;
        if (!sQ[q][6]) continue;
        const Pair &bra = P.pairs[sQ[q][0]];
        const Pair &ket = P.pairs[sQ[q][1]];
        const double s = sym_factor(bra, ket, sQ[q][0], sQ[q][1]);
        const int oa = bra.ca, ob = bra.cb, oc = ket.ca, od = ket.cb;
        const double *g = Z + (size_t)q * NA * NB * NC * ND;
        double v = 0.0;
        if (r < T1) {                       // J[a,b] += 2s sum_cd g D[c,d]
          const int a = r / NB, b = r % NB;
          for (int c = 0; c < NC; ++c)
            for (int d = 0; d < ND; ++d) v = fma(g[(a * NB + b) * NC * ND + c * ND + d], Dm[(size_t)(oc + c) * nc + od + d], v);
          atomic_add(&P.Jc[(size_t)(oa + a) * nc + ob + b], 2.0 * s * v);
          continue;
        }
        r -= T1;
        if (r < T2) {                       // J[c,d] += 2s sum_ab g D[a,b]
          const int c = r / ND, d = r % ND;
          for (int a = 0; a < NA; ++a)
            for (int b = 0; b < NB; ++b) v = fma(g[(a * NB + b) * NC * ND + c * ND + d], Dm[(size_t)(oa + a) * nc + ob + b], v);
          atomic_add(&P.Jc[(size_t)(oc + c) * nc + od + d], 2.0 * s * v);
          continue;
        }
        r -= T2;
        if (r < T3) {                       // K[a,c] += s sum_bd g D[b,d]
          const int a = r / NC, c = r % NC;
          for (int b = 0; b < NB; ++b)
            for (int d = 0; d < ND; ++d) v = fma(g[(a * NB + b) * NC * ND + c * ND + d], Dm[(size_t)(ob + b) * nc + od + d], v);
          atomic_add(&P.Kc[(size_t)(oa + a) * nc + oc + c], s * v);
          continue;
        }
        r -= T3;
        if (r < T4) {                       // K[a,d] += s sum_bc g D[b,c]
          const int a = r / ND, d = r % ND;
          for (int b = 0; b < NB; ++b)
            for (int c = 0; c < NC; ++c) v = fma(g[(a * NB + b) * NC * ND + c * ND + d], Dm[(size_t)(ob + b) * nc + oc + c], v);
          atomic_add(&P.Kc[(size_t)(oa + a) * nc + od + d], s * v);
          continue;
        }
        r -= T4;
        if (r < T5) {                       // K[b,c] += s sum_ad g D[a,d]
          const int b = r / NC, c = r % NC;
          for (int a = 0; a < NA; ++a)
            for (int d = 0; d < ND; ++d) v = fma(g[(a * NB + b) * NC * ND + c * ND + d], Dm[(size_t)(oa + a) * nc + od + d], v);
          atomic_add(&P.Kc[(size_t)(ob + b) * nc + oc + c], s * v);
          continue;
        }
        r -= T5;
        {                                   // K[b,d] += s sum_ac g D[a,c]
          const int b = r / ND, d = r % ND;
          for (int a = 0; a < NA; ++a)
            for (int c = 0; c < NC; ++c) v = fma(g[(a * NB + b) * NC * ND + c * ND + d], Dm[(size_t)(oa + a) * nc + oc + c], v);
          atomic_add(&P.Kc[(size_t)(ob + b) * nc + od + d], s * v);
        }
      }
    } else if constexpr (MODE == MODE_SCHWARZ) {
      if constexpr (LA == LC && LB == LD) {
        for (int t = tid; t < QB * NA * NB; t += BLOCK) {
          const int q = t / (NA * NB), ab = t % (NA * NB);
          if (!sQ[q][6]) continue;
          atomic_max_nonneg(&P.out[sQ[q][0]], fabs(Z[((size_t)q * NA * NB + ab) * NC * ND + ab]));
        }
      }
    } else {
      const size_t nc = P.nc;
      for (int t = tid; t < QB * NA * NB * NC * ND; t += BLOCK) {
        const int q = t / (NA * NB * NC * ND);
        if (!sQ[q][6]) continue;
        const int rem = t % (NA * NB * NC * ND);
        const int ab = rem / (NC * ND), cd = rem % (NC * ND);
        const Pair &bra = P.pairs[sQ[q][0]];
        const Pair &ket = P.pairs[sQ[q][1]];
        const size_t i = bra.ca + ab / NB, j = bra.cb + ab % NB, k = ket.ca + cd / ND, l = ket.cb + cd % ND;
        const double v = Z[(size_t)q * NA * NB * NC * ND + rem];
        P.out[((i * nc + j) * nc + k) * nc + l] = v;
        P.out[((j * nc + i) * nc + k) * nc + l] = v;
        P.out[((i * nc + j) * nc + l) * nc + k] = v;
        P.out[((j * nc + i) * nc + l) * nc + k] = v;
        P.out[((k * nc + l) * nc + i) * nc + j] = v;
        P.out[((l * nc + k) * nc + i) * nc + j] = v;
        P.out[((k * nc + l) * nc + j) * nc + i] = v;
        P.out[((l * nc + k) * nc + j) * nc + i] = v;
      }
    }
    __syncthreads();
  }
}

}  // namespace jk
