// Nuclear gradient of the two-electron energy (paper section 4, Algorithm 4: the derivative
// integrals of a shell quartet contracted with the density at once, twelve accumulators per
// quartet). With D held fixed,
//   dE/dR = sum over kept unique quartets (ab|cd) of sum_abcd W_abcd d(ab|cd)/dR,
//   W_abcd = s [8 D_ab D_cd - 2 D_ac D_bd - 2 D_ad D_bc]   (Cartesian components, D_cart),
// s the eight-fold symmetry factor; E = tr(D (J - K/2)) of the J/K build. A primitive Cartesian
// Gaussian differentiates into a raised and a lowered one,
//   d/dA_x x_A^a exp(-alpha r_A^2) = 2 alpha x_A^(a+1) exp(...) - a x_A^(a-1) exp(...),
// so in the Rys form of section 2 only the one-dimensional integral of the differentiated
// direction changes: I'_x(a,b,c,d) = 2 alpha I_x(a+1,b,c,d) - a I_x(a-1,b,c,d) (likewise for the
// centres B and C with beta, gamma). The one-dimensional integrals come from the 2D recurrence
// table G(e, f), e <= la+lb+1, f <= lc+ld+1 (one quantum above the ERI's), by the binomial
// transfer I(a,b,c,d) = sum_k sum_k' C(b,k) (A-B)^(b-k) C(d,k') (C-D)^(d-k') G(a+k, c+k'). The
// centre D follows from translational invariance: dE/dD = -(dE/dA + dE/dB + dE/dC) per quartet.
#pragma once
#include "jk_device.h"

namespace jk {

struct GradArgs {
  const Pair *pairs;
  const PrimPair *pp;
  const double *ppab;           // [2 per primitive pair] exponent of shell a, of shell b
  const int *kets;              // screened work list (segments per bra pair and ket class)
  const long long *class_off;
  const int *segoff, *segcnt;
  const double *Dc;             // Cartesian density (nc x nc)
  int nc;
  const int *shell_atom;        // per shell: its atom
  double *grad;                 // natom x 3 (accumulated with atomics)
  const int2 *units;            // work units (bra pair, slice) of the launch
  const int *nunits;
  int units_cap;
  int slice;
  int *next;
};

template <int LA, int LB, int LC, int LD>
struct GradCfg {
  static constexpr int E = LA + LB, F = LC + LD, N = (E + F + 1) / 2 + 1;   // derivative: one quantum more
  static constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC), ND = ncart(LD);
  static constexpr int NEL = NA * NB * NC * ND;
  // one-dimensional table I[a'][b'][c'][d'], a' <= LA+1, b' <= LB+1, c' <= LC+1, d' <= LD
  static constexpr int SC = LD + 1, SB = (LC + 2) * SC, SA = (LB + 2) * SB, T1 = (LA + 2) * SA;
  static constexpr int G1 = (E + 2) * (F + 2);   // one direction of the 2D table
  // lane per quartet (tables in registers) for the small classes, else a wave per quartet
  static constexpr bool LANE = NEL <= 27;
  // larger classes: a team of TW waves per quartet (one wave up to 192 elements, else four)
  static constexpr int TW = NEL <= 192 ? 1 : 4;
  static constexpr int EPL = (NEL + 64 * TW - 1) / (64 * TW);   // elements per lane
  static constexpr int WAVE_LDS = 3 * G1 + 3 * T1;              // doubles of LDS per team
};

// d/dX of one Cartesian element for the nine (centre, direction) pairs, accumulated with
// weight w: acc[3 * centre + dir] (centres A, B, C).
__device__ __forceinline__ void grad_element(double w, const double (&i)[3], const double (&dA)[3],
                                             const double (&dB)[3], const double (&dC)[3], double (&acc)[9]) {
  const double wyz = w * i[1] * i[2], wxz = w * i[0] * i[2], wxy = w * i[0] * i[1];
  acc[0] = fma(wyz, dA[0], acc[0]);
  acc[1] = fma(wxz, dA[1], acc[1]);
  acc[2] = fma(wxy, dA[2], acc[2]);
  acc[3] = fma(wyz, dB[0], acc[3]);
  acc[4] = fma(wxz, dB[1], acc[4]);
  acc[5] = fma(wxy, dB[2], acc[5]);
  acc[6] = fma(wyz, dC[0], acc[6]);
  acc[7] = fma(wxz, dC[1], acc[7]);
  acc[8] = fma(wxy, dC[2], acc[8]);
}

// W_abcd of one element (Cartesian indices inside the shells)
__device__ __forceinline__ double grad_weight(const double *Dm, int nc, int ra, int rb, int rc, int rd, double s) {
  const double dab = Dm[(size_t)ra * nc + rb], dcd = Dm[(size_t)rc * nc + rd];
  const double dac = Dm[(size_t)ra * nc + rc], dbd = Dm[(size_t)rb * nc + rd];
  const double dad = Dm[(size_t)ra * nc + rd], dbc = Dm[(size_t)rb * nc + rc];
  return s * (8.0 * dab * dcd - 2.0 * dac * dbd - 2.0 * dad * dbc);
}

// binomial coefficients C(n, k), n <= 5
static __constant__ double BINOM[6][6] = {{1, 0, 0, 0, 0, 0}, {1, 1, 0, 0, 0, 0}, {1, 2, 1, 0, 0, 0},
                                          {1, 3, 3, 1, 0, 0}, {1, 4, 6, 4, 1, 0}, {1, 5, 10, 10, 5, 1}};

// binomial transfer of one direction for compile-time-bounded indices (a+b <= E+1, c+d <= F+1)
template <int LB1, int LD1, int F2>
__device__ __forceinline__ double tr1(const double *G, double ab, double cd, int a, int b, int c, int d) {
  double v = 0.0;
  double pb = 1.0;                        // (A-B)^(b-k), k from b down to 0
#pragma unroll
  for (int k = LB1; k >= 0; --k) {
    if (k > b) continue;
    const double cb = (double)binom(b, k) * pb;
    double inner = 0.0, pd = 1.0;
#pragma unroll
    for (int kk = LD1; kk >= 0; --kk) {
      if (kk > d) continue;
      inner = fma((double)binom(d, kk) * pd, G[(a + k) * F2 + c + kk], inner);
      pd *= cd;
    }
    v = fma(cb, inner, v);
    pb *= ab;
  }
  return v;
}

// ------------------------------------------------------------------ lane per quartet
template <int LA, int LB, int LC, int LD>
__device__ __forceinline__ void grad_lane_quartet(const GradArgs &A, const Pair &bra, int bi, int ki,
                                                  double (&gab)[6]) {
  using C = GradCfg<LA, LB, LC, LD>;
  constexpr int E = C::E, F = C::F, N = C::N, NA = C::NA, NB = C::NB, NC = C::NC, ND = C::ND, NEL = C::NEL;
  constexpr int A0 = CT.start[LA], B0 = CT.start[LB], C0 = CT.start[LC], D0 = CT.start[LD];
  const Pair ket = A.pairs[ki];
  const double s = sym_factor(bra, ket, bi, ki);
  double W[NEL];
#pragma unroll
  for (int e = 0; e < NEL; ++e) {
    const int ia = e / (NB * NC * ND), ib = (e / (NC * ND)) % NB, ic = (e / ND) % NC, id = e % ND;
    W[e] = grad_weight(A.Dc, A.nc, bra.ca + ia, bra.cb + ib, ket.ca + ic, ket.cb + id, s);
  }
  const double AB[3] = {bra.A[0] - bra.B[0], bra.A[1] - bra.B[1], bra.A[2] - bra.B[2]};
  const double CD[3] = {ket.A[0] - ket.B[0], ket.A[1] - ket.B[1], ket.A[2] - ket.B[2]};
  double acc[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) acc[i] = 0.0;
  for (int ik = 0; ik < ket.npp; ++ik) {
    const PrimPair pk = A.pp[ket.pp_off + ik];
    const double gam2 = 2.0 * A.ppab[2 * (ket.pp_off + ik)];
    for (int ib = 0; ib < bra.npp; ++ib) {
      const PrimPair pb = A.pp[bra.pp_off + ib];
      const double al2 = 2.0 * A.ppab[2 * (bra.pp_off + ib)], be2 = 2.0 * A.ppab[2 * (bra.pp_off + ib) + 1];
      PrimQuartet Q;
      prim_quartet(pb, pk, bra.A, ket.A, Q);
      const double hp = 0.5 * pb.ip, hq = 0.5 * pk.ip;
#pragma unroll 1
      for (int n = 0; n < N; ++n) {
        double un, wn;
        rys_root1<N>(Q.T, n, un, wn);
        const double uq = un * Q.pq_inv;
        const double b00 = 0.5 * uq, b10 = hp * (1.0 - uq * Q.q), b01 = hq * (1.0 - uq * Q.p);
        double G[3][E + 2][F + 2];
#pragma unroll
        for (int d = 0; d < 3; ++d)
          vrr2d<E + 1, F + 1>(G[d], d == 2 ? wn * Q.pref : 1.0, Q.PA[d] - uq * Q.q * Q.PQ[d],
                              Q.QC[d] + uq * Q.p * Q.PQ[d], b10, b01, b00);
#pragma unroll
        for (int e = 0; e < NEL; ++e) {
          const int ia = e / (NB * NC * ND), ib2 = (e / (NC * ND)) % NB, ic = (e / ND) % NC, id = e % ND;
          double iv[3], dA[3], dB[3], dC[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const int a = d == 0 ? CT.x[A0 + ia] : d == 1 ? CT.y[A0 + ia] : CT.z[A0 + ia];
            const int b = d == 0 ? CT.x[B0 + ib2] : d == 1 ? CT.y[B0 + ib2] : CT.z[B0 + ib2];
            const int c = d == 0 ? CT.x[C0 + ic] : d == 1 ? CT.y[C0 + ic] : CT.z[C0 + ic];
            const int dd = d == 0 ? CT.x[D0 + id] : d == 1 ? CT.y[D0 + id] : CT.z[D0 + id];
            const double *g = &G[d][0][0];
            iv[d] = tr1<LB + 1, LD, F + 2>(g, AB[d], CD[d], a, b, c, dd);
            dA[d] = al2 * tr1<LB + 1, LD, F + 2>(g, AB[d], CD[d], a + 1, b, c, dd);
            if (a > 0) dA[d] -= a * tr1<LB + 1, LD, F + 2>(g, AB[d], CD[d], a - 1, b, c, dd);
            dB[d] = be2 * tr1<LB + 1, LD, F + 2>(g, AB[d], CD[d], a, b + 1, c, dd);
            if (b > 0) dB[d] -= b * tr1<LB + 1, LD, F + 2>(g, AB[d], CD[d], a, b - 1, c, dd);
            dC[d] = gam2 * tr1<LB + 1, LD, F + 2>(g, AB[d], CD[d], a, b, c + 1, dd);
            if (c > 0) dC[d] -= c * tr1<LB + 1, LD, F + 2>(g, AB[d], CD[d], a, b, c - 1, dd);
          }
          grad_element(W[e], iv, dA, dB, dC, acc);
        }
      }
    }
  }
  // centres C and D of this quartet now, A and B summed over the unit
  const int atc = A.shell_atom[ket.sa], atd = A.shell_atom[ket.sb];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    atomic_add(&A.grad[3 * atc + d], acc[6 + d]);
    atomic_add(&A.grad[3 * atd + d], -(acc[d] + acc[3 + d] + acc[6 + d]));
    gab[d] += acc[d];
    gab[3 + d] += acc[3 + d];
  }
}

// ------------------------------------------------------------------ team of waves per quartet
// TW waves (1, or the whole 256-lane workgroup) evaluate one quartet; sw: WAVE_LDS doubles of
// the team's LDS: G (3 directions) then the 1D tables (3 directions).
template <int TW>
__device__ __forceinline__ void team_sync() {
  if constexpr (TW == 1) {
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

template <int LA, int LB, int LC, int LD>
__device__ __forceinline__ void grad_team_quartet(const GradArgs &A, const Pair &bra, int bi, int ki, double *sw,
                                                  double (&gab)[6]) {
  using C = GradCfg<LA, LB, LC, LD>;
  constexpr int E = C::E, F = C::F, N = C::N, NB = C::NB, NC = C::NC, ND = C::ND, NEL = C::NEL;
  constexpr int TW = C::TW, TL = 64 * TW, EPL = C::EPL;
  constexpr int G1 = C::G1, T1 = C::T1, SA = C::SA, SB = C::SB, SC = C::SC;
  constexpr int A0 = CT.start[LA], B0 = CT.start[LB], C0 = CT.start[LC], D0 = CT.start[LD];
  const int lt = threadIdx.x % TL;              // lane inside the team
  const Pair ket = A.pairs[ki];
  const double s = sym_factor(bra, ket, bi, ki);
  double *sG = sw, *sI = sw + 3 * G1;
  // this lane's elements e = lt + TL j: weight and table offset per direction
  double W[EPL];
  int off[EPL][3];
#pragma unroll
  for (int j = 0; j < EPL; ++j) {
    const int e = lt + TL * j;
    const int ee = e < NEL ? e : 0;
    const int ia = ee / (NB * NC * ND), ib = (ee / (NC * ND)) % NB, ic = (ee / ND) % NC, id = ee % ND;
    W[j] = e < NEL ? grad_weight(A.Dc, A.nc, bra.ca + ia, bra.cb + ib, ket.ca + ic, ket.cb + id, s) : 0.0;
    off[j][0] = CTD.x[A0 + ia] * SA + CTD.x[B0 + ib] * SB + CTD.x[C0 + ic] * SC + CTD.x[D0 + id];
    off[j][1] = T1 + CTD.y[A0 + ia] * SA + CTD.y[B0 + ib] * SB + CTD.y[C0 + ic] * SC + CTD.y[D0 + id];
    off[j][2] = 2 * T1 + CTD.z[A0 + ia] * SA + CTD.z[B0 + ib] * SB + CTD.z[C0 + ic] * SC + CTD.z[D0 + id];
  }
  const double AB[3] = {bra.A[0] - bra.B[0], bra.A[1] - bra.B[1], bra.A[2] - bra.B[2]};
  const double CD[3] = {ket.A[0] - ket.B[0], ket.A[1] - ket.B[1], ket.A[2] - ket.B[2]};
  double acc[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) acc[i] = 0.0;
  for (int ik = 0; ik < ket.npp; ++ik) {
    const PrimPair pk = A.pp[ket.pp_off + ik];
    const double gam2 = 2.0 * A.ppab[2 * (ket.pp_off + ik)];
    for (int ib = 0; ib < bra.npp; ++ib) {
      const PrimPair pb = A.pp[bra.pp_off + ib];
      const double al2 = 2.0 * A.ppab[2 * (bra.pp_off + ib)], be2 = 2.0 * A.ppab[2 * (bra.pp_off + ib) + 1];
      PrimQuartet Q;
      prim_quartet(pb, pk, bra.A, ket.A, Q);
      for (int n = 0; n < N; ++n) {
        double un, wn;
        rys_root1<N>(Q.T, n, un, wn);
        const double uq = un * Q.pq_inv;
        if (lt < 3) {
          const int d = lt;
          vrr2d_store<E + 1, F + 1>(sG + d * G1, d == 2 ? wn * Q.pref : 1.0, Q.PA[d] - uq * Q.q * Q.PQ[d],
                                    Q.QC[d] + uq * Q.p * Q.PQ[d], 0.5 * pb.ip * (1.0 - uq * Q.q),
                                    0.5 * pk.ip * (1.0 - uq * Q.p), 0.5 * uq);
        }
        team_sync<TW>();
        // one-dimensional tables: entries a' + b' <= E + 1 (the others are never read)
        for (int t = lt; t < 3 * T1; t += TL) {
          const int d = t / T1, r = t % T1;
          const int a = r / SA, b = (r / SB) % (LB + 2), c = (r / SC) % (LC + 2), dd = r % SC;
          double v = 0.0;
          if (a + b <= E + 1) {
            const double *g = sG + d * G1 + c;
            double pbp = 1.0;
            for (int k = b; k >= 0; --k) {
              double inner = 0.0, pd = 1.0;
              for (int kk = dd; kk >= 0; --kk) {
                inner = fma(BINOM[dd][kk] * pd, g[(a + k) * (F + 2) + kk], inner);
                pd *= CD[d];
              }
              v = fma(BINOM[b][k] * pbp, inner, v);
              pbp *= AB[d];
            }
          }
          sI[t] = v;
        }
        team_sync<TW>();
#pragma unroll
        for (int j = 0; j < EPL; ++j) {
          if (lt + TL * j < NEL) {
            double iv[3], dA[3], dB[3], dC[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const int o = off[j][d];
              const int r = o - d * T1;
              const int a = r / SA, b = (r / SB) % (LB + 2), c = (r / SC) % (LC + 2);
              iv[d] = sI[o];
              dA[d] = al2 * sI[o + SA] - (a > 0 ? a * sI[o - SA] : 0.0);
              dB[d] = be2 * sI[o + SB] - (b > 0 ? b * sI[o - SB] : 0.0);
              dC[d] = gam2 * sI[o + SC] - (c > 0 ? c * sI[o - SC] : 0.0);
            }
            grad_element(W[j], iv, dA, dB, dC, acc);
          }
        }
        team_sync<TW>();        // every lane has read the tables before the next root rewrites them
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[i] += __shfl_xor(acc[i], o);
  }
  // one value per wave: lane 0 of each wave adds its wave's sums
  if ((threadIdx.x & 63) == 0) {
    const int atc = A.shell_atom[ket.sa], atd = A.shell_atom[ket.sb];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      atomic_add(&A.grad[3 * atc + d], acc[6 + d]);
      atomic_add(&A.grad[3 * atd + d], -(acc[d] + acc[3 + d] + acc[6 + d]));
      gab[d] += acc[d];
      gab[3 + d] += acc[3 + d];
    }
  }
}

// One unit (bra pair, slice of its kets of the class) per workgroup at a time: lanes (lane
// path) or waves (wave path) take the kets; the bra centres' sums are added once per unit.
template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(256) void k_grad(GradArgs A) {
  using C = GradCfg<LA, LB, LC, LD>;
  constexpr int cb = pair_class(LA, LB), ck = pair_class(LC, LD);
  constexpr int NTEAM = C::LANE ? 1 : 4 / C::TW;
  __shared__ double sw[C::LANE ? 1 : NTEAM * C::WAVE_LDS];
  __shared__ int s_unit;
  const int tid = threadIdx.x;
  const int nunits = min(*A.nunits, A.units_cap);
  for (;;) {
    if (tid == 0) s_unit = atomicAdd(A.next, 1);
    __syncthreads();
    const int u = s_unit;
    __syncthreads();
    if (u >= nunits) break;
    const int2 unit = A.units[u];
    const int bi = unit.x;
    const size_t sg = (size_t)bi * NPAIRCLASS + ck;
    const long long n = A.segcnt[sg];
    const long long lo = (long long)unit.y * A.slice, hi = min(lo + (long long)A.slice, n);
    const int *kl = A.kets + A.class_off[qclass_index(cb, ck)] + A.segoff[sg];
    const Pair bra = A.pairs[bi];
    double gab[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (C::LANE) {
      for (long long k = lo + tid; k < hi; k += blockDim.x) grad_lane_quartet<LA, LB, LC, LD>(A, bra, bi, kl[k], gab);
    } else {
      const int team = tid / (64 * C::TW);
      // every team runs the same number of iterations (a team's barriers need all its lanes)
      for (long long k0 = lo; k0 < hi; k0 += NTEAM) {
        const long long k = k0 + team;
        if (k < hi) grad_team_quartet<LA, LB, LC, LD>(A, bra, bi, kl[k], sw + team * C::WAVE_LDS, gab);
      }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) gab[i] += __shfl_xor(gab[i], o);
    }
    if ((tid & 63) == 0) {
      const int ata = A.shell_atom[bra.sa], atb = A.shell_atom[bra.sb];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (gab[d] != 0.0) atomic_add(&A.grad[3 * ata + d], gab[d]);
        if (gab[3 + d] != 0.0) atomic_add(&A.grad[3 * atb + d], gab[3 + d]);
      }
    }
  }
}

}  // namespace jk

namespace jk {
constexpr int GRAD_LMAX = 3;   // gradient kernels exist for shells up to f
typedef hipError_t (*grad_launch_fn)(const GradArgs &args, int grid, hipStream_t stream);
void register_grad(grad_launch_fn *table);   // [NQCLASS]; null where a class has l > GRAD_LMAX
void register_grad_f(grad_launch_fn *table);  // the classes whose bra has an f shell (own unit)
}  // namespace jk
