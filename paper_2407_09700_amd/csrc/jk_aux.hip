// Auxiliary kernels of the J/K build: density transform, block maxima, screening into
// per-class quartet lists, and the final symmetrise + spherical transform.
#include <hip/hip_runtime.h>

#include "jk_aux.h"
#include "jk_device.h"

namespace jk {

// molecule of a flat element index, from the [nmol+1] prefix offsets (binary search)
__device__ __forceinline__ int mol_of(const long long *off, int nmol, long long t) {
  int lo = 0, hi = nmol - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// D_cart[a][b] = sum_{mu in shell(a), nu in shell(b)} T[mu][a] D[mu][nu] T[nu][b]
// (T = identity for Cartesian shells): the density in the Cartesian components, so that
// digestion in the Cartesian basis followed by J = T Jc T^T reproduces the spherical result.
__global__ void k_dcart(ShellInfo S, const double *__restrict__ D, double *__restrict__ Dc, double *__restrict__ Dp) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < S.nc2_tot;
       t += (long long)gridDim.x * blockDim.x) {
    const int m = mol_of(S.mc_off, S.nmol, t);
    const int nc = S.cbase[m + 1] - S.cbase[m], nao = S.abase[m + 1] - S.abase[m];
    const long long r = t - S.mc_off[m];
    const int a = (int)(r / nc), b = (int)(r % nc);
    const int sa = S.cart2shell[S.cbase[m] + a], sb = S.cart2shell[S.cbase[m] + b];
    const int ia = a - S.cart_off[sa], ib = b - S.cart_off[sb];
    const int la = S.l[sa], lb = S.l[sb];
    const bool pa = S.pure[sa] && la >= 2, pb = S.pure[sb] && lb >= 2;
    const int ma = pa ? 2 * la + 1 : 1, mb = pb ? 2 * lb + 1 : 1;
    const double *Ta = pa ? S.tsph + S.toff[la] : nullptr;
    const double *Tb = pb ? S.tsph + S.toff[lb] : nullptr;
    const int na = ncart(la), nb = ncart(lb);
    const double *Dm = D + S.mf_user[m];
    double v = 0.0;
    for (int i = 0; i < ma; ++i) {
      const int mu = S.ao_off[sa] + (pa ? i : ia);
      const double ta = pa ? Ta[i * na + ia] : 1.0;
      if (ta == 0.0) continue;
      double acc = 0.0;
      for (int k = 0; k < mb; ++k) {
        const int nu = S.ao_off[sb] + (pb ? k : ib);
        const double tb = pb ? Tb[k * nb + ib] : 1.0;
        acc = fma(Dm[(size_t)mu * nao + nu], tb, acc);
      }
      v = fma(ta, acc, v);
    }
    Dc[t] = v;
    // the rows of shell sa as one panel stored column by column: element (ia, b) of the panel at
    // b * na + ia, so the block of any shell pair is one contiguous run
    if (Dp) Dp[S.mc_off[m] + (long long)S.cart_off[sa] * nc + (long long)b * na + ia] = v;
  }
}

// Pblk[i][j] = max |D_cart| over the block of shells i, j (per molecule); *gmax = overall max.
__global__ void k_blockmax(ShellInfo S, const double *__restrict__ Dc, double *__restrict__ Pblk, double *gmax) {
  double local = 0.0;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < S.ns2_tot;
       t += (long long)gridDim.x * blockDim.x) {
    const int m = mol_of(S.ps_off, S.nmol, t);
    const int ns = S.sbase[m + 1] - S.sbase[m], nc = S.cbase[m + 1] - S.cbase[m];
    const long long r = t - S.ps_off[m];
    const int i = S.sbase[m] + (int)(r / ns), j = S.sbase[m] + (int)(r % ns);
    const int na = ncart(S.l[i]), nb = ncart(S.l[j]);
    const double *Dm = Dc + S.mc_off[m];
    double mx = 0.0;
    for (int a = 0; a < na; ++a)
      for (int b = 0; b < nb; ++b) mx = fmax(mx, fabs(Dm[(size_t)(S.cart_off[i] + a) * nc + S.cart_off[j] + b]));
    Pblk[t] = mx;
    local = fmax(local, mx);
  }
  atomic_max_nonneg(gmax, local);
}

// pairP[k] = Pblk of kept pair k's own two shells (read by the screen for every ket; one
// coalesced load instead of a scattered one into the molecule's block-maximum matrix).
__global__ void k_pairp(ScreenArgs A) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= A.npairs) return;
  const int m = A.pair_mol[k];
  const int sb0 = A.sbase[m], ns = A.sbase[m + 1] - sb0;
  A.pairP[k] = A.Pblk[A.ps_off[m] + (size_t)(A.pair_sa[k] - sb0) * ns + (A.pair_sb[k] - sb0)];
}

// Number of ket pairs of one class that can pass the screen for one bra pair, under
// the global density bound: kets are sorted by I descending, so they form a prefix.
__device__ __forceinline__ int ket_prefix(const double *__restrict__ Iket, int nket, double Ibra, double pglob,
                                          double tau) {
  if (tau <= 0.0) return nket;
  const double prod = Ibra * pglob;
  if (!(prod > 0.0)) return 0;
  int lo = 0, hi = nket;          // first k with Ibra*Ik*pglob < tau
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (Ibra * Iket[mid] * pglob >= tau) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Candidate kets of bra pair i in one bin (kets of one class, molecule and contraction
// length, sorted by I descending): the prefix that can pass the screen under the global
// density bound; in the bra's own class only kets with index <= i (unique quartets).
__device__ __forceinline__ int bin_candidates(const ScreenArgs &A, int bin, int i, bool same_class, double Ib,
                                              double pglob) {
  const int kb = A.bin_beg[bin];
  int nk = A.bin_beg[bin + 1] - kb;
  if (same_class) {
    if (kb > i) return 0;
    nk = min(nk, i - kb + 1);
  }
  return ket_prefix(A.pairI + kb, nk, Ib, pglob, A.tau);
}

// Segments: for every bra pair and ket class, room for the ket prefixes (one per bin) that
// can pass the screen under the global density bound. Each workgroup adds its per-class
// totals with one global atomic per class and hands out offsets inside its block from LDS.
__global__ __launch_bounds__(256) void k_capacity(ScreenArgs A) {
  __shared__ unsigned long long s_tot[NQCLASS], s_base[NQCLASS];
  for (int t = threadIdx.x; t < NQCLASS; t += blockDim.x) s_tot[t] = 0ull;
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int loc[NPAIRCLASS];
  int cb = -1;
  if (i < A.npairs) {
    cb = A.pair_cls[i];
    const int m = A.pair_mol[i];
    const double Ib = A.pairI[i];
    const double pglob = A.gfix > 0.0 ? A.gfix : *A.gmax * A.gscale;
    for (int ck = 0; ck < NPAIRCLASS; ++ck) {
      loc[ck] = 0;
      if (ck > cb) continue;
      int n = 0;
      const int b1 = A.cm_bin[ck * (A.nmol + 1) + m + 1];
      for (int bin = A.cm_bin[ck * (A.nmol + 1) + m]; bin < b1; ++bin) n += bin_candidates(A, bin, i, ck == cb, Ib, pglob);
      if (n > 0) loc[ck] = (int)atomicAdd(&s_tot[qclass_index(cb, ck)], (unsigned long long)n);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < NQCLASS; t += blockDim.x)
    s_base[t] = s_tot[t] ? atomicAdd(&A.cap[t], s_tot[t]) : 0ull;
  __syncthreads();
  if (i < A.npairs)
    for (int ck = 0; ck <= cb; ++ck) A.segoff[(size_t)i * NPAIRCLASS + ck] = (int)(s_base[qclass_index(cb, ck)] + loc[ck]);
}

// Room of every class region of the work list for this build. The regions (offsets and
// capacities) were laid out when the plan sized its lists; a class whose candidates exceed its
// capacity keeps what fits and raises the overflow flag (the build is then incomplete, which
// the host reports when it checks the plan).
__global__ void k_class_room(const unsigned long long *cap, const long long *capc, long long *room, int *overflow) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= NQCLASS) return;
  const long long n = (long long)cap[c];
  room[c] = n < capc[c] ? n : capc[c];
  if (n > capc[c]) *overflow = 1;
}

// One wave per bra pair: tests the candidates of every ket class with the exact
// predicate I_ab I_cd P >= tau (P = max |D_cart| over the six shell-pair blocks), writes the
// kept kets to the (bra, class) segment -- bin after bin, so that kets of equal contraction
// length sit next to each other -- and its count.
__global__ __launch_bounds__(256) void k_screen(ScreenArgs A) {
  __shared__ int s_cnt[NQCLASS], s_c32[NQCLASS];
  __shared__ unsigned long long s_np[NQCLASS], s_np32[NQCLASS];
  __shared__ int s_pref[4][MAX_BINS + 1];          // per wave: candidate prefix over the bins
  for (int t = threadIdx.x; t < NQCLASS; t += blockDim.x) { s_cnt[t] = 0; s_c32[t] = 0; s_np[t] = 0ull; s_np32[t] = 0ull; }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  int *pref = s_pref[threadIdx.x >> 6];
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (i < A.npairs) {
    const double tau = A.tau;
    const double pglob = *A.gmax;
    const int cb = A.pair_cls[i];
    const int m = A.pair_mol[i];
    const double Ib = A.pairI[i];
    const int sb0 = A.sbase[m];
    const int ns = A.sbase[m + 1] - sb0;
    const double *Pm = A.Pblk + A.ps_off[m];
    const int sa = A.pair_sa[i] - sb0, sb = A.pair_sb[i] - sb0;
    const double *Pa = Pm + (size_t)sa * ns;
    const double *Pb = Pm + (size_t)sb * ns;
    const double pab = Pa[sb];
    const unsigned long long nppb = (unsigned long long)A.pair_npp[i];
    for (int ck = 0; ck <= cb; ++ck) {
      const int b0 = A.cm_bin[ck * (A.nmol + 1) + m];
      const int nb = A.cm_bin[ck * (A.nmol + 1) + m + 1] - b0;   // <= MAX_BINS (plan creation)
      // candidates per bin (one lane per bin), exclusive prefix through the wave
      const int mine = lane < nb ? bin_candidates(A, b0 + lane, i, ck == cb, Ib, pglob) : 0;
      int incl = mine;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
      }
      if (lane < nb) pref[lane + 1] = incl;
      if (lane == 0) pref[0] = 0;
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
      int n = __shfl(incl, 63);
      const int qc = qclass_index(cb, ck);
      const long long so = A.segoff[(size_t)i * NPAIRCLASS + ck];
      {                                       // never write past the class region
        const long long left = A.room[qc] - so;
        if (left < n) n = left > 0 ? (int)left : 0;
      }
      int *out = A.kets + A.class_off[qc] + so;
      const double cut = ((A.f32_classes[qc >> 6] >> (qc & 63)) & 1ull) ? A.fp32_cut : 0.0;
      int kept = 0, kept32 = 0;
      unsigned long long np = 0ull, np32 = 0ull;
      // SU chunks of 64 candidates per pass: the loads of all of them are issued before any is
      // used (two dependent round trips per pass instead of per chunk); the chunks' kept kets are
      // then written in candidate order
      constexpr int SU = 4;
      for (int k0 = 0; k0 < n; k0 += 64 * SU) {
        int kg[SU];
        bool in[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          const int k = k0 + u * 64 + lane;
          in[u] = k < n;
          kg[u] = 0;
          if (in[u]) {
            int lo_b = 0, hi_b = nb - 1;      // last bin with pref[bin] <= k
            while (lo_b < hi_b) {
              const int mid = (lo_b + hi_b + 1) >> 1;
              if (pref[mid] <= k) lo_b = mid; else hi_b = mid - 1;
            }
            kg[u] = A.bin_beg[b0 + lo_b] + (k - pref[lo_b]);
          }
        }
        int sc[SU], sd[SU];
        double ik[SU], pk[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          sc[u] = in[u] ? A.pair_sa[kg[u]] - sb0 : 0;
          sd[u] = in[u] ? A.pair_sb[kg[u]] - sb0 : 0;
          ik[u] = in[u] ? A.pairI[kg[u]] : 0.0;
          pk[u] = in[u] && (A.want & 1) ? A.pairP[kg[u]] : 0.0;
        }
        bool keep[SU], lo[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          // largest density block the quartet's updates read: D[a,b], D[c,d] (Coulomb),
          // D[a,c], D[a,d], D[b,c], D[b,d] (exchange)
          double p = 0.0;
          if (A.want & 1) p = fmax(pab, pk[u]);
          if (A.want & 2) p = fmax(fmax(p, fmax(Pa[sc[u]], Pa[sd[u]])), fmax(Pb[sc[u]], Pb[sd[u]]));
          const double bound = Ib * ik[u] * p;
          keep[u] = in[u] && bound >= tau;
          lo[u] = keep[u] && bound < cut;      // mixed precision: evaluated in FP32
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          if (keep[u]) np += nppb * (unsigned long long)A.pair_npp[kg[u]];
          if (lo[u]) np32 += nppb * (unsigned long long)A.pair_npp[kg[u]];
          // FP64 kets fill the segment from the front, FP32 kets from the back
          const unsigned long long below = (1ull << lane) - 1ull;
          const unsigned long long m64 = __ballot(keep[u] && !lo[u]), m32 = __ballot(lo[u]);
          if (keep[u] && !lo[u]) out[kept + __popcll(m64 & below)] = kg[u];
          if (lo[u]) out[n - 1 - (kept32 + __popcll(m32 & below))] = kg[u];
          kept += __popcll(m64);
          kept32 += __popcll(m32);
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        np += __shfl_xor(np, o);
        np32 += __shfl_xor(np32, o);
      }
      if (lane == 0) {
        const size_t sg = (size_t)i * NPAIRCLASS + ck;
        A.segcnt[sg] = kept;
        if (A.segcnt32) {
          A.segcnt32[sg] = kept32;
          A.segoff32[sg] = (int)(so + n - kept32);
        }
        if (kept + kept32) {
          atomicAdd(&s_cnt[qc], kept + kept32);
          atomicAdd(&s_np[qc], np);
        }
        if (kept32) {
          atomicAdd(&s_c32[qc], kept32);
          atomicAdd(&s_np32[qc], np32);
        }
      }
      __threadfence_block();              // every lane has read pref before the next class rewrites it
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < NQCLASS; t += blockDim.x)
    if (s_cnt[t]) {
      atomicAdd(&A.count[t], s_cnt[t]);
      atomicAdd(&A.nprim[t], s_np[t]);
      if (s_c32[t]) {
        atomicAdd(&A.count32[t], s_c32[t]);
        atomicAdd(&A.nprim[NQCLASS + t], s_np32[t]);
      }
    }
}

// Jt[ca + a][cb + b] = Coulomb pair buffer (each shell pair owns its block of its molecule's Jt).
__global__ void k_fold(FoldArgs F) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < F.npairs; p += gridDim.x * blockDim.x) {
    const int c = F.pair_cls[p];
    const int beg = F.cls_beg[c], np = F.cls_beg[c + 1] - beg;
    const int na = ncart(F.pair_la[p]), nb = ncart(F.pair_lb[p]);
    const int m = F.pair_mol[p];
    const int nc = F.cbase[m + 1] - F.cbase[m];
    double *Jm = F.Jc + F.mc_off[m];
    for (int a = 0; a < na; ++a)
      for (int b = 0; b < nb; ++b)
        Jm[(size_t)(F.pair_ca[p] + a) * nc + F.pair_cb[p] + b] = F.Jpair[F.jp_off[c] + (long long)(a * nb + b) * np + (p - beg)];
  }
}

// The reverse of k_fold for the density: each kept pair's block of the Cartesian density, laid
// out like the Coulomb pair buffer (element-major within a pair class).
__global__ void k_unfold(FoldArgs F) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < F.npairs; p += gridDim.x * blockDim.x) {
    const int c = F.pair_cls[p];
    const int beg = F.cls_beg[c], np = F.cls_beg[c + 1] - beg;
    const int na = ncart(F.pair_la[p]), nb = ncart(F.pair_lb[p]);
    const int m = F.pair_mol[p];
    const int nc = F.cbase[m + 1] - F.cbase[m];
    const double *Dm = F.Dc + F.mc_off[m];
    for (int a = 0; a < na; ++a)
      for (int b = 0; b < nb; ++b)
        F.Dpair[F.jp_off[c] + (long long)(a * nb + b) * np + (p - beg)] = Dm[(size_t)(F.pair_ca[p] + a) * nc + F.pair_cb[p] + b];
  }
}

// J[mu][nu] = sum_{a,b} T[mu][a] (Jc[a][b] + Jc[b][a]) T[nu][b], same for K (per molecule).
__global__ void k_finalize(ShellInfo S, const double *__restrict__ Jc, const double *__restrict__ Kc,
                           double *__restrict__ J, double *__restrict__ K) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < S.nf2_tot;
       t += (long long)gridDim.x * blockDim.x) {
    const int m = mol_of(S.mf_off, S.nmol, t);
    const int nao = S.abase[m + 1] - S.abase[m], nc = S.cbase[m + 1] - S.cbase[m];
    const long long r = t - S.mf_off[m];
    const int mu = (int)(r / nao), nu = (int)(r % nao);
    const int si = S.ao2shell[S.abase[m] + mu], sj = S.ao2shell[S.abase[m] + nu];
    const int im = mu - S.ao_off[si], jn = nu - S.ao_off[sj];
    const int li = S.l[si], lj = S.l[sj];
    const bool pi = S.pure[si] && li >= 2, pj = S.pure[sj] && lj >= 2;
    const int ni = ncart(li), nj = ncart(lj);
    const double *Ti = pi ? S.tsph + S.toff[li] + im * ni : nullptr;
    const double *Tj = pj ? S.tsph + S.toff[lj] + jn * nj : nullptr;
    const int a0 = pi ? 0 : im, a1 = pi ? ni : im + 1;
    const int b0 = pj ? 0 : jn, b1 = pj ? nj : jn + 1;
    const double *Jm = Jc + S.mc_off[m], *Km = Kc + S.mc_off[m];
    double vj = 0.0, vk = 0.0;
    for (int a = a0; a < a1; ++a) {
      const double ta = pi ? Ti[a] : 1.0;
      if (ta == 0.0) continue;
      double rj = 0.0, rk = 0.0;
      const size_t ra = (size_t)(S.cart_off[si] + a);
      for (int b = b0; b < b1; ++b) {
        const double tb = pj ? Tj[b] : 1.0;
        const size_t rb = (size_t)(S.cart_off[sj] + b);
        rj = fma(tb, Jm[ra * nc + rb] + Jm[rb * nc + ra], rj);
        rk = fma(tb, Km[ra * nc + rb] + Km[rb * nc + ra], rk);
      }
      vj = fma(ta, rj, vj);
      vk = fma(ta, rk, vk);
    }
    if (J) J[S.mf_user[m] + r] = vj;
    if (K) K[S.mf_user[m] + r] = vk;
  }
}

__global__ void k_fill_u64(unsigned long long *p, long long n, unsigned long long v) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
    p[t] = v;
}

// Work units of one integral launch: every bra pair of [bra_beg, bra_end) with kets in the
// launch's ket classes (bit ck of mask) and segment parts (parts: 1 FP64, 2 FP32) gives
// ceil(kets / slice) units (bra, slice index).
// Units are handed out with one atomic per wave; their order does not matter.
__global__ void k_units(const int *__restrict__ segcnt, const int *__restrict__ segcnt32, int bra_beg, int bra_end,
                        int mask, int parts, int slice, int2 *__restrict__ units, int units_cap, int *nunits,
                        int *overflow) {
  const int lane = threadIdx.x & 63;
  const int bi = bra_beg + blockIdx.x * blockDim.x + threadIdx.x;
  int n = 0;
  if (bi < bra_end) {
    long long tot = 0;
    for (int ck = 0; ck < NPAIRCLASS; ++ck)
      if ((mask >> ck) & 1) {
        if (parts & 1) tot += segcnt[(size_t)bi * NPAIRCLASS + ck];
        if ((parts & 2) && segcnt32) tot += segcnt32[(size_t)bi * NPAIRCLASS + ck];
      }
    n = (int)((tot + slice - 1) / slice);
  }
  int incl = n;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o);
    if (lane >= o) incl += v;
  }
  const int wave_tot = __shfl(incl, 63);
  int base = 0;
  if (lane == 63 && wave_tot) base = atomicAdd(nunits, wave_tot);
  base = __shfl(base, 63);
  for (int j = 0; j < n; ++j) {
    const long long at = (long long)base + incl - n + j;
    if (at < units_cap) units[at] = make_int2(bi, j);
    else *overflow = 1;        // only a graph replay (list sized at recording) can get here
  }
}

__global__ void k_fill_i32(int *p, long long n, int v) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
    p[t] = v;
}

static int grid_for(long long n, int block) {
  long long g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (int)g;
}

hipError_t launch_dcart(const ShellInfo &S, const double *D, double *Dc, double *Dp, hipStream_t st) {
  hipLaunchKernelGGL(k_dcart, dim3(grid_for(S.nc2_tot, 256)), dim3(256), 0, st, S, D, Dc, Dp);
  return hipGetLastError();
}
hipError_t launch_blockmax(const ShellInfo &S, const double *Dc, double *Pblk, double *gmax, hipStream_t st) {
  hipLaunchKernelGGL(k_blockmax, dim3(grid_for(S.ns2_tot, 256)), dim3(256), 0, st, S, Dc, Pblk, gmax);
  return hipGetLastError();
}
hipError_t launch_capacity(const ScreenArgs &A, hipStream_t st) {
  hipLaunchKernelGGL(k_capacity, dim3((A.npairs + 255) / 256), dim3(256), 0, st, A);
  return hipGetLastError();
}
hipError_t launch_pairp(const ScreenArgs &A, hipStream_t st) {
  hipLaunchKernelGGL(k_pairp, dim3((A.npairs + 255) / 256), dim3(256), 0, st, A);
  return hipGetLastError();
}
hipError_t launch_screen(const ScreenArgs &A, hipStream_t st) {
  hipLaunchKernelGGL(k_screen, dim3((A.npairs + 3) / 4), dim3(256), 0, st, A);
  return hipGetLastError();
}
hipError_t launch_class_room(const unsigned long long *cap, const long long *capc, long long *room, int *overflow,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_class_room, dim3(1), dim3(128), 0, st, cap, capc, room, overflow);
  return hipGetLastError();
}
hipError_t launch_fold(const FoldArgs &F, hipStream_t st) {
  hipLaunchKernelGGL(k_fold, dim3(grid_for(F.npairs, 256)), dim3(256), 0, st, F);
  return hipGetLastError();
}
hipError_t launch_unfold(const FoldArgs &F, hipStream_t st) {
  hipLaunchKernelGGL(k_unfold, dim3(grid_for(F.npairs, 256)), dim3(256), 0, st, F);
  return hipGetLastError();
}
hipError_t launch_finalize(const ShellInfo &S, const double *Jc, const double *Kc, double *J, double *K,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(grid_for(S.nf2_tot, 256)), dim3(256), 0, st, S, Jc, Kc, J, K);
  return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long *p, long long n, unsigned long long v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
hipError_t launch_units(const int *segcnt, const int *segcnt32, int bra_beg, int bra_end, int mask, int parts,
                        int slice, int2 *units, int units_cap, int *nunits, int *overflow, hipStream_t st) {
  if (bra_end <= bra_beg) return hipSuccess;
  hipLaunchKernelGGL(k_units, dim3((bra_end - bra_beg + 255) / 256), dim3(256), 0, st, segcnt, segcnt32, bra_beg,
                     bra_end, mask, parts, slice, units, units_cap, nunits, overflow);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int *p, long long n, int v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace jk
