// Device building blocks of the J/K build on gfx950 (included by the class translation units).
//
// ERI evaluation follows the Rys quadrature of the paper (section 2): for a primitive
// quartet [ab|cd] the integral is a sum over N = floor((la+lb+lc+ld)/2) + 1 roots of
// the product of three 2D integrals. Here the 2D integrals G(e, f) (e quanta on A, f on C)
// come from the Rys two-dimensional recurrence in the variable u = t^2:
//   G(e+1, f) = C00 G(e,f) + e B10 G(e-1,f) + f B00 G(e,f-1)
//   G(e, f+1) = C00' G(e,f) + f B01 G(e,f-1) + e B00 G(e-1,f)
//   B00 = u / (2(p+q)),  B10 = (1 - u q/(p+q)) / (2p),  B01 = (1 - u p/(p+q)) / (2q)
//   C00 = (P-A) - u q/(p+q) (P-Q),  C00' = (Q-C) + u p/(p+q) (P-Q)
// with the Rys weight and the prefactor 2 pi^(5/2) / (p q sqrt(p+q)) K_ab K_cd folded into
// the z direction (paper section 3 folds weights and coefficients into the 2D integrals).
// Products are accumulated over primitives at the [e0|f0] level (e = a + k on centre A,
// f = c + k' on centre C); the transfer to (ab|cd) is applied once per contracted quartet
// with the binomial form of the horizontal relation
//   (a b| = sum_k C(b,k) (A-B)^(b-k) (a+k, 0|   (componentwise), and likewise for |c d).
#pragma once
#include <hip/hip_runtime.h>

#include "jk_common.h"

#define RYS_STORAGE static __device__ const
#include "rys_table.h"
#define BOYS_STORAGE static __device__ const
#include "boys_grid.h"
#undef BOYS_STORAGE

namespace jk {

// ------------------------------------------------------------------ Cartesian tables
struct CartTable {
  int x[165], y[165], z[165];
  int start[10];          // first flat index of each total degree 0..8 (start[9] = 165)
  int idx[9][9][9];       // flat index of (x, y, z)
};

constexpr CartTable make_cart_table() {
  CartTable t{};
  int n = 0;
  for (int L = 0; L <= 8; ++L) {
    t.start[L] = n;
    for (int ax = L; ax >= 0; --ax)
      for (int ay = L - ax; ay >= 0; --ay) {
        t.x[n] = ax; t.y[n] = ay; t.z[n] = L - ax - ay;
        t.idx[ax][ay][L - ax - ay] = n;
        ++n;
      }
  }
  t.start[9] = n;
  return t;
}

static constexpr CartTable CT = make_cart_table();
static __constant__ CartTable CTD = make_cart_table();   // for run-time indexing

// flat index of the component (x, y, z) in the table above, by arithmetic (no table load)
__host__ __device__ __forceinline__ constexpr int cart_flat(int x, int y, int z) {
  const int L = x + y + z;
  return L * (L + 1) * (L + 2) / 6 + (L - x) * (L - x + 1) / 2 + (L - x - y);
}

constexpr __host__ __device__ int range_count(int lo, int hi) {  // components of degrees lo..hi
  int n = 0;
  for (int L = lo; L <= hi; ++L) n += ncart(L);
  return n;
}

constexpr __host__ __device__ int binom(int n, int k) {
  int r = 1;
  for (int i = 0; i < k; ++i) r = r * (n - i) / (i + 1);
  return r;
}

constexpr double PI_2P5_X2 = 34.98683665524972;   // 2 pi^(5/2)

// ------------------------------------------------------------------ Rys roots and weights
// All N roots for one T (compile-time N). Interval k = floor(T) of width 1 carries a
// degree-RYS_DEG polynomial in s = 2(T - k) - 1 per root and weight; beyond RYS_TMAX[N]
// the Gauss-Hermite limit u = s^2 / T, w = W / sqrt(T) holds to double precision.
template <int N>
__device__ __forceinline__ void rys_roots_table(double T, double (&u)[N], double (&w)[N]) {
  if (T >= (double)RYS_TMAX[N]) {
    const double it = 1.0 / T;
    const double isq = sqrt(it);
#pragma unroll
    for (int n = 0; n < N; ++n) {
      u[n] = RYS_HERM_S2[RYS_HOFF[N] + n] * it;
      w[n] = RYS_HERM_W[RYS_HOFF[N] + n] * isq;
    }
  } else {
    const int k = min(max((int)T, 0), RYS_TMAX[N] - 1);   // T is finite and >= 0; the clamp only guards the table
    const double s = 2.0 * (T - (double)k) - 1.0;
    const double *c = RYS_COEF + RYS_OFF[N] + k * (N * 2 * (RYS_DEG + 1));
#pragma unroll
    for (int n = 0; n < N; ++n) {
      const double *cu = c + n * 2 * (RYS_DEG + 1);
      const double *cw = cu + (RYS_DEG + 1);
      double pu = cu[RYS_DEG], pw = cw[RYS_DEG];
#pragma unroll
      for (int d = RYS_DEG - 1; d >= 0; --d) {
        pu = fma(pu, s, cu[d]);
        pw = fma(pw, s, cw[d]);
      }
      u[n] = pu;
      w[n] = pw;
    }
  }
}

// Boys function F_m(T) = int_0^1 t^(2m) exp(-T t^2) dt for m = 0..M (M <= 3), the moments of
// the Rys weight. T < 1: F_M from its Taylor series in T, then the downward relation
// F_(m-1) = (2T F_m + exp(-T)) / (2m-1); T >= 1: F_0 = sqrt(pi/T) erf(sqrt(T)) / 2 and the upward
// relation F_(m+1) = ((2m+1) F_m - exp(-T)) / (2T), stable for T >= 1 and m <= 3.
template <int M>
__host__ __device__ __forceinline__ void boys_low(double T, double (&F)[M + 1]) {
  if (T < 1.0) {
    // F_M(T) = sum_k (-T)^k / (k! (2M+2k+1)); 19 terms reach 1e-17 at T = 1
    double term = 1.0, s = 1.0 / (2 * M + 1);
#pragma unroll
    for (int k = 1; k <= 19; ++k) {
      term *= -T / k;
      s = fma(term, 1.0 / (2 * M + 2 * k + 1), s);
    }
    F[M] = s;
    const double e = exp(-T);
#pragma unroll
    for (int m = M; m > 0; --m) F[m - 1] = (2.0 * T * F[m] + e) / (2 * m - 1);
  } else {
    const double st = sqrt(T);
    const double e = exp(-T);
    const double h = 0.5 / T;
    F[0] = 0.88622692545275801365 / st * erf(st);        // sqrt(pi)/2
#pragma unroll
    for (int m = 0; m < M; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) * h;
  }
}

// Closed-form Rys rules for N = 1, 2 from the moments F_0..F_(2N-1): the N-point Gauss rule
// of the weight whose moments they are (N = 1: u = F1/F0, w = F0; N = 2: the two zeros of the
// monic quadratic orthogonal to 1 and u, and the weights that reproduce F0 and F1).
template <int N>
__host__ __device__ __forceinline__ void rys_closed(double T, double (&u)[N], double (&w)[N]) {
  static_assert(N == 1 || N == 2, "closed form only for one or two roots");
  if constexpr (N == 1) {
    double F[2];
    boys_low<1>(T, F);
    u[0] = F[1] / F[0];
    w[0] = F[0];
  } else {
    double F[4];
    boys_low<3>(T, F);
    const double det = F[0] * F[2] - F[1] * F[1];
    const double c1 = (F[1] * F[2] - F[0] * F[3]) / det;       // u^2 + c1 u + c0
    const double c0 = (F[1] * F[3] - F[2] * F[2]) / det;
    const double disc = sqrt(c1 * c1 - 4.0 * c0);
    // stable pair of roots of u^2 + c1 u + c0 (c1 < 0)
    const double big = 0.5 * (-c1 + disc);
    const double small = c0 / big;
    u[0] = small;
    u[1] = big;
    w[0] = (F[1] - big * F[0]) / (small - big);
    w[1] = F[0] - w[0];
  }
}

// One- and two-root rules for 0 <= T < RYS_TMAX[N] from the Boys moments F_0..F_(2N-1)(T),
// each taken from the grid point T_i = i/8 nearest to T by its Taylor series (dF_m/dT =
// -F_(m+1), nine terms, relative remainder < 5e-17), then the Gauss rule of those moments as
// in rys_closed. grid: BOYS_GRID (device) or its host copy.
template <int N>
__host__ __device__ __forceinline__ void rys_taylor(double T, const double *grid, double (&u)[N], double (&w)[N]) {
  static_assert(N == 1 || N == 2, "grid rule only for one or two roots");
  constexpr int K = 9;                                // Taylor terms
  const int i = (int)(T * BOYS_DT_INV + 0.5);         // T in [0, RYS_TMAX[N]) -> i <= 400
  const double x = (double)i * (1.0 / BOYS_DT_INV) - T;
  const double *f = grid + i * BOYS_NM;
  double g[2 * N + K - 1];
#pragma unroll
  for (int k = 0; k < 2 * N + K - 1; ++k) g[k] = f[k];
  double xk[K];
#pragma unroll
  for (int k = 1; k < K; ++k) xk[k] = x * (1.0 / k);
  double F[2 * N];
#pragma unroll
  for (int m = 0; m < 2 * N; ++m) {
    double v = g[m + K - 1];
#pragma unroll
    for (int k = K - 1; k >= 1; --k) v = fma(xk[k], v, g[m + k - 1]);
    F[m] = v;
  }
  if constexpr (N == 1) {
    u[0] = F[1] / F[0];
    w[0] = F[0];
  } else {
    // zeros of u^2 + c1 u + c0 (the monic quadratic orthogonal to 1 and u), two divisions:
    // small = c0 / big and w0 = (big F0 - F1) / (big - small) share 1 / (big disc), big - small = disc
    const double idet = 1.0 / (F[0] * F[2] - F[1] * F[1]);
    const double c1 = (F[1] * F[2] - F[0] * F[3]) * idet;
    const double c0 = (F[1] * F[3] - F[2] * F[2]) * idet;
    const double disc = sqrt(c1 * c1 - 4.0 * c0);
    const double big = 0.5 * (-c1 + disc);
    const double r = 1.0 / (big * disc);
    u[0] = c0 * disc * r;
    u[1] = big;
    w[0] = (big * F[0] - F[1]) * big * r;
    w[1] = F[0] - w[0];
  }
}

// All N roots (N = 1, 2) by the grid rule, the Gauss-Hermite limit beyond RYS_TMAX[N]. grid:
// BOYS_GRID, or a copy of it in LDS.
template <int N>
__device__ __forceinline__ void rys_low(double T, double (&u)[N], double (&w)[N], const double *grid = BOYS_GRID) {
  if (T >= (double)RYS_TMAX[N]) {
    const double it = 1.0 / T;
    const double isq = sqrt(it);
#pragma unroll
    for (int n = 0; n < N; ++n) {
      u[n] = RYS_HERM_S2[RYS_HOFF[N] + n] * it;
      w[n] = RYS_HERM_W[RYS_HOFF[N] + n] * isq;
    }
  } else {
    rys_taylor<N>(T, grid, u, w);
  }
}

// One root n (run-time) of the N-point rule (table).
// coef: the N-root block of RYS_COEF (RYS_COEF + RYS_OFF[N], or a copy of it in LDS).
template <int N>
__device__ __forceinline__ void rys_root1(double T, int n, double &u, double &w, const double *coef = RYS_COEF + RYS_OFF[N]) {
  if (T >= (double)RYS_TMAX[N]) {
    const double it = 1.0 / T;
    u = RYS_HERM_S2[RYS_HOFF[N] + n] * it;
    w = RYS_HERM_W[RYS_HOFF[N] + n] * sqrt(it);
  } else {
    const int k = min(max((int)T, 0), RYS_TMAX[N] - 1);
    const double s = 2.0 * (T - (double)k) - 1.0;
    const double *cu = coef + k * (N * 2 * (RYS_DEG + 1)) + n * 2 * (RYS_DEG + 1);
    const double *cw = cu + (RYS_DEG + 1);
    double pu = cu[RYS_DEG], pw = cw[RYS_DEG];
#pragma unroll
    for (int d = RYS_DEG - 1; d >= 0; --d) {
      pu = fma(pu, s, cu[d]);
      pw = fma(pw, s, cw[d]);
    }
    u = pu;
    w = pw;
  }
}

// The table the roots of an N-point rule read in the lane bodies: the Boys grid (N <= 2, grid
// rule) or the N-root block of the interpolation table; its size in doubles.
template <int N>
__device__ __forceinline__ const double *root_table() {
  if constexpr (N <= 2) return BOYS_GRID;
  else return RYS_COEF + RYS_OFF[N];
}
template <int N>
constexpr int root_table_doubles() {
  return N <= 2 ? BOYS_NPT * BOYS_NM : RYS_OFF[N + 1] - RYS_OFF[N];
}

// ------------------------------------------------------------------ 2D recurrence
template <int E, int F, typename R = double>
__device__ __forceinline__ void vrr2d(R (&G)[E + 1][F + 1], R g00, R c00, R c00p, R b10, R b01, R b00) {
  G[0][0] = g00;
  if constexpr (E > 0) G[1][0] = c00 * g00;
#pragma unroll
  for (int e = 1; e < E; ++e) G[e + 1][0] = fma(c00, G[e][0], (R)e * b10 * G[e - 1][0]);
#pragma unroll
  for (int f = 0; f < F; ++f) {
#pragma unroll
    for (int e = 0; e <= E; ++e) {
      R v = c00p * G[e][f];
      if (f > 0) v = fma((R)f * b01, G[e][f - 1], v);
      if (e > 0) v = fma((R)e * b00, G[e - 1][f], v);
      G[e][f + 1] = v;
    }
  }
}

// The same table written to dst[e * (F + 1) + f] (LDS) column by column, so that only three
// columns are live in registers (the workgroup bodies hold their accumulators meanwhile).
template <int E, int F>
__device__ __forceinline__ void vrr2d_store(double *dst, double g00, double c00, double c00p, double b10, double b01,
                                            double b00) {
  double prev[E + 1], cur[E + 1];
  cur[0] = g00;
  if constexpr (E > 0) cur[1] = c00 * g00;
#pragma unroll
  for (int e = 1; e < E; ++e) cur[e + 1] = fma(c00, cur[e], (double)e * b10 * cur[e - 1]);
#pragma unroll
  for (int e = 0; e <= E; ++e) {
    dst[e * (F + 1)] = cur[e];
    prev[e] = 0.0;
  }
#pragma unroll
  for (int f = 0; f < F; ++f) {
    double nxt[E + 1];
#pragma unroll
    for (int e = 0; e <= E; ++e) {
      double v = c00p * cur[e];
      if (f > 0) v = fma((double)f * b01, prev[e], v);
      if (e > 0) v = fma((double)e * b00, cur[e - 1], v);
      nxt[e] = v;
      dst[e * (F + 1) + f + 1] = v;
    }
#pragma unroll
    for (int e = 0; e <= E; ++e) {
      prev[e] = cur[e];
      cur[e] = nxt[e];
    }
  }
}

// Per-primitive-quartet scalars shared by the roots.
struct PrimQuartet {
  double p, q, ip, iq, pq_inv, PQ[3], PA[3], QC[3], pref, T;
};

__device__ __forceinline__ void prim_quartet(const PrimPair &b, const PrimPair &k, const double *A, const double *C,
                                             PrimQuartet &o) {
  o.p = b.p;
  o.q = k.p;
  o.ip = b.ip;
  o.iq = k.ip;
  // one reciprocal square root gives both 1/(p+q) and the 1/sqrt(p+q) of the prefactor
  const double r = rsqrt(b.p + k.p);
  o.pq_inv = r * r;
  o.PQ[0] = b.Px - k.Px; o.PQ[1] = b.Py - k.Py; o.PQ[2] = b.Pz - k.Pz;
  o.PA[0] = b.Px - A[0]; o.PA[1] = b.Py - A[1]; o.PA[2] = b.Pz - A[2];
  o.QC[0] = k.Px - C[0]; o.QC[1] = k.Py - C[1]; o.QC[2] = k.Pz - C[2];
  const double rho = b.p * k.p * o.pq_inv;
  o.T = rho * (o.PQ[0] * o.PQ[0] + o.PQ[1] * o.PQ[1] + o.PQ[2] * o.PQ[2]);
  o.pref = PI_2P5_X2 * (b.ip * k.ip) * r * (b.K * k.K);
}

// Symmetry factor of a unique shell quartet: 1 / |stabiliser| in the eight-fold group.
__device__ __forceinline__ double sym_factor(const Pair &bra, const Pair &ket, int bi, int ki) {
  double s = 1.0;
  if (bra.sa == bra.sb) s *= 0.5;
  if (ket.sa == ket.sb) s *= 0.5;
  if (bi == ki) s *= 0.5;
  return s;
}

__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }

__device__ __forceinline__ void atomic_max_nonneg(double *p, double v) {
  atomicMax(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v));
}

}  // namespace jk
