/*
 * jk_oracle.c -- plain CPU oracle for the integral-direct J/K build.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library. It shares no code with the HIP path.
 *
 * What it computes (paper, section 2 and section 3):
 *   (mu nu|la si) = double integral of chi_mu(1) chi_nu(1) / r12 chi_la(2) chi_si(2)
 *   over contracted real basis functions (contraction: section 2, the equation that
 *   sums C_a^i C_b^j C_c^k C_d^l [ab|cd] over primitives), and
 *   J_mu,nu = sum_{la,si} (mu nu|la si) D_la,si,
 *   K_mu,nu = sum_{la,si} (mu la|nu si) D_la,si.
 *
 * Algorithm: NOT Rys quadrature. Primitive integrals come from the Obara-Saika
 * vertical recurrence over the Boys function F_m(T) (Obara & Saika 1986; the
 * electron-transfer-free form of Head-Gordon & Pople 1988), contracted over
 * primitives at the [e0|f0] level and moved to (ab|cd) by the horizontal recurrence
 * (Head-Gordon & Pople 1988). The Boys function is evaluated by its Taylor-type
 * series with downward recursion (small T) or erf plus upward recursion (large T).
 * Spherical functions are obtained by applying caller-supplied Cartesian-to-spherical
 * matrices to every index of the Cartesian block (no other use of them).
 *
 * J/K loops: every ordered shell quartet (i,j,k,l) contributes
 *   J[i,j] += (ij|kl) D[k,l] and K[i,k] += (ij|kl) D[j,l].
 * To avoid evaluating each block eight times the loop runs over unique shell
 * quartets and applies the same updates for every DISTINCT ordered shell tuple in
 * the orbit of the quartet under the 8 index permutations that leave (ij|kl)
 * invariant (section 3 mentions this eight-fold symmetry); the set of ordered tuples
 * visited is therefore exactly the set of all ordered shell quartets.
 *
 * Screening (section 3, Cauchy-Schwarz factor and density-weighted test):
 *   I_ij = max over Cartesian components a in i, b in j of |(ab|ab)|^(1/2),
 *   P(ij|kl) = max |D_cart| over the six shell-pair blocks ij, ik, il, jk, jl, kl,
 *   where D_cart = T^T D T is the density in the Cartesian components.
 *   A quartet is kept iff I_ij > tau, I_kl > tau and I_ij*I_kl*P >= tau.
 *   tau = 0 keeps every quartet whose pair factors are nonzero (exact mode).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC jk_oracle.c -o libjk_oracle.so -lm
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define LMAX 4
#define EMAX (2 * LMAX)                  /* largest |e| on one side of the VRR */
#define MMAX (4 * LMAX)                  /* largest Boys order needed */
#define NCOMP_EMAX 165                   /* number of (ax,ay,az) with ax+ay+az <= 8 */
#define NCOMP_LMAX 35                    /* number of (ax,ay,az) with ax+ay+az <= 4 */

/* ------------------------------------------------------------------ Cartesian indexing */
/* Flat index of (ax,ay,az) among all monomials of total degree <= 8, ordered by total
 * degree, then ax descending, then ay descending. */
static int g_flat[EMAX + 1][EMAX + 1][EMAX + 1];
static int g_comp[NCOMP_EMAX][3];
static int g_level_start[EMAX + 2];
static int g_init = 0;

static void init_tables(void) {
  if (g_init) return;
#pragma omp critical(oracle_init)
  {
    if (!g_init) {
      int n = 0;
      for (int L = 0; L <= EMAX; ++L) {
        g_level_start[L] = n;
        for (int ax = L; ax >= 0; --ax)
          for (int ay = L - ax; ay >= 0; --ay) {
            int az = L - ax - ay;
            g_flat[ax][ay][az] = n;
            g_comp[n][0] = ax; g_comp[n][1] = ay; g_comp[n][2] = az;
            ++n;
          }
      }
      g_level_start[EMAX + 1] = n;
      g_init = 1;
    }
  }
}

static inline int ncart(int l) { return (l + 1) * (l + 2) / 2; }
static inline int nsph(int l, int pure) { return (pure && l >= 2) ? 2 * l + 1 : ncart(l); }

/* ------------------------------------------------------------------ Boys function */
/* F_m(T) = integral_0^1 t^(2m) exp(-T t^2) dt, for m = 0..mmax. */
void oracle_boys(int mmax, double T, double *F) {
  if (T < 1e-300) {
    for (int m = 0; m <= mmax; ++m) F[m] = 1.0 / (2 * m + 1);
    return;
  }
  double e = exp(-T);
  if (T < 45.0) {
    /* F_M(T) = exp(-T) * sum_k (2T)^k / ((2M+1)(2M+3)...(2M+2k+1)), then downward. */
    double term = 1.0 / (2 * mmax + 1), sum = term;
    for (int k = 1; k < 2000; ++k) {
      term *= 2.0 * T / (2 * mmax + 2 * k + 1);
      sum += term;
      if (term < 1e-18 * sum) break;
    }
    F[mmax] = e * sum;
    for (int m = mmax; m > 0; --m) F[m - 1] = (2.0 * T * F[m] + e) / (2 * m - 1);
  } else {
    F[0] = 0.5 * sqrt(M_PI / T) * erf(sqrt(T));
    for (int m = 0; m < mmax; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) / (2.0 * T);
  }
}

/* ------------------------------------------------------------------ basis view */
typedef struct {
  const double *coords;       /* natom x 3 */
  const int *sh_atom, *sh_l, *sh_nprim, *sh_off, *sh_pure;
  const double *pexp, *pcoef;
  const double *tsph;         /* T2 (5x6) | T3 (7x10) | T4 (9x15), row-major */
  int nshell;
} basis_t;

static const double *tsph_of(const basis_t *b, int l) {
  if (l == 2) return b->tsph;
  if (l == 3) return b->tsph + 30;
  if (l == 4) return b->tsph + 30 + 70;
  return NULL;
}

/* ------------------------------------------------------------------ contracted Cartesian ERI block */
/* Workspace for one evaluation (thread private). */
typedef struct {
  double *V;     /* [NCOMP_EMAX][NCOMP_EMAX][MMAX+1] primitive OS table */
  double *E0F0;  /* [NCOMP_EMAX][NCOMP_EMAX] contracted [e0|f0] */
  double *X;     /* bra HRR scratch */
  double *Y;     /* (ab|f0) */
  double *Z;     /* ket HRR scratch */
} work_t;

static void work_alloc(work_t *w) {
  w->V = (double *)malloc(sizeof(double) * NCOMP_EMAX * NCOMP_EMAX * (MMAX + 1));
  w->E0F0 = (double *)malloc(sizeof(double) * NCOMP_EMAX * NCOMP_EMAX);
  w->X = (double *)malloc(sizeof(double) * NCOMP_EMAX * NCOMP_LMAX);
  w->Y = (double *)malloc(sizeof(double) * 15 * 15 * NCOMP_EMAX);
  w->Z = (double *)malloc(sizeof(double) * NCOMP_EMAX * NCOMP_LMAX);
}
static void work_free(work_t *w) { free(w->V); free(w->E0F0); free(w->X); free(w->Y); free(w->Z); }

#define VIDX(e, f, m) (((size_t)(e) * NCOMP_EMAX + (f)) * (MMAX + 1) + (m))

/* Contracted Cartesian block (ab|cd) for shells (i,j,k,l) in this order.
 * out[a][b][c][d] with components in (ax desc, ay desc) order. */
static void eri_cart(const basis_t *B, int si, int sj, int sk, int sl, work_t *w, double *out) {
  const int la = B->sh_l[si], lb = B->sh_l[sj], lc = B->sh_l[sk], ld = B->sh_l[sl];
  const int E = la + lb, F = lc + ld, M = E + F;
  const double *A = B->coords + 3 * B->sh_atom[si], *Bc = B->coords + 3 * B->sh_atom[sj];
  const double *C = B->coords + 3 * B->sh_atom[sk], *D = B->coords + 3 * B->sh_atom[sl];
  const int ne = g_level_start[E + 1], nf = g_level_start[F + 1];
  double AB2 = 0, CD2 = 0;
  for (int x = 0; x < 3; ++x) { AB2 += (A[x] - Bc[x]) * (A[x] - Bc[x]); CD2 += (C[x] - D[x]) * (C[x] - D[x]); }

  memset(w->E0F0, 0, sizeof(double) * NCOMP_EMAX * NCOMP_EMAX);
  double Fm[MMAX + 1];
  for (int pa = 0; pa < B->sh_nprim[si]; ++pa)
  for (int pb = 0; pb < B->sh_nprim[sj]; ++pb) {
    const double a = B->pexp[B->sh_off[si] + pa], b = B->pexp[B->sh_off[sj] + pb];
    const double ca = B->pcoef[B->sh_off[si] + pa], cb = B->pcoef[B->sh_off[sj] + pb];
    const double zeta = a + b;
    double P[3];
    for (int x = 0; x < 3; ++x) P[x] = (a * A[x] + b * Bc[x]) / zeta;
    const double Kab = exp(-a * b / zeta * AB2);
    for (int pc = 0; pc < B->sh_nprim[sk]; ++pc)
    for (int pd = 0; pd < B->sh_nprim[sl]; ++pd) {
      const double c = B->pexp[B->sh_off[sk] + pc], d = B->pexp[B->sh_off[sl] + pd];
      const double cc = B->pcoef[B->sh_off[sk] + pc], cd = B->pcoef[B->sh_off[sl] + pd];
      const double eta = c + d;
      double Q[3], W[3], PQ2 = 0;
      for (int x = 0; x < 3; ++x) {
        Q[x] = (c * C[x] + d * D[x]) / eta;
        W[x] = (zeta * P[x] + eta * Q[x]) / (zeta + eta);
        PQ2 += (P[x] - Q[x]) * (P[x] - Q[x]);
      }
      const double Kcd = exp(-c * d / eta * CD2);
      const double rho = zeta * eta / (zeta + eta);
      const double pref = 2.0 * pow(M_PI, 2.5) / (zeta * eta * sqrt(zeta + eta)) * Kab * Kcd
                          * ca * cb * cc * cd;
      oracle_boys(M, rho * PQ2, Fm);
      double PA[3], WP[3], QC[3], WQ[3];
      for (int x = 0; x < 3; ++x) {
        PA[x] = P[x] - A[x]; WP[x] = W[x] - P[x];
        QC[x] = Q[x] - C[x]; WQ[x] = W[x] - Q[x];
      }
      const double i2z = 0.5 / zeta, i2e = 0.5 / eta, i2ze = 0.5 / (zeta + eta);
      const double rz = rho / zeta, re = rho / eta;
      /* Obara-Saika VRR: fill [e0|f0]^(m) for |e|<=E, |f|<=F, m <= M-|e|-|f|. */
      for (int ef = 0; ef < nf; ++ef) {
        const int fx = g_comp[ef][0], fy = g_comp[ef][1], fz = g_comp[ef][2];
        const int fL = fx + fy + fz;
        for (int ee = 0; ee < ne; ++ee) {
          const int ex = g_comp[ee][0], ey = g_comp[ee][1], ez = g_comp[ee][2];
          const int eL = ex + ey + ez;
          const int mtop = M - eL - fL;
          if (mtop < 0) continue;
          if (fL == 0) {
            if (eL == 0) {
              for (int m = 0; m <= mtop; ++m) w->V[VIDX(0, 0, m)] = pref * Fm[m];
              continue;
            }
            int e1[3] = {ex, ey, ez};
            int i = (ex > 0) ? 0 : ((ey > 0) ? 1 : 2);
            e1[i] -= 1;                                   /* e = e1 + 1_i */
            const int ie1 = g_flat[e1[0]][e1[1]][e1[2]];
            const int n1 = e1[i];
            int ie2 = -1;
            if (n1 > 0) { int e2[3] = {e1[0], e1[1], e1[2]}; e2[i] -= 1; ie2 = g_flat[e2[0]][e2[1]][e2[2]]; }
            for (int m = 0; m <= mtop; ++m) {
              double v = PA[i] * w->V[VIDX(ie1, 0, m)] + WP[i] * w->V[VIDX(ie1, 0, m + 1)];
              if (n1 > 0) v += n1 * i2z * (w->V[VIDX(ie2, 0, m)] - rz * w->V[VIDX(ie2, 0, m + 1)]);
              w->V[VIDX(ee, 0, m)] = v;
            }
          } else {
            int f1[3] = {fx, fy, fz};
            int i = (fx > 0) ? 0 : ((fy > 0) ? 1 : 2);
            f1[i] -= 1;                                   /* f = f1 + 1_i */
            const int if1 = g_flat[f1[0]][f1[1]][f1[2]];
            const int n1 = f1[i];
            int if2 = -1;
            if (n1 > 0) { int f2[3] = {f1[0], f1[1], f1[2]}; f2[i] -= 1; if2 = g_flat[f2[0]][f2[1]][f2[2]]; }
            const int ne1 = (i == 0) ? ex : ((i == 1) ? ey : ez);
            int iem = -1;
            if (ne1 > 0) { int em[3] = {ex, ey, ez}; em[i] -= 1; iem = g_flat[em[0]][em[1]][em[2]]; }
            for (int m = 0; m <= mtop; ++m) {
              double v = QC[i] * w->V[VIDX(ee, if1, m)] + WQ[i] * w->V[VIDX(ee, if1, m + 1)];
              if (n1 > 0) v += n1 * i2e * (w->V[VIDX(ee, if2, m)] - re * w->V[VIDX(ee, if2, m + 1)]);
              if (ne1 > 0) v += ne1 * i2ze * w->V[VIDX(iem, if1, m + 1)];
              w->V[VIDX(ee, ef, m)] = v;
            }
          }
        }
      }
      /* accumulate the contracted [e0|f0] needed by the HRR: la<=|e|<=E, lc<=|f|<=F */
      for (int ee = g_level_start[la]; ee < ne; ++ee)
        for (int ef = g_level_start[lc]; ef < nf; ++ef)
          w->E0F0[ee * NCOMP_EMAX + ef] += w->V[VIDX(ee, ef, 0)];
    }
  }

  /* HRR on the bra: (a, b+1_i| = (a+1_i, b| + (A_i - B_i) (a, b|, for each f. */
  const int na = ncart(la), nb = ncart(lb), nc = ncart(lc), nd = ncart(ld);
  const double ABv[3] = {A[0] - Bc[0], A[1] - Bc[1], A[2] - Bc[2]};
  const double CDv[3] = {C[0] - D[0], C[1] - D[1], C[2] - D[2]};
  /* Y[(a*nb+b)][f] for la-level a, lb-level b, f over all flat <= F */
  for (int ef = g_level_start[lc]; ef < nf; ++ef) {
    /* X[e][b] with b flat over levels 0..lb, e flat */
    for (int ee = g_level_start[la]; ee < ne; ++ee) w->X[ee * NCOMP_LMAX + 0] = w->E0F0[ee * NCOMP_EMAX + ef];
    for (int bL = 1; bL <= lb; ++bL) {
      for (int ib = g_level_start[bL]; ib < g_level_start[bL + 1]; ++ib) {
        int bv[3] = {g_comp[ib][0], g_comp[ib][1], g_comp[ib][2]};
        int i = (bv[0] > 0) ? 0 : ((bv[1] > 0) ? 1 : 2);
        int bm[3] = {bv[0], bv[1], bv[2]}; bm[i] -= 1;
        const int ibm = g_flat[bm[0]][bm[1]][bm[2]];
        for (int ee = g_level_start[la]; ee < g_level_start[E - bL + 1]; ++ee) {
          int ev[3] = {g_comp[ee][0], g_comp[ee][1], g_comp[ee][2]};
          ev[i] += 1;
          const int iep = g_flat[ev[0]][ev[1]][ev[2]];
          w->X[ee * NCOMP_LMAX + ib] = w->X[iep * NCOMP_LMAX + ibm] + ABv[i] * w->X[ee * NCOMP_LMAX + ibm];
        }
      }
    }
    for (int a = 0; a < na; ++a)
      for (int b = 0; b < nb; ++b)
        w->Y[(a * nb + b) * NCOMP_EMAX + ef] =
            w->X[(g_level_start[la] + a) * NCOMP_LMAX + g_level_start[lb] + b];
  }
  /* HRR on the ket for each (a,b). */
  for (int ab = 0; ab < na * nb; ++ab) {
    for (int ef = g_level_start[lc]; ef < nf; ++ef) w->Z[ef * NCOMP_LMAX + 0] = w->Y[ab * NCOMP_EMAX + ef];
    for (int dL = 1; dL <= ld; ++dL) {
      for (int id = g_level_start[dL]; id < g_level_start[dL + 1]; ++id) {
        int dv[3] = {g_comp[id][0], g_comp[id][1], g_comp[id][2]};
        int i = (dv[0] > 0) ? 0 : ((dv[1] > 0) ? 1 : 2);
        int dm[3] = {dv[0], dv[1], dv[2]}; dm[i] -= 1;
        const int idm = g_flat[dm[0]][dm[1]][dm[2]];
        for (int ef = g_level_start[lc]; ef < g_level_start[F - dL + 1]; ++ef) {
          int fv[3] = {g_comp[ef][0], g_comp[ef][1], g_comp[ef][2]};
          fv[i] += 1;
          const int ifp = g_flat[fv[0]][fv[1]][fv[2]];
          w->Z[ef * NCOMP_LMAX + id] = w->Z[ifp * NCOMP_LMAX + idm] + CDv[i] * w->Z[ef * NCOMP_LMAX + idm];
        }
      }
    }
    for (int c = 0; c < nc; ++c)
      for (int d = 0; d < nd; ++d)
        out[(size_t)ab * nc * nd + c * nd + d] = w->Z[(g_level_start[lc] + c) * NCOMP_LMAX + g_level_start[ld] + d];
  }
}

/* Apply the Cartesian-to-spherical matrix of each pure shell to the matching index of
 * a block. in: [n0][n1][n2][n3] Cartesian sizes; out: final sizes. tmp: scratch. */
static void to_final(const basis_t *B, const int sh[4], const double *in, double *out, double *tmp) {
  int dims[4];
  for (int q = 0; q < 4; ++q) dims[q] = ncart(B->sh_l[sh[q]]);
  memcpy(tmp, in, sizeof(double) * dims[0] * dims[1] * dims[2] * dims[3]);
  for (int q = 0; q < 4; ++q) {
    const int l = B->sh_l[sh[q]];
    if (!(B->sh_pure[sh[q]] && l >= 2)) continue;
    const double *T = tsph_of(B, l);
    const int nc = ncart(l), ns = 2 * l + 1;
    int pre = 1, post = 1;
    for (int r = 0; r < q; ++r) pre *= dims[r];
    for (int r = q + 1; r < 4; ++r) post *= dims[r];
    for (int p = 0; p < pre; ++p)
      for (int m = 0; m < ns; ++m)
        for (int s = 0; s < post; ++s) {
          double acc = 0;
          for (int c = 0; c < nc; ++c) acc += T[m * nc + c] * tmp[((size_t)p * nc + c) * post + s];
          out[((size_t)p * ns + m) * post + s] = acc;
        }
    dims[q] = ns;
    memcpy(tmp, out, sizeof(double) * dims[0] * dims[1] * dims[2] * dims[3]);
  }
  memcpy(out, tmp, sizeof(double) * dims[0] * dims[1] * dims[2] * dims[3]);
}

#define BLK_MAX (15 * 15 * 15 * 15)

static void make_basis(basis_t *b, const double *coords, int nshell, const int *sh_atom, const int *sh_l,
                       const int *sh_nprim, const int *sh_off, const int *sh_pure, const double *pexp,
                       const double *pcoef, const double *tsph) {
  b->coords = coords; b->nshell = nshell; b->sh_atom = sh_atom; b->sh_l = sh_l; b->sh_nprim = sh_nprim;
  b->sh_off = sh_off; b->sh_pure = sh_pure; b->pexp = pexp; b->pcoef = pcoef; b->tsph = tsph;
}

static void ao_offsets(const basis_t *B, int *off) {
  off[0] = 0;
  for (int s = 0; s < B->nshell; ++s) off[s + 1] = off[s] + nsph(B->sh_l[s], B->sh_pure[s]);
}

/* Final-basis block of (ij|kl) in the given index order. */
int oracle_eri_block(const double *coords, int nshell, const int *sh_atom, const int *sh_l, const int *sh_nprim,
                     const int *sh_off, const int *sh_pure, const double *pexp, const double *pcoef,
                     const double *tsph, int i, int j, int k, int l, double *out) {
  init_tables();
  basis_t B; make_basis(&B, coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph);
  work_t w; work_alloc(&w);
  double *cart = (double *)malloc(sizeof(double) * BLK_MAX), *tmp = (double *)malloc(sizeof(double) * BLK_MAX);
  int sh[4] = {i, j, k, l};
  eri_cart(&B, i, j, k, l, &w, cart);
  to_final(&B, sh, cart, out, tmp);
  free(cart); free(tmp); work_free(&w);
  return 0;
}

/* Cartesian-block Schwarz factors I[i*nshell+j] = max_{a in i, b in j} |(ab|ab)|^(1/2). */
int oracle_schwarz(const double *coords, int nshell, const int *sh_atom, const int *sh_l, const int *sh_nprim,
                   const int *sh_off, const int *sh_pure, const double *pexp, const double *pcoef,
                   const double *tsph, double *I) {
  init_tables();
  basis_t B; make_basis(&B, coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph);
#pragma omp parallel
  {
    work_t w; work_alloc(&w);
    double *cart = (double *)malloc(sizeof(double) * BLK_MAX);
#pragma omp for schedule(dynamic, 4)
    for (long long ij = 0; ij < (long long)nshell * nshell; ++ij) {
      const int i = (int)(ij / nshell), j = (int)(ij % nshell);
      if (j > i) continue;
      eri_cart(&B, i, j, i, j, &w, cart);
      const int na = ncart(sh_l[i]), nb = ncart(sh_l[j]);
      double mx = 0;
      for (int a = 0; a < na; ++a)
        for (int b = 0; b < nb; ++b) {
          const double v = fabs(cart[(((size_t)a * nb + b) * na + a) * nb + b]);
          if (v > mx) mx = v;
        }
      I[(size_t)i * nshell + j] = I[(size_t)j * nshell + i] = sqrt(mx);
    }
    free(cart); work_free(&w);
  }
  return 0;
}

/* Block maxima of |D_cart| with D_cart = T^T D T per shell block. */
static void density_blockmax(const basis_t *B, const int *off, const double *D, int nbf, double *P) {
  const int ns = B->nshell;
#pragma omp parallel for schedule(dynamic, 8)
  for (int i = 0; i < ns; ++i) {
    double blk[15 * 15], tmp[15 * 15];
    for (int j = 0; j < ns; ++j) {
      const int li = B->sh_l[i], lj = B->sh_l[j];
      const int ni = nsph(li, B->sh_pure[i]), nj = nsph(lj, B->sh_pure[j]);
      const int ci = ncart(li), cj = ncart(lj);
      const double *Ti = (B->sh_pure[i] && li >= 2) ? tsph_of(B, li) : NULL;
      const double *Tj = (B->sh_pure[j] && lj >= 2) ? tsph_of(B, lj) : NULL;
      /* tmp[m][c'] = sum_n D[m][n] Tj[n][c'] */
      for (int m = 0; m < ni; ++m)
        for (int c = 0; c < cj; ++c) {
          double s = 0;
          if (Tj) { for (int n = 0; n < nj; ++n) s += D[(size_t)(off[i] + m) * nbf + off[j] + n] * Tj[n * cj + c]; }
          else s = D[(size_t)(off[i] + m) * nbf + off[j] + c];
          tmp[m * cj + c] = s;
        }
      double mx = 0;
      for (int a = 0; a < ci; ++a)
        for (int c = 0; c < cj; ++c) {
          double s = 0;
          if (Ti) { for (int m = 0; m < ni; ++m) s += Ti[m * ci + a] * tmp[m * cj + c]; }
          else s = tmp[a * cj + c];
          blk[a * cj + c] = s;
          if (fabs(s) > mx) mx = fabs(s);
        }
      P[(size_t)i * ns + j] = mx;
    }
  }
}

/* Density-weighted screen of paper section 3: keep (ij|kl) iff both pair factors exceed tau
 * and I_ij I_kl P >= tau, P the largest |D_cart| over the density blocks the quartet's updates
 * read. want = 3 (J and K): all six blocks D_ij, D_kl, D_ik, D_il, D_jk, D_jl. want = 1 (J only):
 * the Coulomb blocks D_ij, D_kl. want = 2 (K only): the exchange blocks D_ik, D_il, D_jk, D_jl. */
static inline int keep_quartet_want(const double *I, const double *P, int ns, int i, int j, int k, int l,
                                    double tau, int want) {
  const double Iij = I[(size_t)i * ns + j], Ikl = I[(size_t)k * ns + l];
  if (!(Iij > tau) || !(Ikl > tau)) return 0;
  double p = 0.0, t;
  if (want & 1) {
    t = P[(size_t)i * ns + j]; if (t > p) p = t;
    t = P[(size_t)k * ns + l]; if (t > p) p = t;
  }
  if (want & 2) {
    t = P[(size_t)i * ns + k]; if (t > p) p = t;
    t = P[(size_t)i * ns + l]; if (t > p) p = t;
    t = P[(size_t)j * ns + k]; if (t > p) p = t;
    t = P[(size_t)j * ns + l]; if (t > p) p = t;
  }
  return Iij * Ikl * p >= tau;
}

static inline int keep_quartet(const double *I, const double *P, int ns, int i, int j, int k, int l, double tau) {
  return keep_quartet_want(I, P, ns, i, j, k, l, tau, 3);
}

/* Apply J[i,j] += (ij|kl) D[k,l], K[i,k] += (ij|kl) D[j,l] for one ordered tuple.
 * blk is the final-basis block for the tuple (s0,s1,s2,s3) in that index order. */
static void digest(const int *off, int nbf, const double *D, const double *blk, const int s[4],
                   const int n[4], double *J, double *K) {
  for (int p = 0; p < n[0]; ++p)
    for (int q = 0; q < n[1]; ++q)
      for (int r = 0; r < n[2]; ++r)
        for (int t = 0; t < n[3]; ++t) {
          const double g = blk[(((size_t)p * n[1] + q) * n[2] + r) * n[3] + t];
          const int mu = off[s[0]] + p, nu = off[s[1]] + q, la = off[s[2]] + r, si = off[s[3]] + t;
          J[(size_t)mu * nbf + nu] += g * D[(size_t)la * nbf + si];
          K[(size_t)mu * nbf + la] += g * D[(size_t)nu * nbf + si];
        }
}

/* Permute a block stored for (i,j,k,l) into the index order of an image tuple.
 * perm[q] = which original index position supplies image position q. */
static void permute_block(const double *in, const int n[4], const int perm[4], double *out, int nout[4]) {
  for (int q = 0; q < 4; ++q) nout[q] = n[perm[q]];
  int idx[4];
  for (idx[0] = 0; idx[0] < n[0]; ++idx[0])
    for (idx[1] = 0; idx[1] < n[1]; ++idx[1])
      for (idx[2] = 0; idx[2] < n[2]; ++idx[2])
        for (idx[3] = 0; idx[3] < n[3]; ++idx[3]) {
          const double v = in[(((size_t)idx[0] * n[1] + idx[1]) * n[2] + idx[2]) * n[3] + idx[3]];
          const int o0 = idx[perm[0]], o1 = idx[perm[1]], o2 = idx[perm[2]], o3 = idx[perm[3]];
          out[(((size_t)o0 * nout[1] + o1) * nout[2] + o2) * nout[3] + o3] = v;
        }
}

/* The eight index permutations that leave (ij|kl) invariant: positions (0,1,2,3) map to
 * (ij|kl),(ji|kl),(ij|lk),(ji|lk),(kl|ij),(lk|ij),(kl|ji),(lk|ji). */
static const int PERMS[8][4] = {{0, 1, 2, 3}, {1, 0, 2, 3}, {0, 1, 3, 2}, {1, 0, 3, 2},
                                {2, 3, 0, 1}, {3, 2, 0, 1}, {2, 3, 1, 0}, {3, 2, 1, 0}};

/* Full J and K (nbf x nbf, final basis) over the quartets the screen keeps for the outputs
 * `want` (bit 0 J, bit 1 K; both are always accumulated). Returns the number of kept unique
 * quartets. */
long long oracle_jk_want(const double *coords, int nshell, const int *sh_atom, const int *sh_l, const int *sh_nprim,
                         const int *sh_off, const int *sh_pure, const double *pexp, const double *pcoef,
                         const double *tsph, const double *D, double tau, double *J, double *K, int nthreads,
                         int want) {
  init_tables();
  basis_t B; make_basis(&B, coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph);
  int *off = (int *)malloc(sizeof(int) * (nshell + 1));
  ao_offsets(&B, off);
  const int nbf = off[nshell];
  if (nthreads > 0) omp_set_num_threads(nthreads);
  double *I = (double *)malloc(sizeof(double) * nshell * nshell);
  double *P = (double *)malloc(sizeof(double) * nshell * nshell);
  oracle_schwarz(coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph, I);
  density_blockmax(&B, off, D, nbf, P);
  memset(J, 0, sizeof(double) * nbf * nbf);
  memset(K, 0, sizeof(double) * nbf * nbf);
  const long long npair = (long long)nshell * (nshell + 1) / 2;
  long long kept = 0;
#pragma omp parallel reduction(+ : kept)
  {
    work_t w; work_alloc(&w);
    double *cart = (double *)malloc(sizeof(double) * BLK_MAX), *fin = (double *)malloc(sizeof(double) * BLK_MAX);
    double *tmp = (double *)malloc(sizeof(double) * BLK_MAX), *img = (double *)malloc(sizeof(double) * BLK_MAX);
    double *Jt = (double *)calloc((size_t)nbf * nbf, sizeof(double));
    double *Kt = (double *)calloc((size_t)nbf * nbf, sizeof(double));
#pragma omp for schedule(dynamic, 1)
    for (long long ij = 0; ij < npair; ++ij) {
      int i = (int)((sqrt(8.0 * ij + 1) - 1) / 2);
      while ((long long)i * (i + 1) / 2 > ij) --i;
      while ((long long)(i + 1) * (i + 2) / 2 <= ij) ++i;
      const int j = (int)(ij - (long long)i * (i + 1) / 2);
      for (long long kl = 0; kl <= ij; ++kl) {
        int k = (int)((sqrt(8.0 * kl + 1) - 1) / 2);
        while ((long long)k * (k + 1) / 2 > kl) --k;
        while ((long long)(k + 1) * (k + 2) / 2 <= kl) ++k;
        const int l = (int)(kl - (long long)k * (k + 1) / 2);
        if (!keep_quartet_want(I, P, nshell, i, j, k, l, tau, want)) continue;
        ++kept;
        const int sh[4] = {i, j, k, l};
        eri_cart(&B, i, j, k, l, &w, cart);
        to_final(&B, sh, cart, fin, tmp);
        const int n[4] = {nsph(sh_l[i], sh_pure[i]), nsph(sh_l[j], sh_pure[j]),
                          nsph(sh_l[k], sh_pure[k]), nsph(sh_l[l], sh_pure[l])};
        int seen[8][4], nseen = 0;
        for (int p = 0; p < 8; ++p) {
          int t[4];
          for (int q = 0; q < 4; ++q) t[q] = sh[PERMS[p][q]];
          int dup = 0;
          for (int s = 0; s < nseen; ++s)
            if (seen[s][0] == t[0] && seen[s][1] == t[1] && seen[s][2] == t[2] && seen[s][3] == t[3]) dup = 1;
          if (dup) continue;
          memcpy(seen[nseen++], t, sizeof(t));
          int nout[4];
          permute_block(fin, n, PERMS[p], img, nout);
          digest(off, nbf, D, img, t, nout, Jt, Kt);
        }
      }
    }
#pragma omp critical(oracle_reduce)
    {
      for (size_t x = 0; x < (size_t)nbf * nbf; ++x) { J[x] += Jt[x]; K[x] += Kt[x]; }
    }
    free(Jt); free(Kt); free(cart); free(fin); free(tmp); free(img); work_free(&w);
  }
  free(I); free(P); free(off);
  return kept;
}

long long oracle_jk(const double *coords, int nshell, const int *sh_atom, const int *sh_l, const int *sh_nprim,
                    const int *sh_off, const int *sh_pure, const double *pexp, const double *pcoef,
                    const double *tsph, const double *D, double tau, double *J, double *K, int nthreads) {
  return oracle_jk_want(coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph, D, tau, J, K,
                        nthreads, 3);
}

/* Sampled rows: for shells si, sj, the J block J[si,sj] = sum over ALL shells k,l of
 * (si sj|k l) D[k,l] and the K block K[si,sj] = sum over all k,l of (si k|sj l) D[k,l],
 * with the same screening predicate applied to each ordered quartet. Jb, Kb are
 * n_si x n_sj (final basis). I and P may be passed in (nshell^2 each) or NULL. */
int oracle_jk_block(const double *coords, int nshell, const int *sh_atom, const int *sh_l, const int *sh_nprim,
                    const int *sh_off, const int *sh_pure, const double *pexp, const double *pcoef,
                    const double *tsph, const double *D, double tau, const double *Iin, const double *Pin,
                    int si, int sj, double *Jb, double *Kb, int nthreads) {
  init_tables();
  basis_t B; make_basis(&B, coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph);
  int *off = (int *)malloc(sizeof(int) * (nshell + 1));
  ao_offsets(&B, off);
  const int nbf = off[nshell];
  if (nthreads > 0) omp_set_num_threads(nthreads);
  double *I = (double *)Iin, *P = (double *)Pin;
  if (!I) {
    I = (double *)malloc(sizeof(double) * nshell * nshell);
    oracle_schwarz(coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph, I);
  }
  if (!P) { P = (double *)malloc(sizeof(double) * nshell * nshell); density_blockmax(&B, off, D, nbf, P); }
  const int ni = nsph(sh_l[si], sh_pure[si]), nj = nsph(sh_l[sj], sh_pure[sj]);
  memset(Jb, 0, sizeof(double) * ni * nj);
  memset(Kb, 0, sizeof(double) * ni * nj);
#pragma omp parallel
  {
    work_t w; work_alloc(&w);
    double *cart = (double *)malloc(sizeof(double) * BLK_MAX), *fin = (double *)malloc(sizeof(double) * BLK_MAX);
    double *tmp = (double *)malloc(sizeof(double) * BLK_MAX);
    double *Jt = (double *)calloc((size_t)ni * nj, sizeof(double));
    double *Kt = (double *)calloc((size_t)ni * nj, sizeof(double));
#pragma omp for schedule(dynamic, 1)
    for (long long kl = 0; kl < (long long)nshell * nshell; ++kl) {
      const int k = (int)(kl / nshell), l = (int)(kl % nshell);
      const int nk = nsph(sh_l[k], sh_pure[k]), nl = nsph(sh_l[l], sh_pure[l]);
      /* J: (si sj | k l) */
      if (keep_quartet(I, P, nshell, si, sj, k, l, tau)) {
        const int sh[4] = {si, sj, k, l};
        eri_cart(&B, si, sj, k, l, &w, cart);
        to_final(&B, sh, cart, fin, tmp);
        for (int p = 0; p < ni; ++p)
          for (int q = 0; q < nj; ++q) {
            double s = 0;
            for (int r = 0; r < nk; ++r)
              for (int t = 0; t < nl; ++t)
                s += fin[(((size_t)p * nj + q) * nk + r) * nl + t] * D[(size_t)(off[k] + r) * nbf + off[l] + t];
            Jt[p * nj + q] += s;
          }
      }
      /* K: (si k | sj l) */
      if (keep_quartet(I, P, nshell, si, k, sj, l, tau)) {
        const int sh[4] = {si, k, sj, l};
        eri_cart(&B, si, k, sj, l, &w, cart);
        to_final(&B, sh, cart, fin, tmp);
        for (int p = 0; p < ni; ++p)
          for (int q = 0; q < nj; ++q) {
            double s = 0;
            for (int r = 0; r < nk; ++r)
              for (int t = 0; t < nl; ++t)
                s += fin[(((size_t)p * nk + r) * nj + q) * nl + t] * D[(size_t)(off[k] + r) * nbf + off[l] + t];
            Kt[p * nj + q] += s;
          }
      }
    }
#pragma omp critical(oracle_reduce_blk)
    {
      for (int x = 0; x < ni * nj; ++x) { Jb[x] += Jt[x]; Kb[x] += Kt[x]; }
    }
    free(Jt); free(Kt); free(cart); free(fin); free(tmp); work_free(&w);
  }
  if (!Iin) free(I);
  if (!Pin) free(P);
  free(off);
  return 0;
}

/* Screening inputs exposed for tests: Cartesian Schwarz factors and D_cart block maxima. */
int oracle_screen_tables(const double *coords, int nshell, const int *sh_atom, const int *sh_l, const int *sh_nprim,
                         const int *sh_off, const int *sh_pure, const double *pexp, const double *pcoef,
                         const double *tsph, const double *D, double *I, double *P) {
  init_tables();
  basis_t B; make_basis(&B, coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph);
  int *off = (int *)malloc(sizeof(int) * (nshell + 1));
  ao_offsets(&B, off);
  oracle_schwarz(coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph, I);
  density_blockmax(&B, off, D, off[nshell], P);
  free(off);
  return 0;
}

/* Number of unique quartets kept by the predicate for the outputs `want` (counts only). */
long long oracle_count_kept_want(int nshell, const double *I, const double *P, double tau, int want) {
  const long long npair = (long long)nshell * (nshell + 1) / 2;
  long long kept = 0;
#pragma omp parallel for reduction(+ : kept) schedule(dynamic, 16)
  for (long long ij = 0; ij < npair; ++ij) {
    int i = (int)((sqrt(8.0 * ij + 1) - 1) / 2);
    while ((long long)i * (i + 1) / 2 > ij) --i;
    while ((long long)(i + 1) * (i + 2) / 2 <= ij) ++i;
    const int j = (int)(ij - (long long)i * (i + 1) / 2);
    for (long long kl = 0; kl <= ij; ++kl) {
      int k = (int)((sqrt(8.0 * kl + 1) - 1) / 2);
      while ((long long)k * (k + 1) / 2 > kl) --k;
      while ((long long)(k + 1) * (k + 2) / 2 <= kl) ++k;
      const int l = (int)(kl - (long long)k * (k + 1) / 2);
      kept += keep_quartet_want(I, P, nshell, i, j, k, l, tau, want);
    }
  }
  return kept;
}

long long oracle_count_kept(int nshell, const double *I, const double *P, double tau) {
  return oracle_count_kept_want(nshell, I, P, tau, 3);
}

/* ------------------------------------------------------------------ nuclear gradient */
/* Gradient of E = sum over ordered quartets (ij|kl) [D_ij D_kl - D_ik D_jl / 2] with respect to
 * the atomic coordinates, D held fixed (the two-electron part of the nuclear gradient, paper
 * section 4; E is tr(D (J - K/2)) of the J/K build). Every derivative integral comes from the
 * differentiation of a primitive Cartesian Gaussian,
 *   d/dA_x [x_A^a exp(-alpha r_A^2)] = 2 alpha x_A^(a+1) exp(...) - a x_A^(a-1) exp(...),
 * so that d(ij|kl)/dA_x = (i+1_x j|kl) with coefficients 2 alpha c - a_x (i-1_x j|kl), and the
 * same on each of the four centres (no translational invariance used). The shifted shells
 * are extra shells of an extended basis evaluated with the same ERI routine. A unique quartet
 * stands for the 8s distinct ordered quartets of its orbit (s = 1/|stabiliser|), whose weights
 * add up to W_abcd = s [8 D_ab D_cd - 2 D_ac D_bd - 2 D_ad D_bc]. The screen is the J/K
 * build's (six density blocks). Shells up to l = 3 (the raised shell must stay within l = 4).
 * grad: natom x 3, overwritten. Returns the number of kept unique quartets, or -1 if a shell
 * has l > 3. */
long long oracle_grad(const double *coords, int natom, int nshell, const int *sh_atom, const int *sh_l,
                      const int *sh_nprim, const int *sh_off, const int *sh_pure, const double *pexp,
                      const double *pcoef, const double *tsph, const double *D, double tau, double *grad,
                      int nthreads) {
  init_tables();
  if (nshell <= 0 || natom <= 0) return -1;
  for (int s = 0; s < nshell; ++s)
    if (sh_l[s] > LMAX - 1) return -1;
  /* extended basis: shells 0..ns-1 as given, ns + s raised (l+1, coefficients 2 alpha c),
   * 2 ns + s lowered (l-1, coefficients c; unused for l = 0) */
  int nprim_tot = 0;
  for (int s = 0; s < nshell; ++s)
    if (sh_off[s] + sh_nprim[s] > nprim_tot) nprim_tot = sh_off[s] + sh_nprim[s];
  const int ns3 = 3 * nshell;
  int *xa = (int *)malloc(sizeof(int) * ns3), *xl = (int *)malloc(sizeof(int) * ns3);
  int *xn = (int *)malloc(sizeof(int) * ns3), *xo = (int *)malloc(sizeof(int) * ns3);
  int *xp = (int *)calloc((size_t)ns3, sizeof(int));
  double *xe = (double *)malloc(sizeof(double) * 2 * nprim_tot), *xc = (double *)malloc(sizeof(double) * 2 * nprim_tot);
  for (int k = 0; k < nprim_tot; ++k) {
    xe[k] = pexp[k]; xc[k] = pcoef[k];
    xe[nprim_tot + k] = pexp[k]; xc[nprim_tot + k] = 2.0 * pexp[k] * pcoef[k];
  }
  for (int s = 0; s < nshell; ++s) {
    for (int v = 0; v < 3; ++v) {
      const int t = v * nshell + s;
      xa[t] = sh_atom[s]; xn[t] = sh_nprim[s];
      xl[t] = sh_l[s] + (v == 1 ? 1 : v == 2 ? -1 : 0);
      if (xl[t] < 0) xl[t] = 0;
      xo[t] = sh_off[s] + (v == 1 ? nprim_tot : 0);
      xp[t] = 0;                                  /* derivative blocks stay Cartesian */
    }
  }
  basis_t B; make_basis(&B, coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph);
  basis_t X; make_basis(&X, coords, ns3, xa, xl, xn, xo, xp, xe, xc, tsph);
  int *off = (int *)malloc(sizeof(int) * (nshell + 1));
  ao_offsets(&B, off);
  const int nbf = off[nshell];
  if (nthreads > 0) omp_set_num_threads(nthreads);
  double *I = (double *)malloc(sizeof(double) * nshell * nshell);
  double *P = (double *)malloc(sizeof(double) * nshell * nshell);
  oracle_schwarz(coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph, I);
  density_blockmax(&B, off, D, nbf, P);
  memset(grad, 0, sizeof(double) * 3 * natom);
  const long long npair = (long long)nshell * (nshell + 1) / 2;
  long long kept = 0;
#pragma omp parallel reduction(+ : kept)
  {
    work_t w; work_alloc(&w);
    double *raised = (double *)malloc(sizeof(double) * 21 * BLK_MAX / 15);
    double *lowered = (double *)malloc(sizeof(double) * BLK_MAX);
    double *dcart = (double *)malloc(sizeof(double) * BLK_MAX), *fin = (double *)malloc(sizeof(double) * BLK_MAX);
    double *tmp = (double *)malloc(sizeof(double) * BLK_MAX);
    double *g = (double *)calloc((size_t)3 * natom, sizeof(double));
#pragma omp for schedule(dynamic, 1)
    for (long long ij = 0; ij < npair; ++ij) {
      int i = (int)((sqrt(8.0 * ij + 1) - 1) / 2);
      while ((long long)i * (i + 1) / 2 > ij) --i;
      while ((long long)(i + 1) * (i + 2) / 2 <= ij) ++i;
      const int j = (int)(ij - (long long)i * (i + 1) / 2);
      for (long long kl = 0; kl <= ij; ++kl) {
        int k = (int)((sqrt(8.0 * kl + 1) - 1) / 2);
        while ((long long)k * (k + 1) / 2 > kl) --k;
        while ((long long)(k + 1) * (k + 2) / 2 <= kl) ++k;
        const int l = (int)(kl - (long long)k * (k + 1) / 2);
        if (!keep_quartet(I, P, nshell, i, j, k, l, tau)) continue;
        ++kept;
        const int sh[4] = {i, j, k, l};
        const int nc[4] = {ncart(sh_l[i]), ncart(sh_l[j]), ncart(sh_l[k]), ncart(sh_l[l])};
        const int nf[4] = {nsph(sh_l[i], sh_pure[i]), nsph(sh_l[j], sh_pure[j]), nsph(sh_l[k], sh_pure[k]),
                           nsph(sh_l[l], sh_pure[l])};
        const double s = (i == j ? 0.5 : 1.0) * (k == l ? 0.5 : 1.0) * (ij == kl ? 0.5 : 1.0);
        for (int q = 0; q < 4; ++q) {
          const int lq = sh_l[sh[q]];
          int shp[4] = {i, j, k, l}, shm[4] = {i, j, k, l};
          shp[q] = nshell + sh[q];
          shm[q] = 2 * nshell + sh[q];
          eri_cart(&X, shp[0], shp[1], shp[2], shp[3], &w, raised);
          if (lq > 0) eri_cart(&X, shm[0], shm[1], shm[2], shm[3], &w, lowered);
          int np[4] = {nc[0], nc[1], nc[2], nc[3]}, nm[4] = {nc[0], nc[1], nc[2], nc[3]};
          np[q] = ncart(lq + 1);
          nm[q] = lq > 0 ? ncart(lq - 1) : 0;
          for (int x = 0; x < 3; ++x) {
            int idx[4];
            for (idx[0] = 0; idx[0] < nc[0]; ++idx[0])
              for (idx[1] = 0; idx[1] < nc[1]; ++idx[1])
                for (idx[2] = 0; idx[2] < nc[2]; ++idx[2])
                  for (idx[3] = 0; idx[3] < nc[3]; ++idx[3]) {
                    /* component of shell q and its raised / lowered neighbours in direction x */
                    const int cf = g_level_start[lq] + idx[q];
                    int cv[3] = {g_comp[cf][0], g_comp[cf][1], g_comp[cf][2]};
                    int pi[4] = {idx[0], idx[1], idx[2], idx[3]};
                    cv[x] += 1;
                    pi[q] = g_flat[cv[0]][cv[1]][cv[2]] - g_level_start[lq + 1];
                    double v = raised[(((size_t)pi[0] * np[1] + pi[1]) * np[2] + pi[2]) * np[3] + pi[3]];
                    cv[x] -= 2;
                    if (cv[x] >= 0) {
                      int mi[4] = {idx[0], idx[1], idx[2], idx[3]};
                      mi[q] = g_flat[cv[0]][cv[1]][cv[2]] - g_level_start[lq - 1];
                      v -= (cv[x] + 1) * lowered[(((size_t)mi[0] * nm[1] + mi[1]) * nm[2] + mi[2]) * nm[3] + mi[3]];
                    }
                    dcart[(((size_t)idx[0] * nc[1] + idx[1]) * nc[2] + idx[2]) * nc[3] + idx[3]] = v;
                  }
            to_final(&B, sh, dcart, fin, tmp);
            double acc = 0.0;
            for (int a = 0; a < nf[0]; ++a)
              for (int b = 0; b < nf[1]; ++b)
                for (int c = 0; c < nf[2]; ++c)
                  for (int d = 0; d < nf[3]; ++d) {
                    const int A_ = off[i] + a, B_ = off[j] + b, C_ = off[k] + c, D_ = off[l] + d;
                    const double Wt = 8.0 * D[(size_t)A_ * nbf + B_] * D[(size_t)C_ * nbf + D_] -
                                      2.0 * D[(size_t)A_ * nbf + C_] * D[(size_t)B_ * nbf + D_] -
                                      2.0 * D[(size_t)A_ * nbf + D_] * D[(size_t)B_ * nbf + C_];
                    acc += Wt * fin[(((size_t)a * nf[1] + b) * nf[2] + c) * nf[3] + d];
                  }
            g[3 * sh_atom[sh[q]] + x] += s * acc;
          }
        }
      }
    }
#pragma omp critical(oracle_reduce_grad)
    {
      for (int t = 0; t < 3 * natom; ++t) grad[t] += g[t];
    }
    free(g); free(raised); free(lowered); free(dcart); free(fin); free(tmp); work_free(&w);
  }
  free(I); free(P); free(off); free(xa); free(xl); free(xn); free(xo); free(xp); free(xe); free(xc);
  return kept;
}

/* ------------------------------------------------------------------ one-electron integrals */
/* Overlap S, kinetic energy T and nuclear attraction V = -sum_C Z_C (mu|1/|r-C||nu) in the final
 * basis (the one-electron part of an SCF around the J/K build, paper section 4), by the
 * Obara-Saika recurrences (Obara & Saika 1986):
 *   1D overlap: S(0,0) = sqrt(pi/p), S(i+1,j) = PA S(i,j) + (i S(i-1,j) + j S(i,j-1))/(2p),
 *               S(i,j+1) = PB S(i,j) + (i S(i-1,j) + j S(i,j-1))/(2p), times exp(-ab/p AB^2);
 *   kinetic:    the ket Gaussian's second derivative, -1/2 [j(j-1) S(i,j-2) - 2b(2j+1) S(i,j)
 *               + 4b^2 S(i,j+2)] per direction;
 *   attraction: auxiliary integrals Theta^(m)(e) on the bra centre, Theta^(m)(0) = 2 pi/p K F_m(T),
 *               Theta^(m)(e+1_i) = PA_i Theta^(m)(e) - PC_i Theta^(m+1)(e)
 *                                  + e_i/(2p) [Theta^(m)(e-1_i) - Theta^(m+1)(e-1_i)],
 *               then (a|b+1_i) = (a+1_i|b) + (A_i - B_i)(a|b).
 * S, T, V: nbf x nbf; *enuc = sum_{A<B} Z_A Z_B / R_AB. */
static void os_overlap_1d(int imax, int jmax, double PA, double PB, double p, double s00, double out[7][7]) {
  for (int i = 0; i <= imax; ++i)
    for (int j = 0; j <= jmax; ++j) out[i][j] = 0.0;
  out[0][0] = s00;
  for (int i = 0; i <= imax; ++i)
    for (int j = 0; j <= jmax; ++j) {
      if (i == 0 && j == 0) continue;
      if (i > 0) {
        double v = PA * out[i - 1][j];
        if (i > 1) v += (i - 1) * out[i - 2][j] / (2 * p);
        if (j > 0) v += j * out[i - 1][j - 1] / (2 * p);
        out[i][j] = v;
      } else {
        double v = PB * out[i][j - 1];
        if (j > 1) v += (j - 1) * out[i][j - 2] / (2 * p);
        out[i][j] = v;
      }
    }
}

int oracle_one_electron(const double *coords, int natom, int nshell, const int *sh_atom, const int *sh_l,
                        const int *sh_nprim, const int *sh_off, const int *sh_pure, const double *pexp,
                        const double *pcoef, const double *tsph, const double *charges, double *S, double *T,
                        double *V, double *enuc) {
  init_tables();
  basis_t B; make_basis(&B, coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph);
  int *off = (int *)malloc(sizeof(int) * (nshell + 1));
  ao_offsets(&B, off);
  const int nbf = off[nshell];
  /* Cartesian blocks [a][b] of the three operators, then to the final basis */
  double *cb = (double *)malloc(sizeof(double) * 3 * 15 * 15);
  double *th = (double *)malloc(sizeof(double) * NCOMP_EMAX * (EMAX + 1));   /* Theta[e][m] */
  double *e0 = (double *)malloc(sizeof(double) * NCOMP_EMAX);
  double *x = (double *)malloc(sizeof(double) * NCOMP_EMAX * NCOMP_LMAX);
  double fin[15 * 15], tmp[15 * 15];
  for (int i = 0; i < nshell; ++i)
    for (int j = 0; j <= i; ++j) {
      const int la = sh_l[i], lb = sh_l[j], na = ncart(la), nb = ncart(lb), E = la + lb;
      const double *A = coords + 3 * sh_atom[i], *Bc = coords + 3 * sh_atom[j];
      double AB2 = 0, ABv[3];
      for (int d = 0; d < 3; ++d) { ABv[d] = A[d] - Bc[d]; AB2 += ABv[d] * ABv[d]; }
      memset(cb, 0, sizeof(double) * 3 * 15 * 15);
      for (int pa = 0; pa < sh_nprim[i]; ++pa)
        for (int pb = 0; pb < sh_nprim[j]; ++pb) {
          const double a = pexp[sh_off[i] + pa], b = pexp[sh_off[j] + pb];
          const double cc = pcoef[sh_off[i] + pa] * pcoef[sh_off[j] + pb];
          const double p = a + b, K = exp(-a * b / p * AB2);
          double P[3], s1[3][7][7];
          for (int d = 0; d < 3; ++d) {
            P[d] = (a * A[d] + b * Bc[d]) / p;
            os_overlap_1d(la, lb + 2, P[d] - A[d], P[d] - Bc[d], p, sqrt(M_PI / p), s1[d]);
          }
          for (int ca = 0; ca < na; ++ca) {
            const int *ea = g_comp[g_level_start[la] + ca];
            for (int cbb = 0; cbb < nb; ++cbb) {
              const int *eb = g_comp[g_level_start[lb] + cbb];
              double sx[3], tx[3];
              for (int d = 0; d < 3; ++d) {
                const int u = ea[d], v = eb[d];
                sx[d] = s1[d][u][v];
                double t = -2.0 * b * (2 * v + 1) * s1[d][u][v] + 4.0 * b * b * s1[d][u][v + 2];
                if (v >= 2) t += v * (v - 1) * s1[d][u][v - 2];
                tx[d] = -0.5 * t;
              }
              cb[ca * nb + cbb] += cc * K * sx[0] * sx[1] * sx[2];
              cb[225 + ca * nb + cbb] += cc * K * (tx[0] * sx[1] * sx[2] + sx[0] * tx[1] * sx[2] + sx[0] * sx[1] * tx[2]);
            }
          }
          /* nuclear attraction: Theta on the bra centre for |e| <= E, then the transfer */
          const int ne = g_level_start[E + 1];
          for (int e = 0; e < ne; ++e) e0[e] = 0.0;
          for (int c = 0; c < natom; ++c) {
            if (charges[c] == 0.0) continue;
            const double *C = coords + 3 * c;
            double PC[3], PC2 = 0.0, F[EMAX + 2];
            for (int d = 0; d < 3; ++d) { PC[d] = P[d] - C[d]; PC2 += PC[d] * PC[d]; }
            oracle_boys(E, p * PC2, F);
            for (int m = 0; m <= E; ++m) th[0 * (EMAX + 1) + m] = 2.0 * M_PI / p * K * F[m];
            for (int e = 1; e < ne; ++e) {
              const int ev[3] = {g_comp[e][0], g_comp[e][1], g_comp[e][2]};
              const int L = ev[0] + ev[1] + ev[2];
              const int d = ev[0] > 0 ? 0 : (ev[1] > 0 ? 1 : 2);
              int em[3] = {ev[0], ev[1], ev[2]};
              em[d] -= 1;
              const int ie1 = g_flat[em[0]][em[1]][em[2]];
              int ie2 = -1;
              if (em[d] > 0) { int e2[3] = {em[0], em[1], em[2]}; e2[d] -= 1; ie2 = g_flat[e2[0]][e2[1]][e2[2]]; }
              for (int m = 0; m <= E - L; ++m) {
                double v = (P[d] - A[d]) * th[ie1 * (EMAX + 1) + m] - PC[d] * th[ie1 * (EMAX + 1) + m + 1];
                if (ie2 >= 0)
                  v += em[d] / (2.0 * p) * (th[ie2 * (EMAX + 1) + m] - th[ie2 * (EMAX + 1) + m + 1]);
                th[e * (EMAX + 1) + m] = v;
              }
            }
            for (int e = g_level_start[la]; e < ne; ++e) e0[e] -= charges[c] * cc * th[e * (EMAX + 1) + 0];
          }
          /* (a|b): X[e][b] over b levels 0..lb by (a|b+1_i) = (a+1_i|b) + AB_i (a|b) */
          for (int e = g_level_start[la]; e < ne; ++e) x[e * NCOMP_LMAX + 0] = e0[e];
          for (int bL = 1; bL <= lb; ++bL)
            for (int ib = g_level_start[bL]; ib < g_level_start[bL + 1]; ++ib) {
              const int bv[3] = {g_comp[ib][0], g_comp[ib][1], g_comp[ib][2]};
              const int d = bv[0] > 0 ? 0 : (bv[1] > 0 ? 1 : 2);
              int bm[3] = {bv[0], bv[1], bv[2]};
              bm[d] -= 1;
              const int ibm = g_flat[bm[0]][bm[1]][bm[2]];
              for (int e = g_level_start[la]; e < g_level_start[E - bL + 1]; ++e) {
                int ep[3] = {g_comp[e][0], g_comp[e][1], g_comp[e][2]};
                ep[d] += 1;
                const int iep = g_flat[ep[0]][ep[1]][ep[2]];
                x[e * NCOMP_LMAX + ib] = x[iep * NCOMP_LMAX + ibm] + ABv[d] * x[e * NCOMP_LMAX + ibm];
              }
            }
          for (int ca = 0; ca < na; ++ca)
            for (int cbb = 0; cbb < nb; ++cbb)
              cb[450 + ca * nb + cbb] += x[(g_level_start[la] + ca) * NCOMP_LMAX + g_level_start[lb] + cbb];
        }
      /* final basis: transform rows (shell i) and columns (shell j) */
      const int sh[4] = {i, j, i, i};
      (void)sh;
      const double *Ti = (sh_pure[i] && la >= 2) ? tsph_of(&B, la) : NULL;
      const double *Tj = (sh_pure[j] && lb >= 2) ? tsph_of(&B, lb) : NULL;
      const int fi = nsph(la, sh_pure[i]), fj = nsph(lb, sh_pure[j]);
      double *outs[3] = {S, T, V};
      for (int k = 0; k < 3; ++k) {
        const double *blk = cb + 225 * k;
        for (int r = 0; r < fi; ++r)
          for (int c = 0; c < nb; ++c) {
            double v = 0.0;
            if (Ti) { for (int q = 0; q < na; ++q) v += Ti[r * na + q] * blk[q * nb + c]; }
            else v = blk[r * nb + c];
            tmp[r * nb + c] = v;
          }
        for (int r = 0; r < fi; ++r)
          for (int c = 0; c < fj; ++c) {
            double v = 0.0;
            if (Tj) { for (int q = 0; q < nb; ++q) v += tmp[r * nb + q] * Tj[c * nb + q]; }
            else v = tmp[r * nb + c];
            fin[r * fj + c] = v;
            outs[k][(size_t)(off[i] + r) * nbf + off[j] + c] = v;
            outs[k][(size_t)(off[j] + c) * nbf + off[i] + r] = v;
          }
      }
    }
  double e = 0.0;
  for (int a = 0; a < natom; ++a)
    for (int b = 0; b < a; ++b) {
      double r2 = 0.0;
      for (int d = 0; d < 3; ++d) r2 += (coords[3 * a + d] - coords[3 * b + d]) * (coords[3 * a + d] - coords[3 * b + d]);
      e += charges[a] * charges[b] / sqrt(r2);
    }
  *enuc = e;
  free(cb); free(th); free(e0); free(x); free(off);
  return 0;
}

/* Full ERI tensor in the final basis, out[mu][nu][la][si] (nbf^4, small inputs only). */
int oracle_eri_tensor(const double *coords, int nshell, const int *sh_atom, const int *sh_l, const int *sh_nprim,
                      const int *sh_off, const int *sh_pure, const double *pexp, const double *pcoef,
                      const double *tsph, double *out) {
  init_tables();
  basis_t B; make_basis(&B, coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph);
  int *off = (int *)malloc(sizeof(int) * (nshell + 1));
  ao_offsets(&B, off);
  const size_t n = off[nshell];
#pragma omp parallel
  {
    work_t w; work_alloc(&w);
    double *cart = (double *)malloc(sizeof(double) * BLK_MAX), *fin = (double *)malloc(sizeof(double) * BLK_MAX);
    double *tmp = (double *)malloc(sizeof(double) * BLK_MAX);
#pragma omp for schedule(dynamic, 1)
    for (long long ij = 0; ij < (long long)nshell * nshell; ++ij) {
      const int i = (int)(ij / nshell), j = (int)(ij % nshell);
      for (int k = 0; k < nshell; ++k)
        for (int l = 0; l < nshell; ++l) {
          const int sh[4] = {i, j, k, l};
          eri_cart(&B, i, j, k, l, &w, cart);
          to_final(&B, sh, cart, fin, tmp);
          const int ni = off[i + 1] - off[i], nj = off[j + 1] - off[j];
          const int nk = off[k + 1] - off[k], nl = off[l + 1] - off[l];
          for (int p = 0; p < ni; ++p)
            for (int q = 0; q < nj; ++q)
              for (int r = 0; r < nk; ++r)
                for (int t = 0; t < nl; ++t)
                  out[(((off[i] + p) * n + off[j] + q) * n + off[k] + r) * n + off[l] + t] =
                      fin[(((size_t)p * nj + q) * nk + r) * nl + t];
        }
    }
    free(cart); free(fin); free(tmp); work_free(&w);
  }
  free(off);
  return 0;
}

/* Bounded sample of the full J/K loop, for timing: the unique quartets (ij|kl), kl <= ij,
 * of every bra pair index ij with ij % stride == offset, evaluated and digested exactly
 * as in oracle_jk (same screening, same explicit updates into private J/K that are then
 * discarded). Returns the number of kept unique quartets processed. */
long long oracle_jk_sample(const double *coords, int nshell, const int *sh_atom, const int *sh_l, const int *sh_nprim,
                           const int *sh_off, const int *sh_pure, const double *pexp, const double *pcoef,
                           const double *tsph, const double *D, double tau, long long stride, long long offset,
                           int nthreads) {
  init_tables();
  basis_t B; make_basis(&B, coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph);
  int *off = (int *)malloc(sizeof(int) * (nshell + 1));
  ao_offsets(&B, off);
  const int nbf = off[nshell];
  if (nthreads > 0) omp_set_num_threads(nthreads);
  double *I = (double *)malloc(sizeof(double) * nshell * nshell);
  double *P = (double *)malloc(sizeof(double) * nshell * nshell);
  oracle_schwarz(coords, nshell, sh_atom, sh_l, sh_nprim, sh_off, sh_pure, pexp, pcoef, tsph, I);
  density_blockmax(&B, off, D, nbf, P);
  const long long npair = (long long)nshell * (nshell + 1) / 2;
  long long kept = 0;
#pragma omp parallel reduction(+ : kept)
  {
    work_t w; work_alloc(&w);
    double *cart = (double *)malloc(sizeof(double) * BLK_MAX), *fin = (double *)malloc(sizeof(double) * BLK_MAX);
    double *tmp = (double *)malloc(sizeof(double) * BLK_MAX), *img = (double *)malloc(sizeof(double) * BLK_MAX);
    double *Jt = (double *)calloc((size_t)nbf * nbf, sizeof(double));
    double *Kt = (double *)calloc((size_t)nbf * nbf, sizeof(double));
#pragma omp for schedule(dynamic, 1)
    for (long long ij = offset; ij < npair; ij += stride) {
      int i = (int)((sqrt(8.0 * ij + 1) - 1) / 2);
      while ((long long)i * (i + 1) / 2 > ij) --i;
      while ((long long)(i + 1) * (i + 2) / 2 <= ij) ++i;
      const int j = (int)(ij - (long long)i * (i + 1) / 2);
      for (long long kl = 0; kl <= ij; ++kl) {
        int k = (int)((sqrt(8.0 * kl + 1) - 1) / 2);
        while ((long long)k * (k + 1) / 2 > kl) --k;
        while ((long long)(k + 1) * (k + 2) / 2 <= kl) ++k;
        const int l = (int)(kl - (long long)k * (k + 1) / 2);
        if (!keep_quartet(I, P, nshell, i, j, k, l, tau)) continue;
        ++kept;
        const int sh[4] = {i, j, k, l};
        eri_cart(&B, i, j, k, l, &w, cart);
        to_final(&B, sh, cart, fin, tmp);
        const int n[4] = {nsph(sh_l[i], sh_pure[i]), nsph(sh_l[j], sh_pure[j]),
                          nsph(sh_l[k], sh_pure[k]), nsph(sh_l[l], sh_pure[l])};
        int seen[8][4], nseen = 0;
        for (int p = 0; p < 8; ++p) {
          int t[4];
          for (int q = 0; q < 4; ++q) t[q] = sh[PERMS[p][q]];
          int dup = 0;
          for (int s = 0; s < nseen; ++s)
            if (seen[s][0] == t[0] && seen[s][1] == t[1] && seen[s][2] == t[2] && seen[s][3] == t[3]) dup = 1;
          if (dup) continue;
          memcpy(seen[nseen++], t, sizeof(t));
          int nout[4];
          permute_block(fin, n, PERMS[p], img, nout);
          digest(off, nbf, D, img, t, nout, Jt, Kt);
        }
      }
    }
    free(Jt); free(Kt); free(cart); free(fin); free(tmp); free(img); work_free(&w);
  }
  free(I); free(P); free(off);
  return kept;
}
