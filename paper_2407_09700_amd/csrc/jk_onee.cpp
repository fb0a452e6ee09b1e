// One-electron integrals of the SCF around the J/K build (host code: the paper evaluates them on
// the CPU, section 4). Overlap S, kinetic energy T and nuclear attraction V over the contracted
// shells of jk.h, in the final basis, and the nuclear repulsion energy.
//
// Per primitive pair (exponents a, b; P = (aA + bB)/p, p = a + b, K = exp(-ab/p |A-B|^2)) each
// Cartesian direction is the moment of a Gaussian about P: (x-A)^i (x-B)^j expanded binomially
// about P, with the central moments E[(x-P)^n] = (n-1)!! / (2p)^(n/2) (n even) of
// exp(-p (x-P)^2), whose integral is sqrt(pi/p).
//   S = K (pi/p)^(3/2) Sx Sy Sz,
//   T = K (pi/p)^(3/2) (Tx Sy Sz + Sx Ty Sz + Sx Sy Tz),
//       T_x(i,j) = -1/2 [j(j-1) S_x(i,j-2) - 2b(2j+1) S_x(i,j) + 4b^2 S_x(i,j+2)]
//   (the second derivative of the ket Gaussian), and for each nucleus C of charge Z
//   V = -Z (2 pi/p) K sum_n w_n Qx(u_n) Qy(u_n) Qz(u_n):
// the nuclear attraction in the Rys form of section 2 (one centre instead of two): with u = t^2
// the Gaussian moves to mean P + u (C - P) and variance (1 - u)/(2p), Q is the normalised moment
// of (x-A)^i (x-B)^j under it, a polynomial of degree <= i + j in u, and the N-point Rys rule of
// T = p |P-C|^2 (N = floor((la+lb)/2) + 1) integrates the product exactly.
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/jk.h"
#include "jk_host.h"

namespace host_rys {
#define RYS_STORAGE static const
#include "rys_table.h"
#undef RYS_STORAGE
}  // namespace host_rys

namespace {

int ncart_(int l) { return (l + 1) * (l + 2) / 2; }

// the N roots u and weights w of the Rys rule for T (interpolation table, Gauss-Hermite limit)
void rys_rule(int N, double T, double *u, double *w) {
  using namespace host_rys;
  if (T >= (double)RYS_TMAX[N]) {
    for (int n = 0; n < N; ++n) {
      u[n] = RYS_HERM_S2[RYS_HOFF[N] + n] / T;
      w[n] = RYS_HERM_W[RYS_HOFF[N] + n] / std::sqrt(T);
    }
    return;
  }
  const int k = std::min(std::max((int)T, 0), RYS_TMAX[N] - 1);
  const double s = 2.0 * (T - (double)k) - 1.0;
  const double *c = RYS_COEF + RYS_OFF[N] + k * (N * 2 * (RYS_DEG + 1));
  for (int n = 0; n < N; ++n) {
    const double *cu = c + n * 2 * (RYS_DEG + 1), *cw = cu + (RYS_DEG + 1);
    double pu = cu[RYS_DEG], pw = cw[RYS_DEG];
    for (int d = RYS_DEG - 1; d >= 0; --d) {
      pu = pu * s + cu[d];
      pw = pw * s + cw[d];
    }
    u[n] = pu;
    w[n] = pw;
  }
}

// C(n, k) for n <= 8
double binom_(int n, int k) {
  static const double C[9][9] = {{1}, {1, 1}, {1, 2, 1}, {1, 3, 3, 1}, {1, 4, 6, 4, 1}, {1, 5, 10, 10, 5, 1},
                                 {1, 6, 15, 20, 15, 6, 1}, {1, 7, 21, 35, 35, 21, 7, 1},
                                 {1, 8, 28, 56, 70, 56, 28, 8, 1}};
  return C[n][k];
}

// (n-1)!! for even n <= 12 (index n / 2)
const double DFACT[7] = {1.0, 1.0, 3.0, 15.0, 105.0, 945.0, 10395.0};

// E[(x - A)^i (x - B)^j] for a Gaussian of mean m and variance v (v >= 0), i <= 4, j <= 6
double moment(int i, int j, double mA, double mB, double v) {
  double pa[5], pb[7], pv[7];
  pa[0] = pb[0] = pv[0] = 1.0;
  for (int k = 1; k <= i; ++k) pa[k] = pa[k - 1] * mA;
  for (int k = 1; k <= j; ++k) pb[k] = pb[k - 1] * mB;
  for (int k = 1; k <= (i + j) / 2; ++k) pv[k] = pv[k - 1] * v;
  double s = 0.0;
  for (int k = 0; k <= i; ++k)
    for (int q = (k & 1); q <= j; q += 2)      // k + q even
      s += binom_(i, k) * binom_(j, q) * pa[i - k] * pb[j - q] * DFACT[(k + q) / 2] * pv[(k + q) / 2];
  return s;
}

struct Shell {
  int l, nprim, off, pure, atom;
};

// Cartesian exponents of component c of momentum l (ax descending, then ay)
void comp(int l, int c, int *e) {
  int n = 0;
  for (int ax = l; ax >= 0; --ax)
    for (int ay = l - ax; ay >= 0; --ay) {
      if (n++ == c) {
        e[0] = ax; e[1] = ay; e[2] = l - ax - ay;
        return;
      }
    }
}

}  // namespace

extern "C" int jk_one_electron(const jk_basis_t *B, const double *coords, int natom, const double *charges, double *S,
                               double *T, double *V, double *enuc) {
  using jk::set_error;
  if (!B || !coords || !charges || !S || !T || !V || !enuc) return set_error(JK_EINVAL, "NULL argument");
  if (natom <= 0 || B->nshell <= 0) return set_error(JK_EINVAL, "natom and nshell must be positive");
  for (int s = 0; s < B->nshell; ++s) {
    if (B->l[s] < 0 || B->l[s] > 4) return set_error(JK_EUNSUPPORTED, "shell %d: l = %d (0..4)", s, B->l[s]);
    if (B->atom[s] < 0 || B->atom[s] >= natom) return set_error(JK_EINVAL, "shell %d: atom out of range", s);
    if (B->nprim[s] <= 0 || B->prim_off[s] < 0 || B->prim_off[s] + B->nprim[s] > B->nprim_total)
      return set_error(JK_EINVAL, "shell %d: primitive range out of bounds", s);
  }
  for (int a = 0; a < 3 * natom; ++a)
    if (!std::isfinite(coords[a])) return set_error(JK_EINVAL, "coordinate %d is not finite", a);
  // AO offsets (final basis) and the solid-harmonic matrices
  const int ns = B->nshell;
  std::vector<int> off(ns + 1, 0);
  for (int s = 0; s < ns; ++s) {
    const int l = B->l[s];
    off[s + 1] = off[s] + ((B->pure[s] && l >= 2) ? 2 * l + 1 : ncart_(l));
  }
  const int nao = off[ns];
  std::vector<double> tsph[5];
  for (int l = 2; l <= 4; ++l) {
    tsph[l].resize((2 * l + 1) * ncart_(l));
    jk::solid_harmonics_host(l, tsph[l].data());
  }
  const double PI = 3.14159265358979323846;
  std::vector<double> cs(15 * 15), ct(15 * 15), cv(15 * 15);
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j <= i; ++j) {
      const int li = B->l[i], lj = B->l[j], ni = ncart_(li), nj = ncart_(lj);
      const double *A = coords + 3 * B->atom[i], *Bc = coords + 3 * B->atom[j];
      double AB2 = 0.0;
      for (int d = 0; d < 3; ++d) AB2 += (A[d] - Bc[d]) * (A[d] - Bc[d]);
      std::fill(cs.begin(), cs.end(), 0.0);
      std::fill(ct.begin(), ct.end(), 0.0);
      std::fill(cv.begin(), cv.end(), 0.0);
      const int N = (li + lj) / 2 + 1;
      for (int pa = 0; pa < B->nprim[i]; ++pa)
        for (int pb = 0; pb < B->nprim[j]; ++pb) {
          const double a = B->exps[B->prim_off[i] + pa], b = B->exps[B->prim_off[j] + pb];
          const double cc = B->coefs[B->prim_off[i] + pa] * B->coefs[B->prim_off[j] + pb];
          const double p = a + b;
          const double K = std::exp(-a * b / p * AB2);
          double P[3];
          for (int d = 0; d < 3; ++d) P[d] = (a * A[d] + b * Bc[d]) / p;
          // 1D overlap moments about P: Sx(i', j') for i' <= li, j' <= lj + 2
          double s1[3][5][7];
          for (int d = 0; d < 3; ++d)
            for (int x = 0; x <= li; ++x)
              for (int y = 0; y <= lj + 2; ++y) s1[d][x][y] = moment(x, y, P[d] - A[d], P[d] - Bc[d], 0.5 / p);
          const double pref_s = cc * K * std::pow(PI / p, 1.5);
          // nuclear attraction: per nucleus, per Rys root, Q_d(u) for every i' <= li, j' <= lj
          std::vector<double> vblk(ni * nj, 0.0);
          for (int c = 0; c < natom; ++c) {
            const double Z = charges[c];
            if (Z == 0.0) continue;
            const double *C = coords + 3 * c;
            double PC2 = 0.0;
            for (int d = 0; d < 3; ++d) PC2 += (P[d] - C[d]) * (P[d] - C[d]);
            double u[5], w[5];
            rys_rule(N, p * PC2, u, w);
            for (int n = 0; n < N; ++n) {
              double q[3][5][5];
              for (int d = 0; d < 3; ++d) {
                const double m = P[d] + u[n] * (C[d] - P[d]);
                for (int x = 0; x <= li; ++x)
                  for (int y = 0; y <= lj; ++y) q[d][x][y] = moment(x, y, m - A[d], m - Bc[d], (1.0 - u[n]) * 0.5 / p);
              }
              const double f = -Z * 2.0 * PI / p * K * cc * w[n];
              for (int ca = 0; ca < ni; ++ca) {
                int ea[3];
                comp(li, ca, ea);
                for (int cb = 0; cb < nj; ++cb) {
                  int eb[3];
                  comp(lj, cb, eb);
                  vblk[ca * nj + cb] += f * q[0][ea[0]][eb[0]] * q[1][ea[1]][eb[1]] * q[2][ea[2]][eb[2]];
                }
              }
            }
          }
          for (int ca = 0; ca < ni; ++ca) {
            int ea[3];
            comp(li, ca, ea);
            for (int cb = 0; cb < nj; ++cb) {
              int eb[3];
              comp(lj, cb, eb);
              double sx[3], tx[3];
              for (int d = 0; d < 3; ++d) {
                const int x = ea[d], y = eb[d];
                sx[d] = s1[d][x][y];
                double t = -2.0 * b * (2 * y + 1) * s1[d][x][y] + 4.0 * b * b * s1[d][x][y + 2];
                if (y >= 2) t += y * (y - 1) * s1[d][x][y - 2];
                tx[d] = -0.5 * t;
              }
              cs[ca * nj + cb] += pref_s * sx[0] * sx[1] * sx[2];
              ct[ca * nj + cb] += pref_s * (tx[0] * sx[1] * sx[2] + sx[0] * tx[1] * sx[2] + sx[0] * sx[1] * tx[2]);
              cv[ca * nj + cb] += vblk[ca * nj + cb];
            }
          }
        }
      // to the final basis: rows of shell i, columns of shell j
      const bool pi = B->pure[i] && li >= 2, pj = B->pure[j] && lj >= 2;
      const int fi = pi ? 2 * li + 1 : ni, fj = pj ? 2 * lj + 1 : nj;
      double *outs[3] = {S, T, V};
      std::vector<double> *blks[3] = {&cs, &ct, &cv};
      for (int k = 0; k < 3; ++k) {
        const std::vector<double> &blk = *blks[k];
        for (int r = 0; r < fi; ++r)
          for (int c = 0; c < fj; ++c) {
            double v = 0.0;
            for (int ca = 0; ca < ni; ++ca) {
              const double ta = pi ? tsph[li][r * ni + ca] : (ca == r ? 1.0 : 0.0);
              if (ta == 0.0) continue;
              for (int cb = 0; cb < nj; ++cb) {
                const double tb = pj ? tsph[lj][c * nj + cb] : (cb == c ? 1.0 : 0.0);
                if (tb != 0.0) v += ta * tb * blk[ca * nj + cb];
              }
            }
            outs[k][(size_t)(off[i] + r) * nao + off[j] + c] = v;
            outs[k][(size_t)(off[j] + c) * nao + off[i] + r] = v;
          }
      }
    }
  double e = 0.0;
  for (int a = 0; a < natom; ++a)
    for (int b = 0; b < a; ++b) {
      double r2 = 0.0;
      for (int d = 0; d < 3; ++d) r2 += (coords[3 * a + d] - coords[3 * b + d]) * (coords[3 * a + d] - coords[3 * b + d]);
      e += charges[a] * charges[b] / std::sqrt(r2);
    }
  *enuc = e;
  return JK_OK;
}
