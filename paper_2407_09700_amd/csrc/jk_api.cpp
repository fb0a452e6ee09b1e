// Host side of the J/K library: argument validation, shell-pair planning, the
// Cauchy-Schwarz pass, the per-build screening and the class launches (C ABI in jk.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/jk.h"
#include "jk_aux.h"
#include "jk_classes.h"
#include "jk_grad.h"
#include "jk_host.h"
#include "jk_kernels.h"

using namespace jk;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                             \
  do {                                                                                           \
    hipError_t e_ = (expr);                                                                      \
    if (e_ != hipSuccess) {                                                                      \
      if (e_ == hipErrorOutOfMemory) return fail(JK_ENOMEM, "%s: %s", #expr, hipGetErrorString(e_)); \
      return fail(JK_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));                          \
    }                                                                                            \
  } while (0)

ClassInfo g_classes[NQCLASS];
BraInfo g_bras[NPAIRCLASS];
grad_launch_fn g_grad[NQCLASS];
bool g_classes_ready = false;

void ensure_classes() {
  if (g_classes_ready) return;
  register_bra_00(g_classes, g_bras); register_bra_10(g_classes, g_bras); register_bra_11(g_classes, g_bras);
  register_bra_20(g_classes, g_bras); register_bra_21(g_classes, g_bras); register_bra_22(g_classes, g_bras);
  register_bra_30(g_classes, g_bras); register_bra_31(g_classes, g_bras); register_bra_32(g_classes, g_bras);
  register_bra_33(g_classes, g_bras); register_bra_40(g_classes, g_bras); register_bra_41(g_classes, g_bras);
  register_bra_42(g_classes, g_bras); register_bra_43(g_classes, g_bras); register_bra_44(g_classes, g_bras);
  register_grad(g_grad);
  g_classes_ready = true;
}

// ------------------------------------------------------------------ solid harmonics
double fact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}
double binomd(int n, int k) { return (k < 0 || k > n) ? 0.0 : fact(n) / (fact(k) * fact(n - k)); }

int cart_index(int l, int ax, int ay) {   // position of (ax, ay, l-ax-ay) in ax-desc, ay-desc order
  int idx = 0;
  for (int x = l; x > ax; --x) idx += l - x + 1;
  return idx + (l - ax - ay);
}

// Real solid harmonics in Racah normalisation from the closed form of Helgaker,
// Joergensen & Olsen, "Molecular Electronic-Structure Theory", eq. 6.4.47-6.4.50:
// S_lm = N_lm sum_{t,u,v} C^{lm}_{tuv} x^(2t+|m|-2(u+v)) y^(2(u+v)) z^(l-2t-|m|).
void solid_harmonics(int l, double *T) {
  const int nc = (l + 1) * (l + 2) / 2;
  for (int i = 0; i < (2 * l + 1) * nc; ++i) T[i] = 0.0;
  for (int m = -l; m <= l; ++m) {
    const int am = std::abs(m);
    double *row = T + (m + l) * nc;
    const double nlm = 1.0 / (std::pow(2.0, am) * fact(l)) *
                       std::sqrt(2.0 * fact(l + am) * fact(l - am) / (m == 0 ? 2.0 : 1.0));
    const double vm = m < 0 ? 0.5 : 0.0;
    for (int t = 0; t <= (l - am) / 2; ++t)
      for (int u = 0; u <= t; ++u) {
        const int vmax2 = (int)std::floor(am / 2.0 - vm);   // v = vm + j, j = 0..vmax2
        for (int j = 0; j <= vmax2; ++j) {
          const double v = vm + j;
          const int v2 = (int)std::lround(2 * v);
          const double sgn = ((t + (int)std::lround(v - vm)) % 2) ? -1.0 : 1.0;
          const double c = sgn * std::pow(0.25, t) * binomd(l, t) * binomd(l - t, am + t) * binomd(t, u) *
                           binomd(am, v2);
          const int px = 2 * t + am - 2 * u - v2, py = 2 * u + v2, pz = l - 2 * t - am;
          if (px < 0 || py < 0 || pz < 0) continue;
          row[cart_index(l, px, py)] += nlm * c;
        }
      }
    // sign convention: largest-magnitude coefficient positive (first on ties)
    double amax = 0.0;
    for (int k = 0; k < nc; ++k) amax = std::max(amax, std::fabs(row[k]));
    for (int k = 0; k < nc; ++k) {
      if (std::fabs(std::fabs(row[k]) - amax) <= 1e-12 * amax) {
        if (row[k] < 0)
          for (int q = 0; q < nc; ++q) row[q] = -row[q];
        break;
      }
    }
    for (int k = 0; k < nc; ++k)
      if (std::fabs(row[k]) < 1e-15) row[k] = 0.0;
  }
}

// ------------------------------------------------------------------ algorithmic operation counts
// Floating-point operations of the method for one class (an FMA counts 2), counted from its
// steps as an efficient implementation runs them (no divergence, masking or recomputation, no
// multiplication by a constant 1):
//  per primitive quartet:  scalars p, q, P-Q, P-A, Q-C, rho, T, prefactor (24);
//                          per root: interpolated u and w (2 x 11 FMAs = 44), the recurrence
//                          coefficients and the three C00/C00' pairs (14), the 2D recurrence in
//                          three directions (the x and y tables start from 1, so their first
//                          step in e and in f is free; the multiples e b10, e b00, f b01 are
//                          shared by the directions), and the Rys product over the [e0|f0]
//                          elements: one FMA each with the z integral, after one product of the
//                          x and y integrals per distinct (x, y) index set (elements that differ
//                          only in z share it);
//  per contracted quartet: the two binomial transfers, with their coefficients (three products
//                          each) formed once per quartet and a component k = b term of unit
//                          coefficient taken as the start value, and the digestion (six FMAs per
//                          integral, Algorithm 2: two for J, four for K, so a J-only or K-only
//                          build counts only its own).
double vrr_ops(int E, int F) {                               // one direction, table start g00
  double n = E > 0 ? 1 : 0;                                  // G[1][0] = C00 g00
  for (int e = 1; e < E; ++e) n += 1 + 2;                    // (e b10) G[e-1], fma
  for (int f = 0; f < F; ++f)
    for (int e = 0; e <= E; ++e) n += 1 + (f > 0 ? 2 : 0) + (e > 0 ? 2 : 0);
  return n;
}

int range_count_h(int l0, int l1) {
  int n = 0;
  for (int l = l0; l <= l1; ++l) n += ncart(l);
  return n;
}

// transfer terms of one shell: sum over its Cartesian components of (x+1)(y+1)(z+1)
int transfer_terms(int l) {
  int n = 0;
  for (int x = l; x >= 0; --x)
    for (int y = l - x; y >= 0; --y) n += (x + 1) * (y + 1) * (l - x - y + 1);
  return n;
}

// distinct (x, y) index sets of the products Gx[e][f] Gy[e][f] over the [e0|f0] elements
int distinct_xy(int la, int E, int lc, int F) {
  std::vector<char> seen((size_t)(E + 1) * (E + 1) * (F + 1) * (F + 1), 0);
  int n = 0;
  for (int le = la; le <= E; ++le)
    for (int ex = le; ex >= 0; --ex)
      for (int ey = le - ex; ey >= 0; --ey)
        for (int lf = lc; lf <= F; ++lf)
          for (int fx = lf; fx >= 0; --fx)
            for (int fy = lf - fx; fy >= 0; --fy) {
              char &s = seen[(((size_t)ex * (E + 1) + ey) * (F + 1) + fx) * (F + 1) + fy];
              if (!s) {
                s = 1;
                ++n;
              }
            }
  return n;
}

void class_ops(int la, int lb, int lc, int ld, int want, double *per_prim, double *per_quartet) {
  const int E = la + lb, F = lc + ld, N = (E + F) / 2 + 1;
  const int NE = range_count_h(la, E), NF = range_count_h(lc, F);
  const int na = ncart(la), nb = ncart(lb), nc = ncart(lc), nd = ncart(ld);
  const double vrr = 3.0 * vrr_ops(E, F) - 2.0 * ((E > 0) + (F > 0)) + 2.0 * std::max(0, E - 1) + std::max(0, F - 1);
  *per_prim = 24.0 + N * (44.0 + 14.0 + vrr + distinct_xy(la, E, lc, F) + 2.0 * NE * NF);
  // transfer: per output, one FMA per term other than the unit one
  const double bra = 2.0 * na * NF * (transfer_terms(lb) - ncart(lb)) + 3.0 * transfer_terms(lb);
  const double ket = 2.0 * na * nb * nc * (transfer_terms(ld) - ncart(ld)) + 3.0 * transfer_terms(ld);
  const double digest = (want & 1 ? 4.0 : 0.0) + (want & 2 ? 8.0 : 0.0);   // two J and four K FMAs per integral
  *per_quartet = bra + ket + digest * na * nb * nc * nd;
}

// Device memory of the no-allocation entry point: while a call of jk_build_static runs on this
// thread, every device buffer of its plan is carved from the static scratch array (bump
// allocation, no frees) instead of hipMalloc.
struct Arena {
  char *base;     // device address of the array on the current device
  size_t size, used;
};
thread_local Arena *g_arena = nullptr;

template <class T>
int dalloc(T **p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  if (g_arena) {
    const size_t bytes = (n * sizeof(T) + 255) & ~(size_t)255;
    if (bytes > g_arena->size - g_arena->used)
      return fail(JK_ENOMEM, "jk_build_static: the build needs more than the %zu MB of static scratch "
                  "(%zu MB used, %zu more bytes requested); use jk_build", g_arena->size >> 20,
                  g_arena->used >> 20, bytes);
    *p = reinterpret_cast<T *>(g_arena->base + g_arena->used);
    g_arena->used += bytes;
    return JK_OK;
  }
  hipError_t e = hipMalloc((void **)p, n * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? JK_ENOMEM : JK_EDEVICE, "hipMalloc(%zu bytes): %s", n * sizeof(T),
                hipGetErrorString(e));
  }
  return JK_OK;
}

template <class T>
int dupload(T **p, const std::vector<T> &v) {
  int rc = dalloc(p, v.size());
  if (rc) return rc;
  if (!v.empty()) HIPCHK(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return JK_OK;
}

template <class T>
void dfree(T *&p) {
  if (p && !g_arena) (void)hipFree(p);
  p = nullptr;
}

}  // namespace

struct jk_plan {
  int nmol = 0, nshell = 0, nao = 0, nc = 0, nc_max = 0;
  double tau = 1e-12;
  int precision = JK_FP64;
  double fp32_cutoff = 1e-6;
  int flags = 0;
  std::string tune_cache;
  std::vector<int> l, pure, cart_off, ao_off;    // per shell of the batch (offsets inside its molecule)
  std::vector<int> sbase, cbase, abase;          // [nmol+1] first shell / Cartesian AO / AO of each molecule
  std::vector<long long> mc_off, mf_off, ps_off; // [nmol+1] first element of each molecule's nc^2 / nao^2 / ns^2 block
  std::vector<int> mnc;                          // [nmol] Cartesian AO count of each molecule
  std::vector<int> lseg;                         // [nmol * 6] start of each momentum's columns in the molecule's lcols
  // Molecules are kept in ascending Cartesian size (so that, inside a pair class, the pairs
  // of the molecules whose exchange rows fit in LDS come first); perm[i] is the caller's
  // index of molecule i, user_off/user_nao describe the caller's packed D, J, K.
  std::vector<int> perm;
  std::vector<long long> mf_user, user_off;
  std::vector<int> user_nao;
  std::vector<double> schwarz;                   // per molecule ns x ns, at ps_off
  int npairs = 0;
  std::vector<int> cls_beg;                      // [16] first kept pair of each pair class
  std::vector<int> cm_beg;                       // [15 (nmol+1)] first kept pair of each (class, molecule)
  std::vector<char> possible;                    // [120] class can hold quartets (both pair classes in one molecule)
  // device
  Pair *d_pairs = nullptr;
  PrimPair *d_pp = nullptr;
  double *d_pairI = nullptr;
  int *d_pair_cls = nullptr, *d_pair_sa = nullptr, *d_pair_sb = nullptr, *d_cls_beg = nullptr;
  int *d_pair_mol = nullptr, *d_bin_beg = nullptr, *d_cm_bin = nullptr;
  int *d_l = nullptr, *d_pure = nullptr, *d_cart_off = nullptr, *d_ao_off = nullptr;
  int *d_cart2shell = nullptr, *d_ao2shell = nullptr;
  int *d_sbase = nullptr, *d_cbase = nullptr, *d_abase = nullptr, *d_mnc = nullptr;
  int *d_lcol = nullptr, *d_lcols = nullptr, *d_lseg = nullptr;   // compacted exchange rows (JKArgs)
  double *d_ppab = nullptr;            // exponents of the two primitives of every primitive pair
  double *d_pairP = nullptr;           // per kept pair: block maximum of its shells (per build)
  int *d_shell_atom = nullptr;         // per shell: its atom (nuclear gradient)
  int natom = 0, lmax = 0;
  long long *d_mc_off = nullptr, *d_mf_off = nullptr, *d_ps_off = nullptr, *d_mf_user = nullptr;
  double *d_tsph = nullptr;
  double *d_Dp = nullptr;   // Cartesian densities in shell panels (launch_dcart)
  double *d_Dc = nullptr, *d_Jc = nullptr, *d_Kc = nullptr, *d_Pblk = nullptr, *d_gmax = nullptr;
  unsigned long long *d_cap = nullptr, *d_nprim = nullptr;
  int *d_count = nullptr, *d_pair_npp = nullptr;
  int *d_pair_ca = nullptr, *d_pair_cb = nullptr, *d_pair_la = nullptr, *d_pair_lb = nullptr;
  int *d_segoff = nullptr, *d_segcnt = nullptr, *d_next = nullptr;
  int *d_segoff32 = nullptr, *d_segcnt32 = nullptr, *d_count32 = nullptr;   // mixed precision
  int2 *d_units = nullptr;             // work units of the current launch (bra pair, slice)
  int units_cap = 0;
  int *d_nunits = nullptr;             // [NSLOT] unit count per launch slot
  std::vector<int> slice, units_est;   // per launch slot: kets per unit, expected units (last eager build)
  long long *d_class_off = nullptr, *d_jp_off = nullptr, *d_room = nullptr;
  int *d_overflow = nullptr;
  // work-list sizing: class regions are laid out once (plan creation with a density bound, or
  // the first execute) and grow only when a build reports an overflow
  double dmax = 0.0;
  bool sized = false;
  std::vector<long long> capc, class_off_h;      // [120] capacity and first entry of each class region
  long long *d_capc = nullptr;
  bool active[NQCLASS] = {};                     // classes launched by every build (capacity > 0)
  long long overflows = 0;                       // builds reported incomplete by jk_plan_check
  double *d_Jpair = nullptr, *d_Dpair = nullptr;
  long long jp_total = 0;
  std::vector<long long> jp_off;                 // [15]
  hipStream_t last_stream = nullptr;
  // profile events: EV_SETS sets of 2 per launch slot + prep + tail; execute n records into set
  // n mod EV_SETS, jk_profile averages the sets recorded since its last call
  std::vector<hipEvent_t> events;
  int ev_next = 0, ev_count = 0;
  std::vector<int> launched;           // launch slots used by the last eager execute
  std::vector<int> ev_launched;        // launch slots of the builds in the event ring (one launch set)
  std::vector<int> grid;               // per launch slot: workgroups (0 = default)
  bool tuned = false;
  std::vector<char> fuse;              // [NFUSED] lane tier (cb, tier) runs fused (1) or per class (0)
  std::vector<char> shape;             // [NQCLASS] per-class launch shape (SHAPE_* bits; tuner's choice)
  int *d_kets = nullptr;
  long long list_capacity = 0;
  double *d_scratch = nullptr;
  long long scratch_doubles = 0;
  ShellInfo S{};
  jk_stats_t stats{};
  int device = 0;
  // graph replay
  hipStream_t rec_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const double *gD = nullptr;
  double *gJ = nullptr, *gK = nullptr;
  bool graph_stale = false;
  long long replays = 0;
  int rerecords = 0;
};

struct jk_batch {
  jk_plan *p = nullptr;
};

namespace {

void graph_free(jk_plan *p) {
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->gexec = nullptr;
  p->graph = nullptr;
}

void plan_free(jk_plan *p) {
  graph_free(p);
  if (p->rec_stream) (void)hipStreamDestroy(p->rec_stream);
  p->rec_stream = nullptr;
  dfree(p->d_pairs); dfree(p->d_pp); dfree(p->d_pairI); dfree(p->d_pair_cls); dfree(p->d_pair_sa);
  dfree(p->d_pair_sb); dfree(p->d_cls_beg); dfree(p->d_pair_mol); dfree(p->d_bin_beg); dfree(p->d_cm_bin); dfree(p->d_l);
  dfree(p->d_pure); dfree(p->d_cart_off); dfree(p->d_ao_off); dfree(p->d_cart2shell); dfree(p->d_ao2shell);
  dfree(p->d_sbase); dfree(p->d_cbase); dfree(p->d_abase); dfree(p->d_mnc); dfree(p->d_mc_off);
  dfree(p->d_mf_off); dfree(p->d_ps_off); dfree(p->d_mf_user); dfree(p->d_tsph); dfree(p->d_Dc); dfree(p->d_Dp);
  dfree(p->d_Jc); dfree(p->d_Kc); dfree(p->d_Pblk); dfree(p->d_gmax); dfree(p->d_cap); dfree(p->d_count);
  dfree(p->d_kets); dfree(p->d_scratch); dfree(p->d_nprim); dfree(p->d_pair_npp);
  dfree(p->d_pair_ca); dfree(p->d_pair_cb); dfree(p->d_pair_la); dfree(p->d_pair_lb); dfree(p->d_segoff);
  dfree(p->d_segcnt); dfree(p->d_next); dfree(p->d_class_off); dfree(p->d_jp_off); dfree(p->d_Jpair); dfree(p->d_Dpair);
  dfree(p->d_room); dfree(p->d_overflow); dfree(p->d_capc);
  dfree(p->d_lcol); dfree(p->d_lcols); dfree(p->d_lseg); dfree(p->d_ppab); dfree(p->d_shell_atom); dfree(p->d_pairP); dfree(p->d_units); dfree(p->d_nunits); dfree(p->d_segoff32); dfree(p->d_segcnt32); dfree(p->d_count32);
  for (hipEvent_t e : p->events) (void)hipEventDestroy(e);
  p->events.clear();
}

// per-class launches of the lane bodies keep the unit's exchange rows in LDS (compacted to the
// ket class's momenta) when they fit; 0 sends every exchange update to global memory
#ifndef JK_CLS_LDS_ROWS
#define JK_CLS_LDS_ROWS 1
#endif
// default for the lane tiers of a bra class: fused over their ket classes (1: one launch, full
// exchange rows in LDS) or per-class launches with compacted rows (0); the tuner picks per tier
#ifndef JK_FUSE_LANE_TIERS
#define JK_FUSE_LANE_TIERS 0
#endif
constexpr int GRID_SMALL_MAX = 4096;   // workgroups of 256 lanes (lane-per-quartet mode kernels)
constexpr int GRID_TEAM_MAX = 1024;    // persistent workgroups of the J/K kernels and team mode kernels (default)
constexpr size_t FUSED_LDS_MAX = 150 * 1024;   // dynamic LDS of k_bra (the CU has 160 KB)
// Shapes of a per-class lane-body launch with LDS exchange rows, picked per class by the tuner:
// the default (root table in LDS where it fits, rows of a and b in LDS where they fit), or
// without the root table in LDS, or with only the rows of a in LDS (the rows of b keep as many
// leading columns as the rest of the LDS holds).
constexpr int SHAPE_NO_TABLE = 1, SHAPE_ROWS_A = 2, NSHAPE = 3;
constexpr int NFUSED = NPAIRCLASS * NTIERS;     // launch slots of the fused kernels
constexpr int NF32_BASE = NFUSED + NQCLASS;    // slots of the FP32-only fused launches (mixed precision)
constexpr int NSLOT = NF32_BASE + NFUSED;
constexpr int EV_PER_SET = 2 * NSLOT + 4;          // profile events of one execute
constexpr int EV_SETS = 32;                        // executes a profile can average over
const int TUNE_GRIDS[] = {256, 512, 1024, 2048};   // candidates of the grid tuner

int ensure_scratch(jk_plan *p, long long doubles) {
  if (doubles <= p->scratch_doubles) return JK_OK;
  dfree(p->d_scratch);
  p->scratch_doubles = 0;
  p->graph_stale = true;
  int rc = dalloc(&p->d_scratch, (size_t)doubles);
  if (rc) return rc;
  p->scratch_doubles = doubles;
  return JK_OK;
}

// A primitive pair whose Gaussian product factor exp(-ab/(a+b) |AB|^2) is below exp(-60)
// (8.8e-27) is left out of its shell pair: its share of any integral lies some ten orders of
// magnitude below the rounding of the FP64 result.
constexpr double PRIM_EXP_CUT = 60.0;

// Primitive pairs and pair records of every shell pair i >= j of one molecule (canonical
// order l_a >= l_b inside the pair). s0: first shell of the molecule in the batch; shell
// indices of the records are batch-wide, Cartesian offsets are inside the molecule.
void build_pairs(const jk_basis_t *B, const double *coords, const int *cart_off, int s0, int mol,
                 std::vector<Pair> &pairs, std::vector<PrimPair> &pps, std::vector<double> &ppab) {
  const int ns = B->nshell;
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j <= i; ++j) {
      int a = i, b = j;
      if (B->l[i] < B->l[j]) std::swap(a, b);
      Pair P{};
      const double *A = coords + 3 * B->atom[a], *Bc = coords + 3 * B->atom[b];
      double ab2 = 0;
      for (int d = 0; d < 3; ++d) {
        P.A[d] = A[d];
        P.B[d] = Bc[d];
        ab2 += (A[d] - Bc[d]) * (A[d] - Bc[d]);
      }
      P.sa = s0 + a; P.sb = s0 + b;
      P.ca = cart_off[a]; P.cb = cart_off[b];
      P.pp_off = (int)pps.size();
      P.cls = pair_class(B->l[a], B->l[b]);
      P.mol = mol;
      for (int ka = 0; ka < B->nprim[a]; ++ka)
        for (int kb = 0; kb < B->nprim[b]; ++kb) {
          const double ea = B->exps[B->prim_off[a] + ka], eb = B->exps[B->prim_off[b] + kb];
          const double ca = B->coefs[B->prim_off[a] + ka], cb = B->coefs[B->prim_off[b] + kb];
          if (ea * eb / (ea + eb) * ab2 > PRIM_EXP_CUT) continue;
          PrimPair q{};
          q.p = ea + eb;
          q.Px = (ea * A[0] + eb * Bc[0]) / q.p;
          q.Py = (ea * A[1] + eb * Bc[1]) / q.p;
          q.Pz = (ea * A[2] + eb * Bc[2]) / q.p;
          q.K = ca * cb * std::exp(-ea * eb / q.p * ab2);
          q.ip = 1.0 / q.p;
          pps.push_back(q);
          ppab.push_back(ea);      // exponents of the two primitives (nuclear gradient)
          ppab.push_back(eb);
        }
      P.npp = (int)pps.size() - P.pp_off;
      pairs.push_back(P);
    }
}
int validate(const jk_basis_t *B, const double *coords, int natom) {
  if (!B) return fail(JK_EINVAL, "basis is NULL");
  if (!coords) return fail(JK_EINVAL, "coords is NULL");
  if (natom <= 0) return fail(JK_EINVAL, "natom must be positive (got %d)", natom);
  if (B->nshell <= 0) return fail(JK_EINVAL, "nshell must be positive (got %d)", B->nshell);
  if (!B->atom || !B->l || !B->nprim || !B->prim_off || !B->pure || !B->exps || !B->coefs)
    return fail(JK_EINVAL, "a basis array is NULL");
  if (B->nprim_total <= 0) return fail(JK_EINVAL, "nprim_total must be positive");
  for (int a = 0; a < 3 * natom; ++a)
    if (!std::isfinite(coords[a])) return fail(JK_EINVAL, "coordinate %d is not finite", a);
  for (int s = 0; s < B->nshell; ++s) {
    if (B->l[s] < 0) return fail(JK_EINVAL, "shell %d: negative l", s);
    if (B->l[s] > LMAX) return fail(JK_EUNSUPPORTED, "shell %d: l = %d > %d", s, B->l[s], LMAX);
    if (B->nprim[s] <= 0) return fail(JK_EINVAL, "shell %d: nprim must be positive", s);
    if (B->nprim[s] > 64) return fail(JK_EUNSUPPORTED, "shell %d: nprim = %d > 64", s, B->nprim[s]);
    if (B->atom[s] < 0 || B->atom[s] >= natom) return fail(JK_EINVAL, "shell %d: atom %d out of range", s, B->atom[s]);
    if (B->prim_off[s] < 0 || B->prim_off[s] + B->nprim[s] > B->nprim_total)
      return fail(JK_EINVAL, "shell %d: primitive range out of bounds", s);
    if (B->pure[s] != 0 && B->pure[s] != 1) return fail(JK_EINVAL, "shell %d: pure must be 0 or 1", s);
    for (int k = 0; k < B->nprim[s]; ++k) {
      const double e = B->exps[B->prim_off[s] + k], c = B->coefs[B->prim_off[s] + k];
      if (!(e > 0.0) || !std::isfinite(e)) return fail(JK_EINVAL, "shell %d: exponent %d not positive/finite", s, k);
      if (!std::isfinite(c)) return fail(JK_EINVAL, "shell %d: coefficient %d not finite", s, k);
    }
  }
  return JK_OK;
}

int launch_mode_list(jk_plan *p, int qc, int mode, const int2 *list, int count, double *out, hipStream_t st) {
  const ClassInfo &ci = g_classes[qc];
  if (!ci.launch_mode[mode]) return fail(JK_EUNSUPPORTED, "class %d has no launcher for mode %d", qc, mode);
  if (count <= 0) return JK_OK;
  long long g = ((long long)count + ci.per_block - 1) / ci.per_block;
  const int grid = (int)std::max(1LL, std::min(g, (long long)(ci.team ? GRID_TEAM_MAX : GRID_SMALL_MAX)));
  if (ci.scratch_per_wg > 0) {
    int rc = ensure_scratch(p, ci.scratch_per_wg * (long long)grid);
    if (rc) return rc;
  }
  ModeArgs m{};
  m.pairs = p->d_pairs;
  m.pp = p->d_pp;
  m.quartets = list;
  m.count = count;
  m.out = out;
  m.scratch = p->d_scratch;
  m.scratch_per_wg = ci.scratch_per_wg;
  m.nc = p->nc;   // ERI tensor: single-molecule plans only
  HIPCHK(ci.launch_mode[mode](m, grid, st));
  return JK_OK;
}


int parse_opts(const jk_opts_t *opts, jk_plan *p) {
  p->tau = 1e-12;
  p->precision = JK_FP64;
  p->fp32_cutoff = 1e-6;
  p->flags = 0;
  p->dmax = 0.0;
  if (!opts) return JK_OK;
  if (!(opts->thresh >= 0.0) || !std::isfinite(opts->thresh)) return fail(JK_EINVAL, "thresh must be finite and >= 0");
  if (opts->precision != JK_FP64 && opts->precision != JK_MIXED)
    return fail(JK_EINVAL, "unknown precision %d", opts->precision);
  if (!(opts->fp32_cutoff >= 0.0) || !std::isfinite(opts->fp32_cutoff))
    return fail(JK_EINVAL, "fp32_cutoff must be finite and >= 0");
  if (opts->flags & ~(JK_FLAG_PROFILE | JK_FLAG_GRAPH | JK_FLAG_TUNE | JK_FLAG_J_ONLY | JK_FLAG_K_ONLY))
    return fail(JK_EINVAL, "unknown flags 0x%x", opts->flags);
  if ((opts->flags & JK_FLAG_J_ONLY) && (opts->flags & JK_FLAG_K_ONLY))
    return fail(JK_EINVAL, "JK_FLAG_J_ONLY and JK_FLAG_K_ONLY exclude each other");
  if (!(opts->dmax >= 0.0) || !std::isfinite(opts->dmax)) return fail(JK_EINVAL, "dmax must be finite and >= 0");
  p->dmax = opts->dmax;
  p->tau = opts->thresh;
  p->precision = opts->precision;
  p->fp32_cutoff = opts->fp32_cutoff;
  p->flags = opts->flags;
  if (opts->tune_cache) p->tune_cache = opts->tune_cache;
  return JK_OK;
}

int size_lists(jk_plan *p, hipStream_t st, double gfix, double gscale);

// Plan of nmol molecules (a single-molecule plan is the batch of one).
int plan_create(int nmol, const jk_basis_t *const *Bs_in, const double *const *coords_in, const int *natom,
                const jk_opts_t *opts, jk_plan **out) {
  *out = nullptr;
  if (nmol <= 0) return fail(JK_EINVAL, "nmol must be positive (got %d)", nmol);
  if (!Bs_in || !coords_in || !natom) return fail(JK_EINVAL, "basis, coords and natom arrays must not be NULL");
  for (int m = 0; m < nmol; ++m) {
    int rc = validate(Bs_in[m], coords_in[m], natom[m]);
    if (rc) {
      if (nmol > 1) g_err = "molecule " + std::to_string(m) + ": " + g_err;
      return rc;
    }
  }
  jk_plan tmp;
  int rc = parse_opts(opts, &tmp);
  if (rc) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(JK_ENODEV, "no HIP device");
  ensure_classes();
  const auto t0 = std::chrono::steady_clock::now();

  jk_plan *p = new jk_plan();
  p->tau = tmp.tau;
  p->precision = tmp.precision;
  p->fp32_cutoff = tmp.fp32_cutoff;
  p->flags = tmp.flags;
  p->dmax = tmp.dmax;
  p->tune_cache = tmp.tune_cache;
  p->nmol = nmol;
  (void)hipGetDevice(&p->device);
  auto cleanup = [&](int code) {
    plan_free(p);
    delete p;
    return code;
  };

  // caller's packing, then the internal order (ascending Cartesian size, stable)
  p->user_off.assign(nmol + 1, 0);
  p->user_nao.assign(nmol, 0);
  std::vector<int> ncu(nmol, 0);
  for (int m = 0; m < nmol; ++m) {
    int na = 0;
    for (int s = 0; s < Bs_in[m]->nshell; ++s) {
      const int l = Bs_in[m]->l[s];
      ncu[m] += ncart(l);
      na += (Bs_in[m]->pure[s] && l >= 2) ? 2 * l + 1 : ncart(l);
    }
    p->user_nao[m] = na;
    p->user_off[m + 1] = p->user_off[m] + (long long)na * na;
  }
  p->perm.resize(nmol);
  std::iota(p->perm.begin(), p->perm.end(), 0);
  std::stable_sort(p->perm.begin(), p->perm.end(), [&](int x, int y) { return ncu[x] < ncu[y]; });
  std::vector<const jk_basis_t *> Bv(nmol);
  std::vector<const double *> Cv(nmol);
  p->mf_user.resize(nmol);
  for (int i = 0; i < nmol; ++i) {
    Bv[i] = Bs_in[p->perm[i]];
    Cv[i] = coords_in[p->perm[i]];
    p->mf_user[i] = p->user_off[p->perm[i]];
  }
  const jk_basis_t *const *Bs = Bv.data();
  const double *const *coords = Cv.data();

  // per-molecule layout
  std::vector<int> shell_atom;
  p->natom = natom[p->perm[0]];
  p->sbase.assign(nmol + 1, 0); p->cbase.assign(nmol + 1, 0); p->abase.assign(nmol + 1, 0);
  p->mc_off.assign(nmol + 1, 0); p->mf_off.assign(nmol + 1, 0); p->ps_off.assign(nmol + 1, 0);
  p->mnc.assign(nmol, 0);
  for (int m = 0; m < nmol; ++m) {
    const jk_basis_t *B = Bs[m];
    int nc = 0, na = 0;
    for (int s = 0; s < B->nshell; ++s) {
      const int l = B->l[s];
      shell_atom.push_back(B->atom[s]);
      p->lmax = std::max(p->lmax, l);
      p->l.push_back(l);
      p->pure.push_back(B->pure[s]);
      p->cart_off.push_back(nc);
      p->ao_off.push_back(na);
      nc += ncart(l);
      na += (B->pure[s] && l >= 2) ? 2 * l + 1 : ncart(l);
    }
    p->sbase[m + 1] = p->sbase[m] + B->nshell;
    p->cbase[m + 1] = p->cbase[m] + nc;
    p->abase[m + 1] = p->abase[m] + na;
    p->mnc[m] = nc;
    p->nc_max = std::max(p->nc_max, nc);
    p->mc_off[m + 1] = p->mc_off[m] + (long long)nc * nc;
    p->mf_off[m + 1] = p->mf_off[m] + (long long)na * na;
    p->ps_off[m + 1] = p->ps_off[m] + (long long)B->nshell * B->nshell;
  }
  const int ns = p->nshell = p->sbase[nmol];
  p->nc = p->cbase[nmol];
  p->nao = p->abase[nmol];

  // shell tables
  std::vector<int> c2s(p->nc), a2s(p->nao);
  for (int m = 0; m < nmol; ++m)
    for (int s = p->sbase[m]; s < p->sbase[m + 1]; ++s) {
      const int l = p->l[s];
      const int nf = (p->pure[s] && l >= 2) ? 2 * l + 1 : ncart(l);
      for (int k = 0; k < ncart(l); ++k) c2s[p->cbase[m] + p->cart_off[s] + k] = s;
      for (int k = 0; k < nf; ++k) a2s[p->abase[m] + p->ao_off[s] + k] = s;
    }
  // columns by momentum: per molecule, the Cartesian columns of its s shells, then p, ..., g
  // shells (lcols), where each momentum starts (lseg), and each shell's first column inside
  // its momentum's segment (lcol)
  std::vector<int> lcol(ns), lcols(p->nc);
  p->lseg.assign((size_t)nmol * 6, 0);
  for (int m = 0; m < nmol; ++m) {
    int *seg = p->lseg.data() + (size_t)m * 6;
    int pos = 0;
    for (int l = 0; l <= LMAX; ++l) {
      seg[l] = pos;
      for (int s = p->sbase[m]; s < p->sbase[m + 1]; ++s) {
        if (p->l[s] != l) continue;
        lcol[s] = pos - seg[l];
        for (int k = 0; k < ncart(l); ++k) lcols[p->cbase[m] + pos++] = p->cart_off[s] + k;
      }
    }
    seg[LMAX + 1] = pos;
  }
  std::vector<double> tsph(5 * 6 + 7 * 10 + 9 * 15);

  solid_harmonics(2, tsph.data());
  solid_harmonics(3, tsph.data() + 30);
  solid_harmonics(4, tsph.data() + 100);
  if ((rc = dupload(&p->d_l, p->l)) || (rc = dupload(&p->d_pure, p->pure)) ||
      (rc = dupload(&p->d_cart_off, p->cart_off)) || (rc = dupload(&p->d_ao_off, p->ao_off)) ||
      (rc = dupload(&p->d_cart2shell, c2s)) || (rc = dupload(&p->d_ao2shell, a2s)) ||
      (rc = dupload(&p->d_tsph, tsph)) || (rc = dupload(&p->d_sbase, p->sbase)) ||
      (rc = dupload(&p->d_cbase, p->cbase)) || (rc = dupload(&p->d_abase, p->abase)) ||
      (rc = dupload(&p->d_mnc, p->mnc)) || (rc = dupload(&p->d_mc_off, p->mc_off)) ||
      (rc = dupload(&p->d_mf_off, p->mf_off)) || (rc = dupload(&p->d_ps_off, p->ps_off)) ||
      (rc = dupload(&p->d_mf_user, p->mf_user)) || (rc = dupload(&p->d_lcol, lcol)) ||
      (rc = dupload(&p->d_lcols, lcols)) || (rc = dupload(&p->d_lseg, p->lseg)) ||
      (rc = dupload(&p->d_shell_atom, shell_atom)))
    return cleanup(rc);
  ShellInfo &S = p->S;
  S.l = p->d_l; S.pure = p->d_pure; S.cart_off = p->d_cart_off; S.ao_off = p->d_ao_off;
  S.cart2shell = p->d_cart2shell; S.ao2shell = p->d_ao2shell; S.tsph = p->d_tsph;
  S.mc_off = p->d_mc_off; S.mf_off = p->d_mf_off; S.ps_off = p->d_ps_off; S.mf_user = p->d_mf_user;
  S.cbase = p->d_cbase; S.abase = p->d_abase; S.sbase = p->d_sbase;
  S.toff[0] = S.toff[1] = 0; S.toff[2] = 0; S.toff[3] = 30; S.toff[4] = 100;
  S.nmol = nmol;
  S.nc2_tot = p->mc_off[nmol]; S.nf2_tot = p->mf_off[nmol]; S.ns2_tot = p->ps_off[nmol];

  // all shell pairs of every molecule
  std::vector<Pair> all;
  std::vector<PrimPair> pps;
  std::vector<double> ppab;
  for (int m = 0; m < nmol; ++m)
    build_pairs(Bs[m], coords[m], p->cart_off.data() + p->sbase[m], p->sbase[m], m, all, pps, ppab);
  const int nall = (int)all.size();
  if (pps.size() > 0x7fffffffULL) return cleanup(fail(JK_EUNSUPPORTED, "more than 2^31 primitive pairs"));
  if ((rc = dupload(&p->d_pairs, all)) || (rc = dupload(&p->d_pp, pps))) return cleanup(rc);

  // Cauchy-Schwarz factors: the diagonal quartets (ab|ab), one class launch per pair class
  std::vector<double> smax(nall);
  {
    double *d_smax = nullptr;
    int2 *d_diag = nullptr;
    if ((rc = dalloc(&d_smax, nall)) || (rc = dalloc(&d_diag, nall))) {
      dfree(d_smax);
      return cleanup(rc);
    }
    std::vector<int2> diag(nall);
    std::vector<int> cnt(NPAIRCLASS, 0), beg(NPAIRCLASS + 1, 0);
    for (int i = 0; i < nall; ++i) cnt[all[i].cls]++;
    for (int c = 0; c < NPAIRCLASS; ++c) beg[c + 1] = beg[c] + cnt[c];
    std::vector<int> fillp(beg.begin(), beg.end() - 1);
    for (int i = 0; i < nall; ++i) diag[fillp[all[i].cls]++] = make_int2(i, i);
    hipError_t e = hipMemcpy(d_diag, diag.data(), sizeof(int2) * nall, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(d_smax, 0, sizeof(double) * nall);
    if (e != hipSuccess) {
      dfree(d_smax); dfree(d_diag);
      return cleanup(fail(JK_EDEVICE, "Schwarz setup: %s", hipGetErrorString(e)));
    }
    for (int c = 0; c < NPAIRCLASS && !rc; ++c) {
      if (!cnt[c]) continue;
      rc = launch_mode_list(p, qclass_index(c, c), MODE_SCHWARZ, d_diag + beg[c], cnt[c], d_smax, 0);
    }
    if (!rc) {
      e = hipDeviceSynchronize();
      if (e == hipSuccess) e = hipMemcpy(smax.data(), d_smax, sizeof(double) * nall, hipMemcpyDeviceToHost);
      if (e != hipSuccess) rc = fail(JK_EDEVICE, "Schwarz pass: %s", hipGetErrorString(e));
    }
    dfree(d_smax); dfree(d_diag);
    if (rc) return cleanup(rc);
  }
  p->schwarz.assign((size_t)p->ps_off[nmol], 0.0);
  for (int i = 0; i < nall; ++i) {
    const int m = all[i].mol;
    const int nsm = p->sbase[m + 1] - p->sbase[m];
    const int a = all[i].sa - p->sbase[m], b = all[i].sb - p->sbase[m];
    const double I = std::sqrt(smax[i]);
    p->schwarz[(size_t)p->ps_off[m] + (size_t)a * nsm + b] = I;
    p->schwarz[(size_t)p->ps_off[m] + (size_t)b * nsm + a] = I;
  }

  // keep pairs with I > tau, sorted by class, then molecule, then I descending (stable)
  std::vector<int> order;
  order.reserve(nall);
  for (int i = 0; i < nall; ++i)
    if (std::sqrt(smax[i]) > p->tau) order.push_back(i);
  // bins: inside a (class, molecule), pairs of equal contraction length npp are kept
  // together (sorted by I descending inside the bin), so that the kets the screen writes
  // next to each other -- the quartets of neighbouring lanes -- run the same number of
  // primitive quartets. More than MAX_BINS lengths in one (class, molecule): neighbouring
  // lengths share a bin.
  std::vector<int> bucket(nall, 0);
  {
    std::vector<std::vector<int>> lens((size_t)NPAIRCLASS * nmol);
    for (int i : order) lens[(size_t)all[i].cls * nmol + all[i].mol].push_back(all[i].npp);
    std::vector<std::vector<int>> uniq(lens.size());
    for (size_t g = 0; g < lens.size(); ++g) {
      auto &v = lens[g];
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    for (int i : order) {
      const auto &v = lens[(size_t)all[i].cls * nmol + all[i].mol];
      const int r = (int)(std::lower_bound(v.begin(), v.end(), all[i].npp) - v.begin());
      bucket[i] = (int)((long long)r * MAX_BINS / (long long)v.size());   // identity when <= MAX_BINS lengths
    }
  }
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (all[x].cls != all[y].cls) return all[x].cls < all[y].cls;
    if (all[x].mol != all[y].mol) return all[x].mol < all[y].mol;
    if (bucket[x] != bucket[y]) return bucket[x] < bucket[y];
    return smax[x] > smax[y];
  });
  p->npairs = (int)order.size();
  std::vector<Pair> kept(p->npairs);
  std::vector<PrimPair> kpp;
  std::vector<double> kppab;
  std::vector<double> kI(p->npairs);
  std::vector<int> kcls(p->npairs), ksa(p->npairs), ksb(p->npairs), knpp(p->npairs), kca(p->npairs),
      kcb(p->npairs), kla(p->npairs), klb(p->npairs), kmol(p->npairs);
  p->cls_beg.assign(NPAIRCLASS + 1, 0);
  p->cm_beg.assign((size_t)NPAIRCLASS * (nmol + 1), 0);
  std::vector<long long> cmcnt((size_t)NPAIRCLASS * nmol, 0);
  for (int k = 0; k < p->npairs; ++k) {
    Pair P = all[order[k]];
    const int off = (int)kpp.size();
    for (int q = 0; q < P.npp; ++q) {
      kpp.push_back(pps[P.pp_off + q]);
      kppab.push_back(ppab[2 * ((size_t)P.pp_off + q)]);
      kppab.push_back(ppab[2 * ((size_t)P.pp_off + q) + 1]);
    }
    P.pp_off = off;
    kept[k] = P;
    kI[k] = std::sqrt(smax[order[k]]);
    kcls[k] = P.cls; ksa[k] = P.sa; ksb[k] = P.sb; knpp[k] = P.npp;
    kca[k] = P.ca; kcb[k] = P.cb; kla[k] = p->l[P.sa]; klb[k] = p->l[P.sb]; kmol[k] = P.mol;
    p->cls_beg[P.cls + 1]++;
    cmcnt[(size_t)P.cls * nmol + P.mol]++;
  }
  for (int c = 0; c < NPAIRCLASS; ++c) p->cls_beg[c + 1] += p->cls_beg[c];
  for (int c = 0; c < NPAIRCLASS; ++c) {
    int *cm = p->cm_beg.data() + (size_t)c * (nmol + 1);
    cm[0] = p->cls_beg[c];
    for (int m = 0; m < nmol; ++m) cm[m + 1] = cm[m] + (int)cmcnt[(size_t)c * nmol + m];
  }
  // bins and the first bin of every (class, molecule)
  std::vector<int> bin_beg, cm_bin((size_t)NPAIRCLASS * (nmol + 1), 0);
  for (int k = 0; k < p->npairs; ++k)
    if (k == 0 || kcls[k] != kcls[k - 1] || kmol[k] != kmol[k - 1] || bucket[order[k]] != bucket[order[k - 1]])
      bin_beg.push_back(k);
  bin_beg.push_back(p->npairs);
  {
    size_t b = 0;
    for (int c = 0; c < NPAIRCLASS; ++c)
      for (int m = 0; m <= nmol; ++m) {
        const int first = p->cm_beg[(size_t)c * (nmol + 1) + m];   // first pair of (c, m)
        while (b + 1 < bin_beg.size() && bin_beg[b] < first) ++b;
        cm_bin[(size_t)c * (nmol + 1) + m] = (int)b;
      }
  }
  p->possible.assign(NQCLASS, 0);
  for (int cb = 0; cb < NPAIRCLASS; ++cb)
    for (int ck = 0; ck <= cb; ++ck)
      for (int m = 0; m < nmol; ++m)
        if (cmcnt[(size_t)cb * nmol + m] && cmcnt[(size_t)ck * nmol + m]) {
          p->possible[qclass_index(cb, ck)] = 1;
          break;
        }
  dfree(p->d_pairs);
  dfree(p->d_pp);
  if ((rc = dupload(&p->d_pairs, kept)) || (rc = dupload(&p->d_pp, kpp)) || (rc = dupload(&p->d_pairI, kI)) ||
      (rc = dupload(&p->d_ppab, kppab)) ||
      (rc = dupload(&p->d_pair_cls, kcls)) || (rc = dupload(&p->d_pair_sa, ksa)) ||
      (rc = dupload(&p->d_pair_sb, ksb)) || (rc = dupload(&p->d_cls_beg, p->cls_beg)) ||
      (rc = dupload(&p->d_pair_npp, knpp)) || (rc = dupload(&p->d_pair_ca, kca)) ||
      (rc = dupload(&p->d_pair_cb, kcb)) || (rc = dupload(&p->d_pair_la, kla)) ||
      (rc = dupload(&p->d_pair_lb, klb)) || (rc = dupload(&p->d_pair_mol, kmol)) ||
      (rc = dupload(&p->d_bin_beg, bin_beg)) || (rc = dupload(&p->d_cm_bin, cm_bin)))
    return cleanup(rc);
  // Coulomb pair buffer: per pair class, element-major over the pairs of the class
  p->jp_off.assign(NPAIRCLASS, 0);
  long long jt = 0;
  for (int c = 0; c < NPAIRCLASS; ++c) {
    p->jp_off[c] = jt;
    jt += (long long)(p->cls_beg[c + 1] - p->cls_beg[c]) * ncart(pc_la(c)) * ncart(pc_lb(c));
  }
  p->jp_total = jt;
  if ((rc = dupload(&p->d_jp_off, p->jp_off)) || (rc = dalloc(&p->d_Jpair, (size_t)std::max(1LL, jt))) ||
      (rc = dalloc(&p->d_Dpair, (size_t)std::max(1LL, jt))) ||
      (rc = dalloc(&p->d_segoff, (size_t)p->npairs * NPAIRCLASS)) ||
      (rc = dalloc(&p->d_segcnt, (size_t)p->npairs * NPAIRCLASS)) || (rc = dalloc(&p->d_count32, NQCLASS)) ||
      (rc = dalloc(&p->d_pairP, (size_t)std::max(1, p->npairs))))
    return cleanup(rc);
  if (p->precision == JK_MIXED && ((rc = dalloc(&p->d_segoff32, (size_t)p->npairs * NPAIRCLASS)) ||
                                   (rc = dalloc(&p->d_segcnt32, (size_t)p->npairs * NPAIRCLASS))))
    return cleanup(rc);

  // build workspace
  const size_t nc2 = (size_t)p->mc_off[nmol];
  if ((rc = dalloc(&p->d_Dc, nc2)) || (rc = dalloc(&p->d_Dp, nc2)) || (rc = dalloc(&p->d_Jc, nc2)) || (rc = dalloc(&p->d_Kc, nc2)) ||
      (rc = dalloc(&p->d_Pblk, (size_t)p->ps_off[nmol])) || (rc = dalloc(&p->d_gmax, 1)) ||
      (rc = dalloc(&p->d_cap, NQCLASS)) || (rc = dalloc(&p->d_count, NQCLASS)) ||
      (rc = dalloc(&p->d_nprim, 2 * NQCLASS)) || (rc = dalloc(&p->d_class_off, NQCLASS)) ||
      (rc = dalloc(&p->d_room, NQCLASS)) || (rc = dalloc(&p->d_overflow, 1)) || (rc = dalloc(&p->d_capc, NQCLASS)) ||
      (rc = dalloc(&p->d_next, NSLOT)) || (rc = dalloc(&p->d_nunits, NSLOT)))
    return cleanup(rc);
  if (hipMemset(p->d_overflow, 0, sizeof(int)) != hipSuccess) return cleanup(fail(JK_EDEVICE, "hipMemset failed"));
  p->capc.assign(NQCLASS, 0);
  p->class_off_h.assign(NQCLASS, 0);
  p->grid.assign(NSLOT, 0);
  p->slice.assign(NSLOT, 0);
  p->fuse.assign(NFUSED, 0);
  p->shape.assign(NQCLASS, 0);
  for (int f = 0; f < NFUSED; ++f) p->fuse[f] = (f % NTIERS == TEAM_TIER) ? 1 : JK_FUSE_LANE_TIERS;
  p->units_est.assign(NSLOT, 0);
  if (p->flags & (JK_FLAG_PROFILE | JK_FLAG_TUNE)) {
    p->events.resize((size_t)EV_SETS * EV_PER_SET, nullptr);
    for (auto &e : p->events)
      if (hipEventCreate(&e) != hipSuccess) return cleanup(fail(JK_EDEVICE, "hipEventCreate failed"));
  }
  if (p->flags & JK_FLAG_GRAPH) {
    if (hipStreamCreateWithFlags(&p->rec_stream, hipStreamNonBlocking) != hipSuccess) {
      p->rec_stream = nullptr;
      return cleanup(fail(JK_EDEVICE, "hipStreamCreate failed"));
    }
  }
  HIPCHK(hipDeviceSynchronize());
  if (p->dmax > 0.0 && (rc = size_lists(p, nullptr, p->dmax, 0.0))) return cleanup(rc);
  p->stats.npairs_kept = p->npairs;
  p->stats.nao = p->nao;
  p->stats.nao_cart = p->nc;
  p->stats.nshell = ns;
  p->stats.plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = p;
  return JK_OK;
}

// ------------------------------------------------------------------ the integral launches
struct Launch {
  int slot;          // profile/work-counter slot: cb * NTIERS + tier (fused) or NFUSED + qc
  int cb;            // bra pair class
  int tier;          // fused: register tier; per class: -1
  int qc;            // per class: quartet class; fused: -1
  int bra_beg, bra_end;   // bra pairs of the launch
  int mask;          // ket classes of the launch (bit ck)
  int parts;         // segment parts: 1 FP64, 2 FP32, 3 both
  bool f32;          // the FP32-only fused kernel
  int nc_max;        // fused: largest Cartesian size among the launch's molecules
  size_t lds;        // dynamic LDS bytes
  long long scratch_per_wg;
  int kw;            // per class with compacted LDS exchange rows: their length (0: global exchange)
  int krows;         // 1: rows of a and b in LDS, 2: rows of a, and the first kwb columns of the rows of b
  int kwb;
  bool gl;           // per class with LDS rows: the Boys grid in LDS as well
};

// Launches of one build. active[qc]: the class has work (eager) or may have work (recording).
// Inside a pair class the pairs are ordered by molecule size, so the bra pairs of the
// molecules whose two exchange rows fit in LDS form a prefix: that prefix runs in the fused
// kernel, the rest in the per-class kernels.
void plan_launches(const jk_plan *p, const bool *active, std::vector<Launch> &out) {
  out.clear();
  const int nmol = p->nmol;
  for (int cb = 0; cb < NPAIRCLASS; ++cb) {
    const int beg = p->cls_beg[cb], end = p->cls_beg[cb + 1];
    if (beg == end) continue;
    const BraInfo &bi = g_bras[cb];
    const int na = ncart(bi.la), nbb = ncart(bi.lb);
    for (int tier = 0; tier < NTIERS; ++tier) {
      bool any = false;
      for (int ck = 0; ck <= cb; ++ck) any = any || (((bi.tier_mask[tier] >> ck) & 1) && active[qclass_index(cb, ck)]);
      if (!any) continue;
      int split = beg, m_split = 0;
      if (bi.fusable[tier] && p->fuse[cb * NTIERS + tier]) {
        const size_t fixed = (size_t)((na * nbb + 1) & ~1) * 8 + (size_t)bi.pool_bytes[tier];   // jab_s, pool
        const long long fit = fixed < FUSED_LDS_MAX ? (long long)((FUSED_LDS_MAX - fixed) / ((size_t)(na + nbb) * 8)) : 0;
        int m = 0;
        while (m < nmol && p->mnc[m] <= fit) ++m;      // molecules are in ascending size
        split = p->cm_beg[(size_t)cb * (nmol + 1) + m];
        m_split = m;
        if (split > beg) {
          const int ncm = p->mnc[m - 1];
          const size_t lds = (size_t)(na + nbb) * ncm * 8 + fixed;
          // mixed precision: the FP32 parts of the lane tiers run in their own FP32-only kernel
          const bool sep = p->precision == JK_MIXED && bi.launch_bra32[tier] != nullptr;
          out.push_back(Launch{cb * NTIERS + tier, cb, tier, -1, beg, split, bi.tier_mask[tier], sep ? 1 : 3, false,
                               ncm, lds, bi.scratch_per_wg[tier], 0, 0, 0});
          if (sep)
            out.push_back(Launch{NF32_BASE + cb * NTIERS + tier, cb, tier, -1, beg, split, bi.tier_mask[tier], 2, true,
                                 ncm, lds, bi.scratch_per_wg[tier], 0, 0, 0});
        }
      }
      if (split == end) continue;
      for (int ck = 0; ck <= cb; ++ck) {
        const int qc = qclass_index(cb, ck);
        if (!((bi.tier_mask[tier] >> ck) & 1) || !active[qc]) continue;
        const ClassInfo &ci = g_classes[qc];
        const size_t jab = (size_t)((na * nbb + 1) & ~1) * 8;
        const size_t lds = jab + (size_t)ci.team_lds;   // jab_s, pool
        // lane bodies: the exchange rows of the unit in LDS, compacted to the columns of the
        // ket class's momenta, when they fit for every molecule of the launch (the rows of a
        // and b, else those of a)
        int kw = 0, krows = 0;
        if (JK_CLS_LDS_ROWS && ci.launch_clsl) {
          for (int m = m_split; m < nmol; ++m) {
            const int *seg = p->lseg.data() + (size_t)m * 6;
            const int w = seg[ci.lc + 1] - seg[ci.lc] + (ci.lc != ci.ld ? seg[ci.ld + 1] - seg[ci.ld] : 0);
            kw = std::max(kw, w);
          }
          if (kw > 0 && jab + (size_t)(na + nbb) * kw * 8 <= FUSED_LDS_MAX && !(p->shape[qc] & SHAPE_ROWS_A))
            krows = 1;
          else if (kw > 0 && jab + (size_t)na * kw * 8 <= FUSED_LDS_MAX)
            krows = 2;
          else
            kw = 0;
        }
        // lane bodies of few roots: their root table in LDS too, where it fits next to the rows of
        // a and b, or next to the rows of a (the rows of b then keep fewer columns in LDS)
        const size_t gbytes = (size_t)ci.table_lds;
        const bool gl = kw > 0 && ci.launch_clslg && !(p->shape[qc] & SHAPE_NO_TABLE) &&
                        (krows == 1 ? jab + (size_t)(na + nbb) * kw * 8 + gbytes <= FUSED_LDS_MAX
                                    : jab + (size_t)na * kw * 8 + gbytes <= FUSED_LDS_MAX);
        const size_t room = FUSED_LDS_MAX - (gl ? gbytes : 0);
        // rows of a only: the rest of the LDS holds the first kwb columns of the rows of b
        const int kwb = krows == 2 ? (int)std::min<size_t>((size_t)kw, (room - jab - (size_t)na * kw * 8) /
                                                                           ((size_t)nbb * 8))
                                   : 0;
        const size_t klds = jab + ((size_t)(krows == 1 ? na + nbb : na) * kw + (size_t)nbb * kwb) * 8 + (gl ? gbytes : 0);
        out.push_back(Launch{NFUSED + qc, cb, -1, qc, split, end, 1 << ck, 3, false, 0, kw ? klds : lds,
                             ci.scratch_per_wg, kw, krows, kwb, gl});
      }
    }
  }
}

int launch_grid(const jk_plan *p, const Launch &L) {
  const int nu = p->units_est[L.slot] > 0 ? p->units_est[L.slot] : L.bra_end - L.bra_beg;
  const int g = p->grid[L.slot] > 0 ? p->grid[L.slot] : GRID_TEAM_MAX;
  return std::max(1, std::min(nu, g));
}

constexpr long long TARGET_UNITS = 4096;   // work units per launch the slicing aims for (16 per CU)
constexpr int SLICE_MIN = 64;              // fewest kets per unit

// Kets per work unit of a launch from its candidate count (an upper bound of its kets): the
// whole bra when there are many bras, slices of the bra's kets when a few bras carry the work.
void size_units(jk_plan *p, const Launch &L, long long cand, long long *units_need) {
  const long long nbra = L.bra_end - L.bra_beg;
  long long sl = (cand + TARGET_UNITS - 1) / TARGET_UNITS;
  sl = std::max<long long>(SLICE_MIN, (sl + SLICE_MIN - 1) / SLICE_MIN * SLICE_MIN);
  sl = std::min<long long>(sl, 1LL << 30);
  p->slice[L.slot] = (int)sl;
  const long long est = std::min<long long>(nbra + (cand + sl - 1) / sl, 1LL << 30);
  p->units_est[L.slot] = (int)est;
  *units_need = std::max(*units_need, est + 1);
}

// outputs of a build: bit 0 J, bit 1 K
int plan_want(const jk_plan *p) {
  return (p->flags & JK_FLAG_J_ONLY) ? 1 : (p->flags & JK_FLAG_K_ONLY) ? 2 : 3;
}

ScreenArgs screen_args(const jk_plan *p) {
  ScreenArgs A{};
  A.pairI = p->d_pairI;
  A.pair_cls = p->d_pair_cls;
  A.pair_sa = p->d_pair_sa;
  A.pair_sb = p->d_pair_sb;
  A.pair_npp = p->d_pair_npp;
  A.pair_mol = p->d_pair_mol;
  A.bin_beg = p->d_bin_beg;
  A.cm_bin = p->d_cm_bin;
  A.Pblk = p->d_Pblk;
  A.pairP = p->d_pairP;
  A.ps_off = p->d_ps_off;
  A.sbase = p->d_sbase;
  A.gmax = p->d_gmax;
  A.gfix = 0.0;
  A.gscale = 1.0;
  A.cap = p->d_cap;
  A.segoff = p->d_segoff;
  A.segcnt = p->d_segcnt;
  A.segoff32 = p->d_segoff32;
  A.segcnt32 = p->d_segcnt32;
  A.count = p->d_count;
  A.count32 = p->d_count32;
  A.fp32_cut = p->precision == JK_MIXED ? p->fp32_cutoff : 0.0;
  A.f32_classes[0] = A.f32_classes[1] = 0ull;
  for (int qc = 0; qc < NQCLASS; ++qc)   // FP32 bodies exist for the lane-per-quartet classes
    if (!g_classes[qc].team) A.f32_classes[qc >> 6] |= 1ull << (qc & 63);
  A.nprim = p->d_nprim;
  A.class_off = p->d_class_off;
  A.room = p->d_room;
  A.kets = p->d_kets;
  A.tau = p->tau;
  A.npairs = p->npairs;
  A.nmol = p->nmol;
  A.want = plan_want(p);
  return A;
}

// Team scratch for the launches of a build at the current workgroup counts.
int ensure_launch_scratch(jk_plan *p) {
  std::vector<Launch> launches;
  plan_launches(p, p->active, launches);
  long long need = 0;
  for (const Launch &L : launches) need = std::max(need, L.scratch_per_wg * (long long)launch_grid(p, L));
  return need > 0 ? ensure_scratch(p, need) : JK_OK;
}

// Work-list layout. Counts, for every class, the candidate quartets under a density bound
// (gfix, or gscale times the largest |D_cart| of the density already on the device), lays the
// class regions out one after another, and sizes the work-unit list and the team scratch of
// the launches. Regions only grow. Waits for the stream: this runs at plan creation (with a
// caller's bound), on a plan's first execute, and when a check finds an overflow.
int size_lists(jk_plan *p, hipStream_t st, double gfix, double gscale) {
  unsigned long long cap[NQCLASS] = {};
  if (p->npairs > 0) {
    HIPCHK(launch_fill_u64(p->d_cap, NQCLASS, 0ull, st));
    ScreenArgs A = screen_args(p);
    A.gfix = gfix;
    A.gscale = gscale;
    HIPCHK(launch_capacity(A, st));
    HIPCHK(hipMemcpyAsync(cap, p->d_cap, sizeof(cap), hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  bool grew = !p->sized;
  for (int c = 0; c < NQCLASS; ++c) {
    if (cap[c] > 0x7fffffffULL) return fail(JK_EUNSUPPORTED, "class %d: %llu candidate quartets exceed 2^31", c, cap[c]);
    if ((long long)cap[c] > p->capc[c]) {
      p->capc[c] = (long long)cap[c];
      grew = true;
    }
  }
  if (grew) {
    long long total = 0;
    for (int c = 0; c < NQCLASS; ++c) {
      p->class_off_h[c] = total;
      total += p->capc[c];
      p->active[c] = p->capc[c] > 0;
    }
    dfree(p->d_kets);
    p->list_capacity = 0;
    int rc = dalloc(&p->d_kets, (size_t)total + 1);
    if (rc) return rc;
    p->list_capacity = total;
    HIPCHK(hipMemcpy(p->d_class_off, p->class_off_h.data(), sizeof(long long) * NQCLASS, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(p->d_capc, p->capc.data(), sizeof(long long) * NQCLASS, hipMemcpyHostToDevice));
    p->graph_stale = true;
  }
  std::vector<Launch> launches;
  plan_launches(p, p->active, launches);
  long long units_need = 1;
  for (const Launch &L : launches) {
    long long cand = 0;
    for (int ck = 0; ck <= L.cb; ++ck)
      if ((L.mask >> ck) & 1) cand += p->capc[qclass_index(L.cb, ck)];
    size_units(p, L, cand, &units_need);
  }
  if (units_need > 0x7fffffffLL) return fail(JK_EUNSUPPORTED, "%lld work units exceed 2^31", units_need);
  if (units_need > p->units_cap) {
    dfree(p->d_units);
    p->units_cap = 0;
    int rc = dalloc(&p->d_units, (size_t)units_need);
    if (rc) return rc;
    p->units_cap = (int)units_need;
    p->graph_stale = true;
  }
  p->sized = true;
  return ensure_launch_scratch(p);
}

// Enqueue one build on `st`: density transform and block maxima, the screen into the class
// regions, every integral launch, fold and finalisation. Nothing here waits for the device or
// allocates, so the same sequence is recorded into a graph (record = true: no profile events).
// A class whose kept candidates exceed its region raises the device overflow flag.
int enqueue_build(jk_plan *p, const double *D, double *J, double *K, hipStream_t st, bool record) {
  const size_t nc2 = (size_t)p->mc_off[p->nmol];
  const bool prof = !record && !p->events.empty();
  if (!record) p->launched.clear();
  hipEvent_t *ev = prof ? p->events.data() + (size_t)p->ev_next * EV_PER_SET : nullptr;
  if (prof) HIPCHK(hipEventRecord(ev[2 * NSLOT], st));
  HIPCHK(launch_fill_u64((unsigned long long *)p->d_Jc, (long long)nc2, 0ull, st));
  HIPCHK(launch_fill_u64((unsigned long long *)p->d_Kc, (long long)nc2, 0ull, st));
  HIPCHK(launch_fill_u64((unsigned long long *)p->d_Jpair, p->jp_total, 0ull, st));
  HIPCHK(launch_fill_u64((unsigned long long *)p->d_gmax, 1, 0ull, st));
  HIPCHK(launch_fill_u64(p->d_cap, NQCLASS, 0ull, st));
  HIPCHK(launch_fill_u64(p->d_nprim, 2 * NQCLASS, 0ull, st));
  HIPCHK(launch_fill_i32(p->d_count, NQCLASS, 0, st));
  HIPCHK(launch_fill_i32(p->d_count32, NQCLASS, 0, st));
  HIPCHK(launch_fill_i32(p->d_next, NSLOT, 0, st));
  HIPCHK(launch_fill_i32(p->d_nunits, NSLOT, 0, st));
  HIPCHK(launch_fill_i32(p->d_overflow, 1, 0, st));
  HIPCHK(launch_dcart(p->S, D, p->d_Dc, p->d_Dp, st));
  HIPCHK(launch_blockmax(p->S, p->d_Dc, p->d_Pblk, p->d_gmax, st));
  FoldArgs F{};
  F.pair_cls = p->d_pair_cls;
  F.pair_ca = p->d_pair_ca;
  F.pair_cb = p->d_pair_cb;
  F.pair_la = p->d_pair_la;
  F.pair_lb = p->d_pair_lb;
  F.pair_mol = p->d_pair_mol;
  F.cls_beg = p->d_cls_beg;
  F.jp_off = p->d_jp_off;
  F.mc_off = p->d_mc_off;
  F.cbase = p->d_cbase;
  F.Jpair = p->d_Jpair;
  F.Jc = p->d_Jc;
  F.npairs = p->npairs;
  F.Dc = p->d_Dc;
  F.Dpair = p->d_Dpair;
  if (p->npairs > 0) HIPCHK(launch_unfold(F, st));
  ScreenArgs A = screen_args(p);
  if (p->npairs > 0) {
    HIPCHK(launch_capacity(A, st));
    HIPCHK(launch_class_room(p->d_cap, p->d_capc, p->d_room, p->d_overflow, st));
    HIPCHK(launch_pairp(A, st));
    HIPCHK(launch_screen(A, st));
  }
  if (prof) HIPCHK(hipEventRecord(ev[2 * NSLOT + 1], st));

  std::vector<Launch> launches;
  plan_launches(p, p->active, launches);
  JKArgs J_{};
  J_.pairs = p->d_pairs;
  J_.pp = p->d_pp;
  J_.kets = p->d_kets;
  J_.class_off = p->d_class_off;
  J_.segoff = p->d_segoff;
  J_.segcnt = p->d_segcnt;
  J_.segoff32 = p->d_segoff32;
  J_.segcnt32 = p->d_segcnt32;
  J_.Dp = p->d_Dp;
  J_.Kc = p->d_Kc;
  J_.mbase = p->d_mc_off;
  J_.mnc = p->d_mnc;
  J_.Jpair = p->d_Jpair;
  J_.Dpair = p->d_Dpair;
  J_.jp_off = p->d_jp_off;
  J_.cls_beg = p->d_cls_beg;
  J_.scratch = p->d_scratch;
  J_.want = plan_want(p);
  J_.lcol = p->d_lcol;
  J_.lcols = p->d_lcols;
  J_.lseg = p->d_lseg;
  J_.cbase = p->d_cbase;
  for (const Launch &L : launches) {
    const int grid = launch_grid(p, L);
    if (L.scratch_per_wg * (long long)grid > p->scratch_doubles)
      return fail(JK_EDEVICE, "internal: team scratch not sized for launch slot %d", L.slot);
    J_.bra_beg = L.bra_beg;
    J_.bra_end = L.bra_end;
    J_.nc_max = L.nc_max;
    J_.slice = p->slice[L.slot] > 0 ? p->slice[L.slot] : (1 << 30);
    J_.units = p->d_units;
    J_.units_cap = p->units_cap;
    J_.nunits = p->d_nunits + L.slot;
    J_.parts = L.parts;
    HIPCHK(launch_units(p->d_segcnt, p->d_segcnt32, L.bra_beg, L.bra_end, L.mask, L.parts, J_.slice, p->d_units,
                        p->units_cap, p->d_nunits + L.slot, p->d_overflow, st));
    J_.scratch_per_wg = L.scratch_per_wg;
    J_.next = p->d_next + L.slot;
    if (prof) HIPCHK(hipEventRecord(ev[2 * L.slot], st));
    J_.kw = L.kw;
    J_.kwb = L.kwb;
    if (L.qc < 0)
      HIPCHK((L.f32 ? g_bras[L.cb].launch_bra32[L.tier] : g_bras[L.cb].launch_bra[L.tier])(J_, grid, L.lds, st));
    else if (L.kw > 0)
      HIPCHK((L.krows == 1 ? (L.gl ? g_classes[L.qc].launch_clslg : g_classes[L.qc].launch_clsl)
                           : (L.gl ? g_classes[L.qc].launch_clsag : g_classes[L.qc].launch_clsa))(J_, grid, L.lds, st));
    else
      HIPCHK(g_classes[L.qc].launch_cls(J_, grid, L.lds, st));
    if (prof) HIPCHK(hipEventRecord(ev[2 * L.slot + 1], st));
    if (!record) p->launched.push_back(L.slot);
  }
  if (prof) HIPCHK(hipEventRecord(ev[2 * NSLOT + 2], st));
  if (p->npairs > 0 && (J_.want & 1)) HIPCHK(launch_fold(F, st));
  HIPCHK(launch_finalize(p->S, p->d_Jc, p->d_Kc, (J_.want & 1) ? J : nullptr, (J_.want & 2) ? K : nullptr, st));
  if (prof) {
    HIPCHK(hipEventRecord(ev[2 * NSLOT + 3], st));
    // the ring averages builds of one launch set: a build with other launches starts it anew
    if (p->launched != p->ev_launched) {
      p->ev_count = 0;
      p->ev_launched = p->launched;
    }
    p->ev_next = (p->ev_next + 1) % EV_SETS;
    p->ev_count = std::min(p->ev_count + 1, EV_SETS);
  }
  return JK_OK;
}

// Record the build into a HIP graph (on the plan's own stream: the caller's may be the
// legacy default stream, which cannot be recorded). Every buffer already has its size, so
// recording neither allocates nor waits.
int record_graph(jk_plan *p, const double *D, double *J, double *K) {
  graph_free(p);
  HIPCHK(hipStreamBeginCapture(p->rec_stream, hipStreamCaptureModeThreadLocal));
  int rc = enqueue_build(p, D, J, K, p->rec_stream, true);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(p->rec_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(JK_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  p->graph = g;
  const hipError_t e2 = hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    p->gexec = nullptr;
    graph_free(p);
    return fail(JK_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e2));
  }
  p->gD = D;
  p->gJ = J;
  p->gK = K;
  p->graph_stale = false;
  return JK_OK;
}

// ------------------------------------------------------------------ grid tuner
std::string slot_name(int slot) {
  char buf[64];
  if (slot < NFUSED) {
    const BraInfo &bi = g_bras[slot / NTIERS];
    snprintf(buf, sizeof(buf), "k_bra<%d,%d,%d>", bi.la, bi.lb, slot % NTIERS);
  } else if (slot >= NF32_BASE) {
    const BraInfo &bi = g_bras[(slot - NF32_BASE) / NTIERS];
    snprintf(buf, sizeof(buf), "k_bra32<%d,%d,%d>", bi.la, bi.lb, (slot - NF32_BASE) % NTIERS);
  } else {
    const ClassInfo &ci = g_classes[slot - NFUSED];
    snprintf(buf, sizeof(buf), "k_cls<%d,%d,%d,%d>", ci.la, ci.lb, ci.lc, ci.ld);
  }
  return buf;
}

bool load_tune_cache(jk_plan *p) {
  if (p->tune_cache.empty()) return false;
  FILE *f = fopen(p->tune_cache.c_str(), "r");
  if (!f) return false;
  char name[64];
  int g = 0, n = 0;
  while (fscanf(f, "%63s %d", name, &g) == 2) {
    const std::string nm = name;
    if (nm.rfind("fuse:", 0) == 0) {         // fuse:k_bra<la,lb,tier> 0|1
      for (int s = 0; s < NFUSED; ++s)
        if ("fuse:" + slot_name(s) == nm) p->fuse[s] = g != 0;
      continue;
    }
    if (nm.rfind("shape:", 0) == 0) {        // shape:k_cls<la,lb,lc,ld> SHAPE_* bits
      for (int qc = 0; qc < NQCLASS; ++qc)
        if ("shape:" + slot_name(NFUSED + qc) == nm && g >= 0 && g < 4) p->shape[qc] = (char)g;
      continue;
    }
    for (int s = 0; s < NSLOT; ++s)
      if (slot_name(s) == nm && g > 0 && g <= 65536) {
        p->grid[s] = g;
        ++n;
      }
  }
  fclose(f);
  return n > 0;
}

void save_tune_cache(const jk_plan *p) {
  if (p->tune_cache.empty()) return;
  FILE *f = fopen(p->tune_cache.c_str(), "w");
  if (!f) return;
  for (int s = 0; s < NSLOT; ++s)
    if (p->grid[s] > 0) fprintf(f, "%s %d\n", slot_name(s).c_str(), p->grid[s]);
  for (int s = 0; s < NFUSED; ++s)
    if (s % NTIERS != TEAM_TIER && g_bras[s / NTIERS].fusable[s % NTIERS])
      fprintf(f, "fuse:%s %d\n", slot_name(s).c_str(), (int)p->fuse[s]);
  for (int qc = 0; qc < NQCLASS; ++qc)
    if (p->shape[qc]) fprintf(f, "shape:%s %d\n", slot_name(NFUSED + qc).c_str(), (int)p->shape[qc]);
  fclose(f);
}

// Work units and team scratch for the current launch set (after the tuner changed it).
int resize_units(jk_plan *p) {
  std::vector<Launch> launches;
  plan_launches(p, p->active, launches);
  long long units_need = 1;
  for (const Launch &L : launches) {
    long long cand = 0;
    for (int ck = 0; ck <= L.cb; ++ck)
      if ((L.mask >> ck) & 1) cand += p->capc[qclass_index(L.cb, ck)];
    size_units(p, L, cand, &units_need);
  }
  if (units_need > 0x7fffffffLL) return fail(JK_EUNSUPPORTED, "%lld work units exceed 2^31", units_need);
  if (units_need > p->units_cap) {
    dfree(p->d_units);
    p->units_cap = 0;
    int rc = dalloc(&p->d_units, (size_t)units_need);
    if (rc) return rc;
    p->units_cap = (int)units_need;
  }
  p->graph_stale = true;
  return ensure_launch_scratch(p);
}

// Times every launch slot at each candidate workgroup count (one full build per candidate, per-launch
// HIP events): best[slot] and pick[slot].
int time_grids(jk_plan *p, const double *D, double *J, double *K, hipStream_t st, std::vector<float> &best,
               std::vector<int> &pick) {
  best.assign(NSLOT, 1e30f);
  pick.assign(NSLOT, 0);
  for (int g : TUNE_GRIDS) {
    std::fill(p->grid.begin(), p->grid.end(), g);
    int rc = resize_units(p);
    const hipEvent_t *ev = p->events.data() + (size_t)p->ev_next * EV_PER_SET;   // the set this build records
    if (!rc) rc = enqueue_build(p, D, J, K, st, false);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(st));
    for (int slot : p->launched) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev[2 * slot], ev[2 * slot + 1]));
      if (ms < best[slot]) {
        best[slot] = ms;
        pick[slot] = g;
      }
    }
  }
  return JK_OK;
}

// The tuner: for every register tier of lane bodies, whether its ket classes run fused (one
// launch per bra class, full exchange rows in LDS) or per class (compacted rows), for every
// per-class launch its shape (SHAPE_*), and for every launch the workgroup count. Every layout
// and shape is timed at every candidate count; a tier keeps the layout whose launches (fused
// launch and the per-class launches of molecules too large for it, against the per-class
// launches alone) take less time, and each class its fastest shape and count.
int tune_grids(jk_plan *p, const double *D, double *J, double *K, hipStream_t st) {
  std::vector<float> bestF, bestC;
  std::vector<int> pickF, pickC;
  for (int f = 0; f < NFUSED; ++f)
    if (f % NTIERS != TEAM_TIER) p->fuse[f] = 1;
  int rc = time_grids(p, D, J, K, st, bestF, pickF);
  if (rc) return rc;
  for (int f = 0; f < NFUSED; ++f)
    if (f % NTIERS != TEAM_TIER) p->fuse[f] = 0;
  // per-class layout: every launch shape at every count; each class keeps its fastest pair
  std::vector<char> bestShape(NQCLASS, 0);
  for (int sh = 0; sh < NSHAPE; ++sh) {
    std::fill(p->shape.begin(), p->shape.end(), (char)sh);
    std::vector<float> b;
    std::vector<int> pk;
    if ((rc = time_grids(p, D, J, K, st, b, pk))) return rc;
    if (sh == 0) {
      bestC = b;
      pickC = pk;
      continue;
    }
    for (int qc = 0; qc < NQCLASS; ++qc) {
      const int slot = NFUSED + qc;
      if (b[slot] < bestC[slot]) {
        bestC[slot] = b[slot];
        pickC[slot] = pk[slot];
        bestShape[qc] = (char)sh;
      }
    }
  }
  p->shape = bestShape;
  auto t = [](const std::vector<float> &b, int slot) { return b[slot] < 1e29f ? (double)b[slot] : 0.0; };
  std::vector<int> pick = pickC;
  for (int cb = 0; cb < NPAIRCLASS; ++cb)
    for (int tier = 0; tier < TEAM_TIER; ++tier) {
      const BraInfo &bi = g_bras[cb];
      const int f = cb * NTIERS + tier;
      if (!bi.fusable[tier]) continue;
      double costF = t(bestF, f) + t(bestF, NF32_BASE + f), costC = 0.0;
      for (int ck = 0; ck <= cb; ++ck)
        if ((bi.tier_mask[tier] >> ck) & 1) {
          costF += t(bestF, NFUSED + qclass_index(cb, ck));
          costC += t(bestC, NFUSED + qclass_index(cb, ck));
        }
      p->fuse[f] = costF < costC;
      if (p->fuse[f]) {
        pick[f] = pickF[f];
        pick[NF32_BASE + f] = pickF[NF32_BASE + f];
        for (int ck = 0; ck <= cb; ++ck)
          if ((bi.tier_mask[tier] >> ck) & 1) pick[NFUSED + qclass_index(cb, ck)] = pickF[NFUSED + qclass_index(cb, ck)];
      }
    }
  for (int f = 0; f < NFUSED; ++f)   // team tiers: timed in both passes, same layout
    if (f % NTIERS == TEAM_TIER) pick[f] = bestF[f] <= bestC[f] ? pickF[f] : pickC[f];
  p->grid = pick;
  save_tune_cache(p);
  p->ev_count = 0;            // the timing builds are not profiled builds
  return resize_units(p);
}

constexpr double SIZE_HEADROOM = 2.0;   // first-execute sizing: lists hold densities up to twice its largest element

int plan_run(jk_plan *p, const double *D, double *J, double *K, hipStream_t st) {
  const int want = plan_want(p);
  if (!D || (!J && (want & 1)) || (!K && (want & 2)))
    return fail(JK_EINVAL, "D and the requested outputs (J, K) must be device pointers");
  p->last_stream = st;
  if (!p->sized) {
    // the first execute sizes the lists from its own density: transform, block maxima, then
    // the candidate counts under twice its largest element (one wait for the device)
    HIPCHK(launch_fill_u64((unsigned long long *)p->d_gmax, 1, 0ull, st));
    HIPCHK(launch_dcart(p->S, D, p->d_Dc, p->d_Dp, st));
    HIPCHK(launch_blockmax(p->S, p->d_Dc, p->d_Pblk, p->d_gmax, st));
    int rc = size_lists(p, st, 0.0, SIZE_HEADROOM);
    if (rc) return rc;
  }
  if ((p->flags & JK_FLAG_TUNE) && !p->tuned) {
    int rc = load_tune_cache(p) ? resize_units(p) : tune_grids(p, D, J, K, st);
    if (rc) return rc;
    p->tuned = true;
    p->graph_stale = true;
  }
  if (!(p->flags & JK_FLAG_GRAPH)) return enqueue_build(p, D, J, K, st, false);
  if (p->gexec && !p->graph_stale && D == p->gD && J == p->gJ && K == p->gK) {
    ++p->replays;
  } else {
    if (p->gexec) ++p->rerecords;
    int rc = record_graph(p, D, J, K);
    if (rc) return rc;
  }
  p->launched.clear();
  HIPCHK(hipGraphLaunch(p->gexec, st));
  return JK_OK;
}

// Waits for the plan's last build and reports whether its work lists overflowed. On overflow
// the lists grow (sized for twice the largest density element of that build) and the caller
// runs the build again.
int plan_check(jk_plan *p) {
  HIPCHK(hipStreamSynchronize(p->last_stream));
  int ov = 0;
  HIPCHK(hipMemcpy(&ov, p->d_overflow, sizeof(int), hipMemcpyDeviceToHost));
  if (!ov) return JK_OK;
  ++p->overflows;
  int rc = size_lists(p, p->last_stream, 0.0, SIZE_HEADROOM);
  if (rc) return rc;
  HIPCHK(hipMemset(p->d_overflow, 0, sizeof(int)));
  return fail(JK_EOVERFLOW, "the last build needed longer work lists than the plan held, so its J and K are "
              "incomplete; the lists have grown and a new execute completes");
}

// ------------------------------------------------------------------ nuclear gradient
// The screen of the J/K build (six density blocks), then one k_grad launch per quartet class
// over the kept quartets of its work list. grad (natom x 3) is overwritten.
int plan_grad(jk_plan *p, const double *D, double *grad, hipStream_t st) {
  if (!D || !grad) return fail(JK_EINVAL, "D and grad must be device pointers");
  if (p->nmol != 1) return fail(JK_EUNSUPPORTED, "the gradient is built for single-molecule plans");
  if (p->lmax > GRAD_LMAX) return fail(JK_EUNSUPPORTED, "gradient kernels exist for shells up to l = %d (plan has %d)",
                                       GRAD_LMAX, p->lmax);
  if (plan_want(p) != 3) return fail(JK_EINVAL, "the gradient needs a plan made for J and K (no J-only/K-only flag)");
  p->last_stream = st;
  if (!p->sized) {
    HIPCHK(launch_fill_u64((unsigned long long *)p->d_gmax, 1, 0ull, st));
    HIPCHK(launch_dcart(p->S, D, p->d_Dc, p->d_Dp, st));
    HIPCHK(launch_blockmax(p->S, p->d_Dc, p->d_Pblk, p->d_gmax, st));
    int rc = size_lists(p, st, 0.0, SIZE_HEADROOM);
    if (rc) return rc;
  }
  // work units of each class launch: slices sized from the class capacity as for the J/K launches
  std::vector<int> gslice(NQCLASS, 0), gest(NQCLASS, 0);
  long long need = 1;
  for (int qc = 0; qc < NQCLASS; ++qc) {
    if (!p->active[qc] || !g_grad[qc]) continue;
    const int cb = (int)((std::sqrt(8.0 * qc + 1) - 1) / 2);
    const long long nbra = p->cls_beg[cb + 1] - p->cls_beg[cb];
    long long sl = (p->capc[qc] + TARGET_UNITS - 1) / TARGET_UNITS;
    sl = std::max<long long>(SLICE_MIN, (sl + SLICE_MIN - 1) / SLICE_MIN * SLICE_MIN);
    gslice[qc] = (int)std::min<long long>(sl, 1LL << 30);
    gest[qc] = (int)std::min<long long>(nbra + (p->capc[qc] + sl - 1) / sl, 1LL << 30);
    need = std::max(need, (long long)gest[qc] + 1);
  }
  if (need > p->units_cap) {
    HIPCHK(hipStreamSynchronize(st));
    dfree(p->d_units);
    p->units_cap = 0;
    int rc = dalloc(&p->d_units, (size_t)need);
    if (rc) return rc;
    p->units_cap = (int)need;
    p->graph_stale = true;
  }
  HIPCHK(launch_fill_u64((unsigned long long *)grad, 3LL * p->natom, 0ull, st));
  HIPCHK(launch_fill_u64((unsigned long long *)p->d_gmax, 1, 0ull, st));
  HIPCHK(launch_fill_u64(p->d_cap, NQCLASS, 0ull, st));
  HIPCHK(launch_fill_u64(p->d_nprim, 2 * NQCLASS, 0ull, st));
  HIPCHK(launch_fill_i32(p->d_count, NQCLASS, 0, st));
  HIPCHK(launch_fill_i32(p->d_count32, NQCLASS, 0, st));
  HIPCHK(launch_fill_i32(p->d_next, NSLOT, 0, st));
  HIPCHK(launch_fill_i32(p->d_nunits, NSLOT, 0, st));
  HIPCHK(launch_fill_i32(p->d_overflow, 1, 0, st));
  HIPCHK(launch_dcart(p->S, D, p->d_Dc, p->d_Dp, st));
  HIPCHK(launch_blockmax(p->S, p->d_Dc, p->d_Pblk, p->d_gmax, st));
  ScreenArgs A = screen_args(p);
  A.fp32_cut = 0.0;                       // every kept quartet in the FP64 part of its segment
  if (p->npairs > 0) {
    HIPCHK(launch_capacity(A, st));
    HIPCHK(launch_class_room(p->d_cap, p->d_capc, p->d_room, p->d_overflow, st));
    HIPCHK(launch_pairp(A, st));
    HIPCHK(launch_screen(A, st));
  }
  GradArgs G{};
  G.pairs = p->d_pairs;
  G.pp = p->d_pp;
  G.ppab = p->d_ppab;
  G.kets = p->d_kets;
  G.class_off = p->d_class_off;
  G.segoff = p->d_segoff;
  G.segcnt = p->d_segcnt;
  G.Dc = p->d_Dc;
  G.nc = p->nc;
  G.shell_atom = p->d_shell_atom;
  G.grad = grad;
  G.units = p->d_units;
  G.units_cap = p->units_cap;
  for (int qc = 0; qc < NQCLASS; ++qc) {
    if (!p->active[qc] || !g_grad[qc]) continue;
    const int cb = (int)((std::sqrt(8.0 * qc + 1) - 1) / 2), ck = qc - cb * (cb + 1) / 2;
    const int slot = NFUSED + qc;
    G.slice = gslice[qc];
    G.nunits = p->d_nunits + slot;
    G.next = p->d_next + slot;
    HIPCHK(launch_units(p->d_segcnt, nullptr, p->cls_beg[cb], p->cls_beg[cb + 1], 1 << ck, 1, G.slice, p->d_units,
                        p->units_cap, p->d_nunits + slot, p->d_overflow, st));
    HIPCHK(g_grad[qc](G, std::max(1, std::min(gest[qc], GRID_TEAM_MAX)), st));
  }
  return JK_OK;
}

int plan_stats(const jk_plan *plan, jk_stats_t *out) {
  *out = plan->stats;
  if (plan->d_count) {
    int cnt[NQCLASS], c32[NQCLASS], ov = 0;
    unsigned long long np[NQCLASS], cap[NQCLASS];
    HIPCHK(hipStreamSynchronize(plan->last_stream));
    HIPCHK(hipMemcpy(cnt, plan->d_count, sizeof(cnt), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(c32, plan->d_count32, sizeof(c32), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(np, plan->d_nprim, sizeof(np), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(cap, plan->d_cap, sizeof(cap), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&ov, plan->d_overflow, sizeof(int), hipMemcpyDeviceToHost));
    out->kept_quartets = 0;
    out->kept_fp32 = 0;
    out->prim_quartets = 0;
    out->candidate_quartets = 0;
    for (int c = 0; c < NQCLASS; ++c) {
      out->kept_quartets += cnt[c];
      out->kept_fp32 += c32[c];
      out->prim_quartets += (long long)np[c];
      out->candidate_quartets += (long long)cap[c];
    }
    out->overflow = ov;
    out->list_capacity = plan->list_capacity;
  }
  return JK_OK;
}

}  // namespace

namespace jk {
void solid_harmonics_host(int l, double *T) { solid_harmonics(l, T); }
int set_error(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
}  // namespace jk

namespace {

// host copy of the Boys grid for the test hook below
namespace host_boys {
#define BOYS_STORAGE static const
#include "boys_grid.h"
#undef BOYS_STORAGE
}  // namespace host_boys

}  // namespace

extern "C" {

const char *jk_last_error(void) { return g_err.c_str(); }

int jk_rys_grid(int nroots, double T, double *u, double *w) {
  if (!u || !w) return fail(JK_EINVAL, "NULL argument");
  if (nroots != 1 && nroots != 2) return fail(JK_EINVAL, "the grid rule exists for 1 or 2 roots only");
  if (!(T >= 0.0) || !(T < (double)RYS_TMAX[nroots]))
    return fail(JK_EINVAL, "T must be in [0, %d) for %d roots", RYS_TMAX[nroots], nroots);
  if (nroots == 1) {
    double uu[1], ww[1];
    rys_taylor<1>(T, host_boys::BOYS_GRID, uu, ww);
    u[0] = uu[0]; w[0] = ww[0];
  } else {
    double uu[2], ww[2];
    rys_taylor<2>(T, host_boys::BOYS_GRID, uu, ww);
    u[0] = uu[0]; u[1] = uu[1]; w[0] = ww[0]; w[1] = ww[1];
  }
  return JK_OK;
}

int jk_rys_closed(int nroots, double T, double *u, double *w) {
  if (!u || !w) return fail(JK_EINVAL, "NULL argument");
  if (!(T >= 0.0) || !std::isfinite(T)) return fail(JK_EINVAL, "T must be finite and >= 0");
  if (nroots == 1) {
    double uu[1], ww[1];
    rys_closed<1>(T, uu, ww);
    u[0] = uu[0]; w[0] = ww[0];
  } else if (nroots == 2) {
    double uu[2], ww[2];
    rys_closed<2>(T, uu, ww);
    u[0] = uu[0]; u[1] = uu[1]; w[0] = ww[0]; w[1] = ww[1];
  } else {
    return fail(JK_EINVAL, "closed-form roots exist for 1 or 2 roots only");
  }
  return JK_OK;
}

int jk_sph_matrix(int l, double *out) {
  if (!out) return fail(JK_EINVAL, "out is NULL");
  if (l < 2 || l > LMAX) return fail(JK_EINVAL, "l must be in 2..4 (got %d)", l);
  solid_harmonics(l, out);
  return JK_OK;
}

int jk_plan_sizes(const jk_plan_t *plan, int *nao, int *nao_cart) {
  if (!plan) return fail(JK_EINVAL, "plan is NULL");
  if (nao) *nao = plan->nao;
  if (nao_cart) *nao_cart = plan->nc;
  return JK_OK;
}

int jk_stats(const jk_plan_t *plan, jk_stats_t *out) {
  if (!plan || !out) return fail(JK_EINVAL, "NULL argument");
  return plan_stats(plan, out);
}

int jk_profile(jk_plan_t *p, jk_profile_t *out, int max_entries, int *n_entries) {
  if (!p || !out || !n_entries) return fail(JK_EINVAL, "NULL argument");
  if (!(p->flags & JK_FLAG_PROFILE)) return fail(JK_EINVAL, "plan was not created with JK_FLAG_PROFILE");
  if (p->launched.empty() || p->ev_count == 0)
    return fail(JK_EINVAL, "no profiled build since the last profile (graph launches are not profiled)");
  HIPCHK(hipStreamSynchronize(p->last_stream));
  // mean HIP-event time of events (i0, i1) over the executes recorded since the last call
  const int nsets = p->ev_count;
  auto mean_ms = [&](int i0, int i1, double *out_ms) -> int {
    double sum = 0.0;
    for (int k = 1; k <= nsets; ++k) {
      const hipEvent_t *ev = p->events.data() + (size_t)((p->ev_next - k + EV_SETS) % EV_SETS) * EV_PER_SET;
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev[i0], ev[i1]));
      sum += ms;
    }
    *out_ms = sum / nsets;
    return JK_OK;
  };
  int cnt[NQCLASS], c32[NQCLASS];
  unsigned long long np[2 * NQCLASS];
  HIPCHK(hipMemcpy(cnt, p->d_count, sizeof(cnt), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(c32, p->d_count32, sizeof(c32), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(np, p->d_nprim, sizeof(np), hipMemcpyDeviceToHost));
  int n = 0;
  auto push = [&](const jk_profile_t &e) {
    if (n < max_entries) out[n] = e;
    ++n;
  };
  // parts: 3 every kept quartet of the class, 1 its FP64 ones, 2 its FP32 ones
  auto class_flops = [&](int qc, jk_profile_t &r, int parts) {
    const ClassInfo &ci = g_classes[qc];
    double fp = 0.0, fq = 0.0;
    class_ops(ci.la, ci.lb, ci.lc, ci.ld, plan_want(p), &fp, &fq);
    const double q = parts == 3 ? cnt[qc] : parts == 2 ? c32[qc] : cnt[qc] - c32[qc];
    const double pq = parts == 3 ? (double)np[qc] : parts == 2 ? (double)np[NQCLASS + qc]
                                                               : (double)(np[qc] - np[NQCLASS + qc]);
    r.quartets += (long long)q;
    r.prim_quartets += (long long)pq;
    r.flops += pq * fp + q * fq;
  };
  int rc;
  jk_profile_t e{};
  e.kind = 1;
  if ((rc = mean_ms(2 * NSLOT, 2 * NSLOT + 1, &e.ms))) return rc;
  push(e);
  for (int slot : p->launched) {
    jk_profile_t r{};
    r.kind = 0;
    if (slot < NFUSED || slot >= NF32_BASE) {     // fused launch of one tier of a bra class
      const bool f32 = slot >= NF32_BASE;
      const int fs = f32 ? slot - NF32_BASE : slot;
      const int cb = fs / NTIERS, tier = fs % NTIERS;
      const BraInfo &bi = g_bras[cb];
      r.la = bi.la; r.lb = bi.lb; r.lc = -1; r.ld = tier;
      r.team = f32 ? 3 : 2;
      const int parts = f32 ? 2 : (p->precision == JK_MIXED && bi.launch_bra32[tier]) ? 1 : 3;
      for (int ck = 0; ck <= cb; ++ck)
        if ((bi.tier_mask[tier] >> ck) & 1) class_flops(qclass_index(cb, ck), r, parts);
    } else {
      const ClassInfo &ci = g_classes[slot - NFUSED];
      r.la = ci.la; r.lb = ci.lb; r.lc = ci.lc; r.ld = ci.ld;
      r.team = ci.team;
      r.nroots = (ci.la + ci.lb + ci.lc + ci.ld) / 2 + 1;
      class_flops(slot - NFUSED, r, 3);
    }
    if ((rc = mean_ms(2 * slot, 2 * slot + 1, &r.ms))) return rc;
    push(r);
  }
  e = jk_profile_t{};
  e.kind = 2;
  if ((rc = mean_ms(2 * NSLOT + 2, 2 * NSLOT + 3, &e.ms))) return rc;
  push(e);
  p->ev_count = 0;
  *n_entries = n;
  return JK_OK;
}

int jk_schwarz(const jk_plan_t *plan, double *out) {
  if (!plan || !out) return fail(JK_EINVAL, "NULL argument");
  std::memcpy(out, plan->schwarz.data(), sizeof(double) * plan->schwarz.size());
  return JK_OK;
}

void jk_plan_destroy(jk_plan_t *plan) {
  if (!plan) return;
  plan_free(plan);
  delete plan;
}

int jk_plan_create(const jk_basis_t *B, const double *coords, int natom, const jk_opts_t *opts, jk_plan_t **out) {
  if (!out) return fail(JK_EINVAL, "out is NULL");
  *out = nullptr;
  return plan_create(1, &B, &coords, &natom, opts, out);
}

int jk_plan_execute(jk_plan_t *p, const double *D, double *J, double *K, void *stream) {
  if (!p) return fail(JK_EINVAL, "plan is NULL");
  return plan_run(p, D, J, K, (hipStream_t)stream);
}

int jk_plan_check(jk_plan_t *p) {
  if (!p) return fail(JK_EINVAL, "plan is NULL");
  return plan_check(p);
}

int jk_grad(jk_plan_t *p, const double *D, double *grad, void *stream) {
  if (!p) return fail(JK_EINVAL, "plan is NULL");
  return plan_grad(p, D, grad, (hipStream_t)stream);
}

int jk_build(const jk_basis_t *basis, const double *coords, int natom, const double *D, double thresh, double *J,
             double *K, const jk_opts_t *opts, void *stream) {
  jk_opts_t o{};
  if (opts) o = *opts;
  o.thresh = thresh;
  jk_plan_t *p = nullptr;
  int rc = jk_plan_create(basis, coords, natom, &o, &p);
  if (rc) return rc;
  rc = jk_plan_execute(p, D, J, K, stream);
  if (!rc) rc = plan_check(p);
  if (rc == JK_EOVERFLOW) {     // the lists have grown: build again
    rc = jk_plan_execute(p, D, J, K, stream);
    if (!rc) rc = plan_check(p);
  }
  jk_plan_destroy(p);
  return rc;
}

}  // extern "C"

// ------------------------------------------------------------------ no-allocation entry point
namespace {
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)128 << 20;
constexpr int STATIC_MAX_DEVICES = 64;
// One copy per device, held until the process ends. In host code `scratch` only names the
// symbol: its device address comes from hipGetSymbolAddress (static_scratch_ptr).
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];
std::mutex g_static_mu;                          // calls on one device share its array
void *g_static_ptr[STATIC_MAX_DEVICES] = {};

int static_scratch_ptr(int dev, void **out) {
  if (dev < 0 || dev >= STATIC_MAX_DEVICES) return fail(JK_EUNSUPPORTED, "device %d beyond %d", dev, STATIC_MAX_DEVICES);
  if (!g_static_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail(JK_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_static_ptr[dev] = ptr;
  }
  *out = g_static_ptr[dev];
  return JK_OK;
}
}  // namespace

extern "C" {

int jk_build_static(const jk_basis_t *basis, const double *coords, int natom, const double *D, double thresh,
                    double *J, double *K, const jk_opts_t *opts, void *stream) {
  if (opts && (opts->flags & (JK_FLAG_PROFILE | JK_FLAG_GRAPH | JK_FLAG_TUNE)))
    return fail(JK_EINVAL, "jk_build_static: profile, graph and tune flags need allocations");
  if (g_arena) return fail(JK_EINVAL, "jk_build_static: not re-entrant");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_static_mu);
  void *base = nullptr;
  int rc = static_scratch_ptr(dev, &base);
  if (rc) return rc;
  Arena a{static_cast<char *>(base), STATIC_SCRATCH_BYTES, 0};
  g_arena = &a;
  rc = jk_build(basis, coords, natom, D, thresh, J, K, opts, stream);
  g_arena = nullptr;
  return rc;
}

int jk_eri_tensor(jk_plan_t *p, double *eri, void *stream) {
  if (!p || !eri) return fail(JK_EINVAL, "NULL argument");
  if (p->nmol != 1) return fail(JK_EINVAL, "the ERI tensor is defined for single-molecule plans");
  hipStream_t st = (hipStream_t)stream;
  // every (bra, ket) of kept pairs with bra class >= ket class (triangle inside a class)
  std::vector<int2> lst;
  std::vector<long long> off(NQCLASS + 1, 0);
  std::vector<int> cnt(NQCLASS, 0);
  for (int cb = 0; cb < NPAIRCLASS; ++cb)
    for (int ck = 0; ck <= cb; ++ck) {
      const int qc = qclass_index(cb, ck);
      off[qc] = (long long)lst.size();
      for (int i = p->cls_beg[cb]; i < p->cls_beg[cb + 1]; ++i)
        for (int k = p->cls_beg[ck]; k < p->cls_beg[ck + 1]; ++k) {
          if (ck == cb && k > i) break;
          lst.push_back(make_int2(i, k));
        }
      cnt[qc] = (int)((long long)lst.size() - off[qc]);
    }
  int2 *d_lst = nullptr;
  int rc;
  if ((rc = dupload(&d_lst, lst))) return rc;
  const size_t n4 = (size_t)p->nc * p->nc * p->nc * p->nc;
  hipError_t e = hipMemsetAsync(eri, 0, n4 * sizeof(double), st);
  if (e != hipSuccess) rc = fail(JK_EDEVICE, "hipMemsetAsync: %s", hipGetErrorString(e));
  for (int cb = 0; cb < NPAIRCLASS && !rc; ++cb)
    for (int ck = 0; ck <= cb && !rc; ++ck) {
      const int qc = qclass_index(cb, ck);
      if (!cnt[qc]) continue;
      rc = launch_mode_list(p, qc, MODE_ERI, d_lst + off[qc], cnt[qc], eri, st);
    }
  if (!rc) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = fail(JK_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
  }
  dfree(d_lst);
  return rc;
}

int jk_batch_create(int nmol, const jk_basis_t *const *basis, const double *const *coords, const int *natom,
                    const jk_opts_t *opts, jk_batch_t **out) {
  if (!out) return fail(JK_EINVAL, "out is NULL");
  *out = nullptr;
  jk_plan *p = nullptr;
  int rc = plan_create(nmol, basis, coords, natom, opts, &p);
  if (rc) return rc;
  jk_batch *b = new jk_batch();
  b->p = p;
  *out = b;
  return JK_OK;
}

int jk_batch_offsets(const jk_batch_t *b, long long *off, int *nao) {
  if (!b || !b->p) return fail(JK_EINVAL, "batch is NULL");
  const jk_plan *p = b->p;
  for (int m = 0; m <= p->nmol; ++m) {
    if (off) off[m] = p->user_off[m];
    if (nao && m < p->nmol) nao[m] = p->user_nao[m];
  }
  return JK_OK;
}

int jk_batch_execute(jk_batch_t *b, const double *D, double *J, double *K, void *stream) {
  if (!b || !b->p) return fail(JK_EINVAL, "batch is NULL");
  return plan_run(b->p, D, J, K, (hipStream_t)stream);
}

int jk_batch_check(jk_batch_t *b) {
  if (!b || !b->p) return fail(JK_EINVAL, "batch is NULL");
  return plan_check(b->p);
}

int jk_batch_stats(const jk_batch_t *b, jk_stats_t *out) {
  if (!b || !b->p || !out) return fail(JK_EINVAL, "NULL argument");
  return plan_stats(b->p, out);
}

int jk_batch_graph_info(const jk_batch_t *b, int *recorded, long long *replays, int *rerecords) {
  if (!b || !b->p) return fail(JK_EINVAL, "batch is NULL");
  if (recorded) *recorded = b->p->gexec != nullptr;
  if (replays) *replays = b->p->replays;
  if (rerecords) *rerecords = b->p->rerecords;
  return JK_OK;
}

void jk_batch_destroy(jk_batch_t *b) {
  if (!b) return;
  if (b->p) {
    plan_free(b->p);
    delete b->p;
  }
  delete b;
}

}  // extern "C"
