/*
 * jk.h -- C ABI of the MI355X (gfx950) integral-direct Coulomb/exchange builder.
 *
 * Computes, for a symmetric density D over contracted Gaussian shells (l <= 4),
 *     J[mu,nu] = sum_{la,si} (mu nu|la si) D[la,si]
 *     K[mu,nu] = sum_{la,si} (mu la|nu si) D[la,si]
 * with the two-electron integrals evaluated by Rys quadrature (paper section 2: the
 * ERI as an exact N-point quadrature over three 2D integrals, N = floor(L/2) + 1) and
 * contracted with D in the same pass (section 3, Algorithms 2 and 3: the six J/K
 * updates per integral). Shell quartets are screened with the Cauchy-Schwarz factor
 * and the density block maxima (section 3, the pair prescreen I_ab > tau and the
 * density-weighted test I_ab I_cd P >= tau).
 *
 * Conventions (all arguments):
 *  - Atomic units. Row-major. Doubles are IEEE binary64, indices are int32.
 *  - A shell is (atom, l, nprim, prim_off, pure). Its primitives are exps[prim_off +
 *    k], coefs[prim_off + k] for k < nprim. A coefficient multiplies the UNNORMALISED
 *    primitive x^ax y^ay z^az exp(-a r^2) centred on the atom; the library applies no
 *    normalisation of its own.
 *  - Cartesian components of a shell are ordered ax descending, then ay descending
 *    (for l = 2: xx, xy, xz, yy, yz, zz).
 *  - pure = 1 (allowed for any l, acts only for l >= 2): the shell carries the 2l+1
 *    real solid harmonics sqrt(4pi/(2l+1)) r^l Y_lm, m = -l..l (m < 0: sin-type),
 *    written in the Cartesian components with, in each row, the largest-magnitude
 *    coefficient positive (the first in component order on ties). l = 0, 1 are always
 *    Cartesian (s; x, y, z).
 *  - AO order: shells in input order, functions of a shell contiguous. nao is the sum
 *    of the shell sizes (2l+1 for pure l >= 2, else (l+1)(l+2)/2).
 *  - Device buffers (D, J, K, ERI) are caller-owned, on the current HIP device, nao*nao
 *    doubles, contiguous. Host buffers are noted as such.
 *
 * Errors: every int-returning call returns JK_OK (0) or a negative JK_E* code, never
 * aborts and never throws. jk_last_error() returns a thread-local message for the last
 * failure on the calling thread. After an error the outputs are unspecified and any
 * plan remains valid to destroy.
 */
#ifndef JK_H
#define JK_H

#ifdef __cplusplus
extern "C" {
#endif

#define JK_OK 0
#define JK_EINVAL (-1)        /* bad argument: null pointer, size mismatch, non-finite */
#define JK_EUNSUPPORTED (-2)  /* l > 4, nprim > 64, or a feature not built */
#define JK_ENOMEM (-3)        /* host or device allocation failed */
#define JK_EDEVICE (-4)       /* a HIP call failed; the message carries its string */
#define JK_ENODEV (-5)        /* no HIP device */
#define JK_EOVERFLOW (-6)     /* jk_plan_check: the last build's work lists overflowed (see there) */

#define JK_FP64 0
#define JK_MIXED 1

#define JK_FLAG_PROFILE 1     /* jk_opts_t.flags: time every kernel launch of an execute */
#define JK_FLAG_GRAPH 2       /* jk_opts_t.flags: record the build in a HIP graph on the first
                                 execute and replay it afterwards (no host round trip inside) */
#define JK_FLAG_TUNE 4        /* jk_opts_t.flags: on the first execute, time candidate builds
                                 and keep, per register tier, fused or per-class launches, per
                                 class the launch shape (root table and exchange rows in LDS or
                                 not), and per launch the workgroup count */
#define JK_FLAG_J_ONLY 8      /* jk_opts_t.flags: build J only (K is not written and may be NULL);
                                 the density-weighted screen takes the two Coulomb blocks D[a,b],
                                 D[c,d] only */
#define JK_FLAG_K_ONLY 16     /* jk_opts_t.flags: build K only (J is not written and may be NULL);
                                 the screen takes the four exchange blocks D[a,c], D[a,d], D[b,c],
                                 D[b,d] only */

typedef struct {
  int nshell;
  const int *atom;       /* [nshell] atom index of each shell, 0 <= atom < natom */
  const int *l;          /* [nshell] angular momentum, 0..4 */
  const int *nprim;      /* [nshell] contraction order K, 1..64 */
  const int *prim_off;   /* [nshell] first primitive of the shell in exps/coefs */
  const int *pure;       /* [nshell] 0 Cartesian, 1 real solid harmonics */
  int nprim_total;       /* length of exps and coefs */
  const double *exps;    /* [nprim_total] exponents, > 0 */
  const double *coefs;   /* [nprim_total] contraction coefficients (see above) */
} jk_basis_t;            /* all pointers are HOST pointers, read during plan creation only */

typedef struct {
  double thresh;         /* tau: quartet kept iff I_ab > tau, I_cd > tau, I_ab I_cd P >= tau */
  int precision;         /* JK_FP64 (default) or JK_MIXED */
  double fp32_cutoff;    /* JK_MIXED: kept quartets with I_ab I_cd P below this evaluate their
                            2D integrals, products and transfer in FP32 (lane-per-quartet
                            classes; the workgroup-body classes stay FP64); roots, weights and
                            every J/K accumulation stay FP64. >= 0; 0 routes nothing to FP32 */
  int flags;             /* OR of JK_FLAG_* (0: none) */
  const char *tune_cache; /* JK_FLAG_TUNE: HOST path of a text file that keeps the choices
                             between runs (read if present, written after tuning); NULL: none */
  double dmax;           /* > 0: jk_plan_create sizes the screened work lists for densities whose
                            largest element in the Cartesian components is at most dmax, so that
                            no execute waits for the device. 0 (default): the first execute
                            sizes them for twice its own density's largest element, waiting once
                            for the device; later executes never wait */
} jk_opts_t;

typedef struct jk_plan jk_plan_t;
typedef struct jk_batch jk_batch_t;

typedef struct {
  long long kept_quartets;      /* unique shell quartets that passed the screen (last execute) */
  long long candidate_quartets; /* quartets tested by the screen (last execute) */
  long long kept_fp32;          /* of kept_quartets, those evaluated in FP32 (mixed mode) */
  long long prim_quartets;      /* primitive quartets of the kept quartets */
  int npairs_kept;              /* shell pairs with I_ab > tau */
  int nao, nao_cart, nshell;
  double plan_ms;               /* host wall time of jk_plan_create */
  int overflow;                 /* 1 if the last execute's work lists overflowed (jk_plan_check) */
  long long list_capacity;      /* entries of the screened work lists */
} jk_stats_t;

/* Create a plan for one molecule: validates the basis on the host, builds the shell
 * pair tables, uploads them and computes the Cauchy-Schwarz factors on the device
 * (section 3: I_ab = max over the functions of |(ab|ab)|^(1/2)). coords: HOST, natom x 3.
 * opts may be NULL (tau = 1e-12, FP64). The plan owns all device workspace; *out is
 * set only on success. Synchronises the device. */
int jk_plan_create(const jk_basis_t *basis, const double *coords, int natom, const jk_opts_t *opts,
                   jk_plan_t **out);

/* J and K for the density D (DEVICE, nao x nao, symmetric, caller-owned): the Coulomb and
 * exchange sums of section 3 (Algorithms 2 and 3: ERIs of the kept shell quartets evaluated
 * and digested with D in the same pass). J and K are OVERWRITTEN (DEVICE, nao x nao; with
 * JK_FLAG_J_ONLY / JK_FLAG_K_ONLY the other may be NULL). Asynchronous: the build is
 * enqueued on `stream` (a hipStream_t, NULL = default stream) and the call returns without
 * waiting for it, except on a plan's first execute when the plan was created with dmax = 0
 * (that one call sizes the work lists from D and waits for the device once). Results are
 * valid after the stream synchronises. A density whose density-weighted screen keeps more
 * candidates than the lists hold leaves J and K incomplete; jk_plan_check reports this.
 * A plan must not be executed concurrently on two streams. */
int jk_plan_execute(jk_plan_t *plan, const double *D, double *J, double *K, void *stream);

/* Waits for the plan's last execute and returns JK_OK, or JK_EOVERFLOW if its work lists
 * overflowed (its J and K are then incomplete). On JK_EOVERFLOW the plan has already grown
 * its lists (for twice that density's largest element) and a new execute with the same
 * density completes. */
int jk_plan_check(jk_plan_t *plan);

/* Nuclear gradient of the two-electron energy E = tr(D (J - K/2)) with the density held fixed
 * (section 4, Algorithm 4: derivative integrals of each kept quartet, from the raised and
 * lowered primitive Gaussians of the differentiated centre in the Rys form of section 2,
 * contracted with W = s [8 D_ab D_cd - 2 D_ac D_bd - 2 D_ad D_bc] at once; the fourth centre
 * by translational invariance). D: DEVICE nao x nao, symmetric. grad: DEVICE natom x 3
 * doubles (atoms as given to jk_plan_create), OVERWRITTEN. The quartets are those the J/K
 * screen keeps for D (six density blocks). Single-molecule plans made for J and K, shells up
 * to l = 3 (else JK_EUNSUPPORTED / JK_EINVAL). Asynchronous as jk_plan_execute; jk_plan_check
 * reports an overflow of the work lists the same way. */
int jk_grad(jk_plan_t *plan, const double *D, double *grad, void *stream);

/* jk_plan_create + jk_plan_execute + jk_plan_check (executing again after an overflow) +
 * jk_plan_destroy; thresh overrides opts->thresh. Waits for the build. */
int jk_build(const jk_basis_t *basis, const double *coords, int natom, const double *D, double thresh,
             double *J, double *K, const jk_opts_t *opts, void *stream);

/* jk_build for callers that cannot allocate device memory (tight loops, harnesses that forbid
 * hipMalloc): the same plan, build and kernels, with every device buffer the library needs
 * carved from a fixed array of 128 MB per device (a file-scope __device__ array the library
 * holds until the process ends) instead of hipMalloc; nothing is allocated or freed on the
 * device. A molecule whose plan needs more returns JK_ENOMEM with the sizes in the message
 * (outputs untouched beyond that point). opts flags JK_FLAG_PROFILE, GRAPH and TUNE are
 * rejected (JK_EINVAL). Calls on one device share the array: the library serialises them
 * within the process; calls from two processes on one device race. Waits for the build. */
int jk_build_static(const jk_basis_t *basis, const double *coords, int natom, const double *D, double thresh,
                    double *J, double *K, const jk_opts_t *opts, void *stream);

void jk_plan_destroy(jk_plan_t *plan);

/* nao (final basis) and nao_cart (all shells Cartesian) of a plan. */
int jk_plan_sizes(const jk_plan_t *plan, int *nao, int *nao_cart);

/* Statistics of the plan and its last execute (HOST struct). */
int jk_stats(const jk_plan_t *plan, jk_stats_t *out);

/* Per-launch profile of the executes of a plan created with JK_FLAG_PROFILE, averaged over
 * the executes since the previous jk_profile call (at most the last 32). One entry per
 * integral launch (kind 0): either one quartet class (lc, ld >= 0) or one register tier of a
 * bra class fused over its ket classes (lc = -1, ld = tier, team = 2), plus the preparation
 * launches (kind 1: density transform, block maxima, screening) and the final symmetrise and
 * transform (kind 2). ms is the mean HIP-event time of the launch on the caller's stream (the
 * events are recorded inside each execute; reading them here waits for the stream). quartets,
 * prim_quartets and flops are those of the last execute. flops is the algorithmic operation
 * count of the launch's quartets (an FMA counts 2), from the steps of the method: per
 * primitive quartet the pair-quartet scalars, and per Rys root (section 2) the root and
 * weight, the recurrence coefficients, the 2D recurrences in x, y, z and the three-operand
 * product per [e0|f0] element; per contracted quartet the two transfers and the multiply-adds
 * of the digestion (Algorithm 2: two per integral for J, four for K). out is HOST memory of
 * max_entries entries; *n_entries receives the count. Graph launches are not profiled. */
typedef struct {
  int kind;                     /* 0 class kernel, 1 preparation, 2 finalisation */
  int la, lb, lc, ld;           /* class (kind 0); lc = -1, ld = tier for a fused launch */
  int team;                     /* 0 lane-per-quartet, 1 workgroup body, 2 fused bra-class launch,
                                   3 fused launch of the FP32 quartets (mixed precision) */
  int nroots;                   /* Rys roots N of the class */
  long long quartets;           /* kept unique shell quartets */
  long long prim_quartets;      /* their primitive quartets */
  double ms;                    /* kernel time */
  double flops;                 /* algorithmic flops (see above) */
} jk_profile_t;

int jk_profile(jk_plan_t *plan, jk_profile_t *out, int max_entries, int *n_entries);

/* Test hook: full Cartesian ERI tensor (DEVICE, nao_cart^4 doubles, overwritten),
 * unscreened, with the same integral kernels as jk_plan_execute. Small inputs only. */
int jk_eri_tensor(jk_plan_t *plan, double *eri, void *stream);

/* Test hook: Cauchy-Schwarz factors per shell pair (HOST, nshell x nshell, symmetric),
 * computed over the Cartesian components of the shells. */
int jk_schwarz(const jk_plan_t *plan, double *out);

/* Host-only helper: the library's Cartesian -> real-solid-harmonic matrix for l
 * (HOST out, (2l+1) x (l+1)(l+2)/2, row-major). Needs no device. l in 2..4. */
int jk_sph_matrix(int l, double *out);

/* Host-only test hook: the closed-form Rys rule for 1 or 2 roots (paper section 2: the N-point
 * Gauss rule of the weight whose moments are the Boys values F_0..F_(2N-1)(T), here from a
 * series or erf/exp), compiled for the host from the kernels' source. u, w: HOST arrays of
 * nroots entries (u = t^2). */
int jk_rys_closed(int nroots, double T, double *u, double *w);

/* Host-only test hook: the rule the lane-per-quartet kernels use for 1 or 2 roots: the same
 * Gauss rule, with F_0..F_(2N-1)(T) from the Taylor series about the nearest point of a Boys
 * grid (T_i = i/8, gen_boys_grid.py), compiled for the host from the kernels' source.
 * Requires 0 <= T < 40 (one root) or 50 (two roots), beyond which the kernels take the
 * Gauss-Hermite limit; else JK_EINVAL. u, w: HOST arrays of nroots entries (u = t^2). */
int jk_rys_grid(int nroots, double T, double *u, double *w);

/* One-electron integrals of an SCF around the J/K build, on the host (section 4: they are
 * evaluated on the CPU): overlap S, kinetic energy T and nuclear attraction V = -sum_C Z_C
 * (mu|1/|r - R_C||nu) over the shells of `basis` (same conventions as jk_plan_create), in
 * the final basis, and the nuclear repulsion energy. charges: HOST, natom nuclear charges
 * (any real values; 0 leaves a centre out of V). S, T, V: HOST nao x nao, OVERWRITTEN;
 * enuc: HOST scalar. Needs no device. */
int jk_one_electron(const jk_basis_t *basis, const double *coords, int natom, const double *charges, double *S,
                    double *T, double *V, double *enuc);

/* ---- Batched build: many independent molecules in one pass.
 * The shell pairs of all molecules share the class work lists and the persistent
 * integral launches (one launch per class group for the whole batch, not per molecule);
 * each molecule keeps its own density and outputs. This extends the paper's per-class
 * batching of shell quartets (section 3) across molecules. */

/* Create a batch of nmol molecules: basis[m], coords[m] (HOST, natom[m] x 3) as for
 * jk_plan_create. opts (may be NULL) applies to every molecule. With JK_FLAG_GRAPH an
 * execute records the whole build (density transform, screen, integral launches,
 * finalisation) in a HIP graph and launches it; later executes with the same D, J, K
 * pointers launch the recorded graph again. (JK_FLAG_GRAPH acts the same way on a plan.) */
int jk_batch_create(int nmol, const jk_basis_t *const *basis, const double *const *coords, const int *natom,
                    const jk_opts_t *opts, jk_batch_t **out);

/* Packed layout of a batch: molecule m's nao[m] x nao[m] block starts at element off[m]
 * of the packed D, J and K arrays (off has nmol+1 entries; off[nmol] = total length).
 * off and nao are HOST arrays; either may be NULL. */
int jk_batch_offsets(const jk_batch_t *batch, long long *off, int *nao);

/* J and K of every molecule (DEVICE, packed as jk_batch_offsets says, overwritten) for the
 * packed densities D (DEVICE). Asynchronous on `stream`, as jk_plan_execute (including the
 * one wait of a first execute with dmax = 0, and the overflow report of jk_batch_check).
 * Graph launches wait for nothing either. */
int jk_batch_execute(jk_batch_t *batch, const double *D, double *J, double *K, void *stream);

/* jk_plan_check for a batch: waits for its last execute; JK_EOVERFLOW if that build's work
 * lists overflowed (the lists have grown, a graph is recorded again on the next execute). */
int jk_batch_check(jk_batch_t *batch);

/* Statistics of the batch and its last execute, summed over the molecules. */
int jk_batch_stats(const jk_batch_t *batch, jk_stats_t *out);

/* Graph status: *recorded = 1 once a graph exists, *replays = executes that launched an
 * already recorded graph, *rerecords = recordings after the first (grown work lists or new
 * D, J, K pointers). HOST ints, may be NULL. */
int jk_batch_graph_info(const jk_batch_t *batch, int *recorded, long long *replays, int *rerecords);

void jk_batch_destroy(jk_batch_t *batch);

/* Thread-local message of the last failure (never NULL). */
const char *jk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* JK_H */
