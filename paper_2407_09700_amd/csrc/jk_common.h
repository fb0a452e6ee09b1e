// Data layouts shared by the host planner and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jk {

constexpr int LMAX = 4;
constexpr int NPAIRCLASS = 15;            // (la, lb) with la >= lb, la <= 4
constexpr int NQCLASS = 120;              // (bra class >= ket class)

constexpr __host__ __device__ int ncart(int l) { return (l + 1) * (l + 2) / 2; }
constexpr __host__ __device__ int pair_class(int la, int lb) { return la * (la + 1) / 2 + lb; }
constexpr __host__ __device__ int qclass_index(int cb, int ck) { return cb * (cb + 1) / 2 + ck; }   // cb >= ck

// One shell pair after canonical ordering (l_a >= l_b). 80 bytes.
struct alignas(16) Pair {
  double A[3], B[3];     // centres of shell a and shell b
  int sa, sb;            // shell indices (for the symmetry factor)
  int ca, cb;            // first Cartesian AO of shell a / shell b inside the molecule's Cartesian matrices
  int pp_off, npp;       // primitive-pair range in the PrimPair array
  int mol;              // molecule of the pair (index into the per-molecule tables)
  int cls;               // pair class (la, lb)
};

// One primitive pair: exponent sum p = a + b, product centre P = (aA + bB)/p and
// K = c_a c_b exp(-a b |A-B|^2 / p) (the contraction coefficients are folded in).
struct alignas(16) PrimPair {
  double p, Px, Py, Pz, K;
  double ip;             // 1 / p
};

// Parameters of one class launch.
struct ClassArgs {
  const Pair *pairs;
  const PrimPair *pp;
  const int2 *quartets;   // (bra pair, ket pair) indices into pairs
  const int *count;       // device count of entries in quartets
  const double *Dc;       // Cartesian density, nc x nc
  double *Jc, *Kc;        // Cartesian accumulators, nc x nc (unsymmetrised)
  double *out;            // Schwarz maxima per pair (as uint64 bits) or ERI tensor
  double *scratch;        // global scratch for team kernels (per workgroup slices)
  long long scratch_per_wg;
  int nc;                 // Cartesian AO count
  int mode;               // MODE_JK, MODE_SCHWARZ, MODE_ERI
};

enum { MODE_JK = 0, MODE_SCHWARZ = 1, MODE_ERI = 2 };

}  // namespace jk
