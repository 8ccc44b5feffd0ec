// Host side of the fold+FFT formulation of the transform (a variant, not the
// paper's factorisation).
//
// Exchanging the two sums of the explicit matrix (Sec. IV-A, eq.
// SU4ChebyshevTransformExplicitForm) with lambda = g kappa gives
//   X[j] = sum_mu Fh[mu] exp(2 pi i mu.j / n),                          (1)
//   Fh[mu] = (1/24) sum_{(kappa, g): g kappa = mu mod n} x[kappa] exp(2 pi i (g kappa).rst / n),
// a twiddled fold of x onto the n-torus followed by an unnormalised inverse
// 3-D DFT.  The fold only moves kappa inside its orbit under W on the torus,
// so it is block diagonal over those orbits, and its inverse is
//   x = (Fold^H Fold)^{-1} Fold^H Fh,  Fh = DFT(X) / n^3.
// The Gram matrix Fold^H Fold has the entries
//   Gram[k, k'] = (1/24) sum_{h in W: h k = k' mod n} T_{rho_h}(rst),  rho_h = (k' - h k) / n,
// (T the orbit-sum polynomial of Definition 1 at an integer index), so it
// splits into small blocks wherever T vanishes at the wrap vectors.  Folding
// the block inverse and Fold^H into one gather gives, per point k,
//   x[k] = sum_u K_k[u] exp(-2 pi i (u k).rst / n) Fh[u k mod n],        (2)
//   K_k[u] = (1/24) sum_{members m of k's block} Ginv[k, m] exp(-2 pi i (u h_m^{-1} rho_{h_m}).rst),
// with h_m any element taking k to m.  K_k depends on k only through the wrap
// pattern of its orbit (which multiples of n the points u k cross, and which
// u k coincide), so the distinct rows are few; every point stores the index
// of its row.  The device side needs 8 rst integral (the phases of the wraps
// are then 8th roots of unity).
#pragma once
#include <complex>
#include <cstdint>
#include <vector>

#include "fcc_dct.h"

namespace fcc {

// Unfold tables of size n for the skew r8 / 8: pid[k] (flat index) selects the
// row K[pid * 24 + u] of eq. (2), u in the order of the FCC_GROUP table.
//
// For the orbit-block kernels: one representative per orbit of W on the
// torus (its smallest flat index), ordered by the kFoldBox box that holds it
// (boxes and points within a box in lexicographic order), and per image h of
// representative r the row index prid[h * nrep + r] = pid[h r mod n].
constexpr int kFoldBox[3] = {4, 4, 8};
struct FoldTables {
  std::vector<uint8_t> pid;
  std::vector<std::complex<double>> K;
  int npat = 0;
  std::vector<int32_t> reps;
  std::vector<uint8_t> prid;
};
// FCC_ERR_UNSUPPORTED if more than 256 distinct rows occur or a Gram block is
// larger than an orbit; FCC_ERR_SINGULAR_SKEW if a block is singular.
fcc_status fold_tables(int n, const int r8[3], FoldTables* out, bool orbits = false);

}  // namespace fcc
