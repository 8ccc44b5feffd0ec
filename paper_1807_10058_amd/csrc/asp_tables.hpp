// Host-side derivation of the basis-change factors of the radix-2x2x2 FCC
// algorithm (Sec. IV-B, eq. FastAlgorithm) for one node size nl = 2m.
//
// The paper names the basis change B_n(r,s,t) from b_n = (T_k | k in [0,n)^3)
// to b~_n = (T_abc * T_def(T_{m00},T_{0m0},T_{00m})) but leaves it to future
// work.  It is derived here from:
//   - Prop. 1 (vi): T_def(T_{m e1}, T_{m e2}, T_{m e3}) = T_{m*def};
//   - Prop. 1 (iv): T_a T_b = (1/24) sum_g T_{a + g b}  (orbit {g b}, g acting on
//     the column vector, as in the power form A3PowerForm);
//   - Prop. 1 (iii): T_k = T_{gk}, so every index is replaced by its dominant
//     representative (all coordinates >= 0);
//   - the skew ideal <T_{nl e_d} - c_d> of Sec. IV-A (c = (sigma,tau,rho) of the
//     node): for dominant kappa with kappa_d >= nl, lambda = kappa - nl e_d and
//     O_d the orbit of e_d,  c_d T_lambda = (1/|O_d|) sum_{mu in O_d} T_{dom(lambda + nl mu)},
//     solved for T_kappa.
// C = B^{-1} has the product expansions as columns; it is unit-triangular up to
// a constant diagonal in the height order h(k) = 3k1 + 4k2 + 3k3, so B follows
// column by column in increasing height.  Every coefficient is a polynomial in
// (c1,c2,c3) with rational coefficients; the tables keep one id per distinct
// polynomial.
#pragma once
#include <array>
#include <cstdint>
#include <vector>

namespace fcc {

struct LevelTables {
  int nl = 0, m = 0;
  std::vector<int> mono;               // 3 * nmono exponents
  std::vector<double> poly;            // npoly * nmono
  int nmono = 0, npoly = 0;
  std::vector<int> b_rowptr;           // 8 m^3 + 1
  std::vector<uint32_t> b_src;         // packed node-local kappa
  std::vector<uint16_t> b_pid;
  std::vector<int> c_rowptr;           // 8 m^3 + 1
  std::vector<uint32_t> c_src;         // packed node-local position def + 2 abc
  std::vector<uint16_t> c_pid;
};

// Derives (or returns the cached) tables for node size nl (power of two, 2..1024).
// Returns nullptr if nl is invalid or memory runs out.  Thread safe.
const LevelTables* level_tables(int nl);

// Blocks of B_nl: the cubes abc whose gather rows (def, abc) read a common
// source form one block, and no source is read from two blocks, so B_nl is
// block diagonal after permuting rows and sources (for generic abc a block is
// an orbit of 24 cubes under an affine action of W).  C_nl = B_nl^{-1} has the
// transposed structure: row kappa of C reads only the positions def + 2 abc
// of the cubes of the block that reads kappa in B.
struct GatherBlocks {
  std::vector<int> cube;   // m^3: per natural cube (a*m + b)*m + c, the smallest cube of its block
  std::vector<int> kappa;  // nl^3: per node-local source kappa, the block of the B rows that read it
};
// Derived from level_tables(nl) (cached; nullptr on failure).
const GatherBlocks* gather_blocks(int nl);

// W = S_4 as 24 integer 3x3 matrices (row-major), closure of the generators of
// eq. GeneratorMatricesS4.
const std::vector<std::array<int, 9>>& weyl_group();

// Dominant representative of (a,b,c) under W (simple reflections until all >= 0).
void dominant(int& a, int& b, int& c);

inline uint32_t pack3(int x, int y, int z) {
  return (uint32_t(x) << 20) | (uint32_t(y) << 10) | uint32_t(z);
}

}  // namespace fcc
