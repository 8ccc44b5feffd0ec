// Orbit-block form of the basis change of one radix-2x2x2 level (Sec. IV-B,
// eq. FastAlgorithm) for a node of size nl = 2m.
//
// The gather tables of asp_tables.hpp list every row of B_nl and C_nl.  Those
// matrices have much more structure than a sparse table shows:
//
//  * Blocks.  Let W act on the cube grid [0,m)^3 by p -> (g p) mod m.  The rows
//    (def, p) of B_nl for the cubes p of one orbit O read exactly the sources
//    kappa = q + m o, q in O, o in {0,1}^3 (the "octets" of the orbit), and no
//    other rows read them.  So B_nl is block diagonal with one block of size
//    8|O| per orbit, and C_nl = B_nl^{-1} has the same blocks.
//  * Templates.  Label the cube q of an orbit with representative p0 (its
//    smallest cube index) by the first g with (g p0) mod m = q, and the octet
//    point q + m o by (slot of q, o).  In these labels the block's matrix is
//    the same for every orbit of one kind, and for nl >= 16 there are eight
//    kinds (orbit sizes 24, 12, 12, 6, 6, 4, 3, 1) whose matrices do not depend
//    on nl (coefficients are polynomials in c = (sigma, tau, rho) of the node).
//
// These facts were found on the derived tables and are checked against them
// (tests compare the expansion of the templates with the tables row by row).
// The templates are taken from the tables of one small node size (nl_ref = nl
// for nl < 16, 32 otherwise), and the orbits of the target size are
// classified by their label sets, so a level needs no per-row table at all.
#pragma once
#include <array>
#include <cstdint>
#include <vector>

namespace fcc {

struct OrbitTemplate {
  int nc = 0;                   // cubes of the orbit
  std::vector<int> w;           // nc: cube slot j is (W[w_j] p0) mod m
  std::vector<int> key;         // 4*nc: (w_j, floor((W[w_j] p0)_d / m), d = 0..2), the class label set
  std::vector<int> b_rowptr;    // 8 nc + 1: B row j*8 + def (output 2 q_j + def)
  std::vector<uint16_t> b_ent;  // (source slot j'*8 + o) << 8 | poly; source q_j' + m o
  std::vector<int> c_rowptr;    // 8 nc + 1: C row j'*8 + o (output q_j' + m o)
  std::vector<uint16_t> c_ent;  // (cube slot j*8 + def) << 8 | poly; source 2 q_j + def
};

struct OrbitBlocks {
  int nl = 0, m = 0;
  int npoly = 0, nconst = 0;    // polynomial ids below nconst are constants
  std::vector<double> poly;     // npoly * 5, monomials {1, c3, c1, c2, c1 c3}
  std::vector<OrbitTemplate> templ;
  std::vector<std::vector<uint32_t>> reps;  // per template: representatives p0, (x<<20)|(y<<10)|z, Morton order
};

// Templates and orbit lists of node size nl (4 <= nl <= 1024, a power of two),
// cached; nullptr if nl is invalid, memory runs out, or an orbit of nl matches
// no template of the reference size (the structure above would then not hold).
const OrbitBlocks* orbit_blocks(int nl);

}  // namespace fcc
