// Host code of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer: the table derivations the plan runs (basis-change
// rows of Sec. IV-B for node sizes 2..16 and their block structure, the orbit
// templates, the fold+FFT unfold tables), at small sizes.  Exit status 0 and
// "ok" on stdout when every call succeeds; a sanitizer report aborts the run.
#include <cstdio>
#include <vector>

#include "asp_tables.hpp"
#include "fcc_dct.h"
#include "fold_plan.hpp"
#include "orbit_blocks.hpp"

static int fail(const char* what) {
  std::printf("FAILED %s\n", what);
  return 1;
}

int main() {
  for (int nl = 2; nl <= 16; nl *= 2) {
    const fcc::LevelTables* t = fcc::level_tables(nl);
    if (!t) return fail("level_tables");
    const size_t rows = size_t(8) * t->m * t->m * t->m;
    if (t->b_rowptr.size() != rows + 1 || t->c_rowptr.size() != rows + 1) return fail("row pointers");
    if (t->b_src.size() != size_t(t->b_rowptr.back()) || t->c_pid.size() != size_t(t->c_rowptr.back()))
      return fail("entries");
  }
  if (!fcc::gather_blocks(16)) return fail("gather_blocks");
  const fcc::OrbitBlocks* ob = fcc::orbit_blocks(32);
  if (!ob || ob->templ.empty()) return fail("orbit_blocks");
  const int r8[3] = {1, 0, 3};
  for (int n : {4, 8, 16}) {
    fcc::FoldTables ft;
    if (fcc::fold_tables(n, r8, &ft, true) != FCC_OK) return fail("fold_tables");
    if (ft.pid.size() != size_t(n) * n * n || ft.prid.size() != 24 * ft.reps.size()) return fail("fold sizes");
  }
  std::vector<unsigned char> pid(512);
  std::vector<double> K(2 * 256 * 24);
  int npat = 0;
  const double rst[3] = {0.125, 0.0, 0.375};
  if (fcc_fold_unfold_tables(8, rst, pid.data(), K.data(), &npat) != FCC_OK || npat < 1)
    return fail("fcc_fold_unfold_tables");
  std::printf("ok\n");
  return 0;
}
