/* The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: the group
 * closure, T_k, the dense matrix at n = 4 (exact and non-8-rational skews) and
 * sampled rows at n = 8.  Exit status 0 and "ok" when every call succeeds. */
#include <stdio.h>
#include <stdlib.h>

int fcco_group(int* out, int cap);
void fcco_T(const int* k, const double* theta, double* out);
int fcco_matrix(int n, const double* rst, double* F);
int fcco_forward_rows(int n, const double* rst, const double* x, int nrows, const long long* rows, double* out);

int main(void) {
  int W[24 * 9];
  if (fcco_group(W, 24) != 24) { printf("FAILED group\n"); return 1; }
  const int k[3] = {1, 2, 0};
  const double th[3] = {0.1, 0.2, 0.3};
  double t[2];
  fcco_T(k, th, t);
  const double skews[2][3] = {{0.125, 0.0, 0.375}, {0.31, 0.07, 0.23}};
  double* F = malloc(sizeof(double) * 2 * 64 * 64);
  for (int s = 0; s < 2; ++s)
    if (fcco_matrix(4, skews[s], F) != 0) { printf("FAILED matrix\n"); return 1; }
  free(F);
  double* x = calloc(2 * 512, sizeof(double));
  for (int i = 0; i < 512; ++i) x[2 * i] = (double)(i % 7) - 3.0;
  const long long rows[4] = {0, 7, 100, 511};
  double out[8];
  if (fcco_forward_rows(8, skews[0], x, 4, rows, out) != 0) { printf("FAILED rows\n"); return 1; }
  free(x);
  printf("ok\n");
  return 0;
}
