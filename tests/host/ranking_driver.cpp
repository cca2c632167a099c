// Runs the singular-value ranking of the Hankel SVD on values read from stdin.
// Input: n, then n values (text; "nan", "inf", "-inf" allowed).
// Output: the permutation perm[rank] = column, then "finite 1|0".
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ranking.hpp"

int main() {
  int n = 0;
  if (scanf("%d", &n) != 1 || n < 0) return 1;
  std::vector<double> v(n);
  char tok[64];
  for (int i = 0; i < n; ++i) {
    if (scanf("%63s", tok) != 1) return 1;
    v[i] = strtod(tok, nullptr);
  }
  std::vector<int> perm(n, -1);
  for (int j = 0; j < n; ++j) {
    const int r = cbs::desc_rank(n, v.data(), j);
    if (r < 0 || r >= n) return 2;   // out of range: the gather through perm would fault
    perm[r] = j;
  }
  for (int r = 0; r < n; ++r) printf("%d ", perm[r]);
  printf("\nfinite %d\n", cbs::all_finite(n, v.data()) ? 1 : 0);
  return 0;
}
