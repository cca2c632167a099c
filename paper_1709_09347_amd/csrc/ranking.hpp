// Ordering of the Hankel singular values (plain C++, shared by the device SVD kernel and
// the host, and compiled on its own by a CPU test).
//
// The singular values are ranked descending under a strict total order: a non-finite value
// (a linear solve that diverged leaves NaN or Inf in the moments) counts as -1, below every
// column norm, and equal values go by column index.  Distinct columns then get distinct
// ranks in [0, n), so perm[rank(j)] = j is a permutation of 0..n-1 whatever the values are,
// and every later gather through perm stays inside the matrix.
#pragma once

#if defined(__HIPCC__)
#define CBS_HD __host__ __device__
#else
#define CBS_HD
#endif

namespace cbs {

// v itself when finite, -1 otherwise (v - v is 0 only for finite v)
CBS_HD inline double rank_key(double v) { return (v - v == 0.0) ? v : -1.0; }

// rank of column j among the n values v[0..n): the number of columns before it
CBS_HD inline int desc_rank(int n, const double* v, int j) {
  const double sj = rank_key(v[j]);
  int r = 0;
  for (int k = 0; k < n; ++k) {
    const double sk = rank_key(v[k]);
    r += (sk > sj || (sk == sj && k < j)) ? 1 : 0;
  }
  return r;
}

// true when every value is finite: the singular values can be truncated and used; the
// solver reports non-finite moments (CBS_ENONFINITE) otherwise
inline bool all_finite(int n, const double* v) {
  for (int i = 0; i < n; ++i)
    if (!(v[i] - v[i] == 0.0)) return false;
  return true;
}

}  // namespace cbs
