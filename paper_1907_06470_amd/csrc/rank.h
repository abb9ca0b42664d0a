// Descending rank of one eigenvalue among l under a strict total order, shared
// by the small-SVD finishing kernel and its host-side test.
//
// NaN ranks as -infinity and equal values rank by index, so for any input
// (NaN, +-inf, ties) the ranks of 0 .. l-1 are a permutation of 0 .. l-1 and
// every index built from them stays inside the array.  A plain "count the
// larger values" rank gives a NaN rank 0 (every comparison with NaN is
// false) and makes the other ranks collide, leaving slots of the inverse
// permutation unset.
#pragma once

#if defined(__HIPCC__)
#define RSVD_HD __host__ __device__
#else
#define RSVD_HD
#endif

namespace rsvd {

RSVD_HD inline double nan_as_low(double x) { return x == x ? x : -__builtin_inf(); }

// Rank (0 = largest) of lv[i] among lv[0 .. l); lv must already hold
// nan_as_low() of the values.
RSVD_HD inline int desc_rank(const double* lv, int l, int i) {
  const double li = lv[i];
  int rank = 0;
  for (int j = 0; j < l; ++j) {
    const double lj = lv[j];
    rank += (lj > li) || (lj == li && j < i);
  }
  return rank;
}

}  // namespace rsvd
