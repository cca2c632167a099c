// Host-side construction of the grouped projector table of the ket (plain C++, no HIP
// calls, so the CPU tests compile and check it on its own).
//
// Input: the point-major entries of the separable projectors, entries of point n being
// [pt_off[n], pt_off[n+1]) with key atom*4 + (w+1) and four values each.
//
// Grouped ket table: points in groups of kg consecutive indices; group g uses the
// keys [grp_off[g], grp_off[g+1]) (ascending) and, per key, the values of its kg points
// (zero where the point is outside that ball; a ball wider than the transverse period
// reaches a point twice with the same key, and the two values add).  grp_mask holds per
// key one bit per block of 16 points of the group: set where a value of the block is
// nonzero (the matrix-core ket skips the other blocks).

#pragma once

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

namespace cbs {

struct GroupTables {
  std::vector<int32_t> grp_off, grp_key, grp_mask;
  std::vector<double> grp_u;   // [key][kg][4]
};

// Returns an empty string on success, else the reason.
inline std::string build_group_tables(int64_t n_points, const std::vector<int32_t>& pt_off,
                                      const std::vector<int32_t>& pt_key, const std::vector<double>& pt_u,
                                      int kg, GroupTables& t) {
  const int64_t ngroups = (n_points + kg - 1) / kg;
  t.grp_off.assign(ngroups + 1, 0);
  t.grp_key.clear();
  t.grp_mask.clear();
  t.grp_u.clear();
  for (int64_t g = 0; g < ngroups; ++g) {
    const int64_t n0 = g * kg, n1 = std::min<int64_t>(n0 + kg, n_points);
    std::vector<int32_t> keys;
    for (int64_t n = n0; n < n1; ++n)
      for (int32_t e = pt_off[n]; e < pt_off[n + 1]; ++e) keys.push_back(pt_key[e]);
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    const size_t k0 = t.grp_key.size();
    t.grp_key.insert(t.grp_key.end(), keys.begin(), keys.end());
    t.grp_u.resize(t.grp_key.size() * kg * 4, 0.0);
    for (int64_t n = n0; n < n1; ++n)
      for (int32_t e = pt_off[n]; e < pt_off[n + 1]; ++e) {
        const size_t k = k0 + (std::lower_bound(keys.begin(), keys.end(), pt_key[e]) - keys.begin());
        for (int i = 0; i < 4; ++i) t.grp_u[(k * kg + (n - n0)) * 4 + i] += pt_u[4 * (size_t)e + i];
      }
    t.grp_mask.resize(t.grp_key.size(), 0);
    for (size_t k = k0; k < t.grp_key.size(); ++k)
      for (int p = 0; p < kg; ++p)
        for (int i = 0; i < 4; ++i)
          if (t.grp_u[(k * kg + p) * 4 + i] != 0.0) t.grp_mask[k] |= 1 << (p / 16);
    if (t.grp_key.size() >= ((size_t)1 << 31)) return "grouped projector table too large";
    t.grp_off[g + 1] = (int32_t)t.grp_key.size();
  }

  return std::string();
}

}  // namespace cbs
