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

// Chunked bra table: the ball entries regrouped by chunks of tp consecutive points, so
// that one workgroup holding the direction of a chunk (for a group of runs) in LDS can
// contract every entry of the chunk from LDS.
//
// Input: the atom-major entries, segment s (cell shift w = s - 1) of atom a spanning
// [seg[4a+s], seg[4a+s+1]), point idx[e] and four values u[4e..4e+3].
//
// Key k = 3a + s.  A slot is one (chunk, key) pair with at least one entry; slots are
// numbered by chunk, then key.  The entries of a slot (ascending point, then input order)
// are cut into pieces of consecutive entries and nearly equal size: per chunk the smallest
// piece length for which the chunk has at most max_pieces pieces (pl: the longest piece).
//   piece_off[c]..piece_off[c+1]   pieces of chunk c (global piece numbers)
//   piece_beg[q], piece_meta[q]    first entry of piece q; (local slot << 16) | entry count,
//                                  the count padded to a multiple of pad with entries of
//                                  point 0 and zero values (piece_real[q]: the count before)
//   slot_off[c]..slot_off[c+1]     slots of chunk c
//   slot_piece[g]..slot_piece[g+1] pieces of slot g
//   ent_pt[e], ent_u[4e..]         reordered (and padded) entries: point offset within the
//                                  chunk, values
//   key_off[k]..key_off[k+1]       slots of key k (ascending, i.e. in chunk order) in key_slot
struct BraTileTables {
  int32_t tp = 0, pl = 0, nchunks = 0, max_pieces = 0, max_slots = 0;
  std::vector<int32_t> piece_off, piece_beg, piece_meta, piece_real, slot_off, slot_piece, ent_pt, key_off,
      key_slot;
  std::vector<double> ent_u;
};

// Returns an empty string on success, else the reason.
inline std::string build_bra_tile_tables(int64_t n_points, int32_t n_atoms, const std::vector<int32_t>& seg,
                                         const std::vector<int32_t>& idx, const std::vector<double>& u, int tp,
                                         int max_pieces, int pad, BraTileTables& t) {
  if (tp < 1 || max_pieces < 1 || pad < 1) return "bra tile table: bad chunk, piece or padding size";
  const int64_t nnz = (int64_t)idx.size();
  const int64_t nchunks = (n_points + tp - 1) / tp;
  if (nchunks >= ((int64_t)1 << 31)) return "bra tile table: too many chunks";
  const int nkeys = 3 * n_atoms;
  // entries ordered by (chunk, key, point, input order)
  std::vector<int32_t> key_of(nnz);
  for (int a = 0; a < n_atoms; ++a)
    for (int sg = 0; sg < 3; ++sg)
      for (int32_t e = seg[4 * a + sg]; e < seg[4 * a + sg + 1]; ++e) key_of[e] = 3 * a + sg;
  std::vector<int32_t> order(nnz);
  for (int64_t e = 0; e < nnz; ++e) order[e] = (int32_t)e;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const int64_t cx = idx[x] / tp, cy = idx[y] / tp;
    if (cx != cy) return cx < cy;
    if (key_of[x] != key_of[y]) return key_of[x] < key_of[y];
    return idx[x] < idx[y];
  });
  // slots: runs of equal (chunk, key)
  std::vector<int64_t> slot_beg;   // first position in order
  std::vector<int32_t> slot_chunk, slot_key;
  for (int64_t i = 0; i < nnz; ++i) {
    const int32_t e = order[i];
    const int64_t c = idx[e] / tp;
    if (i == 0 || c != idx[order[i - 1]] / tp || key_of[e] != key_of[order[i - 1]]) {
      slot_beg.push_back(i);
      slot_chunk.push_back((int32_t)c);
      slot_key.push_back(key_of[e]);
    }
  }
  const int64_t nslots = (int64_t)slot_beg.size();
  slot_beg.push_back(nnz);
  t.tp = tp;
  t.nchunks = (int32_t)nchunks;
  t.slot_off.assign(nchunks + 1, 0);
  for (int64_t g = 0; g < nslots; ++g) t.slot_off[slot_chunk[g] + 1]++;
  for (int64_t c = 0; c < nchunks; ++c) t.slot_off[c + 1] += t.slot_off[c];
  t.max_slots = 0;
  for (int64_t c = 0; c < nchunks; ++c) t.max_slots = std::max(t.max_slots, t.slot_off[c + 1] - t.slot_off[c]);
  if (t.max_slots > max_pieces) return "bra tile table: more keys in a chunk than pieces allowed";
  if (t.max_slots >= (1 << 15)) return "bra tile table: too many keys in a chunk";
  // pieces: per chunk the smallest length lc for which its slots, each cut into
  // ceil(n / lc) pieces of nearly equal size, give at most max_pieces pieces (so the
  // chunk's work is spread evenly over the threads)
  t.piece_off.assign(nchunks + 1, 0);
  t.piece_beg.clear();
  t.piece_meta.clear();
  t.piece_real.clear();
  t.ent_pt.clear();
  t.ent_u.clear();
  t.slot_piece.assign(nslots + 1, 0);
  t.pl = 0;
  t.max_pieces = 0;
  for (int64_t c = 0; c < nchunks; ++c) {
    const int32_t g0 = t.slot_off[c], g1 = t.slot_off[c + 1];
    int64_t longest = 1;
    for (int32_t g = g0; g < g1; ++g) longest = std::max(longest, slot_beg[g + 1] - slot_beg[g]);
    auto count = [&](int64_t lc) {
      int64_t n = 0;
      for (int32_t g = g0; g < g1; ++g) n += (slot_beg[g + 1] - slot_beg[g] + lc - 1) / lc;
      return n;
    };
    int64_t lo = 1, hi = longest;   // count(longest) = slots <= max_pieces
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (count(mid) <= max_pieces) hi = mid;
      else lo = mid + 1;
    }
    const int64_t lc = lo;
    if (lc + pad >= (1 << 16)) return "bra tile table: a piece would exceed 65535 entries";
    for (int32_t g = g0; g < g1; ++g) {
      t.slot_piece[g] = (int32_t)t.piece_beg.size();
      const int64_t n = slot_beg[g + 1] - slot_beg[g];
      const int64_t np = (n + lc - 1) / lc;
      for (int64_t q = 0; q < np; ++q) {
        const int64_t b = slot_beg[g] + n * q / np, e = slot_beg[g] + n * (q + 1) / np;
        const int64_t padded = (e - b + pad - 1) / pad * pad;
        t.piece_beg.push_back((int32_t)t.ent_pt.size());
        t.piece_meta.push_back(((g - g0) << 16) | (int32_t)padded);
        t.piece_real.push_back((int32_t)(e - b));
        t.pl = std::max<int32_t>(t.pl, (int32_t)padded);
        for (int64_t i = b; i < b + padded; ++i) {
          if (i < e) {
            const int32_t en = order[i];
            t.ent_pt.push_back((int32_t)(idx[en] - (int64_t)(idx[en] / tp) * tp));
            for (int k = 0; k < 4; ++k) t.ent_u.push_back(u[4 * (size_t)en + k]);
          } else {
            t.ent_pt.push_back(0);
            for (int k = 0; k < 4; ++k) t.ent_u.push_back(0.0);
          }
        }
      }
    }
    t.piece_off[c + 1] = (int32_t)t.piece_beg.size();
    t.max_pieces = std::max<int32_t>(t.max_pieces, t.piece_off[c + 1] - t.piece_off[c]);
  }
  t.slot_piece[nslots] = (int32_t)t.piece_beg.size();
  if (t.piece_beg.size() >= ((size_t)1 << 31) || t.ent_pt.size() >= ((size_t)1 << 31))
    return "bra tile table: too many pieces or entries";
  // slots of each key, in chunk order
  t.key_off.assign(nkeys + 1, 0);
  for (int64_t g = 0; g < nslots; ++g) t.key_off[slot_key[g] + 1]++;
  for (int k = 0; k < nkeys; ++k) t.key_off[k + 1] += t.key_off[k];
  t.key_slot.assign(nslots, 0);
  std::vector<int32_t> fill(t.key_off.begin(), t.key_off.end() - 1);
  for (int64_t g = 0; g < nslots; ++g) t.key_slot[fill[slot_key[g]]++] = (int32_t)g;
  return std::string();
}

}  // namespace cbs
