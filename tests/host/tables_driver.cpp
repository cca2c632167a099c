// Runs the host-side table builders on a binary input and writes their tables.
//
// Grouped ket table (argv: in out):
//   input (little endian): int64 n_points, int32 kg, int64 nnz, int32 pt_off[n_points+1],
//   int32 pt_key[nnz], double pt_u[4*nnz];
//   output: for each table, int64 length then the values (grp_off, grp_key, grp_u, grp_mask).
// Chunked bra table (argv: bra in out):
//   input: int64 n_points, int32 n_atoms, int32 tp, int32 max_pieces, int32 pad, int64 nnz,
//   int32 seg[4*n_atoms], int32 idx[nnz], double u[4*nnz];
//   output: the same framing for piece_off, piece_beg, piece_meta, piece_real, slot_off,
//   slot_piece, ent_pt, ent_u, key_off, key_slot, then {pl, max_pieces, max_slots}.
// On failure the reason on stderr, exit 2.
#include <cstdio>
#include <cstring>
#include <vector>

#include "tables.hpp"

template <typename T>
static bool rd(FILE* f, std::vector<T>& v, size_t n) {
  v.resize(n);
  return fread(v.data(), sizeof(T), n, f) == n;
}
template <typename T>
static void wr(FILE* f, const std::vector<T>& v) {
  const long long n = (long long)v.size();
  fwrite(&n, sizeof(n), 1, f);
  fwrite(v.data(), sizeof(T), v.size(), f);
}

static int ket(const char* in, const char* out) {
  FILE* f = fopen(in, "rb");
  if (!f) return 1;
  long long np = 0, nnz = 0;
  int kg = 0;
  if (fread(&np, 8, 1, f) != 1 || fread(&kg, 4, 1, f) != 1 || fread(&nnz, 8, 1, f) != 1) return 1;
  std::vector<int32_t> off, key;
  std::vector<double> u;
  if (!rd(f, off, np + 1) || !rd(f, key, nnz) || !rd(f, u, 4 * nnz)) return 1;
  fclose(f);
  cbs::GroupTables t;
  const std::string why = cbs::build_group_tables(np, off, key, u, kg, t);
  if (!why.empty()) {
    fprintf(stderr, "%s\n", why.c_str());
    return 2;
  }
  FILE* o = fopen(out, "wb");
  wr(o, t.grp_off);
  wr(o, t.grp_key);
  wr(o, t.grp_u);
  wr(o, t.grp_mask);
  fclose(o);
  return 0;
}

static int bra(const char* in, const char* out) {
  FILE* f = fopen(in, "rb");
  if (!f) return 1;
  long long np = 0, nnz = 0;
  int na = 0, tp = 0, maxp = 0, pad = 0;
  if (fread(&np, 8, 1, f) != 1 || fread(&na, 4, 1, f) != 1 || fread(&tp, 4, 1, f) != 1 ||
      fread(&maxp, 4, 1, f) != 1 || fread(&pad, 4, 1, f) != 1 || fread(&nnz, 8, 1, f) != 1)
    return 1;
  std::vector<int32_t> seg, idx;
  std::vector<double> u;
  if (!rd(f, seg, 4 * (size_t)na) || !rd(f, idx, nnz) || !rd(f, u, 4 * nnz)) return 1;
  fclose(f);
  cbs::BraTileTables t;
  const std::string why = cbs::build_bra_tile_tables(np, na, seg, idx, u, tp, maxp, pad, t);
  if (!why.empty()) {
    fprintf(stderr, "%s\n", why.c_str());
    return 2;
  }
  FILE* o = fopen(out, "wb");
  wr(o, t.piece_off);
  wr(o, t.piece_beg);
  wr(o, t.piece_meta);
  wr(o, t.piece_real);
  wr(o, t.slot_off);
  wr(o, t.slot_piece);
  wr(o, t.ent_pt);
  wr(o, t.ent_u);
  wr(o, t.key_off);
  wr(o, t.key_slot);
  wr(o, std::vector<int32_t>{t.pl, t.max_pieces, t.max_slots});
  fclose(o);
  return 0;
}

int main(int argc, char** argv) {
  if (argc == 3) return ket(argv[1], argv[2]);
  if (argc == 4 && strcmp(argv[1], "bra") == 0) return bra(argv[2], argv[3]);
  return 1;
}
