// Runs the host-side grouped-table builder on a binary input and writes its tables.
// Input (little endian): int64 n_points, int32 kg, int64 nnz, int32 pt_off[n_points+1],
// int32 pt_key[nnz], double pt_u[4*nnz].
// Output: for each table, int64 length then the values (grp_off, grp_key, grp_u,
// grp_mask); on
// failure the reason on stderr, exit 2.
#include <cstdio>
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

int main(int argc, char** argv) {
  if (argc != 3) return 1;
  FILE* f = fopen(argv[1], "rb");
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
  FILE* o = fopen(argv[2], "wb");
  wr(o, t.grp_off);
  wr(o, t.grp_key);
  wr(o, t.grp_u);
  wr(o, t.grp_mask);
  fclose(o);
  return 0;
}
