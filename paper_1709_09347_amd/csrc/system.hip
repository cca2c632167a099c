// System set-up (cell blocks of one crystal), error strings, workspace and the
// operator entry points cbs_apply / cbs_apply_parts.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <type_traits>
#include <vector>

#include "cbs_internal.hpp"
#include "tables.hpp"

namespace cbs {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
const char* get_error() { return g_err; }

int32_t Workspace::get(const char* name, size_t bytes, void** out) {
  DevBuf& b = bufs[name];
  if (b.bytes < bytes) {
    if (b.p) {
      if (hipFree(b.p) != hipSuccess) {
        set_error("hipFree of workspace '%s' failed", name);
        return CBS_EHIP;
      }
      b.p = nullptr;
      b.bytes = 0;
    }
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      set_error("device allocation of %zu bytes for '%s' failed", bytes, name);
      return CBS_ENOMEM;
    }
    b.bytes = bytes;
    // CBS_WS_POISON=1 fills new workspace with NaN bytes (a check that no kernel reads a
    // workspace buffer before writing it)
    if (const char* e = getenv("CBS_WS_POISON")) {
      if (e[0] == '1' && hipMemset(b.p, 0xFF, bytes) != hipSuccess) {
        set_error("poisoning workspace '%s' failed", name);
        return CBS_EHIP;
      }
    }
  }
  *out = b.p;
  return CBS_OK;
}

void Workspace::drop(const char* name) {
  auto it = bufs.find(name);
  if (it == bufs.end()) return;
  if (it->second.p) (void)hipFree(it->second.p);
  bufs.erase(it);
}

void Workspace::release() {
  for (auto& kv : bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  bufs.clear();
}

// Central second-derivative weights of half-width p: the closed form
// c_m = 2 (-1)^{m+1} (p!)^2 / (m^2 (p-m)! (p+m)!), c_0 = -2 sum_{m=1}^p 1/m^2.
static void fd_weights(int p, double* c) {
  auto fact = [](int n) {
    double f = 1;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
  };
  double c0 = 0;
  for (int m = 1; m <= p; ++m) {
    const double sgn = (m % 2 == 1) ? 1.0 : -1.0;
    c[m] = 2.0 * sgn * fact(p) * fact(p) / ((double)m * m * fact(p - m) * fact(p + m));
    c0 -= 2.0 / ((double)m * m);
  }
  c[0] = c0;
  for (int m = p + 1; m < 5; ++m) c[m] = 0;
}

template <typename T>
static int32_t upload(const std::vector<T>& h, T** d) {
  *d = nullptr;
  if (h.empty()) return CBS_OK;
  if (hipMalloc(d, h.size() * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    *d = nullptr;
    set_error("device allocation of %zu bytes failed", h.size() * sizeof(T));
    return CBS_ENOMEM;
  }
  CBS_HIP(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return CBS_OK;
}

static int32_t build_projectors(cbs_system* s, const cbs_proj* pr) {
  Projector& P = s->proj;
  if (pr == nullptr || pr->n_atoms == 0) return CBS_OK;
  if (pr->n_proj < 1 || pr->n_proj > 4 || !pr->ball_off || !pr->ball_idx || !pr->ball_w ||
      !pr->ball_val || !pr->coeff) {
    set_error("projectors: need 1..4 projectors per atom and all table pointers");
    return CBS_EINVAL;
  }
  const int A = pr->n_atoms, np = pr->n_proj;
  const int64_t nnz = pr->ball_off[A];
  if (nnz >= (int64_t)1 << 31) {
    set_error("projectors: too many ball entries");
    return CBS_EINVAL;
  }
  std::vector<int32_t> seg(4 * (size_t)A);
  std::vector<int32_t> idx(nnz);
  std::vector<double> u64(4 * (size_t)nnz, 0.0);
  std::vector<double> cf(4 * (size_t)A, 0.0);
  std::vector<int32_t> cnt(s->N + 1, 0);
  int64_t pos = 0;
  for (int a = 0; a < A; ++a) {
    const int64_t lo = pr->ball_off[a], hi = pr->ball_off[a + 1];
    if (hi < lo || lo < 0 || hi > nnz) {
      set_error("projectors: ball_off is not non-decreasing");
      return CBS_EINVAL;
    }
    int wmin = 2, wmax = -2;
    for (int64_t e = lo; e < hi; ++e) {
      const int w = pr->ball_w[e];
      const int64_t n = pr->ball_idx[e];
      if (w < -1 || w > 1 || n < 0 || n >= s->N) {
        set_error("projectors: atom %d entry %lld out of range", a, (long long)e);
        return CBS_EINVAL;
      }
      wmin = std::min(wmin, w);
      wmax = std::max(wmax, w);
    }
    if (hi > lo && wmax - wmin > 1) {
      set_error("projectors: atom %d spans three cells (diameter above the cell length)", a);
      return CBS_EINVAL;
    }
    for (int sidx = 0; sidx < 3; ++sidx) {
      seg[4 * a + sidx] = (int32_t)pos;
      for (int64_t e = lo; e < hi; ++e) {
        if (pr->ball_w[e] != sidx - 1) continue;
        idx[pos] = pr->ball_idx[e];
        for (int i = 0; i < np; ++i) u64[4 * pos + i] = pr->ball_val[e * np + i];
        cnt[pr->ball_idx[e] + 1]++;
        ++pos;
      }
    }
    seg[4 * a + 3] = (int32_t)pos;
    for (int i = 0; i < np; ++i) cf[4 * a + i] = pr->coeff[a * np + i];
  }
  // point-major copy (counting sort by point)
  for (int64_t n = 0; n < s->N; ++n) cnt[n + 1] += cnt[n];
  std::vector<int32_t> pt_key(nnz);
  std::vector<double> pt_u(4 * (size_t)nnz);
  std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
  for (int a = 0; a < A; ++a) {
    for (int sidx = 0; sidx < 3; ++sidx) {
      for (int32_t e = seg[4 * a + sidx]; e < seg[4 * a + sidx + 1]; ++e) {
        const int32_t d = fill[idx[e]]++;
        pt_key[d] = a * 4 + sidx;
        for (int i = 0; i < 4; ++i) pt_u[4 * (size_t)d + i] = u64[4 * (size_t)e + i];
      }
    }
  }
  // grouped ket table (groups of KG consecutive points, keys ascending per group)
  GroupTables gt;
  const std::string why = build_group_tables(s->N, cnt, pt_key, pt_u, KG, gt);
  if (!why.empty()) {
    set_error("projectors: %s", why.c_str());
    return CBS_EINVAL;
  }
  std::vector<int32_t>& grp_off = gt.grp_off;
  std::vector<int32_t>& grp_key = gt.grp_key;
  std::vector<double>& grp_u = gt.grp_u;
  std::vector<int32_t>& grp_mask = gt.grp_mask;
  const int64_t ngroups = (int64_t)grp_off.size() - 1;
  P.grp_nkeys = (int64_t)grp_off[ngroups];
  if (grp_key.empty()) {   // keep the device pointers valid
    grp_key.push_back(0);
    grp_mask.push_back(0);
    grp_u.resize(KG * 4, 0.0);
  }
  std::vector<float> grp_u32(grp_u.begin(), grp_u.end());
  CBS_TRY(upload(grp_off, &P.grp_off));
  CBS_TRY(upload(grp_key, &P.grp_key));
  CBS_TRY(upload(grp_mask, &P.grp_mask));
  CBS_TRY(upload(grp_u, &P.grp_u64));
  CBS_TRY(upload(grp_u32, &P.grp_u32));
  // chunked bra tables for each chunk length; a length whose chunks hold more keys than the
  // pieces allowed is left out (the per-atom bra remains)
  for (int ti = 0; ti < 2; ++ti) {
    BraTileTables bt;
    if (!build_bra_tile_tables(s->N, A, seg, idx, u64, BT_TPS[ti], BT_MAXP, BT_EB, bt).empty() || bt.key_slot.empty())
      continue;
    ChunkTables& d = P.bt[ti];
    std::vector<float> btu32(bt.ent_u.begin(), bt.ent_u.end());
    CBS_TRY(upload(bt.piece_off, &d.piece_off));
    CBS_TRY(upload(bt.piece_beg, &d.piece_beg));
    CBS_TRY(upload(bt.piece_meta, &d.piece_meta));
    CBS_TRY(upload(bt.slot_off, &d.slot_off));
    CBS_TRY(upload(bt.slot_piece, &d.slot_piece));
    CBS_TRY(upload(bt.ent_pt, &d.ent_pt));
    CBS_TRY(upload(bt.ent_u, &d.u64));
    CBS_TRY(upload(btu32, &d.u32));
    std::vector<int32_t> pos(bt.key_slot.size());
    for (size_t t = 0; t < pos.size(); ++t) pos[bt.key_slot[t]] = (int32_t)t;
    CBS_TRY(upload(bt.key_off, &d.key_off));
    CBS_TRY(upload(pos, &d.slot_pos));
    d.tp = BT_TPS[ti];
    d.nchunks = bt.nchunks;
    d.nslots = (int32_t)bt.key_slot.size();
    d.pl = bt.pl;
  }
  std::vector<float> u32(u64.begin(), u64.end()), ptu32(pt_u.begin(), pt_u.end()),
      cf32(cf.begin(), cf.end());
  P.n_atoms = A;
  P.nnz = nnz;
  CBS_TRY(upload(seg, &P.seg));
  CBS_TRY(upload(idx, &P.ball_idx));
  CBS_TRY(upload(u64, &P.ball_u64));
  CBS_TRY(upload(u32, &P.ball_u32));
  CBS_TRY(upload(cf, &P.coeff64));
  CBS_TRY(upload(cf32, &P.coeff32));
  CBS_TRY(upload(cnt, &P.pt_off));
  CBS_TRY(upload(pt_key, &P.pt_key));
  CBS_TRY(upload(pt_u, &P.pt_u64));
  CBS_TRY(upload(ptu32, &P.pt_u32));
  return CBS_OK;
}

static void free_system(cbs_system* s) {
  auto f = [](void* p) {
    if (p) (void)hipFree(p);
  };
  f(s->vloc64);
  f(s->vloc32);
  Projector& P = s->proj;
  f(P.seg);
  f(P.ball_idx);
  f(P.ball_u64);
  f(P.ball_u32);
  f(P.coeff64);
  f(P.coeff32);
  f(P.pt_off);
  f(P.pt_key);
  f(P.pt_u64);
  f(P.pt_u32);
  f(P.grp_off);
  f(P.grp_key);
  f(P.grp_mask);
  f(P.grp_u64);
  f(P.grp_u32);
  for (ChunkTables& d : P.bt) {
    f(d.piece_off);
    f(d.piece_beg);
    f(d.piece_meta);
    f(d.slot_off);
    f(d.slot_piece);
    f(d.ent_pt);
    f(d.u64);
    f(d.u32);
    f(d.key_off);
    f(d.slot_pos);
  }
  f(s->last.vecs);
  s->ws.release();
}

int32_t apply_parts_dev(cbs_system* s, double E, int32_t n_vec, const double2* c0,
                        const double2* cp, const double2* cm, const double2* x, double2* y,
                        hipStream_t st) {
  if (n_vec <= 0) return CBS_OK;
  const int32_t nr = (n_vec + 1) / 2;
  Pair<double>* px = nullptr;
  Pair<double>* pq = nullptr;
  Pair<double>* kt = nullptr;
  RunCoef* coef = nullptr;
  CBS_TRY(ws_get(s->ws, "ap.x", (size_t)nr * s->N, &px));
  CBS_TRY(ws_get(s->ws, "ap.q", (size_t)nr * s->N, &pq));
  CBS_TRY(ws_get(s->ws, "ap.coef", (size_t)nr, &coef));
  if (s->proj.n_atoms > 0) CBS_TRY(ws_get(s->ws, "ap.kt", (size_t)nr * s->proj.n_atoms * 12, &kt));
  std::vector<RunCoef> hc(nr);
  for (int k = 0; k < nr; ++k) {
    for (int h = 0; h < 2; ++h) {
      const int v = 2 * k + h;
      const bool ok = v < n_vec;
      hc[k].c[3 * h + 0] = ok ? c0[v] : make_double2(0, 0);
      hc[k].c[3 * h + 1] = ok ? cp[v] : make_double2(0, 0);
      hc[k].c[3 * h + 2] = ok ? cm[v] : make_double2(0, 0);
    }
    hc[k].E = E;
  }
  CBS_HIP(hipMemcpyAsync(coef, hc.data(), nr * sizeof(RunCoef), hipMemcpyHostToDevice, st));
  CBS_TRY(launch_to_pairs<double>(s->N, n_vec, x, px, st));
  StencilLaunch l{};
  l.nruns = nr;
  l.rin = px;
  l.q = pq;
  l.coef = coef;
  const int32_t ty = s->tile_y[0] ? s->tile_y[0] : default_tile_y(s, sizeof(Pair<double>));
  CBS_TRY(launch_stencil<double>(s, false, l, ty, st));
  if (s->proj.n_atoms > 0) {
    CBS_TRY(launch_bra<double>(s, nr, px, coef, nullptr, 0, kt, nullptr, st, false));
    CBS_TRY(launch_ket_add<double>(s, nr, pq, kt, st));
  }
  CBS_TRY(launch_from_pairs<double>(s->N, n_vec, pq, y, st));
  // the host coefficient array must outlive the asynchronous copy
  CBS_HIP(hipStreamSynchronize(st));
  return CBS_OK;
}

template <typename R>
static int32_t apply_z(cbs_system* s, double E, int32_t n_vec, const double* z, const void* x,
                       void* y, hipStream_t st) {
  const int32_t nr = (n_vec + 1) / 2;
  Pair<R>* px = nullptr;
  Pair<R>* pq = nullptr;
  Pair<R>* kt = nullptr;
  RunCoef* coef = nullptr;
  const char* nx = std::is_same<R, double>::value ? "ap.x" : "ap32.x";
  const char* nq = std::is_same<R, double>::value ? "ap.q" : "ap32.q";
  const char* nk = std::is_same<R, double>::value ? "ap.kt" : "ap32.kt";
  CBS_TRY(ws_get(s->ws, nx, (size_t)nr * s->N, &px));
  CBS_TRY(ws_get(s->ws, nq, (size_t)nr * s->N, &pq));
  CBS_TRY(ws_get(s->ws, "ap.coef", (size_t)nr, &coef));
  if (s->proj.n_atoms > 0) CBS_TRY(ws_get(s->ws, nk, (size_t)nr * s->proj.n_atoms * 12, &kt));
  std::vector<RunCoef> hc(nr);
  for (int k = 0; k < nr; ++k) {
    for (int h = 0; h < 2; ++h) {
      const int v = 2 * k + h;
      double zr = 1, zi = 0;
      if (v < n_vec) {
        zr = z[2 * v];
        zi = z[2 * v + 1];
      }
      const double d = zr * zr + zi * zi;
      hc[k].c[3 * h + 0] = make_double2(v < n_vec ? 1.0 : 0.0, 0.0);
      hc[k].c[3 * h + 1] = make_double2(zr, zi);
      hc[k].c[3 * h + 2] = make_double2(zr / d, -zi / d);
    }
    hc[k].E = E;
  }
  CBS_HIP(hipMemcpyAsync(coef, hc.data(), nr * sizeof(RunCoef), hipMemcpyHostToDevice, st));
  CBS_TRY(launch_to_pairs<R>(s->N, n_vec, x, px, st));
  StencilLaunch l{};
  l.nruns = nr;
  l.rin = px;
  l.q = pq;
  l.coef = coef;
  const int32_t ty = s->tile_y[std::is_same<R, double>::value ? 0 : 1];
  CBS_TRY(launch_stencil<R>(s, false, l, ty ? ty : default_tile_y(s, sizeof(Pair<R>)), st));
  if (s->proj.n_atoms > 0) {
    CBS_TRY(launch_bra<R>(s, nr, px, coef, nullptr, 0, kt, nullptr, st, true));
    CBS_TRY(launch_ket_add<R>(s, nr, pq, kt, st));
  }
  CBS_TRY(launch_from_pairs<R>(s->N, n_vec, pq, y, st));
  CBS_HIP(hipStreamSynchronize(st));
  return CBS_OK;
}

}  // namespace cbs

using namespace cbs;

extern "C" {

const char* cbs_strerror(int32_t code) {
  switch (code) {
    case CBS_OK: return "ok";
    case CBS_EINVAL: return "invalid argument";
    case CBS_ENOMEM: return "out of device memory";
    case CBS_EHIP: return "HIP runtime error";
    case CBS_ENOCONV: return "linear solve did not converge";
    case CBS_EBREAKDOWN: return "BiCG breakdown";
    case CBS_ERANK: return "Hankel rank saturated (subspace too small)";
    case CBS_ETOOMANY: return "more eigenvalues than the output holds";
    case CBS_ENONFINITE: return "non-finite moments";
    case CBS_EEIG: return "dense eigenvalue step failed";
    default: return "unknown error";
  }
}

const char* cbs_last_error(void) { return get_error(); }

void cbs_params_default(cbs_params* p) {
  std::memset(p, 0, sizeof(*p));
  p->lambda_min = 0.5;
  p->n_q = 32;
  p->n_rhs = 16;
  p->n_mom = 8;
  p->delta = 1e-10;
  p->tol = 1e-10;
  p->max_iter = 20000;
  p->precision = CBS_FP64;
  p->extraction = CBS_RR;
  p->half_stop = 0;
  p->inner_tol = 1e-6;
  p->max_refine = 60;
  p->chunk = 8;
  p->conj_nodes = 1;
  p->block = 1;
  p->lo_window = 0;
}

int32_t cbs_system_create(cbs_system** out, int32_t device, const cbs_grid* g, const double* v_loc,
                          const cbs_proj* proj) {
  if (!out || !g || !v_loc) {
    set_error("cbs_system_create: null argument");
    return CBS_EINVAL;
  }
  *out = nullptr;
  const int p = g->fd_order / 2;
  if (g->fd_order % 2 != 0 || p < 1 || p > 4) {
    set_error("fd_order must be 2, 4, 6 or 8 (got %d)", g->fd_order);
    return CBS_EINVAL;
  }
  if (g->nx < 1 || g->nx > 256 || g->ny < 1 || g->nz < p || !(g->h > 0)) {
    set_error("grid %dx%dx%d h=%g unsupported (need 1<=nx<=256, ny>=1, nz>=p=%d, h>0)", g->nx, g->ny,
              g->nz, g->h, p);
    return CBS_EINVAL;
  }
  // the stencil stages one complex128 plane of a tile of full x rows (at least one row and
  // its p halo rows on either side, primal and dual) in LDS
  if ((size_t)(1 + 2 * p) * g->nx * 2 * 16 > 64 * 1024) {
    set_error("grid nx=%d too wide for fd_order %d: one stencil tile needs %zu bytes of LDS (64 KB)", g->nx,
              g->fd_order, (size_t)(1 + 2 * p) * g->nx * 2 * 16);
    return CBS_EINVAL;
  }
  const int64_t N = (int64_t)g->nx * g->ny * g->nz;
  if (N >= ((int64_t)1 << 31)) {
    set_error("grid too large");
    return CBS_EINVAL;
  }
  for (int64_t i = 0; i < N; ++i)
    if (!std::isfinite(v_loc[i])) {
      set_error("cbs_system_create: v_loc[%lld] is not finite", (long long)i);
      return CBS_EINVAL;
    }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    set_error("no HIP device %d", device);
    return CBS_EHIP;
  }
  CBS_HIP(hipSetDevice(device));
  {
    // set-up of cbs_apply_noalloc: the device address of its scratch array on this device
    void* sp = nullptr;
    CBS_TRY(noalloc_scratch(device, &sp));
  }
  cbs_system* s = new cbs_system();
  s->device = device;
  s->nx = g->nx;
  s->ny = g->ny;
  s->nz = g->nz;
  s->p = p;
  s->h = g->h;
  s->N = N;
  fd_weights(p, s->fd);
  std::vector<double> v(v_loc, v_loc + N);
  std::vector<float> vf(v.begin(), v.end());
  int32_t rc = upload(v, &s->vloc64);
  if (rc == CBS_OK) rc = upload(vf, &s->vloc32);
  if (rc == CBS_OK) rc = build_projectors(s, proj);
  if (rc != CBS_OK) {
    free_system(s);
    delete s;
    return rc;
  }
  s->tile_y[0] = default_tile_y(s, sizeof(Pair<double>));
  s->tile_y[1] = default_tile_y(s, sizeof(Pair<float>));
  *out = s;
  return CBS_OK;
}

void cbs_system_destroy(cbs_system* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  free_system(s);
  delete s;
}

int32_t cbs_system_set_vloc(cbs_system* s, const double* v_loc) {
  if (!s || !v_loc) {
    set_error("cbs_system_set_vloc: null argument");
    return CBS_EINVAL;
  }
  for (int64_t i = 0; i < s->N; ++i)
    if (!std::isfinite(v_loc[i])) {
      set_error("cbs_system_set_vloc: v_loc[%lld] is not finite", (long long)i);
      return CBS_EINVAL;
    }
  CBS_HIP(hipSetDevice(s->device));
  std::vector<float> vf(v_loc, v_loc + s->N);
  CBS_HIP(hipMemcpy(s->vloc64, v_loc, s->N * sizeof(double), hipMemcpyHostToDevice));
  CBS_HIP(hipMemcpy(s->vloc32, vf.data(), s->N * sizeof(float), hipMemcpyHostToDevice));
  return CBS_OK;
}

int64_t cbs_system_npoints(const cbs_system* s) { return s ? s->N : -1; }

int64_t cbs_system_solve_id(const cbs_system* s) { return s ? s->solve_id : -1; }

const char* cbs_system_tiling(const cbs_system* s, int32_t* tile_y) {
  if (!s) return "";
  if (tile_y) {
    tile_y[0] = s->tile_y[0];
    tile_y[1] = s->tile_y[1];
  }
  return s->tune_log.c_str();
}

int32_t cbs_apply(cbs_system* s, double E, int32_t n_vec, const double* z, int32_t dtype,
                  const void* x, void* y, void* stream) {
  if (!s || n_vec < 0 || (n_vec > 0 && (!z || !x || !y)) || (dtype != CBS_C128 && dtype != CBS_C64)) {
    set_error("cbs_apply: bad argument");
    return CBS_EINVAL;
  }
  for (int v = 0; v < n_vec; ++v) {
    if (z[2 * v] == 0.0 && z[2 * v + 1] == 0.0) {
      set_error("cbs_apply: z must be nonzero");
      return CBS_EINVAL;
    }
  }
  if (n_vec == 0) return CBS_OK;
  CBS_HIP(hipSetDevice(s->device));
  hipStream_t st = (hipStream_t)stream;
  if (dtype == CBS_C128) return apply_z<double>(s, E, n_vec, z, x, y, st);
  return apply_z<float>(s, E, n_vec, z, x, y, st);
}

int32_t cbs_apply_parts(cbs_system* s, double E, int32_t n_vec, const double* c0, const double* cp,
                        const double* cm, const void* x, void* y, void* stream) {
  if (!s || n_vec < 0 || (n_vec > 0 && (!c0 || !cp || !cm || !x || !y))) {
    set_error("cbs_apply_parts: bad argument");
    return CBS_EINVAL;
  }
  if (n_vec == 0) return CBS_OK;
  CBS_HIP(hipSetDevice(s->device));
  return apply_parts_dev(s, E, n_vec, (const double2*)c0, (const double2*)cp, (const double2*)cm,
                         (const double2*)x, (double2*)y, (hipStream_t)stream);
}

}  // extern "C"
