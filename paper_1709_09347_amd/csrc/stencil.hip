// Local part of the operator P(z) = (H0 - E) + z H+ + z^{-1} H- (paper Sec. 2, Eq. 4):
// the -1/2 finite-difference Laplacian, the local potential and the Bloch phases of
// the z wrap, applied to every run (primal and dual vector side by side).
//
// Kernel design (gfx950):
//  * one workgroup = one run x one tile of TY full x-rows (x periodic inside the tile),
//    marching over all z planes; the y halo (p rows each side) comes through L2;
//  * the plane being processed is staged in LDS (double-buffered, one barrier per plane)
//    for the x and y neighbours; the z direction never touches LDS: every thread keeps
//    a queue of 2p+1 partial outputs in registers, plane m adds c_{m-o} * v_m to the
//    outputs o = m-p..m+p, and output m-p is complete after plane m;
//  * planes below 0 and above nz-1 are the neighbouring cells: they are loaded for the
//    owning column only and carry the coefficients cm (= 1/z) and cp (= z);
//  * BiCG mode fuses p_new = r + beta p_old (dual: conj(beta)), x += xcoef * p_old,
//    the write of p_new and the local part of sigma = pt^H q;
//  * blocks are renumbered so that consecutive tiles of a run land on one XCD, where
//    they share the halo rows in that XCD's L2.
#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "cbs_internal.hpp"

namespace cbs {

template <typename R>
struct StArgs {
  int32_t nx, ny, nz, ty, ntiles, nlogical, nbuf;
  int32_t nzseg;          // z segments per tile (1 for the BiCG stencil)
  int64_t N;
  double kin;   // -1/(2 h^2)
  double c[5];  // c_0..c_p
  const R* vloc;          // local potential in the storage precision
  const double* vloc64;   // and in complex128 arithmetic's precision
  const Pair<R>* rin;
  const Pair<R>* pold;
  Pair<R>* pnew;
  Pair<R>* q;
  Pair<R>* x;
  const RunCoef* coef;
  const double2* beta;
  const double2* xcoef;
  const int32_t* status;
  int32_t need_status;
  double2* sig_part;
  const int32_t* list;    // active runs (ascending) or NULL
  const int32_t* count;   // device count of list entries
};

__device__ __forceinline__ double2 wave_sum2(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// The direction p = r + beta p_old, with the roundings fixed by explicit fused multiply-adds:
// the halo planes recompute what the tile that owns them stored, and the two must agree bit
// for bit (the operator is applied to the stored direction), whatever the compiler would
// contract in either place.
template <typename C>
__device__ __forceinline__ cplx<C> dir_fma(cplx<C> r, cplx<C> b, cplx<C> p) {
  return mkc<C>(fma(-b.y, p.y, fma(b.x, p.x, r.x)), fma(b.y, p.x, fma(b.x, p.y, r.y)));
}

// R: storage precision of the vectors (and of the LDS plane); C: arithmetic precision.
template <typename R, typename C, int P, bool BICG>
__global__ void __launch_bounds__(512) k_stencil(StArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double2 red[8];
  Pair<R>* lds = reinterpret_cast<Pair<R>*>(smem_raw);

  const int per_run = a.ntiles * a.nzseg;
  const int nl = (a.list != nullptr) ? min(a.nlogical, *a.count * per_run) : a.nlogical;
  const int lb = remap_active(blockIdx.x, nl);
  if (lb < 0) return;
  const int slot = lb / per_run;
  const int rem = lb - slot * per_run;
  const int tile = rem / a.nzseg;
  // z segment [z0, z1) of the outputs; the march covers p halo planes on either side
  const int zlen = (a.nz + a.nzseg - 1) / a.nzseg;
  const int z0 = (rem - tile * a.nzseg) * zlen;
  const int z1 = min(z0 + zlen, a.nz);
  if (z0 >= z1) return;
  const int run = (a.list != nullptr) ? a.list[slot] : slot;
  if (a.status != nullptr && a.status[run] != a.need_status) return;

  const int nx = a.nx, ny = a.ny, nz = a.nz, TY = a.ty;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int tx = tid % nx;
  const int ty = tid / nx;
  const int y = tile * TY + ty;
  const bool own = (y < ny);
  const int64_t plane = (int64_t)nx * ny;
  const int64_t base = (int64_t)run * a.N;
  const int rows = TY + 2 * P;
  const int region = rows * nx;
  const int y0 = tile * TY - P;

  const RunCoef cf = a.coef[run];
  const cplx<C> c0a = ccast<C, double>(cf.c[0]), cpa = ccast<C, double>(cf.c[1]),
                cma = ccast<C, double>(cf.c[2]);
  const cplx<C> c0b = ccast<C, double>(cf.c[3]), cpb = ccast<C, double>(cf.c[4]),
                cmb = ccast<C, double>(cf.c[5]);
  const C Erun = (C)cf.E;
  cplx<C> ba = mkc<C>(0, 0), bb = ba, xa = ba, xb = ba;
  bool do_x = false;
  if (BICG) {
    const double2 bt = a.beta[run];
    ba = mkc<C>((C)bt.x, (C)bt.y);
    bb = cconj<C>(ba);
    const double2 xc = a.xcoef[run];
    xa = mkc<C>((C)xc.x, (C)xc.y);
    xb = cconj<C>(xa);
    do_x = (xc.x != 0.0 || xc.y != 0.0);
  }
  const C kin = (C)a.kin;
  C cc[P + 1];
#pragma unroll
  for (int j = 0; j <= P; ++j) cc[j] = (C)a.c[j];
  C zc[2 * P + 1];
#pragma unroll
  for (int d = 0; d <= 2 * P; ++d) zc[d] = kin * cc[d > P ? d - P : P - d];

  Pair<C> acc[2 * P + 1];
#pragma unroll
  for (int d = 0; d <= 2 * P; ++d) {
    acc[d].a = mkc<C>(0, 0);
    acc[d].b = mkc<C>(0, 0);
  }
  cplx<C> pdq[P + 1];
#pragma unroll
  for (int d = 0; d <= P; ++d) pdq[d] = mkc<C>(0, 0);
  double2 sig = make_double2(0.0, 0.0);

  // Plane staging, software-pipelined: the loads of plane m+1 are issued into registers
  // before plane m is computed and committed (direction update, stores, LDS) after it,
  // when every thread holds at most PF elements of the region; otherwise load and commit
  // happen together.
  constexpr int PF = 2;
  const bool pipe = region <= PF * nthr;
  Pair<R> pr_r[PF], pr_p[PF], pr_x[PF];
  auto issue = [&](int mm) {
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int e = tid + k * nthr;
      if (e >= region) break;
      const int r = e / nx;
      const int xx = e - r * nx;
      const int uy = y0 + r;
      int gy = uy % ny;
      if (gy < 0) gy += ny;
      const int64_t n = base + xx + (int64_t)nx * gy + plane * mm;
      pr_r[k] = a.rin[n];
      if (BICG) {
        pr_p[k] = a.pold[n];
        if (do_x && r >= P && r < P + TY && uy < ny) pr_x[k] = a.x[n];
      }
    }
  };
  auto commit = [&](int mm, Pair<R>* buf) {
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int e = tid + k * nthr;
      if (e >= region) break;
      if (BICG) {
        const int r = e / nx;
        const int xx = e - r * nx;
        const int uy = y0 + r;
        int gy = uy % ny;
        if (gy < 0) gy += ny;
        const int64_t n = base + xx + (int64_t)nx * gy + plane * mm;
        Pair<C> v = pcast<C, R>(pr_r[k]);
        const Pair<C> po = pcast<C, R>(pr_p[k]);
        v.a = dir_fma<C>(v.a, ba, po.a);
        v.b = dir_fma<C>(v.b, bb, po.b);
        const Pair<R> vs = pcast<R, C>(v);
        if (r >= P && r < P + TY && uy < ny) {
          a.pnew[n] = vs;
          if (do_x) {
            Pair<C> xv = pcast<C, R>(pr_x[k]);
            xv.a = cfma<C>(xv.a, xa, po.a);
            xv.b = cfma<C>(xv.b, xb, po.b);
            a.x[n] = pcast<R, C>(xv);
          }
        }
        buf[e] = vs;
      } else {
        buf[e] = pr_r[k];
      }
    }
  };
  const int m_end = z1 + P, real_end = min(nz, m_end);
  if (pipe && max(z0 - P, 0) < real_end) issue(max(z0 - P, 0));

  for (int m = z0 - P; m < m_end; ++m) {
    const bool real = (m >= 0) && (m < nz);
    Pair<C> s;
    s.a = mkc<C>(0, 0);
    s.b = s.a;
    Pair<C> inb = s;
    if (real) {
      Pair<R>* buf = lds + ((a.nbuf == 2) ? (m & 1) * region : 0);
      if (a.nbuf == 1 && m > 0) __syncthreads();   // single buffer: previous plane fully read
      if (pipe) {
        commit(m, buf);
        if (m + 1 < real_end) issue(m + 1);
      }
      for (int e = tid; e < region && !pipe; e += nthr) {
        const int r = e / nx;
        const int xx = e - r * nx;
        const int uy = y0 + r;
        int gy = uy % ny;
        if (gy < 0) gy += ny;
        const int64_t n = base + xx + (int64_t)nx * gy + plane * m;
        if (BICG) {
          Pair<C> v = pcast<C, R>(a.rin[n]);
          const Pair<C> po = pcast<C, R>(a.pold[n]);
          v.a = dir_fma<C>(v.a, ba, po.a);
          v.b = dir_fma<C>(v.b, bb, po.b);
          const Pair<R> vs = pcast<R, C>(v);   // the stored direction is the one applied
          if (r >= P && r < P + TY && uy < ny) {
            a.pnew[n] = vs;
            if (do_x) {
              Pair<C> xv = pcast<C, R>(a.x[n]);
              xv.a = cfma<C>(xv.a, xa, po.a);
              xv.b = cfma<C>(xv.b, xb, po.b);
              a.x[n] = pcast<R, C>(xv);
            }
          }
          buf[e] = vs;
        } else {
          buf[e] = a.rin[n];
        }
      }
      __syncthreads();
      if (own) {
        const int row = (ty + P) * nx;
        const Pair<C> v = pcast<C, R>(buf[row + tx]);
        cplx<C> sa = cscale<C>(v.a, (C)2 * cc[0]);
        cplx<C> sb = cscale<C>(v.b, (C)2 * cc[0]);
#pragma unroll
        for (int j = 1; j <= P; ++j) {
          int xl = tx - j;
          xl += (xl < 0) ? nx : 0;
          xl += (xl < 0) ? nx : 0;   // nx may be smaller than p
          xl += (xl < 0) ? nx : 0;
          xl += (xl < 0) ? nx : 0;
          int xr = tx + j;
          xr -= (xr >= nx) ? nx : 0;
          xr -= (xr >= nx) ? nx : 0;
          xr -= (xr >= nx) ? nx : 0;
          xr -= (xr >= nx) ? nx : 0;
          const Pair<C> l = pcast<C, R>(buf[row + xl]);
          const Pair<C> rr = pcast<C, R>(buf[row + xr]);
          const Pair<C> dn = pcast<C, R>(buf[row - j * nx + tx]);
          const Pair<C> up = pcast<C, R>(buf[row + j * nx + tx]);
          const C cj = cc[j];
          sa = cfma_r<C>(sa, cj, cadd<C>(cadd<C>(l.a, rr.a), cadd<C>(dn.a, up.a)));
          sb = cfma_r<C>(sb, cj, cadd<C>(cadd<C>(l.b, rr.b), cadd<C>(dn.b, up.b)));
        }
        const int64_t pt = tx + (int64_t)nx * y + plane * m;
        const C vl = (sizeof(C) == 8) ? (C)a.vloc64[pt] : (C)a.vloc[pt];
        const C vd = vl - Erun;
        sa = cfma_r<C>(cscale<C>(sa, kin), vd, v.a);
        sb = cfma_r<C>(cscale<C>(sb, kin), vd, v.b);
        inb.a = cmul<C>(c0a, sa);
        inb.b = cmul<C>(c0b, sb);
        s.a = cmul<C>(c0a, v.a);
        s.b = cmul<C>(c0b, v.b);
        pdq[P] = v.b;
      }
    } else if (own) {
      const int iz = (m < 0) ? m + nz : m - nz;
      const int64_t n = base + tx + (int64_t)nx * y + plane * iz;
      Pair<C> v = pcast<C, R>(a.rin[n]);
      if (BICG) {
        const Pair<C> po = pcast<C, R>(a.pold[n]);
        v.a = dir_fma<C>(v.a, ba, po.a);
        v.b = dir_fma<C>(v.b, bb, po.b);
        v = pcast<C, R>(pcast<R, C>(v));   // as stored by the tile that owns the plane
      }
      if (m < 0) {
        s.a = cmul<C>(cma, v.a);
        s.b = cmul<C>(cmb, v.b);
      } else {
        s.a = cmul<C>(cpa, v.a);
        s.b = cmul<C>(cpb, v.b);
      }
    }
    if (own) {
#pragma unroll
      for (int d = 0; d <= 2 * P; ++d) {
        acc[d].a = cfma_r<C>(acc[d].a, zc[d], s.a);
        acc[d].b = cfma_r<C>(acc[d].b, zc[d], s.b);
      }
      if (real) {
        acc[P].a = cadd<C>(acc[P].a, inb.a);
        acc[P].b = cadd<C>(acc[P].b, inb.b);
      }
      const int o = m - P;
      if (o >= z0) {
        a.q[base + tx + (int64_t)nx * y + plane * o] = pcast<R, C>(acc[0]);
        if (BICG) {
          const cplx<C> t = cmulc<C>(pdq[0], acc[0].a);
          sig.x += (double)t.x;
          sig.y += (double)t.y;
        }
      }
#pragma unroll
      for (int d = 0; d < 2 * P; ++d) acc[d] = acc[d + 1];
      acc[2 * P].a = mkc<C>(0, 0);
      acc[2 * P].b = mkc<C>(0, 0);
#pragma unroll
      for (int d = 0; d < P; ++d) pdq[d] = pdq[d + 1];
    }
  }

  if (BICG) {
    sig = wave_sum2(sig);
    const int lane = tid & 63, wv = tid >> 6;
    if (lane == 0) red[wv] = sig;
    __syncthreads();
    if (tid == 0) {
      double2 t = make_double2(0.0, 0.0);
      for (int w = 0; w < (nthr + 63) / 64; ++w) {
        t.x += red[w].x;
        t.y += red[w].y;
      }
      a.sig_part[(int64_t)run * a.ntiles + tile] = t;
    }
  }
}

int32_t stencil_tiles(const cbs_system* s, int32_t tile_y) { return (s->ny + tile_y - 1) / tile_y; }

int32_t default_tile_y(const cbs_system* s, int32_t bytes_per_pair) {
  int best = 1;
  double best_cost = 1e30;
  for (int ty = 1; ty <= 16 && ty <= s->ny; ++ty) {
    if (s->nx * ty > 512) break;
    const size_t lds = (size_t)(ty + 2 * s->p) * s->nx * bytes_per_pair;   // single buffer
    if (lds > 64 * 1024) break;
    const int ntile = (s->ny + ty - 1) / ty;
    double cost = (double)(ty + 2 * s->p) / ty * ((double)ntile * ty / s->ny);
    if (s->nx * ty < 128) cost *= 1.25;   // too few waves per workgroup
    if (cost <= best_cost) {
      best_cost = cost;
      best = ty;
    }
  }
  return best;
}

template <typename R, typename C, int P, bool BICG>
static int32_t launch_pc(const cbs_system* s, const StArgs<R>& a, hipStream_t st) {
  const int nthr = s->nx * a.ty;
  const size_t smem = (size_t)a.nbuf * (a.ty + 2 * P) * s->nx * sizeof(Pair<R>);
  if (smem > 64 * 1024) {
    set_error("stencil tile of %d rows x %d needs %zu bytes of LDS", a.ty, s->nx, smem);
    return CBS_EINVAL;
  }
  const int grid = (a.nlogical + 7) / 8 * 8;
  hipLaunchKernelGGL((k_stencil<R, C, P, BICG>), dim3(grid), dim3(nthr), smem, st, a);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

template <typename R, int P, bool BICG>
static int32_t launch_p(const cbs_system* s, const StArgs<R>& a, hipStream_t st) {
  if (std::is_same<R, float>::value && lo_arith_fp32()) return launch_pc<R, float, P, BICG>(s, a, st);
  return launch_pc<R, double, P, BICG>(s, a, st);
}

template <typename R>
int32_t launch_stencil(const cbs_system* s, bool bicg, const StencilLaunch& l, int32_t tile_y,
                       hipStream_t st) {
  if (l.nruns <= 0) return CBS_OK;
  StArgs<R> a;
  a.nx = s->nx;
  a.ny = s->ny;
  a.nz = s->nz;
  a.ty = tile_y;
  a.ntiles = stencil_tiles(s, tile_y);
  a.nbuf = ((size_t)2 * (tile_y + 2 * s->p) * s->nx * sizeof(Pair<R>) <= 64 * 1024) ? 2 : 1;
  a.nzseg = bicg ? 1 : std::max(1, std::min<int32_t>(l.zseg, s->nz));
  a.nlogical = l.nruns * a.ntiles * a.nzseg;
  a.N = s->N;
  a.kin = -0.5 / (s->h * s->h);
  for (int i = 0; i < 5; ++i) a.c[i] = s->fd[i];
  a.vloc = std::is_same<R, double>::value ? (const R*)s->vloc64 : (const R*)s->vloc32;
  a.vloc64 = s->vloc64;
  a.rin = (const Pair<R>*)l.rin;
  a.pold = (const Pair<R>*)l.pold;
  a.pnew = (Pair<R>*)l.pnew;
  a.q = (Pair<R>*)l.q;
  a.x = (Pair<R>*)l.x;
  a.coef = l.coef;
  a.beta = l.beta;
  a.xcoef = l.xcoef;
  a.status = l.status;
  a.need_status = l.need_status;
  a.sig_part = l.sig_part;
  a.list = l.list;
  a.count = l.count;
  if ((a.list == nullptr) != (a.count == nullptr)) {
    set_error("launch_stencil: a run list needs its count");
    return CBS_EINVAL;
  }
  switch (s->p) {
    case 1: return bicg ? launch_p<R, 1, true>(s, a, st) : launch_p<R, 1, false>(s, a, st);
    case 2: return bicg ? launch_p<R, 2, true>(s, a, st) : launch_p<R, 2, false>(s, a, st);
    case 3: return bicg ? launch_p<R, 3, true>(s, a, st) : launch_p<R, 3, false>(s, a, st);
    case 4: return bicg ? launch_p<R, 4, true>(s, a, st) : launch_p<R, 4, false>(s, a, st);
    default: set_error("unsupported finite-difference half-width %d", s->p); return CBS_EINVAL;
  }
}

template int32_t launch_stencil<double>(const cbs_system*, bool, const StencilLaunch&, int32_t,
                                        hipStream_t);
template int32_t launch_stencil<float>(const cbs_system*, bool, const StencilLaunch&, int32_t,
                                       hipStream_t);

}  // namespace cbs

namespace cbs {

// ------------------------------------------------------------------ tile autotuner
// Times the BiCG-mode stencil for every feasible tile height (full x rows, TY y rows,
// double-buffered LDS when it fits) on a scratch batch of runs and keeps the fastest,
// separately for complex128 and complex64.  Candidates are the heights with at most
// 512 threads per workgroup and one plane buffer within 64 KB of LDS.
template <typename R>
static int32_t tune_one(cbs_system* s, hipStream_t st, int32_t* best_ty, std::string& log) {
  const size_t per_run = (size_t)s->N * sizeof(Pair<R>);
  int nr = (int)std::min<size_t>(256, std::max<size_t>(8, ((size_t)2 << 30) / (5 * per_run)));
  Pair<R>* buf = nullptr;
  RunCoef* coef = nullptr;
  double2* sc = nullptr;
  int32_t* status = nullptr;
  double2* sig = nullptr;
  CBS_TRY(ws_get(s->ws, "tune.buf", (size_t)5 * nr * s->N, &buf));
  CBS_TRY(ws_get(s->ws, "tune.coef", (size_t)nr, &coef));
  CBS_TRY(ws_get(s->ws, "tune.sc", (size_t)2 * nr, &sc));
  CBS_TRY(ws_get(s->ws, "tune.status", (size_t)nr, &status));
  CBS_TRY(ws_get(s->ws, "tune.sig", (size_t)nr * s->ny, &sig));
  CBS_HIP(hipMemsetAsync(buf, 0, (size_t)5 * nr * per_run, st));
  CBS_HIP(hipMemsetAsync(sc, 0, (size_t)2 * nr * sizeof(double2), st));
  CBS_HIP(hipMemsetAsync(status, 0, (size_t)nr * sizeof(int32_t), st));
  std::vector<RunCoef> hc(nr);
  for (auto& c : hc) {
    c.c[0] = c.c[3] = make_double2(1, 0);
    c.c[1] = c.c[5] = make_double2(1.5, 1.0);
    c.c[2] = c.c[4] = make_double2(0.4, -0.3);
    c.E = 0.1;
  }
  CBS_HIP(hipMemcpyAsync(coef, hc.data(), nr * sizeof(RunCoef), hipMemcpyHostToDevice, st));
  hipEvent_t e0, e1;
  CBS_HIP(hipEventCreate(&e0));
  CBS_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int bty = default_tile_y(s, sizeof(Pair<R>));
  for (int ty = 1; ty <= 16 && ty <= s->ny; ++ty) {
    if (s->nx * ty > 512) break;
    if ((size_t)(ty + 2 * s->p) * s->nx * sizeof(Pair<R>) > 64 * 1024) break;
    StencilLaunch l{};
    l.nruns = nr;
    l.rin = buf;
    l.pold = buf + (size_t)nr * s->N;
    l.pnew = buf + (size_t)2 * nr * s->N;
    l.q = buf + (size_t)3 * nr * s->N;
    l.x = buf + (size_t)4 * nr * s->N;
    l.coef = coef;
    l.beta = sc;
    l.xcoef = sc + nr;
    l.status = status;
    l.need_status = 0;
    l.sig_part = sig;
    int32_t rc = launch_stencil<R>(s, true, l, ty, st);
    if (rc != CBS_OK) continue;
    CBS_HIP(hipEventRecord(e0, st));
    for (int k = 0; k < 3; ++k) CBS_TRY(launch_stencil<R>(s, true, l, ty, st));
    CBS_HIP(hipEventRecord(e1, st));
    CBS_HIP(hipEventSynchronize(e1));
    float ms = 0;
    CBS_HIP(hipEventElapsedTime(&ms, e0, e1));
    char line[96];
    snprintf(line, sizeof(line), "%s ty=%d %.4f ms; ", sizeof(R) == 8 ? "c128" : "c64", ty, ms / 3);
    log += line;
    if (ms < best) {
      best = ms;
      bty = ty;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *best_ty = bty;
  return CBS_OK;
}

// Times the full-batch projector bra: per atom for 4 or 8 waves per (atom, 16 runs) and the
// two block orders (consecutive workgroups on one XCD or spread over the XCDs), and chunked
// for 4 or 8 runs per workgroup, chunks of 256 or 512 points and table loads per lane or
// shared by quads; and (complex128 only) the residual update for 1024, 2048 and 4096 points
// per chunk.  Keeps the fastest of each.  Same scratch batch as the stencil tiles.
template <typename R>
static int32_t tune_nonlocal(cbs_system* s, hipStream_t st, bool tune_update, std::string& log) {
  const int pi = std::is_same<R, float>::value ? 1 : 0;
  const size_t per_run = (size_t)s->N * sizeof(Pair<R>);
  const int nr = (int)std::min<size_t>(256, std::max<size_t>(8, ((size_t)2 << 30) / (5 * per_run)));
  const int na = s->proj.n_atoms;
  Pair<R>* buf = nullptr;
  Pair<R>* kt = nullptr;
  RunCoef* coef = nullptr;
  double2* dsc = nullptr;
  int32_t* status = nullptr;
  double* part = nullptr;
  CBS_TRY(ws_get(s->ws, "tune.buf", (size_t)5 * nr * s->N, &buf));
  CBS_TRY(ws_get(s->ws, "tune.kt", (size_t)nr * na * 12, &kt));
  CBS_TRY(ws_get(s->ws, "tune.coef", (size_t)nr, &coef));
  CBS_TRY(ws_get(s->ws, "tune.dsc", (size_t)nr * (na + 1), &dsc));
  CBS_TRY(ws_get(s->ws, "tune.status", (size_t)nr, &status));
  CBS_TRY(ws_get(s->ws, "tune.part", (size_t)nr * ((s->N + 1023) / 1024) * 4, &part));
  CBS_HIP(hipMemsetAsync(kt, 0, (size_t)nr * na * 12 * sizeof(Pair<R>), st));
  CBS_HIP(hipMemsetAsync(dsc, 0, (size_t)nr * (na + 1) * sizeof(double2), st));
  hipEvent_t e0, e1;
  CBS_HIP(hipEventCreate(&e0));
  CBS_HIP(hipEventCreate(&e1));
  struct EvG {
    hipEvent_t a, b;
    ~EvG() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } evg{e0, e1};
  const char* tag = sizeof(R) == 8 ? "c128" : "c64";
  float best = 1e30f;
  int bnw = 4, bsp = 1;
  for (int nw : {4, 8})
    for (int sp : {1, 0}) {
      s->bra_nw[pi] = nw;
      s->bra_spread[pi] = sp;
      CBS_TRY(launch_bra<R>(s, nr, buf, coef, status, 0, kt, dsc + nr, st, true));
      CBS_HIP(hipEventRecord(e0, st));
      for (int k = 0; k < 3; ++k) CBS_TRY(launch_bra<R>(s, nr, buf, coef, status, 0, kt, dsc + nr, st, true));
      CBS_HIP(hipEventRecord(e1, st));
      CBS_HIP(hipEventSynchronize(e1));
      float ms = 0;
      CBS_HIP(hipEventElapsedTime(&ms, e0, e1));
      char line[96];
      snprintf(line, sizeof(line), "%s bra nw=%d spread=%d %.4f ms; ", tag, nw, sp, ms / 3);
      log += line;
      if (ms < best) {
        best = ms;
        bnw = nw;
        bsp = sp;
      }
    }
  s->bra_nw[pi] = bnw;
  s->bra_spread[pi] = bsp;
  // the chunked bra with 4 or 8 runs per workgroup, for each chunk length and table-load mode
  int btile = 0, btp = 1, bqx = 0;
  const size_t bpart_bytes = bra_tile_part_bytes(s, nr);
  if (bpart_bytes > 0) {
    unsigned char* bpart = nullptr;
    CBS_TRY(ws_get(s->ws, "tune.bpart", bpart_bytes, &bpart));
    for (int ti = 0; ti < 2; ++ti) {
      if (s->proj.bt[ti].nslots == 0) continue;
      s->bra_tp[pi] = ti;
      for (int rg : {4, 8})
        for (int qx : {0, 1}) {
          s->bra_tile[pi] = rg;
          s->bra_qx[pi] = qx;
          CBS_TRY(launch_bra<R>(s, nr, buf, coef, status, 0, kt, dsc + nr, st, true, nullptr, nullptr, false, bpart));
          CBS_HIP(hipEventRecord(e0, st));
          for (int k = 0; k < 3; ++k)
            CBS_TRY(launch_bra<R>(s, nr, buf, coef, status, 0, kt, dsc + nr, st, true, nullptr, nullptr, false, bpart));
          CBS_HIP(hipEventRecord(e1, st));
          CBS_HIP(hipEventSynchronize(e1));
          float ms = 0;
          CBS_HIP(hipEventElapsedTime(&ms, e0, e1));
          char line[128];
          snprintf(line, sizeof(line), "%s chunked bra %d runs x %d points qx %d %.4f ms; ", tag, rg, BT_TPS[ti],
                   qx, ms / 3);
          log += line;
          if (ms < best) {
            best = ms;
            btile = rg;
            btp = ti;
            bqx = qx;
          }
        }
    }
  }
  s->bra_tile[pi] = btile;
  s->bra_tp[pi] = btp;
  s->bra_qx[pi] = bqx;
  if (tune_update) {
    best = 1e30f;
    int bpts = 2048;
    for (int pts : {1024, 2048, 4096}) {
      s->upd_pts = pts;
      const int nch = update_chunks(s);
      CBS_TRY(launch_update<R>(s, nr, buf, buf + (size_t)nr * s->N, kt, dsc, status, 0, part, nch, st));
      CBS_HIP(hipEventRecord(e0, st));
      for (int k = 0; k < 3; ++k)
        CBS_TRY(launch_update<R>(s, nr, buf, buf + (size_t)nr * s->N, kt, dsc, status, 0, part, nch, st));
      CBS_HIP(hipEventRecord(e1, st));
      CBS_HIP(hipEventSynchronize(e1));
      float ms = 0;
      CBS_HIP(hipEventElapsedTime(&ms, e0, e1));
      char line[96];
      snprintf(line, sizeof(line), "%s update %d pts/chunk %.4f ms; ", tag, pts, ms / 3);
      log += line;
      if (ms < best) {
        best = ms;
        bpts = pts;
      }
    }
    s->upd_pts = bpts;
  }
  return CBS_OK;
}

// CBS_BRA_TILE=<runs>[:<points>[:<qx>]] fixes the full-batch bra after tuning: runs 0 = per
// atom, 4 or 8 = chunked with that many runs per workgroup, on chunks of 256 or 512 points
// (default 512), with table loads per lane (qx 0, the default) or shared by quads (1, see
// k_bra_tile); CBS_BRA_NW (4 or 8) and CBS_BRA_SPREAD (0 or 1) fix the per-atom bra's
// waves and workgroup order.
static int32_t bra_override(cbs_system* s) {
  if (const char* w = getenv("CBS_BRA_NW")) s->bra_nw[0] = s->bra_nw[1] = atoi(w) == 8 ? 8 : 4;
  if (const char* w = getenv("CBS_BRA_SPREAD")) s->bra_spread[0] = s->bra_spread[1] = atoi(w) != 0;
  const char* e = getenv("CBS_BRA_TILE");
  if (e == nullptr || e[0] == 0) return CBS_OK;
  const int rg = atoi(e);
  const char* colon = strchr(e, ':');
  const int tp = colon ? atoi(colon + 1) : 512;
  const char* colon2 = colon ? strchr(colon + 1, ':') : nullptr;
  const int qx = colon2 ? atoi(colon2 + 1) : 0;
  if ((rg != 0 && rg != 4 && rg != 8) || (tp != 256 && tp != 512) || qx < 0 || qx > 1) {
    set_error("CBS_BRA_TILE=%s: expected 0, 4 or 8 runs, optionally :256 or :512 points and :0 or :1", e);
    return CBS_EINVAL;
  }
  const int ti = tp == 256 ? 0 : 1;
  if (rg > 0 && s->proj.bt[ti].nslots == 0) return CBS_OK;   // no chunked tables for this cell
  s->bra_tile[0] = s->bra_tile[1] = rg;
  s->bra_tp[0] = s->bra_tp[1] = ti;
  s->bra_qx[0] = s->bra_qx[1] = qx;
  return CBS_OK;
}

int32_t autotune_tiles(cbs_system* s, hipStream_t st) {
  if (s->tuned) return CBS_OK;
  const char* e = getenv("CBS_AUTOTUNE");
  if (e && e[0] == '0') {
    CBS_TRY(bra_override(s));
    s->tuned = 1;
    return CBS_OK;
  }
  std::string log;
  CBS_TRY(tune_one<double>(s, st, &s->tile_y[0], log));
  CBS_TRY(tune_one<float>(s, st, &s->tile_y[1], log));
  if (s->proj.n_atoms > 0) {
    CBS_TRY(tune_nonlocal<double>(s, st, true, log));
    CBS_TRY(tune_nonlocal<float>(s, st, false, log));
  }
  CBS_HIP(hipStreamSynchronize(st));
  for (const char* n : {"tune.buf", "tune.coef", "tune.sc", "tune.status", "tune.sig", "tune.kt", "tune.dsc",
                        "tune.part", "tune.bpart"})
    s->ws.drop(n);
  CBS_TRY(bra_override(s));
  s->tune_log = log;
  s->tuned = 1;
  return CBS_OK;
}

}  // namespace cbs
