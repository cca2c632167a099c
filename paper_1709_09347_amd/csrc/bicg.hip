// Step 1 of the Sakurai-Sugiura method (paper Sec. 3.1, Eq. 8 and Sec. 3.2,
// Eqs. 9-11): BiCG on P(z_j) y = v for every quadrature node and right-hand side,
// whose dual recurrences solve P(z_j)^H yt = v, i.e. the inner-circle systems
// (P(z)^H = P(1/conj z)).  Every run (node, right-hand side) is a batch entry of the
// same kernel launches (the paper's top and middle layers of parallelism).
//
// Per iteration (all runs at once):
//   A   stencil: p = r + beta p_old (dual conj(beta)), q = local part of P p,
//       x += xcoef p_old, local part of sigma = pt^H q
//   bra projector coefficients of p, nonlocal part of sigma
//   S1  alpha = rho / sigma
//   B   r -= alpha (q + ket), rt -= conj(alpha) (qt + ket); rho, ||r||, ||rt||
//   S2  beta = rho_new / rho; convergence test on the recursive residuals
//   RU  reliable update (residual replacement) for the runs S2 marked: the
//       iterate is accumulated into the complex128 solution y, the true residual
//       v - P y is recomputed in complex128 and replaces r (the search direction is
//       kept, so the Krylov space is not restarted).  In the complex128 path S2 only
//       marks runs whose recursive residual met tol (a final check); in the
//       complex64 path it also marks runs whose residual fell by `ru_factor` since
//       the last replacement: that is the FP64 iterative refinement of the inner
//       single-precision solve.
//   S3  decisions on the true residual (done / continue), count of active runs.
// The iteration sequence is captured once into a HIP graph of `chunk` iterations and
// replayed until no run is active.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <vector>

#include "cbs_internal.hpp"
#include "bicg.hpp"

namespace cbs {

// ------------------------------------------------------------------ pointwise kernels
template <typename T>
__global__ void k_bicg_init(int64_t N, int32_t nruns, int32_t L, const double2* V, Pair<T>* R,
                            Pair<T>* P0, Pair<T>* P1, Pair<T>* X, Pair<double>* Y) {
  const int64_t total = N * nruns;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t run = g / N, n = g - run * N;
    const double2 v = V[(run % L) * N + n];
    Pair<T> r;
    r.a = mkc<T>((T)v.x, (T)v.y);
    r.b = r.a;
    R[g] = r;
    Pair<T> z;
    z.a = mkc<T>(0, 0);
    z.b = z.a;
    P0[g] = z;
    P1[g] = z;
    X[g] = z;
    Pair<double> zd;
    zd.a = make_double2(0, 0);
    zd.b = zd.a;
    Y[g] = zd;
  }
}

// rho = rt^H r, ||r||^2, ||rt||^2 partial sums of the initial residual
template <typename T>
__global__ void __launch_bounds__(256) k_partials(int64_t N, int32_t nchunks, int32_t nlogical,
                                                  const Pair<T>* R, double* part) {
  __shared__ double red[4][4];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  if (lb >= nlogical) return;
  const int run = lb / nchunks, ch = lb - run * nchunks;
  const int64_t chunk = (N + nchunks - 1) / nchunks;
  const int64_t lo = ch * chunk, hi = std::min<int64_t>(lo + chunk, N);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double s[4] = {0, 0, 0, 0};
  for (int64_t n = lo + tid; n < hi; n += 256) {
    const Pair<T> r = R[(int64_t)run * N + n];
    const cplx<T> rho = cmulc<T>(r.b, r.a);
    s[0] += (double)rho.x;
    s[1] += (double)rho.y;
    s[2] += (double)cabs2<T>(r.a);
    s[3] += (double)cabs2<T>(r.b);
  }
  for (int k = 0; k < 4; ++k) s[k] = wsum<double>(s[k]);
  if (lane == 0)
    for (int k = 0; k < 4; ++k) red[wv][k] = s[k];
  __syncthreads();
  if (tid < 4) part[((int64_t)run * nchunks + ch) * 4 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
}

// Reliable update, first half: x += xcoef p (the pending update), y += x, x = 0.
template <typename T>
__global__ void __launch_bounds__(256) k_ru_pre(int64_t N, int32_t nchunks, int32_t nlogical,
                                                const int32_t* status, const double2* xcoef,
                                                const Pair<T>* P, Pair<T>* X, Pair<double>* Y) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  if (lb >= nlogical) return;
  const int run = lb / nchunks, ch = lb - run * nchunks;
  if (status[run] != RUN_RU) return;
  const int64_t chunk = (N + nchunks - 1) / nchunks;
  const int64_t lo = ch * chunk, hi = std::min<int64_t>(lo + chunk, N);
  const double2 xc = xcoef[run];
  const cplx<T> xa = mkc<T>((T)xc.x, (T)xc.y), xb = cconj<T>(xa);
  for (int64_t n = lo + threadIdx.x; n < hi; n += 256) {
    const int64_t g = (int64_t)run * N + n;
    Pair<T> x = X[g];
    const Pair<T> p = P[g];
    x.a = cfma<T>(x.a, xa, p.a);
    x.b = cfma<T>(x.b, xb, p.b);
    Pair<double> y = Y[g];
    y.a = cadd<double>(y.a, ccast<double, T>(x.a));
    y.b = cadd<double>(y.b, ccast<double, T>(x.b));
    Y[g] = y;
    Pair<T> z;
    z.a = mkc<T>(0, 0);
    z.b = z.a;
    X[g] = z;
  }
}

// Reliable update, second half: r = v - P y in complex128 (q64 holds the local part,
// the ket adds the projectors), written back as the working residual.
template <typename T>
__global__ void __launch_bounds__(256) k_ru_post(int64_t N, int32_t nchunks, int32_t nlogical,
                                                 int32_t L, int32_t n_atoms, const int32_t* status,
                                                 const double2* V, const Pair<double>* Q64,
                                                 const Pair<double>* KT64, const int32_t* pt_off,
                                                 const int32_t* pt_key, const double* pt_u,
                                                 Pair<T>* R, double* part) {
  __shared__ double red[4][4];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  if (lb >= nlogical) return;
  const int run = lb / nchunks, ch = lb - run * nchunks;
  if (status[run] != RUN_RU) return;
  const int64_t chunk = (N + nchunks - 1) / nchunks;
  const int64_t lo = ch * chunk, hi = std::min<int64_t>(lo + chunk, N);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double2* v = V + (int64_t)(run % L) * N;
  double s[4] = {0, 0, 0, 0};
  for (int64_t n = lo + tid; n < hi; n += 256) {
    const int64_t g = (int64_t)run * N + n;
    Pair<double> q = Q64[g];
    if (n_atoms > 0) {
      const Pair<double> k = ket_at<double>(n, (int64_t)run * n_atoms * 12, pt_off, pt_key, pt_u, KT64);
      q.a = cadd<double>(q.a, k.a);
      q.b = cadd<double>(q.b, k.b);
    }
    const double2 vv = v[n];
    const double2 ra = csub<double>(vv, q.a), rb = csub<double>(vv, q.b);
    Pair<T> r;
    r.a = ccast<T, double>(ra);
    r.b = ccast<T, double>(rb);
    R[g] = r;
    const cplx<T> rho = cmulc<T>(r.b, r.a);
    s[0] += (double)rho.x;
    s[1] += (double)rho.y;
    s[2] += cabs2<double>(ra);
    s[3] += cabs2<double>(rb);
  }
  for (int k = 0; k < 4; ++k) s[k] = wsum<double>(s[k]);
  if (lane == 0)
    for (int k = 0; k < 4; ++k) red[wv][k] = s[k];
  __syncthreads();
  if (tid < 4) part[((int64_t)run * nchunks + ch) * 4 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
}

// ------------------------------------------------------------------ scalar kernels
__device__ __forceinline__ bool finite2(double2 v) { return isfinite(v.x) && isfinite(v.y); }

__device__ __forceinline__ void sum_part(const double* part, int64_t off, int n, double* s) {
  s[0] = s[1] = s[2] = s[3] = 0;
  for (int c = 0; c < n; ++c)
    for (int k = 0; k < 4; ++k) s[k] += part[(off + c) * 4 + k];
}

__global__ void __launch_bounds__(256) k_s0(BicgScal sc, int32_t nruns, int32_t nchunks,
                                            const double* part, double ru_factor) {
  for (int run = threadIdx.x; run < nruns; run += blockDim.x) {
    double s[4];
    sum_part(part, (int64_t)run * nchunks, nchunks, s);
    sc.rho[run] = make_double2(s[0], s[1]);
    sc.rho_prev[run] = make_double2(s[0], s[1]);
    sc.vn2[run] = s[2];
    sc.beta[run] = make_double2(0, 0);
    sc.alpha[run] = make_double2(0, 0);
    sc.xcoef[run] = make_double2(0, 0);
    sc.iters[run] = 0;
    sc.nru[run] = 0;
    sc.brk[run] = 0;
    sc.halt[run] = 0;
    sc.ru_thr[run] = ru_factor;
    sc.relres[2 * run] = 1.0;
    sc.relres[2 * run + 1] = 1.0;
    sc.status[run] = (s[2] > 0) ? RUN_ACTIVE : RUN_DONE;
    if (s[2] <= 0) {
      sc.relres[2 * run] = 0;
      sc.relres[2 * run + 1] = 0;
    }
  }
}

__global__ void __launch_bounds__(256) k_s1(BicgScal sc, int32_t nruns, int32_t ntiles, int32_t n_atoms,
                                            const double2* sig_part, const double2* signl) {
  for (int run = threadIdx.x; run < nruns; run += blockDim.x) {
    if (sc.status[run] != RUN_ACTIVE) continue;
    double2 sg = make_double2(0, 0);
    for (int t = 0; t < ntiles; ++t) {
      const double2 v = sig_part[(int64_t)run * ntiles + t];
      sg.x += v.x;
      sg.y += v.y;
    }
    for (int a = 0; a < n_atoms; ++a) {
      const double2 v = signl[(int64_t)run * n_atoms + a];
      sg.x += v.x;
      sg.y += v.y;
    }
    if (!(sg.x != 0.0 || sg.y != 0.0) || !finite2(sg)) {
      sc.brk[run] = 1;
      sc.status[run] = RUN_RU;
      sc.alpha[run] = make_double2(0, 0);
      sc.xcoef[run] = make_double2(0, 0);
      continue;
    }
    const double2 al = cdiv<double>(sc.rho[run], sg);
    sc.alpha[run] = al;
    sc.xcoef[run] = al;
  }
}

__global__ void __launch_bounds__(256) k_s2(BicgScal sc, int32_t nruns, int32_t nchunks, const double* part,
                                            double tol, int32_t max_iter) {
  for (int run = threadIdx.x; run < nruns; run += blockDim.x) {
    if (sc.status[run] != RUN_ACTIVE) continue;
    double s[4];
    sum_part(part, (int64_t)run * nchunks, nchunks, s);
    const int it = sc.iters[run] + 1;
    sc.iters[run] = it;
    const double vn = sc.vn2[run];
    const double rr = sqrt(s[2] / vn), rrt = sqrt(s[3] / vn);
    sc.relres[2 * run] = rr;
    sc.relres[2 * run + 1] = rrt;
    const double2 rn = make_double2(s[0], s[1]);
    const double2 ro = sc.rho[run];
    const bool conv = (rr < tol) && (rrt < tol);
    const bool bad = !(rn.x != 0.0 || rn.y != 0.0) || !finite2(rn) || !isfinite(rr) || !isfinite(rrt);
    if (bad && !conv) sc.brk[run] = 1;
    sc.beta[run] = bad ? make_double2(0, 0) : cdiv<double>(rn, ro);
    sc.rho_prev[run] = ro;
    sc.rho[run] = rn;
    if (conv || bad || it >= max_iter || fmax(rr, rrt) < sc.ru_thr[run]) sc.status[run] = RUN_RU;
  }
}

__global__ void __launch_bounds__(256) k_s3(BicgScal sc, int32_t nruns, int32_t nchunks, const double* part,
                                            double tol, int32_t max_iter, int32_t max_ru,
                                            double ru_factor) {
  __shared__ int cnt[4];
  int active = 0;
  for (int run = threadIdx.x; run < nruns; run += blockDim.x) {
    int st = sc.status[run];
    if (st == RUN_RU) {
      double s[4];
      sum_part(part, (int64_t)run * nchunks, nchunks, s);
      const double vn = sc.vn2[run];
      const double rr = sqrt(s[2] / vn), rrt = sqrt(s[3] / vn);
      sc.relres[2 * run] = rr;
      sc.relres[2 * run + 1] = rrt;
      const int nru = sc.nru[run] + 1;
      sc.nru[run] = nru;
      sc.xcoef[run] = make_double2(0, 0);
      const double2 rn = make_double2(s[0], s[1]);
      if (rr < tol && rrt < tol) {
        st = RUN_DONE;
      } else if (sc.brk[run] || !finite2(rn) || !(rn.x != 0.0 || rn.y != 0.0)) {
        st = RUN_BREAKDOWN;
      } else if (sc.halt[run]) {
        st = RUN_HALTED;
      } else if (sc.iters[run] >= max_iter || nru >= max_ru) {
        st = RUN_NOCONV;
      } else {
        st = RUN_ACTIVE;
        sc.beta[run] = cdiv<double>(rn, sc.rho_prev[run]);
        sc.rho[run] = rn;
        sc.ru_thr[run] = fmax(rr, rrt) * ru_factor;
      }
      sc.status[run] = st;
    }
    active += (st == RUN_ACTIVE) ? 1 : 0;
  }
  active = (int)wsum<double>((double)active);
  if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = active;
  __syncthreads();
  if (threadIdx.x == 0) sc.n_active[0] = cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

// Half-of-the-nodes rule (paper Sec. 3.3): within every group of n_q*L runs, once
// more than half of the nodes have all their right-hand sides converged, the
// remaining runs stop.  Stopped runs still get their iterate accumulated (marked
// for a last reliable update with an exhausted budget).
__global__ void __launch_bounds__(256) k_half_stop(BicgScal sc, int32_t ngroups, int32_t n_q, int32_t L) {
  for (int g = threadIdx.x; g < ngroups; g += blockDim.x) {
    int done_nodes = 0;
    for (int j = 0; j < n_q; ++j) {
      bool all = true;
      for (int l = 0; l < L; ++l) all = all && (sc.status[(g * n_q + j) * L + l] == RUN_DONE);
      done_nodes += all ? 1 : 0;
    }
    if (2 * done_nodes > n_q) {
      for (int r = g * n_q * L; r < (g + 1) * n_q * L; ++r) {
        if (sc.status[r] == RUN_ACTIVE) {
          sc.status[r] = RUN_RU;
          sc.halt[r] = 1;
        }
      }
    }
  }
}

__global__ void k_mark_halted(BicgScal sc, int32_t nruns) {
  for (int run = threadIdx.x; run < nruns; run += blockDim.x)
    if (sc.halt[run] && sc.status[run] != RUN_DONE) sc.status[run] = RUN_HALTED;
}

// ------------------------------------------------------------------ host driver
static int32_t grid8(int64_t nlogical) { return (int32_t)((nlogical + 7) / 8 * 8); }

template <typename T>
int32_t bicg_alloc(BicgBatch<T>& b) {
  cbs_system* s = b.sys;
  Workspace& ws = s->ws;
  const size_t nv = (size_t)b.nruns * s->N;
  const bool f32 = std::is_same<T, float>::value;
  const char* pre = f32 ? "b32." : "b64.";
  std::string k = pre;
  CBS_TRY(ws_get(ws, (k + "R").c_str(), nv, &b.R));
  CBS_TRY(ws_get(ws, (k + "P0").c_str(), nv, &b.Pb[0]));
  CBS_TRY(ws_get(ws, (k + "P1").c_str(), nv, &b.Pb[1]));
  CBS_TRY(ws_get(ws, (k + "Q").c_str(), nv, &b.Q));
  CBS_TRY(ws_get(ws, (k + "X").c_str(), nv, &b.X));
  CBS_TRY(ws_get(ws, "bicg.Y", nv, &b.Y));
  const int na = s->proj.n_atoms;
  if (na > 0) CBS_TRY(ws_get(ws, (k + "KT").c_str(), (size_t)b.nruns * na * 12, &b.KT));
  if (f32) {
    CBS_TRY(ws_get(ws, "b32.Q64", nv, &b.Q64));
    if (na > 0) CBS_TRY(ws_get(ws, "b32.KT64", (size_t)b.nruns * na * 12, &b.KT64));
  } else {
    b.Q64 = reinterpret_cast<Pair<double>*>(b.Q);
    b.KT64 = reinterpret_cast<Pair<double>*>(b.KT);
  }
  b.tile_y = s->tile_y[f32 ? 1 : 0];
  b.ntiles = stencil_tiles(s, b.tile_y);
  b.nchunks = update_chunks(s);
  CBS_TRY(ws_get(ws, "bicg.sig", (size_t)b.nruns * b.ntiles, &b.sig_part));
  CBS_TRY(ws_get(ws, "bicg.signl", (size_t)b.nruns * std::max(na, 1), &b.signl));
  CBS_TRY(ws_get(ws, "bicg.upd", (size_t)b.nruns * b.nchunks * 4, &b.upd_part));
  CBS_TRY(ws_get(ws, "bicg.ru", (size_t)b.nruns * b.nchunks * 4, &b.ru_part));
  const size_t R = b.nruns;
  CBS_TRY(ws_get(ws, "sc.alpha", R, &b.sc.alpha));
  CBS_TRY(ws_get(ws, "sc.xcoef", R, &b.sc.xcoef));
  CBS_TRY(ws_get(ws, "sc.beta", R, &b.sc.beta));
  CBS_TRY(ws_get(ws, "sc.rho", R, &b.sc.rho));
  CBS_TRY(ws_get(ws, "sc.rhop", R, &b.sc.rho_prev));
  CBS_TRY(ws_get(ws, "sc.vn2", R, &b.sc.vn2));
  CBS_TRY(ws_get(ws, "sc.relres", 2 * R, &b.sc.relres));
  CBS_TRY(ws_get(ws, "sc.ruthr", R, &b.sc.ru_thr));
  CBS_TRY(ws_get(ws, "sc.status", R, &b.sc.status));
  CBS_TRY(ws_get(ws, "sc.iters", R, &b.sc.iters));
  CBS_TRY(ws_get(ws, "sc.brk", R, &b.sc.brk));
  CBS_TRY(ws_get(ws, "sc.halt", R, &b.sc.halt));
  CBS_TRY(ws_get(ws, "sc.nru", R, &b.sc.nru));
  CBS_TRY(ws_get(ws, "sc.nact", 1, &b.sc.n_active));
  return CBS_OK;
}

template <typename T>
int32_t bicg_enqueue_init(BicgBatch<T>& b, hipStream_t st) {
  cbs_system* s = b.sys;
  const int64_t total = (int64_t)b.nruns * s->N;
  const int g = (int)std::min<int64_t>((total + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_bicg_init<T>, dim3(g), dim3(256), 0, st, s->N, b.nruns, b.L, b.V, b.R, b.Pb[0],
                     b.Pb[1], b.X, b.Y);
  CBS_HIP(hipGetLastError());
  const int nl = b.nruns * b.nchunks;
  hipLaunchKernelGGL(k_partials<T>, dim3(grid8(nl)), dim3(256), 0, st, s->N, b.nchunks, nl,
                     (const Pair<T>*)b.R, b.upd_part);
  CBS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_s0, dim3(1), dim3(256), 0, st, b.sc, b.nruns, b.nchunks, (const double*)b.upd_part,
                     b.ru_factor);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

template <typename T>
int32_t bicg_enqueue_iter(BicgBatch<T>& b, int parity, hipStream_t st) {
  cbs_system* s = b.sys;
  Pair<T>* pnew = b.Pb[parity & 1];
  Pair<T>* pold = b.Pb[(parity + 1) & 1];
  StencilLaunch l{};
  l.nruns = b.nruns;
  l.rin = b.R;
  l.pold = pold;
  l.pnew = pnew;
  l.q = b.Q;
  l.x = b.X;
  l.coef = b.coef;
  l.beta = b.sc.beta;
  l.xcoef = b.sc.xcoef;
  l.status = b.sc.status;
  l.need_status = RUN_ACTIVE;
  l.sig_part = b.sig_part;
  if (b.pev0) CBS_HIP(hipEventRecord(b.pev0, st));
  CBS_TRY(launch_stencil<T>(s, true, l, b.tile_y, st));
  if (b.pev1) CBS_HIP(hipEventRecord(b.pev1, st));
  const int na = s->proj.n_atoms;
  if (na > 0) CBS_TRY(launch_bra<T>(s, b.nruns, pnew, b.coef, b.sc.status, RUN_ACTIVE, b.KT, b.signl, st));
  hipLaunchKernelGGL(k_s1, dim3(1), dim3(256), 0, st, b.sc, b.nruns, b.ntiles, na,
                     (const double2*)b.sig_part, (const double2*)b.signl);
  CBS_HIP(hipGetLastError());
  CBS_TRY(launch_update<T>(s, b.nruns, b.R, b.Q, b.KT, b.sc.alpha, b.sc.status, b.upd_part, b.nchunks, st));
  hipLaunchKernelGGL(k_s2, dim3(1), dim3(256), 0, st, b.sc, b.nruns, b.nchunks, (const double*)b.upd_part,
                     b.tol, b.max_iter);
  CBS_HIP(hipGetLastError());
  if (b.half_stop && b.n_q > 0) {
    hipLaunchKernelGGL(k_half_stop, dim3(1), dim3(256), 0, st, b.sc, b.nruns / (b.n_q * b.L), b.n_q, b.L);
    CBS_HIP(hipGetLastError());
  }
  // reliable update of the marked runs
  const int nl = b.nruns * b.nchunks;
  hipLaunchKernelGGL(k_ru_pre<T>, dim3(grid8(nl)), dim3(256), 0, st, s->N, b.nchunks, nl,
                     (const int32_t*)b.sc.status, (const double2*)b.sc.xcoef, (const Pair<T>*)pnew, b.X, b.Y);
  CBS_HIP(hipGetLastError());
  StencilLaunch r{};
  r.nruns = b.nruns;
  r.rin = b.Y;
  r.q = b.Q64;
  r.coef = b.coef;
  r.status = b.sc.status;
  r.need_status = RUN_RU;
  CBS_TRY(launch_stencil<double>(s, false, r, s->tile_y[0], st));
  if (na > 0) CBS_TRY(launch_bra<double>(s, b.nruns, b.Y, b.coef, b.sc.status, RUN_RU, b.KT64, nullptr, st));
  hipLaunchKernelGGL(k_ru_post<T>, dim3(grid8(nl)), dim3(256), 0, st, s->N, b.nchunks, nl, b.L, na,
                     (const int32_t*)b.sc.status, b.V, (const Pair<double>*)b.Q64,
                     (const Pair<double>*)b.KT64, s->proj.pt_off, s->proj.pt_key,
                     (const double*)s->proj.pt_u64, b.R, b.ru_part);
  CBS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_s3, dim3(1), dim3(256), 0, st, b.sc, b.nruns, b.nchunks, (const double*)b.ru_part,
                     b.tol, b.max_iter, b.max_ru, b.ru_factor);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

static bool use_graphs() {
  const char* e = getenv("CBS_NO_GRAPH");
  return !(e && e[0] == '1');
}

// Runs the whole iteration on an internal stream ordered after `user` and before
// its return point.  Several batches (systems) advance in the same graph.
// Profile mode: iterations are launched one by one (no graph); every stencil launch of
// every batch is bracketed by events on the stream it runs on, and the active-run count
// is read back after each iteration to account the launch's algorithmic bytes.
template <typename T>
static int32_t bicg_run_profiled(std::vector<BicgBatch<T>*>& batches, hipStream_t st, int32_t max_iter) {
  std::vector<int32_t> active(batches.size());
  for (size_t i = 0; i < batches.size(); ++i) {
    active[i] = batches[i]->nruns;
    CBS_HIP(hipEventCreate(&batches[i]->pev0));
    CBS_HIP(hipEventCreate(&batches[i]->pev1));
  }
  int32_t rc = CBS_OK;
  for (int it = 0; it <= max_iter + 1 && rc == CBS_OK; ++it) {
    int any = 0;
    for (size_t i = 0; i < batches.size() && rc == CBS_OK; ++i) {
      BicgBatch<T>& b = *batches[i];
      if (active[i] == 0) continue;
      rc = bicg_enqueue_iter<T>(b, it, st);
      if (rc != CBS_OK) break;
      int32_t na = 0;
      CBS_HIP(hipMemcpyAsync(&na, b.sc.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      CBS_HIP(hipStreamSynchronize(st));
      float ms = 0;
      CBS_HIP(hipEventElapsedTime(&ms, b.pev0, b.pev1));
      const double passes = (it == 0) ? 4.0 : 6.0;
      b.prof_ms += ms;
      b.prof_launches += 1;
      b.prof_bytes += (double)active[i] * passes * b.sys->N * sizeof(Pair<T>) + (double)b.sys->N * sizeof(T);
      active[i] = na;
      any += na;
    }
    if (any == 0) break;
  }
  for (auto* b : batches) {
    (void)hipEventDestroy(b->pev0);
    (void)hipEventDestroy(b->pev1);
    b->pev0 = b->pev1 = nullptr;
  }
  return rc;
}

template <typename T>
int32_t bicg_run(std::vector<BicgBatch<T>*>& batches, hipStream_t user, int32_t chunk, int32_t max_iter,
                 double* elapsed_ms, bool profile) {
  if (batches.empty()) return CBS_OK;
  if (chunk < 2) chunk = 2;
  if (chunk % 2) chunk += 1;
  hipStream_t st = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  CBS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  struct Guard {
    hipStream_t& s;
    hipEvent_t& a;
    hipEvent_t& b;
    ~Guard() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      if (s) (void)hipStreamDestroy(s);
    }
  } guard{st, ev0, ev1};
  CBS_HIP(hipEventCreate(&ev0));
  CBS_HIP(hipEventCreate(&ev1));
  CBS_HIP(hipEventRecord(ev0, user));
  CBS_HIP(hipStreamWaitEvent(st, ev0, 0));
  for (auto* b : batches) CBS_TRY(bicg_enqueue_init<T>(*b, st));
  int32_t* hact = nullptr;
  CBS_HIP(hipHostMalloc(&hact, sizeof(int32_t) * batches.size(), hipHostMallocDefault));
  struct HGuard {
    int32_t* p;
    ~HGuard() {
      if (p) (void)hipHostFree(p);
    }
  } hg{hact};

  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  const bool graphs = use_graphs() && !profile;
  if (graphs) {
    CBS_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
    int32_t rc = CBS_OK;
    for (int k = 0; k < chunk && rc == CBS_OK; ++k)
      for (auto* b : batches)
        if (rc == CBS_OK) rc = bicg_enqueue_iter<T>(*b, k, st);
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc != CBS_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    CBS_HIP(e);
    CBS_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  auto t0 = std::chrono::steady_clock::now();
  int32_t rc = CBS_OK;
  const int max_chunks = profile ? 0 : (max_iter + 2) / chunk + 2;
  if (profile) rc = bicg_run_profiled<T>(batches, st, max_iter);
  for (int c = 0; c < max_chunks; ++c) {
    if (graphs) {
      if (hipGraphLaunch(exec, st) != hipSuccess) {
        set_error("hipGraphLaunch failed");
        rc = CBS_EHIP;
        break;
      }
    } else {
      for (int k = 0; k < chunk && rc == CBS_OK; ++k)
        for (auto* b : batches)
          if (rc == CBS_OK) rc = bicg_enqueue_iter<T>(*b, k, st);
      if (rc != CBS_OK) break;
    }
    for (size_t i = 0; i < batches.size(); ++i)
      if (hipMemcpyAsync(hact + i, batches[i]->sc.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, st) !=
          hipSuccess) {
        rc = CBS_EHIP;
        set_error("copy of the active-run count failed");
      }
    if (rc != CBS_OK) break;
    if (hipStreamSynchronize(st) != hipSuccess) {
      set_error("BiCG iteration failed: %s", hipGetErrorString(hipGetLastError()));
      rc = CBS_EHIP;
      break;
    }
    int any = 0;
    for (size_t i = 0; i < batches.size(); ++i) any += hact[i];
    if (any == 0) break;
  }
  if (rc == CBS_OK) {
    for (auto* b : batches) {
      if (b->half_stop) {
        hipLaunchKernelGGL(k_mark_halted, dim3(1), dim3(256), 0, st, b->sc, b->nruns);
        CBS_HIP(hipGetLastError());
      }
    }
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  CBS_HIP(hipStreamSynchronize(st));
  auto t1 = std::chrono::steady_clock::now();
  if (elapsed_ms) *elapsed_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  CBS_HIP(hipEventRecord(ev1, st));
  CBS_HIP(hipStreamWaitEvent(user, ev1, 0));
  return rc;
}

// Summaries copied to the host after a run.
template <typename T>
int32_t bicg_collect(BicgBatch<T>& b, std::vector<int32_t>& iters, std::vector<double>& relres,
                     std::vector<int32_t>& status, hipStream_t st) {
  iters.resize(b.nruns);
  relres.resize(2 * (size_t)b.nruns);
  status.resize(b.nruns);
  CBS_HIP(hipMemcpyAsync(iters.data(), b.sc.iters, b.nruns * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CBS_HIP(hipMemcpyAsync(relres.data(), b.sc.relres, 2 * b.nruns * sizeof(double), hipMemcpyDeviceToHost, st));
  CBS_HIP(hipMemcpyAsync(status.data(), b.sc.status, b.nruns * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CBS_HIP(hipStreamSynchronize(st));
  return CBS_OK;
}

template int32_t bicg_alloc<double>(BicgBatch<double>&);
template int32_t bicg_alloc<float>(BicgBatch<float>&);
template int32_t bicg_run<double>(std::vector<BicgBatch<double>*>&, hipStream_t, int32_t, int32_t, double*, bool);
template int32_t bicg_run<float>(std::vector<BicgBatch<float>*>&, hipStream_t, int32_t, int32_t, double*, bool);
template int32_t bicg_collect<double>(BicgBatch<double>&, std::vector<int32_t>&, std::vector<double>&,
                                      std::vector<int32_t>&, hipStream_t);
template int32_t bicg_collect<float>(BicgBatch<float>&, std::vector<int32_t>&, std::vector<double>&,
                                     std::vector<int32_t>&, hipStream_t);

// ------------------------------------------------------------------ node coefficients
void node_coefs(const double2* z, int32_t n_z, int32_t L, double E, std::vector<RunCoef>& out) {
  out.resize((size_t)n_z * L);
  for (int j = 0; j < n_z; ++j) {
    const double zr = z[j].x, zi = z[j].y, d = zr * zr + zi * zi;
    RunCoef c{};
    // primal P(z): (1, z, 1/z); dual P(z)^H = P(1/conj z): (1, 1/conj z, conj z)
    c.c[0] = make_double2(1, 0);
    c.c[1] = make_double2(zr, zi);
    c.c[2] = make_double2(zr / d, -zi / d);
    c.c[3] = make_double2(1, 0);
    c.c[4] = make_double2(zr / d, zi / d);
    c.c[5] = make_double2(zr, -zi);
    c.E = E;
    for (int l = 0; l < L; ++l) out[(size_t)j * L + l] = c;
  }
}

__global__ void k_split_pairs(int64_t N, int32_t nruns, const Pair<double>* Y, double2* ya, double2* yb) {
  const int64_t total = N * nruns;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const Pair<double> v = Y[g];
    ya[g] = v.a;
    yb[g] = v.b;
  }
}

int32_t split_pairs(int64_t N, int32_t nruns, const Pair<double>* Y, double2* ya, double2* yb, hipStream_t st) {
  const int64_t total = N * nruns;
  if (total == 0) return CBS_OK;
  const int g = (int)std::min<int64_t>((total + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_split_pairs, dim3(g), dim3(256), 0, st, N, nruns, Y, ya, yb);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

// Complete step-1 solve of one system at one energy, shared by cbs_bicg and cbs_solve.
int32_t solve_nodes(cbs_system* s, double E, const double2* z, int32_t n_z, int32_t L, const double2* V,
                    const cbs_params* prm, hipStream_t st, NodeSolve& out) {
  std::vector<RunCoef> hc;
  node_coefs(z, n_z, L, E, hc);
  RunCoef* coef = nullptr;
  const int32_t nruns = n_z * L;
  CBS_TRY(ws_get(s->ws, "bicg.coef", (size_t)nruns, &coef));
  CBS_HIP(hipMemcpyAsync(coef, hc.data(), nruns * sizeof(RunCoef), hipMemcpyHostToDevice, st));
  const bool mixed = prm->precision == CBS_MIXED;
  const int32_t max_ru = mixed ? std::max(prm->max_refine, 1) : 1 << 30;
  int32_t rc = CBS_OK;
  if (mixed) {
    BicgBatch<float> b{};
    b.sys = s;
    b.nruns = nruns;
    b.L = L;
    b.n_q = n_z;
    b.V = V;
    b.coef = coef;
    b.tol = prm->tol;
    b.ru_factor = prm->inner_tol;
    b.max_iter = prm->max_iter;
    b.max_ru = max_ru;
    b.half_stop = prm->half_stop;
    CBS_TRY(bicg_alloc<float>(b));
    std::vector<BicgBatch<float>*> v{&b};
    rc = bicg_run<float>(v, st, prm->chunk, prm->max_iter, &out.ms, prm->profile != 0);
    if (rc != CBS_OK) return rc;
    CBS_TRY(bicg_collect<float>(b, out.iters, out.relres, out.status, st));
    out.Y = b.Y;
    out.prof_launches = b.prof_launches;
    out.prof_ms = b.prof_ms;
    out.prof_bytes = b.prof_bytes;
  } else {
    BicgBatch<double> b{};
    b.sys = s;
    b.nruns = nruns;
    b.L = L;
    b.n_q = n_z;
    b.V = V;
    b.coef = coef;
    b.tol = prm->tol;
    b.ru_factor = 0.0;
    b.max_iter = prm->max_iter;
    b.max_ru = max_ru;
    b.half_stop = prm->half_stop;
    CBS_TRY(bicg_alloc<double>(b));
    std::vector<BicgBatch<double>*> v{&b};
    rc = bicg_run<double>(v, st, prm->chunk, prm->max_iter, &out.ms, prm->profile != 0);
    if (rc != CBS_OK) return rc;
    CBS_TRY(bicg_collect<double>(b, out.iters, out.relres, out.status, st));
    out.Y = b.Y;
    out.prof_launches = b.prof_launches;
    out.prof_ms = b.prof_ms;
    out.prof_bytes = b.prof_bytes;
  }
  out.nruns = nruns;
  return CBS_OK;
}

int32_t check_params(const cbs_params* p, bool need_moments) {
  if (!p) {
    set_error("params is NULL");
    return CBS_EINVAL;
  }
  if (!(p->lambda_min > 0 && p->lambda_min < 1) || p->n_q < 1 || p->n_rhs < 1 || !(p->tol > 0) ||
      p->max_iter < 1 || (p->precision != CBS_FP64 && p->precision != CBS_MIXED) ||
      (p->precision == CBS_MIXED && !(p->inner_tol > 0 && p->inner_tol < 1))) {
    set_error("invalid solver parameters");
    return CBS_EINVAL;
  }
  if (need_moments) {
    if (p->n_mom < 1 || 2 * p->n_mom > p->n_q || p->n_rhs * p->n_mom > 256 || !(p->delta > 0) ||
        (p->extraction != CBS_RR && p->extraction != CBS_HANKEL)) {
      set_error("invalid moment parameters (need 2*n_mom <= n_q, n_rhs*n_mom <= 256)");
      return CBS_EINVAL;
    }
  }
  return CBS_OK;
}

}  // namespace cbs

using namespace cbs;

extern "C" int32_t cbs_bicg(cbs_system* s, double E, int32_t n_z, const double* z, int32_t n_rhs,
                            const void* V, const cbs_params* prm, void* Y, void* Yt, int32_t* iters,
                            double* relres, cbs_info* info, void* stream) {
  if (!s || n_z < 1 || !z || n_rhs < 1 || !V || !Y || !Yt) {
    set_error("cbs_bicg: bad argument");
    return CBS_EINVAL;
  }
  CBS_TRY(check_params(prm, false));
  for (int j = 0; j < n_z; ++j) {
    if (z[2 * j] == 0 && z[2 * j + 1] == 0) {
      set_error("cbs_bicg: z must be nonzero");
      return CBS_EINVAL;
    }
  }
  CBS_HIP(hipSetDevice(s->device));
  hipStream_t st = (hipStream_t)stream;
  NodeSolve ns;
  CBS_TRY(solve_nodes(s, E, (const double2*)z, n_z, n_rhs, (const double2*)V, prm, st, ns));
  CBS_TRY(split_pairs(s->N, ns.nruns, ns.Y, (double2*)Y, (double2*)Yt, st));
  CBS_HIP(hipStreamSynchronize(st));
  bool noconv = false;
  for (int r = 0; r < ns.nruns; ++r) {
    if (iters) iters[r] = ns.iters[r];
    if (relres) {
      relres[2 * r] = ns.relres[2 * r];
      relres[2 * r + 1] = ns.relres[2 * r + 1];
    }
    noconv = noconv || ns.status[r] != RUN_DONE;
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    double mx = 0, sum = 0;
    int im = 0;
    for (int r = 0; r < ns.nruns; ++r) {
      mx = std::max(mx, std::max(ns.relres[2 * r], ns.relres[2 * r + 1]));
      im = std::max(im, ns.iters[r]);
      sum += ns.iters[r];
    }
    info->iters_max = im;
    info->iters_mean = sum / ns.nruns;
    info->max_solve_resid = mx;
    info->t_solve_ms = ns.ms;
    info->matvecs = (int64_t)(2 * sum);
    info->stencil_launches = ns.prof_launches;
    info->stencil_ms = ns.prof_ms;
    info->stencil_bytes = ns.prof_bytes;
  }
  if (noconv) {
    set_error("cbs_bicg: %s", "some runs missed the tolerance");
    return CBS_ENOCONV;
  }
  return CBS_OK;
}
