// Step 1 of the Sakurai-Sugiura method (paper Sec. 3.1, Eq. 8 and Sec. 3.2, Eqs. 9-11):
// BiCG on P(z_j) y = v for every quadrature node and right-hand side, whose dual
// recurrences solve P(z_j)^H yt = v, i.e. the inner-circle systems (P(z)^H = P(1/conj z)).
// Every run (node, right-hand side, energy) is a batch entry of the same kernel launches
// (the paper's top and middle layers of parallelism become one batch dimension).
//
// Per iteration, for every precision phase that has runs:
//   A   stencil: p = r + beta p_old (dual conj(beta)), q = local part of P p,
//       x += xcoef p_old, local part of sigma = pt^H q
//   bra projector coefficients of p, nonlocal part of sigma
// then
//   S1  alpha = rho / sigma
//   B   r -= alpha (q + ket), rt -= conj(alpha) (qt + ket); rho, ||r||^2, ||rt||^2
//   S2  beta = rho_new / rho; tests on the recursive residuals
//   RU  residual replacement for the runs S2 marked (a compact list, launches shaped for
//       few runs): the iterate is accumulated into the complex128 solution y, the true
//       residual v - P y is recomputed in complex128 and replaces r; the search direction
//       is kept, so the Krylov space is not restarted.
//   S3  decisions on the true residual (done / continue / change phase), active counts.
// Precision (mixed mode) follows the relaxation of inexact Krylov methods: the error
// allowed in an operator application grows as the residual shrinks.  Every run starts
// with complex128 vectors; once its residual is below `narrow_tol` its vectors are
// rounded to complex64 and the same recurrence continues in single precision (the
// search direction is kept, so the Krylov space is not restarted).  In that phase a
// replacement is triggered whenever the recursive residual has dropped by `ru_factor`
// since the last one: the FP64 iterative refinement that keeps the gap between the
// single-precision recursive residual and the true residual below the tolerance.  A run
// whose true residual stops falling in complex64 restarts in complex128.  The complex64
// phase computes in FP32 (CBS_LO_ARITH=64: FP64 arithmetic on complex64 data).  FP64
// mode stays in the complex128 phase, where S2 only marks runs whose recursive residual
// met tol.
// The iteration is captured once into a HIP graph of `chunk` iterations and replayed
// until no run is active.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "bicg.hpp"
#include "cbs_internal.hpp"

namespace cbs {

static int32_t grid8(int64_t nlogical) { return (int32_t)((nlogical + 7) / 8 * 8); }

// ------------------------------------------------------------------ pointwise kernels
template <typename T>
__global__ void k_bicg_init(int64_t N, int32_t nruns, int32_t L, const double2* V, const double2* Vd, Pair<T>* R,
                            Pair<T>* P0, Pair<T>* P1, Pair<T>* X, Pair<double>* Y) {
  const int64_t total = N * nruns;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t run = g / N, n = g - run * N;
    const double2 v = V[(run % L) * N + n];
    const double2 vd = Vd[(run % L) * N + n];
    Pair<T> r;
    r.a = mkc<T>((T)v.x, (T)v.y);
    r.b = mkc<T>((T)vd.x, (T)vd.y);
    R[g] = r;
    Pair<T> z;
    z.a = mkc<T>(0, 0);
    z.b = z.a;
    P0[g] = z;
    P1[g] = z;
    X[g] = z;
    if (Y != nullptr) {
      Pair<double> zd;
      zd.a = make_double2(0, 0);
      zd.b = zd.a;
      Y[g] = zd;
    }
  }
}

// rho = rt^H r, ||r||^2, ||rt||^2 partial sums of the initial residual
template <typename T>
__global__ void __launch_bounds__(256) k_partials(int64_t N, int32_t nchunks, int32_t nlogical, const Pair<T>* R,
                                                  double* part) {
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

// Residual replacement, first half: x += xcoef p (the pending update), y += x, x = 0.
// The run's latest direction p is in the buffer of the iteration that marked it (ru_par);
// marked on the previous iteration, it is also copied to this iteration's buffer, the one
// the run's next stencil pass reads as p_old.  Work items: (entry of the replacement list,
// chunk of points), taken grid-stride by a bounded grid (the list is short); runs of the
// other phase are skipped.
template <typename T>
__global__ void __launch_bounds__(256) k_ru_pre(int64_t N, int32_t nchunks, int32_t nlogical, const int32_t* list,
                                                const int32_t* count, const int32_t* status, int32_t need,
                                                const double2* xcoef, const int32_t* ru_par, int32_t parity,
                                                Pair<T>* P0, Pair<T>* P1, Pair<T>* X, Pair<double>* Y) {
  const int nl = min(nlogical, *count * nchunks);
  for (int lb = blockIdx.x; lb < nl; lb += gridDim.x) {
    const int slot = lb / nchunks, ch = lb - slot * nchunks;
    const int run = list[slot];
    if (status[run] != need) continue;
    const int64_t chunk = (N + nchunks - 1) / nchunks;
    const int64_t lo = ch * chunk, hi = std::min<int64_t>(lo + chunk, N);
    const double2 xc = xcoef[run];
    const cplx<T> xa = mkc<T>((T)xc.x, (T)xc.y), xb = cconj<T>(xa);
    const int rp = ru_par[run];
    const Pair<T>* P = rp ? P1 : P0;
    Pair<T>* Pnow = (parity & 1) ? P1 : P0;
    const bool copy = rp != (parity & 1);
    for (int64_t n = lo + threadIdx.x; n < hi; n += 256) {
      const int64_t g = (int64_t)run * N + n;
      Pair<T> x = X[g];
      const Pair<T> p = P[g];
      if (copy) Pnow[g] = p;
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
}

// Residual replacement, second half: r = v - P y in complex128 (Q64 holds the local
// part; the ket of the projectors is added over the grouped table, 64-point groups with
// lane = point and the coefficients of each key read uniformly); written as the working
// residual R (precision T) and, when R64 is given, also in complex128 (needed when the
// run changes phase).  Work items: (entry of the replacement list, chunk of groups), taken
// grid-stride by a bounded grid; the chunks are fine (one 64-point group per wave), so a
// few replaced runs spread over many workgroups.
template <typename T>
__global__ void __launch_bounds__(256) k_ru_post(int64_t N, int32_t nchunks, int32_t nlogical, const int32_t* list,
                                                 const int32_t* count, int32_t L, const int32_t* rhs,
                                                 int32_t n_atoms, const int32_t* status, int32_t need, const double2* V,
                                                 const double2* Vd, const Pair<double>* Q64,
                                                 const Pair<double>* KT64, const int32_t* grp_off,
                                                 const int32_t* grp_key, const double* grp_u, Pair<T>* R,
                                                 Pair<double>* R64, double* part) {
  __shared__ double red[4][4];
  const int nl = min(nlogical, *count * nchunks);
  for (int lb = blockIdx.x; lb < nl; lb += gridDim.x) {
    const int slot = lb / nchunks, ch = lb - slot * nchunks;
    const int run = __builtin_amdgcn_readfirstlane(list[slot]);
    if (status[run] != need) continue;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l = (rhs != nullptr) ? rhs[run] : run % L;   // the run's right-hand side
    const double2* v = V + (int64_t)l * N;
    const double2* vdual = Vd + (int64_t)l * N;
    typedef const CBS_CONST_AS int32_t* cint_p;
    typedef const CBS_CONST_AS Pair<double>* ckt_p;
    const cint_p goff = (cint_p)grp_off;
    const cint_p gkey = (cint_p)grp_key;
    const int64_t ngroups = (N + KG - 1) / KG;
    const int64_t gpc = (ngroups + nchunks - 1) / nchunks;
    const int64_t g0 = ch * gpc;
    const int64_t g1 = (g0 + gpc < ngroups) ? g0 + gpc : ngroups;
    double s[4] = {0, 0, 0, 0};
    for (int64_t g = g0 + wv; g < g1; g += 4) {
      const int64_t n = g * KG + lane;
      Pair<double> k;
      k.a = make_double2(0, 0);
      k.b = k.a;
      if (n_atoms > 0) {
        const ckt_p kt = (ckt_p)KT64 + (int64_t)run * n_atoms * 12;
        const int e0 = goff[g], e1 = goff[g + 1];
        for (int e = e0; e < e1; ++e) {
          const int key = gkey[e];
          const double4 uu = reinterpret_cast<const double4*>(grp_u)[(int64_t)e * KG + lane];
          const double us[4] = {uu.x, uu.y, uu.z, uu.w};
          const ckt_p kp = kt + (int64_t)(key >> 2) * 12 + (key & 3) * 4;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const Pair<double> kk = kp[i];
            k.a = cfma_r<double>(k.a, us[i], kk.a);
            k.b = cfma_r<double>(k.b, us[i], kk.b);
          }
        }
      }
      if (n < N) {
        const int64_t gi = (int64_t)run * N + n;
        const Pair<double> q = Q64[gi];
        Pair<double> r64;
        r64.a = csub<double>(v[n], cadd<double>(q.a, k.a));
        r64.b = csub<double>(vdual[n], cadd<double>(q.b, k.b));
        Pair<T> r;
        r.a = ccast<T, double>(r64.a);
        r.b = ccast<T, double>(r64.b);
        R[gi] = r;
        if (R64 != nullptr) R64[gi] = r64;
        const cplx<T> rho = cmulc<T>(r.b, r.a);
        s[0] += (double)rho.x;
        s[1] += (double)rho.y;
        s[2] += cabs2<double>(r64.a);
        s[3] += cabs2<double>(r64.b);
      }
    }
    for (int k = 0; k < 4; ++k) s[k] = wsum<double>(s[k]);
    if (lane == 0)
      for (int k = 0; k < 4; ++k) red[wv][k] = s[k];
    __syncthreads();
    if (tid < 4) part[((int64_t)run * nchunks + ch) * 4 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();   // red is reused by the next work item
  }
}

// Phase changes decided this iteration (conv flags, cleared by the next k_s2):
//   conv == 1: the run went back to complex128 and restarts from its replaced residual;
//              the old complex128 direction is cleared (beta is 0, and a stale value must
//              not turn 0 * p into NaN);
//   conv == 2: the run entered the complex64 phase: r and the latest search direction are
//              rounded to complex64, the complex128 iterate is accumulated into y and both
//              iterates restart from zero.
__global__ void __launch_bounds__(256) k_phase(int64_t N, int32_t nchunks, int32_t nlogical, const int32_t* conv,
                                               const Pair<double>* Rhi, Pair<double>* Phi, Pair<double>* Xhi,
                                               Pair<float>* Rlo, Pair<float>* Plo, Pair<float>* Xlo,
                                               Pair<double>* Y) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  if (lb >= nlogical) return;
  const int run = lb / nchunks, ch = lb - run * nchunks;
  const int cv = conv[run];
  if (cv != 1 && cv != 2) return;
  const int64_t chunk = (N + nchunks - 1) / nchunks;
  const int64_t lo = ch * chunk, hi = std::min<int64_t>(lo + chunk, N);
  Pair<double> zd;
  zd.a = make_double2(0, 0);
  zd.b = zd.a;
  if (cv == 1) {
    for (int64_t n = lo + threadIdx.x; n < hi; n += 256) Phi[(int64_t)run * N + n] = zd;
    return;
  }
  for (int64_t n = lo + threadIdx.x; n < hi; n += 256) {
    const int64_t g = (int64_t)run * N + n;
    const Pair<double> r = Rhi[g], p = Phi[g], x = Xhi[g];
    Pair<float> rf, pf, zf;
    rf.a = ccast<float, double>(r.a);
    rf.b = ccast<float, double>(r.b);
    pf.a = ccast<float, double>(p.a);
    pf.b = ccast<float, double>(p.b);
    zf.a = mkc<float>(0, 0);
    zf.b = zf.a;
    Rlo[g] = rf;
    Plo[g] = pf;
    Xlo[g] = zf;
    Pair<double> y = Y[g];
    y.a = cadd<double>(y.a, x.a);
    y.b = cadd<double>(y.b, x.b);
    Y[g] = y;
    Xhi[g] = zd;
  }
}

// ------------------------------------------------------------------ scalar kernels
__device__ __forceinline__ bool finite2(double2 v) { return isfinite(v.x) && isfinite(v.y); }

__device__ __forceinline__ void sum_part(const double* part, int64_t off, int n, double* s) {
  s[0] = s[1] = s[2] = s[3] = 0;
  for (int c = 0; c < n; ++c)
    for (int k = 0; k < 4; ++k) s[k] += part[(off + c) * 4 + k];
}

__device__ __forceinline__ bool is_active(int st) { return st == ST_ACT_LO || st == ST_ACT_HI; }

// Compact lists of the active runs of each phase (ascending) and their counts, so the
// iteration kernels launch over full groups of active runs.  One block of 256 threads.
__device__ void build_lists(BicgScal& sc, int32_t nruns) {
  __shared__ int wcnt[2][4];
  __shared__ int base[2];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) base[0] = base[1] = 0;
  __syncthreads();
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r0 = 0; r0 < nruns; r0 += 256) {
    const int run = r0 + tid;
    const int st = (run < nruns) ? sc.status[run] : -1;
    const bool lo = st == ST_ACT_LO, hi = st == ST_ACT_HI;
    const unsigned long long mlo = __ballot(lo), mhi = __ballot(hi);
    if (lane == 0) {
      wcnt[0][wv] = __popcll(mlo);
      wcnt[1][wv] = __popcll(mhi);
    }
    __syncthreads();
    int olo = base[0], ohi = base[1];
    for (int w = 0; w < wv; ++w) {
      olo += wcnt[0][w];
      ohi += wcnt[1][w];
    }
    if (lo) sc.list[olo + __popcll(mlo & below)] = run;
    if (hi) sc.list[nruns + ohi + __popcll(mhi & below)] = run;
    __syncthreads();
    if (tid == 0) {
      base[0] += wcnt[0][0] + wcnt[0][1] + wcnt[0][2] + wcnt[0][3];
      base[1] += wcnt[1][0] + wcnt[1][1] + wcnt[1][2] + wcnt[1][3];
    }
    __syncthreads();
  }
  if (tid == 0) {
    sc.n_active[0] = base[0];
    sc.n_active[1] = base[1];
  }
}
__device__ __forceinline__ bool is_ru(int st) { return st == ST_RU_LO || st == ST_RU_HI; }

// Compact list of the runs marked for residual replacement (either phase, ascending) in
// list[2][.], count n_active[2].  One block of 256 threads.
__device__ void build_ru_list(BicgScal& sc, int32_t nruns) {
  __shared__ int wcnt[4];
  __shared__ int base;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) base = 0;
  __syncthreads();
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r0 = 0; r0 < nruns; r0 += 256) {
    const int run = r0 + tid;
    const bool ru = (run < nruns) && is_ru(sc.status[run]);
    const unsigned long long m = __ballot(ru);
    if (lane == 0) wcnt[wv] = __popcll(m);
    __syncthreads();
    int o = base;
    for (int w = 0; w < wv; ++w) o += wcnt[w];
    if (ru) sc.list[2 * (int64_t)nruns + o + __popcll(m & below)] = run;
    __syncthreads();
    if (tid == 0) base += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  if (tid == 0) sc.n_active[2] = base;
}

__global__ void __launch_bounds__(256) k_s0(BicgScal sc, int32_t nruns, int32_t nchunks, const double* part,
                                            int32_t start, const double* vref) {
  for (int run = threadIdx.x; run < nruns; run += blockDim.x) {
    double s[4];
    sum_part(part, (int64_t)run * nchunks, nchunks, s);
    sc.rho[run] = make_double2(s[0], s[1]);
    sc.rho_prev[run] = make_double2(s[0], s[1]);
    sc.vn2[run] = (vref != nullptr && vref[run] > 0) ? vref[run] : s[2];
    sc.beta[run] = make_double2(0, 0);
    sc.alpha[run] = make_double2(0, 0);
    sc.xcoef[run] = make_double2(0, 0);
    sc.iters[run] = 0;
    sc.nru[run] = 0;
    sc.brk[run] = 0;
    sc.halt[run] = 0;
    sc.conv[run] = 0;
    sc.ru_it[run] = 0;
    sc.nrestart[run] = 0;
    sc.ru_thr[run] = 0.0;
    // a zero right-hand side is solved by zero; a non-finite one is not "zero" and ends in
    // a breakdown at the first scalar test
    const bool zero = s[2] == 0.0 && s[3] == 0.0;
    const double vn = sc.vn2[run];
    sc.relres[2 * run] = zero ? 0.0 : (vn > 0 ? sqrt(s[2] / vn) : 1.0);
    sc.relres[2 * run + 1] = zero ? 0.0 : (vn > 0 ? sqrt(s[3] / vn) : 1.0);
    sc.rmin[run] = fmax(sc.relres[2 * run], sc.relres[2 * run + 1]);
    sc.status[run] = zero ? ST_DONE : start;
  }
  __syncthreads();
  build_lists(sc, nruns);
}

// One wavefront per run: the lanes add the stencil's per-tile and the bra's per-atom
// partials of sigma = pt^H q, lane 0 sets alpha.
__global__ void __launch_bounds__(256) k_s1(BicgScal sc, int32_t nruns, int32_t n_atoms, const double2* sig_lo,
                                            int32_t nt_lo, const double2* sig_hi, int32_t nt_hi,
                                            const double2* signl, int32_t parity) {
  const int lane = threadIdx.x & 63;
  const int run = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (run >= nruns) return;
  const int st = sc.status[run];
  if (!is_active(st)) return;
  const double2* sp = (st == ST_ACT_LO) ? sig_lo : sig_hi;
  const int nt = (st == ST_ACT_LO) ? nt_lo : nt_hi;
  double2 sg = make_double2(0, 0);
  for (int t = lane; t < nt; t += 64) {
    const double2 v = sp[(int64_t)run * nt + t];
    sg.x += v.x;
    sg.y += v.y;
  }
  if (signl != nullptr)
    for (int a = lane; a < n_atoms; a += 64) {
      const double2 v = signl[(int64_t)run * n_atoms + a];
      sg.x += v.x;
      sg.y += v.y;
    }
  sg.x = wsum<double>(sg.x);
  sg.y = wsum<double>(sg.y);
  if (lane != 0) return;
  if (!(sg.x != 0.0 || sg.y != 0.0) || !finite2(sg)) {
    sc.brk[run] = 1;
    sc.status[run] = (st == ST_ACT_LO) ? ST_RU_LO : ST_RU_HI;
    sc.ru_par[run] = parity & 1;
    sc.alpha[run] = make_double2(0, 0);
    sc.xcoef[run] = make_double2(0, 0);
    return;
  }
  const double2 al = cdiv<double>(sc.rho[run], sg);
  sc.alpha[run] = al;
  sc.xcoef[run] = al;
}

// One wavefront per run: the lanes add the update's per-chunk partials, lane 0 takes the
// decisions.  The list of runs marked for replacement is built afterwards (k_ru_list).
__global__ void __launch_bounds__(256) k_s2(BicgScal sc, int32_t nruns, int32_t nchunks, const double* part,
                                            double tol, int32_t max_iter, double narrow_tol, double ru_factor,
                                            int32_t lo_window, double div_factor, double* hist, int32_t hstride,
                                            int32_t hrows, int32_t parity) {
  const int lane = threadIdx.x & 63;
  const int run = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (run >= nruns) return;
  const int st = sc.status[run];
  if (!is_active(st)) {
    if (lane == 0) sc.conv[run] = 0;   // the previous iteration's phase changes are done
    return;
  }
  double s[4] = {0, 0, 0, 0};
  for (int c = lane; c < nchunks; c += 64)
    for (int k = 0; k < 4; ++k) s[k] += part[((int64_t)run * nchunks + c) * 4 + k];
  for (int k = 0; k < 4; ++k) s[k] = wsum<double>(s[k]);
  if (lane != 0) return;
  sc.conv[run] = 0;
  const int it = sc.iters[run] + 1;
  sc.iters[run] = it;
  const double vn = sc.vn2[run];
  const double rr = sqrt(s[2] / vn), rrt = sqrt(s[3] / vn);
  sc.relres[2 * run] = rr;
  sc.relres[2 * run + 1] = rrt;
  // optional convergence history: row it / hstride - 1 holds this iteration's residuals
  if (hist != nullptr && it % hstride == 0 && it / hstride <= hrows) {
    const int64_t at = ((int64_t)(it / hstride - 1) * nruns + run) * 2;
    hist[at] = rr;
    hist[at + 1] = rrt;
  }
  const double2 rn = make_double2(s[0], s[1]);
  const double2 ro = sc.rho[run];
  const bool conv = (rr < tol) && (rrt < tol);
  const bool bad = !(rn.x != 0.0 || rn.y != 0.0) || !finite2(rn) || !isfinite(rr) || !isfinite(rrt);
  if (bad && !conv) sc.brk[run] = 1;
  sc.beta[run] = bad ? make_double2(0, 0) : cdiv<double>(rn, ro);
  sc.rho_prev[run] = ro;
  sc.rho[run] = rn;
  const bool stalled = (st == ST_ACT_LO) && (it - sc.ru_it[run] >= lo_window);
  // a residual div_factor (1e6) times above the smallest since the last replacement, 20
  // iterations or more after it (a restarted BiCG rises above its starting residual at
  // first): the run is diverging (near a breakdown); the replacement restarts it from its
  // accumulated solution
  const double cur = fmax(rr, rrt);
  const double mn = fmin(sc.rmin[run], cur);
  sc.rmin[run] = mn;
  const bool diverged = it - sc.ru_it[run] >= 20 && cur > div_factor * mn;
  if (conv || bad || it >= max_iter || cur < sc.ru_thr[run] || stalled || diverged) {
    sc.status[run] = (st == ST_ACT_LO) ? ST_RU_LO : ST_RU_HI;
    sc.ru_par[run] = parity & 1;
  } else if (st == ST_ACT_HI && narrow_tol > 0.0 && sc.ru_thr[run] >= 0.0 && fmax(rr, rrt) < narrow_tol &&
             (parity & 1)) {
    // the residual is small enough for complex64 vectors and operator applications (on odd
    // iterations, where k_phase runs)
    sc.status[run] = ST_ACT_LO;
    sc.conv[run] = 2;
    sc.ru_it[run] = it;
    sc.ru_thr[run] = fmax(rr, rrt) * ru_factor;
  }
}

// The list of runs marked for replacement, and the active lists without them (the
// replacement itself runs on odd iterations only; k_s3 rebuilds the lists after it).
__global__ void __launch_bounds__(256) k_ru_list(BicgScal sc, int32_t nruns) {
  build_ru_list(sc, nruns);
  build_lists(sc, nruns);
}

__global__ void __launch_bounds__(256) k_s3(BicgScal sc, int32_t nruns, int32_t nchunks, double* part,
                                            double tol, int32_t max_iter, int32_t max_ru, double ru_factor) {
  // the partial sums of each replaced run (listed by k_ru_list): the whole block adds them up and
  // leaves the totals in the run's first chunk slot
  __shared__ double red[4][4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nlist = sc.n_active[2];
  for (int i = 0; i < nlist; ++i) {
    const int run = sc.list[2 * (int64_t)nruns + i];
    double t[4] = {0, 0, 0, 0};
    for (int c = tid; c < nchunks; c += 256)
      for (int k = 0; k < 4; ++k) t[k] += part[((int64_t)run * nchunks + c) * 4 + k];
    for (int k = 0; k < 4; ++k) t[k] = wsum<double>(t[k]);
    if (lane == 0)
      for (int k = 0; k < 4; ++k) red[wv][k] = t[k];
    __syncthreads();
    if (tid < 4) part[(int64_t)run * nchunks * 4 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();
  }
  for (int run = threadIdx.x; run < nruns; run += blockDim.x) {
    int st = sc.status[run];
    if (is_ru(st)) {
      double s[4];
      for (int k = 0; k < 4; ++k) s[k] = part[(int64_t)run * nchunks * 4 + k];
      const double vn = sc.vn2[run];
      const double rr = sqrt(s[2] / vn), rrt = sqrt(s[3] / vn);
      sc.relres[2 * run] = rr;
      sc.relres[2 * run + 1] = rrt;
      const int nru = sc.nru[run] + 1;
      sc.nru[run] = nru;
      sc.ru_it[run] = sc.iters[run];
      sc.rmin[run] = fmax(rr, rrt);
      sc.xcoef[run] = make_double2(0, 0);
      const double2 rn = make_double2(s[0], s[1]);
      if (rr < tol && rrt < tol) {
        st = ST_DONE;
      } else if (sc.brk[run] || !finite2(rn) || !(rn.x != 0.0 || rn.y != 0.0)) {
        st = ST_BREAKDOWN;
      } else if (sc.halt[run]) {
        st = ST_HALTED;
      } else if (sc.iters[run] >= max_iter || nru >= max_ru) {
        st = ST_NOCONV;
      } else {
        sc.beta[run] = cdiv<double>(rn, sc.rho_prev[run]);
        sc.rho[run] = rn;
        const double tr = fmax(rr, rrt);
        if (st == ST_RU_LO && tr > 0.5 * sc.ru_thr[run] / ru_factor) {
          // the complex64 recurrence stopped reducing the true residual: restart BiCG in
          // complex128 from the accumulated solution (the replaced residual is in R64,
          // beta = 0 makes the true residual the first search direction)
          st = ST_ACT_HI;
          sc.conv[run] = 1;
          sc.nrestart[run] += 1;
          sc.ru_thr[run] = -1.0;
          sc.beta[run] = make_double2(0, 0);
        } else if (st == ST_RU_LO) {
          st = ST_ACT_LO;
          sc.ru_thr[run] = tr * ru_factor;
        } else {
          st = ST_ACT_HI;
          if (tr > 100.0 * tol) {
            // a complex128 run is replaced once its recursive residual is below tol, or when
            // it diverges (k_s2); a true residual far above tol means the recurrence lost its
            // accuracy (a near-breakdown made the iterate a sum of large, cancelling terms):
            // restart BiCG from the accumulated solution, the true residual as the first
            // search direction, instead of continuing recurrences whose scalars no longer
            // match the residual (in mixed mode k_phase also clears the old direction)
            sc.beta[run] = make_double2(0, 0);
            sc.conv[run] = 1;
            sc.nrestart[run] += 1;
          }
          sc.ru_thr[run] = (sc.ru_thr[run] < 0.0) ? -1.0 : 0.0;
        }
      }
      sc.status[run] = st;
    }
  }
  __syncthreads();
  build_lists(sc, nruns);
}

// Half-of-the-nodes rule (paper Sec. 3.3): within every group of n_q*L runs, once more
// than half of the nodes have all their right-hand sides converged, the remaining runs
// stop (their iterate is still accumulated by a last replacement).  A run that changes
// phase this iteration (conv != 0: its complex64 vectors are written only at the end of
// the iteration) is stopped at the next one.
__global__ void __launch_bounds__(256) k_half_stop(BicgScal sc, int32_t ngroups, int32_t n_q, int32_t L,
                                                   int32_t parity) {
  for (int g = threadIdx.x; g < ngroups; g += blockDim.x) {
    int done_nodes = 0;
    for (int j = 0; j < n_q; ++j) {
      bool all = true;
      for (int l = 0; l < L; ++l) all = all && (sc.status[(g * n_q + j) * L + l] == ST_DONE);
      done_nodes += all ? 1 : 0;
    }
    if (2 * done_nodes > n_q) {
      for (int r = g * n_q * L; r < (g + 1) * n_q * L; ++r) {
        const int st = sc.status[r];
        if ((st == ST_ACT_LO || st == ST_ACT_HI) && sc.conv[r] == 0) {
          sc.status[r] = (st == ST_ACT_LO) ? ST_RU_LO : ST_RU_HI;
          sc.ru_par[r] = parity & 1;
          sc.halt[r] = 1;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ work queue
// A batched solve holds more items (energy, node, right-hand side) than slots.  After every
// iteration: the slots whose item finished record its iterations, residuals and state
// (k_q_retire), add its solution to the moments of its energy (k_q_accum), and take the
// next items of the queue (k_q_refill: coefficients, right-hand side; k_q_init: r = v,
// p = x = y = 0 and the first partial sums; k_q_s0: the scalar state of a new run and the
// active lists).  The queue is a counter on the device, so no host step is involved; the
// host only reads the active count once per replayed chunk of iterations.
__device__ __forceinline__ bool is_final(int st) {
  return st == ST_DONE || st == ST_NOCONV || st == ST_BREAKDOWN || st == ST_HALTED;
}

// Slots (ascending) whose item finished, compacted into rlist; head[1] = their count.
// One block of 256 threads.
__global__ void __launch_bounds__(256) k_q_retire(BicgScal sc, QueueState q, int32_t nruns) {
  __shared__ int wcnt[4];
  __shared__ int base;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) base = 0;
  __syncthreads();
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r0 = 0; r0 < nruns; r0 += 256) {
    const int run = r0 + tid;
    const int item = (run < nruns) ? q.slot_item[run] : -1;
    const bool ret = item >= 0 && is_final(sc.status[run]);
    if (ret) {
      q.item_iters[item] = sc.iters[run];
      q.item_status[item] = sc.status[run];
      q.item_relres[2 * item] = sc.relres[2 * run];
      q.item_relres[2 * item + 1] = sc.relres[2 * run + 1];
    }
    const unsigned long long m = __ballot(ret);
    if (lane == 0) wcnt[wv] = __popcll(m);
    __syncthreads();
    int o = base;
    for (int w = 0; w < wv; ++w) o += wcnt[w];
    if (ret) q.rlist[o + __popcll(m & below)] = run;
    __syncthreads();
    if (tid == 0) base += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  if (tid == 0) q.head[1] = base;
}

// S[e][k][l] += w1_j z1_j^k y - w2_j z2_j^k yt (2 Re of it when the mirrored nodes are
// taken by conjugation) for every retiring slot, in list order: a thread owns its points
// for all slots, so items with the same (e, l) add in a fixed order.
__global__ void __launch_bounds__(256) k_q_accum(int64_t N, QueueState q, const Pair<double>* Y) {
  const int cnt = q.head[1];
  if (cnt == 0) return;
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
    for (int i = 0; i < cnt; ++i) {
      const int slot = q.rlist[i];
      const int item = q.slot_item[slot];
      const int l = item % q.L, j = (item / q.L) % q.nq, e = item / (q.L * q.nq);
      const Pair<double> y = Y[(int64_t)slot * N + n];
      for (int k = 0; k < q.M2; ++k) {
        const double2 t = csub<double>(cmul<double>(q.ca[j * q.M2 + k], y.a), cmul<double>(q.cb[j * q.M2 + k], y.b));
        double2* sp = q.S + (((int64_t)e * q.M2 + k) * q.L + l) * N + n;
        double2 sv = *sp;
        if (q.conj) {
          sv.x += 2.0 * t.x;
        } else {
          sv.x += t.x;
          sv.y += t.y;
        }
        *sp = sv;
      }
    }
  }
}

// Frees the retired slots, then gives the free slots (ascending) the next items; rlist /
// head[1] then list the refilled slots.  One block of 256 threads.
__global__ void __launch_bounds__(256) k_q_refill(QueueState q, int32_t nruns) {
  __shared__ int wcnt[4];
  __shared__ int base;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nret = q.head[1];
  for (int i = tid; i < nret; i += 256) q.slot_item[q.rlist[i]] = -1;
  if (tid == 0) base = 0;
  __syncthreads();
  const int next = q.head[0];
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r0 = 0; r0 < nruns; r0 += 256) {
    const int run = r0 + tid;
    const bool fr = run < nruns && q.slot_item[run] < 0;
    const unsigned long long m = __ballot(fr);
    if (lane == 0) wcnt[wv] = __popcll(m);
    __syncthreads();
    int o = base;
    for (int w = 0; w < wv; ++w) o += wcnt[w];
    const int pos = o + __popcll(m & below);
    const int item = next + pos;
    if (fr && item < q.n_items) {
      q.slot_item[run] = item;
      q.slot_rhs[run] = item % q.L;
      q.coef_w[run] = q.item_coef[item / q.L];
      q.rlist[pos] = run;
    }
    __syncthreads();
    if (tid == 0) base += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  if (tid == 0) {
    const int take = min(base, q.n_items - next);
    q.head[0] = next + take;
    q.head[1] = take;
  }
}

// The refilled slots' vectors (complex128 phase): r = (v, v), p_old = p_new = x = y = 0, and
// the partial sums of rho = rt^H r, ||r||^2, ||rt||^2 per (slot, chunk) as k_partials makes them.
__global__ void __launch_bounds__(256) k_q_init(int64_t N, int32_t nchunks, QueueState q, const double2* V,
                                                const double2* Vd, Pair<double>* R, Pair<double>* P0,
                                                Pair<double>* P1, Pair<double>* X, Pair<double>* Y, double* part) {
  __shared__ double red[4][4];
  const int cnt = q.head[1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int lb = blockIdx.x; lb < cnt * nchunks; lb += gridDim.x) {
    const int i = lb / nchunks, ch = lb - i * nchunks;
    const int run = q.rlist[i];
    const int l = q.slot_rhs[run];
    const int64_t chunk = (N + nchunks - 1) / nchunks;
    const int64_t lo = ch * chunk, hi = std::min<int64_t>(lo + chunk, N);
    double s[4] = {0, 0, 0, 0};
    Pair<double> z;
    z.a = make_double2(0, 0);
    z.b = z.a;
    for (int64_t n = lo + tid; n < hi; n += 256) {
      const int64_t g = (int64_t)run * N + n;
      Pair<double> r;
      r.a = V[(int64_t)l * N + n];
      r.b = Vd[(int64_t)l * N + n];
      R[g] = r;
      P0[g] = z;
      P1[g] = z;
      X[g] = z;
      Y[g] = z;
      const double2 rho = cmulc<double>(r.b, r.a);
      s[0] += rho.x;
      s[1] += rho.y;
      s[2] += cabs2<double>(r.a);
      s[3] += cabs2<double>(r.b);
    }
    for (int k = 0; k < 4; ++k) s[k] = wsum<double>(s[k]);
    if (lane == 0)
      for (int k = 0; k < 4; ++k) red[wv][k] = s[k];
    __syncthreads();
    if (tid < 4) part[((int64_t)run * nchunks + ch) * 4 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    __syncthreads();
  }
}

// Scalar state of the refilled slots (as k_s0 for a new run), then the active lists.
__global__ void __launch_bounds__(256) k_q_s0(BicgScal sc, QueueState q, int32_t nruns, int32_t nchunks,
                                              const double* part) {
  const int cnt = q.head[1];
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const int run = q.rlist[i];
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
    sc.conv[run] = 0;
    sc.ru_it[run] = 0;
    sc.nrestart[run] = 0;
    sc.ru_thr[run] = 0.0;
    const bool zero = s[2] == 0.0 && s[3] == 0.0;
    sc.relres[2 * run] = zero ? 0.0 : 1.0;
    sc.relres[2 * run + 1] = zero ? 0.0 : 1.0;
    sc.rmin[run] = 1.0;
    sc.status[run] = zero ? ST_DONE : ST_ACT_HI;
  }
  __syncthreads();
  build_lists(sc, nruns);
}

__global__ void k_q_setup(int32_t nruns, QueueState q, BicgScal sc) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < nruns; r += gridDim.x * blockDim.x) {
    q.slot_item[r] = -1;
    q.slot_rhs[r] = 0;
    sc.status[r] = ST_DONE;
    sc.iters[r] = 0;
    sc.relres[2 * r] = 0.0;
    sc.relres[2 * r + 1] = 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    q.head[0] = 0;
    q.head[1] = 0;
  }
}

__global__ void k_fill_c(int64_t n, double2* p) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_double2(0.0, 0.0);
}

static int32_t enqueue_queue_step(BicgSolve& b, hipStream_t st, bool retire) {
  QueueState& q = *b.q;
  const int64_t N = b.sys->N;
  if (retire) {
    hipLaunchKernelGGL(k_q_retire, dim3(1), dim3(256), 0, st, b.sc, q, b.nruns);
    hipLaunchKernelGGL(k_q_accum, dim3((int)std::min<int64_t>((N + 255) / 256, 2048)), dim3(256), 0, st, N, q,
                       (const Pair<double>*)b.Y);
  }
  hipLaunchKernelGGL(k_q_refill, dim3(1), dim3(256), 0, st, q, b.nruns);
  hipLaunchKernelGGL(k_q_init, dim3(std::min(b.nruns * b.nchunks, 4096)), dim3(256), 0, st, N, b.nchunks, q, b.V,
                     b.Vd ? b.Vd : b.V, b.hi.R, b.hi.Pb[0], b.hi.Pb[1], b.hi.X, b.Y, b.upd_part);
  hipLaunchKernelGGL(k_q_s0, dim3(1), dim3(256), 0, st, b.sc, q, b.nruns, b.nchunks, (const double*)b.upd_part);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

int32_t queue_alloc(BicgSolve& b, QueueState& q, const std::vector<RunCoef>& item_coef,
                    const std::vector<double2>& ca, const std::vector<double2>& cb, const char* tag,
                    hipStream_t st) {
  Workspace& ws = b.sys->ws;
  const std::string t = tag;
  RunCoef* ic = nullptr;
  double2 *dca = nullptr, *dcb = nullptr;
  CBS_TRY(ws_get(ws, (t + ".slot_item").c_str(), (size_t)b.nruns, &q.slot_item));
  CBS_TRY(ws_get(ws, (t + ".slot_rhs").c_str(), (size_t)b.nruns, &q.slot_rhs));
  CBS_TRY(ws_get(ws, (t + ".head").c_str(), 2, &q.head));
  CBS_TRY(ws_get(ws, (t + ".rlist").c_str(), (size_t)b.nruns, &q.rlist));
  CBS_TRY(ws_get(ws, (t + ".icoef").c_str(), item_coef.size(), &ic));
  CBS_TRY(ws_get(ws, (t + ".coefw").c_str(), (size_t)b.nruns, &q.coef_w));
  CBS_TRY(ws_get(ws, (t + ".iiters").c_str(), (size_t)q.n_items, &q.item_iters));
  CBS_TRY(ws_get(ws, (t + ".istat").c_str(), (size_t)q.n_items, &q.item_status));
  CBS_TRY(ws_get(ws, (t + ".irel").c_str(), 2 * (size_t)q.n_items, &q.item_relres));
  CBS_TRY(ws_get(ws, (t + ".ca").c_str(), ca.size(), &dca));
  CBS_TRY(ws_get(ws, (t + ".cb").c_str(), cb.size(), &dcb));
  const size_t ns = (size_t)q.nE * q.M2 * q.L * b.sys->N;
  CBS_TRY(ws_get(ws, (t + ".S").c_str(), ns, &q.S));
  CBS_HIP(hipMemcpyAsync(ic, item_coef.data(), item_coef.size() * sizeof(RunCoef), hipMemcpyHostToDevice, st));
  CBS_HIP(hipMemcpyAsync(dca, ca.data(), ca.size() * sizeof(double2), hipMemcpyHostToDevice, st));
  CBS_HIP(hipMemcpyAsync(dcb, cb.data(), cb.size() * sizeof(double2), hipMemcpyHostToDevice, st));
  q.item_coef = ic;
  q.ca = dca;
  q.cb = dcb;
  hipLaunchKernelGGL(k_fill_c, dim3((int)std::min<size_t>((ns + 255) / 256, 1 << 16)), dim3(256), 0, st,
                     (int64_t)ns, q.S);
  CBS_HIP(hipGetLastError());
  b.coef = q.coef_w;
  b.q = &q;
  return CBS_OK;
}

// ------------------------------------------------------------------ host driver
template <typename T>
static int32_t alloc_vecs(cbs_system* s, BicgVecs<T>& v, size_t nruns, const std::string& pre) {
  Workspace& ws = s->ws;
  const size_t nv = nruns * s->N;
  CBS_TRY(ws_get(ws, (pre + "R").c_str(), nv, &v.R));
  CBS_TRY(ws_get(ws, (pre + "P0").c_str(), nv, &v.Pb[0]));
  CBS_TRY(ws_get(ws, (pre + "P1").c_str(), nv, &v.Pb[1]));
  CBS_TRY(ws_get(ws, (pre + "Q").c_str(), nv, &v.Q));
  CBS_TRY(ws_get(ws, (pre + "X").c_str(), nv, &v.X));
  if (s->proj.n_atoms > 0) CBS_TRY(ws_get(ws, (pre + "KT").c_str(), nruns * s->proj.n_atoms * 12, &v.KT));
  v.tile_y = s->tile_y[std::is_same<T, float>::value ? 1 : 0];
  v.ntiles = stencil_tiles(s, v.tile_y);
  CBS_TRY(ws_get(ws, (pre + "sig").c_str(), nruns * v.ntiles, &v.sig));
  return CBS_OK;
}

int32_t bicg_alloc(BicgSolve& b, const char* tag) {
  cbs_system* s = b.sys;
  Workspace& ws = s->ws;
  const std::string t = tag;
  const size_t R = b.nruns;
  CBS_TRY(autotune_tiles(s, nullptr));
  if (b.mixed) CBS_TRY(alloc_vecs<float>(s, b.lo, R, t + ".lo."));
  CBS_TRY(alloc_vecs<double>(s, b.hi, R, t + ".hi."));
  CBS_TRY(ws_get(ws, (t + ".Y").c_str(), R * s->N, &b.Y));
  b.nchunks = update_chunks(s);
  const int na = s->proj.n_atoms;
  CBS_TRY(ws_get(ws, (t + ".signl").c_str(), R * std::max(na, 1), &b.signl));
  CBS_TRY(ws_get(ws, (t + ".upd").c_str(), R * b.nchunks * 4, &b.upd_part));
  b.bra_part = nullptr;
  if (s->bra_tile[0] > 0 || s->bra_tile[1] > 0) {
    unsigned char* bp = nullptr;
    CBS_TRY(ws_get(ws, (t + ".brapart").c_str(), bra_tile_part_bytes(s, (int32_t)R), &bp));
    b.bra_part = bp;
  }
  b.ru_chunks = (int32_t)(((s->N + KG - 1) / KG + 3) / 4);   // one group per wave
  CBS_TRY(ws_get(ws, (t + ".ru").c_str(), R * b.ru_chunks * 4, &b.ru_part));
  CBS_TRY(ws_get(ws, (t + ".alpha").c_str(), R, &b.sc.alpha));
  CBS_TRY(ws_get(ws, (t + ".xcoef").c_str(), R, &b.sc.xcoef));
  CBS_TRY(ws_get(ws, (t + ".beta").c_str(), R, &b.sc.beta));
  CBS_TRY(ws_get(ws, (t + ".rho").c_str(), R, &b.sc.rho));
  CBS_TRY(ws_get(ws, (t + ".rhop").c_str(), R, &b.sc.rho_prev));
  CBS_TRY(ws_get(ws, (t + ".vn2").c_str(), R, &b.sc.vn2));
  CBS_TRY(ws_get(ws, (t + ".relres").c_str(), 2 * R, &b.sc.relres));
  CBS_TRY(ws_get(ws, (t + ".ruthr").c_str(), R, &b.sc.ru_thr));
  CBS_TRY(ws_get(ws, (t + ".rmin").c_str(), R, &b.sc.rmin));
  CBS_TRY(ws_get(ws, (t + ".rupar").c_str(), R, &b.sc.ru_par));
  CBS_TRY(ws_get(ws, (t + ".status").c_str(), R, &b.sc.status));
  CBS_TRY(ws_get(ws, (t + ".iters").c_str(), R, &b.sc.iters));
  CBS_TRY(ws_get(ws, (t + ".brk").c_str(), R, &b.sc.brk));
  CBS_TRY(ws_get(ws, (t + ".halt").c_str(), R, &b.sc.halt));
  CBS_TRY(ws_get(ws, (t + ".nru").c_str(), R, &b.sc.nru));
  CBS_TRY(ws_get(ws, (t + ".conv").c_str(), R, &b.sc.conv));
  CBS_TRY(ws_get(ws, (t + ".nact").c_str(), 3, &b.sc.n_active));
  CBS_TRY(ws_get(ws, (t + ".ruit").c_str(), R, &b.sc.ru_it));
  CBS_TRY(ws_get(ws, (t + ".nrst").c_str(), R, &b.sc.nrestart));
  CBS_TRY(ws_get(ws, (t + ".list").c_str(), 3 * R, &b.sc.list));
  return CBS_OK;
}

static int32_t enqueue_init(BicgSolve& b, hipStream_t st) {
  cbs_system* s = b.sys;
  if (b.q != nullptr) {
    // every slot empty and final, then the first refill
    hipLaunchKernelGGL(k_q_setup, dim3(std::max(1, std::min((b.nruns + 255) / 256, 1024))), dim3(256), 0, st,
                       b.nruns, *b.q, b.sc);
    CBS_HIP(hipGetLastError());
    return enqueue_queue_step(b, st, false);
  }
  const int64_t total = (int64_t)b.nruns * s->N;
  const int g = (int)std::min<int64_t>((total + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_bicg_init<double>, dim3(g), dim3(256), 0, st, s->N, b.nruns, b.L, b.V, b.Vd ? b.Vd : b.V, b.hi.R, b.hi.Pb[0],
                     b.hi.Pb[1], b.hi.X, b.Y);
  CBS_HIP(hipGetLastError());
  const int nl = b.nruns * b.nchunks;
  hipLaunchKernelGGL(k_partials<double>, dim3(grid8(nl)), dim3(256), 0, st, s->N, b.nchunks, nl,
                     (const Pair<double>*)b.hi.R, b.upd_part);
  CBS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_s0, dim3(1), dim3(256), 0, st, b.sc, b.nruns, b.nchunks, (const double*)b.upd_part,
                     (int32_t)ST_ACT_HI, b.vn2_ref);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

template <typename T>
static int32_t enqueue_stencil_bra(BicgSolve& b, BicgVecs<T>& v, int32_t need, int parity, hipStream_t st) {
  cbs_system* s = b.sys;
  StencilLaunch l{};
  l.nruns = b.nruns;
  l.rin = v.R;
  l.pold = v.Pb[(parity + 1) & 1];
  l.pnew = v.Pb[parity & 1];
  l.q = v.Q;
  l.x = v.X;
  l.coef = b.coef;
  l.beta = b.sc.beta;
  l.xcoef = b.sc.xcoef;
  l.status = b.sc.status;
  l.need_status = need;
  l.sig_part = v.sig;
  const int ph = (need == ST_ACT_LO) ? 0 : 1;
  l.list = b.sc.list + (size_t)ph * b.nruns;
  l.count = b.sc.n_active + ph;
  if (v.ev0) CBS_HIP(hipEventRecord(v.ev0, st));
  CBS_TRY(launch_stencil<T>(s, true, l, v.tile_y, st));
  if (v.ev1) CBS_HIP(hipEventRecord(v.ev1, st));
  if (s->proj.n_atoms > 0)
    CBS_TRY(launch_bra<T>(s, b.nruns, v.Pb[parity & 1], b.coef, b.sc.status, need, v.KT, b.signl, st, true,
                          l.list, l.count, false, b.bra_part));
  return CBS_OK;
}

// Residual replacement of the runs on the list built by k_ru_list: the pending x update and
// y += x, the true residual v - P(z) y in complex128 (stencil and bra over the short list),
// and k_s3's decisions.
static int32_t enqueue_replacement(BicgSolve& b, int parity, hipStream_t st) {
  cbs_system* s = b.sys;
  const int na = s->proj.n_atoms;
  const int32_t* rul = b.sc.list + 2 * (size_t)b.nruns;
  const int32_t* ruc = b.sc.n_active + 2;
  const int nlr = b.nruns * b.ru_chunks;
  const int gru = std::min(grid8(nlr), 2048);
  if (b.mixed)
    hipLaunchKernelGGL(k_ru_pre<float>, dim3(gru), dim3(256), 0, st, s->N, b.ru_chunks, nlr, rul, ruc,
                       (const int32_t*)b.sc.status, (int32_t)ST_RU_LO, (const double2*)b.sc.xcoef,
                       (const int32_t*)b.sc.ru_par, parity, b.lo.Pb[0], b.lo.Pb[1], b.lo.X, b.Y);
  hipLaunchKernelGGL(k_ru_pre<double>, dim3(gru), dim3(256), 0, st, s->N, b.ru_chunks, nlr, rul, ruc,
                     (const int32_t*)b.sc.status, (int32_t)ST_RU_HI, (const double2*)b.sc.xcoef,
                     (const int32_t*)b.sc.ru_par, parity, b.hi.Pb[0], b.hi.Pb[1], b.hi.X, b.Y);
  CBS_HIP(hipGetLastError());
  {
    StencilLaunch r{};
    r.nruns = b.nruns;
    r.rin = b.Y;
    r.q = b.hi.Q;
    r.coef = b.coef;
    r.list = rul;
    r.count = ruc;
    r.zseg = 4;   // the list is short: four z segments per tile shorten each workgroup's march
    CBS_TRY(launch_stencil<double>(s, false, r, b.hi.tile_y, st));
    if (na > 0)
      CBS_TRY(launch_bra<double>(s, b.nruns, b.Y, b.coef, nullptr, 0, b.hi.KT, nullptr, st, true, rul, ruc,
                                 true));
  }
  if (b.mixed)
    hipLaunchKernelGGL(k_ru_post<float>, dim3(gru), dim3(256), 0, st, s->N, b.ru_chunks, nlr, rul, ruc, b.L,
                       b.q ? (const int32_t*)b.q->slot_rhs : (const int32_t*)nullptr, na,
                       (const int32_t*)b.sc.status, (int32_t)ST_RU_LO, b.V, b.Vd ? b.Vd : b.V,
                       (const Pair<double>*)b.hi.Q, (const Pair<double>*)b.hi.KT, s->proj.grp_off, s->proj.grp_key,
                       (const double*)s->proj.grp_u64, b.lo.R, b.hi.R, b.ru_part);
  hipLaunchKernelGGL(k_ru_post<double>, dim3(gru), dim3(256), 0, st, s->N, b.ru_chunks, nlr, rul, ruc, b.L,
                     b.q ? (const int32_t*)b.q->slot_rhs : (const int32_t*)nullptr, na,
                     (const int32_t*)b.sc.status, (int32_t)ST_RU_HI, b.V, b.Vd ? b.Vd : b.V,
                     (const Pair<double>*)b.hi.Q, (const Pair<double>*)b.hi.KT, s->proj.grp_off, s->proj.grp_key,
                     (const double*)s->proj.grp_u64, b.hi.R, (Pair<double>*)nullptr, b.ru_part);
  CBS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_s3, dim3(1), dim3(256), 0, st, b.sc, b.nruns, b.ru_chunks, b.ru_part, b.tol,
                     b.max_iter, b.max_ru, b.ru_factor);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

static int32_t enqueue_iter(BicgSolve& b, int parity, hipStream_t st) {
  cbs_system* s = b.sys;
  const int na = s->proj.n_atoms;
  const int nl = b.nruns * b.nchunks;
  if (b.mixed) CBS_TRY(enqueue_stencil_bra<float>(b, b.lo, ST_ACT_LO, parity, st));
  CBS_TRY(enqueue_stencil_bra<double>(b, b.hi, ST_ACT_HI, parity, st));
  hipLaunchKernelGGL(k_s1, dim3((b.nruns + 3) / 4), dim3(256), 0, st, b.sc, b.nruns, na, (const double2*)b.lo.sig,
                     b.lo.ntiles, (const double2*)b.hi.sig, b.hi.ntiles, (const double2*)b.signl, parity);
  CBS_HIP(hipGetLastError());
  if (b.mixed)
    CBS_TRY(launch_update<float>(s, b.nruns, b.lo.R, b.lo.Q, b.lo.KT, b.sc.alpha, b.sc.status, ST_ACT_LO,
                                 b.upd_part, b.nchunks, st, b.sc.list, b.sc.n_active));
  CBS_TRY(launch_update<double>(s, b.nruns, b.hi.R, b.hi.Q, b.hi.KT, b.sc.alpha, b.sc.status, ST_ACT_HI,
                                b.upd_part, b.nchunks, st, b.sc.list + b.nruns, b.sc.n_active + 1));
  hipLaunchKernelGGL(k_s2, dim3((b.nruns + 3) / 4), dim3(256), 0, st, b.sc, b.nruns, b.nchunks,
                     (const double*)b.upd_part, b.tol, b.max_iter, b.narrow_tol, b.ru_factor, b.lo_window,
                     b.div_factor, b.hist, b.hist_stride, b.hist_rows, parity);
  CBS_HIP(hipGetLastError());
  if (b.half_stop && b.n_q > 0) {
    hipLaunchKernelGGL(k_half_stop, dim3(1), dim3(256), 0, st, b.sc, b.nruns / (b.n_q * b.L), b.n_q, b.L, parity);
    CBS_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_ru_list, dim3(1), dim3(256), 0, st, b.sc, b.nruns);
  CBS_HIP(hipGetLastError());
  // residual replacement of the runs on the list built by k_ru_list, on odd iterations only
  // (each of its launches costs a few microseconds even when the list is empty): a run marked
  // on an even iteration sits out the next one, whose replacement takes it and moves its
  // direction to that iteration's buffer (k_ru_pre).  Chunks of iterations are even, so
  // every chunk ends with a replacement.
  if (parity & 1) CBS_TRY(enqueue_replacement(b, parity, st));
  // phase changes (narrowing in k_s2, restarts in k_s3) and the work queue (items finished in
  // k_s3) come about on odd iterations only, so their launches are kept to those
  if (b.mixed && (parity & 1)) {
    hipLaunchKernelGGL(k_phase, dim3(grid8(nl)), dim3(256), 0, st, s->N, b.nchunks, nl, (const int32_t*)b.sc.conv,
                       (const Pair<double>*)b.hi.R, b.hi.Pb[parity & 1], b.hi.X, b.lo.R, b.lo.Pb[parity & 1],
                       b.lo.X, b.Y);
    CBS_HIP(hipGetLastError());
  }
  if (b.q != nullptr && (parity & 1)) CBS_TRY(enqueue_queue_step(b, st, true));
  return CBS_OK;
}

static bool use_graphs() {
  const char* e = getenv("CBS_NO_GRAPH");
  return !(e && e[0] == '1');
}

// Profile mode: iterations launched one by one; each stencil launch is bracketed by
// events on the stream it runs on and the active-run counts are read back after every
// iteration to account each launch's algorithmic bytes.
static int32_t run_profiled(std::vector<BicgSolve*>& solves, hipStream_t st, int32_t max_iter) {
  std::vector<int32_t> act(2 * solves.size());
  for (size_t i = 0; i < solves.size(); ++i) {
    BicgSolve& b = *solves[i];
    act[2 * i] = 0;
    act[2 * i + 1] = b.nruns;
    CBS_HIP(hipEventCreate(&b.hi.ev0));
    CBS_HIP(hipEventCreate(&b.hi.ev1));
    if (b.mixed) {
      CBS_HIP(hipEventCreate(&b.lo.ev0));
      CBS_HIP(hipEventCreate(&b.lo.ev1));
    }
  }
  int32_t rc = CBS_OK;
  int32_t hna[2];
  for (int it = 0; it <= max_iter + 3 && rc == CBS_OK; ++it) {
    int any = 0;
    for (size_t i = 0; i < solves.size() && rc == CBS_OK; ++i) {
      BicgSolve& b = *solves[i];
      // (an odd iteration still runs: it replaces the runs marked on the even one before it)
      if (act[2 * i] + act[2 * i + 1] == 0 && (it & 1) == 0) continue;
      rc = enqueue_iter(b, it, st);
      if (rc != CBS_OK) break;
      CBS_HIP(hipMemcpyAsync(hna, b.sc.n_active, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      CBS_HIP(hipStreamSynchronize(st));
      const double passes = (it == 0) ? 4.0 : 6.0;   // r, p_old (+ x) in; p_new, q (+ x) out
      float ms = 0;
      if (b.mixed && act[2 * i] > 0) {
        CBS_HIP(hipEventElapsedTime(&ms, b.lo.ev0, b.lo.ev1));
        b.lo.prof_ms += ms;
        b.lo.prof_launches += 1;
        b.lo.prof_bytes += (double)act[2 * i] * passes * b.sys->N * sizeof(Pair<float>) + b.sys->N * sizeof(float);
      }
      if (act[2 * i + 1] > 0) {
        CBS_HIP(hipEventElapsedTime(&ms, b.hi.ev0, b.hi.ev1));
        b.hi.prof_ms += ms;
        b.hi.prof_launches += 1;
        b.hi.prof_bytes += (double)act[2 * i + 1] * passes * b.sys->N * sizeof(Pair<double>) + b.sys->N * sizeof(double);
      }
      act[2 * i] = hna[0];
      act[2 * i + 1] = hna[1];
      any += hna[0] + hna[1];
    }
    // runs marked on an even iteration are replaced on the odd one: stop after an odd one
    if (any == 0 && (it & 1)) break;
  }
  for (auto* b : solves) {
    hipEvent_t evs[4] = {b->hi.ev0, b->hi.ev1, b->lo.ev0, b->lo.ev1};
    for (auto e : evs)
      if (e) (void)hipEventDestroy(e);
    b->hi.ev0 = b->hi.ev1 = b->lo.ev0 = b->lo.ev1 = nullptr;
  }
  return rc;
}

// Runs all solves to completion on an internal stream ordered after `user` (and `user`
// waits for it at the end).  Several solves (systems) advance in the same graph.
int32_t bicg_run(std::vector<BicgSolve*>& solves, hipStream_t user, int32_t chunk, int32_t max_iter,
                 double* elapsed_ms, bool profile) {
  if (solves.empty()) return CBS_OK;
  if (chunk < 2) chunk = 2;
  if (chunk % 2) chunk += 1;
  hipStream_t st = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int32_t* hact = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  struct Guard {
    hipStream_t& s;
    hipEvent_t& a;
    hipEvent_t& b;
    int32_t*& h;
    hipGraphExec_t& x;
    hipGraph_t& g;
    ~Guard() {
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
      if (h) (void)hipHostFree(h);
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      if (s) (void)hipStreamDestroy(s);
    }
  } guard{st, ev0, ev1, hact, exec, graph};
  CBS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  CBS_HIP(hipEventCreate(&ev0));
  CBS_HIP(hipEventCreate(&ev1));
  CBS_HIP(hipEventRecord(ev0, user));
  CBS_HIP(hipStreamWaitEvent(st, ev0, 0));
  for (auto* b : solves) CBS_TRY(enqueue_init(*b, st));
  // two slots of active counts: the count of chunk c is read while chunk c + 1 runs
  CBS_HIP(hipHostMalloc(&hact, sizeof(int32_t) * 4 * solves.size(), hipHostMallocDefault));
  const bool graphs = use_graphs() && !profile;
  // CBS_VERBOSE=2: a progress line every 500 iterations (long solves); 3: one line per chunk
  // with the complex128 / complex64 active-run counts and the chunk's wall time
  const char* vb = getenv("CBS_VERBOSE");
  const int progress = (vb && vb[0] == '2') ? 500 : 0;
  const bool trace = vb && vb[0] == '3';
  auto tc = std::chrono::steady_clock::now();
  if (graphs) {
    CBS_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
    int32_t rc = CBS_OK;
    for (int k = 0; k < chunk && rc == CBS_OK; ++k)
      for (auto* b : solves)
        if (rc == CBS_OK) rc = enqueue_iter(*b, k, st);
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc != CBS_OK) return rc;
    CBS_HIP(e);
    CBS_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  auto t0 = std::chrono::steady_clock::now();
  int32_t rc = CBS_OK;
  if (profile) {
    rc = run_profiled(solves, st, max_iter);
  } else {
    // Chunk c + 1 is queued before the host waits for the active count of chunk c, so the
    // device never idles on the poll; one chunk past the end runs with empty run lists.
    const int max_chunks = (max_iter + 2) / chunk + 2;
    const size_t ns2 = 2 * solves.size();
    hipEvent_t evc[2] = {nullptr, nullptr};
    struct EvGuard {
      hipEvent_t* e;
      ~EvGuard() {
        for (int i = 0; i < 2; ++i)
          if (e[i]) (void)hipEventDestroy(e[i]);
      }
    } evguard{evc};
    CBS_HIP(hipEventCreateWithFlags(&evc[0], hipEventDisableTiming));
    CBS_HIP(hipEventCreateWithFlags(&evc[1], hipEventDisableTiming));
    auto launch_chunk = [&](int c) -> int32_t {
      if (graphs) {
        if (hipGraphLaunch(exec, st) != hipSuccess) {
          set_error("hipGraphLaunch failed");
          return CBS_EHIP;
        }
      } else {
        for (int k = 0; k < chunk; ++k)
          for (auto* b : solves) CBS_TRY(enqueue_iter(*b, k, st));
      }
      int32_t* slot = hact + (size_t)(c & 1) * ns2;
      for (size_t i = 0; i < solves.size(); ++i)
        if (hipMemcpyAsync(slot + 2 * i, solves[i]->sc.n_active, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st) !=
            hipSuccess) {
          set_error("copy of the active-run count failed");
          return CBS_EHIP;
        }
      CBS_HIP(hipEventRecord(evc[c & 1], st));
      return CBS_OK;
    };
    rc = launch_chunk(0);
    int launched = 1;
    for (int c = 0; c < max_chunks && rc == CBS_OK; ++c) {
      if (launched < max_chunks) {
        rc = launch_chunk(launched);
        ++launched;
        if (rc != CBS_OK) break;
      }
      if (hipEventSynchronize(evc[c & 1]) != hipSuccess) {
        set_error("BiCG iteration failed: %s", hipGetErrorString(hipGetLastError()));
        rc = CBS_EHIP;
        break;
      }
      const int32_t* cnt = hact + (size_t)(c & 1) * ns2;
      int any = 0;
      for (size_t i = 0; i < ns2; ++i) any += cnt[i];
      if (trace) {
        int hi = 0, lo = 0;
        for (size_t i = 0; i < solves.size(); ++i) lo += cnt[2 * i], hi += cnt[2 * i + 1];
        const auto now = std::chrono::steady_clock::now();
        fprintf(stderr, "[cbs] chunk end %d: active complex128 %d complex64 %d, %.3f ms\n", (c + 1) * chunk, hi,
                lo, std::chrono::duration<double, std::milli>(now - tc).count());
        tc = now;
      }
      if (any == 0) break;
      if (progress > 0 && (c + 1) * chunk % progress == 0) {
        fprintf(stderr, "[cbs] BiCG iteration %d: %d runs active\n", (c + 1) * chunk, any);
        fflush(stderr);
      }
    }
  }
  CBS_HIP(hipStreamSynchronize(st));
  auto t1 = std::chrono::steady_clock::now();
  if (elapsed_ms) *elapsed_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  CBS_HIP(hipEventRecord(ev1, st));
  CBS_HIP(hipStreamWaitEvent(user, ev1, 0));
  return rc;
}

int32_t bicg_collect(BicgSolve& b, NodeSolve& out, hipStream_t st) {
  out.nruns = b.nruns;
  out.iters.resize(b.nruns);
  out.relres.resize(2 * (size_t)b.nruns);
  out.status.resize(b.nruns);
  std::vector<int32_t> nru(b.nruns), nrst(b.nruns);
  CBS_HIP(hipMemcpyAsync(out.iters.data(), b.sc.iters, b.nruns * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CBS_HIP(hipMemcpyAsync(out.relres.data(), b.sc.relres, 2 * b.nruns * sizeof(double), hipMemcpyDeviceToHost, st));
  CBS_HIP(hipMemcpyAsync(out.status.data(), b.sc.status, b.nruns * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CBS_HIP(hipMemcpyAsync(nru.data(), b.sc.nru, b.nruns * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CBS_HIP(hipMemcpyAsync(nrst.data(), b.sc.nrestart, b.nruns * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CBS_HIP(hipStreamSynchronize(st));
  out.n_ru = 0;
  for (int v : nru) out.n_ru = std::max(out.n_ru, v);
  out.restarts = 0;
  for (int v : nrst) out.restarts += v;
  const char* verbose = getenv("CBS_VERBOSE");
  if (verbose && (verbose[0] == '1' || verbose[0] == '2')) {
    // diagnostics: final states, iteration spread, the slowest runs
    int cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int v : out.status) cnt[(v >= 0 && v < 8) ? v : 0] += 1;
    std::vector<int> order(b.nruns);
    for (int r = 0; r < b.nruns; ++r) order[r] = r;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return out.iters[x] < out.iters[y]; });
    fprintf(stderr, "[cbs] %d runs: done %d noconv %d breakdown %d halted %d; iters min %d median %d max %d\n",
            b.nruns, cnt[ST_DONE], cnt[ST_NOCONV], cnt[ST_BREAKDOWN], cnt[ST_HALTED], out.iters[order[0]],
            out.iters[order[b.nruns / 2]], out.iters[order[b.nruns - 1]]);
    for (int k = std::max(0, b.nruns - 5); k < b.nruns; ++k) {
      const int r = order[k];
      fprintf(stderr, "[cbs]   run %d: status %d iters %d replacements %d relres %.2e %.2e\n", r, out.status[r],
              out.iters[r], nru[r], out.relres[2 * r], out.relres[2 * r + 1]);
    }
  }
  out.Y = b.Y;
  out.prof_launches = b.hi.prof_launches;
  out.prof_ms = b.hi.prof_ms;
  out.prof_bytes = b.hi.prof_bytes;
  out.prof_lo_launches = b.lo.prof_launches;
  out.prof_lo_ms = b.lo.prof_ms;
  out.prof_lo_bytes = b.lo.prof_bytes;
  return CBS_OK;
}

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
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
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

void configure_solve(BicgSolve& b, const cbs_params* prm) {
  b.mixed = prm->precision == CBS_MIXED;
  b.tol = prm->tol;
  b.ru_factor = 1e-2;
  b.narrow_tol = b.mixed ? std::max(prm->inner_tol, prm->tol) : 0.0;
  b.max_iter = prm->max_iter;
  b.max_ru = std::max(prm->max_refine, 1);
  b.half_stop = prm->half_stop;
  b.lo_window = prm->lo_window > 0 ? prm->lo_window : 300;
  // CBS_DIVERGE_FACTOR overrides the divergence guard's factor (tests set it low to drive the
  // restart path on ordinary residual bumps)
  b.div_factor = 1e6;
  if (const char* e = getenv("CBS_DIVERGE_FACTOR")) {
    const double f = atof(e);
    if (f > 1.0) b.div_factor = f;
  }
}

__global__ void k_fill_nan(int64_t n, double* p) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = __builtin_nan("");
}

// Step-1 solve of one system at one energy, shared by cbs_bicg, cbs_bicg_history and cbs_solve.
int32_t solve_nodes(cbs_system* s, double E, const double2* z, int32_t n_z, int32_t L, const double2* V,
                    const cbs_params* prm, hipStream_t st, NodeSolve& out, const HistReq* hist) {
  std::vector<RunCoef> hc;
  node_coefs(z, n_z, L, E, hc);
  RunCoef* coef = nullptr;
  const int32_t nruns = n_z * L;
  CBS_TRY(ws_get(s->ws, "bicg.coef", (size_t)nruns, &coef));
  CBS_HIP(hipMemcpyAsync(coef, hc.data(), nruns * sizeof(RunCoef), hipMemcpyHostToDevice, st));
  BicgSolve b;
  b.sys = s;
  b.nruns = nruns;
  b.L = L;
  b.n_q = n_z;
  b.V = V;
  b.coef = coef;
  configure_solve(b, prm);
  CBS_TRY(bicg_alloc(b, "bicg"));
  const size_t hn = hist ? (size_t)hist->rows * nruns * 2 : 0;
  if (hn > 0) {
    // rows a run does not reach keep NaN (filled by a kernel: the buffer is not part of a graph)
    CBS_TRY(ws_get(s->ws, "bicg.hist", hn, &b.hist));
    hipLaunchKernelGGL(k_fill_nan, dim3((int)std::min<size_t>((hn + 255) / 256, 4096)), dim3(256), 0, st,
                       (int64_t)hn, b.hist);
    CBS_HIP(hipGetLastError());
    b.hist_stride = hist->stride;
    b.hist_rows = hist->rows;
  }
  std::vector<BicgSolve*> v{&b};
  CBS_TRY(bicg_run(v, st, prm->chunk, prm->max_iter, &out.ms, prm->profile != 0));
  CBS_TRY(bicg_collect(b, out, st));
  if (hn > 0) CBS_HIP(hipMemcpyAsync(hist->host, b.hist, hn * sizeof(double), hipMemcpyDeviceToHost, st));
  // the host coefficient array must outlive the asynchronous copy
  CBS_HIP(hipStreamSynchronize(st));
  if (hn > 0) s->ws.drop("bicg.hist");
  return CBS_OK;
}

int32_t check_params(const cbs_params* p, bool need_moments) {
  if (!p) {
    set_error("params is NULL");
    return CBS_EINVAL;
  }
  if (!(p->lambda_min > 0 && p->lambda_min < 1) || p->n_q < 1 || p->n_rhs < 1 || !(p->tol > 0) || p->max_iter < 1 ||
      (p->precision != CBS_FP64 && p->precision != CBS_MIXED) ||
      (p->precision == CBS_MIXED && !(p->inner_tol > 0 && p->inner_tol < 1)) ||
      (p->conj_nodes != 0 && p->conj_nodes != 1) || p->lo_window < 0 ||
      (p->block != 1 && p->block != p->n_rhs)) {
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

static int32_t bicg_entry(cbs_system* s, double E, int32_t n_z, const double* z, int32_t n_rhs, const void* V,
                          const cbs_params* prm, void* Y, void* Yt, int32_t* iters, double* relres, cbs_info* info,
                          void* stream, const HistReq* hist) {
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
  if (prm->block > 1) {
    if (hist) {
      set_error("cbs_bicg_history: block BiCG keeps no per-run histories");
      return CBS_EINVAL;
    }
    CBS_TRY(solve_nodes_block(s, E, (const double2*)z, n_z, n_rhs, (const double2*)V, prm, st, ns));
  } else {
    CBS_TRY(solve_nodes(s, E, (const double2*)z, n_z, n_rhs, (const double2*)V, prm, st, ns, hist));
  }
  CBS_TRY(split_pairs(s->N, ns.nruns, ns.Y, (double2*)Y, (double2*)Yt, st));
  CBS_HIP(hipStreamSynchronize(st));
  bool noconv = false;
  for (int r = 0; r < ns.nruns; ++r) {
    if (iters) iters[r] = ns.iters[r];
    if (relres) {
      relres[2 * r] = ns.relres[2 * r];
      relres[2 * r + 1] = ns.relres[2 * r + 1];
    }
    noconv = noconv || ns.status[r] != ST_DONE;
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
    info->refine_steps = ns.n_ru;
    info->restarts = (int32_t)std::min<int64_t>(ns.restarts, INT32_MAX);
    info->t_solve_ms = ns.ms;
    info->matvecs = (int64_t)(2 * sum);
    info->stencil_launches = ns.prof_launches;
    info->stencil_ms = ns.prof_ms;
    info->stencil_bytes = ns.prof_bytes;
    info->stencil_lo_launches = ns.prof_lo_launches;
    info->stencil_lo_ms = ns.prof_lo_ms;
    info->stencil_lo_bytes = ns.prof_lo_bytes;
  }
  if (noconv) {
    set_error("cbs_bicg: some runs missed the tolerance");
    return CBS_ENOCONV;
  }
  return CBS_OK;
}

extern "C" int32_t cbs_bicg(cbs_system* s, double E, int32_t n_z, const double* z, int32_t n_rhs, const void* V,
                            const cbs_params* prm, void* Y, void* Yt, int32_t* iters, double* relres, cbs_info* info,
                            void* stream) {
  return bicg_entry(s, E, n_z, z, n_rhs, V, prm, Y, Yt, iters, relres, info, stream, nullptr);
}

// The residual norm of every run along the iterations (the per-node convergence histories
// of Sec. 4.1), recorded by the iteration's scalar kernel as it computes them.
extern "C" int32_t cbs_bicg_history(cbs_system* s, double E, int32_t n_z, const double* z, int32_t n_rhs,
                                    const void* V, const cbs_params* prm, int32_t stride, int32_t max_rows,
                                    double* hist, void* Y, void* Yt, int32_t* iters, double* relres,
                                    cbs_info* info, void* stream) {
  if (stride < 1 || max_rows < 1 || !hist || n_z < 1 || n_rhs < 1 ||
      (int64_t)max_rows * n_z * n_rhs * 2 >= ((int64_t)1 << 31)) {
    set_error("cbs_bicg_history: bad argument (stride >= 1, max_rows >= 1, hist not NULL, "
              "max_rows * runs * 2 < 2^31)");
    return CBS_EINVAL;
  }
  HistReq h;
  h.stride = stride;
  h.rows = max_rows;
  h.host = hist;
  return bicg_entry(s, E, n_z, z, n_rhs, V, prm, Y, Yt, iters, relres, info, stream, &h);
}
