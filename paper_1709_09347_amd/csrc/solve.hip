// The Sakurai-Sugiura method at one energy (paper Sec. 3.1, Algorithm 1, on the ring
// contour of Sec. 3.2):
//   1. BiCG with duals at the outer-circle nodes (bicg.hip): Y_j^(1) primal, Y_j^(2) dual
//   2. moments S_k = sum_j w1_j z1_j^k Y_j^(1) - sum_j w2_j z2_j^k Y_j^(2), k < 2M, and
//      mu_k = V^H S_k (block inner products on MFMA)
//   3. block Hankel T_ij = mu_{i+j}, T<_ij = mu_{i+j+1}; SVD T = U S W^H truncated at
//      sigma > delta sigma_1; reduced problem U1^H T< W1 S1^-1 phi = tau phi
//   4. eigenpairs: Hankel (lambda, S W1 S1^-1 phi) or, by default, Rayleigh-Ritz: the
//      QEP projected onto Q = orth(S W1) and solved densely through its linearisation
//   5. residuals ||P(lambda) psi|| in complex128, the annulus of Eq. 5, sorting.
// Everything between the solves and the host copy of lambda runs on the device in FP64.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "bicg.hpp"
#include "cbs_internal.hpp"
#include "dense.hpp"
#include "ranking.hpp"

namespace cbs {

using c64 = double2;

// Trapezoid nodes and weights on both circles: theta_j = 2 pi (j - 1/2)/n_q,
// z1 = e^{i theta}/lambda_min, z2 = lambda_min e^{i theta} = 1/conj(z1), w = z/n_q
// (the trapezoid rule of (1/2 pi i) \oint dz, dz = i z d theta).
static void quadrature(double lmin, int n_q, std::vector<c64>& z1, std::vector<c64>& w1, std::vector<c64>& z2,
                       std::vector<c64>& w2) {
  z1.resize(n_q);
  w1.resize(n_q);
  z2.resize(n_q);
  w2.resize(n_q);
  for (int j = 0; j < n_q; ++j) {
    const double th = 2.0 * M_PI * (j + 0.5) / n_q;
    const double c = cos(th), s = sin(th);
    z1[j] = make_double2(c / lmin, s / lmin);
    z2[j] = make_double2(c * lmin, s * lmin);
    w1[j] = make_double2(z1[j].x / n_q, z1[j].y / n_q);
    w2[j] = make_double2(z2[j].x / n_q, z2[j].y / n_q);
  }
}

// S[k][l][n] for k in [k0, k0+nk): coefficient tables ca[j][k] = w1 z1^k, cb[j][k] = w2 z2^k,
// over the n_q solved nodes; with conj, each solved node stands for itself and its mirror
// conj z_j (real right-hand sides and real blocks: the mirror's solution is conj y and its
// weight conj w), so the pair adds t + conj t = 2 Re t.
constexpr int MOM_CHUNK = 8;
__global__ void __launch_bounds__(256) k_moments(int64_t N, int32_t L, int32_t n_q, int32_t conj, int32_t nk_total,
                                                 int32_t k0, int32_t nk, const Pair<double>* Y, const c64* ca,
                                                 const c64* cb, c64* S) {
  const int64_t total = N * L;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = g / N, n = g - l * N;
    c64 acc[MOM_CHUNK];
#pragma unroll
    for (int k = 0; k < MOM_CHUNK; ++k) acc[k] = make_double2(0, 0);
    for (int j = 0; j < n_q; ++j) {
      const Pair<double> y = Y[((int64_t)j * L + l) * N + n];
#pragma unroll
      for (int k = 0; k < MOM_CHUNK; ++k) {
        if (k < nk) {
          const c64 a = ca[j * nk_total + k0 + k], b = cb[j * nk_total + k0 + k];
          acc[k] = cadd<double>(acc[k], csub<double>(cmul<double>(a, y.a), cmul<double>(b, y.b)));
        }
      }
    }
#pragma unroll
    for (int k = 0; k < MOM_CHUNK; ++k)
      if (k < nk) S[((int64_t)(k0 + k) * L + l) * N + n] = conj ? make_double2(2.0 * acc[k].x, 0.0) : acc[k];
  }
}

// flag[0] = 1 if any imaginary part of the n values is nonzero; flag[1] = 1 if any value
// is not finite
__global__ void __launch_bounds__(256) k_any_imag(int64_t n, const c64* v, int32_t* flag) {
  bool any = false, bad = false;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
    const c64 x = v[g];
    any = any || !(x.y == 0.0);
    bad = bad || !(isfinite(x.x) && isfinite(x.y));
  }
  if (any) flag[0] = 1;
  if (bad) flag[1] = 1;
}

__global__ void k_clear_flag(int32_t* flag) {
  flag[0] = 0;
  flag[1] = 0;
}

static int32_t launch_grid(int64_t work);

// Quadrature nodes per circle to solve: half of them (0 < theta < pi) when the mirrored
// nodes can be taken from conjugation (conj_nodes, even n_q, every right-hand side real).
// Right-hand sides holding a non-finite value are rejected (CBS_EINVAL).
static int32_t nodes_to_solve(cbs_system* s, const cbs_params* prm, const c64* const* V, int n_v, int64_t count,
                              hipStream_t st, int32_t* nq_solved) {
  *nq_solved = prm->n_q;
  int32_t* flag = nullptr;
  CBS_TRY(ws_get(s->ws, "rhs.imag", 2, &flag));
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, st, flag);
  for (int i = 0; i < n_v; ++i)
    hipLaunchKernelGGL(k_any_imag, dim3(launch_grid(count)), dim3(256), 0, st, count, V[i], flag);
  CBS_HIP(hipGetLastError());
  int32_t h[2] = {1, 1};
  CBS_HIP(hipMemcpyAsync(h, flag, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CBS_HIP(hipStreamSynchronize(st));
  if (h[1] != 0) {
    set_error("the right-hand sides V hold a non-finite value");
    return CBS_EINVAL;
  }
  if (prm->conj_nodes && prm->n_q % 2 == 0 && h[0] == 0) *nq_solved = prm->n_q / 2;
  return CBS_OK;
}

// Block Hankel matrices from mu (C[a + (k L + b) L] = mu_k[a][b]).
__global__ void k_hankel(int32_t L, int32_t M, const c64* C, c64* T, c64* Tl) {
  const int n = L * M;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n * n; t += gridDim.x * blockDim.x) {
    const int r = t % n, c = t / n;
    const int i = r / L, a = r % L, j = c / L, b = c % L;
    T[r + (int64_t)c * n] = C[a + (int64_t)((i + j) * L + b) * L];
    Tl[r + (int64_t)c * n] = C[a + (int64_t)((i + j + 1) * L + b) * L];
  }
}

__global__ void k_gather_cols(int32_t n, int32_t m, const c64* src, int32_t lds, const int32_t* perm, c64* dst,
                              int32_t ldd) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n * m; t += gridDim.x * blockDim.x) {
    const int i = t % n, j = t / n;
    dst[i + (int64_t)j * ldd] = src[i + (int64_t)perm[j] * lds];
  }
}

// coef = W1 diag(1/s) phi  (n x m)
__global__ void k_scale_rows_gemm(int32_t n, int32_t m, const c64* W1, const double* sig, const c64* phi, c64* out) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n * m; t += gridDim.x * blockDim.x) {
    const int i = t % n, j = t / n;
    c64 acc = make_double2(0, 0);
    for (int k = 0; k < m; ++k)
      acc = cadd<double>(acc, cscale<double>(cmul<double>(W1[i + (int64_t)k * n], phi[k + (int64_t)j * m]), 1.0 / sig[k]));
    out[i + (int64_t)j * n] = acc;
  }
}

// Companion linearisation of A- + lam A0 + lam^2 A+ and its shift: X = (A - s B), RHS = B.
__global__ void k_linearize(int32_t m, const c64* A0, const c64* Ap, const c64* Am, c64 sft, c64* X, c64* B) {
  const int n = 2 * m;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n * n; t += gridDim.x * blockDim.x) {
    const int r = t % n, c = t / n;
    c64 a = make_double2(0, 0), b = make_double2(0, 0);
    if (r < m && c < m) {
      b = make_double2(r == c ? 1.0 : 0.0, 0);
    } else if (r < m && c >= m) {
      a = make_double2(r == c - m ? 1.0 : 0.0, 0);
    } else if (r >= m && c < m) {
      a = cscale<double>(Am[(r - m) + (int64_t)c * m], -1.0);
    } else {
      a = cscale<double>(A0[(r - m) + (int64_t)(c - m) * m], -1.0);
      b = Ap[(r - m) + (int64_t)(c - m) * m];
    }
    X[r + (int64_t)c * n] = csub<double>(a, cmul<double>(sft, b));
    B[r + (int64_t)c * n] = b;
  }
}

// Per-vector 2-norm, index of the largest entry; optionally normalise so that entry is real positive.
__global__ void __launch_bounds__(256) k_vec_norm(int64_t N, const c64* V, int64_t ldv, double* norms, int32_t fix,
                                                  c64* out, int64_t ldo) {
  __shared__ double s2[4], smax[4];
  __shared__ int64_t sidx[4];
  __shared__ c64 sph;
  __shared__ double snorm;
  const int v = blockIdx.x, tid = threadIdx.x;
  const c64* x = V + (int64_t)v * ldv;
  double acc = 0, best = -1;
  int64_t bi = 0;
  for (int64_t n = tid; n < N; n += 256) {
    const double a = cabs2<double>(x[n]);
    acc += a;
    if (a > best) {
      best = a;
      bi = n;
    }
  }
  acc = wsum<double>(acc);
  for (int o = 1; o < 64; o <<= 1) {
    const double ob = __shfl_xor(best, o, 64);
    const int64_t oi = __shfl_xor(bi, o, 64);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  if ((tid & 63) == 0) {
    s2[tid >> 6] = acc;
    smax[tid >> 6] = best;
    sidx[tid >> 6] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    double t = s2[0] + s2[1] + s2[2] + s2[3];
    double b = smax[0];
    int64_t ii = sidx[0];
    for (int w = 1; w < 4; ++w)
      if (smax[w] > b || (smax[w] == b && sidx[w] < ii)) {
        b = smax[w];
        ii = sidx[w];
      }
    const double nr = sqrt(t);
    norms[v] = nr;
    snorm = nr;
    const c64 e = x[ii];
    const double ae = sqrt(cabs2<double>(e));
    sph = (ae > 0) ? make_double2(e.x / ae, -e.y / ae) : make_double2(1, 0);   // conj phase
  }
  __syncthreads();
  if (fix && snorm > 0) {
    const c64 f = cscale<double>(sph, 1.0 / snorm);
    for (int64_t n = tid; n < N; n += 256) out[(int64_t)v * ldo + n] = cmul<double>(f, x[n]);
  }
}

static int32_t vec_norms(int64_t N, int32_t nv, const c64* V, int64_t ldv, double* norms, bool fix, c64* out,
                         int64_t ldo, hipStream_t st) {
  if (nv <= 0) return CBS_OK;
  hipLaunchKernelGGL(k_vec_norm, dim3(nv), dim3(256), 0, st, N, V, ldv, norms, (int32_t)fix, out, ldo);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

static int32_t launch_grid(int64_t work) { return (int32_t)std::min<int64_t>((work + 255) / 256, 4096); }

// Diagnostics: with CBS_DUMP=<dir>, intermediate arrays of the extraction are written
// there as raw little-endian files (<name>.bin) for offline comparison.
static void dump(const char* name, const void* dev, size_t bytes, hipStream_t st) {
  const char* dir = getenv("CBS_DUMP");
  if (!dir || !dir[0] || !dev || bytes == 0) return;
  std::vector<char> h(bytes);
  if (hipMemcpyAsync(h.data(), dev, bytes, hipMemcpyDeviceToHost, st) != hipSuccess) return;
  if (hipStreamSynchronize(st) != hipSuccess) return;
  std::string path = std::string(dir) + "/" + name + ".bin";
  FILE* f = fopen(path.c_str(), "wb");
  if (!f) return;
  fwrite(h.data(), 1, bytes, f);
  fclose(f);
}

struct Extracted {
  std::vector<c64> lam;      // candidates kept (in the annulus, residual-filtered), sorted
  std::vector<double> res;
  c64* vecs = nullptr;       // device, [cnt][N] normalised, in sorted order (workspace)
  int32_t rank = 0;
  double sig1 = 0, sig_ratio = 0;
};

// Moment weights w1_j z1_j^k and w2_j z2_j^k of the first nq nodes, k < nk (host, [j][k]).
static void moment_weights(const cbs_params* prm, int nq, int nk, std::vector<c64>& ca, std::vector<c64>& cb) {
  std::vector<c64> z1, w1, z2, w2;
  quadrature(prm->lambda_min, prm->n_q, z1, w1, z2, w2);
  ca.assign((size_t)nq * nk, make_double2(0, 0));
  cb.assign((size_t)nq * nk, make_double2(0, 0));
  for (int j = 0; j < nq; ++j) {
    c64 pa = w1[j], pb = w2[j];
    for (int k = 0; k < nk; ++k) {
      ca[(size_t)j * nk + k] = pa;
      cb[(size_t)j * nk + k] = pb;
      pa = cmul<double>(pa, z1[j]);
      pb = cmul<double>(pb, z2[j]);
    }
  }
}

int32_t extract_S(cbs_system* s, double E, const cbs_params* prm, double noise, const c64* V, const c64* S,
                  hipStream_t st, Extracted& out, double* t_mom_ms, std::chrono::steady_clock::time_point t0);

// The largest primal relative residual of the runs [r0, r1) (relres: [run][primal, dual]),
// finite values only: the noise level of the moments built from those solutions.
static double solve_noise(const std::vector<double>& relres, int64_t r0, int64_t r1) {
  double m = 0;
  for (int64_t r = r0; r < r1; ++r)
    if (std::isfinite(relres[2 * r])) m = std::max(m, relres[2 * r]);
  return m;
}

// Steps 2-5 for one system / energy; Y = node solutions (pairs, run = j*L + l); noise: the
// largest relative residual of those solutions.
int32_t extract(cbs_system* s, double E, const cbs_params* prm, double noise, const c64* V, const Pair<double>* Y,
                int32_t nq_solved, hipStream_t st, Extracted& out, double* t_mom_ms) {
  const int L = prm->n_rhs, M = prm->n_mom, nq = nq_solved, nk = 2 * M;
  const int32_t conj = nq_solved != prm->n_q;
  const int64_t N = s->N;
  Workspace& ws = s->ws;
  auto t0 = std::chrono::steady_clock::now();
  std::vector<c64> ca, cb;
  moment_weights(prm, nq, nk, ca, cb);
  c64 *dca = nullptr, *dcb = nullptr, *S = nullptr;
  CBS_TRY(ws_get(ws, "mom.ca", ca.size(), &dca));
  CBS_TRY(ws_get(ws, "mom.cb", cb.size(), &dcb));
  CBS_TRY(ws_get(ws, "mom.S", (size_t)nk * L * N, &S));
  CBS_HIP(hipMemcpyAsync(dca, ca.data(), ca.size() * sizeof(c64), hipMemcpyHostToDevice, st));
  CBS_HIP(hipMemcpyAsync(dcb, cb.data(), cb.size() * sizeof(c64), hipMemcpyHostToDevice, st));
  for (int k0 = 0; k0 < nk; k0 += MOM_CHUNK) {
    hipLaunchKernelGGL(k_moments, dim3(launch_grid(N * L)), dim3(256), 0, st, N, L, nq, conj, nk, k0,
                       std::min(MOM_CHUNK, nk - k0), Y, (const c64*)dca, (const c64*)dcb, S);
    CBS_HIP(hipGetLastError());
  }
  return extract_S(s, E, prm, noise, V, S, st, out, t_mom_ms, t0);
}

// Steps 2 (mu_k = V^H S_k) to 5 from the moments S [2M][L][N] of one system / energy.
int32_t extract_S(cbs_system* s, double E, const cbs_params* prm, double noise, const c64* V, const c64* S,
                  hipStream_t st, Extracted& out, double* t_mom_ms, std::chrono::steady_clock::time_point t0) {
  const int L = prm->n_rhs, M = prm->n_mom, nk = 2 * M, n = L * M;
  const int64_t N = s->N;
  Workspace& ws = s->ws;
  c64* C = nullptr;
  CBS_TRY(ws_get(ws, "mom.C", (size_t)L * nk * L, &C));
  CBS_TRY(gram(s, N, L, V, N, nk * L, S, N, C, L, st));
  CBS_HIP(hipStreamSynchronize(st));
  dump("S", S, (size_t)nk * L * N * sizeof(c64), st);
  dump("mu", C, (size_t)L * nk * L * sizeof(c64), st);
  auto t1 = std::chrono::steady_clock::now();
  if (t_mom_ms) *t_mom_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();

  // --- Hankel SVD
  c64 *T = nullptr, *Tl = nullptr, *W = nullptr;
  double* sig = nullptr;
  int32_t *perm = nullptr, *info = nullptr;
  CBS_TRY(ws_get(ws, "hk.T", (size_t)n * n, &T));
  CBS_TRY(ws_get(ws, "hk.Tl", (size_t)n * n, &Tl));
  CBS_TRY(ws_get(ws, "hk.W", (size_t)n * n, &W));
  CBS_TRY(ws_get(ws, "hk.sig", 1024, &sig));
  CBS_TRY(ws_get(ws, "hk.perm", 512, &perm));
  CBS_TRY(ws_get(ws, "hk.info", 4, &info));
  CBS_HIP(hipMemsetAsync(info, 0, 4 * sizeof(int32_t), st));
  hipLaunchKernelGGL(k_hankel, dim3(launch_grid((int64_t)n * n)), dim3(256), 0, st, L, M, (const c64*)C, T, Tl);
  CBS_HIP(hipGetLastError());
  dump("T", T, (size_t)n * n * sizeof(c64), st);
  dump("Tl", Tl, (size_t)n * n * sizeof(c64), st);
  CBS_TRY(svd(n, T, n, W, n, sig, perm, st));
  dump("U", T, (size_t)n * n * sizeof(c64), st);
  dump("W", W, (size_t)n * n * sizeof(c64), st);
  dump("sigma", sig, (size_t)n * sizeof(double), st);
  dump("perm", perm, (size_t)n * sizeof(int32_t), st);
  std::vector<double> hsig(n);
  CBS_HIP(hipMemcpyAsync(hsig.data(), sig, n * sizeof(double), hipMemcpyDeviceToHost, st));
  CBS_HIP(hipStreamSynchronize(st));
  if (!all_finite(n, hsig.data())) {
    set_error("non-finite singular values of the Hankel matrix (a linear solve diverged)");
    return CBS_ENONFINITE;
  }
  // rank: singular values above delta sigma_1 and above the noise floor of the moments,
  // the solves' largest residual relative to sigma_1: directions below it carry no
  // information, and in the Rayleigh-Ritz basis they let spurious pairs mix with true ones.
  // Where the floor is ambiguous (between 10x and 100x that residual) both ranks are tried and
  // the one giving more eigenpairs, then the smaller largest residual, is kept.
  auto rank_above = [&](double rel) {
    const double thr = std::max(prm->delta, std::isfinite(noise) ? rel * noise : 0.0);
    int r = 0;
    for (int i = 0; i < n; ++i)
      if (hsig[i] > thr * hsig[0]) ++r;
    return r;
  };
  const int m_hi = rank_above(100.0), m_lo = rank_above(10.0);
  out.sig1 = hsig[0];
  out.lam.clear();
  out.res.clear();
  if (m_lo == 0 || !(hsig[0] > 0)) {
    out.rank = m_lo;
    out.sig_ratio = 0.0;
    return CBS_OK;
  }
  auto extract_rank = [&](const int m, const char* out_name, Extracted& out) -> int32_t {
    out.rank = m;
    out.sig1 = hsig[0];
    out.sig_ratio = (m > 0 && hsig[0] > 0) ? hsig[m - 1] / hsig[0] : 0.0;
    out.lam.clear();
    out.res.clear();
    if (m == 0) return CBS_OK;

    // --- reduced Hankel problem
    c64 *Up = nullptr, *Wp = nullptr, *TW = nullptr, *Bred = nullptr, *tau = nullptr, *phi = nullptr;
    CBS_TRY(ws_get(ws, "hk.Up", (size_t)n * m, &Up));
    CBS_TRY(ws_get(ws, "hk.Wp", (size_t)n * m, &Wp));
    CBS_TRY(ws_get(ws, "hk.TW", (size_t)n * m, &TW));
    CBS_TRY(ws_get(ws, "hk.B", (size_t)m * m, &Bred));
    CBS_TRY(ws_get(ws, "hk.tau", (size_t)2 * n, &tau));
    CBS_TRY(ws_get(ws, "hk.phi", (size_t)m * m, &phi));
    hipLaunchKernelGGL(k_gather_cols, dim3(launch_grid((int64_t)n * m)), dim3(256), 0, st, n, m, (const c64*)T, n,
                       (const int32_t*)perm, Up, n);
    hipLaunchKernelGGL(k_gather_cols, dim3(launch_grid((int64_t)n * m)), dim3(256), 0, st, n, m, (const c64*)W, n,
                       (const int32_t*)perm, Wp, n);
    CBS_HIP(hipGetLastError());
    CBS_TRY(small_gemm(n, m, n, Tl, n, false, Wp, n, TW, n, nullptr, nullptr, st));
    // Bred = Up^H TW diag(1/sigma)
    std::vector<double> inv(m);
    for (int i = 0; i < m; ++i) inv[i] = 1.0 / hsig[i];
    double* dinv = nullptr;
    CBS_TRY(ws_get(ws, "hk.inv", (size_t)m, &dinv));
    CBS_HIP(hipMemcpyAsync(dinv, inv.data(), m * sizeof(double), hipMemcpyHostToDevice, st));
    CBS_TRY(small_gemm(m, m, n, Up, n, true, TW, n, Bred, m, dinv, nullptr, st));
    dump("Bred", Bred, (size_t)m * m * sizeof(c64), st);
    if (prm->extraction == CBS_HANKEL) {
      // the reduced Hankel eigenpairs are the result only for the Hankel extraction; the
      // Rayleigh-Ritz extraction uses the SVD basis alone
      CBS_TRY(eig(s, m, Bred, m, tau, phi, m, info, st));
      dump("tau", tau, (size_t)m * sizeof(c64), st);
      dump("phi", phi, (size_t)m * m * sizeof(c64), st);
    }

    std::vector<c64> cand;
    c64* basis = nullptr;   // N x ncand candidate vectors (not normalised)
    int ncand = 0;
    const int64_t capv = std::max<int64_t>(2 * m, 1);
    CBS_TRY(ws_get(ws, "ex.vec", (size_t)capv * N, &basis));
    if (prm->extraction == CBS_HANKEL) {
      c64* coef = nullptr;
      CBS_TRY(ws_get(ws, "hk.coef", (size_t)n * m, &coef));
      hipLaunchKernelGGL(k_scale_rows_gemm, dim3(launch_grid((int64_t)n * m)), dim3(256), 0, st, n, m, (const c64*)Wp,
                         (const double*)sig, (const c64*)phi, coef);
      CBS_HIP(hipGetLastError());
      CBS_TRY(tall_gemm(N, n, m, S, N, coef, n, basis, N, st));
      cand.resize(m);
      CBS_HIP(hipMemcpyAsync(cand.data(), tau, m * sizeof(c64), hipMemcpyDeviceToHost, st));
      ncand = m;
    } else {
      // --- Rayleigh-Ritz on Q = orth(S_{<M} W1): shifted Cholesky QR, then two plain passes
      c64 *Qa = nullptr, *Qb = nullptr, *G = nullptr, *Ri = nullptr;
      CBS_TRY(ws_get(ws, "rr.Qa", (size_t)m * N, &Qa));
      CBS_TRY(ws_get(ws, "rr.Qb", (size_t)m * N, &Qb));
      CBS_TRY(ws_get(ws, "rr.G", (size_t)m * m, &G));
      CBS_TRY(ws_get(ws, "rr.Ri", (size_t)m * m, &Ri));
      CBS_TRY(tall_gemm(N, n, m, S, N, Wp, n, Qa, N, st));
      for (int pass = 0; pass < 3; ++pass) {
        CBS_TRY(gram(s, N, m, Qa, N, m, Qa, N, G, m, st));
        double shift = 0;
        if (pass == 0) {
          std::vector<c64> hg((size_t)m * m);
          CBS_HIP(hipMemcpyAsync(hg.data(), G, hg.size() * sizeof(c64), hipMemcpyDeviceToHost, st));
          CBS_HIP(hipStreamSynchronize(st));
          double tr = 0;
          for (int i = 0; i < m; ++i) tr += hg[(size_t)i * m + i].x;
          shift = 11.0 * ((double)N * m + (double)m * (m + 1)) * 1.1102230246251565e-16 * tr;
        }
        CBS_TRY(chol_inv(m, G, m, shift, Ri, info, st));
        CBS_TRY(tall_gemm(N, m, m, Qa, N, Ri, m, Qb, N, st));
        std::swap(Qa, Qb);
      }
      // projected blocks A0 = Q^H (H0-E) Q, A+ = Q^H H+ Q, A- = Q^H H- Q
      c64 *HQ = nullptr, *A3 = nullptr;
      CBS_TRY(ws_get(ws, "rr.HQ", (size_t)3 * m * N, &HQ));
      CBS_TRY(ws_get(ws, "rr.A3", (size_t)3 * m * m, &A3));
      std::vector<c64> one(m, make_double2(1, 0)), zero(m, make_double2(0, 0));
      CBS_TRY(apply_parts_dev(s, E, m, one.data(), zero.data(), zero.data(), Qa, HQ, st));
      CBS_TRY(apply_parts_dev(s, E, m, zero.data(), one.data(), zero.data(), Qa, HQ + (size_t)m * N, st));
      CBS_TRY(apply_parts_dev(s, E, m, zero.data(), zero.data(), one.data(), Qa, HQ + (size_t)2 * m * N, st));
      for (int p = 0; p < 3; ++p)
        CBS_TRY(gram(s, N, m, Qa, N, m, HQ + (size_t)p * m * N, N, A3 + (size_t)p * m * m, m, st));
      const int n2 = 2 * m;
      c64 *X = nullptr, *Bl = nullptr, *th = nullptr, *vv = nullptr;
      CBS_TRY(ws_get(ws, "rr.X", (size_t)n2 * n2, &X));
      CBS_TRY(ws_get(ws, "rr.B", (size_t)n2 * n2, &Bl));
      CBS_TRY(ws_get(ws, "rr.th", (size_t)n2, &th));
      CBS_TRY(ws_get(ws, "rr.vv", (size_t)n2 * n2, &vv));
      const c64 sft = make_double2(0.83 * cos(0.7654), 0.83 * sin(0.7654));
      hipLaunchKernelGGL(k_linearize, dim3(launch_grid((int64_t)n2 * n2)), dim3(256), 0, st, m, (const c64*)A3,
                         (const c64*)(A3 + (size_t)m * m), (const c64*)(A3 + (size_t)2 * m * m), sft, X, Bl);
      CBS_HIP(hipGetLastError());
      dump("Q", Qa, (size_t)m * N * sizeof(c64), st);
      dump("A3", A3, (size_t)3 * m * m * sizeof(c64), st);
      CBS_TRY(lu_solve(n2, X, n2, Bl, n2, n2, info, st));
      dump("Minv", Bl, (size_t)n2 * n2 * sizeof(c64), st);
      CBS_TRY(eig(s, n2, Bl, n2, th, vv, n2, info, st));
      dump("theta", th, (size_t)n2 * sizeof(c64), st);
      std::vector<c64> hth(n2);
      CBS_HIP(hipMemcpyAsync(hth.data(), th, n2 * sizeof(c64), hipMemcpyDeviceToHost, st));
      CBS_HIP(hipStreamSynchronize(st));
      double thmax = 0;
      for (auto& t : hth) thmax = std::max(thmax, sqrt(cabs2<double>(t)));
      // keep finite eigenvalues inside (a slightly widened) annulus; x = top half of v
      std::vector<int32_t> keep;
      const double lmin = prm->lambda_min;
      for (int i = 0; i < n2; ++i) {
        if (!(sqrt(cabs2<double>(hth[i])) > 1e-13 * thmax)) continue;
        const c64 lam = cadd<double>(sft, cdiv<double>(make_double2(1, 0), hth[i]));
        const double a = sqrt(cabs2<double>(lam));
        if (a > lmin * (1 - 1e-9) && a < (1 + 1e-9) / lmin) {
          keep.push_back(i);
          cand.push_back(lam);
        }
      }
      ncand = (int)keep.size();
      if (ncand > 0) {
        int32_t* dkeep = nullptr;
        c64* Xt = nullptr;
        CBS_TRY(ws_get(ws, "rr.keep", (size_t)ncand, &dkeep));
        CBS_TRY(ws_get(ws, "rr.Xt", (size_t)m * ncand, &Xt));
        CBS_HIP(hipMemcpyAsync(dkeep, keep.data(), ncand * sizeof(int32_t), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_gather_cols, dim3(launch_grid((int64_t)m * ncand)), dim3(256), 0, st, m, ncand,
                           (const c64*)vv, n2, (const int32_t*)dkeep, Xt, m);
        CBS_HIP(hipGetLastError());
        CBS_TRY(tall_gemm(N, m, ncand, Qa, N, Xt, m, basis, N, st));
      }
    }
    int32_t hinfo[4];
    CBS_HIP(hipMemcpyAsync(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, st));
    CBS_HIP(hipStreamSynchronize(st));
    if (hinfo[0] != 0) {
      // info[0] = 1: QR iteration did not converge, 2: singular LU pivot, 3: Cholesky QR of
      // the Ritz basis lost positive definiteness
      set_error("extraction: %s", hinfo[0] == 1   ? "QR iteration of the reduced eigenproblem did not converge"
                                  : hinfo[0] == 2 ? "the linearised projected QEP is singular at the shift"
                                                  : "Cholesky QR of the Ritz basis failed");
      return CBS_EEIG;
    }
    if (ncand == 0) return CBS_OK;
    // --- normalise, residuals ||P(lambda) psi||, annulus, sorting
    double* norms = nullptr;
    c64* psi = nullptr;
    c64* Ppsi = nullptr;
    CBS_TRY(ws_get(ws, "ex.norm", (size_t)ncand, &norms));
    CBS_TRY(ws_get(ws, "ex.psi", (size_t)ncand * N, &psi));
    CBS_TRY(ws_get(ws, "ex.Ppsi", (size_t)ncand * N, &Ppsi));
    CBS_TRY(vec_norms(N, ncand, basis, N, norms, true, psi, N, st));
    std::vector<c64> c0(ncand, make_double2(1, 0)), cm(ncand);
    for (int i = 0; i < ncand; ++i) cm[i] = cdiv<double>(make_double2(1, 0), cand[i]);
    CBS_TRY(apply_parts_dev(s, E, ncand, c0.data(), cand.data(), cm.data(), psi, Ppsi, st));
    std::vector<double> rn(ncand);
    CBS_TRY(vec_norms(N, ncand, Ppsi, N, norms, false, nullptr, 0, st));
    CBS_HIP(hipMemcpyAsync(rn.data(), norms, ncand * sizeof(double), hipMemcpyDeviceToHost, st));
    CBS_HIP(hipStreamSynchronize(st));
    if (getenv("CBS_DUMP")) {
      std::string dir = getenv("CBS_DUMP");
      FILE* f = fopen((dir + "/cand.txt").c_str(), "w");
      if (f) {
        fprintf(f, "info %d %d %d %d\n", hinfo[0], hinfo[1], hinfo[2], hinfo[3]);
        for (int i = 0; i < ncand; ++i) fprintf(f, "%.17g %.17g %.6e\n", cand[i].x, cand[i].y, rn[i]);
        fclose(f);
      }
    }
    // operator scale for the spurious-pair filter
    double cs = std::fabs(s->fd[0]);
    for (int m2 = 1; m2 <= s->p; ++m2) cs += 2 * std::fabs(s->fd[m2]);
    const double pscale = 3.0 * 0.5 * cs / (s->h * s->h) + std::fabs(E) + 10.0;
    const double keep_tol = (prm->extraction == CBS_HANKEL ? 1e-2 : 1e-6) * pscale;
    std::vector<int> idx;
    const double lmin = prm->lambda_min;
    for (int i = 0; i < ncand; ++i) {
      const double a = sqrt(cabs2<double>(cand[i]));
      if (!(a > lmin && a < 1.0 / lmin)) continue;   // strict annulus (Eq. 5)
      if (!(rn[i] <= keep_tol)) continue;
      idx.push_back(i);
    }
    // Order: decay |ln|lambda|| (propagating modes first), then the Bloch phase arg(lambda),
    // then |lambda| (the inner partner of a pair lambda, 1/conj(lambda) before the outer
    // one).  Values equal to 1e-9 count as ties, so partners whose |ln|lambda|| differ only
    // by rounding keep a stable order; insertion sort, which needs no strict weak order.
    auto before = [&](int a, int b) {
      const double aa = sqrt(cabs2<double>(cand[a])), ab = sqrt(cabs2<double>(cand[b]));
      const double la = std::fabs(std::log(aa)), lb = std::fabs(std::log(ab));
      if (std::fabs(la - lb) > 1e-9 * (1.0 + std::max(la, lb))) return la < lb;
      const double pa = atan2(cand[a].y, cand[a].x), pb = atan2(cand[b].y, cand[b].x);
      if (std::fabs(pa - pb) > 1e-9) return pa < pb;
      return aa < ab;
    };
    for (size_t i = 1; i < idx.size(); ++i)
      for (size_t j = i; j > 0 && before(idx[j], idx[j - 1]); --j) std::swap(idx[j], idx[j - 1]);
    out.lam.resize(idx.size());
    out.res.resize(idx.size());
    CBS_TRY(ws_get(ws, out_name, std::max<size_t>(idx.size(), 1) * N, &out.vecs));
    for (size_t k = 0; k < idx.size(); ++k) {
      out.lam[k] = cand[idx[k]];
      out.res[k] = rn[idx[k]];
      CBS_HIP(hipMemcpyAsync(out.vecs + k * N, psi + (size_t)idx[k] * N, N * sizeof(c64), hipMemcpyDeviceToDevice, st));
    }
    CBS_HIP(hipStreamSynchronize(st));
    return CBS_OK;
  };
  CBS_TRY(extract_rank(m_hi, "ex.out", out));
  if (m_lo != m_hi) {
    Extracted alt;
    CBS_TRY(extract_rank(m_lo, "ex.out2", alt));
    auto worst = [](const Extracted& x) {
      double w = 0;
      for (double r : x.res) w = std::max(w, r);
      return w;
    };
    if (alt.lam.size() > out.lam.size() || (alt.lam.size() == out.lam.size() && worst(alt) < worst(out)))
      out = std::move(alt);
  }
  return CBS_OK;
}

int32_t store_last(cbs_system* s, double E, const Extracted& ex, hipStream_t st) {
  LastSolve& L = s->last;
  const size_t cnt = ex.lam.size();
  if (L.cap < cnt) {
    if (L.vecs) (void)hipFree(L.vecs);
    L.vecs = nullptr;
    L.cap = 0;
    if (hipMalloc(&L.vecs, std::max<size_t>(cnt, 1) * s->N * sizeof(c64)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("allocation for the stored eigenpairs failed");
      return CBS_ENOMEM;
    }
    L.cap = cnt;
  }
  L.n = (int32_t)cnt;
  L.E = E;
  s->solve_id += 1;
  L.lambda = ex.lam;
  if (cnt) CBS_HIP(hipMemcpyAsync(L.vecs, ex.vecs, cnt * s->N * sizeof(c64), hipMemcpyDeviceToDevice, st));
  return CBS_OK;
}

}  // namespace cbs

using namespace cbs;

extern "C" int32_t cbs_solve(cbs_system* s, double E, const cbs_params* prm, const void* V, int32_t max_eigs,
                             double* lambda, double* resid, void* vecs, int32_t* n_eigs, cbs_info* info,
                             void* stream) {
  if (!s || !V || max_eigs < 0 || (max_eigs > 0 && !lambda) || !n_eigs) {
    set_error("cbs_solve: bad argument");
    return CBS_EINVAL;
  }
  CBS_TRY(check_params(prm, true));
  CBS_HIP(hipSetDevice(s->device));
  hipStream_t st = (hipStream_t)stream;
  std::vector<c64> z1, w1, z2, w2;
  quadrature(prm->lambda_min, prm->n_q, z1, w1, z2, w2);
  const c64* Vc = (const c64*)V;
  int32_t nqs = prm->n_q;
  CBS_TRY(nodes_to_solve(s, prm, &Vc, 1, (int64_t)prm->n_rhs * s->N, st, &nqs));
  NodeSolve ns;
  if (prm->block > 1)
    CBS_TRY(solve_nodes_block(s, E, z1.data(), nqs, prm->n_rhs, Vc, prm, st, ns));
  else
    CBS_TRY(solve_nodes(s, E, z1.data(), nqs, prm->n_rhs, Vc, prm, st, ns));
  Extracted ex;
  double tmom = 0;
  auto t0 = std::chrono::steady_clock::now();
  CBS_TRY(extract(s, E, prm, solve_noise(ns.relres, 0, ns.nruns), Vc, ns.Y, nqs, st, ex, &tmom));
  auto t1 = std::chrono::steady_clock::now();
  CBS_TRY(store_last(s, E, ex, st));
  const int cnt = (int)ex.lam.size();
  *n_eigs = cnt;
  bool noconv = false, brk = false;
  double mx = 0, sum = 0;
  int im = 0;
  for (int r = 0; r < ns.nruns; ++r) {
    noconv = noconv || (ns.status[r] != ST_DONE && ns.status[r] != ST_HALTED);
    brk = brk || ns.status[r] == ST_BREAKDOWN;
    mx = std::max(mx, std::max(ns.relres[2 * r], ns.relres[2 * r + 1]));
    im = std::max(im, ns.iters[r]);
    sum += ns.iters[r];
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->rank = ex.rank;
    info->n_eigs = cnt;
    info->iters_max = im;
    info->iters_mean = sum / std::max(1, ns.nruns);
    info->max_solve_resid = mx;
    double er = 0;
    for (double r : ex.res) er = std::max(er, r);
    info->max_eig_resid = er;
    info->sigma_first = ex.sig1;
    info->sigma_ratio = ex.sig_ratio;
    info->t_solve_ms = ns.ms;
    info->t_moments_ms = tmom;
    info->t_extract_ms = std::chrono::duration<double, std::milli>(t1 - t0).count() - tmom;
    info->matvecs = (int64_t)(2 * sum);
    info->refine_steps = ns.n_ru;
    info->restarts = (int32_t)std::min<int64_t>(ns.restarts, INT32_MAX);
    info->stencil_launches = ns.prof_launches;
    info->stencil_ms = ns.prof_ms;
    info->stencil_bytes = ns.prof_bytes;
    info->stencil_lo_launches = ns.prof_lo_launches;
    info->stencil_lo_ms = ns.prof_lo_ms;
    info->stencil_lo_bytes = ns.prof_lo_bytes;
    info->nodes_solved = nqs;
  }
  int32_t rc = CBS_OK;
  if (cnt > max_eigs) rc = CBS_ETOOMANY;
  else if (brk) rc = CBS_EBREAKDOWN;
  else if (noconv) rc = CBS_ENOCONV;
  else if (ex.rank >= prm->n_rhs * prm->n_mom) rc = CBS_ERANK;
  if (info) info->status = rc;
  if (cnt > max_eigs) {
    set_error("cbs_solve: %d eigenvalues, output holds %d", cnt, max_eigs);
    return CBS_ETOOMANY;
  }
  for (int k = 0; k < cnt; ++k) {
    lambda[2 * k] = ex.lam[k].x;
    lambda[2 * k + 1] = ex.lam[k].y;
    if (resid) resid[k] = ex.res[k];
  }
  if (vecs && cnt)
    CBS_HIP(hipMemcpyAsync(vecs, ex.vecs, (size_t)cnt * s->N * sizeof(c64), hipMemcpyDeviceToDevice, st));
  CBS_HIP(hipStreamSynchronize(st));
  if (brk) {
    set_error("cbs_solve: BiCG breakdown in some runs");
    return CBS_EBREAKDOWN;
  }
  if (noconv) {
    set_error("cbs_solve: some linear solves missed the tolerance");
    return CBS_ENOCONV;
  }
  if (ex.rank >= prm->n_rhs * prm->n_mom) {
    set_error("cbs_solve: Hankel rank %d reached L*M; enlarge L or M", ex.rank);
    return CBS_ERANK;
  }
  return CBS_OK;
}

// ------------------------------------------------------------------ batching
static int severity(int32_t rc) {
  switch (rc) {
    case CBS_EBREAKDOWN: return 6;
    case CBS_ENONFINITE: return 5;
    case CBS_EEIG: return 4;
    case CBS_ENOCONV: return 3;
    case CBS_ETOOMANY: return 2;
    case CBS_ERANK: return 1;
    default: return 0;
  }
}

// Batched solve through the work queue: per system one BiCG solve whose slots take the
// (energy, node, right-hand side) items in turn (bicg.hip); the moments of every energy
// are accumulated as its items finish, then each (system, energy) pair is extracted.
static int32_t solve_batched_queue(int32_t n_sys, cbs_system* const* systems, int32_t n_E, const double* E,
                                   const cbs_params* prm, const void* const* V, int32_t max_eigs, double* lambda,
                                   int32_t* n_eigs, cbs_info* info, hipStream_t st, int nq, double per_pt,
                                   double budget) {
  const int L = prm->n_rhs, M2 = 2 * prm->n_mom;
  const int32_t conj = nq != prm->n_q;
  // device memory: the moments of every energy first, the slots share what is left in
  // proportion to each system's work (items x points)
  double mom_bytes = 0, weight = 0;
  for (int s = 0; s < n_sys; ++s) {
    mom_bytes += (double)n_E * M2 * L * systems[s]->N * 16.0;
    weight += (double)n_E * nq * L * systems[s]->N;
  }
  const double slot_budget = std::max(budget - mom_bytes, 0.0);
  std::vector<c64> ca, cb;
  moment_weights(prm, nq, M2, ca, cb);
  std::vector<c64> z1, w1, z2, w2;
  quadrature(prm->lambda_min, prm->n_q, z1, w1, z2, w2);
  std::vector<BicgSolve> solves(n_sys);
  std::vector<QueueState> qs(n_sys);
  std::vector<BicgSolve*> ptrs;
  int64_t max_total = 0;
  for (int s = 0; s < n_sys; ++s) {
    cbs_system* sy = systems[s];
    const int n_items = n_E * nq * L;
    const double share = slot_budget * ((double)n_items * sy->N / weight);
    int slots = (int)std::min<double>(n_items, std::floor(share / ((double)sy->N * per_pt)));
    if (const char* e = getenv("CBS_QUEUE_SLOTS")) slots = std::min(n_items, std::max(1, atoi(e)));
    if (slots < 1) {
      set_error("cbs_solve_batched: not enough device memory for one run of system %d", s);
      return CBS_ENOMEM;
    }
    std::vector<RunCoef> item_coef;
    for (int e = 0; e < n_E; ++e) {
      std::vector<RunCoef> one;
      node_coefs(z1.data(), nq, 1, E[e], one);
      item_coef.insert(item_coef.end(), one.begin(), one.end());
    }
    BicgSolve& b = solves[s];
    b.sys = sy;
    b.nruns = slots;
    b.L = L;
    b.n_q = nq;
    b.V = (const c64*)V[s];
    configure_solve(b, prm);
    b.coef = nullptr;
    CBS_TRY(bicg_alloc(b, "bicg"));
    QueueState& q = qs[s];
    q.n_items = n_items;
    q.nq = nq;
    q.L = L;
    q.nE = n_E;
    q.M2 = M2;
    q.conj = conj;
    CBS_TRY(queue_alloc(b, q, item_coef, ca, cb, "queue", st));
    ptrs.push_back(&b);
    max_total = std::max<int64_t>(max_total, (int64_t)prm->max_iter * ((n_items + slots - 1) / slots + 1));
    if (getenv("CBS_VERBOSE"))
      fprintf(stderr, "[cbs] queue: system %d, %d items in %d slots\n", s, n_items, slots);
  }
  double ms = 0;
  CBS_TRY(bicg_run(ptrs, st, prm->chunk, (int32_t)std::min<int64_t>(max_total, INT32_MAX / 2), &ms, false));
  int32_t worst = CBS_OK;
  auto note = [&](int32_t rc) {
    if (rc != CBS_OK && (worst == CBS_OK || severity(rc) > severity(worst))) worst = rc;
  };
  for (int s = 0; s < n_sys; ++s) {
    cbs_system* sy = systems[s];
    QueueState& q = qs[s];
    std::vector<int32_t> it(q.n_items), stt(q.n_items);
    std::vector<double> rr(2 * (size_t)q.n_items);
    CBS_HIP(hipMemcpyAsync(it.data(), q.item_iters, it.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CBS_HIP(hipMemcpyAsync(stt.data(), q.item_status, stt.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CBS_HIP(hipMemcpyAsync(rr.data(), q.item_relres, rr.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    CBS_HIP(hipStreamSynchronize(st));
    for (int e = 0; e < n_E; ++e) {
      const int ie = s * n_E + e;
      Extracted ex;
      double tmom = 0;
      auto t0 = std::chrono::steady_clock::now();
      const c64* Se = q.S + (size_t)e * M2 * L * sy->N;
      const int32_t rc = extract_S(sy, E[e], prm, solve_noise(rr, (int64_t)e * nq * L, (int64_t)(e + 1) * nq * L),
                                   (const c64*)V[s], Se, st, ex, &tmom, t0);
      if (rc == CBS_EHIP || rc == CBS_ENOMEM || rc == CBS_EINVAL) return rc;
      bool noconv = false, brk = false;
      double mx = 0, sum = 0;
      int im = 0;
      for (int k = e * nq * L; k < (e + 1) * nq * L; ++k) {
        noconv = noconv || (stt[k] != ST_DONE && stt[k] != ST_HALTED);
        brk = brk || stt[k] == ST_BREAKDOWN;
        mx = std::max(mx, std::max(rr[2 * k], rr[2 * k + 1]));
        im = std::max(im, it[k]);
        sum += it[k];
      }
      if (info) {
        cbs_info& in = info[ie];
        std::memset(&in, 0, sizeof(in));
        in.iters_max = im;
        in.iters_mean = sum / (nq * L);
        in.max_solve_resid = mx;
        in.t_solve_ms = ms;   // shared by the whole batch
        in.t_moments_ms = tmom;
        in.matvecs = (int64_t)(2 * sum);
        in.nodes_solved = nq;
      }
      if (rc != CBS_OK) {
        n_eigs[ie] = 0;
        if (info) info[ie].status = rc;
        note(rc);
        continue;
      }
      auto t1 = std::chrono::steady_clock::now();
      CBS_TRY(store_last(sy, E[e], ex, st));
      const int cnt = (int)ex.lam.size();
      n_eigs[ie] = cnt;
      if (info) {
        cbs_info& in = info[ie];
        in.rank = ex.rank;
        in.n_eigs = cnt;
        for (double r : ex.res) in.max_eig_resid = std::max(in.max_eig_resid, r);
        in.sigma_first = ex.sig1;
        in.sigma_ratio = ex.sig_ratio;
        in.t_extract_ms = std::chrono::duration<double, std::milli>(t1 - t0).count() - tmom;
      }
      int32_t prc = CBS_OK;
      if (cnt > max_eigs) {
        prc = CBS_ETOOMANY;
      } else {
        double* out = lambda + (size_t)ie * 2 * max_eigs;
        for (int k = 0; k < cnt; ++k) {
          out[2 * k] = ex.lam[k].x;
          out[2 * k + 1] = ex.lam[k].y;
        }
        if (brk) prc = CBS_EBREAKDOWN;
        else if (noconv) prc = CBS_ENOCONV;
        else if (ex.rank >= L * prm->n_mom) prc = CBS_ERANK;
      }
      if (info) info[ie].status = prc;
      note(prc);
    }
  }
  CBS_HIP(hipStreamSynchronize(st));
  if (worst != CBS_OK) set_error("cbs_solve_batched: %s in at least one (system, energy) pair", cbs_strerror(worst));
  return worst;
}

// Every (system, energy) pair with the same parameters.  The BiCG runs of all
// energies of a system form one batch (each run carries its own energy), and the
// batches of all systems advance in the same captured graph, so one replay moves
// every quadrature node, right-hand side, energy and grid of the wave.  Energies
// are taken in waves sized to a device-memory budget (CBS_BATCH_BYTES, default 60%
// of the free memory); the extraction then runs per (system, energy).
extern "C" int32_t cbs_solve_batched(int32_t n_sys, cbs_system* const* systems, int32_t n_E, const double* E,
                                     const cbs_params* prm, const void* const* V, int32_t max_eigs, double* lambda,
                                     int32_t* n_eigs, cbs_info* info, void* stream) {
  if (n_sys < 1 || !systems || n_E < 1 || !E || !V || max_eigs < 0 || (max_eigs > 0 && !lambda) || !n_eigs) {
    set_error("cbs_solve_batched: bad argument");
    return CBS_EINVAL;
  }
  CBS_TRY(check_params(prm, true));
  if (prm->block > 1) {
    set_error("cbs_solve_batched: block BiCG runs per (system, energy) through cbs_solve");
    return CBS_EINVAL;
  }
  for (int s = 0; s < n_sys; ++s) {
    if (!systems[s] || !V[s] || systems[s]->device != systems[0]->device) {
      set_error("cbs_solve_batched: null system/V or systems on different devices");
      return CBS_EINVAL;
    }
  }
  CBS_HIP(hipSetDevice(systems[0]->device));
  hipStream_t st = (hipStream_t)stream;
  const int L = prm->n_rhs;
  const bool mixed = prm->precision == CBS_MIXED;
  // conjugate nodes only when every system's right-hand sides are real
  bool halve = true;
  for (int s = 0; s < n_sys; ++s) {
    int32_t q = prm->n_q;
    const c64* Vs = (const c64*)V[s];
    CBS_TRY(nodes_to_solve(systems[s], prm, &Vs, 1, (int64_t)L * systems[s]->N, st, &q));
    halve = halve && q != prm->n_q;
  }
  const int nq = halve ? prm->n_q / 2 : prm->n_q;
  // memory per energy for all systems
  const double per_pt = mixed ? (5 * 16 + 5 * 32 + 32) : (5 * 32 + 32);
  double per_energy = 0;
  for (int s = 0; s < n_sys; ++s) per_energy += (double)systems[s]->N * nq * L * per_pt;
  double budget = 0;
  if (const char* e = getenv("CBS_BATCH_BYTES")) budget = atof(e);
  if (!(budget > 0)) {
    size_t fr = 0, tot = 0;
    CBS_HIP(hipMemGetInfo(&fr, &tot));
    budget = 0.6 * (double)fr;
  }
  // the work queue (default); the energy waves below for the half-of-the-nodes stop (whose
  // groups are whole energies), profiling, or CBS_QUEUE=0
  const char* qenv = getenv("CBS_QUEUE");
  if (!prm->half_stop && !prm->profile && !(qenv && qenv[0] == '0'))
    return solve_batched_queue(n_sys, systems, n_E, E, prm, V, max_eigs, lambda, n_eigs, info, st, nq, per_pt,
                               budget);
  const int wave = std::max(1, std::min(n_E, (int)(budget / per_energy)));
  std::vector<c64> z1, w1, z2, w2;
  quadrature(prm->lambda_min, prm->n_q, z1, w1, z2, w2);
  // overall code: the most severe of the pairs' codes
  int32_t worst = CBS_OK;
  auto note = [&](int32_t rc) {
    if (rc != CBS_OK && (worst == CBS_OK || severity(rc) > severity(worst))) worst = rc;
  };
  for (int e0 = 0; e0 < n_E; e0 += wave) {
    const int ne = std::min(wave, n_E - e0);
    std::vector<BicgSolve> solves(n_sys);
    std::vector<std::vector<RunCoef>> coefs(n_sys);
    std::vector<BicgSolve*> ptrs;
    for (int s = 0; s < n_sys; ++s) {
      cbs_system* sy = systems[s];
      std::vector<RunCoef>& hc = coefs[s];
      for (int e = 0; e < ne; ++e) {
        std::vector<RunCoef> one;
        node_coefs(z1.data(), nq, L, E[e0 + e], one);
        hc.insert(hc.end(), one.begin(), one.end());
      }
      RunCoef* coef = nullptr;
      CBS_TRY(ws_get(sy->ws, "batch.coef", hc.size(), &coef));
      CBS_HIP(hipMemcpyAsync(coef, hc.data(), hc.size() * sizeof(RunCoef), hipMemcpyHostToDevice, st));
      BicgSolve& b = solves[s];
      b.sys = sy;
      b.nruns = ne * nq * L;
      b.L = L;
      b.n_q = nq;
      b.V = (const c64*)V[s];
      b.coef = coef;
      configure_solve(b, prm);
      CBS_TRY(bicg_alloc(b, "bicg"));
      ptrs.push_back(&b);
    }
    double ms = 0;
    CBS_TRY(bicg_run(ptrs, st, prm->chunk, prm->max_iter, &ms, prm->profile != 0));
    for (int s = 0; s < n_sys; ++s) {
      cbs_system* sy = systems[s];
      NodeSolve ns;
      CBS_TRY(bicg_collect(solves[s], ns, st));
      for (int e = 0; e < ne; ++e) {
        const int ie = s * n_E + e0 + e;
        Extracted ex;
        double tmom = 0;
        auto t0 = std::chrono::steady_clock::now();
        const Pair<double>* Ye = ns.Y + (size_t)e * nq * L * sy->N;
        const int32_t rc = extract(sy, E[e0 + e], prm,
                                   solve_noise(ns.relres, (int64_t)e * nq * L, (int64_t)(e + 1) * nq * L),
                                   (const c64*)V[s], Ye, nq, st, ex, &tmom);
        if (rc == CBS_EHIP || rc == CBS_ENOMEM || rc == CBS_EINVAL) return rc;
        if (rc != CBS_OK) {
          // this pair has no eigenpairs (non-finite moments or a failed dense step); the
          // other pairs go on
          n_eigs[ie] = 0;
          if (info) {
            std::memset(&info[ie], 0, sizeof(cbs_info));
            info[ie].status = rc;
            info[ie].nodes_solved = nq;
          }
          note(rc);
          continue;
        }
        auto t1 = std::chrono::steady_clock::now();
        CBS_TRY(store_last(sy, E[e0 + e], ex, st));
        const int cnt = (int)ex.lam.size();
        n_eigs[ie] = cnt;
        bool noconv = false, brk = false;
        double mx = 0, sum = 0;
        int im = 0;
        for (int r = e * nq * L; r < (e + 1) * nq * L; ++r) {
          noconv = noconv || (ns.status[r] != ST_DONE && ns.status[r] != ST_HALTED);
          brk = brk || ns.status[r] == ST_BREAKDOWN;
          mx = std::max(mx, std::max(ns.relres[2 * r], ns.relres[2 * r + 1]));
          im = std::max(im, ns.iters[r]);
          sum += ns.iters[r];
        }
        if (info) {
          cbs_info& in = info[ie];
          std::memset(&in, 0, sizeof(in));
          in.rank = ex.rank;
          in.n_eigs = cnt;
          in.iters_max = im;
          in.iters_mean = sum / (nq * L);
          in.max_solve_resid = mx;
          for (double r : ex.res) in.max_eig_resid = std::max(in.max_eig_resid, r);
          in.sigma_first = ex.sig1;
          in.sigma_ratio = ex.sig_ratio;
          in.t_solve_ms = ms;   // shared by the whole wave
          in.t_moments_ms = tmom;
          in.t_extract_ms = std::chrono::duration<double, std::milli>(t1 - t0).count() - tmom;
          in.matvecs = (int64_t)(2 * sum);
          in.refine_steps = ns.n_ru;
          in.restarts = (int32_t)std::min<int64_t>(ns.restarts, INT32_MAX);
          in.nodes_solved = nq;
        }
        int32_t prc = CBS_OK;
        if (cnt > max_eigs) {
          prc = CBS_ETOOMANY;
        } else {
          double* out = lambda + (size_t)ie * 2 * max_eigs;
          for (int k = 0; k < cnt; ++k) {
            out[2 * k] = ex.lam[k].x;
            out[2 * k + 1] = ex.lam[k].y;
          }
          if (brk) prc = CBS_EBREAKDOWN;
          else if (noconv) prc = CBS_ENOCONV;
          else if (ex.rank >= L * prm->n_mom) prc = CBS_ERANK;
        }
        if (info) info[ie].status = prc;
        note(prc);
      }
    }
  }
  CBS_HIP(hipStreamSynchronize(st));
  if (worst != CBS_OK) set_error("cbs_solve_batched: %s in at least one (system, energy) pair", cbs_strerror(worst));
  return worst;
}

// Complex wave number of a Bloch factor (Sec. 2): lambda = exp(i k a) with a the cell
// length, so k = -i ln(lambda) / a = (arg lambda - i ln|lambda|) / a on the principal
// branch of the logarithm.
extern "C" int32_t cbs_lambda_to_k(int32_t n, const double* lambda, double cell_length, double* k) {
  if (n < 0 || (n > 0 && (!lambda || !k)) || !(cell_length > 0.0) || !std::isfinite(cell_length)) {
    set_error("cbs_lambda_to_k: bad argument");
    return CBS_EINVAL;
  }
  for (int32_t i = 0; i < n; ++i) {
    const double re = lambda[2 * i], im = lambda[2 * i + 1];
    if (!std::isfinite(re) || !std::isfinite(im) || (re == 0.0 && im == 0.0)) {
      set_error("cbs_lambda_to_k: lambda[%d] is zero or not finite", i);
      return CBS_EINVAL;
    }
  }
  for (int32_t i = 0; i < n; ++i) {
    const double re = lambda[2 * i], im = lambda[2 * i + 1];
    k[2 * i] = std::atan2(im, re) / cell_length;
    k[2 * i + 1] = -std::log(std::hypot(re, im)) / cell_length;
  }
  return CBS_OK;
}

// Branches of the complex band structure (Sec. 2; the curves k(E) of the CBS figures of
// Sec. 4.1 and 5): the k of consecutive energies are joined by a greedy assignment on the
// distance to each open branch's linear prediction (Re k compared modulo 2 pi / a).
extern "C" int32_t cbs_connect_branches(int32_t n_E, const double* E, const int32_t* n_k, const double* k,
                                        double cell_length, double max_jump, int32_t* branch,
                                        int32_t* n_branches) {
  if (n_E < 0 || (n_E > 0 && (!E || !n_k)) || !(cell_length > 0.0) || !std::isfinite(cell_length) ||
      !(max_jump > 0.0) || !n_branches) {
    set_error("cbs_connect_branches: bad argument");
    return CBS_EINVAL;
  }
  int64_t total = 0;
  for (int e = 0; e < n_E; ++e) {
    if (n_k[e] < 0 || !std::isfinite(E[e]) || (e > 0 && !(E[e] > E[e - 1]))) {
      set_error("cbs_connect_branches: counts must be >= 0 and energies finite and increasing");
      return CBS_EINVAL;
    }
    total += n_k[e];
  }
  if (total > 0 && (!k || !branch)) {
    set_error("cbs_connect_branches: bad argument");
    return CBS_EINVAL;
  }
  for (int64_t i = 0; i < 2 * total; ++i)
    if (!std::isfinite(k[i])) {
      set_error("cbs_connect_branches: k[%lld] is not finite", (long long)(i / 2));
      return CBS_EINVAL;
    }
  const double period = 2.0 * M_PI / cell_length;
  auto wrap = [&](double d) { return d - period * std::floor(d / period + 0.5); };
  struct Open {
    int id;
    double kr, ki, pr, pi, e, pe;   // last point, previous point (pe < -1e300: none)
  };
  std::vector<Open> open;
  int next_id = 0;
  int64_t off = 0;
  for (int e = 0; e < n_E; ++e) {
    const int n = n_k[e];
    std::vector<int> take(n, -1);
    std::vector<char> used(open.size(), 0);
    // candidate pairs (open branch, new point) within max_jump of the prediction
    struct Cand {
      double d;
      int b, p;
    };
    std::vector<Cand> cand;
    for (size_t b = 0; b < open.size(); ++b) {
      const Open& o = open[b];
      double qr = o.kr, qi = o.ki;
      if (o.pe > -1e300) {
        const double f = (E[e] - o.e) / (o.e - o.pe);
        qr = o.kr + wrap(o.kr - o.pr) * f;
        qi = o.ki + (o.ki - o.pi) * f;
      }
      for (int p = 0; p < n; ++p) {
        const double dr = wrap(k[2 * (off + p)] - qr), di = k[2 * (off + p) + 1] - qi;
        const double d = std::sqrt(dr * dr + di * di);
        if (d <= max_jump) cand.push_back({d, (int)b, p});
      }
    }
    std::stable_sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) { return a.d < b.d; });
    std::vector<Open> nxt;
    for (const Cand& c : cand) {
      if (used[c.b] || take[c.p] >= 0) continue;
      used[c.b] = 1;
      take[c.p] = open[c.b].id;
      const Open& o = open[c.b];
      nxt.push_back({o.id, k[2 * (off + c.p)], k[2 * (off + c.p) + 1], o.kr, o.ki, E[e], o.e});
    }
    for (int p = 0; p < n; ++p) {
      if (take[p] < 0) {
        take[p] = next_id++;
        nxt.push_back({take[p], k[2 * (off + p)], k[2 * (off + p) + 1], 0.0, 0.0, E[e], -1e308});
      }
      branch[off + p] = take[p];
    }
    open.swap(nxt);
    off += n;
  }
  *n_branches = next_id;
  return CBS_OK;
}
