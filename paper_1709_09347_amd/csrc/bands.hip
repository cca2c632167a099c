// Conventional band structure on the device: the lowest eigenvalues of the Hermitian
// H(k) = H0 + e^{ika} H+ + e^{-ika} H- at real wave numbers k (paper Sec. 2: a propagating
// Bloch state lambda = e^{ika} of the QEP at energy E is an eigenvector of H(k) with
// eigenvalue E; Sec. 4.1 checks the complex band structure against these bands).
//
// Method: Chebyshev-filtered subspace iteration.  A block of m = n_bands + guard vectors
// is filtered by the Chebyshev polynomial of H(k) that is bounded by 1 on [cut, upper]
// (cut: the largest Ritz value of the block, upper: a bound of the spectrum) and grows
// fast below cut, then orthonormalised (Cholesky QR, three passes, the first shifted) and
// rotated by the Rayleigh-Ritz eigenvectors of Q^H H(k) Q.  The small Hermitian
// eigenproblem uses the one-sided Jacobi SVD of Q^H H Q + s I, positive definite for s
// above its spectral radius, whose right singular vectors are eigenvectors (orthogonal
// also for clustered bands).  The filter uses the scaled three-term recurrence, so the
// block's magnitude stays bounded.  Each band stops when ||H x - theta x|| <= tol
// (|theta| + 1); all operator applications are the complex128 kernels of cbs_apply_parts.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "cbs_internal.hpp"
#include "dense.hpp"

namespace cbs {

using c64 = double2;

// out = alpha (HY - c Y) + beta X (vectors [m][N])
__global__ void k_cheb(int64_t total, const c64* HY, const c64* Y, const c64* X, c64* out, double c, double alpha,
                       double beta) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const c64 hy = HY[g], y = Y[g];
    c64 o = make_double2(alpha * (hy.x - c * y.x), alpha * (hy.y - c * y.y));
    if (X != nullptr) {
      const c64 x = X[g];
      o.x += beta * x.x;
      o.y += beta * x.y;
    }
    out[g] = o;
  }
}

// A' = G + s I for the Hermitian G (m x m, column-major), symmetrised
__global__ void k_shift_herm(int32_t m, const c64* G, double s, c64* A) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < m * m; t += gridDim.x * blockDim.x) {
    const int i = t % m, j = t / m;
    const c64 a = G[i + (int64_t)j * m], b = G[j + (int64_t)i * m];
    c64 v = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    if (i == j) v = make_double2(v.x + s, 0.0);
    A[t] = v;
  }
}

// R = HX - X diag(theta) column norms (partial per column, one block per column)
__global__ void __launch_bounds__(256) k_ritz_res(int64_t N, const c64* HX, const c64* X, const double* theta,
                                                  double* res) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  const double th = theta[j];
  double s = 0;
  for (int64_t n = threadIdx.x; n < N; n += 256) {
    const c64 h = HX[(int64_t)j * N + n], x = X[(int64_t)j * N + n];
    const double rx = h.x - th * x.x, ry = h.y - th * x.y;
    s += rx * rx + ry * ry;
  }
  s = wsum<double>(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) res[j] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

// theta (ascending) and the eigenvector matrix U (columns in that order) from the SVD of
// G + s I: sigma descending with perm, so rank r from the bottom is eigenvalue r
__global__ void k_ritz_order(int32_t m, const double* sigma, const int32_t* perm, const c64* W, double s,
                             double* theta, c64* U) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < m * m; t += gridDim.x * blockDim.x) {
    const int i = t % m, r = t / m;   // row, ascending rank
    const int src = perm[m - 1 - r];
    U[i + (int64_t)r * m] = W[i + (int64_t)src * m];
    if (i == 0) theta[r] = sigma[m - 1 - r] - s;
  }
}

// deterministic start vectors (splitmix64 of the index), complex, unit scale
__global__ void k_start_block(int64_t total, uint64_t seed, c64* X) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(g + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double a = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    const double b = (double)((z << 21) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    X[g] = make_double2(a, b);
  }
}

static int grid_of(int64_t work) { return (int)std::min<int64_t>((work + 255) / 256, 4096); }

// Largest eigenvalue of a symmetric tridiagonal matrix (diagonal a, off-diagonal b) by
// bisection on the Sturm sequence count.
static double tridiag_max(const std::vector<double>& a, const std::vector<double>& b) {
  const int n = (int)a.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto below = [&](double x) {   // eigenvalues below x
    int c = 0;
    double d = 1.0;
    for (int i = 0; i < n; ++i) {
      d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
      if (d == 0.0) d = 1e-300;
      if (d < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-12 * (1.0 + std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) >= n) hi = mid;
    else lo = mid;
  }
  return hi;
}

// Upper bound of the spectrum of the Hermitian H(k) (phase ph = e^{ika}): k steps of
// Lanczos from a fixed start vector give the largest Ritz value theta; theta + |b_k| (the
// last off-diagonal) bounds the spectrum from above for a Lanczos run that has captured
// the top of it; 10% of the spread is added as margin.
static int32_t spectrum_upper(cbs_system* s, c64 ph, hipStream_t st, double* upper) {
  const int64_t N = s->N;
  const int steps = 16;
  c64 *dv = nullptr, *dw = nullptr;
  CBS_TRY(ws_get(s->ws, "bd.lz_v", (size_t)N, &dv));
  CBS_TRY(ws_get(s->ws, "bd.lz_w", (size_t)N, &dw));
  std::vector<c64> v(N), vp(N, make_double2(0, 0)), w(N);
  double nrm = 0;
  for (int64_t n = 0; n < N; ++n) {
    // a fixed, non-smooth start vector
    const double t = std::sin(0.7 * (double)n + 0.3) + 0.5 * std::cos(1.3 * (double)n);
    v[n] = make_double2(t, 0.25 * t);
    nrm += t * t * 1.0625;
  }
  nrm = std::sqrt(nrm);
  for (auto& x : v) x = make_double2(x.x / nrm, x.y / nrm);
  std::vector<double> al, be;
  double beta = 0;
  const c64 one = make_double2(1, 0), phc = make_double2(ph.x, -ph.y);
  for (int k = 0; k < steps; ++k) {
    CBS_HIP(hipMemcpyAsync(dv, v.data(), N * sizeof(c64), hipMemcpyHostToDevice, st));
    CBS_TRY(apply_parts_dev(s, 0.0, 1, &one, &ph, &phc, dv, dw, st));
    CBS_HIP(hipMemcpyAsync(w.data(), dw, N * sizeof(c64), hipMemcpyDeviceToHost, st));
    CBS_HIP(hipStreamSynchronize(st));
    double alpha = 0;
    for (int64_t n = 0; n < N; ++n) alpha += v[n].x * w[n].x + v[n].y * w[n].y;   // Re v^H w
    double bn = 0;
    for (int64_t n = 0; n < N; ++n) {
      w[n].x -= alpha * v[n].x + beta * vp[n].x;
      w[n].y -= alpha * v[n].y + beta * vp[n].y;
      bn += w[n].x * w[n].x + w[n].y * w[n].y;
    }
    al.push_back(alpha);
    beta = std::sqrt(bn);
    if (k + 1 < steps) be.push_back(beta);
    if (!(beta > 0)) break;
    vp = v;
    for (int64_t n = 0; n < N; ++n) v[n] = make_double2(w[n].x / beta, w[n].y / beta);
  }
  be.resize(al.size() > 0 ? al.size() - 1 : 0);
  const double tmax = tridiag_max(al, be);
  double tmin = tmax;
  for (double a : al) tmin = std::min(tmin, a);
  *upper = tmax + std::fabs(beta) + 0.1 * (tmax - tmin);
  return CBS_OK;
}

}  // namespace cbs

using namespace cbs;

extern "C" int32_t cbs_bands(cbs_system* s, int32_t n_k, const double* k, int32_t n_bands, double tol,
                             int32_t max_iter, double* eps, double* resid, void* vecs, int32_t* iters,
                             void* stream) {
  if (!s || n_k < 1 || !k || n_bands < 1 || !eps || !(tol > 0) || max_iter < 1) {
    set_error("cbs_bands: bad argument");
    return CBS_EINVAL;
  }
  for (int i = 0; i < n_k; ++i)
    if (!std::isfinite(k[i])) {
      set_error("cbs_bands: k[%d] is not finite", i);
      return CBS_EINVAL;
    }
  const int guard = std::max(4, (n_bands + 3) / 4);
  int m = n_bands + guard;
  m += m & 1;
  if (m > 256 || (int64_t)m > s->N) {
    set_error("cbs_bands: %d bands need a block of %d vectors (at most 256 and at most N)", n_bands, m);
    return CBS_EINVAL;
  }
  CBS_HIP(hipSetDevice(s->device));
  hipStream_t st = (hipStream_t)stream;
  const int64_t N = s->N;
  Workspace& ws = s->ws;
  c64 *X = nullptr, *Y = nullptr, *Z = nullptr, *HY = nullptr, *G = nullptr, *A = nullptr, *W = nullptr,
      *Ri = nullptr, *U = nullptr;
  double *sig = nullptr, *theta = nullptr, *res = nullptr;
  int32_t *perm = nullptr, *info = nullptr;
  const size_t blk = (size_t)m * N;
  CBS_TRY(ws_get(ws, "bd.X", blk, &X));
  CBS_TRY(ws_get(ws, "bd.Y", blk, &Y));
  CBS_TRY(ws_get(ws, "bd.Z", blk, &Z));
  CBS_TRY(ws_get(ws, "bd.HY", blk, &HY));
  CBS_TRY(ws_get(ws, "bd.G", (size_t)m * m, &G));
  CBS_TRY(ws_get(ws, "bd.A", (size_t)m * m, &A));
  CBS_TRY(ws_get(ws, "bd.W", (size_t)m * m, &W));
  CBS_TRY(ws_get(ws, "bd.Ri", (size_t)m * m, &Ri));
  CBS_TRY(ws_get(ws, "bd.U", (size_t)m * m, &U));
  CBS_TRY(ws_get(ws, "bd.sig", 1024, &sig));
  CBS_TRY(ws_get(ws, "bd.theta", (size_t)m, &theta));
  CBS_TRY(ws_get(ws, "bd.res", (size_t)m, &res));
  CBS_TRY(ws_get(ws, "bd.perm", 512, &perm));
  CBS_TRY(ws_get(ws, "bd.info", 4, &info));
  // lowest local potential (below it lies no band of the local part)
  std::vector<double> vl(N);
  CBS_HIP(hipMemcpyAsync(vl.data(), s->vloc64, N * sizeof(double), hipMemcpyDeviceToHost, st));
  CBS_HIP(hipStreamSynchronize(st));
  const double vmin = *std::min_element(vl.begin(), vl.end());
  const double a_cell = s->nz * s->h;
  const int degree = 16;
  for (int ik = 0; ik < n_k; ++ik) {
    const c64 ph = make_double2(std::cos(k[ik] * a_cell), std::sin(k[ik] * a_cell));
    const c64 phc = make_double2(ph.x, -ph.y);
    double upper = 0;
    CBS_TRY(spectrum_upper(s, ph, st, &upper));
    std::vector<c64> c0(m, make_double2(1, 0)), cp(m, ph), cm(m, phc);
    auto applyH = [&](const c64* in, c64* out) { return apply_parts_dev(s, 0.0, m, c0.data(), cp.data(), cm.data(), in, out, st); };
    // orthonormalise the columns of Y into X (Cholesky QR: a shifted pass, then two plain ones)
    auto orthonormalise = [&](c64* src, c64* dst) -> int32_t {
      c64* a = src;
      c64* b = dst;
      for (int pass = 0; pass < 3; ++pass) {
        CBS_TRY(gram(s, N, m, a, N, m, a, N, G, m, st));
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
        CBS_TRY(tall_gemm(N, m, m, a, N, Ri, m, b, N, st));
        std::swap(a, b);
      }
      // an odd number of passes leaves the result in dst (src is overwritten)
      return CBS_OK;
    };
    // Rayleigh-Ritz on the orthonormal X: theta ascending, X := X U, HY := H X
    auto rayleigh_ritz = [&]() -> int32_t {
      CBS_TRY(applyH(X, HY));
      CBS_TRY(gram(s, N, m, X, N, m, HY, N, G, m, st));
      std::vector<c64> hg((size_t)m * m);
      CBS_HIP(hipMemcpyAsync(hg.data(), G, hg.size() * sizeof(c64), hipMemcpyDeviceToHost, st));
      CBS_HIP(hipStreamSynchronize(st));
      double fro = 0;
      for (auto& v : hg) fro += v.x * v.x + v.y * v.y;
      const double shift = std::sqrt(fro) + 1.0;
      hipLaunchKernelGGL(k_shift_herm, dim3(grid_of((int64_t)m * m)), dim3(256), 0, st, m, (const c64*)G, shift, A);
      CBS_HIP(hipGetLastError());
      CBS_TRY(svd(m, A, m, W, m, sig, perm, st));
      hipLaunchKernelGGL(k_ritz_order, dim3(grid_of((int64_t)m * m)), dim3(256), 0, st, m, (const double*)sig,
                         (const int32_t*)perm, (const c64*)W, shift, theta, U);
      CBS_HIP(hipGetLastError());
      CBS_TRY(tall_gemm(N, m, m, X, N, U, m, Z, N, st));
      std::swap(X, Z);
      CBS_TRY(tall_gemm(N, m, m, HY, N, U, m, Z, N, st));
      std::swap(HY, Z);
      return CBS_OK;
    };
    CBS_HIP(hipMemsetAsync(info, 0, 4 * sizeof(int32_t), st));
    hipLaunchKernelGGL(k_start_block, dim3(grid_of((int64_t)blk)), dim3(256), 0, st, (int64_t)blk,
                       (uint64_t)(0x5EED0000 + ik), Y);
    CBS_HIP(hipGetLastError());
    CBS_TRY(orthonormalise(Y, X));
    CBS_TRY(rayleigh_ritz());
    std::vector<double> hth(m), hres(m);
    int it = 0;
    bool done = false;
    for (; it < max_iter && !done; ++it) {
      CBS_HIP(hipMemcpyAsync(hth.data(), theta, m * sizeof(double), hipMemcpyDeviceToHost, st));
      hipLaunchKernelGGL(k_ritz_res, dim3(m), dim3(256), 0, st, N, (const c64*)HY, (const c64*)X,
                         (const double*)theta, res);
      CBS_HIP(hipGetLastError());
      CBS_HIP(hipMemcpyAsync(hres.data(), res, m * sizeof(double), hipMemcpyDeviceToHost, st));
      CBS_HIP(hipStreamSynchronize(st));
      done = true;
      for (int b = 0; b < n_bands; ++b) done = done && hres[b] <= tol * (std::fabs(hth[b]) + 1.0);
      if (done) break;
      // Chebyshev filter of degree `degree` on [cut, upper], scaled recurrence
      const double cut = hth[m - 1];
      const double low = std::min(hth[0], vmin) - 1.0;
      if (!(cut < upper)) {
        set_error("cbs_bands: %d bands reach the top of the spectrum at k[%d]", n_bands, ik);
        return CBS_EINVAL;
      }
      const double e = 0.5 * (upper - cut), c = 0.5 * (upper + cut);
      double sigma = e / (low - c);
      const double sigma1 = sigma, gamma = 2.0 / sigma1;
      // Y = (H X - c X) sigma1 / e ; H X is HY after the last Rayleigh-Ritz step
      hipLaunchKernelGGL(k_cheb, dim3(grid_of((int64_t)blk)), dim3(256), 0, st, (int64_t)blk, (const c64*)HY,
                         (const c64*)X, (const c64*)nullptr, Y, c, sigma1 / e, 0.0);
      CBS_HIP(hipGetLastError());
      // three-term recurrence over the buffers (prev, cur, next), rotated each step; the
      // starting block X is only read by the first step, so all three take turns
      c64* prev = X;
      c64* cur = Y;
      c64* nxt = Z;
      for (int d = 2; d <= degree; ++d) {
        const double sigma2 = 1.0 / (gamma - sigma);
        CBS_TRY(applyH(cur, HY));
        // next = 2 (H cur - c cur) sigma2 / e - sigma sigma2 prev
        hipLaunchKernelGGL(k_cheb, dim3(grid_of((int64_t)blk)), dim3(256), 0, st, (int64_t)blk, (const c64*)HY,
                           (const c64*)cur, (const c64*)prev, nxt, c, 2.0 * sigma2 / e, -sigma * sigma2);
        CBS_HIP(hipGetLastError());
        c64* freed = prev;
        prev = cur;
        cur = nxt;
        nxt = freed;
        sigma = sigma2;
      }
      // the filtered block is in cur: orthonormalised into nxt, which becomes X
      CBS_TRY(orthonormalise(cur, nxt));
      X = nxt;
      Y = cur;
      Z = prev;
      CBS_TRY(rayleigh_ritz());
    }
    int32_t hinfo[4];
    CBS_HIP(hipMemcpyAsync(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost, st));
    CBS_HIP(hipMemcpyAsync(hth.data(), theta, m * sizeof(double), hipMemcpyDeviceToHost, st));
    hipLaunchKernelGGL(k_ritz_res, dim3(m), dim3(256), 0, st, N, (const c64*)HY, (const c64*)X,
                       (const double*)theta, res);
    CBS_HIP(hipMemcpyAsync(hres.data(), res, m * sizeof(double), hipMemcpyDeviceToHost, st));
    CBS_HIP(hipStreamSynchronize(st));
    if (hinfo[0] != 0) {
      set_error("cbs_bands: Cholesky QR of the filtered block failed at k[%d]", ik);
      return CBS_EEIG;
    }
    for (int b = 0; b < n_bands; ++b) {
      eps[(size_t)ik * n_bands + b] = hth[b];
      if (resid) resid[(size_t)ik * n_bands + b] = hres[b];
    }
    if (iters) iters[ik] = it;
    if (vecs)
      CBS_HIP(hipMemcpyAsync((c64*)vecs + (size_t)ik * n_bands * N, X, (size_t)n_bands * N * sizeof(c64),
                             hipMemcpyDeviceToDevice, st));
    if (!done) {
      CBS_HIP(hipStreamSynchronize(st));
      set_error("cbs_bands: k[%d] not converged in %d filter steps", ik, max_iter);
      return CBS_ENOCONV;
    }
  }
  CBS_HIP(hipStreamSynchronize(st));
  return CBS_OK;
}
