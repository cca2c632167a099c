// Adjoint of the eigenvalues with respect to the local potential.
//
// For a simple eigenvalue lambda with P(lambda) x = 0 and y^H P(lambda) = 0,
// differentiating P(lambda(V); V) x = 0 and projecting on y gives
//     d lambda / d V(r) = - conj(y(r)) x(r) / (y^H P'(lambda) x),  P' = H+ - lambda^-2 H-,
// since V(r) only enters the diagonal of H0.  P(lambda)^H = P(1/conj lambda) (paper
// Sec. 3.2), so y is the right eigenvector of the partner 1/conj(lambda), which lies
// in the same annulus and is returned by the same solve (for |lambda| = 1 it is x
// itself).  The denominator uses the complex128 operator kernels (parts form), the
// gradient itself is one pointwise kernel; the optional vector-Jacobian product
// contracts the per-eigenvalue gradients with the incoming weights in the same pass.
#include <cmath>
#include <vector>

#include "cbs_internal.hpp"
#include "dense.hpp"

namespace cbs {

__global__ void k_grad(int64_t N, int32_t k, const double2* X, const double2* Yl, const double2* den, double2* out,
                       const double2* w, double* vjp) {
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0;
    for (int i = 0; i < k; ++i) {
      const double2 x = X[(int64_t)i * N + n], y = Yl[(int64_t)i * N + n];
      // -conj(y) x / den
      const double2 g = cscale<double>(cdiv<double>(cmulc<double>(y, x), den[i]), -1.0);
      if (out) out[(int64_t)i * N + n] = g;
      if (vjp) {
        const double2 wi = w[i];
        acc += wi.x * g.x + wi.y * g.y;   // Re(w conj(g))
      }
    }
    if (vjp) vjp[n] = acc;
  }
}

}  // namespace cbs

using namespace cbs;

extern "C" int32_t cbs_grad_vloc(cbs_system* s, int32_t n_sel, const int32_t* sel, void* out, const double* weights,
                                 void* vjp, void* stream) {
  if (!s || n_sel < 0 || (n_sel > 0 && !sel) || (!out && !vjp) || (vjp && !weights)) {
    set_error("cbs_grad_vloc: bad argument");
    return CBS_EINVAL;
  }
  const LastSolve& L = s->last;
  if (L.n <= 0 || !L.vecs) {
    set_error("cbs_grad_vloc: no stored solve");
    return CBS_EINVAL;
  }
  if (n_sel == 0) return CBS_OK;
  CBS_HIP(hipSetDevice(s->device));
  hipStream_t st = (hipStream_t)stream;
  const int64_t N = s->N;
  std::vector<int32_t> partner(n_sel);
  for (int k = 0; k < n_sel; ++k) {
    const int i = sel[k];
    if (i < 0 || i >= L.n) {
      set_error("cbs_grad_vloc: index %d out of range (%d eigenpairs)", i, L.n);
      return CBS_EINVAL;
    }
    const double2 li = L.lambda[i];
    const double2 target = cdiv<double>(make_double2(1, 0), cconj<double>(li));
    const double scale = std::sqrt(cabs2<double>(li));
    int best = -1;
    double bd = 1e300;
    for (int j = 0; j < L.n; ++j) {
      const double d = std::sqrt(cabs2<double>(csub<double>(L.lambda[j], target)));
      if (d < bd) {
        bd = d;
        best = j;
      }
    }
    // simple eigenvalue: nothing else within 1e-7 relative of lambda_i or of its partner
    int near_i = 0, near_p = 0;
    for (int j = 0; j < L.n; ++j) {
      near_i += (std::sqrt(cabs2<double>(csub<double>(L.lambda[j], li))) <= 1e-7 * scale) ? 1 : 0;
      near_p += (std::sqrt(cabs2<double>(csub<double>(L.lambda[j], target))) <= 1e-7 * scale) ? 1 : 0;
    }
    if (best < 0 || bd > 1e-7 * scale || near_i != 1 || near_p != 1) {
      set_error("cbs_grad_vloc: eigenvalue %d has no simple partner 1/conj(lambda)", i);
      return CBS_EINVAL;
    }
    partner[k] = best;
  }
  double2 *X = nullptr, *Yl = nullptr, *PX = nullptr, *G = nullptr, *den = nullptr, *w = nullptr;
  CBS_TRY(ws_get(s->ws, "adj.x", (size_t)n_sel * N, &X));
  CBS_TRY(ws_get(s->ws, "adj.y", (size_t)n_sel * N, &Yl));
  CBS_TRY(ws_get(s->ws, "adj.px", (size_t)n_sel * N, &PX));
  CBS_TRY(ws_get(s->ws, "adj.g", (size_t)n_sel * n_sel, &G));
  CBS_TRY(ws_get(s->ws, "adj.den", (size_t)n_sel, &den));
  CBS_TRY(ws_get(s->ws, "adj.w", (size_t)n_sel, &w));
  std::vector<double2> c0(n_sel, make_double2(0, 0)), cp(n_sel, make_double2(1, 0)), cm(n_sel);
  for (int k = 0; k < n_sel; ++k) {
    CBS_HIP(hipMemcpyAsync(X + (size_t)k * N, L.vecs + (size_t)sel[k] * N, N * sizeof(double2),
                           hipMemcpyDeviceToDevice, st));
    CBS_HIP(hipMemcpyAsync(Yl + (size_t)k * N, L.vecs + (size_t)partner[k] * N, N * sizeof(double2),
                           hipMemcpyDeviceToDevice, st));
    const double2 l = L.lambda[sel[k]];
    const double2 inv2 = cdiv<double>(make_double2(1, 0), cmul<double>(l, l));
    cm[k] = make_double2(-inv2.x, -inv2.y);
  }
  // P'(lambda) x = H+ x - lambda^-2 H- x, then y^H P' x (diagonal of a block inner product)
  CBS_TRY(apply_parts_dev(s, L.E, n_sel, c0.data(), cp.data(), cm.data(), X, PX, st));
  CBS_TRY(gram(s, N, n_sel, Yl, N, n_sel, PX, N, G, n_sel, st));
  std::vector<double2> hg((size_t)n_sel * n_sel), hd(n_sel);
  CBS_HIP(hipMemcpyAsync(hg.data(), G, hg.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
  CBS_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < n_sel; ++k) {
    hd[k] = hg[(size_t)k * n_sel + k];
    if (!(cabs2<double>(hd[k]) > 0)) {
      set_error("cbs_grad_vloc: y^H P'(lambda) x vanishes for eigenvalue %d (defective)", sel[k]);
      return CBS_EINVAL;
    }
  }
  CBS_HIP(hipMemcpyAsync(den, hd.data(), n_sel * sizeof(double2), hipMemcpyHostToDevice, st));
  if (vjp) CBS_HIP(hipMemcpyAsync(w, weights, n_sel * sizeof(double2), hipMemcpyHostToDevice, st));
  const int g = (int)std::min<int64_t>((N + 255) / 256, 4096);
  hipLaunchKernelGGL(k_grad, dim3(g), dim3(256), 0, st, N, n_sel, (const double2*)X, (const double2*)Yl,
                     (const double2*)den, (double2*)out, (const double2*)w, (double*)vjp);
  CBS_HIP(hipGetLastError());
  CBS_HIP(hipStreamSynchronize(st));
  return CBS_OK;
}
