// Dense FP64 pieces of the extraction (paper Sec. 3.1, Algorithm 1):
//  * block inner products C = A^H B of tall vector blocks (moments mu_k = V^H S_k,
//    Gram matrices of the Rayleigh-Ritz basis) on FP64 MFMA, split over the long axis;
//  * tall-skinny products out = A W (Ritz vectors, basis changes);
//  * single-workgroup complex dense kernels for the small matrices (n <= 512):
//    one-sided Jacobi SVD, Hessenberg reduction + shifted QR (Schur form) with
//    eigenvectors, LU with partial pivoting, Cholesky.
// Small matrices are column-major: element (i, j) at a[i + j*lda].
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "cbs_internal.hpp"
#include "dense.hpp"
#include "ranking.hpp"

namespace cbs {

using c64 = double2;

__device__ __forceinline__ c64 zmul(c64 a, c64 b) { return cmul<double>(a, b); }
__device__ __forceinline__ c64 zmulc(c64 a, c64 b) { return cmulc<double>(a, b); }   // conj(a) b
__device__ __forceinline__ c64 zadd(c64 a, c64 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ c64 zsub(c64 a, c64 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ c64 zconj(c64 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ c64 zscale(c64 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double zabs(c64 a) { return hypot(a.x, a.y); }
__device__ __forceinline__ c64 zdiv(c64 a, c64 b) { return cdiv<double>(a, b); }
__device__ __forceinline__ c64 zsqrt(c64 a) {
  const double r = zabs(a);
  if (r == 0.0) return make_double2(0, 0);
  double re = sqrt(0.5 * (r + fabs(a.x)));
  double im = a.y / (2.0 * re);
  if (a.x < 0) {
    const double t = fabs(im);
    im = (a.y >= 0) ? re : -re;
    re = t;
  }
  return make_double2(re, im);
}

// ------------------------------------------------------------------ block inner products
typedef double f64x4 __attribute__((ext_vector_type(4)));

// One 16x16 complex tile of C = A^H B per workgroup (4 waves), over a slice of the long
// axis.  MFMA f64 16x16x4: lane l feeds A[l%16][k=l/16] and B[k=l/16][l%16] and holds
// D[4*v + l/16][l%16], v = 0..3.  The k slot of a lane walks 4 consecutive points of its
// vector over 4 instructions, so each lane streams 64 contiguous bytes per step.
// C_re = Ar^T Br + Ai^T Bi, C_im = Ar^T Bi - Ai^T Br.
__global__ void __launch_bounds__(256) k_gram_mfma(int64_t N, int32_t na, int32_t nb, const c64* A,
                                                   int64_t lda, const c64* B, int64_t ldb, int32_t tiles_b,
                                                   int32_t nsplit, int64_t span, double* part) {
  __shared__ double red[4][2][64][4];
  const int tile = blockIdx.x / nsplit, sp = blockIdx.x - tile * nsplit;
  const int ta = tile / tiles_b, tb = tile - ta * tiles_b;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int row = ta * 16 + (lane & 15);
  const int col = tb * 16 + (lane & 15);
  const int kk = lane >> 4;
  const bool ra = row < na, cb = col < nb;
  const c64* pa = A + (int64_t)(ra ? row : 0) * lda;
  const c64* pb = B + (int64_t)(cb ? col : 0) * ldb;
  const int64_t lo = sp * span, hi = std::min<int64_t>(lo + span, N);
  f64x4 cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
  // each wave takes every 4th block of 16 points
  for (int64_t n0 = lo + wv * 16; n0 < hi; n0 += 64) {
    c64 av[4], bv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t n = n0 + 4 * kk + s;
      const bool ok = n < hi;
      av[s] = (ok && ra) ? pa[n] : make_double2(0, 0);
      bv[s] = (ok && cb) ? pb[n] : make_double2(0, 0);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      cre = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s].x, bv[s].x, cre, 0, 0, 0);
      cre = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s].y, bv[s].y, cre, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s].x, bv[s].y, cim, 0, 0, 0);
      cim = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[s].y, bv[s].x, cim, 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    red[wv][0][lane][v] = cre[v];
    red[wv][1][lane][v] = cim[v];
  }
  __syncthreads();
  if (tid < 64) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double re = red[0][0][tid][v] + red[1][0][tid][v] + red[2][0][tid][v] + red[3][0][tid][v];
      const double im = red[0][1][tid][v] + red[1][1][tid][v] + red[2][1][tid][v] + red[3][1][tid][v];
      const int i = ta * 16 + mfma16_row<double>(tid, v);
      const int j = tb * 16 + (tid & 15);
      if (i < na && j < nb) {
        double* o = part + (((int64_t)sp * na + i) * nb + j) * 2;
        o[0] = re;
        o[1] = im;
      }
    }
  }
}

// Plain reference version of the same tile (no MFMA), selected with CBS_NO_MFMA=1.
__global__ void __launch_bounds__(256) k_gram_plain(int64_t N, int32_t na, int32_t nb, const c64* A,
                                                    int64_t lda, const c64* B, int64_t ldb, int32_t tiles_b,
                                                    int32_t nsplit, int64_t span, double* part) {
  const int tile = blockIdx.x / nsplit, sp = blockIdx.x - tile * nsplit;
  const int ta = tile / tiles_b, tb = tile - ta * tiles_b;
  const int i = ta * 16 + (threadIdx.x >> 4), j = tb * 16 + (threadIdx.x & 15);
  const int64_t lo = sp * span, hi = std::min<int64_t>(lo + span, N);
  if (i >= na || j >= nb) return;
  c64 acc = make_double2(0, 0);
  for (int64_t n = lo; n < hi; ++n) acc = zadd(acc, zmulc(A[(int64_t)i * lda + n], B[(int64_t)j * ldb + n]));
  double* o = part + (((int64_t)sp * na + i) * nb + j) * 2;
  o[0] = acc.x;
  o[1] = acc.y;
}

__global__ void k_gram_reduce(int32_t na, int32_t nb, int32_t nsplit, const double* part, c64* C, int64_t ldc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= na * nb) return;
  const int i = t / nb, j = t - i * nb;
  double re = 0, im = 0;
  for (int s = 0; s < nsplit; ++s) {
    const double* o = part + (((int64_t)s * na + i) * nb + j) * 2;
    re += o[0];
    im += o[1];
  }
  C[i + (int64_t)j * ldc] = make_double2(re, im);
}

static bool no_mfma() {
  const char* e = getenv("CBS_NO_MFMA");
  return e && e[0] == '1';
}

int32_t gram(cbs_system* s, int64_t N, int32_t na, const c64* A, int64_t lda, int32_t nb, const c64* B,
             int64_t ldb, c64* C, int64_t ldc, hipStream_t st) {
  if (na <= 0 || nb <= 0) return CBS_OK;
  const int tiles_a = (na + 15) / 16, tiles_b = (nb + 15) / 16;
  const int tiles = tiles_a * tiles_b;
  int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>((2048 + tiles - 1) / tiles, (N + 255) / 256));
  const int64_t span = ((N + nsplit - 1) / nsplit + 63) / 64 * 64;
  nsplit = (int)((N + span - 1) / span);
  double* part = nullptr;
  CBS_TRY(ws_get(s->ws, "gram.part", (size_t)nsplit * na * nb * 2, &part));
  if (no_mfma())
    hipLaunchKernelGGL(k_gram_plain, dim3(tiles * nsplit), dim3(256), 0, st, N, na, nb, A, lda, B, ldb, tiles_b,
                       nsplit, span, part);
  else
    hipLaunchKernelGGL(k_gram_mfma, dim3(tiles * nsplit), dim3(256), 0, st, N, na, nb, A, lda, B, ldb, tiles_b,
                       nsplit, span, part);
  CBS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_gram_reduce, dim3((na * nb + 255) / 256), dim3(256), 0, st, na, nb, nsplit,
                     (const double*)part, C, ldc);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

// ------------------------------------------------------------------ tall-skinny product
// out[c][n] = sum_k A[k][n] W[k + c*ldw] for c < nc; W staged in LDS per column tile.
constexpr int TG_C = 16;
__global__ void __launch_bounds__(256) k_tall_gemm(int64_t N, int32_t K, int32_t nc, const c64* A, int64_t lda,
                                                   const c64* W, int32_t ldw, c64* out, int64_t ldo) {
  extern __shared__ c64 w_s[];   // [K][TG_C]
  const int c0 = blockIdx.y * TG_C;
  const int ncl = std::min(TG_C, nc - c0);
  for (int t = threadIdx.x; t < K * TG_C; t += blockDim.x) {
    const int k = t / TG_C, c = t - k * TG_C;
    w_s[t] = (c < ncl) ? W[k + (int64_t)(c0 + c) * ldw] : make_double2(0, 0);
  }
  __syncthreads();
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
    c64 acc[TG_C];
#pragma unroll
    for (int c = 0; c < TG_C; ++c) acc[c] = make_double2(0, 0);
    for (int k = 0; k < K; ++k) {
      const c64 a = A[(int64_t)k * lda + n];
#pragma unroll
      for (int c = 0; c < TG_C; ++c) acc[c] = zadd(acc[c], zmul(a, w_s[k * TG_C + c]));
    }
    for (int c = 0; c < ncl; ++c) out[(int64_t)(c0 + c) * ldo + n] = acc[c];
  }
}

int32_t tall_gemm(int64_t N, int32_t K, int32_t nc, const c64* A, int64_t lda, const c64* W, int32_t ldw, c64* out,
                  int64_t ldo, hipStream_t st) {
  if (nc <= 0 || N <= 0) return CBS_OK;
  const size_t smem = (size_t)K * TG_C * sizeof(c64);
  if (smem > 64 * 1024) {
    set_error("tall_gemm: inner dimension %d too large", K);
    return CBS_EINVAL;
  }
  const int gx = (int)std::min<int64_t>((N + 255) / 256, 2048);
  hipLaunchKernelGGL(k_tall_gemm, dim3(gx, (nc + TG_C - 1) / TG_C), dim3(256), smem, st, N, K, nc, A, lda, W, ldw,
                     out, ldo);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

// ------------------------------------------------------------------ single-workgroup helpers
constexpr int SWG = 256;   // threads of the single-workgroup kernels

template <int WG>
__device__ double block_max_wg(double v, double* sh) {
  v = fmax(v, __shfl_xor(v, 1, 64));
  for (int o = 2; o < 64; o <<= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
  for (int w = 1; w < WG / 64; ++w) r = fmax(r, sh[w]);
  __syncthreads();
  return r;
}

__device__ double block_max(double v, double* sh) { return block_max_wg<SWG>(v, sh); }

__device__ double block_sum(double v, double* sh) {
  for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0;
  for (int w = 0; w < SWG / 64; ++w) r += sh[w];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------ one-sided Jacobi SVD
// A (n x n, lda) is overwritten by U*Sigma, V starts as the identity and becomes W with
// A_in W = U Sigma.  Columns are paired round-robin (slot 0 fixed, the others rotating by
// one per round, so the slot of every column follows from the round number); each round's
// n/2 disjoint pairs are handled by groups of JWG/(n/2) threads.  Output: sigma sorted
// descending (perm gives the source column of each sorted position), U columns normalised
// in place.
constexpr int JWG = 1024;
__global__ void __launch_bounds__(JWG) k_jacobi_svd(int32_t n, c64* A, int32_t lda, c64* V, int32_t ldv,
                                                     double* sigma, int32_t* perm, int32_t max_sweeps) {
  __shared__ double sh[JWG / 64];
  __shared__ double sflag;
  const int tid = threadIdx.x;
  for (int t = tid; t < n * n; t += JWG) {
    const int i = t % n, j = t / n;
    V[i + (int64_t)j * ldv] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  const int m = (n + 1) / 2 * 2;   // even number of slots (a dummy column when n is odd)
  __syncthreads();
  const int npairs = m / 2;
  int gsize = 1;   // threads per pair: a power of two, so xor shuffles stay inside the group
  while (gsize * 2 * npairs <= JWG && gsize < 64) gsize *= 2;
  // column in slot k after r rotations: slot 0 holds column 0, slot k >= 1 holds
  // column 1 + ((k - 1 - r) mod (m - 1))
  auto slot_col = [&](int k, int r) {
    if (k == 0) return 0;
    int c = (k - 1 - r) % (m - 1);
    if (c < 0) c += m - 1;
    return 1 + c;
  };
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double offmax = 0;
    for (int round = 0; round < m - 1; ++round) {
      // pairs of this round: (slot k, slot m-1-k)
      for (int pidx = tid / gsize; pidx < npairs; pidx += JWG / gsize) {
        const int sub = tid % gsize;
        int p = slot_col(pidx, round), q = slot_col(m - 1 - pidx, round);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double al = 0, be = 0;
        c64 ga = make_double2(0, 0);
        if (q < n) {
#pragma unroll 4
          for (int i = sub; i < n; i += gsize) {
            const c64 ap = A[i + (int64_t)p * lda], aq = A[i + (int64_t)q * lda];
            al += cabs2<double>(ap);
            be += cabs2<double>(aq);
            ga = zadd(ga, zmulc(ap, aq));
          }
        }
        // reduce inside the group (groups are contiguous lanes; gsize divides 64 or is a multiple)
        for (int o = 1; o < gsize; o <<= 1) {
          al += __shfl_xor(al, o, 64);
          be += __shfl_xor(be, o, 64);
          ga.x += __shfl_xor(ga.x, o, 64);
          ga.y += __shfl_xor(ga.y, o, 64);
        }
        if (q >= n) continue;
        const double g = zabs(ga);
        if (!(g > 1e-15 * sqrt(al * be)) || g == 0.0) continue;
        offmax = fmax(offmax, g / sqrt(al * be));
        const double zeta = (be - al) / (2.0 * g);
        const double t = ((zeta >= 0) ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
        const c64 e = make_double2(ga.x / g, -ga.y / g);   // e^{-i phi}
        // two rows at a time: all their loads are issued before the first store (the
        // compiler cannot tell that the stores do not alias the next rows' loads)
        for (int i0 = sub; i0 < n; i0 += 2 * gsize) {
          c64 ap[2], aq[2], vp[2], vq[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int i = min(i0 + u * gsize, n - 1);
            ap[u] = A[i + (int64_t)p * lda];
            aq[u] = A[i + (int64_t)q * lda];
            vp[u] = V[i + (int64_t)p * ldv];
            vq[u] = V[i + (int64_t)q * ldv];
          }
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int i = i0 + u * gsize;
            if (i >= n) break;
            const c64 aqe = zmul(e, aq[u]), vqe = zmul(e, vq[u]);
            A[i + (int64_t)p * lda] = zsub(zscale(ap[u], c), zscale(aqe, sn));
            A[i + (int64_t)q * lda] = zadd(zscale(ap[u], sn), zscale(aqe, c));
            V[i + (int64_t)p * ldv] = zsub(zscale(vp[u], c), zscale(vqe, sn));
            V[i + (int64_t)q * ldv] = zadd(zscale(vp[u], sn), zscale(vqe, c));
          }
        }
      }
      __syncthreads();
    }
    const double om = block_max_wg<JWG>(offmax, sh);
    if (tid == 0) sflag = om;
    __syncthreads();
    if (sflag < 1e-13) break;
  }
  // column norms, sort descending (simple selection by rank)
  for (int j = tid; j < n; j += JWG) {
    double s2 = 0;
    for (int i = 0; i < n; ++i) s2 += cabs2<double>(A[i + (int64_t)j * lda]);
    sigma[512 + j] = sqrt(s2);   // scratch area after the output
  }
  __syncthreads();
  // ranks under a strict total order (ranking.hpp), so perm is a permutation of 0..n-1
  // whatever the values are
  for (int j = tid; j < n; j += JWG) perm[desc_rank(n, sigma + 512, j)] = j;
  __syncthreads();
  for (int r = tid; r < n; r += JWG) sigma[r] = sigma[512 + perm[r]];
  __syncthreads();
  // normalise U columns
  for (int j = tid; j < n; j += JWG) {
    const double sj = sigma[512 + j];
    if (sj > 0)
      for (int i = 0; i < n; ++i) A[i + (int64_t)j * lda] = zscale(A[i + (int64_t)j * lda], 1.0 / sj);
  }
}

// ------------------------------------------------------------------ block one-sided Jacobi SVD
// The same factorisation A W = U Sigma, with the columns in nb blocks of bs: blocks are
// paired round-robin (as the columns above), one workgroup per block pair copies the pair's
// 2 bs columns of A and of W into LDS, runs one full one-sided Jacobi sweep over them (every
// column pair, round-robin inside the pair) and writes them back.  nb - 1 launches make an
// outer sweep; the largest |a_p^H a_q| / (|a_p| |a_q|) of the sweep decides convergence.  The
// single-workgroup kernel above moves both matrices through one CU's caches every round;
// here the rotations run in LDS on nb / 2 CUs.
__global__ void k_svd_init(int32_t n, c64* V, int32_t ldv, unsigned long long* flag) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n * n; t += gridDim.x * blockDim.x) {
    const int i = t % n, j = t / n;
    V[i + (int64_t)j * ldv] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0ull;
}

// slot k of nslots after r rotations holds: slot 0 item 0, slot k >= 1 item
// 1 + ((k - 1 - r) mod (nslots - 1))
__device__ __forceinline__ int rr_slot(int k, int r, int nslots) {
  if (k == 0) return 0;
  int c = (k - 1 - r) % (nslots - 1);
  if (c < 0) c += nslots - 1;
  return 1 + c;
}

constexpr int BJ_THREADS = 1024;
constexpr size_t BJ_LDS = 128 * 1024;   // the block pair's columns of A and W

__global__ void __launch_bounds__(BJ_THREADS) k_svd_block(int32_t n, int32_t bs, int32_t nb, int32_t round, c64* A,
                                                          int32_t lda, c64* V, int32_t ldv,
                                                          unsigned long long* flag) {
  __shared__ c64 bj_lds[BJ_LDS / sizeof(c64)];
  __shared__ double sh[BJ_THREADS / 64];
  c64* la = bj_lds;                       // [2 bs][n]
  c64* lv = la + (size_t)2 * bs * n;      // [2 bs][n]
  int bp = rr_slot(blockIdx.x, round, nb), bq = rr_slot(nb - 1 - blockIdx.x, round, nb);
  const int tid = threadIdx.x;
  const int cols = 2 * bs;
  // local column c: block bp's columns first, then bq's; columns at or past n are padding
  auto gcol = [&](int c) { return (c < bs) ? bp * bs + c : bq * bs + (c - bs); };
  for (int t = tid; t < cols * n; t += BJ_THREADS) {
    const int c = t / n, i = t - c * n;
    const int g = gcol(c);
    la[t] = (g < n) ? A[i + (int64_t)g * lda] : make_double2(0, 0);
    lv[t] = (g < n) ? V[i + (int64_t)g * ldv] : make_double2(0, 0);
  }
  __syncthreads();
  // threads per column pair: a power of two up to 64 (one wave), bs pairs per inner round
  int gsize = 64;
  while (gsize * bs > BJ_THREADS) gsize >>= 1;
  const int pidx = tid / gsize, sub = tid % gsize;
  double offmax = 0;
  for (int ir = 0; ir < cols - 1; ++ir) {
    if (pidx < bs) {
      int p = rr_slot(pidx, ir, cols), q = rr_slot(cols - 1 - pidx, ir, cols);
      if (p > q) {
        const int t = p;
        p = q;
        q = t;
      }
      const bool valid = gcol(p) < n && gcol(q) < n;
      c64* ap = la + (size_t)p * n;
      c64* aq = la + (size_t)q * n;
      double al = 0, be = 0;
      c64 ga = make_double2(0, 0);
      if (valid) {
        for (int i = sub; i < n; i += gsize) {
          const c64 x = ap[i], y = aq[i];
          al += cabs2<double>(x);
          be += cabs2<double>(y);
          ga = zadd(ga, zmulc(x, y));
        }
      }
      for (int o = 1; o < gsize; o <<= 1) {
        al += __shfl_xor(al, o, 64);
        be += __shfl_xor(be, o, 64);
        ga.x += __shfl_xor(ga.x, o, 64);
        ga.y += __shfl_xor(ga.y, o, 64);
      }
      const double g = zabs(ga);
      if (valid && g > 1e-15 * sqrt(al * be) && g != 0.0) {
        offmax = fmax(offmax, g / sqrt(al * be));
        const double zeta = (be - al) / (2.0 * g);
        const double t = ((zeta >= 0) ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
        const c64 e = make_double2(ga.x / g, -ga.y / g);   // e^{-i phi}
        c64* vp = lv + (size_t)p * n;
        c64* vq = lv + (size_t)q * n;
        for (int i = sub; i < n; i += gsize) {
          const c64 x = ap[i], y = zmul(e, aq[i]);
          ap[i] = zsub(zscale(x, c), zscale(y, sn));
          aq[i] = zadd(zscale(x, sn), zscale(y, c));
          const c64 u = vp[i], w = zmul(e, vq[i]);
          vp[i] = zsub(zscale(u, c), zscale(w, sn));
          vq[i] = zadd(zscale(u, sn), zscale(w, c));
        }
      }
    }
    __syncthreads();
  }
  for (int t = tid; t < cols * n; t += BJ_THREADS) {
    const int c = t / n, i = t - c * n;
    const int g = gcol(c);
    if (g < n) {
      A[i + (int64_t)g * lda] = la[t];
      V[i + (int64_t)g * ldv] = lv[t];
    }
  }
  const double om = block_max_wg<BJ_THREADS>(offmax, sh);
  // values are non-negative, so their bit patterns order like the values
  if (tid == 0 && om > 0) atomicMax(flag, (unsigned long long)__double_as_longlong(om));
}

// column norms, sigma sorted descending with its permutation, U columns normalised (the
// tail of the single-workgroup kernel)
__global__ void __launch_bounds__(JWG) k_svd_finish(int32_t n, c64* A, int32_t lda, double* sigma, int32_t* perm) {
  const int tid = threadIdx.x;
  for (int j = tid; j < n; j += JWG) {
    double s2 = 0;
    for (int i = 0; i < n; ++i) s2 += cabs2<double>(A[i + (int64_t)j * lda]);
    sigma[512 + j] = sqrt(s2);
  }
  __syncthreads();
  for (int j = tid; j < n; j += JWG) perm[desc_rank(n, sigma + 512, j)] = j;
  __syncthreads();
  for (int r = tid; r < n; r += JWG) sigma[r] = sigma[512 + perm[r]];
  __syncthreads();
  for (int j = tid; j < n; j += JWG) {
    const double sj = sigma[512 + j];
    if (sj > 0)
      for (int i = 0; i < n; ++i) A[i + (int64_t)j * lda] = zscale(A[i + (int64_t)j * lda], 1.0 / sj);
  }
}

// ------------------------------------------------------------------ small GEMM (one workgroup)
// C = op(A) * B (+ scale of columns), op = identity or conjugate transpose.
__global__ void __launch_bounds__(SWG) k_small_gemm(int32_t m, int32_t n, int32_t k, const c64* A, int32_t lda,
                                                     int32_t transA, const c64* B, int32_t ldb, c64* C,
                                                     int32_t ldc, const double* colscale, const int32_t* bperm) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < m * n; t += gridDim.x * blockDim.x) {
    const int i = t % m, j = t / m;
    const int jb = bperm ? bperm[j] : j;
    c64 acc = make_double2(0, 0);
    for (int l = 0; l < k; ++l) {
      const c64 a = transA ? zconj(A[l + (int64_t)i * lda]) : A[i + (int64_t)l * lda];
      acc = zadd(acc, zmul(a, B[l + (int64_t)jb * ldb]));
    }
    if (colscale) acc = zscale(acc, colscale[j]);
    C[i + (int64_t)j * ldc] = acc;
  }
}

int32_t small_gemm(int32_t m, int32_t n, int32_t k, const c64* A, int32_t lda, bool transA, const c64* B,
                   int32_t ldb, c64* C, int32_t ldc, const double* colscale, const int32_t* bperm, hipStream_t st) {
  if (m <= 0 || n <= 0) return CBS_OK;
  const int g = std::min(1024, (m * n + 255) / 256);
  hipLaunchKernelGGL(k_small_gemm, dim3(g), dim3(256), 0, st, m, n, k, A, lda, (int32_t)transA, B, ldb, C, ldc,
                     colscale, bperm);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

// ------------------------------------------------------------------ eigen-decomposition
// Complex Schur form by Householder reduction to Hessenberg form and single-shift QR
// with Wilkinson shifts and deflation; eigenvectors by back substitution on the
// triangular factor and the accumulated unitary Z.  A (n x n) is destroyed; w receives
// the eigenvalues, Vout the unit-norm eigenvectors.  work: n*n (Z) + n*n (Y).
__global__ void __launch_bounds__(SWG) k_eig(int32_t n, c64* H, int32_t ldh, c64* w, c64* Vout, int32_t ldv,
                                              c64* Z, c64* Y, int32_t* info) {
  __shared__ double sh[SWG / 64];
  __shared__ c64 sv[512];
  __shared__ c64 sg[1];
  __shared__ c64 sxy[2];   // (x, y) of the next Givens rotation of the sweep
  __shared__ int s_lo, s_hi, s_iter, s_done;
  const int tid = threadIdx.x;
  for (int t = tid; t < n * n; t += SWG) {
    const int i = t % n, j = t / n;
    Z[i + (int64_t)j * n] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // --- Householder reduction to upper Hessenberg form
  for (int k = 0; k + 2 < n; ++k) {
    double nx2 = 0;
    for (int i = k + 1 + tid; i < n; i += SWG) nx2 += cabs2<double>(H[i + (int64_t)k * ldh]);
    nx2 = block_sum(nx2, sh);
    const c64 x0 = H[k + 1 + (int64_t)k * ldh];
    const double nx = sqrt(nx2);
    if (nx == 0.0) continue;
    const double a0 = zabs(x0);
    const c64 ph = (a0 > 0) ? make_double2(x0.x / a0, x0.y / a0) : make_double2(1, 0);
    const c64 alpha = zscale(ph, -nx);   // new subdiagonal value
    // v = x - alpha e1, normalised
    for (int i = k + 1 + tid; i < n; i += SWG) {
      c64 v = H[i + (int64_t)k * ldh];
      if (i == k + 1) v = zsub(v, alpha);
      sv[i] = v;
    }
    __syncthreads();
    double vn2 = 0;
    for (int i = k + 1 + tid; i < n; i += SWG) vn2 += cabs2<double>(sv[i]);
    vn2 = block_sum(vn2, sh);
    if (vn2 == 0.0) continue;
    const double inv = 1.0 / sqrt(vn2);
    for (int i = k + 1 + tid; i < n; i += SWG) sv[i] = zscale(sv[i], inv);
    __syncthreads();
    // left: H[k+1:, j] -= 2 v (v^H H[k+1:, j]) for j >= k
    for (int j = k + tid; j < n; j += SWG) {
      c64 d = make_double2(0, 0);
      for (int i = k + 1; i < n; ++i) d = zadd(d, zmulc(sv[i], H[i + (int64_t)j * ldh]));
      d = zscale(d, 2.0);
      for (int i = k + 1; i < n; ++i) H[i + (int64_t)j * ldh] = zsub(H[i + (int64_t)j * ldh], zmul(sv[i], d));
    }
    __syncthreads();
    // right: H[i, k+1:] -= 2 (H[i, k+1:] v) v^H for all i; same for Z
    for (int i = tid; i < 2 * n; i += SWG) {
      c64* M = (i < n) ? H : Z;
      const int r = (i < n) ? i : i - n;
      const int ld = (i < n) ? ldh : n;
      c64 d = make_double2(0, 0);
      for (int j = k + 1; j < n; ++j) d = zadd(d, zmul(M[r + (int64_t)j * ld], sv[j]));
      d = zscale(d, 2.0);
      for (int j = k + 1; j < n; ++j) M[r + (int64_t)j * ld] = zsub(M[r + (int64_t)j * ld], zmul(d, zconj(sv[j])));
    }
    __syncthreads();
    for (int i = k + 2 + tid; i < n; i += SWG) H[i + (int64_t)k * ldh] = make_double2(0, 0);
    __syncthreads();
  }
  // --- shifted QR on the Hessenberg matrix (full Schur form)
  if (tid == 0) {
    s_hi = n - 1;
    s_iter = 0;
    s_done = 0;
  }
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  int total_iter = 0;
  while (true) {
    if (tid == 0) {
      int hi = s_hi;
      while (hi >= 0) {
        if (hi == 0) {
          w[0] = H[0];
          hi = -1;
          break;
        }
        int l = hi;
        while (l > 0) {
          const double sd = zabs(H[l + (int64_t)(l - 1) * ldh]);
          const double dd = zabs(H[l + (int64_t)l * ldh]) + zabs(H[l - 1 + (int64_t)(l - 1) * ldh]);
          if (sd <= eps * dd || sd < 1e-300) break;
          --l;
        }
        if (l > 0) H[l + (int64_t)(l - 1) * ldh] = make_double2(0, 0);
        if (l == hi) {
          w[hi] = H[hi + (int64_t)hi * ldh];
          --hi;
          s_iter = 0;
          continue;
        }
        // shift from the trailing 2x2 block of the active window [l, hi]
        const c64 a = H[hi - 1 + (int64_t)(hi - 1) * ldh], b = H[hi - 1 + (int64_t)hi * ldh];
        const c64 c = H[hi + (int64_t)(hi - 1) * ldh], d = H[hi + (int64_t)hi * ldh];
        c64 mu;
        if (s_iter > 0 && s_iter % 11 == 0) {
          mu = zadd(d, make_double2(0.75 * zabs(c), 0.0));   // exceptional shift
        } else {
          const c64 hd = zscale(zsub(a, d), 0.5);
          const c64 disc = zsqrt(zadd(zmul(hd, hd), zmul(b, c)));
          const c64 m1 = zadd(zscale(zadd(a, d), 0.5), disc), m2 = zsub(zscale(zadd(a, d), 0.5), disc);
          mu = (zabs(zsub(m1, d)) < zabs(zsub(m2, d))) ? m1 : m2;
        }
        sg[0] = mu;
        s_lo = l;
        sxy[0] = zsub(H[l + (int64_t)l * ldh], mu);
        sxy[1] = H[l + 1 + (int64_t)l * ldh];
        break;
      }
      s_hi = hi;
      if (hi < 0) s_done = 1;
    }
    __syncthreads();
    if (s_done) break;
    if (++total_iter > 60 * n) {
      if (tid == 0) info[0] = 1;   // QR failed to converge
      break;
    }
    const int lo = s_lo, hi = s_hi;
    const c64 mu = sg[0];
    if (tid == 0) s_iter = s_iter + 1;
    // implicit single-shift sweep: Givens rotations chase the bulge from lo to hi.  The
    // pair (x, y) that defines rotation k comes from the column update of rotation k-1
    // (rows k and k+1 of column k-1, through LDS), so every thread forms (c, s) itself.
    for (int k = lo; k < hi; ++k) {
      const c64 x = sxy[0], y = sxy[1];
      const double nx = zabs(x), ny = zabs(y);
      const double r = hypot(nx, ny);
      double c;   // G = [[c, s], [-conj(s), c]] with c real: G [x; y] = [r'; 0]
      c64 s;
      if (r == 0.0) {
        c = 1.0;
        s = make_double2(0, 0);
      } else if (nx == 0.0) {
        c = 0.0;
        s = zscale(zconj(y), 1.0 / ny);
      } else {
        c = nx / r;
        const c64 ux = make_double2(x.x / nx, x.y / nx);   // phase of x
        s = zscale(zmul(ux, zconj(y)), 1.0 / r);
      }
      // rows k, k+1: [hk; hk1] <- [c hk + s hk1; -conj(s) hk + c hk1], columns max(k-1,0)..n-1
      const int j0 = (k > lo) ? k - 1 : lo;
      for (int j = j0 + tid; j < n; j += SWG) {
        const c64 hk = H[k + (int64_t)j * ldh], hk1 = H[k + 1 + (int64_t)j * ldh];
        H[k + (int64_t)j * ldh] = zadd(zscale(hk, c), zmul(s, hk1));
        H[k + 1 + (int64_t)j * ldh] = zsub(zscale(hk1, c), zmul(zconj(s), hk));
      }
      __syncthreads();
      // columns k, k+1 of H (rows 0..min(k+2, hi)) and of Z: M G^H
      const int rmax = std::min(k + 2, hi);
      for (int i = tid; i <= rmax + n; i += SWG) {
        c64* M;
        int r2, ld;
        if (i <= rmax) {
          M = H;
          r2 = i;
          ld = ldh;
        } else {
          M = Z;
          r2 = i - rmax - 1;
          ld = n;
          if (r2 >= n) continue;
        }
        const c64 mk = M[r2 + (int64_t)k * ld], mk1 = M[r2 + (int64_t)(k + 1) * ld];
        const c64 nk = zadd(zscale(mk, c), zmul(zconj(s), mk1));
        M[r2 + (int64_t)k * ld] = nk;
        M[r2 + (int64_t)(k + 1) * ld] = zsub(zscale(mk1, c), zmul(s, mk));
        if (i <= rmax && r2 == k + 1) sxy[0] = nk;   // x of rotation k+1
        if (i <= rmax && r2 == k + 2) sxy[1] = nk;   // y of rotation k+1 (the bulge)
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // --- eigenvectors of the triangular T = H: T y = w_k y, y_k = 1, y_i = 0 for i > k
  double tnorm = 0;
  for (int t = tid; t < n * n; t += SWG) {
    const int i = t % n, j = t / n;
    if (i <= j) tnorm = fmax(tnorm, zabs(H[i + (int64_t)j * ldh]));
  }
  tnorm = block_max(tnorm, sh);
  const double smin = fmax(eps * tnorm, 1e-300);
  for (int k = tid; k < n; k += SWG) {
    const c64 lam = H[k + (int64_t)k * ldh];
    for (int i = n - 1; i > k; --i) Y[i + (int64_t)k * n] = make_double2(0, 0);
    Y[k + (int64_t)k * n] = make_double2(1, 0);
    for (int i = k - 1; i >= 0; --i) {
      c64 acc = H[i + (int64_t)k * ldh];
      for (int j = i + 1; j < k; ++j) acc = zadd(acc, zmul(H[i + (int64_t)j * ldh], Y[j + (int64_t)k * n]));
      c64 d = zsub(H[i + (int64_t)i * ldh], lam);
      if (zabs(d) < smin) d = make_double2(smin, 0);
      Y[i + (int64_t)k * n] = zscale(zdiv(acc, d), -1.0);
    }
  }
  __syncthreads();
  // V = Z Y, columns normalised
  for (int t = tid; t < n * n; t += SWG) {
    const int i = t % n, k = t / n;
    c64 acc = make_double2(0, 0);
    for (int j = 0; j <= k; ++j) acc = zadd(acc, zmul(Z[i + (int64_t)j * n], Y[j + (int64_t)k * n]));
    Vout[i + (int64_t)k * ldv] = acc;
  }
  __syncthreads();
  for (int k = tid; k < n; k += SWG) {
    double s2 = 0;
    for (int i = 0; i < n; ++i) s2 += cabs2<double>(Vout[i + (int64_t)k * ldv]);
    const double inv = (s2 > 0) ? 1.0 / sqrt(s2) : 0.0;
    for (int i = 0; i < n; ++i) Vout[i + (int64_t)k * ldv] = zscale(Vout[i + (int64_t)k * ldv], inv);
  }
}

int32_t eig(cbs_system* s, int32_t n, c64* H, int32_t ldh, c64* w, c64* V, int32_t ldv, int32_t* info_dev,
            hipStream_t st) {
  if (n <= 0) return CBS_OK;
  if (n > 512) {
    set_error("eig: order %d above 512", n);
    return CBS_EINVAL;
  }
  c64* Z = nullptr;
  c64* Y = nullptr;
  CBS_TRY(ws_get(s->ws, "eig.Z", (size_t)n * n, &Z));
  CBS_TRY(ws_get(s->ws, "eig.Y", (size_t)n * n, &Y));
  hipLaunchKernelGGL(k_eig, dim3(1), dim3(SWG), 0, st, n, H, ldh, w, V, ldv, Z, Y, info_dev);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

int32_t svd(int32_t n, c64* A, int32_t lda, c64* V, int32_t ldv, double* sigma, int32_t* perm, hipStream_t st) {
  if (n <= 0) return CBS_OK;
  if (n > 512) {
    set_error("svd: order %d above 512", n);
    return CBS_EINVAL;
  }
  if (n < 4 || getenv("CBS_SVD_SINGLE")) {
    hipLaunchKernelGGL(k_jacobi_svd, dim3(1), dim3(JWG), 0, st, n, A, lda, V, ldv, sigma, perm, 60);
    CBS_HIP(hipGetLastError());
    return CBS_OK;
  }
  // block size: the pair's 2 bs columns of A and W in at most 128 KB of LDS, at least 2
  // blocks; an odd block count gets a padding block
  int bs = 1;
  while (bs * 2 * (int64_t)n * 2 * 2 * sizeof(c64) <= BJ_LDS && bs * 2 * 2 <= n) bs *= 2;
  int nb = (n + bs - 1) / bs;
  nb += nb & 1;
  unsigned long long* flag = nullptr;
  CBS_HIP(hipMalloc(&flag, sizeof(unsigned long long)));
  struct Free {
    unsigned long long* p;
    ~Free() { (void)hipFree(p); }
  } fr{flag};
  hipLaunchKernelGGL(k_svd_init, dim3(std::min(1024, (n * n + 255) / 256)), dim3(256), 0, st, n, V, ldv, flag);
  CBS_HIP(hipGetLastError());
  int sweeps = 0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    for (int r = 0; r < nb - 1; ++r) {
      hipLaunchKernelGGL(k_svd_block, dim3(nb / 2), dim3(BJ_THREADS), 0, st, n, bs, nb, r, A, lda, V, ldv, flag);
      CBS_HIP(hipGetLastError());
    }
    unsigned long long h = 0;
    CBS_HIP(hipMemcpyAsync(&h, flag, sizeof(h), hipMemcpyDeviceToHost, st));
    CBS_HIP(hipStreamSynchronize(st));
    double om = 0;
    std::memcpy(&om, &h, sizeof(om));
    sweeps = sweep + 1;
    if (!(om >= 1e-13)) break;   // converged (or nothing rotated)
    CBS_HIP(hipMemsetAsync(flag, 0, sizeof(unsigned long long), st));
  }
  if (const char* v = getenv("CBS_VERBOSE"))
    if (v[0] == '3') fprintf(stderr, "[cbs] svd: order %d, %d blocks of %d, %d sweeps\n", n, nb, bs, sweeps);
  hipLaunchKernelGGL(k_svd_finish, dim3(1), dim3(JWG), 0, st, n, A, lda, sigma, perm);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

// ------------------------------------------------------------------ LU solve
// B := A^{-1} B for n x n A (destroyed) and nrhs columns, partial pivoting.
__global__ void __launch_bounds__(SWG) k_lu_solve(int32_t n, c64* A, int32_t lda, c64* B, int32_t ldb,
                                                   int32_t nrhs, int32_t* info) {
  __shared__ double sh[SWG / 64];
  __shared__ int sidx[SWG / 64];
  __shared__ int piv;
  const int tid = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    // pivot search
    double best = -1;
    int bi = k;
    for (int i = k + tid; i < n; i += SWG) {
      const double v = zabs(A[i + (int64_t)k * lda]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int o = 1; o < 64; o <<= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if ((tid & 63) == 0) {
      sh[tid >> 6] = best;
      sidx[tid >> 6] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double b = sh[0];
      int ii = sidx[0];
      for (int w = 1; w < SWG / 64; ++w)
        if (sh[w] > b || (sh[w] == b && sidx[w] < ii)) {
          b = sh[w];
          ii = sidx[w];
        }
      piv = ii;
      if (b == 0.0) info[0] = 2;   // singular
    }
    __syncthreads();
    const int p = piv;
    if (p != k) {
      for (int j = tid; j < n + nrhs; j += SWG) {
        c64* M = (j < n) ? A : B;
        const int col = (j < n) ? j : j - n;
        const int ld = (j < n) ? lda : ldb;
        const c64 t = M[k + (int64_t)col * ld];
        M[k + (int64_t)col * ld] = M[p + (int64_t)col * ld];
        M[p + (int64_t)col * ld] = t;
      }
    }
    __syncthreads();
    const c64 d = A[k + (int64_t)k * lda];
    const bool ok = zabs(d) > 0;
    for (int i = k + 1 + tid; i < n; i += SWG)
      A[i + (int64_t)k * lda] = ok ? zdiv(A[i + (int64_t)k * lda], d) : make_double2(0, 0);
    __syncthreads();
    // trailing update of A and B
    const int cols = (n - k - 1) + nrhs;
    const int rows = n - k - 1;
    for (int t = tid; t < rows * cols; t += SWG) {
      const int i = k + 1 + t % rows;
      const int cj = t / rows;
      c64* M;
      int col, ld;
      if (cj < n - k - 1) {
        M = A;
        col = k + 1 + cj;
        ld = lda;
      } else {
        M = B;
        col = cj - (n - k - 1);
        ld = ldb;
      }
      M[i + (int64_t)col * ld] = zsub(M[i + (int64_t)col * ld], zmul(A[i + (int64_t)k * lda], M[k + (int64_t)col * ld]));
    }
    __syncthreads();
  }
  // back substitution U x = y, one right-hand side per thread
  for (int c = tid; c < nrhs; c += SWG) {
    for (int i = n - 1; i >= 0; --i) {
      c64 acc = B[i + (int64_t)c * ldb];
      for (int j = i + 1; j < n; ++j) acc = zsub(acc, zmul(A[i + (int64_t)j * lda], B[j + (int64_t)c * ldb]));
      const c64 d = A[i + (int64_t)i * lda];
      B[i + (int64_t)c * ldb] = (zabs(d) > 0) ? zdiv(acc, d) : make_double2(0, 0);
    }
  }
}

int32_t lu_solve(int32_t n, c64* A, int32_t lda, c64* B, int32_t ldb, int32_t nrhs, int32_t* info_dev,
                 hipStream_t st) {
  if (n <= 0) return CBS_OK;
  hipLaunchKernelGGL(k_lu_solve, dim3(1), dim3(SWG), 0, st, n, A, lda, B, ldb, nrhs, info_dev);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

// ------------------------------------------------------------------ Cholesky + inverse
// G = R^H R (upper R), Rinv = R^{-1} (upper); G destroyed.  A shift is added to the
// diagonal first (shifted Cholesky QR).
__global__ void __launch_bounds__(SWG) k_chol_inv(int32_t n, c64* G, int32_t ldg, double shift, c64* Rinv,
                                                   int32_t* info) {
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += SWG) G[i + (int64_t)i * ldg].x += shift;
  __syncthreads();
  // right-looking: for k, R[k][k] = sqrt(G[k][k]); R[k][j] = G[k][j]/R[k][k]; G[i][j] -= conj(R[k][i]) R[k][j]
  for (int k = 0; k < n; ++k) {
    const double d = G[k + (int64_t)k * ldg].x;
    const double r = (d > 0) ? sqrt(d) : 0.0;
    if (tid == 0 && !(d > 0)) info[0] = 3;
    __syncthreads();
    for (int j = k + 1 + tid; j < n; j += SWG)
      G[k + (int64_t)j * ldg] = (r > 0) ? zscale(G[k + (int64_t)j * ldg], 1.0 / r) : make_double2(0, 0);
    __syncthreads();
    if (tid == 0) G[k + (int64_t)k * ldg] = make_double2(r, 0);
    const int m = n - k - 1;
    for (int t = tid; t < m * m; t += SWG) {
      const int i = k + 1 + t % m, j = k + 1 + t / m;
      if (i <= j)
        G[i + (int64_t)j * ldg] = zsub(G[i + (int64_t)j * ldg], zmulc(G[k + (int64_t)i * ldg], G[k + (int64_t)j * ldg]));
    }
    __syncthreads();
  }
  // inverse of the upper triangle, one column per thread
  for (int c = tid; c < n; c += SWG) {
    for (int i = n - 1; i >= 0; --i) {
      c64 acc = make_double2(i == c ? 1.0 : 0.0, 0.0);
      for (int j = i + 1; j <= c; ++j) acc = zsub(acc, zmul(G[i + (int64_t)j * ldg], Rinv[j + (int64_t)c * n]));
      const double d = G[i + (int64_t)i * ldg].x;
      Rinv[i + (int64_t)c * n] = (i > c) ? make_double2(0, 0) : ((d > 0) ? zscale(acc, 1.0 / d) : make_double2(0, 0));
    }
  }
}

int32_t chol_inv(int32_t n, c64* G, int32_t ldg, double shift, c64* Rinv, int32_t* info_dev, hipStream_t st) {
  if (n <= 0) return CBS_OK;
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(SWG), 0, st, n, G, ldg, shift, Rinv, info_dev);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

}  // namespace cbs
