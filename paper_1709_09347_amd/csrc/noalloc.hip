// Operator application without device allocation (cbs_apply_noalloc).
//
// cbs_apply stages its vectors in the system's grow-only workspace, which calls hipMalloc
// the first time a size is seen.  This variant runs the same kernels with every staging
// buffer inside one fixed device array, `scratch`, so a call allocates nothing: callers
// that cannot allocate (code under graph capture, tight serving loops) use it.
//
// The array is a file-scope __device__ symbol: in host code its name is only a stand-in,
// so its device address is looked up once per device with hipGetSymbolAddress (at system
// creation, with that device current) and that address is what the kernels receive.
// Every call on one device shares the array and leaves its contents behind; calls that
// overlap on one device race.
#include <mutex>
#include <type_traits>
#include <vector>

#include "cbs_internal.hpp"

namespace cbs {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // CBS_APPLY_NOALLOC_BYTES in cbs.h
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static void* g_scratch[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Device address of the scratch array on `device` (which must be current); looked up once.
int32_t noalloc_scratch(int32_t device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) {
    set_error("device %d beyond the %d devices the allocation-free entry points track", device, kMaxDevices);
    return CBS_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      set_error("hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
      return CBS_EHIP;
    }
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return CBS_OK;
}

// Run coefficients of up to kCoefChunk runs, passed by value as kernel arguments (no host
// staging copy) and written into the scratch array by one small kernel.
constexpr int kCoefChunk = 24;
struct CoefChunk {
  RunCoef c[kCoefChunk];
};

__global__ void k_put_coef(CoefChunk chunk, int32_t n, RunCoef* dst) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = chunk.c[i];
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of scratch one call needs: run coefficients, the two pair buffers and the ket
// coefficients, each 256-byte aligned.
static size_t need_bytes(const cbs_system* s, int32_t n_vec, size_t pair_bytes) {
  const size_t nr = (size_t)(n_vec + 1) / 2;
  size_t b = align256(nr * sizeof(RunCoef));
  b += 2 * align256(nr * (size_t)s->N * pair_bytes);
  if (s->proj.n_atoms > 0) b += align256(nr * (size_t)s->proj.n_atoms * 12 * pair_bytes);
  return b;
}

template <typename R>
static int32_t apply_noalloc(cbs_system* s, double E, int32_t n_vec, const double* z, const void* x, void* y,
                             unsigned char* base, hipStream_t st) {
  const int32_t nr = (n_vec + 1) / 2;
  size_t off = 0;
  RunCoef* coef = reinterpret_cast<RunCoef*>(base + off);
  off += align256((size_t)nr * sizeof(RunCoef));
  Pair<R>* px = reinterpret_cast<Pair<R>*>(base + off);
  off += align256((size_t)nr * s->N * sizeof(Pair<R>));
  Pair<R>* pq = reinterpret_cast<Pair<R>*>(base + off);
  off += align256((size_t)nr * s->N * sizeof(Pair<R>));
  Pair<R>* kt = (s->proj.n_atoms > 0) ? reinterpret_cast<Pair<R>*>(base + off) : nullptr;
  // P(z) coefficients per half (primal = even vector, dual slot = odd vector); a missing
  // odd vector gets c0 = 0 and z = 1, and its output half is not copied back
  for (int k0 = 0; k0 < nr; k0 += kCoefChunk) {
    CoefChunk ch;
    const int n = std::min(kCoefChunk, nr - k0);
    for (int k = 0; k < n; ++k) {
      RunCoef& c = ch.c[k];
      for (int h = 0; h < 2; ++h) {
        const int v = 2 * (k0 + k) + h;
        double zr = 1, zi = 0;
        if (v < n_vec) {
          zr = z[2 * v];
          zi = z[2 * v + 1];
        }
        const double d = zr * zr + zi * zi;
        c.c[3 * h + 0] = make_double2(v < n_vec ? 1.0 : 0.0, 0.0);
        c.c[3 * h + 1] = make_double2(zr, zi);
        c.c[3 * h + 2] = make_double2(zr / d, -zi / d);
      }
      c.E = E;
      c.pad = 0;
    }
    hipLaunchKernelGGL(k_put_coef, dim3(1), dim3(kCoefChunk), 0, st, ch, (int32_t)n, coef + k0);
    CBS_HIP(hipGetLastError());
  }
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
  return CBS_OK;
}

}  // namespace cbs

using namespace cbs;

extern "C" int32_t cbs_apply_noalloc(cbs_system* s, double E, int32_t n_vec, const double* z, int32_t dtype,
                                     const void* x, void* y, void* stream) {
  if (!s || n_vec < 0 || (n_vec > 0 && (!z || !x || !y)) || (dtype != CBS_C128 && dtype != CBS_C64)) {
    set_error("cbs_apply_noalloc: bad argument");
    return CBS_EINVAL;
  }
  for (int v = 0; v < n_vec; ++v) {
    if (z[2 * v] == 0.0 && z[2 * v + 1] == 0.0) {
      set_error("cbs_apply_noalloc: z must be nonzero");
      return CBS_EINVAL;
    }
  }
  if (n_vec == 0) return CBS_OK;
  const size_t pb = (dtype == CBS_C128) ? sizeof(Pair<double>) : sizeof(Pair<float>);
  const size_t need = need_bytes(s, n_vec, pb);
  if (need > kScratchBytes) {
    set_error("cbs_apply_noalloc: %d vectors of %lld points need %zu bytes of scratch, the fixed array holds %zu",
              n_vec, (long long)s->N, need, kScratchBytes);
    return CBS_EINVAL;
  }
  CBS_HIP(hipSetDevice(s->device));
  void* base = nullptr;
  CBS_TRY(noalloc_scratch(s->device, &base));
  hipStream_t st = (hipStream_t)stream;
  if (dtype == CBS_C128) return apply_noalloc<double>(s, E, n_vec, z, x, y, (unsigned char*)base, st);
  return apply_noalloc<float>(s, E, n_vec, z, x, y, (unsigned char*)base, st);
}
