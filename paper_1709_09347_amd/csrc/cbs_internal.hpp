// Internal declarations of the MI355X Sakurai-Sugiura CBS library.
//
// Vector storage on the device is "pair-interleaved": for every BiCG run
// (quadrature node j, right-hand side l) the primal vector and its dual are
// stored side by side per grid point, Pair{primal, dual}, so one thread
// handles both recurrences of a run and the dual's scalars (conj(alpha),
// conj(beta)) come for free.  Run r occupies points [r*N, (r+1)*N).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "cbs.h"

namespace cbs {

// ---------------------------------------------------------------- complex
template <typename R> struct cvec;
template <> struct cvec<double> { using T = double2; };
template <> struct cvec<float> { using T = float2; };
template <typename R> using cplx = typename cvec<R>::T;

template <typename R>
__host__ __device__ __forceinline__ cplx<R> mkc(R re, R im) { cplx<R> c; c.x = re; c.y = im; return c; }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return mkc<R>(a.x + b.x, a.y + b.y); }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return mkc<R>(a.x - b.x, a.y - b.y); }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return mkc<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cmulc(cplx<R> a, cplx<R> b) {
  return mkc<R>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cconj(cplx<R> a) { return mkc<R>(a.x, -a.y); }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return mkc<R>(a.x * s, a.y * s); }
// a + s * b (s real)
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cfma_r(cplx<R> a, R s, cplx<R> b) {
  return mkc<R>(a.x + s * b.x, a.y + s * b.y);
}
// a + c * b (c complex)
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cfma(cplx<R> a, cplx<R> c, cplx<R> b) {
  return mkc<R>(a.x + c.x * b.x - c.y * b.y, a.y + c.x * b.y + c.y * b.x);
}
template <typename R>
__host__ __device__ __forceinline__ R cabs2(cplx<R> a) { return a.x * a.x + a.y * a.y; }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cdiv(cplx<R> a, cplx<R> b) {
  R d = b.x * b.x + b.y * b.y;
  return mkc<R>((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
template <typename Ro, typename Ri>
__host__ __device__ __forceinline__ cplx<Ro> ccast(cplx<Ri> a) { return mkc<Ro>((Ro)a.x, (Ro)a.y); }

template <typename R>
struct alignas(2 * sizeof(cplx<R>)) Pair {
  cplx<R> a;  // primal
  cplx<R> b;  // dual
};

template <typename Ro, typename Ri>
__host__ __device__ __forceinline__ Pair<Ro> pcast(const Pair<Ri>& p) {
  Pair<Ro> o;
  o.a = ccast<Ro, Ri>(p.a);
  o.b = ccast<Ro, Ri>(p.b);
  return o;
}

// Coefficient triple of one vector: y = c0 (H0-E) x + cp H+ x + cm H- x.
// Per run: [primal c0, cp, cm, dual c0, cp, cm] as complex doubles.
struct RunCoef {
  double2 c[6];
  double E;        // energy of the run (batched solves mix energies)
  double pad;
};

template <typename R> struct vec4;
template <> struct vec4<double> { using T = double4; };
template <> struct vec4<float> { using T = float4; };

// Output layout of the 16x16x4 MFMA instructions (one block, 4 accumulators per lane,
// column = lane % 16): the FP64 variant holds row 4*v + lane/16 in accumulator v, the
// FP32 variant row 4*(lane/16) + v.  Operands: lane l feeds A[l%16][l/16] and
// B[l/16][l%16] in both.
template <typename R>
__device__ __forceinline__ int mfma16_row(int lane, int v) {
  return sizeof(R) == 8 ? 4 * v + (lane >> 4) : 4 * (lane >> 4) + v;
}

// Address space for data read at wave-uniform addresses (the compiler then uses scalar
// loads); the host pass of the same source has no address spaces.
#if defined(__HIP_DEVICE_COMPILE__)
#define CBS_CONST_AS __attribute__((address_space(4)))
#else
#define CBS_CONST_AS
#endif

// Arithmetic precision of the complex64-storage kernels: FP32 by default (complex64
// operator applications and updates; the phase starts once the residual is small enough
// for them); CBS_LO_ARITH=64 computes in FP64 on the complex64 data.
inline bool lo_arith_fp32() {
  const char* e = getenv("CBS_LO_ARITH");
  return !(e && e[0] == '6' && e[1] == '4');
}

// Remap a block id so that consecutive logical blocks run on one XCD (the
// dispatcher hands blocks to the 8 XCDs round-robin); gridDim must be a
// multiple of 8.
__device__ __forceinline__ int xcd_remap(int bid, int nb) { return (bid & 7) * (nb >> 3) + (bid >> 3); }

// Logical block of a launch whose first nl logical blocks carry work (nl may be below the
// grid when the work comes from a device-side count of active runs): the nl blocks are
// spread over the 8 XCDs (hardware block b runs on XCD b % 8) so that consecutive logical
// blocks share one XCD; -1 for blocks without work.
__device__ __forceinline__ int remap_active(int bid, int nl) {
  const int per = (nl + 7) >> 3;
  if ((bid >> 3) >= per) return -1;
  const int lb = (bid & 7) * per + (bid >> 3);
  return (lb < nl) ? lb : -1;
}

template <typename R>
__device__ __forceinline__ R wsum(R v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Ket of the nonlocal projectors at point n (see nonlocal.hip).
template <typename R>
__device__ __forceinline__ Pair<R> ket_at(int64_t n, int64_t ktbase, const int32_t* pt_off,
                                          const int32_t* pt_key, const R* pt_u, const Pair<R>* kt) {
  Pair<R> q;
  q.a = mkc<R>(0, 0);
  q.b = q.a;
  const int lo = pt_off[n], hi = pt_off[n + 1];
  for (int e = lo; e < hi; ++e) {
    const int key = pt_key[e];
    const typename vec4<R>::T uu = reinterpret_cast<const typename vec4<R>::T*>(pt_u)[e];
    const Pair<R>* k = kt + ktbase + (int64_t)(key >> 2) * 12 + (key & 3) * 4;
    const R us[4] = {uu.x, uu.y, uu.z, uu.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const Pair<R> kk = k[i];
      q.a = cfma_r<R>(q.a, us[i], kk.a);
      q.b = cfma_r<R>(q.b, us[i], kk.b);
    }
  }
  return q;
}

// ------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
const char* get_error();

#define CBS_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::cbs::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call, hipGetErrorString(e_)); \
      return CBS_EHIP;                                                                 \
    }                                                                                  \
  } while (0)

#define CBS_TRY(expr)               \
  do {                              \
    int32_t rc_ = (expr);           \
    if (rc_ != CBS_OK) return rc_;  \
  } while (0)

// ------------------------------------------------------------- buffers
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Grow-only device workspace keyed by name.
struct Workspace {
  std::map<std::string, DevBuf> bufs;
  int32_t get(const char* name, size_t bytes, void** out);
  void drop(const char* name);
  void release();
};

template <typename T>
int32_t ws_get(Workspace& ws, const char* name, size_t count, T** out) {
  void* p = nullptr;
  int32_t rc = ws.get(name, count * sizeof(T) + 256, &p);
  *out = static_cast<T*>(p);
  return rc;
}

// ------------------------------------------------------------- system
struct ChunkTables {
  int32_t tp = 0, nchunks = 0, nslots = 0, pl = 0;
  int32_t* piece_off = nullptr;   // [nchunks+1]
  int32_t* piece_beg = nullptr;   // [npieces]
  int32_t* piece_meta = nullptr;  // [npieces] (local slot << 16) | entry count (a multiple of BT_EB)
  int32_t* slot_off = nullptr;    // [nchunks+1]
  int32_t* slot_piece = nullptr;  // [nslots+1]
  int32_t* ent_pt = nullptr;      // [entries] point within the chunk (padding: 0)
  double* u64 = nullptr;          // [entries][4] (padding: 0)
  float* u32 = nullptr;
  int32_t* key_off = nullptr;     // [3*n_atoms+1] slots of key k: [key_off[k], key_off[k+1]) in key order
  int32_t* slot_pos = nullptr;    // [nslots] position of slot g in key order (chunk order within a key)
};

struct Projector {
  int32_t n_atoms = 0;
  int64_t nnz = 0;
  // atom-major, entries of each atom ordered by shift w: segment s (w = s-1)
  // of atom a spans [seg[4a+s], seg[4a+s+1]).
  int32_t* seg = nullptr;        // [4*n_atoms]
  int32_t* ball_idx = nullptr;   // [nnz] cell point
  double* ball_u64 = nullptr;    // [nnz*4] (padded to 4 projectors)
  float* ball_u32 = nullptr;
  double* coeff64 = nullptr;     // [n_atoms*4]
  float* coeff32 = nullptr;
  // point-major index for the ket: entries of point n are [pt_off[n], pt_off[n+1])
  int32_t* pt_off = nullptr;     // [N+1]
  int32_t* pt_key = nullptr;     // [nnz] atom*4 + (w+1)
  double* pt_u64 = nullptr;      // [nnz*4]
  float* pt_u32 = nullptr;
  int32_t max_atom_entries = 0;
  // grouped ket tables: points in groups of KG consecutive indices; group g uses the
  // keys [grp_off[g], grp_off[g+1]) (atom*4 + (w+1), ascending) and for each key the
  // values of its KG points (zero where the point is outside that ball); grp_mask: per key
  // one bit per 16-point block of the group with a nonzero value
  int32_t* grp_off = nullptr;    // [ngroups+1]
  int32_t* grp_key = nullptr;    // [nkeys]
  int32_t* grp_mask = nullptr;   // [nkeys]
  double* grp_u64 = nullptr;     // [nkeys][KG][4]
  float* grp_u32 = nullptr;
  int64_t grp_nkeys = 0;
  // chunked bra tables (see tables.hpp), one set per chunk length BT_TPS[i]: the entries
  // of every chunk by key, cut into pieces, at most BT_MAXP pieces per chunk; nslots
  // (chunk, key) slots in all (0: no tables of that length)
  ChunkTables bt[2];
};
constexpr int KG = 64;        // points per ket group (one wavefront)
constexpr int BT_TPS[2] = {256, 512};   // points per chunk of the chunked bra
constexpr int BT_MAXP = 128;             // pieces per chunk of the chunked bra
constexpr int BT_EB = 4;                 // entries per batch of the chunked bra (pieces padded to it)

struct LastSolve {
  int32_t n = 0;
  double E = 0;
  std::vector<double2> lambda;
  double2* vecs = nullptr;   // device [n][N], owned
  size_t cap = 0;
};

}  // namespace cbs

struct cbs_system {
  int32_t device = 0;
  int32_t nx = 0, ny = 0, nz = 0, p = 0;
  double h = 0;
  int64_t N = 0;
  double fd[5] = {0, 0, 0, 0, 0};   // c_0 .. c_p of the central second derivative
  double* vloc64 = nullptr;
  float* vloc32 = nullptr;
  cbs::Projector proj;
  cbs::Workspace ws;
  cbs::LastSolve last;
  int32_t tile_y[2] = {0, 0};       // stencil tile rows per precision (0 = double, 1 = float)
  int32_t bra_nw[2] = {4, 4};       // waves per (atom, 16 runs) of the full-batch bra, per precision
  int32_t bra_spread[2] = {1, 1};   // 1: consecutive bra workgroups on different XCDs (same runs)
  int32_t bra_tile[2] = {0, 0};     // full-batch bra: 0 = per atom (MFMA), else runs per chunked workgroup
  int32_t bra_tp[2] = {1, 1};       // chunked bra: which chunk length (index into BT_TPS)
  int32_t bra_qx[2] = {0, 0};       // chunked bra: table loads per lane (0) or shared by quads (1)
  int32_t upd_pts = 2048;           // points per chunk of the residual update (its partial sums)
  int32_t tuned = 0;                // tile heights picked by the autotuner
  int64_t solve_id = 0;             // stored solves so far (see cbs_system_solve_id)
  std::string tune_log;
};

namespace cbs {

// ---------------------------------------------------------------- host API of the kernels
// Launch helpers (all asynchronous on `stream`).

// Local operator (stencil) of every run's pair: see stencil.hip.
struct StencilLaunch {
  int32_t nruns;
  const void* rin;          // BiCG: r; apply: x
  const void* pold;         // BiCG: previous search direction
  void* pnew;               // BiCG: new search direction
  void* q;                  // output: local part of P(z) p
  void* x;                  // BiCG: x += xcoef * pold
  const RunCoef* coef;      // [nruns]
  const double2* beta;      // BiCG [nruns]
  const double2* xcoef;     // BiCG [nruns]
  const int32_t* status;    // [nruns] or NULL (no filter)
  int32_t need_status;      // blocks of runs whose status differs return at once
  double2* sig_part;        // BiCG [nruns*ntiles]
  const int32_t* list;      // device [nruns] active runs (ascending) or NULL: all runs
  const int32_t* count;     // device: entries of list (with list)
  int32_t zseg;             // apply only: z segments per tile (0 or 1: one), for short run lists
};
template <typename R>
int32_t launch_stencil(const cbs_system* s, bool bicg, const StencilLaunch& a, int32_t tile_y,
                       hipStream_t st);
int32_t stencil_tiles(const cbs_system* s, int32_t tile_y);
int32_t default_tile_y(const cbs_system* s, int32_t bytes_per_pair);
// Times every feasible tile height once per system and precision (CBS_AUTOTUNE=0: keep defaults).
int32_t autotune_tiles(cbs_system* s, hipStream_t st);

// Nonlocal part: bra (coefficients of every atom) then ket tables.
// tile_part: scratch of bra_tile_part_bytes(s, nruns) bytes for the chunked bra (used for
// full batches of P(z) when the tables exist and the autotuner chose it), or NULL.
template <typename R>
int32_t launch_bra(const cbs_system* s, int32_t nruns, const void* v, const RunCoef* coef,
                   const int32_t* status, int32_t need_status, void* kt, double2* signl,
                   hipStream_t st, bool phased, const int32_t* list = nullptr,
                   const int32_t* count = nullptr, bool short_list = false, void* tile_part = nullptr);
size_t bra_tile_part_bytes(const cbs_system* s, int32_t nruns);

// Fused pointwise kernels.
template <typename R>
int32_t launch_update(const cbs_system* s, int32_t nruns, void* r, const void* q, const void* kt,
                      const double2* alpha, const int32_t* status, int32_t need_status, double* part,
                      int32_t nchunks, hipStream_t st, const int32_t* list = nullptr,
                      const int32_t* count = nullptr);
template <typename R>
int32_t launch_ket_add(const cbs_system* s, int32_t nruns, void* q, const void* kt, hipStream_t st);

int32_t update_chunks(const cbs_system* s);

// Utility conversions between vector-major [v][N] and pair layout.
template <typename R>
int32_t launch_to_pairs(int64_t N, int32_t nvec, const void* x, void* pairs, hipStream_t st);
template <typename R>
int32_t launch_from_pairs(int64_t N, int32_t nvec, const void* pairs, void* y, hipStream_t st);

// Device address of the fixed scratch array of cbs_apply_noalloc on `device` (current),
// looked up once per device (noalloc.hip).
int32_t noalloc_scratch(int32_t device, void** out);

// Parts-form apply on complex128 vectors (used by the solver's Rayleigh-Ritz step).
int32_t apply_parts_dev(cbs_system* s, double E, int32_t n_vec, const double2* c0,
                        const double2* cp, const double2* cm, const double2* x, double2* y,
                        hipStream_t st);

}  // namespace cbs
