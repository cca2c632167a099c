// Separable nonlocal projectors (paper Sec. 4: norm-conserving pseudopotentials) and the
// pointwise kernels that consume them.
//
// With the ball values of atom a split by cell shift w (u_{a,i,w}), the nonlocal part
// of c0 (H0-E) + cp H+ + cm H- is
//     sum_{a,i} h_ai sum_{w,w'} coef(w'-w) u_{a,i,w} u_{a,i,w'}^T,
// coef(0) = c0, coef(1) = cp, coef(-1) = cm (P(z): 1, z, 1/z).  It is applied in two
// passes per run:
//   bra:  G[a][w'][i] = u_{a,i,w'}^T v            (one workgroup per atom and 16 runs,
//                                                  MFMA; a plain kernel per atom and run)
//         K[a][w][i]  = h_ai sum_w' coef(w'-w) G[a][w'][i]
//   ket:  y(n) += sum_{entries e at point n} sum_i u_{e,i} K[a_e][w_e][i]
// The ket runs inside the pointwise kernels (BiCG residual update, apply), reading
// point-ordered tables (per point, or per 64-point group and key in the update) so no two
// threads ever add into the same point.
// For BiCG the bra also yields the nonlocal part of sigma = pt^H P p:
//   sum_{a,i} h_ai conj(ct_ai) c_ai,  c = G_0 + z G_1 + z^-1 G_-1 (dual: 1/conj z).
#include <algorithm>
#include <type_traits>

#include "cbs_internal.hpp"

namespace cbs {

// ------------------------------------------------------------------------- bra
template <typename R>
struct BraArgs {
  int32_t n_atoms, nlogical, need_status, nruns;
  int64_t N;
  const int32_t* seg;
  const int32_t* idx;
  const R* u;          // [nnz][4]
  const R* coeff;      // [n_atoms][4]
  const Pair<R>* v;
  const RunCoef* coef;
  const int32_t* status;
  Pair<R>* kt;         // [run][atom][3][4]
  double2* signl;      // [run][atom] or NULL
  const int32_t* list;    // MFMA bra: active runs (ascending) or NULL
  const int32_t* count;   // device count of list entries
  int32_t spread;         // MFMA bra: 1 = consecutive blocks on different XCDs
};

template <typename R>
__global__ void __launch_bounds__(256) k_bra(BraArgs<R> a) {
  __shared__ R red[4][16];
  __shared__ cplx<R> G[3][4][2];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int nl = (a.list != nullptr) ? min(a.nlogical, *a.count * a.n_atoms) : a.nlogical;
  if (lb >= nl) return;
  const int slot = lb / a.n_atoms;
  const int atom = lb - slot * a.n_atoms;
  const int run = (a.list != nullptr) ? a.list[slot] : slot;
  if (a.status != nullptr && a.status[run] != a.need_status) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t base = (int64_t)run * a.N;
  for (int sgi = 0; sgi < 3; ++sgi) {
    const int lo = a.seg[4 * atom + sgi], hi = a.seg[4 * atom + sgi + 1];
    R acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0;
    for (int e = lo + tid; e < hi; e += 256) {
      const typename vec4<R>::T uu = reinterpret_cast<const typename vec4<R>::T*>(a.u)[e];
      const Pair<R> v = a.v[base + a.idx[e]];
      const R us[4] = {uu.x, uu.y, uu.z, uu.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        acc[4 * i + 0] += us[i] * v.a.x;
        acc[4 * i + 1] += us[i] * v.a.y;
        acc[4 * i + 2] += us[i] * v.b.x;
        acc[4 * i + 3] += us[i] * v.b.y;
      }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = wsum<R>(acc[k]);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 16; ++k) red[wv][k] = acc[k];
    }
    __syncthreads();
    if (tid < 16) {
      const R t = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
      const int i = tid >> 2, part = tid & 3;
      R* g = reinterpret_cast<R*>(&G[sgi][i][part >> 1]);
      g[part & 1] = t;
    }
    __syncthreads();
  }
  const RunCoef cf = a.coef[run];
  if (tid < 24) {
    // tid -> (w shift s of the ket entry, projector i, half)
    const int half = tid & 1, i = (tid >> 1) & 3, sw = tid >> 3;
    const cplx<R> c0 = ccast<R, double>(cf.c[3 * half + 0]);
    const cplx<R> cp = ccast<R, double>(cf.c[3 * half + 1]);
    const cplx<R> cm = ccast<R, double>(cf.c[3 * half + 2]);
    cplx<R> k = mkc<R>(0, 0);
#pragma unroll
    for (int s2 = 0; s2 < 3; ++s2) {
      const int d = s2 - sw;   // w' - w
      const cplx<R> cc = (d == 0) ? c0 : (d == 1) ? cp : (d == -1) ? cm : mkc<R>(0, 0);
      k = cfma<R>(k, cc, G[s2][i][half]);
    }
    k = cscale<R>(k, a.coeff[4 * atom + i]);
    cplx<R>* dst = reinterpret_cast<cplx<R>*>(&a.kt[((int64_t)run * a.n_atoms + atom) * 12 + sw * 4 + i]);
    dst[half] = k;
  }
  if (a.signl != nullptr && tid == 32) {
    double2 sg = make_double2(0.0, 0.0);
    const cplx<R> zpa = ccast<R, double>(cf.c[1]), zma = ccast<R, double>(cf.c[2]);
    const cplx<R> zpb = ccast<R, double>(cf.c[4]), zmb = ccast<R, double>(cf.c[5]);
    for (int i = 0; i < 4; ++i) {
      cplx<R> ca = cadd<R>(G[1][i][0], cadd<R>(cmul<R>(zpa, G[2][i][0]), cmul<R>(zma, G[0][i][0])));
      cplx<R> cb = cadd<R>(G[1][i][1], cadd<R>(cmul<R>(zpb, G[2][i][1]), cmul<R>(zmb, G[0][i][1])));
      const cplx<R> t = cscale<R>(cmulc<R>(cb, ca), a.coeff[4 * atom + i]);
      sg.x += (double)t.x;
      sg.y += (double)t.y;
    }
    a.signl[(int64_t)run * a.n_atoms + atom] = sg;
  }
}

// MFMA bra for operators of the form P(z) (c0 = 1, cp = z, cm = 1/z per half): then
// K[w][i] = h_ai z^-w c_ai with c_ai = sum_e u_{e,i} z^{w_e} v(idx_e), so the Bloch
// phase is applied to the gathered vector and one contraction per atom remains:
//   C[(run, half, re/im)][i] = sum_e A[(run, half, re/im)][e] U[e][i],
// a [16 x n_ball] x [n_ball x 4] product per wave (4 runs x 2 halves x re/im rows),
// 4 waves = 16 runs per workgroup sharing every table read.  MFMA 16x16x4: lane l
// feeds A[l%16][k=l/16] and U[k=l/16][l%16] (columns 4..15 are zero padding) and holds
// C[mfma16_row(l, v)][l%16].
template <typename R> struct mf4;
template <> struct mf4<double> { typedef double T __attribute__((ext_vector_type(4))); };
template <> struct mf4<float> { typedef float T __attribute__((ext_vector_type(4))); };

__device__ __forceinline__ mf4<double>::T mfma16x16x4(double a, double b, mf4<double>::T c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mf4<float>::T mfma16x16x4(float a, float b, mf4<float>::T c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// R: storage precision (vectors, tables, K); C: arithmetic precision (MFMA, sums).
// NW waves per workgroup share each (atom, 16 runs): 4 for full batches; 16 when the run
// list is short (residual replacement), so the few workgroups walk their balls 4x faster.
template <typename R, typename C, int NW>
__global__ void __launch_bounds__(64 * NW) k_bra_mfma(BraArgs<R> a) {
  __shared__ cplx<C> cs[16][2][4];
  __shared__ int srun[16];
  // slots: the runs themselves, or the entries of the active-run list
  const int nslots = (a.list != nullptr) ? *a.count : a.nruns;
  const int nl = min(a.nlogical, ((nslots + 15) / 16) * a.n_atoms);
  // spread: all XCDs work on the same 16 runs at a time (different atoms), so the
  // overlapping balls of neighbouring atoms are re-read from the memory-side cache
  const int lb = a.spread ? ((int)blockIdx.x < nl ? (int)blockIdx.x : -1) : remap_active(blockIdx.x, nl);
  if (lb < 0) return;
  const int chunk = lb / a.n_atoms;
  const int atom = lb - chunk * a.n_atoms;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int any = 0;
  if (tid < 16) {
    const int slot = chunk * 16 + tid;
    int run = -1;
    if (slot < nslots) {
      run = (a.list != nullptr) ? a.list[slot] : slot;
      if (a.status != nullptr && a.status[run] != a.need_status) run = -1;
    }
    srun[tid] = run;
    any = run >= 0;
  }
  if (!__syncthreads_or(any)) return;
  // Every wave covers all 16 runs (four groups g of 4 runs: four independent MFMA chains
  // that share each table load) over every NW-th step of 4 ball entries; the waves'
  // partial products are summed through LDS.  The ball's entries come in three segments
  // by cell shift w = -1, 0, +1; each segment is contracted without its Bloch phase, which
  // multiplies the segment's complex sums afterwards (c += z^w c_w), so the inner loop
  // holds no phase factors.
  __shared__ C red[NW][4][16][4];
  __shared__ cplx<C> cw[16][2][4];
  const int row = lane & 15, kslot = lane >> 4, col = lane & 15;
  const int half = (row >> 1) & 1, reim = row & 1;
  // lane's component of the gathered vector: run (row >> 2) of group g, primal or dual
  // (half), real or imaginary part (reim); entry idx is at vrow[g][4 * idx]
  const R* vrow[4];
  bool rvalid[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int run = srun[4 * g + (row >> 2)];
    rvalid[g] = run >= 0;
    vrow[g] = reinterpret_cast<const R*>(a.v + (int64_t)(rvalid[g] ? run : 0) * a.N) + 2 * half + reim;
  }
  if (tid < 128) (&cs[0][0][0])[tid] = mkc<C>(0, 0);
  for (int sg = 0; sg < 3; ++sg) {
    const int sa = a.seg[4 * atom + sg], sb = a.seg[4 * atom + sg + 1];
    if (sa == sb) continue;   // uniform over the workgroup
    typename mf4<C>::T acc[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) acc[g] = {0, 0, 0, 0};
    if constexpr (sizeof(C) == 8) {
      // FP64 arithmetic: the table entries (point index, projector value) of the next
      // step are loaded while the gathers of this step are in flight, so each step waits
      // for one memory latency rather than for the table load and then the gather that
      // depends on it.  (With FP32 arithmetic the plain loop is faster: more waves fit.)
      // Loads are unconditional (indices clamped into the segment), so the waits count
      // only the gathers and leave the next step's loads in flight.  Entries past the
      // segment carry a zero projector value and rows of empty run slots are discarded,
      // so the gathered values need no masking.
      const int e_first = sa + 4 * wv + kslot;
      constexpr int STEP = 4 * NW;   // entries per step of the whole workgroup
      const int el = min(e_first, sb - 1);
      int idx0 = a.idx[el];
      C bv0 = (e_first < sb && col < 4) ? (C)a.u[4 * (int64_t)el + (col & 3)] : (C)0;
      for (int e = e_first; e - kslot < sb; e += STEP) {
        C vv[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) vv[g] = (C)vrow[g][4 * (int64_t)idx0];
        const int e1 = e + STEP;
        const int e1l = min(e1, sb - 1);
        const int idx1 = a.idx[e1l];
        const C u1 = (C)a.u[4 * (int64_t)e1l + (col & 3)];
        const C bv1 = (e1 < sb && col < 4) ? u1 : (C)0;
#pragma unroll
        for (int g = 0; g < 4; ++g) acc[g] = mfma16x16x4(vv[g], bv0, acc[g]);
        idx0 = idx1;
        bv0 = bv1;
      }
    } else {
      for (int e0 = sa + 4 * wv; e0 < sb; e0 += 4 * NW) {
        const int e = e0 + kslot;
        const bool ok = e < sb;
        const int elc = min(e, sb - 1);
        const int idx = a.idx[elc];
        const C u = (C)a.u[4 * (int64_t)elc + (col & 3)];
        const C bv = (ok && col < 4) ? u : (C)0;
        C vv[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) vv[g] = (C)vrow[g][4 * (int64_t)idx];
#pragma unroll
        for (int g = 0; g < 4; ++g) acc[g] = mfma16x16x4(vv[g], bv, acc[g]);
      }
    }
    // only the lanes of output columns 0..3 (the four projectors) carry results
    if ((lane & 15) < 4) {
      const int q = (lane >> 4) * 4 + (lane & 15);
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wv][g][q][v] = acc[g][v];
    }
    __syncthreads();
    {
      // thread t < 256: group g = t/64 reduces lane t%64 over the NW waves
      const int g = tid >> 6, l2 = tid & 63;
      if (tid < 256 && (l2 & 15) < 4) {
        const int q = (l2 >> 4) * 4 + (l2 & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          C sum = 0;
#pragma unroll
          for (int w = 0; w < NW; ++w) sum += red[w][g][q][v];
          const int r = mfma16_row<C>(l2, v);   // output row held by lane l2
          C* dst = reinterpret_cast<C*>(&cw[4 * g + (r >> 2)][(r >> 1) & 1][l2 & 15]);
          dst[r & 1] = sum;
        }
      }
    }
    __syncthreads();
    if (tid < 128) {
      // c[run][half][i] += z^w c_w: w = -1 -> 1/z (primal) or conj z (dual), +1 -> z or 1/conj z
      const int r2 = tid >> 3, h2 = (tid >> 2) & 1, i = tid & 3;
      const int rr = srun[r2];
      if (rr >= 0) {
        const cplx<C> c = cw[r2][h2][i];
        cplx<C> t = c;
        if (sg != 1) t = cmul<C>(ccast<C, double>(a.coef[rr].c[3 * h2 + (sg == 0 ? 2 : 1)]), c);
        cs[r2][h2][i] = cadd<C>(cs[r2][h2][i], t);
      }
    }
    __syncthreads();
  }
  const RunCoef* cfp = a.coef;
  for (int t = tid; t < 16 * 24; t += 64 * NW) {
    const int r2 = t / 24, rem = t - r2 * 24;
    const int h2 = rem & 1, i = (rem >> 1) & 3, sw = rem >> 3;
    const int rr = srun[r2];
    if (rr < 0) continue;
    const RunCoef& cf = cfp[rr];
    // K[w][i] = h z^-w c: w = -1 -> cp, 0 -> c0, +1 -> cm
    const cplx<C> f = ccast<C, double>(cf.c[3 * h2 + (sw == 0 ? 1 : sw == 1 ? 0 : 2)]);
    const cplx<C> k = cscale<C>(cmul<C>(f, cs[r2][h2][i]), (C)a.coeff[4 * atom + i]);
    cplx<R>* dst = reinterpret_cast<cplx<R>*>(&a.kt[((int64_t)rr * a.n_atoms + atom) * 12 + sw * 4 + i]);
    dst[h2] = ccast<R, C>(k);
  }
  if (a.signl != nullptr && tid < 16) {
    const int rr = srun[tid];
    if (rr >= 0) {
      double2 sg = make_double2(0.0, 0.0);
      for (int i = 0; i < 4; ++i) {
        const cplx<C> t = cscale<C>(cmulc<C>(cs[tid][1][i], cs[tid][0][i]), (C)a.coeff[4 * atom + i]);
        sg.x += (double)t.x;
        sg.y += (double)t.y;
      }
      a.signl[(int64_t)rr * a.n_atoms + atom] = sg;
    }
  }
}

// ------------------------------------------------------------- chunked bra
// The same coefficients as k_bra_mfma, computed chunk by chunk: a workgroup copies the
// direction of RG runs on TP consecutive points into LDS (one coalesced pass over the
// vector, instead of a gather per ball entry: the balls overlap, every point lies in
// about five of them) and contracts every ball entry of the chunk from LDS.  A thread takes
// one piece (consecutive entries of one key) for one run and sums the sixteen products
// u_i * (primal, dual; re, im) over its entries; the pieces of a key are then added in
// order through LDS and each (run, chunk, key) sum is written to the partial array.  The
// finishing kernel adds a key's chunk sums in chunk order and applies the Bloch phases as
// k_bra_mfma does.  Workgroups of one chunk (its runs in groups of RG) are consecutive on
// one XCD, so the chunk's table is read from that XCD's L2.
template <typename R, typename C>
struct BraTileArgs {
  int32_t nruns, nchunks, nslots, need_status, nlogical;
  int64_t N;
  const int32_t* piece_off;
  const int32_t* piece_beg;
  const int32_t* piece_meta;
  const int32_t* slot_off;
  const int32_t* slot_piece;
  const int32_t* slot_pos;
  const int32_t* ent_pt;
  const R* ent_u;
  const Pair<R>* v;
  const int32_t* status;
  const int32_t* list;
  const int32_t* count;
  C* part;   // [run][slot in key order][16]: u_i times (primal re, primal im, dual re, dual im), i major
};

// Value of lane I of this lane's quad (quad_perm DPP: every lane of the quad reads lane I).
template <int I>
__device__ __forceinline__ int quad_pick(int v) {
  return __builtin_amdgcn_mov_dpp(v, I * 0x55, 0xF, 0xF, true);
}
template <int I>
__device__ __forceinline__ float quad_pick(float v) {
  return __int_as_float(quad_pick<I>(__float_as_int(v)));
}
template <int I>
__device__ __forceinline__ double quad_pick(double v) {
  return __hiloint2double(quad_pick<I>(__double2hiint(v)), quad_pick<I>(__double2loint(v)));
}

// Entry Q of a group of four consecutive entries, whose point and projector values lane Q of
// the quad loaded: the sixteen products with this lane's run, added in entry order.
template <int Q, typename R, typename C, typename U4>
__device__ __forceinline__ void bt_entry(C (&acc)[16], const Pair<R>* vj, int ptm, const U4& um) {
  const Pair<R> x = vj[quad_pick<Q>(ptm)];
  const C u4[4] = {(C)quad_pick<Q>(um.x), (C)quad_pick<Q>(um.y), (C)quad_pick<Q>(um.z), (C)quad_pick<Q>(um.w)};
  const C xs[4] = {(C)x.a.x, (C)x.a.y, (C)x.b.x, (C)x.b.y};
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[4 * i + k] += u4[i] * xs[k];
}
template <typename R, typename C, typename U4>
__device__ __forceinline__ void bt_group(C (&acc)[16], const Pair<R>* vj, int ptm, const U4& um) {
  bt_entry<0, R, C, U4>(acc, vj, ptm, um);
  bt_entry<1, R, C, U4>(acc, vj, ptm, um);
  bt_entry<2, R, C, U4>(acc, vj, ptm, um);
  bt_entry<3, R, C, U4>(acc, vj, ptm, um);
}

// BT_MAXP x RG threads: thread t takes piece t / RG of the chunk (at most BT_MAXP) for run
// t % RG of the group, so the RG threads of a piece read the same table entries.  The
// piece's bounds are requested before the staging barrier, so their latency overlaps the
// staging loads.  QX = 0: every thread loads each entry of its piece itself; QX = 1: the
// four lanes of a quad (one piece, RG a multiple of 4) load one entry each of a group of
// four and pass them round by DPP (a quarter of the table traffic and registers), the next
// group requested while the current one is used.  Both add the products in the same order.
template <typename R, typename C, int RG, int TP, int QX>
__global__ void __launch_bounds__(BT_MAXP * RG, 4) k_bra_tile(BraTileArgs<R, C> a) {
  static_assert(BT_MAXP * RG <= 1024, "one piece per thread row");
  // the staged directions (rows padded by one point against bank conflicts between the
  // runs of a piece), then in the same space the piece sums
  constexpr int VB = RG * (TP + 1) * (int)sizeof(Pair<R>);
  constexpr int SB = BT_MAXP * RG * 16 * (int)sizeof(C);
  constexpr int LDSB = VB > SB ? VB : SB;
  static_assert(LDSB <= 160 * 1024, "staging exceeds LDS");
  constexpr int NT = BT_MAXP * RG;
  constexpr int EB = BT_EB;   // entries whose table loads are issued together (pieces are padded to it)
  using U4 = typename vec4<R>::T;
  __shared__ __attribute__((aligned(16))) unsigned char lds[LDSB];
  __shared__ int srun[RG];
  const int nsl = (a.list != nullptr) ? *a.count : a.nruns;
  const int ngr = (nsl + RG - 1) / RG;
  const int nl = min(a.nlogical, ngr * a.nchunks);
  const int lb = remap_active(blockIdx.x, nl);
  if (lb < 0) return;
  const int c = lb / ngr;
  const int rg = lb - c * ngr;
  const int tid = threadIdx.x;
  int any = 0;
  if (tid < RG) {
    const int slot = rg * RG + tid;
    int run = -1;
    if (slot < nsl) {
      run = (a.list != nullptr) ? a.list[slot] : slot;
      if (a.status != nullptr && a.status[run] != a.need_status) run = -1;
    }
    srun[tid] = run;
    any = run >= 0;
  }
  if (!__syncthreads_or(any)) return;
  Pair<R>* vs = reinterpret_cast<Pair<R>*>(lds);
  const int64_t p0 = (int64_t)c * TP;
  const int np = (int)min<int64_t>(TP, a.N - p0);
  const int j = tid % RG, lp = tid / RG;
  const int run = srun[j];
  // this thread's piece
  const int pb = a.piece_off[c];
  const int npc = a.piece_off[c + 1] - pb;
  // with the quad exchange the lanes of a piece walk it together, also for an empty run slot
  // (staged from run 0's row, its sums never stored)
  const bool work = lp < npc && (QX > 0 || run >= 0);
  int beg = 0, end = 1;
  if (work) {
    beg = a.piece_beg[pb + lp];
    end = beg + (a.piece_meta[pb + lp] & 0xffff);
  }
  const U4* ut = reinterpret_cast<const U4*>(a.ent_u);
  {
    // every thread's share of the chunk is loaded before any of it is stored (loads are
    // unconditional, from a valid run and point: rows of empty run slots and points past
    // the cell's end are staged but never read)
    constexpr int SPT = RG * TP / NT;
    static_assert(SPT * NT == RG * TP, "staging covers the chunk");
    int rows[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) rows[q] = max(srun[(tid + q * NT) / TP], 0);
    Pair<R> tmp[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int i = tid + q * NT;
      const int pt = min(i % TP, np - 1);
      tmp[q] = a.v[(int64_t)rows[q] * a.N + p0 + pt];
    }
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int i = tid + q * NT;
      const int jj = i / TP, pt = i - jj * TP;
      vs[jj * (TP + 1) + pt] = tmp[q];
    }
  }
  __syncthreads();
  const Pair<R>* vj = vs + j * (TP + 1);
  C acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0;
  static_assert(QX == 0 || (EB == 4 && RG % 4 == 0), "quad exchange: groups of four entries, quads of one piece");
  if (QX == 1 && work) {
    const int ql = tid & 3;
    int pn = a.ent_pt[beg + ql];
    U4 un = ut[beg + ql];
    for (int e0 = beg; e0 < end; e0 += 4) {
      const int pc = pn;
      const U4 uc = un;
      if (e0 + 4 < end) {
        pn = a.ent_pt[e0 + 4 + ql];
        un = ut[e0 + 4 + ql];
      }
      bt_group<R, C, U4>(acc, vj, pc, uc);
    }
  } else if (QX == 0 && work) {
    for (int e0 = beg; e0 < end; e0 += EB) {
      int pts[EB];
      U4 us[EB];
#pragma unroll
      for (int q = 0; q < EB; ++q) {
        pts[q] = a.ent_pt[e0 + q];
        us[q] = ut[e0 + q];
      }
#pragma unroll
      for (int q = 0; q < EB; ++q) {
        const Pair<R> x = vj[pts[q]];
        const C u4[4] = {(C)us[q].x, (C)us[q].y, (C)us[q].z, (C)us[q].w};
        const C xs[4] = {(C)x.a.x, (C)x.a.y, (C)x.b.x, (C)x.b.y};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[4 * i + k] += u4[i] * xs[k];
      }
    }
  }
  __syncthreads();   // every thread is done with the staged directions
  C* psum = reinterpret_cast<C*>(lds);   // [local piece][run of the group][16]
  if (lp < npc) {
#pragma unroll
    for (int k = 0; k < 16; ++k) psum[(lp * RG + j) * 16 + k] = acc[k];
  }
  __syncthreads();
  const int so = a.slot_off[c];
  const int nsc = a.slot_off[c + 1] - so;
  for (int i = tid; i < nsc * RG * 16; i += NT) {
    const int ls = i / (RG * 16);
    const int rem = i - ls * (RG * 16);
    const int jj = rem >> 4, k = rem & 15;
    const int rr = srun[jj];
    if (rr < 0) continue;
    const int g = so + ls;
    const int q0 = a.slot_piece[g] - pb, q1 = a.slot_piece[g + 1] - pb;
    C sum = 0;
    for (int q = q0; q < q1; ++q) sum += psum[(q * RG + jj) * 16 + k];
    a.part[((int64_t)rr * a.nslots + a.slot_pos[g]) * 16 + k] = sum;
  }
}

template <typename R, typename C>
struct BraFinArgs {
  int32_t nruns, n_atoms, nslots, need_status, nlogical;
  const int32_t* key_off;
  const C* part;
  const R* coeff;
  const RunCoef* coef;
  const int32_t* status;
  const int32_t* list;
  const int32_t* count;
  Pair<R>* kt;
  double2* signl;
};

// One wave per (run, atom), four per workgroup: lane 16 s + k adds value k of segment s
// (cell shift w = s - 1) over the key's chunks in chunk order; then the Bloch phases, K
// and the nonlocal part of sigma exactly as at the end of k_bra_mfma.
template <typename R, typename C>
__global__ void __launch_bounds__(256) k_bra_fin(BraFinArgs<R, C> a) {
  __shared__ C gs[4][3][16];
  __shared__ cplx<C> cs[4][2][4];
  const int nsl = (a.list != nullptr) ? *a.count : a.nruns;
  const int nl = min(a.nlogical, nsl * ((a.n_atoms + 3) / 4));
  const int lb = remap_active(blockIdx.x, nl);
  if (lb < 0) return;
  const int agr = (a.n_atoms + 3) / 4;
  const int slot = lb / agr;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int atom = (lb - slot * agr) * 4 + wv;
  int run = (a.list != nullptr) ? a.list[slot] : slot;
  if (a.status != nullptr && a.status[run] != a.need_status) run = -1;
  const bool ok = run >= 0 && atom < a.n_atoms;
  if (ok && lane < 48) {
    const int sg = lane >> 4, k = lane & 15;
    const int key = 3 * atom + sg;
    C sum = 0;
    const C* pr = a.part + (int64_t)run * a.nslots * 16 + k;
    const int t0 = a.key_off[key], t1 = a.key_off[key + 1];
    // the key's chunk sums are contiguous; sixteen at a time, loads in flight together, the
    // additions in chunk order
    constexpr int FB = 16;
    for (int t = t0; t < t1; t += FB) {
      C x[FB];
#pragma unroll
      for (int q = 0; q < FB; ++q) x[q] = pr[(int64_t)min(t + q, t1 - 1) * 16];
#pragma unroll
      for (int q = 0; q < FB; ++q)
        if (t + q < t1) sum += x[q];
    }
    gs[wv][sg][k] = sum;
  }
  __syncthreads();
  if (ok && lane < 8) {
    // c[half][i] = sum_s z^w c_s: w = -1 -> 1/z (primal) or conj z (dual), +1 -> z or 1/conj z
    const int h2 = lane >> 2, i = lane & 3;
    const RunCoef& cf = a.coef[run];
    cplx<C> acc = mkc<C>(0, 0);
    for (int sg = 0; sg < 3; ++sg) {
      const cplx<C> c = mkc<C>(gs[wv][sg][4 * i + 2 * h2], gs[wv][sg][4 * i + 2 * h2 + 1]);
      cplx<C> t = c;
      if (sg != 1) t = cmul<C>(ccast<C, double>(cf.c[3 * h2 + (sg == 0 ? 2 : 1)]), c);
      acc = cadd<C>(acc, t);
    }
    cs[wv][h2][i] = acc;
  }
  __syncthreads();
  if (ok && lane < 24) {
    const int h2 = lane & 1, i = (lane >> 1) & 3, sw = lane >> 3;
    const RunCoef& cf = a.coef[run];
    // K[w][i] = h z^-w c: w = -1 -> cp, 0 -> c0, +1 -> cm
    const cplx<C> f = ccast<C, double>(cf.c[3 * h2 + (sw == 0 ? 1 : sw == 1 ? 0 : 2)]);
    const cplx<C> k = cscale<C>(cmul<C>(f, cs[wv][h2][i]), (C)a.coeff[4 * atom + i]);
    cplx<R>* dst = reinterpret_cast<cplx<R>*>(&a.kt[((int64_t)run * a.n_atoms + atom) * 12 + sw * 4 + i]);
    dst[h2] = ccast<R, C>(k);
  }
  if (ok && a.signl != nullptr && lane == 32) {
    double2 sg = make_double2(0.0, 0.0);
    for (int i = 0; i < 4; ++i) {
      const cplx<C> t = cscale<C>(cmulc<C>(cs[wv][1][i], cs[wv][0][i]), (C)a.coeff[4 * atom + i]);
      sg.x += (double)t.x;
      sg.y += (double)t.y;
    }
    a.signl[(int64_t)run * a.n_atoms + atom] = sg;
  }
}

size_t bra_tile_part_bytes(const cbs_system* s, int32_t nruns) {
  const int32_t ns = std::max(s->proj.bt[0].nslots, s->proj.bt[1].nslots);
  return (size_t)std::max(nruns, 0) * (size_t)ns * 16 * sizeof(double);
}

template <typename R, typename C, int RG, int QX>
static void launch_tile_qx(int tp, int grid, hipStream_t st, const BraTileArgs<R, C>& t) {
  if (tp == 256)
    hipLaunchKernelGGL((k_bra_tile<R, C, RG, 256, QX>), dim3(grid), dim3(BT_MAXP * RG), 0, st, t);
  else
    hipLaunchKernelGGL((k_bra_tile<R, C, RG, 512, QX>), dim3(grid), dim3(BT_MAXP * RG), 0, st, t);
}

template <typename R, typename C, int RG>
static void launch_tile_tp(int tp, int qx, int grid, hipStream_t st, const BraTileArgs<R, C>& t) {
  switch (qx) {
    case 1: launch_tile_qx<R, C, RG, 1>(tp, grid, st, t); break;
    default: launch_tile_qx<R, C, RG, 0>(tp, grid, st, t); break;
  }
}

template <typename R, typename C>
static int32_t launch_bra_tile(const cbs_system* s, const ChunkTables& d, int rg, int32_t nruns, const void* v,
                               const RunCoef* coef, const int32_t* status, int32_t need_status, void* kt,
                               double2* signl, hipStream_t st, const int32_t* list, const int32_t* count,
                               void* part) {
  const Projector& pr = s->proj;
  if (d.tp != 256 && d.tp != 512) {
    set_error("chunked bra: chunk length %d unsupported", d.tp);
    return CBS_EINVAL;
  }
  BraTileArgs<R, C> t;
  t.nruns = nruns;
  t.nchunks = d.nchunks;
  t.nslots = d.nslots;
  t.need_status = need_status;
  t.nlogical = ((nruns + rg - 1) / rg) * d.nchunks;
  t.N = s->N;
  t.piece_off = d.piece_off;
  t.piece_beg = d.piece_beg;
  t.piece_meta = d.piece_meta;
  t.slot_off = d.slot_off;
  t.slot_piece = d.slot_piece;
  t.slot_pos = d.slot_pos;
  t.ent_pt = d.ent_pt;
  t.ent_u = std::is_same<R, double>::value ? (const R*)d.u64 : (const R*)d.u32;
  t.v = (const Pair<R>*)v;
  t.status = status;
  t.list = list;
  t.count = count;
  t.part = (C*)part;
  const int grid = (t.nlogical + 7) / 8 * 8;
  const int qx = s->bra_qx[std::is_same<R, float>::value ? 1 : 0];
  if (rg == 4)
    launch_tile_tp<R, C, 4>(d.tp, qx, grid, st, t);
  else if (rg == 8)
    launch_tile_tp<R, C, 8>(d.tp, qx, grid, st, t);
  else {
    set_error("chunked bra: %d runs per workgroup unsupported", rg);
    return CBS_EINVAL;
  }
  CBS_HIP(hipGetLastError());
  BraFinArgs<R, C> f;
  f.nruns = nruns;
  f.n_atoms = pr.n_atoms;
  f.nslots = d.nslots;
  f.need_status = need_status;
  f.nlogical = nruns * ((pr.n_atoms + 3) / 4);
  f.key_off = d.key_off;
  f.part = (const C*)part;
  f.coeff = std::is_same<R, double>::value ? (const R*)pr.coeff64 : (const R*)pr.coeff32;
  f.coef = coef;
  f.status = status;
  f.list = list;
  f.count = count;
  f.kt = (Pair<R>*)kt;
  f.signl = signl;
  const int fgrid = (f.nlogical + 7) / 8 * 8;
  hipLaunchKernelGGL((k_bra_fin<R, C>), dim3(fgrid), dim3(256), 0, st, f);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

static bool bra_plain() {
  const char* e = getenv("CBS_NO_MFMA");
  return e && e[0] == '1';
}

template <typename R>
int32_t launch_bra(const cbs_system* s, int32_t nruns, const void* v, const RunCoef* coef,
                   const int32_t* status, int32_t need_status, void* kt, double2* signl,
                   hipStream_t st, bool phased, const int32_t* list, const int32_t* count,
                   bool short_list, void* tile_part) {
  const Projector& pr = s->proj;
  if (pr.n_atoms == 0 || nruns <= 0) return CBS_OK;
  const int pi = std::is_same<R, float>::value ? 1 : 0;
  if (tile_part != nullptr && phased && !short_list && !bra_plain() && s->bra_tile[pi] > 0 &&
      pr.bt[s->bra_tp[pi]].nslots > 0) {
    const ChunkTables& d = pr.bt[s->bra_tp[pi]];
    if ((list == nullptr) != (count == nullptr)) {
      set_error("launch_bra: a run list needs its count");
      return CBS_EINVAL;
    }
    if constexpr (std::is_same<R, float>::value) {
      if (lo_arith_fp32())
        return launch_bra_tile<R, float>(s, d, s->bra_tile[pi], nruns, v, coef, status, need_status, kt, signl,
                                         st, list, count, tile_part);
    }
    return launch_bra_tile<R, double>(s, d, s->bra_tile[pi], nruns, v, coef, status, need_status, kt, signl,
                                      st, list, count, tile_part);
  }
  BraArgs<R> a;
  a.nruns = nruns;
  a.n_atoms = pr.n_atoms;
  a.nlogical = nruns * pr.n_atoms;
  a.need_status = need_status;
  a.N = s->N;
  a.seg = pr.seg;
  a.idx = pr.ball_idx;
  a.u = std::is_same<R, double>::value ? (const R*)pr.ball_u64 : (const R*)pr.ball_u32;
  a.coeff = std::is_same<R, double>::value ? (const R*)pr.coeff64 : (const R*)pr.coeff32;
  a.v = (const Pair<R>*)v;
  a.coef = coef;
  a.status = status;
  a.kt = (Pair<R>*)kt;
  a.signl = signl;
  a.list = list;   // runs: the list entries, or all runs (both filtered by status if given)
  a.count = count;
  const char* bm = getenv("CBS_BRA_MAP");
  a.spread = bm ? !(bm[0] == 'x') : (s->bra_spread[pi] != 0);
  if ((list == nullptr) != (count == nullptr)) {
    set_error("launch_bra: a run list needs its count");
    return CBS_EINVAL;
  }
  if (phased && !bra_plain()) {
    a.nlogical = ((nruns + 15) / 16) * pr.n_atoms;
    const int grid = (a.nlogical + 7) / 8 * 8;
    const bool f32 = std::is_same<R, float>::value && lo_arith_fp32();
    if (short_list && f32)
      hipLaunchKernelGGL((k_bra_mfma<R, float, 16>), dim3(grid), dim3(1024), 0, st, a);
    else if (short_list)
      hipLaunchKernelGGL((k_bra_mfma<R, double, 16>), dim3(grid), dim3(1024), 0, st, a);
    else if (f32 && s->bra_nw[pi] == 8)
      hipLaunchKernelGGL((k_bra_mfma<R, float, 8>), dim3(grid), dim3(512), 0, st, a);
    else if (f32)
      hipLaunchKernelGGL((k_bra_mfma<R, float, 4>), dim3(grid), dim3(256), 0, st, a);
    else if (s->bra_nw[pi] == 8)
      hipLaunchKernelGGL((k_bra_mfma<R, double, 8>), dim3(grid), dim3(512), 0, st, a);
    else
      hipLaunchKernelGGL((k_bra_mfma<R, double, 4>), dim3(grid), dim3(256), 0, st, a);
  } else {
    const int grid = (a.nlogical + 7) / 8 * 8;
    hipLaunchKernelGGL(k_bra<R>, dim3(grid), dim3(256), 0, st, a);
  }
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

// --------------------------------------------------------------- BiCG residual update
// r -= alpha q, rt -= conj(alpha) qt with q = local part + ket; partial sums of
// rho = rt^H r, ||r||^2, ||rt||^2 per (run, chunk).
template <typename R>
struct UpdArgs {
  int32_t nchunks, nlogical, n_atoms, need_status, nruns;
  int64_t N;
  Pair<R>* r;
  const Pair<R>* q;
  const Pair<R>* kt;
  const double2* alpha;
  const int32_t* status;
  double* part;   // [run][chunk][4]
  const int32_t* list;    // active runs (ascending) or NULL
  const int32_t* count;   // device count of list entries
  const int32_t* grp_off;   // grouped ket tables (see Projector)
  const int32_t* grp_key;
  const int32_t* grp_mask;
  const R* grp_u;
};

// One workgroup updates UR = 4 runs (consecutive active-list slots) over a chunk of point
// groups; a wave takes one group of KG = 64 points at a time.  The ket of a group is a
// small product on the matrix cores: for each of the group's keys (atom, shift), U [64
// points x 4 projectors] (the grouped table) times K [4 projectors x 16 columns] (4 runs x
// primal/dual x re/im), accumulated over the keys with MFMA 16x16x4 in four 16-point row
// blocks.  One vector load brings a key's K operand for all four runs; keys go in
// batches of four whose loads are issued while the previous batch is on the matrix cores.
// The 64 x 16 result goes through LDS to lane = point for the update of r.
constexpr int UR = 4;

template <typename R, typename C>
__global__ void __launch_bounds__(256) k_update(UpdArgs<R> a) {
  constexpr int KB = 4;   // keys per batch
  __shared__ double red[4][UR][4];
  __shared__ C tile[4][KG][17];
  const int nslots = (a.list != nullptr) ? *a.count : a.nruns;
  const int nrc = (nslots + UR - 1) / UR;
  const int nl = min(a.nlogical, nrc * a.nchunks);
  const int lb = remap_active(blockIdx.x, nl);
  if (lb < 0) return;
  // run groups vary fastest: the workgroups that one XCD has in flight share a chunk of
  // point groups, so its slice of the grouped table is fetched into that XCD's L2 once
  // rather than once per run group
  const int ch = lb / nrc;
  const int rc = lb - ch * nrc;
  int run[UR];
  bool act[UR];
  bool any = false;
#pragma unroll
  for (int k = 0; k < UR; ++k) {
    const int slot = rc * UR + k;
    run[k] = 0;
    act[k] = false;
    if (slot < nslots) {
      run[k] = (a.list != nullptr) ? a.list[slot] : slot;
      act[k] = a.status[run[k]] == a.need_status;
    }
    any = any || act[k];
  }
  if (!any) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  cplx<C> aa[UR];
#pragma unroll
  for (int k = 0; k < UR; ++k) {
    run[k] = __builtin_amdgcn_readfirstlane(run[k]);
    const double2 al = act[k] ? a.alpha[run[k]] : make_double2(0, 0);
    aa[k] = mkc<C>((C)al.x, (C)al.y);
  }
  typedef const CBS_CONST_AS int32_t* cint_p;
  const cint_p goff = (cint_p)a.grp_off;
  const cint_p gkey = (cint_p)a.grp_key;
  const int64_t ngroups = (a.N + KG - 1) / KG;
  const int64_t gpc = (ngroups + a.nchunks - 1) / a.nchunks;
  const int64_t g0 = ch * gpc;
  const int64_t g1 = (g0 + gpc < ngroups) ? g0 + gpc : ngroups;
  const int64_t kstride = (int64_t)a.n_atoms * 12;
  // MFMA operand roles: lane l feeds U[point l%16 of a row block][projector l/16] and
  // K[projector l/16][column l%16], column c = 4 * run slot + 2 * (dual) + (imaginary)
  const int orow = lane & 15, ok4 = lane >> 4;
  const int bslot = orow >> 2;
  const int krun = bslot == 0 ? run[0] : bslot == 1 ? run[1] : bslot == 2 ? run[2] : run[3];
  const R* kcol = (a.kt != nullptr)
                      ? reinterpret_cast<const R*>(a.kt + (int64_t)krun * kstride) + (orow & 3) + 4 * ok4
                      : nullptr;
  double s[UR][4];
#pragma unroll
  for (int k = 0; k < UR; ++k) s[k][0] = s[k][1] = s[k][2] = s[k][3] = 0;
  for (int64_t g = g0 + wv; g < g1; g += 4) {
    typename mf4<C>::T acc[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = {0, 0, 0, 0};
    if (kcol != nullptr) {
      const int e0 = goff[g], e1 = goff[g + 1];
      for (int eb = e0; eb < e1; eb += 64) {
        // up to 64 keys of the group in one vector load (lane j holds key eb + j); the
        // batches read them with readlane, so no scalar load waits inside the loop
        const int nk = min(64, e1 - eb);
        const int keyv = (lane < nk) ? a.grp_key[eb + lane] : 0;
        const int maskv = (lane < nk) ? a.grp_mask[eb + lane] : 0;
        C kbA[KB], ubA[KB][4], kbB[KB], ubB[KB][4];
        int mA[KB], mB[KB];
        // operands of keys j0 .. j0+KB-1 of this chunk (no blocks past the last key; the
        // 16-point blocks where the key's table is zero are neither loaded nor multiplied)
        auto load = [&](int j0, C (&kb)[KB], C (&ub)[KB][4], int (&m)[KB]) {
#pragma unroll
          for (int j = 0; j < KB; ++j) {
            const bool valid = j0 + j < nk;   // wave-uniform
            const int jj = valid ? j0 + j : 0;
            const int key = __builtin_amdgcn_readlane(keyv, jj);
            m[j] = valid ? __builtin_amdgcn_readlane(maskv, jj) : 0;
            const int koff = (key >> 2) * 12 + (key & 3) * 4;
            kb[j] = (C)kcol[4 * koff];
            const R* up = a.grp_u + ((int64_t)(eb + jj) * KG + orow) * 4 + ok4;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) ub[j][rb] = ((m[j] >> rb) & 1) ? (C)up[64 * rb] : (C)0;
          }
        };
        auto mma = [&](const C (&kb)[KB], const C (&ub)[KB][4], const int (&m)[KB]) {
#pragma unroll
          for (int j = 0; j < KB; ++j)
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
              if ((m[j] >> rb) & 1) acc[rb] = mfma16x16x4(ub[j][rb], kb[j], acc[rb]);
        };
        // two register buffers: the loads of the next batch are in flight while the
        // MFMAs of the current one run
        load(0, kbA, ubA, mA);
        for (int j0 = 0; j0 < nk; j0 += 2 * KB) {
          load(j0 + KB, kbB, ubB, mB);
          mma(kbA, ubA, mA);
          if (j0 + KB >= nk) break;
          load(j0 + 2 * KB, kbA, ubA, mA);
          mma(kbB, ubB, mB);
        }
      }
    }
    // the 64 x 16 ket tile to lane = point (wave-private LDS rows)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) tile[wv][16 * rb + mfma16_row<C>(lane, v)][orow] = acc[rb][v];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const C* kt = tile[wv][lane];
    const int64_t n = g * KG + lane;
    if (n < a.N) {
      Pair<C> q[UR], r[UR];
#pragma unroll
      for (int k = 0; k < UR; ++k) {
        const int64_t gi = (int64_t)run[k] * a.N + n;
        q[k] = pcast<C, R>(a.q[gi]);
        r[k] = pcast<C, R>(a.r[gi]);
      }
#pragma unroll
      for (int k = 0; k < UR; ++k) {
        if (!act[k]) continue;
        Pair<C> qk = q[k];
        qk.a = cadd<C>(qk.a, mkc<C>(kt[4 * k], kt[4 * k + 1]));
        qk.b = cadd<C>(qk.b, mkc<C>(kt[4 * k + 2], kt[4 * k + 3]));
        Pair<C> rk = r[k];
        rk.a = csub<C>(rk.a, cmul<C>(aa[k], qk.a));
        rk.b = csub<C>(rk.b, cmul<C>(cconj<C>(aa[k]), qk.b));
        const Pair<R> rs = pcast<R, C>(rk);
        a.r[(int64_t)run[k] * a.N + n] = rs;
        rk = pcast<C, R>(rs);   // the dots of the stored residual
        const cplx<C> rho = cmulc<C>(rk.b, rk.a);
        s[k][0] += (double)rho.x;
        s[k][1] += (double)rho.y;
        s[k][2] += (double)cabs2<C>(rk.a);
        s[k][3] += (double)cabs2<C>(rk.b);
      }
    }
    // the tile rows are rewritten by the next group
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
#pragma unroll
  for (int k = 0; k < UR; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double t = wsum<double>(s[k][j]);
      if (lane == 0) red[wv][k][j] = t;
    }
  __syncthreads();
  if (tid < 4 * UR) {
    const int k = tid >> 2, j = tid & 3;
    if (act[k])
      a.part[((int64_t)run[k] * a.nchunks + ch) * 4 + j] = red[0][k][j] + red[1][k][j] + red[2][k][j] + red[3][k][j];
  }
}

int32_t update_chunks(const cbs_system* s) {
  const int64_t per = std::max<int64_t>(s->upd_pts, 256);
  return (int32_t)((s->N + per - 1) / per);
}

template <typename R>
int32_t launch_update(const cbs_system* s, int32_t nruns, void* r, const void* q, const void* kt,
                      const double2* alpha, const int32_t* status, int32_t need_status, double* part,
                      int32_t nchunks, hipStream_t st, const int32_t* list, const int32_t* count) {
  if ((list == nullptr) != (count == nullptr)) {
    set_error("launch_update: a run list needs its count");
    return CBS_EINVAL;
  }
  if (nruns <= 0) return CBS_OK;
  UpdArgs<R> a;
  a.need_status = need_status;
  a.nchunks = nchunks;
  a.nruns = nruns;
  a.nlogical = ((nruns + UR - 1) / UR) * nchunks;
  a.n_atoms = s->proj.n_atoms;
  a.N = s->N;
  a.r = (Pair<R>*)r;
  a.q = (const Pair<R>*)q;
  a.kt = (s->proj.n_atoms > 0) ? (const Pair<R>*)kt : nullptr;
  a.alpha = alpha;
  a.status = status;
  a.part = part;
  a.list = list;
  a.count = count;
  a.grp_off = s->proj.grp_off;
  a.grp_key = s->proj.grp_key;
  a.grp_mask = s->proj.grp_mask;
  a.grp_u = std::is_same<R, double>::value ? (const R*)s->proj.grp_u64 : (const R*)s->proj.grp_u32;
  const int grid = (a.nlogical + 7) / 8 * 8;
  if (std::is_same<R, float>::value && lo_arith_fp32())
    hipLaunchKernelGGL((k_update<R, float>), dim3(grid), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_update<R, double>), dim3(grid), dim3(256), 0, st, a);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

// ------------------------------------------------------------------ apply: q += ket
template <typename R>
__global__ void __launch_bounds__(256) k_ket_add(int64_t N, int32_t nruns, int32_t n_atoms, Pair<R>* q,
                                                 const Pair<R>* kt, const int32_t* pt_off,
                                                 const int32_t* pt_key, const R* pt_u) {
  const int64_t total = N * nruns;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t run = g / N, n = g - run * N;
    const Pair<R> k = ket_at<R>(n, run * n_atoms * 12, pt_off, pt_key, pt_u, kt);
    Pair<R> v = q[g];
    v.a = cadd<R>(v.a, k.a);
    v.b = cadd<R>(v.b, k.b);
    q[g] = v;
  }
}

template <typename R>
int32_t launch_ket_add(const cbs_system* s, int32_t nruns, void* q, const void* kt, hipStream_t st) {
  if (s->proj.n_atoms == 0 || nruns <= 0) return CBS_OK;
  const int64_t total = s->N * nruns;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_ket_add<R>, dim3(grid), dim3(256), 0, st, s->N, nruns, s->proj.n_atoms,
                     (Pair<R>*)q, (const Pair<R>*)kt, s->proj.pt_off, s->proj.pt_key,
                     std::is_same<R, double>::value ? (const R*)s->proj.pt_u64 : (const R*)s->proj.pt_u32);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

// ------------------------------------------------------------------ layout conversions
template <typename R>
__global__ void k_to_pairs(int64_t N, int32_t nvec, const cplx<R>* x, Pair<R>* p) {
  const int64_t npair = (nvec + 1) / 2;
  const int64_t total = npair * N;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = g / N, n = g - k * N;
    Pair<R> v;
    v.a = x[(2 * k) * N + n];
    v.b = (2 * k + 1 < nvec) ? x[(2 * k + 1) * N + n] : mkc<R>(0, 0);
    p[g] = v;
  }
}

template <typename R>
__global__ void k_from_pairs(int64_t N, int32_t nvec, const Pair<R>* p, cplx<R>* y) {
  const int64_t npair = (nvec + 1) / 2;
  const int64_t total = npair * N;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = g / N, n = g - k * N;
    const Pair<R> v = p[g];
    y[(2 * k) * N + n] = v.a;
    if (2 * k + 1 < nvec) y[(2 * k + 1) * N + n] = v.b;
  }
}

template <typename R>
int32_t launch_to_pairs(int64_t N, int32_t nvec, const void* x, void* pairs, hipStream_t st) {
  const int64_t total = (int64_t)((nvec + 1) / 2) * N;
  if (total == 0) return CBS_OK;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_to_pairs<R>, dim3(grid), dim3(256), 0, st, N, nvec, (const cplx<R>*)x,
                     (Pair<R>*)pairs);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

template <typename R>
int32_t launch_from_pairs(int64_t N, int32_t nvec, const void* pairs, void* y, hipStream_t st) {
  const int64_t total = (int64_t)((nvec + 1) / 2) * N;
  if (total == 0) return CBS_OK;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_from_pairs<R>, dim3(grid), dim3(256), 0, st, N, nvec, (const Pair<R>*)pairs,
                     (cplx<R>*)y);
  CBS_HIP(hipGetLastError());
  return CBS_OK;
}

#define INST(R)                                                                                   \
  template int32_t launch_bra<R>(const cbs_system*, int32_t, const void*, const RunCoef*,         \
                                 const int32_t*, int32_t, void*, double2*, hipStream_t, bool,     \
                                 const int32_t*, const int32_t*, bool, void*);                    \
  template int32_t launch_update<R>(const cbs_system*, int32_t, void*, const void*, const void*,  \
                                    const double2*, const int32_t*, int32_t, double*, int32_t,    \
                                    hipStream_t, const int32_t*, const int32_t*);                 \
  template int32_t launch_ket_add<R>(const cbs_system*, int32_t, void*, const void*, hipStream_t); \
  template int32_t launch_to_pairs<R>(int64_t, int32_t, const void*, void*, hipStream_t);         \
  template int32_t launch_from_pairs<R>(int64_t, int32_t, const void*, void*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace cbs
