// BiCG batch state shared by the step-1 driver and the solver.
#pragma once

#include <vector>

#include "cbs_internal.hpp"

namespace cbs {

// Per-run scalars of the BiCG recurrences (device arrays, one entry per run).
struct BicgScal {
  double2* alpha;
  double2* xcoef;     // pending x update coefficient (applied by the next stencil pass)
  double2* beta;
  double2* rho;
  double2* rho_prev;
  double* vn2;        // ||v||^2 of the run's right-hand side
  double* relres;     // [2*run]: primal, dual relative residual (last known)
  double* ru_thr;     // next reliable update when the recursive residual falls below this
  int32_t* status;
  int32_t* iters;
  int32_t* brk;
  int32_t* halt;
  int32_t* nru;
  int32_t* n_active;  // [1]
};

template <typename T>
struct BicgBatch {
  cbs_system* sys;
  int32_t nruns, L, n_q, ntiles, nchunks, tile_y;
  const double2* V;            // [L][N] right-hand sides
  const RunCoef* coef;         // [nruns]
  Pair<T>* R;
  Pair<T>* Pb[2];
  Pair<T>* Q;
  Pair<T>* X;
  Pair<T>* KT;
  Pair<double>* Y;             // solutions (primal, dual), complex128
  Pair<double>* Q64;
  Pair<double>* KT64;
  double2* sig_part;
  double2* signl;
  double* upd_part;
  double* ru_part;
  BicgScal sc;
  double tol, ru_factor;
  int32_t max_iter, max_ru, half_stop;
  // profiling of the stencil launches (events recorded around each one when set)
  hipEvent_t pev0 = nullptr, pev1 = nullptr;
  int64_t prof_launches = 0;
  double prof_ms = 0, prof_bytes = 0;
};

struct NodeSolve {
  int32_t nruns = 0;
  Pair<double>* Y = nullptr;   // workspace-owned, valid until the next solve on the system
  std::vector<int32_t> iters, status;
  std::vector<double> relres;
  double ms = 0;
  int64_t prof_launches = 0;
  double prof_ms = 0, prof_bytes = 0;
};

template <typename T> int32_t bicg_alloc(BicgBatch<T>& b);
template <typename T>
int32_t bicg_run(std::vector<BicgBatch<T>*>& batches, hipStream_t user, int32_t chunk, int32_t max_iter,
                 double* elapsed_ms, bool profile = false);
template <typename T>
int32_t bicg_collect(BicgBatch<T>& b, std::vector<int32_t>& iters, std::vector<double>& relres,
                     std::vector<int32_t>& status, hipStream_t st);
void node_coefs(const double2* z, int32_t n_z, int32_t L, double E, std::vector<RunCoef>& out);
int32_t solve_nodes(cbs_system* s, double E, const double2* z, int32_t n_z, int32_t L, const double2* V,
                    const cbs_params* prm, hipStream_t st, NodeSolve& out);
int32_t split_pairs(int64_t N, int32_t nruns, const Pair<double>* Y, double2* ya, double2* yb, hipStream_t st);
int32_t check_params(const cbs_params* p, bool need_moments);

}  // namespace cbs
