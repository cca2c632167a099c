// BiCG state shared by the step-1 driver and the solver.
#pragma once

#include <vector>

#include "cbs_internal.hpp"

namespace cbs {

// Run states.  A run lives in the low-precision phase (complex64 recurrences) or the
// high-precision phase (complex128); the state encodes the phase so every kernel
// filters its runs with one comparison.
enum BicgState : int32_t {
  ST_ACT_LO = 0,   // iterating in complex64 (residual already small)
  ST_RU_LO = 1,    // complex64 run marked for a residual replacement this iteration
  ST_DONE = 2,     // true complex128 residual below tol (primal and dual)
  ST_NOCONV = 3,   // iteration or replacement cap reached
  ST_BREAKDOWN = 4,
  ST_HALTED = 5,   // stopped by the half-of-the-nodes rule
  ST_ACT_HI = 6,   // iterating in complex128
  ST_RU_HI = 7     // complex128 run marked for the final true-residual check
};

// Per-run scalars of the BiCG recurrences (device arrays, one entry per run).
struct BicgScal {
  double2* alpha;
  double2* xcoef;     // pending x update coefficient (applied by the next stencil pass)
  double2* beta;
  double2* rho;
  double2* rho_prev;
  double* vn2;        // ||v||^2 of the run's right-hand side
  double* relres;     // [2*run]: primal, dual relative residual (last known)
  double* ru_thr;     // complex64 phase: next replacement below this; -1: kept in complex128
  double* rmin;       // smallest max(primal, dual) residual since the last replacement
  int32_t* status;
  int32_t* iters;
  int32_t* brk;
  int32_t* halt;
  int32_t* nru;
  int32_t* conv;      // phase change this iteration: 1 widen to complex128, 2 narrow to complex64
  int32_t* ru_it;     // iteration of the last replacement (complex64 stagnation guard)
  int32_t* nrestart;  // complex64 -> complex128 restarts of the run
  int32_t* ru_par;    // parity of the iteration that marked the run for replacement (where its
                      // latest search direction is)
  int32_t* n_active;  // [3]: active runs in the complex64 / complex128 phase; runs marked
                      // for residual replacement
  int32_t* list;      // [3][nruns]: the runs of each of those sets, ascending (n_active entries)
};

// Vectors of one precision (pairs: primal, dual per point, run-major).
template <typename T>
struct BicgVecs {
  Pair<T>* R = nullptr;
  Pair<T>* Pb[2] = {nullptr, nullptr};
  Pair<T>* Q = nullptr;
  Pair<T>* X = nullptr;
  Pair<T>* KT = nullptr;
  double2* sig = nullptr;   // [run][tile] stencil partials of sigma
  int32_t tile_y = 0, ntiles = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;   // profiling of the stencil launches
  int64_t prof_launches = 0;
  double prof_ms = 0, prof_bytes = 0;
};

// Work queue of a batched solve: the solve's runs are slots, each holding one item
// (energy e, node j, right-hand side l) at a time; a slot whose item finished hands the
// item's solution to the moments of its energy and takes the next item.
struct QueueState {
  int32_t n_items = 0, nq = 0, L = 1, nE = 0, M2 = 0, conj = 0;
  int32_t* slot_item = nullptr;       // [nruns] item held by the slot, -1: none
  int32_t* slot_rhs = nullptr;        // [nruns] right-hand side l of the slot's item
  int32_t* head = nullptr;            // [2]: next item to issue, entries of rlist
  int32_t* rlist = nullptr;           // [nruns] slots retiring or refilled this iteration
  const RunCoef* item_coef = nullptr; // [nE * nq] coefficients of (energy, node)
  RunCoef* coef_w = nullptr;          // [nruns] the slots' coefficients (the solve's coef)
  int32_t* item_iters = nullptr;      // [n_items]
  int32_t* item_status = nullptr;     // [n_items]
  double* item_relres = nullptr;      // [2 n_items]
  double2* S = nullptr;               // [nE][M2][L][N] moments
  const double2* ca = nullptr;        // [nq][M2] w1 z1^k
  const double2* cb = nullptr;        // [nq][M2] w2 z2^k
  int32_t init_chunks = 0;            // point chunks of the refill initialisation
};

// One BiCG solve over a set of runs of one system (energies and nodes mixed freely:
// every run carries its own coefficients and energy).
struct BicgSolve {
  cbs_system* sys = nullptr;
  int32_t nruns = 0, L = 1, n_q = 0, nchunks = 0;
  int32_t ru_chunks = 0;   // work chunks per run of the residual replacement (ru_part)
  const double2* V = nullptr;       // [L][N]; run r uses right-hand side r % L
  const double2* Vd = nullptr;      // dual right-hand sides (same indexing), NULL: V
  const RunCoef* coef = nullptr;    // [nruns]
  const double* vn2_ref = nullptr;  // [nruns] ||v||^2 the residuals are measured against (NULL: the
                                    // initial residual's; set when solving for a correction)
  bool mixed = false;               // start in the complex64 phase
  BicgVecs<float> lo;               // complex64 phase (mixed only)
  BicgVecs<double> hi;              // complex128 phase (also the FP64 residual buffers)
  Pair<double>* Y = nullptr;        // solutions (primal, dual), complex128
  double2* signl = nullptr;
  double* upd_part = nullptr;
  double* ru_part = nullptr;
  void* bra_part = nullptr;   // chunk sums of the chunked bra (NULL: the per-atom bra)
  BicgScal sc{};
  double tol = 1e-10, ru_factor = 1e-2, narrow_tol = 0.0;
  double div_factor = 1e6;   // a residual this far above its smallest since the last replacement: diverging
  int32_t max_iter = 10000, max_ru = 1000, half_stop = 0;
  int32_t lo_window = 300;   // complex64 iterations without a 100x drop before a forced replacement
  double* hist = nullptr;    // [hist_rows][nruns][2] recursive relative residuals, NULL: not recorded
  int32_t hist_stride = 0, hist_rows = 0;   // row i holds iteration (i + 1) * hist_stride
  QueueState* q = nullptr;   // batched work queue, NULL: every run is its own item
};

// Optional residual-history request of solve_nodes (device buffer owned by the workspace).
struct HistReq {
  int32_t stride = 0, rows = 0;
  double* host = nullptr;    // [rows][nruns][2], receives the rows after the solve
};

struct NodeSolve {
  int32_t nruns = 0;
  Pair<double>* Y = nullptr;   // workspace-owned, valid until the next solve on the system
  std::vector<int32_t> iters, status;
  std::vector<double> relres;
  double ms = 0;
  int64_t prof_launches = 0, prof_lo_launches = 0;   // complex128 / complex64 stencil
  double prof_ms = 0, prof_bytes = 0, prof_lo_ms = 0, prof_lo_bytes = 0;
  int32_t n_ru = 0;
  int64_t restarts = 0;   // complex64 -> complex128 restarts, summed over the runs
};

int32_t bicg_alloc(BicgSolve& b, const char* tag);
// Work queue: allocation (item tables, moments) and the initial fill of the slots.
int32_t queue_alloc(BicgSolve& b, QueueState& q, const std::vector<RunCoef>& item_coef,
                    const std::vector<double2>& ca, const std::vector<double2>& cb, const char* tag,
                    hipStream_t st);
int32_t bicg_run(std::vector<BicgSolve*>& solves, hipStream_t user, int32_t chunk, int32_t max_iter,
                 double* elapsed_ms, bool profile);
int32_t bicg_collect(BicgSolve& b, NodeSolve& out, hipStream_t st);
void node_coefs(const double2* z, int32_t n_z, int32_t L, double E, std::vector<RunCoef>& out);
int32_t solve_nodes(cbs_system* s, double E, const double2* z, int32_t n_z, int32_t L, const double2* V,
                    const cbs_params* prm, hipStream_t st, NodeSolve& out, const HistReq* hist = nullptr);
// Block BiCG over the L columns of each node (block.hip); same output as solve_nodes.
int32_t solve_nodes_block(cbs_system* s, double E, const double2* z, int32_t n_z, int32_t L, const double2* V,
                          const cbs_params* prm, hipStream_t st, NodeSolve& out);
int32_t split_pairs(int64_t N, int32_t nruns, const Pair<double>* Y, double2* ya, double2* yb, hipStream_t st);
int32_t check_params(const cbs_params* p, bool need_moments);
void configure_solve(BicgSolve& b, const cbs_params* prm);

}  // namespace cbs
