/*
 * cbs.h - C ABI of the MI355X Sakurai-Sugiura complex-band-structure library.
 *
 * The library computes, at a real energy E, the Bloch factors lambda with
 * lambda_min < |lambda| < 1/lambda_min of the quadratic eigenvalue problem
 * (Iwase et al., SC17, Sec. 2, Eqs. 4-5)
 *
 *     P(lambda) psi = [ (H0 - E) + lambda H+ + lambda^{-1} H- ] psi = 0,
 *
 * where H0, H+ and H- = H+^T are the cell blocks of a real-space
 * finite-difference Kohn-Sham Hamiltonian: -1/2 Laplacian by central finite
 * differences of order fd_order (x, y periodic with phase 1, z coupled to the
 * neighbouring cells), a local potential V_loc on the diagonal, and separable
 * nonlocal projectors V_nl = sum_{a,i} h_ai |u_ai><u_ai| summed over the
 * periodic images of each atom.  (P is the negative of the paper's Eq. 4
 * operator; the eigenpairs are the same.)
 *
 * Method (paper Sec. 3): BiCG solves of P(z_j) Y_j = V at the trapezoid
 * nodes z_j of the outer circle, whose dual systems P(z_j)^H Yt_j = V are the
 * inner-circle solves because P(z)^H = P(1/conj z) (Sec. 3.2, Eq. 11); the
 * moments S_k = sum_j w_j z_j^k Y_j over the ring contour (Sec. 3.2, Eq. 7);
 * block Hankel matrices of mu_k = V^H S_k, their truncated SVD and the
 * reduced eigenproblem (Sec. 3.1, Algorithm 1); optionally a Rayleigh-Ritz
 * projection of the QEP onto the span of the Hankel Ritz vectors.
 *
 * Conventions
 *   - Complex numbers are interleaved (re, im) pairs of double (complex128)
 *     or float (complex64).
 *   - Grid point index n = ix + nx*(iy + ny*iz), N = nx*ny*nz.
 *   - A block of k vectors of length N is stored vector-major: element
 *     (vector v, point n) at offset v*N + n (in complex elements).
 *   - "device" pointers are HIP device memory on the system's device, owned
 *     by the caller; "host" pointers are ordinary host memory, owned by the
 *     caller.  No call keeps a caller pointer after it returns.
 *   - stream: a hipStream_t (NULL = the default stream).  Calls that return
 *     host results synchronise that stream before returning.
 *   - Every function returns CBS_OK (0) or a negative error code; on error no
 *     output is guaranteed except where stated.  cbs_strerror() names codes,
 *     cbs_last_error() gives a message for the last failure on this thread.
 */
#ifndef CBS_H
#define CBS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CBS_OK = 0,
  CBS_EINVAL = -1,      /* bad argument or unsupported shape */
  CBS_ENOMEM = -2,      /* device allocation failed */
  CBS_EHIP = -3,        /* HIP runtime error */
  CBS_ENOCONV = -4,     /* a linear solve missed its tolerance (results written) */
  CBS_EBREAKDOWN = -5,  /* BiCG breakdown (zero rho or sigma) */
  CBS_ERANK = -6,       /* Hankel rank reached L*M: subspace too small (results written) */
  CBS_ETOOMANY = -7,    /* more eigenvalues than max_eigs (count written) */
  CBS_ENONFINITE = -8,  /* non-finite moments (a linear solve diverged); no eigenpairs */
  CBS_EEIG = -9         /* a small dense step of the extraction failed (QR iteration of the
                           reduced eigenproblem, Cholesky QR of the Ritz basis or the LU of the
                           linearised projected QEP); no eigenpairs */
};

enum { CBS_C128 = 0, CBS_C64 = 1 };          /* element type of cbs_apply vectors */
enum { CBS_FP64 = 0, CBS_MIXED = 1 };        /* solve precision */
enum { CBS_RR = 0, CBS_HANKEL = 1 };         /* eigenpair extraction */

typedef struct cbs_system cbs_system;

/* Grid of one periodic cell.  fd_order in {2, 4, 6, 8} (half-width p = fd_order/2);
 * requires nz >= p, 1 <= nx <= 256, ny >= 1, h > 0. */
typedef struct {
  int32_t nx, ny, nz, fd_order;
  double h;
} cbs_grid;

/* Separable nonlocal projectors (paper Sec. 4: norm-conserving pseudopotentials),
 * host arrays, CSR over atoms.  Ball entry e of atom a (ball_off[a] <= e <
 * ball_off[a+1]) sits at cell point ball_idx[e] of the cell shifted by
 * ball_w[e] in {-1, 0, 1} along z, and carries the values ball_val[e*n_proj + i]
 * of the atom's n_proj (<= 4) projectors (grid-normalised u = h^{3/2} p).
 * coeff[a*n_proj + i] is h_ai.  Each atom's entries must span at most two
 * adjacent shifts (projector diameter below the cell length), so that only
 * nearest cells couple. */
typedef struct {
  int32_t n_atoms, n_proj;
  const int64_t* ball_off;   /* [n_atoms+1] */
  const int32_t* ball_idx;   /* [nnz] */
  const int8_t* ball_w;      /* [nnz] */
  const double* ball_val;    /* [nnz*n_proj] */
  const double* coeff;       /* [n_atoms*n_proj] */
} cbs_proj;

/* Contour and solver parameters (paper Sec. 3 and 4.1; defaults from
 * cbs_params_default: lambda_min 0.5, n_q 32, n_rhs 16, n_mom 8, delta 1e-10,
 * tol 1e-10). */
typedef struct {
  double lambda_min;    /* annulus lambda_min < |lambda| < 1/lambda_min, 0 < lambda_min < 1 */
  int32_t n_q;          /* trapezoid nodes per circle (N_int) */
  int32_t n_rhs;        /* right-hand sides L (N_rh) */
  int32_t n_mom;        /* moments M (N_mm); Hankel size L*M <= 256; 2*M <= n_q */
  double delta;         /* SVD rank threshold, relative to the largest singular value (raised to
                           100x the largest relative residual of the solves when that is higher) */
  double tol;           /* per-column relative residual of every solve (primal and dual) */
  int32_t max_iter;     /* BiCG iteration cap (per inner solve) */
  int32_t precision;    /* CBS_FP64, or CBS_MIXED: complex128 BiCG until a run's residual is
                           below inner_tol, then complex64 vectors and operator applications
                           with FP64 residual replacement (iterative refinement) to tol */
  int32_t extraction;   /* CBS_RR (default) or CBS_HANKEL */
  int32_t half_stop;    /* 1: stop all solves at one energy once more than half of the solved
                           nodes have every right-hand side converged (Sec. 3.3); the stopped
                           runs keep their iterate (true residual in cbs_info.max_solve_resid).
                           cbs_solve counts them as finished, cbs_bicg as missing tol.  0
                           (default): every run to tol. */
  double inner_tol;     /* CBS_MIXED: residual below which a run continues in complex64 (1e-6) */
  int32_t max_refine;   /* cap on FP64 residual replacements per run (60) */
  int32_t chunk;        /* iterations per captured graph between convergence polls (even) */
  int32_t profile;      /* 1: no graph; HIP events time every BiCG stencil launch (cbs_info.stencil_*) */
  int32_t conj_nodes;   /* 1 (default): when every right-hand side is real (imaginary parts exactly
                           zero), solve only the nodes with 0 < theta_j < pi.  The blocks H0, H+, H-
                           are real, so P(conj z) = conj P(z): the solutions at the mirrored nodes
                           conj z_j are the complex conjugates, and each mirrored pair adds
                           2 Re(w z^k y) to the moments (Sec. 3.1 Eq. 7 summed in pairs).  Same
                           result, half the linear solves.  0: solve every node. */
  int32_t block;        /* 1 (default): every right-hand side is its own BiCG run (the paper's
                           Sec. 3.1 solver).  n_rhs: block BiCG over the n_rhs columns of each node
                           (block Krylov space of P(z_j) on V, n_rhs x n_rhs coefficient matrices
                           from block inner products); other values: CBS_EINVAL. */
  int32_t lo_window;    /* CBS_MIXED: complex64 iterations without a 100x residual drop before a
                           forced complex128 residual replacement (0: 300) */
} cbs_params;

/* Per-solve diagnostics. */
typedef struct {
  int32_t rank;             /* numerical rank m of the Hankel matrix */
  int32_t n_eigs;           /* eigenpairs returned (inside the annulus) */
  int32_t iters_max;        /* largest BiCG iteration count over all runs (summed over refinement) */
  int32_t refine_steps;     /* FP64 refinement steps (CBS_MIXED) */
  double iters_mean;        /* mean BiCG iterations per run */
  double max_solve_resid;   /* max over all solves of ||v - P(z)y|| / ||v|| (recursive, or FP64 recomputed for CBS_MIXED) */
  double max_eig_resid;     /* max ||P(lambda) psi|| / ||psi|| over returned pairs */
  double sigma_first;       /* largest singular value of the Hankel matrix */
  double sigma_ratio;       /* sigma_m / sigma_1 of the last kept singular value */
  double t_solve_ms, t_moments_ms, t_extract_ms;   /* wall time of the three steps */
  int64_t matvecs;          /* operator applications (vectors) in the solves */
  /* params.profile = 1 only: the BiCG stencil kernel, timed per launch with HIP events on
   * the stream it runs on; bytes are its algorithmic traffic (per active run: read r,
   * p_old, x and write p_new, q, x once, plus V_loc once per launch).  stencil_*: the
   * complex128 kernel, stencil_lo_*: the complex64 kernel (CBS_MIXED). */
  int64_t stencil_launches;
  double stencil_ms;
  double stencil_bytes;
  int64_t stencil_lo_launches;
  double stencil_lo_ms;
  double stencil_lo_bytes;
  int32_t nodes_solved;     /* nodes per circle whose systems were solved: n_q, or n_q/2 with conj_nodes */
  int32_t restarts;         /* CBS_MIXED: runs whose complex64 phase stopped reducing the true residual
                               and that restarted BiCG in complex128 (summed over the runs) */
  int32_t status;           /* return code of this solve: of the call (cbs_solve) or of this
                               (system, energy) pair (cbs_solve_batched) */
} cbs_info;

/* ---- errors ---------------------------------------------------------- */
const char* cbs_strerror(int32_t code);
const char* cbs_last_error(void);

/* ---- systems (paper Sec. 2: the cell blocks of one crystal) ---------- */

/* Uploads the grid, local potential (host [N] double) and projector tables
 * (host, may be NULL) to `device` and builds the point-major projector index.
 * Not timed in a solve.  Errors: CBS_EINVAL (shape, or a non-finite v_loc,
 * checked before the device is touched), CBS_ENOMEM, CBS_EHIP. */
int32_t cbs_system_create(cbs_system** out, int32_t device, const cbs_grid* grid,
                          const double* v_loc, const cbs_proj* proj);
void cbs_system_destroy(cbs_system* sys);
/* Replace V_loc (host [N] double); keeps projectors and workspace.
 * CBS_EINVAL (nothing changed) if a value is not finite. */
int32_t cbs_system_set_vloc(cbs_system* sys, const double* v_loc);
int64_t cbs_system_npoints(const cbs_system* sys);
/* Number of solves whose eigenpairs the system has stored for cbs_grad_vloc so far: it
 * changes whenever cbs_solve or cbs_solve_batched replaces them.  0 before the first
 * solve, -1 for a NULL handle. */
int64_t cbs_system_solve_id(const cbs_system* sys);
/* Stencil tiling: tile_y[0] (complex128) and tile_y[1] (complex64) full-x rows per
 * workgroup, and the autotuner's timings ("" before the first solve tuned them;
 * CBS_AUTOTUNE=0 keeps the heuristic defaults).  The string lives until the next
 * solve on sys. */
const char* cbs_system_tiling(const cbs_system* sys, int32_t* tile_y);

void cbs_params_default(cbs_params* p);

/* ---- operator (Eq. 4) --------------------------------------------------
 * y_v = P(z_v) x_v for a batch of n_vec vectors (device, [n_vec][N], dtype
 * CBS_C128 or CBS_C64), z host [2*n_vec] (re, im), z_v != 0.  x and y must not
 * overlap.  complex64 runs the single-precision kernels end to end.  The
 * staging buffers come from the system's workspace (allocated on first use). */
int32_t cbs_apply(cbs_system* sys, double E, int32_t n_vec, const double* z,
                  int32_t dtype, const void* x, void* y, void* stream);

/* Allocation-free variant of cbs_apply, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and result as cbs_apply; it calls no hipMalloc or hipFree: its
 * staging buffers (run coefficients, the two pair-interleaved vector buffers and the
 * projector coefficients) live in one fixed device array of CBS_APPLY_NOALLOC_BYTES per
 * device, held from the first cbs_system_create on that device until the process ends.
 * A call needs, each part rounded up to 256 bytes,
 *   ceil(n_vec/2) * 112  +  2 * ceil(n_vec/2) * N * b  +  ceil(n_vec/2) * n_atoms * 12 * b
 * bytes, b = 32 (CBS_C128) or 16 (CBS_C64); a larger call returns CBS_EINVAL before
 * touching the device.  Every call on one device shares the array and leaves its contents
 * behind; calls that overlap on one device (several streams or threads) race. */
#define CBS_APPLY_NOALLOC_BYTES (64u << 20)
int32_t cbs_apply_noalloc(cbs_system* sys, double E, int32_t n_vec, const double* z,
                          int32_t dtype, const void* x, void* y, void* stream);

/* y_v = c0_v (H0 - E) x_v + cp_v H+ x_v + cm_v H- x_v, coefficients host
 * [2*n_vec] each (re, im); complex128 only.  The z-split form of cbs_apply,
 * used for Rayleigh-Ritz projections. */
int32_t cbs_apply_parts(cbs_system* sys, double E, int32_t n_vec, const double* c0,
                        const double* cp, const double* cm, const void* x, void* y,
                        void* stream);

/* ---- step 1: BiCG with duals (Sec. 3.2, Eqs. 9-11) ---------------------
 * For every node z_j (host [2*n_z]) and right-hand side v_l (device [L][N]
 * complex128) solves P(z_j) y = v_l and, as the BiCG dual, P(z_j)^H yt = v_l,
 * to params->tol (precision CBS_FP64 or CBS_MIXED as in cbs_solve).  Y, Yt
 * device [n_z][L][N] complex128.  iters (host [n_z*L], may be NULL) receives
 * the iteration count of each run and relres (host [2*n_z*L], may be NULL) the
 * final relative residuals (primal, dual).  Returns CBS_ENOCONV if a run
 * missed tol within max_iter or was stopped by params->half_stop (results
 * still written). */
int32_t cbs_bicg(cbs_system* sys, double E, int32_t n_z, const double* z, int32_t n_rhs,
                 const void* V, const cbs_params* params, void* Y, void* Yt,
                 int32_t* iters, double* relres, cbs_info* info, void* stream);

/* As cbs_bicg, and also the convergence history of every run (the per-node
 * residual curves of Sec. 4.1): hist (host [max_rows][n_z*n_rhs][2], primal
 * then dual) receives the recursive relative residual ||r|| / ||v|| of each run
 * after iterations stride, 2*stride, ... (row i = iteration (i+1)*stride), as
 * the solver computes it (complex64 recurrences in the complex64 phase of
 * CBS_MIXED, the true residual right after a replacement).  Rows past a run's
 * last iteration, or past max_rows, hold NaN / are not recorded.  The solve is
 * the same as cbs_bicg's; the device keeps max_rows*runs*2 doubles during the
 * call.  CBS_EINVAL if stride < 1, max_rows < 1, hist is NULL or
 * max_rows*runs*2 >= 2^31; otherwise as cbs_bicg. */
int32_t cbs_bicg_history(cbs_system* sys, double E, int32_t n_z, const double* z, int32_t n_rhs,
                         const void* V, const cbs_params* params, int32_t stride, int32_t max_rows,
                         double* hist, void* Y, void* Yt, int32_t* iters, double* relres,
                         cbs_info* info, void* stream);

/* ---- the whole method at one energy (Algorithm 1 on the ring contour) --
 * V: device [L][N] complex128 right-hand sides (L = params->n_rhs); when every
 * imaginary part is zero and params->conj_nodes is set, half of the nodes are
 * solved and the mirrored ones taken by conjugation (cbs_info.nodes_solved).
 * lambda: host [2*max_eigs], resid: host [max_eigs] (may be NULL),
 * vecs: device [max_eigs][N] complex128 (may be NULL), unit 2-norm, largest
 * component real positive.  Eigenvalues are sorted by |ln|lambda||, then by
 * arg lambda.  Returns CBS_ETOOMANY with *n_eigs = needed count when
 * max_eigs is too small; CBS_ERANK when the Hankel rank equals L*M (results
 * written, subspace too small; also at an energy whose annulus holds no
 * eigenvalue, where the moments are noise: then *n_eigs = 0); CBS_ENOCONV
 * when a solve missed tol (results written).  The last solve's eigenpairs stay on the system for
 * cbs_grad_vloc. */
int32_t cbs_solve(cbs_system* sys, double E, const cbs_params* params, const void* V,
                  int32_t max_eigs, double* lambda, double* resid, void* vecs,
                  int32_t* n_eigs, cbs_info* info, void* stream);

/* ---- batching: energies x systems in one pass ------------------------
 * Solves every (system s, energy e) pair with the same parameters.  All
 * quadrature nodes, right-hand sides, energies and systems share each BiCG
 * kernel launch.  V[s]: device [L][N_s] complex128.  lambda: host
 * [n_sys][n_E][2*max_eigs]; n_eigs: host [n_sys*n_E]; info: host [n_sys*n_E]
 * (may be NULL); info[i].status holds each pair's own code.  A pair whose
 * extraction fails (CBS_ENONFINITE, CBS_EEIG) gets n_eigs = 0 and the other pairs
 * are still solved.  Returns the most severe pair code (CBS_EBREAKDOWN, then
 * CBS_ENONFINITE, CBS_EEIG, CBS_ENOCONV, CBS_ETOOMANY, CBS_ERANK), or
 * CBS_EINVAL / CBS_ENOMEM / CBS_EHIP at once. */
int32_t cbs_solve_batched(int32_t n_sys, cbs_system* const* systems, int32_t n_E,
                          const double* E, const cbs_params* params,
                          const void* const* V, int32_t max_eigs, double* lambda,
                          int32_t* n_eigs, cbs_info* info, void* stream);

/* ---- complex band structure (Sec. 2) ----------------------------------
 * The complex wave number of each Bloch factor: lambda = exp(i k a) with a the
 * cell length along the transport direction (N_z h), so
 * k = (arg lambda - i ln|lambda|) / a on the principal branch, Re k in
 * [-pi/a, pi/a].  Propagating states (|lambda| = 1) have real k, states decaying
 * along +z (|lambda| < 1) have Im k > 0.  Scanning E with cbs_solve_batched and
 * converting each energy's eigenvalues gives the complex band structure.
 * lambda, k: host [2*n] (re, im pairs; k may alias lambda).  Host arithmetic
 * only.  CBS_EINVAL (nothing written) if n < 0, cell_length is not a positive
 * finite number, or a lambda is zero or not finite. */
int32_t cbs_lambda_to_k(int32_t n, const double* lambda, double cell_length, double* k);

/* Branches of the complex band structure: the curves k(E) (Sec. 2; the CBS figures of
 * Sec. 4.1 and 5) from the k of a scan of increasing energies.  E: host [n_E]; n_k: host
 * [n_E] counts; k: host [sum n_k][2] (re, im), energy by energy.  Each k is joined to the
 * open branch whose linear prediction (from its last two points) it is nearest to, Re k
 * compared modulo 2 pi / cell_length, in increasing order of that distance (a greedy
 * assignment); a point farther than max_jump (1/bohr) from every prediction starts a new
 * branch, a branch that takes no point ends.  branch: host [sum n_k] branch ids (0 ..
 * n_branches - 1, in order of appearance).  Host arithmetic only; CBS_EINVAL if a count
 * is negative, the energies are not increasing or a value is not finite. */
int32_t cbs_connect_branches(int32_t n_E, const double* E, const int32_t* n_k, const double* k,
                             double cell_length, double max_jump, int32_t* branch, int32_t* n_branches);

/* ---- conventional band structure (Sec. 2; the cross-check of Sec. 4.1) --
 * The lowest n_bands eigenvalues of the Hermitian H(k) = H0 + e^{ika} H+ + e^{-ika} H-
 * (a = nz h, the cell length) at the real wave numbers k (host [n_k], 1/bohr).  A
 * propagating Bloch factor lambda = e^{ika} of the QEP at energy E makes E an eigenvalue
 * of H(k), so these bands check the complex band structure where no dense H(k) can be
 * diagonalised.  Chebyshev-filtered subspace iteration on the device: a block of n_bands
 * plus guard vectors, a degree-16 filter per step bounded on [largest Ritz value, a
 * Lanczos bound of the spectrum], Cholesky QR and Rayleigh-Ritz through a Jacobi SVD; the
 * operator is cbs_apply_parts's complex128 kernels.  Each band stops when
 * ||H x - eps x|| <= tol (|eps| + 1); a k takes at most max_iter filter steps.
 * eps: host [n_k][n_bands], ascending; resid: host [n_k][n_bands] residual norms (may
 * be NULL); vecs: device [n_k][n_bands][N] complex128 unit eigenvectors (may be NULL);
 * iters: host [n_k] filter steps (may be NULL).  Returns CBS_ENOCONV when a k missed tol
 * (that k and the earlier ones written), CBS_EINVAL for n_bands beyond ~200 or the grid
 * size, CBS_EEIG if the Cholesky QR of a filtered block failed. */
int32_t cbs_bands(cbs_system* sys, int32_t n_k, const double* k, int32_t n_bands, double tol,
                  int32_t max_iter, double* eps, double* resid, void* vecs, int32_t* iters, void* stream);

/* ---- adjoint --------------------------------------------------------
 * d lambda_i / d V_loc(r) for eigenpairs sel[k] (host indices into the last
 * cbs_solve's output) = -conj(y_i(r)) x_i(r) / (y_i^H P'(lambda_i) x_i) with
 * P'(lambda) = H+ - lambda^{-2} H- and y_i the eigenvector of the pair
 * partner 1/conj(lambda_i), which is a left eigenvector of lambda_i because
 * P(lambda)^H = P(1/conj lambda) (Sec. 3.2): the inner-circle (dual) solves
 * already carry it, no extra solve is made.
 * out: device [n_sel][N] complex128 (may be NULL).  If weights (host
 * [2*n_sel], complex g_k) and vjp (device [N] double) are given, also writes
 * the vector-Jacobian product vjp(r) = sum_k Re(g_k conj(d lambda_k/d V(r))),
 * the gradient of a real loss whose conjugate-Wirtinger derivative with
 * respect to lambda_k is g_k (PyTorch's convention for complex outputs).
 * CBS_EINVAL if no solve is stored, an index is out of range, or a selected
 * eigenvalue has no simple partner (degenerate within 1e-7 relative). */
int32_t cbs_grad_vloc(cbs_system* sys, int32_t n_sel, const int32_t* sel, void* out,
                      const double* weights, void* vjp, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CBS_H */
