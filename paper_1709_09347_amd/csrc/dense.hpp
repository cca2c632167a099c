// Dense FP64 helpers of the extraction step (see dense.hip).
#pragma once

#include "cbs_internal.hpp"

namespace cbs {

// C (na x nb, ldc) = A^H B, A: na vectors of length N (stride lda), B: nb vectors (stride ldb).
int32_t gram(cbs_system* s, int64_t N, int32_t na, const double2* A, int64_t lda, int32_t nb, const double2* B,
             int64_t ldb, double2* C, int64_t ldc, hipStream_t st);
// out[c] = sum_k A[k] W[k + c*ldw], vectors of length N.
int32_t tall_gemm(int64_t N, int32_t K, int32_t nc, const double2* A, int64_t lda, const double2* W, int32_t ldw,
                  double2* out, int64_t ldo, hipStream_t st);
// C (m x n) = op(A) B[:, bperm] * diag(colscale).
int32_t small_gemm(int32_t m, int32_t n, int32_t k, const double2* A, int32_t lda, bool transA, const double2* B,
                   int32_t ldb, double2* C, int32_t ldc, const double* colscale, const int32_t* bperm,
                   hipStream_t st);
// A = U diag(sigma) W^H: A overwritten by U (columns in source order), V by W; sigma[0..n)
// sorted descending with perm[r] = source column of rank r; sigma needs 1024 doubles.
int32_t svd(int32_t n, double2* A, int32_t lda, double2* V, int32_t ldv, double* sigma, int32_t* perm,
            hipStream_t st);
// Eigenvalues w and unit eigenvectors V of a general complex matrix H (destroyed).
int32_t eig(cbs_system* s, int32_t n, double2* H, int32_t ldh, double2* w, double2* V, int32_t ldv,
            int32_t* info_dev, hipStream_t st);
int32_t lu_solve(int32_t n, double2* A, int32_t lda, double2* B, int32_t ldb, int32_t nrhs, int32_t* info_dev,
                 hipStream_t st);
int32_t chol_inv(int32_t n, double2* G, int32_t ldg, double shift, double2* Rinv, int32_t* info_dev,
                 hipStream_t st);

}  // namespace cbs
