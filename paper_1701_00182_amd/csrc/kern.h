// Task descriptors and launchers of the batched device kernels.
//
// Every batched kernel takes a device array of small descriptors, one per
// independent matrix operation, so that all blocks of a hierarchical-matrix
// depth across all planes of a cyclic-reduction level run in one launch.
// Matrices are column-major with explicit leading dimensions.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace acr {

// C = alpha * op(A) * op(B) + beta * C   (op = transpose when ta / tb is set)
struct GemmTask {
  const void* A;
  const void* B;
  void* C;
  int64_t lda, ldb, ldc;
  int m, n, k;
  int ta, tb;
  double alpha, beta;
};

// dst = alpha * diag(rs) * src * diag(cs) (+ dst if accumulate); rs / cs may be
// null; a null src stands for the identity (alpha on the diagonal, 0 elsewhere)
struct CopyTask {
  const void* src;
  void* dst;
  const void* rs;
  const void* cs;
  int64_t lds, ldd;
  int m, n;
  int accumulate;
  double alpha;
};

// In-place inverse of an s x s matrix (Gauss-Jordan, partial pivoting)
struct InvTask {
  void* A;
  int64_t lda;
  int s;
  int flag_slot;
};

// Householder QR of an m x r panel; reflectors overwrite the panel below the
// diagonal, R above it; tau has min(m, r) entries
struct QrTask {
  void* A;
  void* tau;
  int64_t lda;
  int m, r;
};

// Truncated SVD of the core Ru * Rv^T (p x q, p = min(mu, r), q = min(mv, r))
// by one-sided Jacobi in FP64; writes Zu = X_k Sigma_k (p x k), Zv = Y_k (q x k)
struct SvdTask {
  const void* Ru;   // panel holding R of the U stack (ld ldu)
  const void* Rv;   // panel holding R of the V stack (ld ldv)
  int64_t ldu, ldv;
  int p, q, r;
  double* C;        // p x q workspace (becomes X * Sigma)
  double* Y;        // q x q workspace (right rotations)
  double* sig;      // q workspace
  int* rank_out;
  int max_rank;     // 0 = unlimited
};

// out (m x k) = Q * [Z; 0] with Q the product of the panel's reflectors
struct ApplyQTask {
  const void* Aq;   // reflectors (panel after QR)
  const void* tau;
  const double* Z;  // p x k, ld ldz
  void* out;        // m x k, ld ldo
  int64_t lda, ldz, ldo;
  int m, p, k;
};

enum : int { FLAG_SINGULAR = 0, FLAG_RANK = 1, FLAG_NONFINITE = 2, FLAG_INVALID = 3, NFLAGS = 8 };

template <class T> void launch_gemm(const GemmTask* d_tasks, const int* d_tile_task,
                                    const int* d_first_tile, int ntiles, hipStream_t s);
template <class T> void launch_copy(const CopyTask* d_tasks, int ntasks, hipStream_t s);
template <class T> void launch_inverse(const InvTask* d_tasks, int ntasks, int max_s,
                                       int* d_flags, hipStream_t s);
template <class T> void launch_qr(const QrTask* d_tasks, int ntasks, hipStream_t s);
template <class T> void launch_svd(const SvdTask* d_tasks, int ntasks, double eps,
                                   int* d_flags, hipStream_t s);
template <class T> void launch_applyq(const ApplyQTask* d_tasks, int ntasks, hipStream_t s);

}  // namespace acr
