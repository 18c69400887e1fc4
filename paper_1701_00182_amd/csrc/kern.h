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
  int lowp;   // FP32 data only: 1 = BF16, 2 = FP16 matrix-core inputs with block scaling; 0 = the
              // launch's default (Exec::prod_lowp), -1 = always FP32
};

// C = alpha * sum_s op_s(A_s) B_s + beta * C: one output block with the inner
// dimension concatenated from up to kMaxSeg (A, B) segment pairs -- a leaf's
// rows of H X in one pass (the dense leaf times the leaf's part of X, then each
// ancestor block's U-slice times that block's V^T X).  op_s transposes A_s when
// ta has bit s set.
constexpr int kMaxSeg = 21;
struct SegGemmTask {
  void* C;
  int64_t ldc;
  int m, n;
  double alpha, beta;
  int nseg;
  unsigned ta;
  const void* A[kMaxSeg];
  const void* B[kMaxSeg];
  int64_t lda[kMaxSeg], ldb[kMaxSeg];
  int k[kMaxSeg];
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

// Truncated SVD of the core C = Ru * Rv^T (p x q) in FP64: column-pivoted QR of
// C, then one-sided Jacobi; writes Zu = X_k Sigma_k (p x k, at C + p*q, ld p) and
// Zv = Y_k (q x k, at Y + q*q, ld q)
struct SvdTask {
  const void* Ru;   // R factor of the U stack (ld ldu)
  const void* Rv;   // R factor of the V stack (ld ldv)
  int64_t ldu, ldv;
  int p, q, r;
  double* C;        // 2 p q workspace
  double* Y;        // 2 q q workspace
  double* sig;      // q workspace
  int* perm;        // q workspace (column pivots)
  int* t_out;       // numerical rank found by the pivoted QR
  int* rank_out;
  int max_rank;     // 0 = unlimited
  int mode;         // 0: Ru, Rv upper-trapezoidal panels in T; 1: full FP64 factors
  int tc;           // host copy of *t_out (used to size the Jacobi stage)
  unsigned long long* sweep_ctr;  // optional: += rows * pairs visited (timing table)
  unsigned long long* flop_ctr;   // += flops counted on the device (sweeps, small cores, left factor)
};

// dst (n x n, ld n) = upper triangle of src (ld lds), zeros below; the next
// n x n doubles of dst are cleared
struct TriCopyTask {
  const double* src;
  double* dst;
  int64_t lds;
  int n;
};
void launch_tri_copy(const TriCopyTask* d_tasks, int ntasks, hipStream_t s);

// out (m x k) = Q * [Z; 0] with Q the product of the panel's reflectors
struct ApplyQTask {
  const void* Aq;   // reflectors (panel after QR)
  const void* tau;
  const double* Z;  // p x k, ld ldz
  void* out;        // m x k, ld ldo
  int64_t lda, ldz, ldo;
  int m, p, k;
};

// S^T S of an m x r stack in FP64, from per-chunk partial sums reduced in order
struct GramTask {
  const void* A;
  int64_t lda;
  int m, r;
  int rows_per_chunk;
  double* part;   // nchunk x r x r
  double* G;      // r x r
};

// Pivoted Cholesky G[perm, perm] ~= L L^T (L r x rank), then R (rank x r) in the
// original column order
struct PcholTask {
  const double* G;
  double* L;       // r x r workspace
  int* perm;       // r
  double* d;       // r workspace
  int* rank_out;
  int r;
  int r1;          // rank (host fills it in before materialising R)
  double* R;       // r1 x r
};

// W (r x k, precision T) = P1 L11^{-T} Z  (Z r1 x k FP64, overwritten)
struct WtTask {
  const double* L;
  const int* perm;
  double* Z;
  int64_t ldz;
  void* W;
  int r, r1, k;
};

// t (k x c, ld k) = V^T x for one off-diagonal block (solve sweeps)
struct InnerTask {
  const void* V;
  int64_t ldv;
  int rows, k;
  const void* x;
  int64_t ldx;
  void* t;
  int c;
};

constexpr int kMaxDepth = 20;
// alpha * H x restricted to one leaf's rows: dense leaf (or diagonal) times the
// leaf part of x, plus the U-slices of the leaf's ancestors times their t
struct LeafTerm {
  const void* leaf;
  const void* diag;
  const void* x;
  int64_t ldx;
  int trans;
  int nd;
  double alpha;
  const void* up[kMaxDepth];
  const void* tp[kMaxDepth];
  int64_t ldu[kMaxDepth];
  int kd[kMaxDepth];
};

// y_leaf = beta * yin_leaf + sum of up to two terms
struct LeafTask {
  void* y;
  const void* yin;
  int64_t ldy;
  int n, c;
  double beta;
  int nterm;
  LeafTerm term[2];
};

enum : int { FLAG_SINGULAR = 0, FLAG_RANK = 1, FLAG_NONFINITE = 2, FLAG_INVALID = 3, NFLAGS = 8 };

// matrix-core GEMM over the same tile map; lowp selects the 16-bit input
// variant for FP32 data (0 = FP32 / FP64 inputs)
template <class T> void launch_gemm_mfma(const GemmTask* d_tasks, const int* d_tile_task, const int* d_first_tile,
                                         int ntiles, int lowp, hipStream_t s);
// FP32 GEMM in 128 x 32 output tiles for outputs at most 32 columns wide
// (tile map: ceil(m / 128) tiles per task)
void launch_gemm_narrow(const GemmTask* d_tasks, const int* d_tile_task, const int* d_first_tile, int ntiles,
                        hipStream_t s);
template <class T> void launch_seg_gemm(const SegGemmTask* d_tasks, const int* d_tile_task, const int* d_first_tile,
                                        int ntiles, hipStream_t s);
// Work units of a copy: columns of at most kCopyUnit elements go whole, as
// many as fit in kCopyUnit elements per unit; longer columns in kCopyUnit-row
// chunks.
constexpr int kCopyUnit = 2048;
__host__ __device__ inline int copy_cols_per_unit(int m) { return m >= kCopyUnit || m <= 0 ? 1 : kCopyUnit / m; }
__host__ __device__ inline int64_t copy_units(int m, int n) {
  if (m <= 0 || n <= 0) return 0;
  if (m > kCopyUnit) return (int64_t)n * ((m + kCopyUnit - 1) / kCopyUnit);
  const int cpu = copy_cols_per_unit(m);
  return (n + cpu - 1) / cpu;
}
// units: workgroups per task (each takes the task's units in turn)
template <class T> void launch_copy(const CopyTask* d_tasks, int ntasks, int units, hipStream_t s);
// unblocked = true forces the unblocked Gauss-Jordan kernel
template <class T> void launch_inverse(const InvTask* d_tasks, int ntasks, int max_s,
                                       int* d_flags, hipStream_t s, bool unblocked);
// LDS-resident variants; `lds` is the dynamic shared memory per workgroup
template <class T> void launch_qr_lds(const QrTask* d_tasks, int ntasks, size_t lds, hipStream_t s);
// max_q: the widest core (the global-memory variant keeps its pivot map in LDS)
template <class T> void launch_qrcp(const SvdTask* d_tasks, int ntasks, double delta, size_t lds, int max_q,
                                    hipStream_t s);
// threads: the workgroup size that gives every core of the launch one pass
// per round of its LDS-resident sweeps (rounded up to 256, 512 or 1024); for
// the blocked sweeps in global memory (lds = 0), above 512 when a vector is
// longer than kJBRegRows
constexpr int kJBRegRows = 256;   // longest vectors of the register-resident blocked visit
template <class T> void launch_jacobi(const SvdTask* d_tasks, int ntasks, double eps, int* d_flags, size_t lds,
                                      int threads, hipStream_t s);
// Cores whose C fits in LDS: the pivoted QR, the sweeps and the right vectors
// in one workgroup per core (one wavefront when p, q, r <= kSvdWave), with no
// host round trip; larger cores: launch_qrcp, then launch_jacobi
template <class T> void launch_svd_wave(const SvdTask* d_tasks, int ntasks, double delta, double eps, int* d_flags,
                                        size_t lds, hipStream_t s);
template <class T> void launch_svd_block(const SvdTask* d_tasks, int ntasks, double delta, double eps, int* d_flags,
                                         size_t lds, hipStream_t s);
// Zu = Ru (Rv^T Zv) for the kept columns, kc columns per workgroup
template <class T> void launch_core_left(const SvdTask* d_tasks, int ntasks, int kc, int nchunks, size_t lds,
                                         unsigned long long* ctr, hipStream_t s);
template <class T> void launch_applyq_lds(const ApplyQTask* d_tasks, int ntasks, size_t lds, hipStream_t s);
// reduce_wgs: workgroups per task of the ordered sum of the chunk partials
// (each takes 32 x 32 tiles of the upper triangle in turn)
template <class T> void launch_gram(const GramTask* d_tasks, int ntasks, const int* d_tile_task,
                                   const int* d_first_tile, int ntiles, int reduce_wgs, hipStream_t s);
// chunk partials of the Gram on the matrix cores (workgroup map: four
// wavefronts per workgroup, one per row chunk x upper pair of 32-column blocks)
template <class T> void launch_gram_mfma(const GramTask* d_tasks, const int* d_tile_task, const int* d_first_tile,
                                        int ntiles, hipStream_t s);
// lds_packed > 0: the Gram matrices in LDS (packed, right-looking; lds_packed
// = max over the tasks of lds_bytes_pchol_packed); 0: left-looking with L in
// global memory (max_r bounds the tasks' orders)
void launch_pchol(const PcholTask* d_tasks, int ntasks, int max_r, double tol, size_t lds_packed, hipStream_t s);
// register-tiled pivoted Cholesky (no swaps): kind 0 for orders up to
// kPcholRegSmall (256-thread workgroups, 4 x 4 tiles), kind 3 up to
// kPcholRegMid (512 threads, 5 x 5 tiles), kind 2 up to kPcholReg1024 (1024
// threads, 5 x 5 tiles), kind 1 up to kPcholReg (512 threads, 8 x 8 tiles):
// the same arithmetic per entry whatever the tiling; overwrites the tasks'
// Gram buffers (the columns of L in original row order)
constexpr int kPcholRegSmall = 88;
constexpr int kPcholRegMid = 155;
constexpr int kPcholReg1024 = 220;
constexpr int kPcholReg = 248;
void launch_pchol_reg(const PcholTask* d_tasks, int ntasks, int max_r, double tol, int kind, hipStream_t s);
void launch_materialize_r(const PcholTask* d_tasks, int ntasks, int wgs, hipStream_t s);
template <class T> void launch_wtilde(const WtTask* d_tasks, int ntasks, int kc, int nchunks, size_t lds,
                                      hipStream_t s);
// vec: the 16-byte vector kernels (every task's sizes, leading dimensions and
// addresses multiples of 16 bytes; no transposed leaf)
template <class T> void launch_inner(const InnerTask* d_tasks, const int* d_wave_task, const int* d_first_wave,
                                    int nwaves, bool vec, hipStream_t s);
template <class T> void launch_apply_leaf(const LeafTask* d_tasks, int ntasks, bool vec, hipStream_t s);
constexpr size_t kLdsBudget = 156 * 1024;
constexpr size_t kLdsPerCu = 160 * 1024;   // LDS of one compute unit
constexpr size_t kSmallLds = 32 * 1024;   // LDS-resident tasks up to this size use 256-thread workgroups
constexpr size_t kMidLds = 80 * 1024;     // pivoted QR of cores up to this size on 512-thread workgroups
inline size_t lds_bytes_qr(const QrTask& t, size_t w) { return (size_t)t.m * t.r * w; }
// Row stride of W^T (q x t) in LDS for the scalar sweeps: q rounded up to 8
// modulo 16 doubles, so that the vectors that the 8-lane groups of a
// wavefront read together start in different LDS banks (q itself where the
// padding would not fit)
__host__ __device__ inline int jacobi_ld(int q, int t) {
  const int ld = q + ((8 - q) % 16 + 16) % 16;
  return (size_t)ld * t * 8 <= kLdsBudget ? ld : q;
}
inline size_t lds_bytes_jacobi(const SvdTask& t) { return (size_t)jacobi_ld(t.q, t.tc) * t.tc * 8; }
inline size_t lds_bytes_pchol_packed(int r) { return (size_t)r * (r + 1) / 2 * 8 + (size_t)r * 4; }
// register-tiled pivoted Cholesky: the scaled column, the pivot diagonals and
// kPcholChunk buffered columns of L (doubles), perm, posof, alive (ints)
constexpr int kPcholChunk = 32;
inline size_t lds_bytes_pchol_reg(int r) { return (size_t)r * ((2 + kPcholChunk) * 8 + 3 * 4); }
constexpr int kSvdWave = 64;
inline bool svd_wave_ok(const SvdTask& t) {
  return t.mode == 0 && t.p <= kSvdWave && t.q <= kSvdWave && t.r <= kSvdWave;
}
inline size_t lds_bytes_svd_wave(const SvdTask& t, size_t w) {
  (void)w;
  const size_t lc = t.p | 1;
  return (lc * t.q + t.q) * 8 + (size_t)2 * t.q * 4;
}
// default LDS limit of the one-workgroup path for cores beyond the wavefront
// size (0: such cores take the two-kernel path, the faster one at the n = 128
// benchmark shapes; acr_options_t.svd_fused_lds / acr_autotune change it)
constexpr size_t kFusedLds = 0;
// C (ld p|1), q norms, q pivots, the q-entry position -> column map
inline size_t lds_bytes_qrcp(const SvdTask& t) { return ((size_t)(t.p | 1) * t.q + t.q) * 8 + (size_t)t.q * 8; }
inline size_t lds_bytes_svd_block(const SvdTask& t) {
  const size_t lc = t.p | 1;
  return (lc * t.q + t.q) * 8 + (size_t)2 * t.q * 4;
}
inline size_t lds_bytes_applyq(const ApplyQTask& t, size_t w) { return ((size_t)t.m * t.p + (size_t)t.m * t.k) * w; }

}  // namespace acr
