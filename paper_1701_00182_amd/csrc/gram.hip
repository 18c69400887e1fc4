// Gram-based compression of large stacked low-rank sums.
//
// For a stack S (m x r) too large for one workgroup's local memory, the
// triangular factor is obtained from the FP64 Gram matrix S^T S (computed by
// many workgroups, each over a chunk of rows, then reduced in a fixed order)
// and a pivoted Cholesky factorisation that stops at the numerical rank:
//   S P = Q [L11^T L21^T],  Q = S P1 L11^{-T}.
// The core (L-factors of both stacks) then goes through the same one-sided
// Jacobi SVD as the Householder path, and the truncated bases are rebuilt with
// one GEMM each: U_new = S W with W = P1 L11^{-T} Z.
#include <cmath>

#include "kern.h"

namespace acr {

namespace {

constexpr int kGT = 32;  // Gram tile

template <class T>
__global__ __launch_bounds__(256) void k_gram_partial(const GramTask* __restrict__ tasks,
                                                      const int* __restrict__ tile_task,
                                                      const int* __restrict__ first_tile) {
  const int tile = blockIdx.x;
  const int ti = tile_task[tile];
  const GramTask t = tasks[ti];
  int local = tile - first_tile[ti];
  const int nb = (t.r + kGT - 1) / kGT;
  const int ntri = nb * (nb + 1) / 2;
  const int chunk = local / ntri;
  int tri = local - chunk * ntri;
  // tri -> (bi, bj) with bi <= bj
  int bi = 0;
  while (tri >= nb - bi) { tri -= nb - bi; ++bi; }
  const int bj = bi + tri;
  const int r0 = chunk * t.rows_per_chunk;
  const int r1 = min(t.m, r0 + t.rows_per_chunk);
  const T* A = static_cast<const T*>(t.A);
  __shared__ double Ai[kGT][kGT + 1];
  __shared__ double Aj[kGT][kGT + 1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // ty in 0..7
  double acc[4] = {0, 0, 0, 0};
  for (int row = r0; row < r1; row += kGT) {
    for (int e = threadIdx.x; e < kGT * kGT; e += 256) {
      const int rr = e & 31, cc = e >> 5;
      const int gr = row + rr;
      const int ci = bi * kGT + cc, cj = bj * kGT + cc;
      Ai[rr][cc] = (gr < r1 && ci < t.r) ? (double)A[gr + (int64_t)ci * t.lda] : 0.0;
      Aj[rr][cc] = (gr < r1 && cj < t.r) ? (double)A[gr + (int64_t)cj * t.lda] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < kGT; ++rr) {
      const double b = Aj[rr][tx];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += Ai[rr][ty + 8 * q] * b;
    }
    __syncthreads();
  }
  double* P = t.part + (int64_t)chunk * t.r * t.r;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = bi * kGT + ty + 8 * q, j = bj * kGT + tx;
    if (i < t.r && j < t.r) P[i + (int64_t)j * t.r] = acc[q];
  }
}

__global__ __launch_bounds__(256) void k_gram_reduce(const GramTask* __restrict__ tasks) {
  const GramTask t = tasks[blockIdx.x];
  const int nchunk = (t.m + t.rows_per_chunk - 1) / t.rows_per_chunk;
  const int64_t rr = (int64_t)t.r * t.r;
  for (int64_t e = threadIdx.x + (int64_t)blockIdx.y * 256; e < rr; e += (int64_t)gridDim.y * 256) {
    const int i = (int)(e % t.r), j = (int)(e / t.r);
    if (i > j) continue;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += t.part[c * rr + e];
    t.G[i + (int64_t)j * t.r] = s;
    t.G[j + (int64_t)i * t.r] = s;
  }
}

// Pivoted Cholesky of an r x r FP64 Gram matrix, stopped when the largest
// remaining diagonal falls to tol * (largest initial diagonal).
__global__ __launch_bounds__(256) void k_pchol(const PcholTask* __restrict__ tasks, double tol) {
  const PcholTask t = tasks[blockIdx.x];
  const int r = t.r;
  const double* G = t.G;
  double* L = t.L;
  int* perm = t.perm;
  double* d = t.d;
  __shared__ double rv[256];
  __shared__ int ri[256];
  __shared__ double sh_ljj;
  __shared__ int sh_stop;
  for (int64_t e = threadIdx.x; e < (int64_t)r * r; e += 256) L[e] = 0.0;
  for (int i = threadIdx.x; i < r; i += 256) {
    perm[i] = i;
    d[i] = G[i + (int64_t)i * r];
  }
  __syncthreads();
  double mx = 0.0;
  for (int i = threadIdx.x; i < r; i += 256) mx = fmax(mx, d[i]);
  rv[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) rv[threadIdx.x] = fmax(rv[threadIdx.x], rv[threadIdx.x + w]);
    __syncthreads();
  }
  const double thr = tol * rv[0];
  const bool zero = !(rv[0] > 0.0);
  __syncthreads();
  int rank = 0;
  for (int j = 0; j < r && !zero; ++j) {
    double best = -1.0;
    int bp = j;
    for (int i = j + threadIdx.x; i < r; i += 256) {
      const double v = d[perm[i]];
      if (v > best) { best = v; bp = i; }
    }
    rv[threadIdx.x] = best;
    ri[threadIdx.x] = bp;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        const double o = rv[threadIdx.x + w];
        const int oi = ri[threadIdx.x + w];
        if (o > rv[threadIdx.x] || (o == rv[threadIdx.x] && oi < ri[threadIdx.x])) {
          rv[threadIdx.x] = o;
          ri[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    const int p = ri[0];
    if (threadIdx.x == 0) {
      sh_stop = !(rv[0] > thr);
      if (!sh_stop) {
        const int tmp = perm[j];
        perm[j] = perm[p];
        perm[p] = tmp;
      }
    }
    __syncthreads();
    if (sh_stop) break;
    if (p != j)
      for (int l = threadIdx.x; l < j; l += 256) {
        const double a = L[j + (int64_t)l * r];
        L[j + (int64_t)l * r] = L[p + (int64_t)l * r];
        L[p + (int64_t)l * r] = a;
      }
    __syncthreads();
    if (threadIdx.x == 0) {
      sh_ljj = sqrt(d[perm[j]]);
      L[j + (int64_t)j * r] = sh_ljj;
    }
    __syncthreads();
    const double ljj = sh_ljj;
    const int pj = perm[j];
    for (int i = j + 1 + threadIdx.x; i < r; i += 256) {
      const int pi = perm[i];
      double s = G[pi + (int64_t)pj * r];
      for (int l = 0; l < j; ++l) s -= L[i + (int64_t)l * r] * L[j + (int64_t)l * r];
      const double lij = s / ljj;
      L[i + (int64_t)j * r] = lij;
      d[pi] -= lij * lij;
    }
    __syncthreads();
    rank = j + 1;
  }
  if (threadIdx.x == 0) *t.rank_out = rank;
}

// R (r1 x r, original column order): R[a, perm[i]] = L[i, a] for i >= a.
__global__ __launch_bounds__(256) void k_materialize_r(const PcholTask* __restrict__ tasks) {
  const PcholTask t = tasks[blockIdx.x];
  const int r = t.r, r1 = t.r1;
  for (int64_t e = threadIdx.x + (int64_t)blockIdx.y * 256; e < (int64_t)r1 * r; e += (int64_t)gridDim.y * 256) {
    const int a = (int)(e % r1), i = (int)(e / r1);
    t.R[a + (int64_t)t.perm[i] * r1] = i >= a ? t.L[i + (int64_t)a * r] : 0.0;
  }
}

// W = P1 L11^{-T} Z scattered into r x k (precision T): back-substitution per column.
template <class T>
__global__ __launch_bounds__(256) void k_wtilde(const WtTask* __restrict__ tasks) {
  const WtTask t = tasks[blockIdx.x];
  const int r = t.r, r1 = t.r1, k = t.k;
  T* W = static_cast<T*>(t.W);
  for (int64_t e = threadIdx.x; e < (int64_t)r * k; e += 256) W[e] = T(0);
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += 256) {
    double* z = t.Z + (int64_t)c * t.ldz;   // overwritten with the solution
    for (int a = r1 - 1; a >= 0; --a) {
      double s = z[a];
      for (int b = a + 1; b < r1; ++b) s -= t.L[b + (int64_t)a * r] * z[b];
      z[a] = s / t.L[a + (int64_t)a * r];
    }
    for (int a = 0; a < r1; ++a) W[t.perm[a] + (int64_t)c * r] = T(z[a]);
  }
}

}  // namespace

template <class T>
void launch_gram(const GramTask* d_tasks, int ntasks, const int* d_tile_task, const int* d_first_tile, int ntiles,
                 hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_gram_partial<T>, dim3(ntiles), dim3(256), 0, s, d_tasks, d_tile_task, d_first_tile);
  hipLaunchKernelGGL(k_gram_reduce, dim3(ntasks, 16), dim3(256), 0, s, d_tasks);
}

void launch_pchol(const PcholTask* d_tasks, int ntasks, double tol, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_pchol, dim3(ntasks), dim3(256), 0, s, d_tasks, tol);
}

void launch_materialize_r(const PcholTask* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_materialize_r, dim3(ntasks, 8), dim3(256), 0, s, d_tasks);
}

template <class T> void launch_wtilde(const WtTask* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_wtilde<T>, dim3(ntasks), dim3(256), 0, s, d_tasks);
}

template void launch_gram<float>(const GramTask*, int, const int*, const int*, int, hipStream_t);
template void launch_gram<double>(const GramTask*, int, const int*, const int*, int, hipStream_t);
template void launch_wtilde<float>(const WtTask*, int, hipStream_t);
template void launch_wtilde<double>(const WtTask*, int, hipStream_t);

}  // namespace acr
