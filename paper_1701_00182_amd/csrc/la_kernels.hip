// Batched dense linear-algebra kernels for the hierarchical block operations.
//
// One launch processes a list of independent small problems (all blocks of one
// hierarchical depth over all planes of a cyclic-reduction level).  Kernels:
//   k_gemm     tiled C = alpha op(A) op(B) + beta C over a tile map
//   k_copy     scaled copies / accumulations of sub-matrices (stack assembly)
//   k_inverse  Gauss-Jordan inverse with partial pivoting (dense leaves,
//              the small capacitance matrices of the HODLR inverse)
// The compression kernels (Householder QR, pivoted-QR + Jacobi SVD, apply-Q,
// Gram path) live in la_lds.hip, svd.hip and gram.hip.
#include "kern.h"

#include <cfloat>
#include <cmath>

namespace acr {

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the 256 threads of a workgroup; every thread gets the result.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

template <class T>
__global__ __launch_bounds__(256) void k_gemm(const GemmTask* __restrict__ tasks,
                                              const int* __restrict__ tile_task,
                                              const int* __restrict__ first_tile) {
  const int tile = blockIdx.x;
  const int ti = tile_task[tile];
  const GemmTask t = tasks[ti];
  const int local = tile - first_tile[ti];
  const int ntn = (t.n + 63) >> 6;
  const int row0 = (local / ntn) * 64, col0 = (local % ntn) * 64;
  __shared__ T As[16][65];
  __shared__ T Bs[16][65];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  T acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = T(0);
  const T* A = static_cast<const T*>(t.A);
  const T* B = static_cast<const T*>(t.B);
  for (int k0 = 0; k0 < t.k; k0 += 16) {
    for (int e = tid; e < 1024; e += 256) {
      int i, kk;
      if (!t.ta) { i = e & 63; kk = e >> 6; } else { kk = e & 15; i = e >> 4; }
      const int gi = row0 + i, gk = k0 + kk;
      T v = T(0);
      if (gi < t.m && gk < t.k)
        v = t.ta ? A[gk + (int64_t)gi * t.lda] : A[gi + (int64_t)gk * t.lda];
      As[kk][i] = v;
    }
    for (int e = tid; e < 1024; e += 256) {
      int j, kk;
      if (!t.tb) { kk = e & 15; j = e >> 4; } else { j = e & 63; kk = e >> 6; }
      const int gj = col0 + j, gk = k0 + kk;
      T v = T(0);
      if (gj < t.n && gk < t.k)
        v = t.tb ? B[gj + (int64_t)gk * t.ldb] : B[gk + (int64_t)gj * t.ldb];
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][tx + 16 * q];
        b[q] = Bs[kk][ty + 16 * q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
    }
    __syncthreads();
  }
  T* C = static_cast<T*>(t.C);
  const T alpha = T(t.alpha), beta = T(t.beta);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gj = col0 + ty + 16 * q;
    if (gj >= t.n) continue;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int gi = row0 + tx + 16 * p;
      if (gi >= t.m) continue;
      T* c = C + gi + (int64_t)gj * t.ldc;
      T v = alpha * acc[p][q];
      if (t.beta != 0.0) v += beta * *c;
      *c = v;
    }
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_copy(const CopyTask* __restrict__ tasks) {
  const CopyTask t = tasks[blockIdx.x];
  const int64_t total = (int64_t)t.m * t.n;
  const T* src = static_cast<const T*>(t.src);
  T* dst = static_cast<T*>(t.dst);
  const T* rs = static_cast<const T*>(t.rs);
  const T* cs = static_cast<const T*>(t.cs);
  const T alpha = T(t.alpha);
  for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.y * 256) {
    const int i = (int)(e % t.m), j = (int)(e / t.m);
    T v = src ? alpha * src[i + (int64_t)j * t.lds] : (i == j ? alpha : T(0));
    if (rs) v *= rs[i];
    if (cs) v *= cs[j];
    T* d = dst + i + (int64_t)j * t.ldd;
    if (t.accumulate) v += *d;
    *d = v;
  }
}

// Gauss-Jordan inversion with partial pivoting.  LDS=true stages the matrix in
// shared memory (s * s elements), otherwise it works on the global copy.
template <class T, bool LDS>
__global__ __launch_bounds__(256) void k_inverse(const InvTask* __restrict__ tasks, int* flags) {
  extern __shared__ double smem_d[];
  const InvTask t = tasks[blockIdx.x];
  const int s = t.s;
  if (s == 0) return;
  T* g = static_cast<T*>(t.A);
  T* a;
  int64_t la;
  int* piv;
  if (LDS) {
    a = reinterpret_cast<T*>(smem_d);
    la = s;
    piv = reinterpret_cast<int*>(a + (int64_t)s * s);
    for (int e = threadIdx.x; e < s * s; e += 256) a[e] = g[(e % s) + (int64_t)(e / s) * t.lda];
  } else {
    a = g;
    la = t.lda;
    piv = reinterpret_cast<int*>(smem_d);
  }
  __shared__ double rv[256];
  __shared__ int ri[256];
  __shared__ int sh_p;
  __syncthreads();
  bool bad = false;
  for (int j = 0; j < s; ++j) {
    double best = -1.0;
    int bi = j;
    for (int i = j + threadIdx.x; i < s; i += 256) {
      const double v = fabs((double)a[i + j * la]);
      if (v > best) { best = v; bi = i; }
    }
    rv[threadIdx.x] = best;
    ri[threadIdx.x] = bi;
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
    if (threadIdx.x == 0) { sh_p = ri[0]; piv[j] = ri[0]; }
    __syncthreads();
    const int p = sh_p;
    if (p != j) {
      for (int c = threadIdx.x; c < s; c += 256) {
        const T tmp = a[j + c * la];
        a[j + c * la] = a[p + c * la];
        a[p + c * la] = tmp;
      }
    }
    __syncthreads();
    const T pv = a[j + j * la];
    if (!(pv != T(0)) || !isfinite((double)pv)) bad = true;
    const T inv = T(1) / pv;
    __syncthreads();
    for (int c = threadIdx.x; c < s; c += 256)
      if (c != j) a[j + c * la] *= inv;
    __syncthreads();
    for (int64_t e = threadIdx.x; e < (int64_t)s * s; e += 256) {
      const int i = (int)(e % s), c = (int)(e / s);
      if (i != j && c != j) a[i + c * la] -= a[i + j * la] * a[j + c * la];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < s; i += 256)
      if (i != j) a[i + j * la] = -a[i + j * la] * inv;
    if (threadIdx.x == 0) a[j + j * la] = inv;
    __syncthreads();
  }
  for (int j = s - 1; j >= 0; --j) {
    const int p = piv[j];
    if (p != j) {
      for (int r = threadIdx.x; r < s; r += 256) {
        const T tmp = a[r + j * la];
        a[r + j * la] = a[r + p * la];
        a[r + p * la] = tmp;
      }
    }
    __syncthreads();
  }
  if (LDS) {
    for (int e = threadIdx.x; e < s * s; e += 256) g[(e % s) + (int64_t)(e / s) * t.lda] = a[e];
  }
  if (bad && threadIdx.x == 0) atomicOr(&flags[FLAG_SINGULAR], 1);
}

}  // namespace

template <class T>
void launch_gemm(const GemmTask* d_tasks, const int* d_tile_task, const int* d_first_tile, int ntiles,
                 hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_gemm<T>, dim3(ntiles), dim3(256), 0, s, d_tasks, d_tile_task, d_first_tile);
}

template <class T>
void launch_copy(const CopyTask* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_copy<T>, dim3(ntasks, 8), dim3(256), 0, s, d_tasks);
}

template <class T>
void launch_inverse(const InvTask* d_tasks, int ntasks, int max_s, int* d_flags, hipStream_t s) {
  if (ntasks <= 0) return;
  const size_t lds_bytes = (size_t)max_s * max_s * sizeof(T) + (size_t)max_s * sizeof(int);
  if (lds_bytes <= 60 * 1024) {
    hipLaunchKernelGGL((k_inverse<T, true>), dim3(ntasks), dim3(256), lds_bytes, s, d_tasks, d_flags);
  } else {
    hipLaunchKernelGGL((k_inverse<T, false>), dim3(ntasks), dim3(256), (size_t)max_s * sizeof(int), s,
                       d_tasks, d_flags);
  }
}

#define ACR_INST(T)                                                                              \
  template void launch_gemm<T>(const GemmTask*, const int*, const int*, int, hipStream_t);      \
  template void launch_copy<T>(const CopyTask*, int, hipStream_t);                              \
  template void launch_inverse<T>(const InvTask*, int, int, int*, hipStream_t);

ACR_INST(float)
ACR_INST(double)
#undef ACR_INST

}  // namespace acr
