// Batched dense linear-algebra kernels for the hierarchical block operations.
//
// One launch processes a list of independent small problems (all blocks of one
// hierarchical depth over all planes of a cyclic-reduction level).  Kernels:
//   k_copy     scaled copies / accumulations of sub-matrices (stack assembly)
//   k_inverse  Gauss-Jordan inverse with partial pivoting (dense leaves,
//              the small capacitance matrices of the HODLR inverse)
// The compression kernels (Householder QR, pivoted-QR + Jacobi SVD, apply-Q,
// Gram path) live in la_lds.hip, svd.hip and gram.hip; the matrix-core GEMM
// in gemm_mfma.hip.
#include "kern.h"
#include "wave.h"

#include <cfloat>
#include <cmath>

namespace acr {

namespace {

// 16-byte vector of T
template <class T> struct Vec16;
template <> struct Vec16<float> { using type = float4; static constexpr int n = 4; };
template <> struct Vec16<double> { using type = double2; static constexpr int n = 2; };

template <class T>
__device__ inline bool aligned16(const T* p) {
  return p == nullptr || (reinterpret_cast<uintptr_t>(p) & 15) == 0;
}

template <class T>
__global__ __launch_bounds__(256) void k_copy(const CopyTask* __restrict__ tasks) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  const CopyTask t = tasks[blockIdx.x];
  const T* src = static_cast<const T*>(t.src);
  T* dst = static_cast<T*>(t.dst);
  const T* rs = static_cast<const T*>(t.rs);
  const T* cs = static_cast<const T*>(t.cs);
  const T alpha = T(t.alpha);
  // units of (column, 2048-row chunk): one division per unit, none per element
  const int ich = (t.m + 2047) / 2048;
  const int64_t units = (int64_t)t.n * ich;
  for (int64_t u = blockIdx.y; u < units; u += gridDim.y) {
    const int j = (int)(u / ich), i0 = (int)(u % ich) * 2048;
    const int i1 = t.m < i0 + 2048 ? t.m : i0 + 2048;
    const T csj = cs ? cs[j] : T(1);
    const T* sc = src ? src + (int64_t)j * t.lds : nullptr;
    T* dc = dst + (int64_t)j * t.ldd;
    int i = i0 + threadIdx.x;
    // 16-byte vectors when every column pointer is aligned at the chunk start
    if (sc && aligned16(sc + i0) && aligned16(dc + i0) && (!rs || aligned16(rs + i0))) {
      const int nv = (i1 - i0) / VN;
      for (int e = threadIdx.x; e < nv; e += 256) {
        const int ib = i0 + e * VN;
        V x = *reinterpret_cast<const V*>(sc + ib);
        T* xv = reinterpret_cast<T*>(&x);
        V rv;
        if (rs) rv = *reinterpret_cast<const V*>(rs + ib);
        const T* rsv = reinterpret_cast<const T*>(&rv);
        V y;
        if (t.accumulate) y = *reinterpret_cast<const V*>(dc + ib);
        T* yv = reinterpret_cast<T*>(&y);
        V o;
        T* ov = reinterpret_cast<T*>(&o);
#pragma unroll
        for (int c = 0; c < VN; ++c) {
          T v = alpha * xv[c];
          if (rs) v *= rsv[c];
          v *= csj;
          if (t.accumulate) v += yv[c];
          ov[c] = v;
        }
        *reinterpret_cast<V*>(dc + ib) = o;
      }
      i = i0 + nv * VN + threadIdx.x;
    }
    for (; i < i1; i += 256) {
      T v = sc ? alpha * sc[i] : (i == j ? alpha : T(0));
      if (rs) v *= rs[i];
      v *= csj;
      if (t.accumulate) v += dc[i];
      dc[i] = v;
    }
  }
}

// Gauss-Jordan inversion with partial pivoting.  LDS=true stages the matrix in
// shared memory (s * s elements), otherwise it works on the global copy.
// Gauss-Jordan inverse with partial pivoting, in place (LDS copy when it fits).
// Per pivot: a wavefront-shuffle argmax, the row swap, the rank-1 update of
// every entry outside row / column j (row j scaled on the fly), then row j and
// column j: three workgroup barriers plus the argmax's two.
template <class T, bool LDS, int NT>
__global__ __launch_bounds__(NT) void k_inverse(const InvTask* __restrict__ tasks, int* flags) {
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
    staged_copy<NT>(
        (int64_t)s * s, [&](int64_t e) { return g[(int)e % s + (int64_t)((int)e / s) * t.lda]; },
        [&](int64_t e, T v) { a[e] = v; });
  } else {
    a = g;
    la = t.lda;
    piv = reinterpret_cast<int*>(smem_d);
  }
  __shared__ double red[NT / 64];
  __shared__ int redi[NT / 64];
  __syncthreads();
  bool bad = false;
  for (int j = 0; j < s; ++j) {
    double best = -1.0;
    int bi = j;
    for (int i = j + threadIdx.x; i < s; i += NT) {
      const double v = fabs((double)a[i + j * la]);
      if (v > best) { best = v; bi = i; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (o > best || (o == best && oi < bi)) { best = o; bi = oi; }
    }
    if ((threadIdx.x & 63) == 0) { red[threadIdx.x >> 6] = best; redi[threadIdx.x >> 6] = bi; }
    __syncthreads();
    best = red[0];
    int p = redi[0];
    for (int w = 1; w < NT / 64; ++w)
      if (red[w] > best || (red[w] == best && redi[w] < p)) { best = red[w]; p = redi[w]; }
    if (threadIdx.x == 0) piv[j] = p;
    if (p != j) {
      for (int c = threadIdx.x; c < s; c += NT) {
        const T tmp = a[j + c * la];
        a[j + c * la] = a[p + c * la];
        a[p + c * la] = tmp;
      }
    }
    __syncthreads();
    const T pv = a[j + j * la];
    if (!(pv != T(0)) || !isfinite((double)pv)) bad = true;
    const T inv = T(1) / pv;
    // a[i, c] -= a[i, j] (a[j, c] / pivot) for i, c != j: a wavefront per
    // column, lanes down the rows; column j's entries for a lane's rows are
    // read once per step (kInvRows per lane in registers, larger s in a loop)
    {
      constexpr int NW = NT / 64, kInvRows = 4;
      const int lane = threadIdx.x & 63;
      T aj[kInvRows];
#pragma unroll
      for (int u = 0; u < kInvRows; ++u) {
        const int i = lane + 64 * u;
        aj[u] = i < s ? a[i + j * la] : T(0);
      }
      for (int c = threadIdx.x >> 6; c < s; c += NW) {
        if (c == j) continue;
        T* col = a + c * la;
        const T rj = col[j] * inv;
#pragma unroll
        for (int u = 0; u < kInvRows; ++u) {
          const int i = lane + 64 * u;
          if (i < s && i != j) col[i] -= aj[u] * rj;
        }
        for (int i = lane + 64 * kInvRows; i < s; i += 64)
          if (i != j) col[i] -= a[i + j * la] * rj;
      }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < s; c += NT)
      if (c != j) {
        a[j + c * la] *= inv;
        a[c + j * la] = -a[c + j * la] * inv;
      }
    if (threadIdx.x == 0) a[j + j * la] = inv;
    __syncthreads();
  }
  for (int j = s - 1; j >= 0; --j) {
    const int p = piv[j];
    if (p != j) {
      for (int r = threadIdx.x; r < s; r += NT) {
        const T tmp = a[r + j * la];
        a[r + j * la] = a[r + p * la];
        a[r + p * la] = tmp;
      }
    }
    __syncthreads();
  }
  if (LDS) {
    for (int c = threadIdx.x >> 6; c < s; c += NT / 64)
      for (int i = threadIdx.x & 63; i < s; i += 64) g[i + (int64_t)c * t.lda] = a[i + c * s];
  }
  if (bad && threadIdx.x == 0) atomicOr(&flags[FLAG_SINGULAR], 1);
}

}  // namespace


template <class T>
void launch_copy(const CopyTask* d_tasks, int ntasks, int units, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_copy<T>, dim3(ntasks, units), dim3(256), 0, s, d_tasks);
}

template <class T>
void launch_inverse(const InvTask* d_tasks, int ntasks, int max_s, int* d_flags, hipStream_t s) {
  if (ntasks <= 0) return;
  const size_t lds_bytes = (size_t)max_s * max_s * sizeof(T) + (size_t)max_s * sizeof(int);
  if (lds_bytes <= kLdsBudget) {
    if (max_s < 96) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_inverse<T, true, 256>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
      hipLaunchKernelGGL((k_inverse<T, true, 256>), dim3(ntasks), dim3(256), lds_bytes, s, d_tasks, d_flags);
    } else {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_inverse<T, true, 1024>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
      hipLaunchKernelGGL((k_inverse<T, true, 1024>), dim3(ntasks), dim3(1024), lds_bytes, s, d_tasks, d_flags);
    }
  } else {
    hipLaunchKernelGGL((k_inverse<T, false, 1024>), dim3(ntasks), dim3(1024), (size_t)max_s * sizeof(int), s,
                       d_tasks, d_flags);
  }
}

#define ACR_INST(T)                                                                              \
  template void launch_copy<T>(const CopyTask*, int, int, hipStream_t);                         \
  template void launch_inverse<T>(const InvTask*, int, int, int*, hipStream_t);

ACR_INST(float)
ACR_INST(double)
#undef ACR_INST

}  // namespace acr
