// Fused HODLR matrix-vector kernels for the solve sweeps (few right-hand sides).
//
// A HODLR product y = H x splits into (i) one small inner product per
// off-diagonal block, t_b = V_b^T x[cols_b], and (ii) for every leaf row range,
// y_leaf = H_leaf x_leaf + sum over the leaf's ancestors of U_b[leaf rows] t_b.
// k_inner computes all t_b of a level (one wavefront per column of V_b).
// k_apply_leaf computes, per (plane, leaf), beta * y_in + sum of up to two
// alpha * H x terms (the E and F couplings of one plane), reading each leaf
// and each U-slice exactly once: the forward reduction and back-substitution
// of Eq. elim / Eq. all_backSubs become two streaming launches per step.
//
// Both have a 16-byte vector form (float4 / double2 rows per lane) used when
// every leaf size, leading dimension and base address of a batch allows it:
// k_apply_leaf_vec spreads a leaf's columns over the 256 threads of a
// workgroup (rows in 16-byte vectors, columns interleaved over lane groups,
// partial sums reduced through LDS), k_inner_vec reads V and x as vectors.
#include "kern.h"

namespace acr {

namespace {

template <class T>
__global__ __launch_bounds__(256) void k_inner(const InnerTask* __restrict__ tasks, const int* __restrict__ wave_task,
                                               const int* __restrict__ first_wave, int nwaves) {
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (wv >= nwaves) return;
  const int ti = wave_task[wv];
  const InnerTask t = tasks[ti];
  const int col = wv - first_wave[ti];
  const T* v = static_cast<const T*>(t.V) + (int64_t)col * t.ldv;
  const T* x = static_cast<const T*>(t.x);
  T* out = static_cast<T*>(t.t);
  for (int j = 0; j < t.c; ++j) {
    const T* xj = x + (int64_t)j * t.ldx;
    float accf = 0.f;
    double accd = 0.0;
    for (int i = lane; i < t.rows; i += 64) {
      if (sizeof(T) == 4) accf += (float)v[i] * (float)xj[i];
      else accd += (double)v[i] * (double)xj[i];
    }
    double acc = sizeof(T) == 4 ? (double)accf : accd;
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) out[col + (int64_t)j * t.k] = T(acc);
  }
}

template <class T>
__global__ __launch_bounds__(64) void k_apply_leaf(const LeafTask* __restrict__ tasks) {
  const LeafTask& t = tasks[blockIdx.x];
  const int n = t.n, c = t.c;
  T* y = static_cast<T*>(t.y);
  const T* yin = static_cast<const T*>(t.yin);
  for (int i = threadIdx.x; i < n; i += 64) {
    for (int j = 0; j < c; ++j) {
      T acc = (t.beta != 0.0 && yin) ? T(t.beta) * yin[i + (int64_t)j * t.ldy] : T(0);
      for (int q = 0; q < t.nterm; ++q) {
        const LeafTerm& tm = t.term[q];
        const T* x = static_cast<const T*>(tm.x) + (int64_t)j * tm.ldx;
        T s = T(0);
        if (tm.diag) {
          s = static_cast<const T*>(tm.diag)[i] * x[i];
        } else {
          const T* Lf = static_cast<const T*>(tm.leaf);
          if (!tm.trans) {
            for (int l = 0; l < n; ++l) s += Lf[i + (int64_t)l * n] * x[l];
          } else {
            for (int l = 0; l < n; ++l) s += Lf[l + (int64_t)i * n] * x[l];
          }
          for (int d = 0; d < tm.nd; ++d) {
            const T* U = static_cast<const T*>(tm.up[d]);
            const T* tv = static_cast<const T*>(tm.tp[d]) + (int64_t)j * tm.kd[d];
            const int64_t ld = tm.ldu[d];
            for (int col = 0; col < tm.kd[d]; ++col) s += U[i + (int64_t)col * ld] * tv[col];
          }
        }
        acc += T(tm.alpha) * s;
      }
      y[i + (int64_t)j * t.ldy] = acc;
    }
  }
}

template <class T> struct Vec16;
template <> struct Vec16<float> {
  typedef float V __attribute__((ext_vector_type(4)));
  static constexpr int W = 4;
};
template <> struct Vec16<double> {
  typedef double V __attribute__((ext_vector_type(2)));
  static constexpr int W = 2;
};

template <class T>
__device__ inline T hsum(typename Vec16<T>::V v) {
  T s = v[0];
#pragma unroll
  for (int i = 1; i < Vec16<T>::W; ++i) s += v[i];
  return s;
}

template <class T>
__global__ __launch_bounds__(256) void k_inner_vec(const InnerTask* __restrict__ tasks,
                                                   const int* __restrict__ wave_task,
                                                   const int* __restrict__ first_wave, int nwaves) {
  typedef typename Vec16<T>::V V;
  constexpr int W = Vec16<T>::W;
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (wv >= nwaves) return;
  const int ti = wave_task[wv];
  const InnerTask t = tasks[ti];
  const int col = wv - first_wave[ti];
  const V* v = reinterpret_cast<const V*>(static_cast<const T*>(t.V) + (int64_t)col * t.ldv);
  const int rv = t.rows / W;
  T* out = static_cast<T*>(t.t);
  for (int j = 0; j < t.c; ++j) {
    const V* xj = reinterpret_cast<const V*>(static_cast<const T*>(t.x) + (int64_t)j * t.ldx);
    V a0 = V(0), a1 = V(0);
    int i = lane;
    for (; i + 64 < rv; i += 128) {
      a0 += v[i] * xj[i];
      a1 += v[i + 64] * xj[i + 64];
    }
    if (i < rv) a0 += v[i] * xj[i];
    double acc = (double)hsum<T>(a0 + a1);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) out[col + (int64_t)j * t.k] = T(acc);
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_apply_leaf_vec(const LeafTask* __restrict__ tasks) {
  typedef typename Vec16<T>::V V;
  constexpr int W = Vec16<T>::W;
  __shared__ V part[256];
  const LeafTask& t = tasks[blockIdx.x];
  const int n = t.n, rv = n / W;
  const int ng = 256 / rv;
  const int r = threadIdx.x % rv, g = threadIdx.x / rv;
  for (int j = 0; j < t.c; ++j) {
    V acc = V(0);
    if (g < ng) {
      for (int q = 0; q < t.nterm; ++q) {
        const LeafTerm& tm = t.term[q];
        const T a = T(tm.alpha);
        const T* x = static_cast<const T*>(tm.x) + (int64_t)j * tm.ldx;
        if (tm.diag) {
          if (g == 0) {
            const V d = reinterpret_cast<const V*>(tm.diag)[r];
            const V xv = reinterpret_cast<const V*>(x)[r];
            acc += a * d * xv;
          }
          continue;
        }
        const T* Lf = static_cast<const T*>(tm.leaf);
        for (int l = g; l < n; l += ng) acc += (a * x[l]) * reinterpret_cast<const V*>(Lf + (int64_t)l * n)[r];
        for (int d = 0; d < tm.nd; ++d) {
          const T* U = static_cast<const T*>(tm.up[d]);
          const T* tv = static_cast<const T*>(tm.tp[d]) + (int64_t)j * tm.kd[d];
          const int64_t ld = tm.ldu[d];
          for (int col = g; col < tm.kd[d]; col += ng)
            acc += (a * tv[col]) * reinterpret_cast<const V*>(U + (int64_t)col * ld)[r];
        }
      }
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < rv) {
      V s = part[threadIdx.x];
      for (int g2 = 1; g2 < ng; ++g2) s += part[threadIdx.x + g2 * rv];
      if (t.beta != 0.0 && t.yin)
        s += T(t.beta) * reinterpret_cast<const V*>(static_cast<const T*>(t.yin) + (int64_t)j * t.ldy)[r];
      reinterpret_cast<V*>(static_cast<T*>(t.y) + (int64_t)j * t.ldy)[r] = s;
    }
    __syncthreads();
  }
}

}  // namespace

template <class T>
void launch_inner(const InnerTask* d_tasks, const int* d_wave_task, const int* d_first_wave, int nwaves, bool vec,
                  hipStream_t s) {
  if (nwaves <= 0) return;
  if (vec)
    hipLaunchKernelGGL(k_inner_vec<T>, dim3((nwaves + 3) / 4), dim3(256), 0, s, d_tasks, d_wave_task, d_first_wave,
                       nwaves);
  else
    hipLaunchKernelGGL(k_inner<T>, dim3((nwaves + 3) / 4), dim3(256), 0, s, d_tasks, d_wave_task, d_first_wave,
                       nwaves);
}

template <class T> void launch_apply_leaf(const LeafTask* d_tasks, int ntasks, bool vec, hipStream_t s) {
  if (ntasks <= 0) return;
  if (vec)
    hipLaunchKernelGGL(k_apply_leaf_vec<T>, dim3(ntasks), dim3(256), 0, s, d_tasks);
  else
    hipLaunchKernelGGL(k_apply_leaf<T>, dim3(ntasks), dim3(64), 0, s, d_tasks);
}

template void launch_inner<float>(const InnerTask*, const int*, const int*, int, bool, hipStream_t);
template void launch_inner<double>(const InnerTask*, const int*, const int*, int, bool, hipStream_t);
template void launch_apply_leaf<float>(const LeafTask*, int, bool, hipStream_t);
template void launch_apply_leaf<double>(const LeafTask*, int, bool, hipStream_t);

}  // namespace acr
