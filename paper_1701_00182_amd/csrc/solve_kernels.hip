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

}  // namespace

template <class T>
void launch_inner(const InnerTask* d_tasks, const int* d_wave_task, const int* d_first_wave, int nwaves,
                  hipStream_t s) {
  if (nwaves <= 0) return;
  hipLaunchKernelGGL(k_inner<T>, dim3((nwaves + 3) / 4), dim3(256), 0, s, d_tasks, d_wave_task, d_first_wave, nwaves);
}

template <class T> void launch_apply_leaf(const LeafTask* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_apply_leaf<T>, dim3(ntasks), dim3(64), 0, s, d_tasks);
}

template void launch_inner<float>(const InnerTask*, const int*, const int*, int, hipStream_t);
template void launch_inner<double>(const InnerTask*, const int*, const int*, int, hipStream_t);
template void launch_apply_leaf<float>(const LeafTask*, int, hipStream_t);
template void launch_apply_leaf<double>(const LeafTask*, int, hipStream_t);

}  // namespace acr
