// Householder QR of stacked bases and the reconstruction Q [Z; 0], in an
// LDS-resident instantiation for panels that fit the 160 KB local data share of
// a CDNA4 compute unit and a global-memory one otherwise.  Trailing columns are
// processed concurrently by groups of G lanes that reduce with intra-group
// shuffles, so one workgroup keeps its 1024 lanes busy even on 64 x 64 panels.
#include <cmath>

#include "kern.h"

namespace acr {

namespace {

__device__ inline double gsum(double v, int G) {
  for (int off = G >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

template <int NT> __device__ inline double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

// Lanes per column group for one step over `cols` columns of `rows` live rows
// with nt threads: enough groups to take every column at once (short shuffle
// reductions, no column queue per group), and enough lanes that a column slice
// fits kRC registers.
constexpr int kRC = 16;
__device__ inline int step_lanes(int rows, int cols, int nt) {
  int G = 4;
  while (G < 64 && 2 * G * cols <= nt) G <<= 1;
  while (G < 64 && rows > G * kRC) G <<= 1;
  return G;
}

template <class T, bool LDS, int NT>
__global__ __launch_bounds__(NT) void k_qr_lds(const QrTask* __restrict__ tasks) {
  extern __shared__ double smq[];
  const QrTask t = tasks[blockIdx.x];
  T* A = static_cast<T*>(t.A);
  T* tau = static_cast<T*>(t.tau);
  const int m = t.m, r = t.r;
  T* a = LDS ? reinterpret_cast<T*>(smq) : A;
  const int64_t la = LDS ? m : t.lda;
  if (LDS)
    for (int e = threadIdx.x; e < m * r; e += NT) a[e] = A[(e % m) + (int64_t)(e / m) * t.lda];
  __shared__ double red[NT / 64];
  __shared__ double sh_sig[2];
  const int nref = m < r ? m : r;
  __syncthreads();
  // sigma_j = squared norm of column j below the diagonal; for j > 0 it comes
  // from the group that updated column j in the previous step
  double sigma = 0.0;
  {
    double ps = 0.0;
    for (int i = 1 + threadIdx.x; i < m; i += NT) {
      const double v = (double)a[i];
      ps += v * v;
    }
    sigma = block_sum<NT>(ps, red);
  }
  for (int j = 0; j < nref; ++j) {
    T* col = a + j * la;
    const double x0 = (double)col[j];
    double tj = 0.0, scale = 0.0, beta = x0;
    if (sigma != 0.0) {
      const double nrm = sqrt(x0 * x0 + sigma);
      beta = x0 >= 0.0 ? -nrm : nrm;
      tj = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    if (threadIdx.x == 0) tau[j] = T(tj);
    // v = (1, x_{j+1..} * scale) rounded to T as it will be stored, applied to
    // the trailing columns on the fly; each lane's slice of v and of the column
    // sits in registers when it fits
    const int G = step_lanes(m - j, r - j - 1, NT), groups = NT / G;
    const int gi = threadIdx.x / G, gl = threadIdx.x % G;
    if (m - j <= G * kRC) {
      double v[kRC];
#pragma unroll
      for (int u = 0; u < kRC; ++u) {
        const int i = j + gl + u * G;
        v[u] = i < m ? (i == j ? 1.0 : (double)T((double)col[i] * scale)) : 0.0;
      }
      for (int c = j + 1 + gi; c < r; c += groups) {
        T* ac = a + c * la;
        double x[kRC];
#pragma unroll
        for (int u = 0; u < kRC; ++u) {
          const int i = j + gl + u * G;
          x[u] = i < m ? (double)ac[i] : 0.0;
        }
        if (tj != 0.0) {
          double w = 0.0;
#pragma unroll
          for (int u = 0; u < kRC; ++u) w += v[u] * x[u];
          w = gsum(w, G) * tj;
#pragma unroll
          for (int u = 0; u < kRC; ++u) {
            const int i = j + gl + u * G;
            x[u] = (double)T(x[u] - w * v[u]);
            if (i < m) ac[i] = T(x[u]);
          }
        }
        if (c == j + 1) {
          double sn = 0.0;
#pragma unroll
          for (int u = 0; u < kRC; ++u) sn += (gl + u * G >= 2) ? x[u] * x[u] : 0.0;
          sn = gsum(sn, G);
          if (gl == 0) sh_sig[j & 1] = sn;
        }
      }
    } else {
      for (int c = j + 1 + gi; c < r; c += groups) {
        T* ac = a + c * la;
        if (tj != 0.0) {
          double w = 0.0;
          for (int i = j + gl; i < m; i += G) w += (i == j ? 1.0 : (double)T((double)col[i] * scale)) * (double)ac[i];
          w = gsum(w, G) * tj;
          for (int i = j + gl; i < m; i += G)
            ac[i] = T((double)ac[i] - w * (i == j ? 1.0 : (double)T((double)col[i] * scale)));
        }
        if (c == j + 1) {
          double sn = 0.0;
          for (int i = j + 2 + gl; i < m; i += G) {
            const double v = (double)ac[i];
            sn += v * v;
          }
          sn = gsum(sn, G);
          if (gl == 0) sh_sig[j & 1] = sn;
        }
      }
    }
    __syncthreads();
    // column j is no longer read: store its reflector and the diagonal of R
    if (tj != 0.0)
      for (int i = j + 1 + threadIdx.x; i < m; i += NT) col[i] = T((double)col[i] * scale);
    if (threadIdx.x == 0) col[j] = T(beta);
    sigma = sh_sig[j & 1];
  }
  __syncthreads();
  if (LDS)
    for (int e = threadIdx.x; e < m * r; e += NT) A[(e % m) + (int64_t)(e / m) * t.lda] = a[e];
}

template <class T, bool LDS, int NT>
__global__ __launch_bounds__(NT) void k_applyq_lds(const ApplyQTask* __restrict__ tasks) {
  extern __shared__ double sma[];
  const ApplyQTask t = tasks[blockIdx.x];
  const int m = t.m, p = t.p, k = t.k;
  if (k == 0 || m == 0) return;
  const T* Aq = static_cast<const T*>(t.Aq);
  const T* tau = static_cast<const T*>(t.tau);
  T* out = static_cast<T*>(t.out);
  const T* v = LDS ? reinterpret_cast<T*>(sma) : Aq;
  const int64_t lv = LDS ? m : t.lda;
  T* o = LDS ? reinterpret_cast<T*>(sma) + m * p : out;
  const int64_t lo = LDS ? m : t.ldo;
  if (LDS)
    for (int e = threadIdx.x; e < m * p; e += NT)
      reinterpret_cast<T*>(sma)[e] = Aq[(e % m) + (int64_t)(e / m) * t.lda];
  for (int e = threadIdx.x; e < m * k; e += NT) {
    const int i = e % m, c = e / m;
    o[i + c * lo] = i < p ? T(t.Z[i + (int64_t)c * t.ldz]) : T(0);
  }
  __syncthreads();
  for (int j = p - 1; j >= 0; --j) {
    const double tj = (double)tau[j];
    if (tj == 0.0) continue;
    const T* vj = v + j * lv;
    const int G = step_lanes(m - j, k, NT), groups = NT / G;
    const int gi = threadIdx.x / G, gl = threadIdx.x % G;
    if (m - j <= G * kRC) {
      double vr[kRC];
#pragma unroll
      for (int u = 0; u < kRC; ++u) {
        const int i = j + gl + u * G;
        vr[u] = i < m ? (i == j ? 1.0 : (double)vj[i]) : 0.0;
      }
      for (int c = gi; c < k; c += groups) {
        T* oc = o + c * lo;
        double x[kRC];
        double w = 0.0;
#pragma unroll
        for (int u = 0; u < kRC; ++u) {
          const int i = j + gl + u * G;
          x[u] = i < m ? (double)oc[i] : 0.0;
          w += vr[u] * x[u];
        }
        w = gsum(w, G) * tj;
#pragma unroll
        for (int u = 0; u < kRC; ++u) {
          const int i = j + gl + u * G;
          if (i < m) oc[i] = T(x[u] - w * vr[u]);
        }
      }
    } else {
      for (int c = gi; c < k; c += groups) {
        T* oc = o + c * lo;
        double w = 0.0;
        for (int i = j + gl; i < m; i += G) w += (i == j ? 1.0 : (double)vj[i]) * (double)oc[i];
        w = gsum(w, G) * tj;
        for (int i = j + gl; i < m; i += G) oc[i] = T((double)oc[i] - w * (i == j ? 1.0 : (double)vj[i]));
      }
    }
    __syncthreads();
  }
  if (LDS)
    for (int e = threadIdx.x; e < m * k; e += NT) out[(e % m) + (int64_t)(e / m) * t.ldo] = o[e];
}

template <class K> void allow_lds(K kernel, size_t bytes) {
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

}  // namespace

// lds == 0 selects the global-memory instantiation (same algorithm).  Panels
// of up to kSmallLds bytes run with 256 threads (several workgroups share a
// compute unit), larger ones with 1024.
template <class T> void launch_qr_lds(const QrTask* d_tasks, int ntasks, size_t lds, hipStream_t s) {
  if (ntasks <= 0) return;
  if (lds == 0) {
    hipLaunchKernelGGL((k_qr_lds<T, false, 1024>), dim3(ntasks), dim3(1024), 0, s, d_tasks);
    return;
  }
  if (lds <= kSmallLds) {
    allow_lds(k_qr_lds<T, true, 256>, lds);
    hipLaunchKernelGGL((k_qr_lds<T, true, 256>), dim3(ntasks), dim3(256), lds, s, d_tasks);
    return;
  }
  allow_lds(k_qr_lds<T, true, 1024>, lds);
  hipLaunchKernelGGL((k_qr_lds<T, true, 1024>), dim3(ntasks), dim3(1024), lds, s, d_tasks);
}

template <class T> void launch_applyq_lds(const ApplyQTask* d_tasks, int ntasks, size_t lds, hipStream_t s) {
  if (ntasks <= 0) return;
  if (lds == 0) {
    hipLaunchKernelGGL((k_applyq_lds<T, false, 1024>), dim3(ntasks), dim3(1024), 0, s, d_tasks);
    return;
  }
  if (lds <= kSmallLds) {
    allow_lds(k_applyq_lds<T, true, 256>, lds);
    hipLaunchKernelGGL((k_applyq_lds<T, true, 256>), dim3(ntasks), dim3(256), lds, s, d_tasks);
    return;
  }
  allow_lds(k_applyq_lds<T, true, 1024>, lds);
  hipLaunchKernelGGL((k_applyq_lds<T, true, 1024>), dim3(ntasks), dim3(1024), lds, s, d_tasks);
}

#define ACR_LDS_INST(T)                                                                           \
  template void launch_qr_lds<T>(const QrTask*, int, size_t, hipStream_t);                        \
  template void launch_applyq_lds<T>(const ApplyQTask*, int, size_t, hipStream_t);
ACR_LDS_INST(float)
ACR_LDS_INST(double)
#undef ACR_LDS_INST

}  // namespace acr
