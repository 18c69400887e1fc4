// Householder QR of stacked bases and the reconstruction Q [Z; 0], in an
// LDS-resident instantiation for panels that fit the 160 KB local data share of
// a CDNA4 compute unit and a global-memory one otherwise.  Trailing columns are
// processed concurrently by groups of G lanes that reduce with intra-group
// shuffles, so one workgroup keeps its 1024 lanes busy even on 64 x 64 panels.
#include <cmath>

#include "kern.h"
#include "wave.h"

namespace acr {

namespace {

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
// fits `cap` registers (16 for panels in LDS, 8 in global memory, whose 64-bit
// addresses take more registers).
__device__ inline int step_lanes(int rows, int cols, int nt, int cap) {
  int G = 4;
  while (G < 64 && 2 * G * cols <= nt) G <<= 1;
  while (G < 64 && rows > G * cap) G <<= 1;
  return G;
}

// Reflector j, v = (1, T(x_{j+1..} * scale)) with factor tj, applied to the
// trailing columns j+1.. of the panel a (m rows, column stride la) by groups
// of G lanes; the group that updates column j+1 also leaves the squared norm
// of its rows j+2.. in *sig_next.  With NU > 0 each lane holds
// NU = ceil((m - j) / G) rows of v and of the column in registers and the
// loops unroll without branches (rows of lanes before the last are full, the
// last loads through a clamped index and stores under a mask); NU = 0
// streams the rows.
template <class T, int NT, int NU>
__device__ __forceinline__ void qr_update(T* a, int64_t la, int m, int r, int j, const T* col, double scale,
                                          double tj, int G, double* sig_next) {
  const int groups = NT / G, gi = threadIdx.x / G, gl = threadIdx.x % G;
  if (NU == 0) {
    for (int c = j + 1 + gi; c < r; c += groups) {
      T* ac = a + c * la;
      if (tj != 0.0) {
        double w = 0.0;
        for (int i = j + gl; i < m; i += G) w += (i == j ? 1.0 : (double)T((double)col[i] * scale)) * (double)ac[i];
        w = gsum_dpp(w, G) * tj;
        for (int i = j + gl; i < m; i += G)
          ac[i] = T((double)ac[i] - w * (i == j ? 1.0 : (double)T((double)col[i] * scale)));
      }
      if (c == j + 1) {
        double sn = 0.0;
        for (int i = j + 2 + gl; i < m; i += G) {
          const double v = (double)ac[i];
          sn += v * v;
        }
        sn = gsum_dpp(sn, G);
        if (gl == 0) *sig_next = sn;
      }
    }
    return;
  }
  constexpr int R = NU > 0 ? NU : 1;
  const int il = j + gl + (R - 1) * G;
  const bool tail_ok = il < m;
  const int ic = tail_ok ? il : j;
  double v[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const double x = (double)(u + 1 < R ? col[j + gl + u * G] : col[ic]);
    const double vv = (u == 0 && gl == 0) ? 1.0 : (double)T(x * scale);
    v[u] = (u + 1 < R || tail_ok) ? vv : 0.0;
  }
  for (int c = j + 1 + gi; c < r; c += groups) {
    T* ac = a + c * la;
    double x[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const double y = (double)(u + 1 < R ? ac[j + gl + u * G] : ac[ic]);
      x[u] = (u + 1 < R || tail_ok) ? y : 0.0;
    }
    if (tj != 0.0) {
      double w = 0.0;
#pragma unroll
      for (int u = 0; u < R; ++u) w = fma(v[u], x[u], w);
      w = gsum_dpp(w, G) * tj;
#pragma unroll
      for (int u = 0; u < R; ++u) x[u] = (double)T(x[u] - w * v[u]);
#pragma unroll
      for (int u = 0; u + 1 < R; ++u) ac[j + gl + u * G] = T(x[u]);
      if (tail_ok) ac[il] = T(x[R - 1]);
    }
    if (c == j + 1) {
      double sn = 0.0;
#pragma unroll
      for (int u = 0; u < R; ++u) sn = (u == 0 && gl < 2) ? sn : fma(x[u], x[u], sn);
      sn = gsum_dpp(sn, G);
      if (gl == 0) *sig_next = sn;
    }
  }
}

// Reflector j (vj, factor tj) applied to the k columns of o (m rows, column
// stride lo), rows j..m-1; same register scheme as qr_update.
template <class T, int NT, int NU>
__device__ __forceinline__ void applyq_update(T* o, int64_t lo, int m, int k, int j, const T* vj, double tj,
                                              int G) {
  const int groups = NT / G, gi = threadIdx.x / G, gl = threadIdx.x % G;
  if (NU == 0) {
    for (int c = gi; c < k; c += groups) {
      T* oc = o + c * lo;
      double w = 0.0;
      for (int i = j + gl; i < m; i += G) w += (i == j ? 1.0 : (double)vj[i]) * (double)oc[i];
      w = gsum_dpp(w, G) * tj;
      for (int i = j + gl; i < m; i += G) oc[i] = T((double)oc[i] - w * (i == j ? 1.0 : (double)vj[i]));
    }
    return;
  }
  constexpr int R = NU > 0 ? NU : 1;
  const int il = j + gl + (R - 1) * G;
  const bool tail_ok = il < m;
  const int ic = tail_ok ? il : j;
  double v[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const double x = (double)(u + 1 < R ? vj[j + gl + u * G] : vj[ic]);
    const double vv = (u == 0 && gl == 0) ? 1.0 : x;
    v[u] = (u + 1 < R || tail_ok) ? vv : 0.0;
  }
  for (int c = gi; c < k; c += groups) {
    T* oc = o + c * lo;
    double x[R];
    double w = 0.0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const double y = (double)(u + 1 < R ? oc[j + gl + u * G] : oc[ic]);
      x[u] = (u + 1 < R || tail_ok) ? y : 0.0;
      w = fma(v[u], x[u], w);
    }
    w = gsum_dpp(w, G) * tj;
#pragma unroll
    for (int u = 0; u + 1 < R; ++u) oc[j + gl + u * G] = T(x[u] - w * v[u]);
    if (tail_ok) oc[il] = T(x[R - 1] - w * v[R - 1]);
  }
}

#define ACR_NU_CASES(M) M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16)

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
    staged_copy<NT>(
        (int64_t)m * r, [&](int64_t e) { return A[(int)e % m + (int64_t)((int)e / m) * t.lda]; },
        [&](int64_t e, T v) { a[e] = v; });
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
    // the trailing columns on the fly
    constexpr int kCap = LDS ? 16 : 8;
    const int G = step_lanes(m - j, r - j - 1, NT, kCap);
    double* sn = &sh_sig[j & 1];
    const int nu = (m - j + G - 1) / G;
    switch (nu <= kCap ? nu : 0) {
#define ACR_QR_CASE(k) \
  case k: qr_update<T, NT, (k <= kCap ? k : 0)>(a, la, m, r, j, col, scale, tj, G, sn); break;
      ACR_NU_CASES(ACR_QR_CASE)
#undef ACR_QR_CASE
      default: qr_update<T, NT, 0>(a, la, m, r, j, col, scale, tj, G, sn); break;
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
    staged_copy<NT>(
        (int64_t)m * p, [&](int64_t e) { return Aq[(int)e % m + (int64_t)((int)e / m) * t.lda]; },
        [&](int64_t e, T x) { reinterpret_cast<T*>(sma)[e] = x; });
  staged_copy<NT>(
      (int64_t)m * k,
      [&](int64_t e) {
        const int i = (int)e % m, c = (int)e / m;
        return i < p ? T(t.Z[i + (int64_t)c * t.ldz]) : T(0);
      },
      [&](int64_t e, T x) { o[(int)e % m + ((int)e / m) * lo] = x; });
  __syncthreads();
  for (int j = p - 1; j >= 0; --j) {
    const double tj = (double)tau[j];
    if (tj == 0.0) continue;
    const T* vj = v + j * lv;
    constexpr int kCap = LDS ? 16 : 8;
    const int G = step_lanes(m - j, k, NT, kCap);
    const int nu = (m - j + G - 1) / G;
    switch (nu <= kCap ? nu : 0) {
#define ACR_AQ_CASE(kk) \
  case kk: applyq_update<T, NT, (kk <= kCap ? kk : 0)>(o, lo, m, k, j, vj, tj, G); break;
      ACR_NU_CASES(ACR_AQ_CASE)
#undef ACR_AQ_CASE
      default: applyq_update<T, NT, 0>(o, lo, m, k, j, vj, tj, G); break;
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
