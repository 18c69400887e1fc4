// Batched dense linear-algebra kernels for the hierarchical block operations.
//
// One launch processes a list of independent small problems (all blocks of one
// hierarchical depth over all planes of a cyclic-reduction level).  Kernels:
//   k_gemm     tiled C = alpha op(A) op(B) + beta C over a tile map
//   k_copy     scaled copies / accumulations of sub-matrices (stack assembly)
//   k_inverse  Gauss-Jordan inverse with partial pivoting (dense leaves,
//              the small capacitance matrices of the HODLR inverse)
//   k_qr       Householder QR of tall panels (stacked low-rank bases)
//   k_svd      one-sided Jacobi SVD in FP64 of the core R_u R_v^T, ordering,
//              and truncation at a relative tolerance
//   k_applyq   reconstruction Q [Z; 0] of the truncated bases
// Compression by SVD of low-rank sums follows Section 2.1 of the paper; the
// QR + Jacobi organisation is this library's choice.
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

// Householder QR (LAPACK sign convention: beta = -sign(x0) ||x||,
// tau = (beta - x0) / beta, v = x / (x0 - beta) below the diagonal).
template <class T>
__global__ __launch_bounds__(256) void k_qr(const QrTask* __restrict__ tasks) {
  const QrTask t = tasks[blockIdx.x];
  T* A = static_cast<T*>(t.A);
  T* tau = static_cast<T*>(t.tau);
  const int m = t.m, r = t.r;
  const int64_t ld = t.lda;
  const int nref = m < r ? m : r;
  __shared__ double red[4];
  __shared__ double sh_tau, sh_scale, sh_beta;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < nref; ++j) {
    T* col = A + (int64_t)j * ld;
    double ps = 0.0;
    for (int i = j + 1 + threadIdx.x; i < m; i += 256) {
      const double v = (double)col[i];
      ps += v * v;
    }
    const double sigma = block_sum(ps, red);
    if (threadIdx.x == 0) {
      const double x0 = (double)col[j];
      if (sigma == 0.0) {
        sh_tau = 0.0;
        sh_beta = x0;
        sh_scale = 0.0;
      } else {
        const double nrm = sqrt(x0 * x0 + sigma);
        const double beta = x0 >= 0.0 ? -nrm : nrm;
        sh_tau = (beta - x0) / beta;
        sh_scale = 1.0 / (x0 - beta);
        sh_beta = beta;
      }
      tau[j] = T(sh_tau);
    }
    __syncthreads();
    const double tj = sh_tau;
    if (tj != 0.0) {
      const T sc = T(sh_scale);
      for (int i = j + 1 + threadIdx.x; i < m; i += 256) col[i] *= sc;
    }
    if (threadIdx.x == 0) col[j] = T(sh_beta);
    __syncthreads();
    if (tj != 0.0) {
      for (int c = j + 1 + wave; c < r; c += 4) {
        T* ac = A + (int64_t)c * ld;
        double w = 0.0;
        for (int i = j + lane; i < m; i += 64) {
          const double vi = (i == j) ? 1.0 : (double)col[i];
          w += vi * (double)ac[i];
        }
        w = wave_sum(w) * tj;
        for (int i = j + lane; i < m; i += 64) {
          const double vi = (i == j) ? 1.0 : (double)col[i];
          ac[i] = T((double)ac[i] - w * vi);
        }
      }
    }
    __syncthreads();
  }
}

// One-sided Jacobi SVD of C = Ru Rv^T followed by ordering and truncation.
template <class T>
__global__ __launch_bounds__(256) void k_svd(const SvdTask* __restrict__ tasks, double eps, int* flags) {
  const SvdTask t = tasks[blockIdx.x];
  const int p = t.p, q = t.q, r = t.r;
  const T* Ru = static_cast<const T*>(t.Ru);
  const T* Rv = static_cast<const T*>(t.Rv);
  double* C = t.C;
  double* Y = t.Y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ double red[4];
  __shared__ int sh_rot;
  __shared__ double sh_smax;
  if (p == 0 || q == 0) {
    if (threadIdx.x == 0) *t.rank_out = 0;
    return;
  }
  for (int64_t e = threadIdx.x; e < (int64_t)p * q; e += 256) {
    const int a = (int)(e % p), b = (int)(e / p);
    double acc = 0.0;
    for (int l = (a > b ? a : b); l < r; ++l)
      acc += (double)Ru[a + (int64_t)l * t.ldu] * (double)Rv[b + (int64_t)l * t.ldv];
    C[a + (int64_t)b * p] = acc;
  }
  for (int64_t e = threadIdx.x; e < (int64_t)q * q; e += 256) Y[e] = (e % q == e / q) ? 1.0 : 0.0;
  __syncthreads();
  const double tol = fmax(1e-15, 2.3e-16 * (double)p);
  const int qe = q + (q & 1);
  for (int sweep = 0; sweep < 60 && q > 1; ++sweep) {
    if (threadIdx.x == 0) sh_rot = 0;
    __syncthreads();
    for (int round = 0; round < qe - 1; ++round) {
      for (int pi = wave; pi < qe / 2; pi += 4) {
        const int pa = pi, pb = qe - 1 - pi;
        int ia = pa == 0 ? 0 : ((pa - 1 + round) % (qe - 1)) + 1;
        int ib = pb == 0 ? 0 : ((pb - 1 + round) % (qe - 1)) + 1;
        if (ia >= q || ib >= q) continue;
        if (ia > ib) { const int tmp = ia; ia = ib; ib = tmp; }
        double* ca = C + (int64_t)ia * p;
        double* cb = C + (int64_t)ib * p;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < p; i += 64) {
          const double x = ca[i], y = cb[i];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (ga == 0.0 || !(fabs(ga) > tol * sqrt(al * be))) continue;
        const double zeta = (be - al) / (2.0 * ga);
        double tt;
        if (fabs(zeta) > 1e150) tt = 0.5 / zeta;
        else tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
        for (int i = lane; i < p; i += 64) {
          const double x = ca[i], y = cb[i];
          ca[i] = cs * x - sn * y;
          cb[i] = sn * x + cs * y;
        }
        double* ya = Y + (int64_t)ia * q;
        double* yb = Y + (int64_t)ib * q;
        for (int i = lane; i < q; i += 64) {
          const double x = ya[i], y = yb[i];
          ya[i] = cs * x - sn * y;
          yb[i] = sn * x + cs * y;
        }
        if (lane == 0) sh_rot = 1;
      }
      __syncthreads();
    }
    const int rot = sh_rot;
    __syncthreads();
    if (!rot) break;
  }
  double* sig = t.sig;
  for (int i = wave; i < q; i += 4) {
    const double* ci = C + (int64_t)i * p;
    double ss = 0.0;
    for (int l = lane; l < p; l += 64) ss += ci[l] * ci[l];
    ss = wave_sum(ss);
    if (lane == 0) sig[i] = sqrt(ss);
  }
  __syncthreads();
  double mx = 0.0;
  for (int i = threadIdx.x; i < q; i += 256) mx = fmax(mx, sig[i]);
  // max reduction through the shared slots
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if (lane == 0) red[wave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) sh_smax = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  const double smax = sh_smax;
  const double thr = eps > 0.0 ? eps * smax : 0.0;
  int cnt = 0;
  for (int i = threadIdx.x; i < q; i += 256) cnt += (smax > 0.0 && sig[i] > thr) ? 1 : 0;
  const int k_all = (int)block_sum((double)cnt, red);
  int k = k_all;
  if (t.max_rank > 0 && k > t.max_rank) {
    if (threadIdx.x == 0) atomicOr(&flags[FLAG_RANK], 1);
    k = t.max_rank;
  }
  // place column i at its rank position (descending sigma, ties by index)
  double* Zu = C + (int64_t)p * q;   // caller sizes C as p*q + p*q
  double* Zv = Y + (int64_t)q * q;   // and Y as q*q + q*q
  for (int i = wave; i < q; i += 4) {
    const double si = sig[i];
    int pos = 0;
    for (int j = lane; j < q; j += 64) {
      const double sj = sig[j];
      pos += (sj > si || (sj == si && j < i)) ? 1 : 0;
    }
    pos = (int)wave_sum((double)pos);
    if (pos < k) {
      for (int l = lane; l < p; l += 64) Zu[l + (int64_t)pos * p] = C[l + (int64_t)i * p];
      for (int l = lane; l < q; l += 64) Zv[l + (int64_t)pos * q] = Y[l + (int64_t)i * q];
    }
  }
  if (threadIdx.x == 0) *t.rank_out = k;
}

template <class T>
__global__ __launch_bounds__(256) void k_applyq(const ApplyQTask* __restrict__ tasks) {
  const ApplyQTask t = tasks[blockIdx.x];
  const int m = t.m, p = t.p, k = t.k;
  if (k == 0 || m == 0) return;
  const T* Aq = static_cast<const T*>(t.Aq);
  const T* tau = static_cast<const T*>(t.tau);
  T* out = static_cast<T*>(t.out);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t e = threadIdx.x; e < (int64_t)m * k; e += 256) {
    const int i = (int)(e % m), c = (int)(e / m);
    out[i + (int64_t)c * t.ldo] = i < p ? T(t.Z[i + (int64_t)c * t.ldz]) : T(0);
  }
  __syncthreads();
  for (int j = p - 1; j >= 0; --j) {
    const double tj = (double)tau[j];
    if (tj == 0.0) continue;
    const T* v = Aq + (int64_t)j * t.lda;
    for (int c = wave; c < k; c += 4) {
      T* oc = out + (int64_t)c * t.ldo;
      double w = 0.0;
      for (int i = j + lane; i < m; i += 64) w += (i == j ? 1.0 : (double)v[i]) * (double)oc[i];
      w = wave_sum(w) * tj;
      for (int i = j + lane; i < m; i += 64) oc[i] = T((double)oc[i] - w * (i == j ? 1.0 : (double)v[i]));
    }
    __syncthreads();
  }
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

template <class T>
void launch_qr(const QrTask* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_qr<T>, dim3(ntasks), dim3(256), 0, s, d_tasks);
}

template <class T>
void launch_svd(const SvdTask* d_tasks, int ntasks, double eps, int* d_flags, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_svd<T>, dim3(ntasks), dim3(256), 0, s, d_tasks, eps, d_flags);
}

template <class T>
void launch_applyq(const ApplyQTask* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_applyq<T>, dim3(ntasks), dim3(256), 0, s, d_tasks);
}

#define ACR_INST(T)                                                                              \
  template void launch_gemm<T>(const GemmTask*, const int*, const int*, int, hipStream_t);      \
  template void launch_copy<T>(const CopyTask*, int, hipStream_t);                              \
  template void launch_inverse<T>(const InvTask*, int, int, int*, hipStream_t);                 \
  template void launch_qr<T>(const QrTask*, int, hipStream_t);                                  \
  template void launch_svd<T>(const SvdTask*, int, double, int*, hipStream_t);                  \
  template void launch_applyq<T>(const ApplyQTask*, int, hipStream_t);
ACR_INST(float)
ACR_INST(double)
#undef ACR_INST

}  // namespace acr
