// Truncated SVD of the compression core C = Ru Rv^T (FP64).
//
// Stage 1 (k_qrcp): Householder QR with column pivoting of C, stopped when the
// largest remaining column norm drops below delta times the largest initial
// one; C P ~= Q [R11 R12].  Stage 2 (k_jacobi): one-sided Jacobi on the
// columns of W^T = P [R11 R12]^T (q x t), whose singular values are those of C
// up to the dropped tail.  QR with column pivoting both removes the directions
// far below the truncation level and preconditions the Jacobi iteration, which
// then converges in a few sweeps.  The right singular vectors are the
// normalised rotated columns; the left factor is recomputed as C Zv = U Sigma.
#include <cmath>

#include "kern.h"

namespace acr {

namespace {

__device__ inline double gsum2(double v, int G) {
  for (int off = G >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

__device__ inline int lanes_for(int m) {
  int G = 4;
  while (G < 64 && G * 4 < m) G <<= 1;
  return G;
}

template <class T>
__device__ inline double core_entry(const SvdTask& t, int a, int b) {
  double acc = 0.0;
  if (t.mode == 0) {
    const T* Ru = static_cast<const T*>(t.Ru);
    const T* Rv = static_cast<const T*>(t.Rv);
    for (int l = (a > b ? a : b); l < t.r; ++l)
      acc += (double)Ru[a + (int64_t)l * t.ldu] * (double)Rv[b + (int64_t)l * t.ldv];
  } else {
    const double* Ru = static_cast<const double*>(t.Ru);
    const double* Rv = static_cast<const double*>(t.Rv);
    for (int l = 0; l < t.r; ++l) acc += Ru[a + (int64_t)l * t.ldu] * Rv[b + (int64_t)l * t.ldv];
  }
  return acc;
}

template <class T, bool LDS>
__global__ __launch_bounds__(256) void k_qrcp(const SvdTask* __restrict__ tasks, double delta) {
  extern __shared__ double smc[];
  const SvdTask t = tasks[blockIdx.x];
  const int p = t.p, q = t.q;
  const int mn = p < q ? p : q;
  if (p == 0 || q == 0) {
    if (threadIdx.x == 0) *t.t_out = 0;
    return;
  }
  double* C = LDS ? smc : t.C;
  double* nrm = LDS ? smc + (int64_t)p * q : t.sig;
  int* perm = LDS ? reinterpret_cast<int*>(nrm + q) : t.perm;
  __shared__ double rv[256];
  __shared__ int ri[256];
  __shared__ double sh_tau, sh_scale, sh_beta;
  __shared__ int sh_stop;
  for (int64_t e = threadIdx.x; e < (int64_t)p * q; e += 256) C[e] = core_entry<T>(t, (int)(e % p), (int)(e / p));
  __syncthreads();
  const int G = lanes_for(p), groups = 256 / G;
  const int gi = threadIdx.x / G, gl = threadIdx.x % G;
  for (int c = gi; c < q; c += groups) {
    double s = 0.0;
    for (int i = gl; i < p; i += G) s += C[i + (int64_t)c * p] * C[i + (int64_t)c * p];
    s = gsum2(s, G);
    if (gl == 0) { nrm[c] = s; perm[c] = c; }
  }
  __syncthreads();
  double mx = 0.0;
  for (int c = threadIdx.x; c < q; c += 256) mx = fmax(mx, nrm[c]);
  rv[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) rv[threadIdx.x] = fmax(rv[threadIdx.x], rv[threadIdx.x + w]);
    __syncthreads();
  }
  // dropped tail: Frobenius norm <= sqrt(q) * sqrt(thr2) = delta * (largest column norm)
  const double thr2 = delta * delta * rv[0] / (double)q;
  __syncthreads();
  int tcount = 0;
  for (int j = 0; j < mn; ++j) {
    double best = -1.0;
    int bc = j;
    for (int c = j + threadIdx.x; c < q; c += 256)
      if (nrm[c] > best) { best = nrm[c]; bc = c; }
    rv[threadIdx.x] = best;
    ri[threadIdx.x] = bc;
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
    const int pc = ri[0];
    if (threadIdx.x == 0) sh_stop = !(rv[0] > thr2) || !(rv[0] > 0.0);
    __syncthreads();
    if (sh_stop) break;
    if (pc != j) {
      for (int i = threadIdx.x; i < p; i += 256) {
        const double a = C[i + (int64_t)j * p];
        C[i + (int64_t)j * p] = C[i + (int64_t)pc * p];
        C[i + (int64_t)pc * p] = a;
      }
      if (threadIdx.x == 0) {
        const double a = nrm[j];
        nrm[j] = nrm[pc];
        nrm[pc] = a;
        const int b = perm[j];
        perm[j] = perm[pc];
        perm[pc] = b;
      }
    }
    __syncthreads();
    double* col = C + (int64_t)j * p;
    double ps = 0.0;
    for (int i = j + 1 + threadIdx.x; i < p; i += 256) ps += col[i] * col[i];
    rv[threadIdx.x] = ps;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) rv[threadIdx.x] += rv[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double sigma = rv[0], x0 = col[j];
      if (sigma == 0.0) {
        sh_tau = 0.0;
        sh_scale = 0.0;
        sh_beta = x0;
      } else {
        const double nr = sqrt(x0 * x0 + sigma);
        const double beta = x0 >= 0.0 ? -nr : nr;
        sh_tau = (beta - x0) / beta;
        sh_scale = 1.0 / (x0 - beta);
        sh_beta = beta;
      }
    }
    __syncthreads();
    const double tj = sh_tau;
    if (tj != 0.0)
      for (int i = j + 1 + threadIdx.x; i < p; i += 256) col[i] *= sh_scale;
    __syncthreads();
    if (threadIdx.x == 0) col[j] = sh_beta;
    for (int c = j + 1 + gi; c < q; c += groups) {
      double* ac = C + (int64_t)c * p;
      if (tj != 0.0) {
        double w = 0.0;
        for (int i = j + gl; i < p; i += G) w += (i == j ? 1.0 : col[i]) * ac[i];
        w = gsum2(w, G) * tj;
        for (int i = j + gl; i < p; i += G) ac[i] -= w * (i == j ? 1.0 : col[i]);
      }
      double s = 0.0;
      for (int i = j + 1 + gl; i < p; i += G) s += ac[i] * ac[i];
      s = gsum2(s, G);
      if (gl == 0) nrm[c] = s;
    }
    __syncthreads();
    tcount = j + 1;
  }
  // W^T (q x tcount), rows in the original column order of C
  double* Wt = t.Y;
  for (int64_t e = threadIdx.x; e < (int64_t)q * tcount; e += 256) {
    const int c = (int)(e % q), a = (int)(e / q);
    Wt[perm[c] + (int64_t)a * q] = c >= a ? C[a + (int64_t)c * p] : 0.0;
  }
  if (threadIdx.x == 0) *t.t_out = tcount;
}

template <class T, bool LDS>
__global__ __launch_bounds__(256) void k_jacobi(const SvdTask* __restrict__ tasks, double eps, int* flags) {
  extern __shared__ double smj[];
  const SvdTask t = tasks[blockIdx.x];
  const int rows = t.q;
  const int n = *t.t_out;
  if (n == 0 || rows == 0) {
    if (threadIdx.x == 0) *t.rank_out = 0;
    return;
  }
  double* A = LDS ? smj : t.Y;
  double* sig = t.sig;
  __shared__ double red[4];
  __shared__ int sh_rot;
  if (LDS)
    for (int64_t e = threadIdx.x; e < (int64_t)rows * n; e += 256) A[e] = t.Y[e];
  __syncthreads();
  const int ne = n + (n & 1), npairs = ne / 2;
  int G = 64;
  while (G > 1 && G * npairs > 256) G >>= 1;
  if (!LDS && G < 16) G = 16;
  while (G > 1 && G > 2 * rows) G >>= 1;
  const int groups = 256 / G;
  const int gi = threadIdx.x / G, gl = threadIdx.x % G;
  const double tol = fmax(1e-15, 2.3e-16 * (double)rows);
  int sweeps = 0;
  for (int sweep = 0; sweep < 60 && n > 1; ++sweep) {
    if (threadIdx.x == 0) sh_rot = 0;
    __syncthreads();
    ++sweeps;
    for (int round = 0; round < ne - 1; ++round) {
      for (int pi = gi; pi < npairs; pi += groups) {
        const int pa = pi, pb = ne - 1 - pi;
        int ia = pa == 0 ? 0 : ((pa - 1 + round) % (ne - 1)) + 1;
        int ib = pb == 0 ? 0 : ((pb - 1 + round) % (ne - 1)) + 1;
        if (ia >= n || ib >= n) continue;
        if (ia > ib) { const int tmp = ia; ia = ib; ib = tmp; }
        double* ca = A + (int64_t)ia * rows;
        double* cb = A + (int64_t)ib * rows;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = gl; i < rows; i += G) {
          const double x = ca[i], y = cb[i];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        al = gsum2(al, G);
        be = gsum2(be, G);
        ga = gsum2(ga, G);
        if (ga == 0.0 || !(fabs(ga) > tol * sqrt(al * be))) continue;
        const double zeta = (be - al) / (2.0 * ga);
        double tt;
        if (fabs(zeta) > 1e150) tt = 0.5 / zeta;
        else tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
        for (int i = gl; i < rows; i += G) {
          const double x = ca[i], y = cb[i];
          ca[i] = cs * x - sn * y;
          cb[i] = sn * x + cs * y;
        }
        if (gl == 0) sh_rot = 1;
      }
      __syncthreads();
    }
    const int rot = sh_rot;
    __syncthreads();
    if (!rot) break;
  }
  for (int i = gi; i < n; i += groups) {
    const double* ci = A + (int64_t)i * rows;
    double ss = 0.0;
    for (int l = gl; l < rows; l += G) ss += ci[l] * ci[l];
    ss = gsum2(ss, G);
    if (gl == 0) sig[i] = sqrt(ss);
  }
  __syncthreads();
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) mx = fmax(mx, sig[i]);
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  __shared__ double sh_mx[4];
  if ((threadIdx.x & 63) == 0) sh_mx[threadIdx.x >> 6] = mx;
  __syncthreads();
  const double smax = fmax(fmax(sh_mx[0], sh_mx[1]), fmax(sh_mx[2], sh_mx[3]));
  const double thr = eps > 0.0 ? eps * smax : 0.0;
  int cnt = 0;
  for (int i = threadIdx.x; i < n; i += 256) cnt += (smax > 0.0 && sig[i] > thr) ? 1 : 0;
  double cs_ = (double)cnt;
  for (int off = 32; off > 0; off >>= 1) cs_ += __shfl_xor(cs_, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cs_;
  __syncthreads();
  int k = (int)(red[0] + red[1] + red[2] + red[3]);
  if (t.max_rank > 0 && k > t.max_rank) {
    if (threadIdx.x == 0) atomicOr(&flags[FLAG_RANK], 1);
    k = t.max_rank;
  }
  // right vectors: normalised rotated columns, ordered by decreasing sigma
  const int q = t.q, p = t.p;
  double* Zv = t.Y + (int64_t)q * q;
  for (int i = gi; i < n; i += groups) {
    const double si = sig[i];
    double pos = 0.0;
    for (int j = gl; j < n; j += G) {
      const double sj = sig[j];
      pos += (sj > si || (sj == si && j < i)) ? 1.0 : 0.0;
    }
    const int ps = (int)gsum2(pos, G);
    if (ps < k) {
      const double inv = 1.0 / si;
      for (int l = gl; l < rows; l += G) Zv[l + (int64_t)ps * q] = A[l + (int64_t)i * rows] * inv;
    }
  }
  __syncthreads();
  // left factor: Zu = C Zv = Ru (Rv^T Zv)
  double* Zu = t.C + (int64_t)p * q;
  double* tmp = t.tmp;
  for (int c = 0; c < k; ++c) {
    const double* zv = Zv + (int64_t)c * q;
    for (int l = threadIdx.x; l < t.r; l += 256) {
      double s = 0.0;
      if (t.mode == 0) {
        const T* Rv = static_cast<const T*>(t.Rv);
        const int bmax = l < q - 1 ? l : q - 1;
        for (int b = 0; b <= bmax; ++b) s += (double)Rv[b + (int64_t)l * t.ldv] * zv[b];
      } else {
        const double* Rv = static_cast<const double*>(t.Rv);
        for (int b = 0; b < q; ++b) s += Rv[b + (int64_t)l * t.ldv] * zv[b];
      }
      tmp[l] = s;
    }
    __syncthreads();
    for (int a = threadIdx.x; a < p; a += 256) {
      double s = 0.0;
      if (t.mode == 0) {
        const T* Ru = static_cast<const T*>(t.Ru);
        for (int l = a; l < t.r; ++l) s += (double)Ru[a + (int64_t)l * t.ldu] * tmp[l];
      } else {
        const double* Ru = static_cast<const double*>(t.Ru);
        for (int l = 0; l < t.r; ++l) s += Ru[a + (int64_t)l * t.ldu] * tmp[l];
      }
      Zu[a + (int64_t)c * p] = s;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *t.rank_out = k;
    if (t.sweep_ctr)
      atomicAdd(t.sweep_ctr, (unsigned long long)sweeps * (unsigned long long)(n * (n - 1) / 2) * (unsigned long long)rows);
  }
}

template <class K> void allow(K kernel, size_t bytes) {
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

}  // namespace

template <class T>
void launch_qrcp(const SvdTask* d_tasks, int ntasks, double delta, size_t lds, hipStream_t s) {
  if (ntasks <= 0) return;
  if (lds == 0) {
    hipLaunchKernelGGL((k_qrcp<T, false>), dim3(ntasks), dim3(256), 0, s, d_tasks, delta);
    return;
  }
  allow(k_qrcp<T, true>, lds);
  hipLaunchKernelGGL((k_qrcp<T, true>), dim3(ntasks), dim3(256), lds, s, d_tasks, delta);
}

template <class T>
void launch_jacobi(const SvdTask* d_tasks, int ntasks, double eps, int* d_flags, size_t lds, hipStream_t s) {
  if (ntasks <= 0) return;
  if (lds == 0) {
    hipLaunchKernelGGL((k_jacobi<T, false>), dim3(ntasks), dim3(256), 0, s, d_tasks, eps, d_flags);
    return;
  }
  allow(k_jacobi<T, true>, lds);
  hipLaunchKernelGGL((k_jacobi<T, true>), dim3(ntasks), dim3(256), lds, s, d_tasks, eps, d_flags);
}

template void launch_qrcp<float>(const SvdTask*, int, double, size_t, hipStream_t);
template void launch_qrcp<double>(const SvdTask*, int, double, size_t, hipStream_t);
template void launch_jacobi<float>(const SvdTask*, int, double, int*, size_t, hipStream_t);
template void launch_jacobi<double>(const SvdTask*, int, double, int*, size_t, hipStream_t);

}  // namespace acr
