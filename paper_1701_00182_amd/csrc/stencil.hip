// Stencil-side kernels (see stencil.h).
#include <cmath>

#include "kern.h"
#include "stencil.h"

namespace acr {

namespace {

__device__ inline void grid_ijk(const Grid& g, int64_t r, int& i, int& j, int& k) {
  const int64_t M = g.M();
  k = (int)(r / M);
  const int64_t rem = r - (int64_t)k * M;
  j = (int)(rem / g.nx);
  i = (int)(rem - (int64_t)j * g.nx);
}

__global__ void k_validate(Grid g, const double* __restrict__ coef, int* flags) {
  const int64_t N = g.N();
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k;
    grid_ijk(g, r, i, j, k);
    const bool outside[7] = {false, i == 0, i == g.nx - 1, j == 0, j == g.ny - 1, k == 0, k == g.nz - 1};
    bool nonfinite = false, invalid = false;
    for (int s = 0; s < 7; ++s) {
      const double v = coef[s * N + r];
      if (!isfinite(v)) nonfinite = true;
      if (outside[s] && v != 0.0) invalid = true;
    }
    if (nonfinite) atomicOr(&flags[FLAG_NONFINITE], 1);
    if (invalid) atomicOr(&flags[FLAG_INVALID], 1);
  }
}

// 27-point validation: entries reaching outside the grid must be zero
__global__ void k_validate27(Grid g, const double* __restrict__ coef, int* flags) {
  const int64_t N = g.N();
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k;
    grid_ijk(g, r, i, j, k);
    bool nonfinite = false, invalid = false;
    for (int s = 0; s < 27; ++s) {
      const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
      const bool out = i + dx < 0 || i + dx >= g.nx || j + dy < 0 || j + dy >= g.ny || k + dz < 0 || k + dz >= g.nz;
      const double v = coef[s * N + r];
      if (!isfinite(v)) nonfinite = true;
      if (out && v != 0.0) invalid = true;
    }
    if (nonfinite) atomicOr(&flags[FLAG_NONFINITE], 1);
    if (invalid) atomicOr(&flags[FLAG_INVALID], 1);
  }
}

template <class T>
__global__ void k_conv_leaves(Grid g, const double* __restrict__ coef, const LeafEnt* __restrict__ ents, int nent,
                              T* const* __restrict__ leafptr, int nleaf) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (e >= nent) return;
  const LeafEnt en = ents[e];
  T* lp = leafptr[(int64_t)k * nleaf + en.leaf];
  if (!lp) return;   // absent block of this plane
  const double v = coef[en.slot * g.N() + (int64_t)k * g.M() + en.nat];
  lp[en.a + (int64_t)en.b * en.n] = T(v);
}

template <class T>
__global__ void k_cut9_fill(Grid g, const double* __restrict__ coef, const Cut9Ent* __restrict__ ents, int nent,
                            int nblk, T* const* __restrict__ uptr, T* const* __restrict__ vptr,
                            const int* __restrict__ rows, const int* __restrict__ cols) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (e >= nent) return;
  const Cut9Ent en = ents[e];
  T* U = uptr[(int64_t)k * nblk + en.blk];
  T* V = vptr[(int64_t)k * nblk + en.blk];
  if (!U || !V) return;
  // entries sharing a column select the same row: equal writes
  U[en.r + (int64_t)en.j * rows[en.blk]] = T(1);
  V[en.c + (int64_t)en.j * cols[en.blk]] = T(coef[en.slot * g.N() + (int64_t)k * g.M() + en.nat]);
}

__global__ void k_cut_rank(Grid g, const double* __restrict__ coef, const CutEnt* __restrict__ ents,
                           const int* __restrict__ first, int nblk, double eps, int* ranks) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (b >= nblk) return;
  const int64_t base = (int64_t)k * g.M();
  double mx = 0.0;
  for (int e = first[b]; e < first[b + 1]; ++e) mx = fmax(mx, fabs(coef[ents[e].slot * g.N() + base + ents[e].nat]));
  int cnt = 0;
  if (mx > 0.0) {
    const double thr = eps * mx;
    for (int e = first[b]; e < first[b + 1]; ++e)
      cnt += fabs(coef[ents[e].slot * g.N() + base + ents[e].nat]) > thr ? 1 : 0;
  }
  ranks[(int64_t)k * nblk + b] = cnt;
}

template <class T>
__global__ void k_cut_fill(Grid g, const double* __restrict__ coef, const CutEnt* __restrict__ ents,
                           const int* __restrict__ first, int nblk, double eps, T* const* uptr, T* const* vptr,
                           const int* __restrict__ rows, const int* __restrict__ cols) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (b >= nblk) return;
  const int64_t base = (int64_t)k * g.M();
  double mx = 0.0;
  for (int e = first[b]; e < first[b + 1]; ++e) mx = fmax(mx, fabs(coef[ents[e].slot * g.N() + base + ents[e].nat]));
  if (mx == 0.0) return;
  const double thr = eps * mx;
  T* U = uptr[(int64_t)k * nblk + b];
  T* V = vptr[(int64_t)k * nblk + b];
  int col = 0;
  for (int e = first[b]; e < first[b + 1]; ++e) {
    const CutEnt en = ents[e];
    const double v = coef[en.slot * g.N() + base + en.nat];
    if (fabs(v) > thr) {
      U[en.r + (int64_t)col * rows[b]] = T(v);
      V[en.c + (int64_t)col * cols[b]] = T(1);
      ++col;
    }
  }
}

template <class T>
__global__ void k_diag(Grid g, const double* __restrict__ coef, int slot, const int* __restrict__ perm, T* out) {
  const int64_t N = g.N(), M = g.M();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / M, pos = e - k * M;
    out[e] = T(coef[slot * N + k * M + perm[pos]]);
  }
}

template <class T>
__global__ void k_perm_in(Grid g, int nrhs, const double* __restrict__ b, int64_t ldb, const int* __restrict__ perm,
                          T* W) {
  const int64_t N = g.N(), M = g.M();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N * nrhs; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / N, rr = e - c * N, k = rr / M, pos = rr - k * M;
    W[(k * nrhs + c) * M + pos] = T(b[k * M + perm[pos] + c * ldb]);
  }
}

template <class T>
__global__ void k_perm_out(Grid g, int nrhs, const T* __restrict__ W, const int* __restrict__ perm, double* x,
                           int64_t ldx) {
  const int64_t N = g.N(), M = g.M();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N * nrhs; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / N, rr = e - c * N, k = rr / M, pos = rr - k * M;
    x[k * M + perm[pos] + c * ldx] = (double)W[(k * nrhs + c) * M + pos];
  }
}

__global__ void k_residual(Grid g, const double* __restrict__ coef, const double* __restrict__ x,
                           const double* __restrict__ b, double* r, int transpose) {
  const int64_t N = g.N(), M = g.M();
  const int64_t off[7] = {0, -1, 1, -(int64_t)g.nx, (int64_t)g.nx, -M, M};
  // slot read at the neighbour for the transposed operator
  const int tslot[7] = {0, 2, 1, 4, 3, 6, 5};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k;
    grid_ijk(g, e, i, j, k);
    const bool in[7] = {true, i > 0, i < g.nx - 1, j > 0, j < g.ny - 1, k > 0, k < g.nz - 1};
    double acc = coef[e] * x[e];
    for (int s = 1; s < 7; ++s) {
      if (!in[s]) continue;
      const int64_t nb = e + off[s];
      const double a = transpose ? coef[tslot[s] * N + nb] : coef[s * N + e];
      acc += a * x[nb];
    }
    r[e] = b[e] - acc;
  }
}

// r = b - A x for a 27-point stencil; the transpose reads, for the neighbour
// q = r + o(s), the slot of q whose offset points back to r (26 - s)
__global__ void k_residual27(Grid g, const double* __restrict__ coef, const double* __restrict__ x,
                             const double* __restrict__ b, double* r, int transpose) {
  const int64_t N = g.N(), M = g.M();
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k;
    grid_ijk(g, e, i, j, k);
    double acc = 0.0;
    for (int s = 0; s < 27; ++s) {
      const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
      if (i + dx < 0 || i + dx >= g.nx || j + dy < 0 || j + dy >= g.ny || k + dz < 0 || k + dz >= g.nz) continue;
      const int64_t nb = e + dx + (int64_t)dy * g.nx + (int64_t)dz * M;
      const double a = transpose ? coef[(26 - s) * N + nb] : coef[s * N + e];
      acc += a * x[nb];
    }
    r[e] = b[e] - acc;
  }
}

__global__ void k_multidot(int64_t n, int nvec, const double* __restrict__ X, int64_t ldx,
                           const double* __restrict__ y, double* part) {
  __shared__ double red[256];
  const int i = blockIdx.y;
  const double* xi = X + (int64_t)i * ldx;
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) acc += xi[e] * y[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)i * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_reduce_parts(const double* __restrict__ part, int nblocks, double* out) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) acc += part[(int64_t)i * nblocks + b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

__global__ void k_gemv_sub(int64_t n, int nvec, const double* __restrict__ X, int64_t ldx,
                           const double* __restrict__ h, double* y) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < nvec; ++i) acc += X[(int64_t)i * ldx + e] * h[i];
    y[e] -= acc;
  }
}

__global__ void k_axpby(int64_t n, double alpha, const double* __restrict__ x, double beta, double* y) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = alpha * x[e] + (beta == 0.0 ? 0.0 : beta * y[e]);
}

__global__ void k_scale_copy(int64_t n, const double* __restrict__ x, const double* alpha_dev, int invert,
                             double* y) {
  const double a = invert ? 1.0 / *alpha_dev : *alpha_dev;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = a * x[e];
}

__global__ void k_assemble(Grid g, const double* __restrict__ kappa, double* coef) {
  const int64_t N = g.N(), M = g.M();
  const int64_t off[7] = {0, -1, 1, -(int64_t)g.nx, (int64_t)g.nx, -M, M};
  const double h[3] = {1.0 / (g.nx + 1), 1.0 / (g.ny + 1), 1.0 / (g.nz + 1)};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k;
    grid_ijk(g, e, i, j, k);
    const bool in[7] = {true, i > 0, i < g.nx - 1, j > 0, j < g.ny - 1, k > 0, k < g.nz - 1};
    const double kr = kappa[e];
    double c = 0.0;
    for (int s = 1; s < 7; ++s) {
      const double ih2 = 1.0 / (h[(s - 1) / 2] * h[(s - 1) / 2]);
      if (in[s]) {
        const double ks = kappa[e + off[s]];
        const double kf = 2.0 * kr * ks / (kr + ks);
        c += kf * ih2;
        coef[s * N + e] = -kf * ih2;
      } else {
        c += kr * ih2;
        coef[s * N + e] = 0.0;
      }
    }
    coef[e] = c;
  }
}

__global__ void k_kappa_grad(Grid g, const double* __restrict__ kappa, const double* __restrict__ u,
                             const double* __restrict__ lam, double* grad) {
  const int64_t N = g.N(), M = g.M();
  const int64_t off[7] = {0, -1, 1, -(int64_t)g.nx, (int64_t)g.nx, -M, M};
  const double h[3] = {1.0 / (g.nx + 1), 1.0 / (g.ny + 1), 1.0 / (g.nz + 1)};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N; e += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k;
    grid_ijk(g, e, i, j, k);
    const bool in[7] = {true, i > 0, i < g.nx - 1, j > 0, j < g.ny - 1, k > 0, k < g.nz - 1};
    const double kc = kappa[e], lc = lam[e], uc = u[e];
    double acc = 0.0;
    for (int s = 1; s < 7; ++s) {
      const double ih2 = 1.0 / (h[(s - 1) / 2] * h[(s - 1) / 2]);
      if (in[s]) {
        const int64_t nb = e + off[s];
        const double ks = kappa[nb];
        const double dk = 2.0 * ks * ks / ((kc + ks) * (kc + ks));
        acc += dk * (lc - lam[nb]) * (uc - u[nb]) * ih2;
      } else {
        acc += lc * uc * ih2;
      }
    }
    grad[e] = -acc;
  }
}

inline int nblocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

void launch_validate(Grid g, const double* coef, int* flags, hipStream_t s) {
  if (g.ns == 27)
    hipLaunchKernelGGL(k_validate27, dim3(nblocks_for(g.N())), dim3(256), 0, s, g, coef, flags);
  else
    hipLaunchKernelGGL(k_validate, dim3(nblocks_for(g.N())), dim3(256), 0, s, g, coef, flags);
}

template <class T>
void launch_cut9_fill(Grid g, const double* coef, const Cut9Ent* ents, int nent, int nblk, T* const* uptr,
                      T* const* vptr, const int* rows, const int* cols, hipStream_t s) {
  if (nent == 0) return;
  hipLaunchKernelGGL(k_cut9_fill<T>, dim3((nent + 255) / 256, g.nz), dim3(256), 0, s, g, coef, ents, nent, nblk,
                     uptr, vptr, rows, cols);
}

template <class T>
void launch_conv_leaves(Grid g, const double* coef, const LeafEnt* ents, int nent, T* const* leafptr, int nleaf,
                        hipStream_t s) {
  if (nent == 0) return;
  hipLaunchKernelGGL(k_conv_leaves<T>, dim3((nent + 255) / 256, g.nz), dim3(256), 0, s, g, coef, ents, nent, leafptr,
                     nleaf);
}

void launch_cut_rank(Grid g, const double* coef, const CutEnt* ents, const int* first, int nblk, double eps,
                     int* ranks, hipStream_t s) {
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_cut_rank, dim3((nblk + 63) / 64, g.nz), dim3(64), 0, s, g, coef, ents, first, nblk, eps, ranks);
}

template <class T>
void launch_cut_fill(Grid g, const double* coef, const CutEnt* ents, const int* first, int nblk, double eps,
                     T* const* uptr, T* const* vptr, const int* rows, const int* cols, hipStream_t s) {
  if (nblk == 0) return;
  hipLaunchKernelGGL(k_cut_fill<T>, dim3((nblk + 63) / 64, g.nz), dim3(64), 0, s, g, coef, ents, first, nblk, eps,
                     uptr, vptr, rows, cols);
}

template <class T>
void launch_diag(Grid g, const double* coef, int slot, const int* perm, T* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag<T>, dim3(nblocks_for(g.N())), dim3(256), 0, s, g, coef, slot, perm, out);
}

template <class T>
void launch_perm_in(Grid g, int nrhs, const double* b, int64_t ldb, const int* perm, T* W, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_in<T>, dim3(nblocks_for(g.N() * nrhs)), dim3(256), 0, s, g, nrhs, b, ldb, perm, W);
}

template <class T>
void launch_perm_out(Grid g, int nrhs, const T* W, const int* perm, double* x, int64_t ldx, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_out<T>, dim3(nblocks_for(g.N() * nrhs)), dim3(256), 0, s, g, nrhs, W, perm, x, ldx);
}

void launch_residual(Grid g, const double* coef, const double* x, const double* b, double* r, int transpose,
                     hipStream_t s) {
  if (g.ns == 27)
    hipLaunchKernelGGL(k_residual27, dim3(nblocks_for(g.N())), dim3(256), 0, s, g, coef, x, b, r, transpose);
  else
    hipLaunchKernelGGL(k_residual, dim3(nblocks_for(g.N())), dim3(256), 0, s, g, coef, x, b, r, transpose);
}

void launch_multidot(int64_t n, int nvec, const double* X, int64_t ldx, const double* y, double* part, int nblocks,
                     hipStream_t s) {
  if (nvec == 0) return;
  hipLaunchKernelGGL(k_multidot, dim3(nblocks, nvec), dim3(256), 0, s, n, nvec, X, ldx, y, part);
}

void launch_reduce_parts(int nvec, const double* part, int nblocks, double* out, hipStream_t s) {
  if (nvec == 0) return;
  hipLaunchKernelGGL(k_reduce_parts, dim3(nvec), dim3(256), 0, s, part, nblocks, out);
}

void launch_gemv_sub(int64_t n, int nvec, const double* X, int64_t ldx, const double* h, double* y, hipStream_t s) {
  if (nvec == 0) return;
  hipLaunchKernelGGL(k_gemv_sub, dim3(nblocks_for(n)), dim3(256), 0, s, n, nvec, X, ldx, h, y);
}

void launch_axpby(int64_t n, double alpha, const double* x, double beta, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(nblocks_for(n)), dim3(256), 0, s, n, alpha, x, beta, y);
}

void launch_scale_copy(int64_t n, const double* x, const double* alpha_dev, int invert, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_copy, dim3(nblocks_for(n)), dim3(256), 0, s, n, x, alpha_dev, invert, y);
}

void launch_assemble(Grid g, const double* kappa, double* coef, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble, dim3(nblocks_for(g.N())), dim3(256), 0, s, g, kappa, coef);
}

void launch_kappa_grad(Grid g, const double* kappa, const double* u, const double* lam, double* grad,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_kappa_grad, dim3(nblocks_for(g.N())), dim3(256), 0, s, g, kappa, u, lam, grad);
}

#define ACR_ST_INST(T)                                                                                          \
  template void launch_conv_leaves<T>(Grid, const double*, const LeafEnt*, int, T* const*, int, hipStream_t);  \
  template void launch_cut_fill<T>(Grid, const double*, const CutEnt*, const int*, int, double, T* const*,      \
                                   T* const*, const int*, const int*, hipStream_t);                            \
  template void launch_diag<T>(Grid, const double*, int, const int*, T*, hipStream_t);                          \
  template void launch_cut9_fill<T>(Grid, const double*, const Cut9Ent*, int, int, T* const*, T* const*,        \
                                    const int*, const int*, hipStream_t);                                       \
  template void launch_perm_in<T>(Grid, int, const double*, int64_t, const int*, T*, hipStream_t);             \
  template void launch_perm_out<T>(Grid, int, const T*, const int*, double*, int64_t, hipStream_t);
ACR_ST_INST(float)
ACR_ST_INST(double)
#undef ACR_ST_INST

}  // namespace acr
