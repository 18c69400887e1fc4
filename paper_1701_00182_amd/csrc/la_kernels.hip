// Batched dense linear-algebra kernels for the hierarchical block operations.
//
// One launch processes a list of independent small problems (all blocks of one
// hierarchical depth over all planes of a cyclic-reduction level).  Kernels:
//   k_copy     scaled copies / accumulations of sub-matrices (stack assembly)
//   k_inverse_blk  blocked Gauss-Jordan inverse with partial pivoting, the
//              update outside each panel on the matrix cores (dense leaves,
//              the capacitance matrices of the HODLR inverse)
//   k_inverse  unblocked Gauss-Jordan (matrices whose panels exceed LDS)
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
  const int64_t units = copy_units(t.m, t.n);
  const int ich = (t.m + kCopyUnit - 1) / kCopyUnit;
  const int cpu = copy_cols_per_unit(t.m);
  // one VN-element slot: rows i .. i + nv - 1 of column j, 16-byte accesses
  // when the whole slot is there and aligned
  struct Slot {
    T x[VN], r[VN], y[VN];
    T* d;
    T csj;
    int i, j, nv;
    bool vec;
  };
  auto load = [&](Slot& q) {
    const T* sc = src ? src + (int64_t)q.j * t.lds + q.i : nullptr;
    q.d = dst + (int64_t)q.j * t.ldd + q.i;
    q.csj = cs ? cs[q.j] : T(1);
    q.vec = q.nv == VN && aligned16(sc) && aligned16(q.d) && (!rs || aligned16(rs + q.i));
    if (q.vec) {
      if (sc) *reinterpret_cast<V*>(q.x) = *reinterpret_cast<const V*>(sc);
      if (rs) *reinterpret_cast<V*>(q.r) = *reinterpret_cast<const V*>(rs + q.i);
      if (t.accumulate) *reinterpret_cast<V*>(q.y) = *reinterpret_cast<const V*>(q.d);
    } else {
      // unrolled with a predicate per element, so the slot stays in registers
#pragma unroll
      for (int c = 0; c < VN; ++c) {
        if (c < q.nv) {
          if (sc) q.x[c] = sc[c];
          if (rs) q.r[c] = rs[q.i + c];
          if (t.accumulate) q.y[c] = q.d[c];
        }
      }
    }
    if (!sc)
#pragma unroll
      for (int c = 0; c < VN; ++c) q.x[c] = q.i + c == q.j ? T(1) : T(0);
  };
  auto store = [&](Slot& q) {
    T o[VN];
#pragma unroll
    for (int c = 0; c < VN; ++c) {
      T v = alpha * q.x[c];
      if (rs) v *= q.r[c];
      v *= q.csj;
      if (t.accumulate) v += q.y[c];
      o[c] = v;
    }
    if (q.vec) {
      *reinterpret_cast<V*>(q.d) = *reinterpret_cast<const V*>(o);
    } else {
#pragma unroll
      for (int c = 0; c < VN; ++c)
        if (c < q.nv) q.d[c] = o[c];
    }
  };
  for (int64_t u = blockIdx.y; u < units; u += gridDim.y) {
    // the unit's columns c0 .. c1 - 1, rows r0 .. r1 - 1 of each
    int c0, c1, r0, r1;
    if (t.m > kCopyUnit) {
      c0 = (int)(u / ich);
      c1 = c0 + 1;
      r0 = (int)(u % ich) * kCopyUnit;
      r1 = t.m < r0 + kCopyUnit ? t.m : r0 + kCopyUnit;
    } else {
      c0 = (int)u * cpu;
      c1 = t.n < c0 + cpu ? t.n : c0 + cpu;
      r0 = 0;
      r1 = t.m;
    }
    const int spc = (r1 - r0 + VN - 1) / VN;   // slots per column
    const int cnt = (c1 - c0) * spc;
    // two slots per thread per pass, both loaded before either is stored
    for (int e = threadIdx.x; e < cnt; e += 512) {
      Slot a, b;
      const bool hb = e + 256 < cnt;
      {
        const int jj = e / spc, v = e - jj * spc;
        a.j = c0 + jj;
        a.i = r0 + v * VN;
        a.nv = r1 - a.i < VN ? r1 - a.i : VN;
      }
      if (hb) {
        const int e2 = e + 256, jj = e2 / spc, v = e2 - jj * spc;
        b.j = c0 + jj;
        b.i = r0 + v * VN;
        b.nv = r1 - b.i < VN ? r1 - b.i : VN;
      }
      load(a);
      if (hb) load(b);
      store(a);
      if (hb) store(b);
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

// Blocked Gauss-Jordan inverse with partial pivoting on the matrix cores.
// The columns are taken in panels of NB (32 in FP32, 16 in FP64).  A panel's
// pivots run on the vector units: each step picks the pivot row, swaps it
// with row j across the whole matrix, and applies the elimination step E_j to
// the panel columns only, which then hold the columns of T_P = E_last...E_first
// (in-place Gauss-Jordan).  Every other column c is then updated at once by
// C <- T_P C, a rank-NB product on the matrix cores (v_mfma_f32_32x32x2_f32 /
// v_mfma_f64_16x16x4_f64, one 32 x 32 tile of C per wavefront, C[P, :] saved
// in LDS beforehand): rows outside the panel take C + T_P[i, P] C[P, :], the
// panel's rows are written as T_P[P, P] C[P, :] directly -- forming them as
// C + (T_P - I)[P, P] C[P, :] would cancel nearly all of C[P, :] when the
// pivots are large and lose digits in FP32.  Row swaps commute
// with the deferred update because they are applied to whole rows, the stored
// panel factors included.  The matrix lives in LDS (LDS = true) or in place in
// global memory; the panel and the saved rows are in LDS either way.  After the
// last panel the columns are swapped back in reverse pivot order.
template <class T> struct InvNb { static constexpr int value = 32; };
template <> struct InvNb<double> { static constexpr int value = 16; };

template <class T, bool LDS, int NT>
__global__ __launch_bounds__(NT) void k_inverse_blk(const InvTask* __restrict__ tasks, int* flags) {
  constexpr int NB = InvNb<T>::value;
  constexpr int NW = NT / 64;
  extern __shared__ double smem_d[];
  const InvTask t = tasks[blockIdx.x];
  const int s = t.s;
  if (s == 0) return;
  T* g = static_cast<T*>(t.A);
  // LDS: [a (s x s, LDS = true)] W (s x NB, the panel) | R (NB x s, saved rows) | piv (s)
  T* a;
  int64_t la;
  T* W;
  if (LDS) {
    a = reinterpret_cast<T*>(smem_d);
    la = s;
    W = a + (int64_t)s * s;
  } else {
    a = g;
    la = t.lda;
    W = reinterpret_cast<T*>(smem_d);
  }
  T* R = W + (int64_t)s * NB;
  int* piv = reinterpret_cast<int*>(R + (int64_t)NB * s);
  __shared__ double red[NW];
  __shared__ int redi[NW];
  if (LDS)
    staged_copy<NT>(
        (int64_t)s * s, [&](int64_t e) { return g[(int)e % s + (int64_t)((int)e / s) * t.lda]; },
        [&](int64_t e, T v) { a[e] = v; });
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  bool bad = false;
  for (int j0 = 0; j0 < s; j0 += NB) {
    const int jn = s - j0 < NB ? s - j0 : NB;
    __syncthreads();
    // the panel into W (columns beyond jn zero)
    for (int e = threadIdx.x; e < s * NB; e += NT) {
      const int i = e % s, c = e / s;
      W[i + (int64_t)c * s] = c < jn ? a[i + (int64_t)(j0 + c) * la] : T(0);
    }
    __syncthreads();
    for (int jj = 0; jj < jn; ++jj) {
      const int j = j0 + jj;
      double best = -1.0;
      int bi = j;
      for (int i = j + threadIdx.x; i < s; i += NT) {
        const double v = fabs((double)W[i + (int64_t)jj * s]);
        if (v > best) { best = v; bi = i; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (o > best || (o == best && oi < bi)) { best = o; bi = oi; }
      }
      if (lane == 0) { red[wave] = best; redi[wave] = bi; }
      __syncthreads();
      best = red[0];
      int p = redi[0];
      for (int w = 1; w < NW; ++w)
        if (red[w] > best || (red[w] == best && redi[w] < p)) { best = red[w]; p = redi[w]; }
      if (threadIdx.x == 0) piv[j] = p;
      if (p != j) {
        // rows j and p: the panel in W, every other column in a
        for (int c = threadIdx.x; c < s; c += NT) {
          if (c >= j0 && c < j0 + jn) continue;
          const T x = a[j + (int64_t)c * la];
          a[j + (int64_t)c * la] = a[p + (int64_t)c * la];
          a[p + (int64_t)c * la] = x;
        }
        for (int c = threadIdx.x; c < jn; c += NT) {
          const T x = W[j + (int64_t)c * s];
          W[j + (int64_t)c * s] = W[p + (int64_t)c * s];
          W[p + (int64_t)c * s] = x;
        }
      }
      __syncthreads();
      const T pv = W[j + (int64_t)jj * s];
      if (!(pv != T(0)) || !isfinite((double)pv)) bad = true;
      const T inv = T(1) / pv;
      // E_j on the panel columns c != jj: W[i, c] -= W[i, jj] W[j, c] / pv, i != j
      for (int e = threadIdx.x; e < s * jn; e += NT) {
        const int i = e % s, c = e / s;
        if (c == jj || i == j) continue;
        W[i + (int64_t)c * s] -= W[i + (int64_t)jj * s] * (W[j + (int64_t)c * s] * inv);
      }
      __syncthreads();
      for (int c = threadIdx.x; c < jn; c += NT)
        if (c != jj) W[j + (int64_t)c * s] *= inv;
      for (int i = threadIdx.x; i < s; i += NT)
        if (i != j) W[i + (int64_t)jj * s] = -W[i + (int64_t)jj * s] * inv;
      if (threadIdx.x == 0) W[j + (int64_t)jj * s] = inv;
      __syncthreads();
    }
    // rows P of the other columns
    for (int e = threadIdx.x; e < NB * s; e += NT) {
      const int k = e % NB, c = e / NB;
      R[k + (int64_t)c * NB] = (k < jn && (c < j0 || c >= j0 + jn)) ? a[j0 + k + (int64_t)c * la] : T(0);
    }
    __syncthreads();
    // C <- W R (+ C outside the panel's rows) on the matrix cores over the
    // columns outside the panel: one 32 x 32 tile of C per wavefront (the
    // transposed product, as in the GEMM kernels: rows of C on the lanes)
    const int nt = (s + 31) / 32;
    for (int tile = wave; tile < nt * nt; tile += NW) {
      const int r0 = (tile % nt) * 32, c0 = (tile / nt) * 32;
      if (c0 >= j0 && c0 + 32 <= j0 + jn) continue;   // a tile inside the panel
      if constexpr (sizeof(T) == 4) {
        typedef float f32x16 __attribute__((ext_vector_type(16)));
        const int row = r0 + (lane & 31);
        f32x16 acc;
        const bool prow = row >= j0 && row < j0 + jn;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int col = c0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          acc[v] = (row < s && col < s && !prow) ? (float)a[row + (int64_t)col * la] : 0.f;
        }
#pragma unroll
        for (int kk = 0; kk < NB; kk += 2) {
          const int k = kk + (lane >> 5);
          const float wa = row < s ? (float)W[row + (int64_t)k * s] : 0.f;
          const int cb = c0 + (lane & 31);
          const float rb = cb < s ? (float)R[k + (int64_t)cb * NB] : 0.f;
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(rb, wa, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int col = c0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          if (row < s && col < s && (col < j0 || col >= j0 + jn)) a[row + (int64_t)col * la] = (T)acc[v];
        }
      } else {
        typedef double f64x4 __attribute__((ext_vector_type(4)));
        f64x4 acc[2][2];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = r0 + 16 * x + (lane & 15), col = c0 + 16 * y + (lane >> 4) + 4 * v;
              const bool prow = row >= j0 && row < j0 + jn;
              acc[x][y][v] = (row < s && col < s && !prow) ? (double)a[row + (int64_t)col * la] : 0.0;
            }
#pragma unroll
        for (int kk = 0; kk < NB; kk += 4) {
          const int k = kk + (lane >> 4);
          double wa[2], rb[2];
#pragma unroll
          for (int x = 0; x < 2; ++x) {
            const int row = r0 + 16 * x + (lane & 15);
            wa[x] = row < s ? (double)W[row + (int64_t)k * s] : 0.0;
            const int cb = c0 + 16 * x + (lane & 15);
            rb[x] = cb < s ? (double)R[k + (int64_t)cb * NB] : 0.0;
          }
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
              acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(rb[y], wa[x], acc[x][y], 0, 0, 0);
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = r0 + 16 * x + (lane & 15), col = c0 + 16 * y + (lane >> 4) + 4 * v;
              if (row < s && col < s && (col < j0 || col >= j0 + jn)) a[row + (int64_t)col * la] = (T)acc[x][y][v];
            }
      }
    }
    __syncthreads();
    // the panel's columns: T_P[:, P]
    for (int e = threadIdx.x; e < s * jn; e += NT) {
      const int i = e % s, c = e / s;
      a[i + (int64_t)(j0 + c) * la] = W[i + (int64_t)c * s];
    }
  }
  __syncthreads();
  for (int j = s - 1; j >= 0; --j) {
    const int p = piv[j];
    if (p != j) {
      for (int r = threadIdx.x; r < s; r += NT) {
        const T tmp = a[r + (int64_t)j * la];
        a[r + (int64_t)j * la] = a[r + (int64_t)p * la];
        a[r + (int64_t)p * la] = tmp;
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

template <class T, bool LDS, int NT>
void launch_inverse_blk(const InvTask* d_tasks, int ntasks, size_t lds_bytes, int* d_flags, hipStream_t s) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_inverse_blk<T, LDS, NT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  hipLaunchKernelGGL((k_inverse_blk<T, LDS, NT>), dim3(ntasks), dim3(NT), lds_bytes, s, d_tasks, d_flags);
}

template <class T>
void launch_inverse(const InvTask* d_tasks, int ntasks, int max_s, int* d_flags, hipStream_t s, bool unblocked) {
  if (ntasks <= 0) return;
  // blocked Gauss-Jordan: the matrix, the panel and the saved rows in LDS when
  // they fit, else the panel and the saved rows only
  const size_t nb = InvNb<T>::value;
  const size_t side = 2 * (size_t)max_s * nb * sizeof(T) + (size_t)max_s * sizeof(int);
  const size_t full = side + (size_t)max_s * max_s * sizeof(T);
  if (!unblocked && full <= kLdsBudget) {
    if (max_s < 96)
      launch_inverse_blk<T, true, 256>(d_tasks, ntasks, full, d_flags, s);
    else
      launch_inverse_blk<T, true, 1024>(d_tasks, ntasks, full, d_flags, s);
    return;
  }
  if (!unblocked && side <= kLdsBudget) {
    launch_inverse_blk<T, false, 1024>(d_tasks, ntasks, side, d_flags, s);
    return;
  }
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
  template void launch_inverse<T>(const InvTask*, int, int, int*, hipStream_t, bool);

ACR_INST(float)
ACR_INST(double)
#undef ACR_INST

}  // namespace acr
