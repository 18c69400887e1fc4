// Batched GEMM on the CDNA4 matrix cores: C = alpha op(A) op(B) + beta C over a
// list of independent problems (every block product of one hierarchical depth
// across all planes of a reduction level goes into one launch).
//
// Each workgroup (4 wavefronts) computes one 64 x 64 output tile; wavefront w
// owns the 32 x 32 quadrant (w & 1, w >> 1).  Operand blocks are loaded with
// 16-byte vectors into registers one block ahead (the next block's loads are
// in flight while the current one is multiplied).  The matrix cores compute the
// transposed quadrant (B-panel columns as the first operand), so that
// consecutive lanes hold consecutive rows of the column-major C and the
// stores coalesce.  K advances in blocks staged through LDS, converted to the
// matrix-core input type on the way in:
//   FP64 data            v_mfma_f64_16x16x4_f64   (2 x 2 per wavefront)
//   FP32 data            v_mfma_f32_32x32x2_f32
//   FP32 data, 16-bit    v_mfma_f32_32x32x16_{bf16,f16}: each K block of the
//                        A row panel and of the B column panel of the tile is
//                        scaled by a power of two that brings its largest
//                        magnitude into [0.5, 1), rounded to nearest even; the
//                        block's product is accumulated in FP32 with the
//                        scales removed exactly.
// Operand / accumulator lane layouts (64 lanes, lane l):
//   32x32xK: A[i = l % 32][k = kb * (l / 32) + 0..kb-1], B[k ...][j = l % 32],
//            D[v] = C[8 (v / 4) + 4 (l / 32) + v % 4][l % 32]  (v = 0..15)
//   16x16x4: A[i = l % 16][k = l / 16], B[k = l / 16][j = l % 16],
//            D[v] = C[l / 16 + 4 v][l % 16]  (v = 0..3)
#include <cmath>

#include "kern.h"

namespace acr {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <class T>
__device__ inline T load_a(const GemmTask& t, const T* A, int i, int k) {
  return (i < t.m && k < t.k) ? (t.ta ? A[k + (int64_t)i * t.lda] : A[i + (int64_t)k * t.lda]) : T(0);
}
template <class T>
__device__ inline T load_b(const GemmTask& t, const T* B, int k, int j) {
  return (j < t.n && k < t.k) ? (t.tb ? B[j + (int64_t)k * t.ldb] : B[k + (int64_t)j * t.ldb]) : T(0);
}

__device__ inline void tile_of(const GemmTask& t, int local, int& row0, int& col0) {
  const int ntn = (t.n + 63) >> 6;
  row0 = (local / ntn) * 64;
  col0 = (local % ntn) * 64;
}

// A wavefront's 32 x 32 FP32 accumulator, computed transposed (D[v] holds
// row r = lane row, column c0 + 8 (v / 4) + 4 (l / 32) + v % 4): C = alpha acc
// + beta C with one row pointer per lane.
__device__ inline void store_acc32(const GemmTask& t, int r, int c0, const f32x16& acc) {
  const int lane = threadIdx.x & 63;
  if (r >= t.m) return;
  float* base = static_cast<float*>(t.C) + r;
  const float al = (float)t.alpha, be = (float)t.beta;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int c = c0 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (c >= t.n) continue;
    float* p = base + (int64_t)c * t.ldc;
    float x = al * acc[v];
    if (t.beta != 0.0) x += be * *p;
    *p = x;
  }
}

// C(i, j) of the tile = alpha * v + beta * C(i, j)
template <class T>
__device__ inline void store_tile(const GemmTask& t, int row0, int col0, int i, int j, T v) {
  const int gi = row0 + i, gj = col0 + j;
  if (gi >= t.m || gj >= t.n) return;
  T* c = static_cast<T*>(t.C) + gi + (int64_t)gj * t.ldc;
  T r = T(t.alpha) * v;
  if (t.beta != 0.0) r += T(t.beta) * *c;
  *c = r;
}

// Register-staged operand tile: P positions p (rows of op(A) or columns of
// op(B)) x KB values of k, element (p, k) at base[p * sp + k * sk] with one of
// sp / sk equal to 1.  Each thread moves NV vectors of VEC consecutive elements
// along the contiguous dimension (one 16-byte load when aligned and inside the
// matrix, element loads with zero fill otherwise); the values are held in
// registers while the previous block is multiplied, then written to LDS.
template <class T, int KB, int P = 64> struct Stage {
  static constexpr int VEC = 16 / sizeof(T);
  static constexpr int NV = P * KB / (VEC * 256);
  static_assert(NV >= 1 && NV * VEC * 256 == P * KB, "tile not a multiple of the workgroup's vectors");
  T v[NV][VEC];

  __device__ inline void load(const T* base, int64_t sp, int64_t sk, int np, int K, int p0, int k0) {
    const bool pc = sp == 1;
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      const int e = threadIdx.x + s * 256;
      int p, k;
      if (pc) { p = (e % (P / VEC)) * VEC; k = e / (P / VEC); }
      else { k = (e % (KB / VEC)) * VEC; p = e / (KB / VEC); }
      const int gp = p0 + p, gk = k0 + k;
      const T* ptr = base + gp * sp + gk * sk;
      const bool full = pc ? (gp + VEC <= np && gk < K) : (gp < np && gk + VEC <= K);
      if (full && (((uintptr_t)ptr & 15) == 0)) {
        typedef T V __attribute__((ext_vector_type(VEC)));
        const V x = *reinterpret_cast<const V*>(ptr);
#pragma unroll
        for (int u = 0; u < VEC; ++u) v[s][u] = x[u];
      } else {
        // element u sits at ptr + u along the contiguous dimension
#pragma unroll
        for (int u = 0; u < VEC; ++u) {
          const int qp = pc ? gp + u : gp, qk = pc ? gk : gk + u;
          v[s][u] = (qp < np && qk < K) ? ptr[u] : T(0);
        }
      }
    }
  }
  // into lds[k][p] (row stride LD), converted to the LDS element type
  template <class L, int LD> __device__ inline void store(L (*lds)[LD], bool pc) const {
#pragma unroll
    for (int s = 0; s < NV; ++s) {
      const int e = threadIdx.x + s * 256;
      int p, k;
      if (pc) { p = (e % (P / VEC)) * VEC; k = e / (P / VEC); }
      else { k = (e % (KB / VEC)) * VEC; p = e / (KB / VEC); }
#pragma unroll
      for (int u = 0; u < VEC; ++u) {
        if (pc) lds[k][p + u] = L(v[s][u]);
        else lds[k + u][p] = L(v[s][u]);
      }
    }
  }
};

// operand geometry of op(A) (rows p, inner k) and op(B) (columns p, inner k)
__device__ inline void a_geom(const GemmTask& t, int64_t& sp, int64_t& sk) {
  if (t.ta) { sp = t.lda; sk = 1; } else { sp = 1; sk = t.lda; }
}
__device__ inline void b_geom(const GemmTask& t, int64_t& sp, int64_t& sk) {
  if (t.tb) { sp = 1; sk = t.ldb; } else { sp = t.ldb; sk = 1; }
}

// FP32 data, FP32 matrix cores.
__global__ __launch_bounds__(256) void k_gemm_f32(const GemmTask* __restrict__ tasks, const int* __restrict__ tile_task,
                                                  const int* __restrict__ first_tile) {
  constexpr int KB = 32;
  const int ti = tile_task[blockIdx.x];
  const GemmTask t = tasks[ti];
  int row0, col0;
  tile_of(t, blockIdx.x - first_tile[ti], row0, col0);
  __shared__ float As[KB][64 + 4];
  __shared__ float Bs[KB][64 + 4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
  const float* A = static_cast<const float*>(t.A);
  const float* B = static_cast<const float*>(t.B);
  int64_t asp, ask, bsp, bsk;
  a_geom(t, asp, ask);
  b_geom(t, bsp, bsk);
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  Stage<float, KB> sa, sb;
  if (t.k > 0) {
    sa.load(A, asp, ask, t.m, t.k, row0, 0);
    sb.load(B, bsp, bsk, t.n, t.k, col0, 0);
  }
  for (int k0 = 0; k0 < t.k; k0 += KB) {
    sa.store(As, asp == 1);
    sb.store(Bs, bsp == 1);
    __syncthreads();
    if (k0 + KB < t.k) {   // next block in flight during the products
      sa.load(A, asp, ask, t.m, t.k, row0, k0 + KB);
      sb.load(B, bsp, bsk, t.n, t.k, col0, k0 + KB);
    }
#pragma unroll
    for (int kk = 0; kk < KB; kk += 2) {
      const float a = As[kk + (lane >> 5)][wr + (lane & 31)];
      const float b = Bs[kk + (lane >> 5)][wc + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(b, a, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  store_acc32(t, row0 + wr + (lane & 31), col0 + wc, acc);
}

// FP32 data, FP32 matrix cores, for outputs at most 32 columns wide (the
// low-rank side of most factorisation products): 128 x 32 output tiles, wave
// w owning rows 32 w .. 32 w + 31, so that no matrix-core work goes to the
// empty half of a 64 x 64 tile.
__global__ __launch_bounds__(256) void k_gemm_f32_n32(const GemmTask* __restrict__ tasks,
                                                      const int* __restrict__ tile_task,
                                                      const int* __restrict__ first_tile) {
  constexpr int KB = 32;
  const int ti = tile_task[blockIdx.x];
  const GemmTask t = tasks[ti];
  const int row0 = (blockIdx.x - first_tile[ti]) * 128;
  __shared__ float As[KB][128 + 4];
  __shared__ float Bs[KB][32 + 4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w * 32;
  const float* A = static_cast<const float*>(t.A);
  const float* B = static_cast<const float*>(t.B);
  int64_t asp, ask, bsp, bsk;
  a_geom(t, asp, ask);
  b_geom(t, bsp, bsk);
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  Stage<float, KB, 128> sa;
  Stage<float, KB, 32> sb;
  if (t.k > 0) {
    sa.load(A, asp, ask, t.m, t.k, row0, 0);
    sb.load(B, bsp, bsk, t.n, t.k, 0, 0);
  }
  for (int k0 = 0; k0 < t.k; k0 += KB) {
    sa.store(As, asp == 1);
    sb.store(Bs, bsp == 1);
    __syncthreads();
    if (k0 + KB < t.k) {   // next block in flight during the products
      sa.load(A, asp, ask, t.m, t.k, row0, k0 + KB);
      sb.load(B, bsp, bsk, t.n, t.k, 0, k0 + KB);
    }
#pragma unroll
    for (int kk = 0; kk < KB; kk += 2) {
      const float a = As[kk + (lane >> 5)][wr + (lane & 31)];
      const float b = Bs[kk + (lane >> 5)][lane & 31];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(b, a, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  store_acc32(t, row0 + wr + (lane & 31), 0, acc);
}

// FP64 data, FP64 matrix cores.
__global__ __launch_bounds__(256) void k_gemm_f64(const GemmTask* __restrict__ tasks, const int* __restrict__ tile_task,
                                                  const int* __restrict__ first_tile) {
  constexpr int KB = 16;
  const int ti = tile_task[blockIdx.x];
  const GemmTask t = tasks[ti];
  int row0, col0;
  tile_of(t, blockIdx.x - first_tile[ti], row0, col0);
  __shared__ double As[KB][64 + 2];
  __shared__ double Bs[KB][64 + 2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
  const double* A = static_cast<const double*>(t.A);
  const double* B = static_cast<const double*>(t.B);
  int64_t asp, ask, bsp, bsk;
  a_geom(t, asp, ask);
  b_geom(t, bsp, bsk);
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.0;
  Stage<double, KB> sa, sb;
  if (t.k > 0) {
    sa.load(A, asp, ask, t.m, t.k, row0, 0);
    sb.load(B, bsp, bsk, t.n, t.k, col0, 0);
  }
  for (int k0 = 0; k0 < t.k; k0 += KB) {
    sa.store(As, asp == 1);
    sb.store(Bs, bsp == 1);
    __syncthreads();
    if (k0 + KB < t.k) {
      sa.load(A, asp, ask, t.m, t.k, row0, k0 + KB);
      sb.load(B, bsp, bsk, t.n, t.k, col0, k0 + KB);
    }
#pragma unroll
    for (int kk = 0; kk < KB; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        a[s] = As[kk + (lane >> 4)][wr + 16 * s + (lane & 15)];
        b[s] = Bs[kk + (lane >> 4)][wc + 16 * s + (lane & 15)];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[y], a[x], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        store_tile<double>(t, row0, col0, wr + 16 * x + (lane & 15), wc + 16 * y + (lane >> 4) + 4 * v, acc[x][y][v]);
}

template <class H> struct Mfma16;
template <> struct Mfma16<__bf16> {
  typedef bf16x8 V;
  static __device__ inline f32x16 run(V a, V b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0); }
};
template <> struct Mfma16<_Float16> {
  typedef f16x8 V;
  static __device__ inline f32x16 run(V a, V b, f32x16 c) { return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0); }
};

// Exponent e with max * 2^-e in [0.5, 1) (0 for an all-zero or non-finite block).
__device__ inline int block_exponent(float mx) {
  if (!(mx > 0.f) || !isfinite(mx)) return 0;
  int e;
  (void)frexpf(mx, &e);
  return e;
}

// FP32 data through 16-bit matrix-core inputs.  The operands are staged with
// the FP32 kernel's 16-byte register loads; each K block of the A row panel
// and of the B column panel is scaled by a power of two that brings its
// largest magnitude into [0.5, 1) (a workgroup maximum over the staged
// values), rounded to nearest even into LDS (k contiguous, so that each lane
// reads its 8 k values at once), multiplied into a fresh FP32 accumulator, and
// that block's product is added to the tile with the scales removed (exactly:
// a power of two).
template <class H>
__global__ __launch_bounds__(256) void k_gemm_lowp(const GemmTask* __restrict__ tasks, const int* __restrict__ tile_task,
                                                   const int* __restrict__ first_tile) {
  constexpr int KB = 32;
  typedef Stage<float, KB> S;
  const int ti = tile_task[blockIdx.x];
  const GemmTask t = tasks[ti];
  int row0, col0;
  tile_of(t, blockIdx.x - first_tile[ti], row0, col0);
  __shared__ __attribute__((aligned(16))) H As[64][KB + 8];
  __shared__ __attribute__((aligned(16))) H Bs[64][KB + 8];
  __shared__ float red[2][4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
  const float* A = static_cast<const float*>(t.A);
  const float* B = static_cast<const float*>(t.B);
  int64_t asp, ask, bsp, bsk;
  a_geom(t, asp, ask);
  b_geom(t, bsp, bsk);
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  typedef typename Mfma16<H>::V V;
  S sa, sb;
  if (t.k > 0) {
    sa.load(A, asp, ask, t.m, t.k, row0, 0);
    sb.load(B, bsp, bsk, t.n, t.k, col0, 0);
  }
  // staged element (p, k) of the thread's slot (s, u), as in Stage::store
  auto pos = [&](bool pc, int s, int u, int& p, int& k) {
    const int e = tid + s * 256;
    if (pc) { p = (e % (64 / S::VEC)) * S::VEC + u; k = e / (64 / S::VEC); }
    else { k = (e % (KB / S::VEC)) * S::VEC + u; p = e / (KB / S::VEC); }
  };
  for (int k0 = 0; k0 < t.k; k0 += KB) {
    float ma = 0.f, mb = 0.f;
#pragma unroll
    for (int s = 0; s < S::NV; ++s)
#pragma unroll
      for (int u = 0; u < S::VEC; ++u) {
        ma = fmaxf(ma, fabsf(sa.v[s][u]));
        mb = fmaxf(mb, fabsf(sb.v[s][u]));
      }
    for (int off = 32; off > 0; off >>= 1) {
      ma = fmaxf(ma, __shfl_xor(ma, off, 64));
      mb = fmaxf(mb, __shfl_xor(mb, off, 64));
    }
    if (lane == 0) { red[0][w] = ma; red[1][w] = mb; }
    __syncthreads();
    const int ea = block_exponent(fmaxf(fmaxf(red[0][0], red[0][1]), fmaxf(red[0][2], red[0][3])));
    const int eb = block_exponent(fmaxf(fmaxf(red[1][0], red[1][1]), fmaxf(red[1][2], red[1][3])));
    const bool apc = asp == 1, bpc = bsp == 1;
#pragma unroll
    for (int s = 0; s < S::NV; ++s)
#pragma unroll
      for (int u = 0; u < S::VEC; ++u) {
        int p, k;
        pos(apc, s, u, p, k);
        As[p][k] = H(ldexpf(sa.v[s][u], -ea));
        pos(bpc, s, u, p, k);
        Bs[p][k] = H(ldexpf(sb.v[s][u], -eb));
      }
    __syncthreads();
    if (k0 + KB < t.k) {   // next block in flight during the products
      sa.load(A, asp, ask, t.m, t.k, row0, k0 + KB);
      sb.load(B, bsp, bsk, t.n, t.k, col0, k0 + KB);
    }
    f32x16 blk;
#pragma unroll
    for (int v = 0; v < 16; ++v) blk[v] = 0.f;
#pragma unroll
    for (int kk = 0; kk < KB; kk += 16) {
      const V a = *reinterpret_cast<const V*>(&As[wr + (lane & 31)][kk + 8 * (lane >> 5)]);
      const V b = *reinterpret_cast<const V*>(&Bs[wc + (lane & 31)][kk + 8 * (lane >> 5)]);
      blk = Mfma16<H>::run(b, a, blk);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] += ldexpf(blk[v], ea + eb);
    __syncthreads();
  }
  store_acc32(t, row0 + wr + (lane & 31), col0 + wc, acc);
}

// Segmented GEMM: the inner dimension runs over the task's (A_s, B_s) pairs,
// each in K blocks (zero-padded at a segment's end), with the same register
// prefetch; FP32 data on 32x32x2 FP32 MFMA, FP64 data on 16x16x4 FP64 MFMA.
template <class T>
__global__ __launch_bounds__(256) void k_seg_gemm(const SegGemmTask* __restrict__ tasks,
                                                  const int* __restrict__ tile_task,
                                                  const int* __restrict__ first_tile) {
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int KB = F32 ? 32 : 16;
  constexpr int PAD = F32 ? 4 : 2;
  const int ti = tile_task[blockIdx.x];
  const SegGemmTask& t = tasks[ti];
  const int local = blockIdx.x - first_tile[ti];
  const int ntn = (t.n + 63) >> 6;
  const int row0 = (local / ntn) * 64, col0 = (local % ntn) * 64;
  __shared__ T As[KB][64 + PAD];
  __shared__ T Bs[KB][64 + PAD];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
  f32x16 accf;
  f64x4 accd[2][2];
#pragma unroll
  for (int v = 0; v < 16; ++v) accf[v] = 0.f;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) accd[a][b][v] = 0.0;
  // cursor over (segment, k block)
  int cs = 0, ck = 0;
  while (cs < t.nseg && t.k[cs] <= 0) ++cs;
  Stage<T, KB> sa, sb;
  auto load = [&](int seg, int k0) {
    const int64_t asp = ((t.ta >> seg) & 1) ? t.lda[seg] : 1, ask = ((t.ta >> seg) & 1) ? 1 : t.lda[seg];
    sa.load(static_cast<const T*>(t.A[seg]), asp, ask, t.m, t.k[seg], row0, k0);
    sb.load(static_cast<const T*>(t.B[seg]), t.ldb[seg], 1, t.n, t.k[seg], col0, k0);
  };
  if (cs < t.nseg) load(cs, 0);
  while (cs < t.nseg) {
    // the same contiguity test as in load()
    const bool apc = (((t.ta >> cs) & 1) ? t.lda[cs] : 1) == 1;
    sa.store(As, apc);
    sb.store(Bs, t.ldb[cs] == 1);
    __syncthreads();
    // advance the cursor and prefetch the next block
    int ns = cs, nk = ck + KB;
    if (nk >= t.k[ns]) {
      ++ns;
      nk = 0;
      while (ns < t.nseg && t.k[ns] <= 0) ++ns;
    }
    if (ns < t.nseg) load(ns, nk);
    if constexpr (F32) {
#pragma unroll
      for (int kk = 0; kk < KB; kk += 2) {
        const float a = As[kk + (lane >> 5)][wr + (lane & 31)];
        const float b = Bs[kk + (lane >> 5)][wc + (lane & 31)];
        accf = __builtin_amdgcn_mfma_f32_32x32x2f32(b, a, accf, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < KB; kk += 4) {
        double a[2], b[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          a[s] = As[kk + (lane >> 4)][wr + 16 * s + (lane & 15)];
          b[s] = Bs[kk + (lane >> 4)][wc + 16 * s + (lane & 15)];
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            accd[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[y], a[x], accd[x][y], 0, 0, 0);
      }
    }
    __syncthreads();
    cs = ns;
    ck = nk;
  }
  auto put = [&](int i, int j, T v) {
    const int gi = row0 + i, gj = col0 + j;
    if (gi >= t.m || gj >= t.n) return;
    T* c = static_cast<T*>(t.C) + gi + (int64_t)gj * t.ldc;
    T r = T(t.alpha) * v;
    if (t.beta != 0.0) r += T(t.beta) * *c;
    *c = r;
  };
  if constexpr (F32) {
#pragma unroll
    for (int v = 0; v < 16; ++v) put(wr + (lane & 31), wc + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), accf[v]);
  } else {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) put(wr + 16 * x + (lane & 15), wc + 16 * y + (lane >> 4) + 4 * v, accd[x][y][v]);
  }
}

// FP64 Gram partials on the FP64 matrix cores.  One wavefront per unit (a
// chunk of rows of a stack S, m x r in precision T, and an upper-triangle pair
// bi <= bj of 32-column blocks): part[chunk][i + j r] = sum over the chunk's
// rows of S[row, i] S[row, j], FP64 products of the FP32 / FP64 entries.
// Any assignment of rows to the k slots of the 16x16x4 products gives the same
// sums as long as both operands use it, so lane l takes the RPL consecutive
// rows starting at RPL (l / 16) of column l % 16 of each 16-column half, read
// straight into registers with 16-byte loads (no LDS), one row group ahead.
// A diagonal pair (bi == bj) reads one block and skips the 16 x 16 part
// below its diagonal, which the reduction never reads.  Narrow stacks (r of a
// few tens) waste at most a 32-wide tile instead of a 64-wide one.
template <class T, int RPL> struct RowSlice {
  T v[2][RPL];
  __device__ inline void load(const T* const (&p)[2], int k0, bool vec) {
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const T* q = p[x] + k0;
      if (vec) {
        typedef T V __attribute__((ext_vector_type(16 / sizeof(T))));
        constexpr int W = 16 / sizeof(T);
#pragma unroll
        for (int u = 0; u < RPL / W; ++u) {
          const V y = *reinterpret_cast<const V*>(q + u * W);
#pragma unroll
          for (int w = 0; w < W; ++w) v[x][u * W + w] = y[w];
        }
      } else {
#pragma unroll
        for (int u = 0; u < RPL; ++u) v[x][u] = q[u];
      }
    }
  }
  // rows past the chunk's end (kmax rows from the slice start) read as zero
  __device__ inline void load_tail(const T* const (&p)[2], int k0, int kmax) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int u = 0; u < RPL; ++u) v[x][u] = u < kmax ? p[x][k0 + u] : T(0);
  }
};

template <class T, int RPL>
__device__ inline void gram_step(f64x4 (&acc)[2][2], const RowSlice<T, RPL>& a, const RowSlice<T, RPL>& b,
                                 bool diag) {
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const double a0 = (double)a.v[0][u], a1 = (double)a.v[1][u];
    const double b0 = (double)b.v[0][u], b1 = (double)b.v[1][u];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a0, acc[0][1], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a1, acc[1][1], 0, 0, 0);
    if (!diag) acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a1, acc[1][0], 0, 0, 0);
  }
}

template <class T>
__global__ __launch_bounds__(256) void k_gram_mfma(const GramTask* __restrict__ tasks,
                                                   const int* __restrict__ block_task,
                                                   const int* __restrict__ first_block) {
  constexpr int RPL = 32 / sizeof(T);   // rows per lane and row group: 32 bytes
  constexpr int RW = 4 * RPL;           // rows per row group
  const int ti = block_task[blockIdx.x];
  const GramTask t = tasks[ti];
  const int lane = threadIdx.x & 63;
  const int nb = (t.r + 31) / 32, ntri = nb * (nb + 1) / 2;
  const int nch = (t.m + t.rows_per_chunk - 1) / t.rows_per_chunk;
  const int unit = (blockIdx.x - first_block[ti]) * 4 + (threadIdx.x >> 6);
  if (unit >= nch * ntri) return;   // no workgroup barrier below
  const int chunk = unit / ntri;
  int tri = unit - chunk * ntri;
  int bi = 0;
  while (tri >= nb - bi) { tri -= nb - bi; ++bi; }
  const int bj = bi + tri;
  const bool diag = bi == bj;
  const int r0 = chunk * t.rows_per_chunk;
  const int K = min(t.m, r0 + t.rows_per_chunk) - r0;
  const T* S = static_cast<const T*>(t.A);
  const bool vec = ((reinterpret_cast<uintptr_t>(S) | (uintptr_t)(t.lda * (int64_t)sizeof(T)) |
                     (uintptr_t)(t.rows_per_chunk * (int64_t)sizeof(T))) & 15) == 0;
  // columns past r repeat column r - 1; their sums are never written
  const int c = lane & 15, g = lane >> 4;
  const T* pa[2];
  const T* pb[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    pa[x] = S + (int64_t)min(bi * 32 + 16 * x + c, t.r - 1) * t.lda + r0 + g * RPL;
    pb[x] = S + (int64_t)min(bj * 32 + 16 * x + c, t.r - 1) * t.lda + r0 + g * RPL;
  }
  f64x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[x][y][v] = 0.0;
  const int full = K / RW * RW;
  RowSlice<T, RPL> a, b;
  if (full > 0) {
    a.load(pa, 0, vec);
    if (!diag) b.load(pb, 0, vec);
  }
  for (int k0 = 0; k0 < full; k0 += RW) {
    RowSlice<T, RPL> an, bn;
    const bool more = k0 + RW < full;
    if (more) {
      an.load(pa, k0 + RW, vec);
      if (!diag) bn.load(pb, k0 + RW, vec);
    }
    gram_step(acc, a, diag ? a : b, diag);
    if (more) {
      a = an;
      if (!diag) b = bn;
    }
  }
  if (full < K) {
    const int kmax = K - full - g * RPL;   // rows of this lane's slice inside the chunk
    a.load_tail(pa, full, kmax);
    if (!diag) b.load_tail(pb, full, kmax);
    gram_step(acc, a, diag ? a : b, diag);
  }
  double* P = t.part + (int64_t)chunk * t.r * t.r;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      if (diag && x == 1 && y == 0) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = bi * 32 + 16 * x + c, j = bj * 32 + 16 * y + g + 4 * v;
        if (i < t.r && j < t.r) P[i + (int64_t)j * t.r] = acc[x][y][v];
      }
    }
}

}  // namespace

template <>
void launch_gemm_mfma<float>(const GemmTask* d_tasks, const int* d_tile_task, const int* d_first_tile, int ntiles,
                             int lowp, hipStream_t s) {
  if (ntiles <= 0) return;
  if (lowp == 1)
    hipLaunchKernelGGL(k_gemm_lowp<__bf16>, dim3(ntiles), dim3(256), 0, s, d_tasks, d_tile_task, d_first_tile);
  else if (lowp == 2)
    hipLaunchKernelGGL(k_gemm_lowp<_Float16>, dim3(ntiles), dim3(256), 0, s, d_tasks, d_tile_task, d_first_tile);
  else
    hipLaunchKernelGGL(k_gemm_f32, dim3(ntiles), dim3(256), 0, s, d_tasks, d_tile_task, d_first_tile);
}

void launch_gemm_narrow(const GemmTask* d_tasks, const int* d_tile_task, const int* d_first_tile, int ntiles,
                        hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_gemm_f32_n32, dim3(ntiles), dim3(256), 0, s, d_tasks, d_tile_task, d_first_tile);
}

template <>
void launch_gemm_mfma<double>(const GemmTask* d_tasks, const int* d_tile_task, const int* d_first_tile, int ntiles,
                              int lowp, hipStream_t s) {
  (void)lowp;
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_gemm_f64, dim3(ntiles), dim3(256), 0, s, d_tasks, d_tile_task, d_first_tile);
}

}  // namespace acr

namespace acr {
template <class T>
void launch_gram_mfma(const GramTask* d_tasks, const int* d_tile_task, const int* d_first_tile, int ntiles,
                      hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_gram_mfma<T>, dim3(ntiles), dim3(256), 0, s, d_tasks, d_tile_task, d_first_tile);
}
template void launch_gram_mfma<float>(const GramTask*, const int*, const int*, int, hipStream_t);
template void launch_gram_mfma<double>(const GramTask*, const int*, const int*, int, hipStream_t);
}  // namespace acr

namespace acr {
template <class T>
void launch_seg_gemm(const SegGemmTask* d_tasks, const int* d_tile_task, const int* d_first_tile, int ntiles,
                     hipStream_t s) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_seg_gemm<T>, dim3(ntiles), dim3(256), 0, s, d_tasks, d_tile_task, d_first_tile);
}
template void launch_seg_gemm<float>(const SegGemmTask*, const int*, const int*, int, hipStream_t);
template void launch_seg_gemm<double>(const SegGemmTask*, const int*, const int*, int, hipStream_t);
}  // namespace acr
