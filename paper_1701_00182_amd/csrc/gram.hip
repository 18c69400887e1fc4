// Gram-based compression of large stacked low-rank sums.
//
// For a stack S (m x r) too large for one workgroup's local memory, the
// triangular factor is obtained from the FP64 Gram matrix S^T S (computed on
// the FP64 matrix cores by many wavefronts, each over a chunk of rows and a
// pair of 32-column blocks -- gemm_mfma.hip -- then reduced in a fixed order)
// and a pivoted Cholesky factorisation that stops at the numerical rank:
//   S P = Q [L11^T L21^T],  Q = S P1 L11^{-T}.
// The core (L-factors of both stacks) then goes through the same one-sided
// Jacobi SVD as the Householder path, and the truncated bases are rebuilt with
// one GEMM each: U_new = S W with W = P1 L11^{-T} Z.
#include <cmath>

#include "kern.h"
#include "wave.h"

namespace acr {

namespace {

__global__ __launch_bounds__(256) void k_gram_reduce(const GramTask* __restrict__ tasks) {
  __shared__ double tile[32][33];
  const GramTask t = tasks[blockIdx.x];
  const int r = t.r;
  const int nchunk = (t.m + t.rows_per_chunk - 1) / t.rows_per_chunk;
  // r^2 fits 32 bits (the host rejects wider stacks)
  const int rr = r * r;
  const int nb = (r + 31) / 32, ntile = nb * (nb + 1) / 2;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // 32 x 32 tiles (bi, bj), bi <= bj, of the upper triangle, column by
  // column: the sums of the chunk partials in chunk order for the entries
  // i <= j, stored in place and, through the LDS tile, at the mirrored
  // position, both with consecutive lanes on consecutive rows
  for (int tt = blockIdx.y; tt < ntile; tt += gridDim.y) {
    int bj = (int)((sqrtf(8.0f * (float)tt + 1.0f) - 1.0f) * 0.5f);
    while (bj > 0 && bj * (bj + 1) / 2 > tt) --bj;
    while ((bj + 1) * (bj + 2) / 2 <= tt) ++bj;
    const int bi = tt - bj * (bj + 1) / 2;
    const int i = bi * 32 + tx;
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < r) {
      const double* p = t.part + i;
#pragma unroll 4
      for (int c = 0; c < nchunk; ++c) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int j = bj * 32 + ty + 8 * k;
          if (j < r) sum[k] += p[(int64_t)c * rr + (int64_t)j * r];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int j = bj * 32 + ty + 8 * k;
      if (i < r && j < r && (bi < bj || i <= j)) t.G[i + (int64_t)j * r] = sum[k];
      tile[ty + 8 * k][tx] = sum[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // entry (row, col) = (bj * 32 + tx, bi * 32 + ty + 8 k) mirrors (col, row)
      const int row = bj * 32 + tx, col = bi * 32 + ty + 8 * k;
      if (row < r && col < r && (bi < bj || col < row)) t.G[row + (int64_t)col * r] = tile[tx][ty + 8 * k];
    }
    __syncthreads();
  }
}

__device__ inline double gsumw(double v, int G) {
  for (int off = G >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

// Pivoted Cholesky of an r x r FP64 Gram matrix, stopped when the largest
// remaining diagonal falls to tol * (largest initial diagonal).  Left-looking:
// column j of L is formed from the rows of the previous columns, G lanes per
// row (G chosen so that the remaining rows fill the workgroup).  Only the
// entries on and below the diagonal of the first `rank` columns are written.
template <int NT>
__global__ __launch_bounds__(NT) void k_pchol(const PcholTask* __restrict__ tasks, double tol) {
  extern __shared__ double smp[];
  const PcholTask t = tasks[blockIdx.x];
  const int r = t.r;
  const double* G = t.G;
  double* L = t.L;
  // the remaining diagonal and the pivot order live in LDS during the loop
  double* d = smp;
  int* perm = reinterpret_cast<int*>(smp + r);
  __shared__ double red[NT / 64];
  __shared__ int redi[NT / 64];
  double mx = 0.0;
  for (int i = threadIdx.x; i < r; i += NT) {
    perm[i] = i;
    d[i] = G[i + (int64_t)i * r];
    mx = fmax(mx, d[i]);
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = 0.0;
  for (int w = 0; w < NT / 64; ++w) mx = fmax(mx, red[w]);
  const double thr = tol * mx;
  const bool zero = !(mx > 0.0);
  int rank = 0;
  for (int j = 0; j < r && !zero; ++j) {
    double best = -1.0;
    int bp = j;
    for (int i = j + threadIdx.x; i < r; i += NT) {
      const double v = d[perm[i]];
      if (v > best) { best = v; bp = i; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bp, off, 64);
      if (o > best || (o == best && oi < bp)) { best = o; bp = oi; }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { red[threadIdx.x >> 6] = best; redi[threadIdx.x >> 6] = bp; }
    __syncthreads();
    best = red[0];
    bp = redi[0];
    for (int w = 1; w < NT / 64; ++w)
      if (red[w] > best || (red[w] == best && redi[w] < bp)) { best = red[w]; bp = redi[w]; }
    if (!(best > thr)) break;
    const int p = bp;
    if (p != j) {
      for (int l = threadIdx.x; l < j; l += NT) {
        const double a = L[j + (int64_t)l * r];
        L[j + (int64_t)l * r] = L[p + (int64_t)l * r];
        L[p + (int64_t)l * r] = a;
      }
      if (threadIdx.x == 0) {
        const int tmp = perm[j];
        perm[j] = perm[p];
        perm[p] = tmp;
      }
    }
    __syncthreads();
    const int pj = perm[j];
    const double ljj = sqrt(d[pj]);
    if (threadIdx.x == 0) L[j + (int64_t)j * r] = ljj;
    const int rem = r - j - 1;
    int Gl = 16;
    while (Gl > 1 && Gl * rem > NT) Gl >>= 1;
    const int groups = NT / Gl, gi = threadIdx.x / Gl, gl = threadIdx.x % Gl;
    for (int i = j + 1 + gi; i < r; i += groups) {
      // four independent partial sums keep four loads of each row in flight
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int l = gl;
      for (; l + 3 * Gl < j; l += 4 * Gl) {
        s0 += L[i + (int64_t)l * r] * L[j + (int64_t)l * r];
        s1 += L[i + (int64_t)(l + Gl) * r] * L[j + (int64_t)(l + Gl) * r];
        s2 += L[i + (int64_t)(l + 2 * Gl) * r] * L[j + (int64_t)(l + 2 * Gl) * r];
        s3 += L[i + (int64_t)(l + 3 * Gl) * r] * L[j + (int64_t)(l + 3 * Gl) * r];
      }
      for (; l < j; l += Gl) s0 += L[i + (int64_t)l * r] * L[j + (int64_t)l * r];
      double s = gsumw((s0 + s1) + (s2 + s3), Gl);
      if (gl == 0) {
        const int pi = perm[i];
        const double lij = (G[pi + (int64_t)pj * r] - s) / ljj;
        L[i + (int64_t)j * r] = lij;
        d[pi] -= lij * lij;
      }
    }
    __syncthreads();
    rank = j + 1;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < r; i += NT) {
    t.perm[i] = perm[i];
    t.d[i] = d[i];
  }
  if (threadIdx.x == 0) *t.rank_out = rank;
}

// R (r1 x r, original column order): R[a, perm[i]] = L[i, a] for i >= a.
// Pivoted Cholesky with the Gram matrix in LDS: its lower triangle packed by
// columns, kept in pivot order (the rows and columns of each pivot are swapped
// into place), and right-looking rank-1 updates of the trailing block.  The
// finished columns stay in LDS, unscaled, and their rows follow every later
// pivot swap there; L is written to global memory once, at the end, so that no
// step waits on global memory.  Same outputs as k_pchol: L (r x rank, pivot
// order, column-major in global memory), perm, the remaining diagonal d in the
// original order, the rank.  One workgroup barrier per step (two when the
// pivot moves).  LDS: r (r + 1) / 2 doubles and r ints.
__device__ inline int packed(int r, int i, int k) { return k * (2 * r - k - 1) / 2 + i; }   // i >= k

template <int NT>
__global__ __launch_bounds__(NT) void k_pchol_lds(const PcholTask* __restrict__ tasks, double tol) {
  extern __shared__ double spk[];
  const PcholTask t = tasks[blockIdx.x];
  const int r = t.r;
  double* S = spk;
  int* perm = reinterpret_cast<int*>(S + (size_t)r * (r + 1) / 2);
  auto* L = to_global(t.L);
  constexpr int NW = NT / 64;
  // per-wavefront pivot candidates, double buffered by step parity: the
  // wavefront that updates a column's diagonal proposes it for the next step
  __shared__ double cand[2][NW];
  __shared__ int candi[2][NW];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // G (column-major) into the packed triangle
  const auto* Gg = to_global(t.G);
  staged_copy<NT>(
      (int64_t)r * r, [&](int64_t e) { return Gg[e]; },
      [&](int64_t e, double v) {
        const int k = (int)e / r, i = (int)e - k * r;
        if (i >= k) S[packed(r, i, k)] = v;
      });
  for (int i = threadIdx.x; i < r; i += NT) perm[i] = i;
  __syncthreads();
  {
    double v = -INFINITY;
    int vi = 0x7fffffff;
    for (int i = threadIdx.x; i < r; i += NT) {
      const double x = S[packed(r, i, i)];
      if (x > v) { v = x; vi = i; }
    }
    wave_argmax(v, vi);
    if (lane == 0) { cand[0][wave] = v; candi[0][wave] = vi; }
  }
  __syncthreads();
  double mx;
  {
    int dummy;
    mx = lane < NW ? cand[0][lane] : -INFINITY;
    dummy = lane < NW ? candi[0][lane] : 0x7fffffff;
    wave_argmax(mx, dummy);
  }
  const double thr = tol * mx;
  const bool zero = !(mx > 0.0);
  int rank = 0;
  for (int j = 0; j < r && !zero; ++j) {
    // the pivot: argmax over the NW candidates, read from the first lane
    double best = lane < NW ? cand[j & 1][lane] : -INFINITY;
    int p = lane < NW ? candi[j & 1][lane] : 0x7fffffff;
    group_argmax<NW>(best, p);
    best = read_first_lane(best);
    p = __builtin_amdgcn_readfirstlane(p);
    if (!(best > thr)) break;
    if (p != j) {
      // swap positions j and p among the remaining ones (rows and columns of
      // the packed trailing block), their diagonals, the pivot order, and
      // rows j and p of the columns of L already computed
      for (int x = j + 1 + threadIdx.x; x < r; x += NT) {
        if (x == p) continue;
        const int aj = packed(r, x, j);
        const int ap = packed(r, x > p ? x : p, x > p ? p : x);
        const double tmp = S[aj];
        S[aj] = S[ap];
        S[ap] = tmp;
      }
      for (int l = threadIdx.x; l < j; l += NT) {
        const int aj = packed(r, j, l), ap = packed(r, p, l);
        const double a = S[aj];
        S[aj] = S[ap];
        S[ap] = a;
      }
      if (threadIdx.x == 0) {
        const double a = S[packed(r, j, j)];
        S[packed(r, j, j)] = S[packed(r, p, p)];
        S[packed(r, p, p)] = a;
        const int b = perm[j];
        perm[j] = perm[p];
        perm[p] = b;
      }
      __syncthreads();
    }
    const double ljj = sqrt(S[packed(r, j, j)]);
    const double inv = 1.0 / ljj;
    const double* cj = S + packed(r, 0, j);   // column j (rows j..), not modified in this step
    // S(i, k) -= l_i l_k for j < k <= i, l_i = S(i, j) / l_jj: a wavefront per
    // column, lanes down it.  Row k of column k is lane 0's first row, so lane
    // 0 alone holds the wavefront's candidate for the next pivot (the largest
    // new diagonal, the first column on ties).  Two or four columns per pass
    // with their reads in flight together measured no faster.
    double v = -INFINITY;
    int vi = 0x7fffffff;
    for (int k = j + 1 + wave; k < r; k += NW) {
      const double lk = cj[k] * inv;
      double* col = S + packed(r, 0, k);
      for (int i = k + lane; i < r; i += 64) {
        const double x = col[i] - (cj[i] * inv) * lk;
        col[i] = x;
        if (i == k && x > v) { v = x; vi = k; }
      }
    }
    if (lane == 0) { cand[(j + 1) & 1][wave] = v; candi[(j + 1) & 1][wave] = vi; }
    __syncthreads();
    rank = j + 1;
  }
  // column j of L: the packed column j (rows moved with every later pivot)
  // over the square root of its pivot
  for (int j = 0; j < rank; ++j) {
    const double ljj = sqrt(S[packed(r, j, j)]);
    const double inv = 1.0 / ljj;
    const double* cj = S + packed(r, 0, j);
    for (int i = j + threadIdx.x; i < r; i += NT) L[i + (int64_t)j * r] = i == j ? ljj : cj[i] * inv;
  }
  for (int i = threadIdx.x; i < r; i += NT) {
    t.perm[i] = perm[i];
    t.d[perm[i]] = S[packed(r, i, i)];
  }
  if (threadIdx.x == 0) *t.rank_out = rank;
}

// Pivoted Cholesky with the Gram matrix held in registers and no row or column
// swaps.  The lower triangle (with the upper halves of the diagonal blocks,
// kept symmetric) is cut into TB x TB tiles, one per thread, fixed for the
// whole factorisation.  Step j: the pivot p is the remaining index with the
// largest diagonal (ties: the lowest position in the order the swap-based
// kernels produce, tracked in perm / posof); its column scaled by 1 / l_pp,
// with zeros at indices already eliminated, goes to LDS from the tiles that
// hold column p (row p left of the diagonal block); every tile then takes the
// rank-1 update S(i, k) -= l_i l_k (2 TB LDS reads and TB^2 multiply-adds per
// thread, the same arithmetic as the right-looking update), and the diagonal
// tiles propose the next pivot.  The columns of L are written in original row
// order into the Gram buffer, which is not read after the start, and gathered
// into pivot order at the end: the outputs are those of the swap-based kernels.
// The columns collect in LDS and go to global memory every kPcholChunk steps:
// a workgroup barrier waits for the thread's outstanding global stores, so a
// store per step would put a memory round trip into every step.
template <int NT, int TB>
__global__ __launch_bounds__(NT) void k_pchol_reg(const PcholTask* __restrict__ tasks, double tol) {
  extern __shared__ double spr[];
  const PcholTask t = tasks[blockIdx.x];
  const int r = t.r;
  double* lv = spr;                                // pivot column / l_pp, 0 at eliminated indices
  double* dpiv = lv + r;                           // diagonal of each pivot when it was taken
  double* lbuf = dpiv + r;                         // the last kPcholChunk columns of L
  int* perm = reinterpret_cast<int*>(lbuf + (int64_t)kPcholChunk * r);   // position -> original index
  int* posof = perm + r;                           // original index -> position
  int* alive = posof + r;                          // 1 until the index is eliminated
  constexpr int NW = NT / 64;
  __shared__ double cand[2][NW];
  __shared__ int candi[2][NW];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // this thread's tile: block row R >= block column C, tile index R (R + 1) / 2 + C
  const int nb = (r + TB - 1) / TB;
  int R = -1, C = -1;
  if ((int)threadIdx.x < nb * (nb + 1) / 2) {
    int rr = 0;
    while ((rr + 1) * (rr + 2) / 2 <= (int)threadIdx.x) ++rr;
    R = rr;
    C = (int)threadIdx.x - rr * (rr + 1) / 2;
  }
  const int i0 = R * TB, k0 = C * TB;
  const auto* Gg = to_global(t.G);
  double v[TB][TB];
#pragma unroll
  for (int a = 0; a < TB; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) {
      const int i = i0 + a, k = k0 + b;
      v[a][b] = (R >= 0 && i < r && k < r) ? Gg[i + (int64_t)k * r] : 0.0;
    }
  for (int x = threadIdx.x; x < r; x += NT) {
    perm[x] = x;
    posof[x] = x;
    alive[x] = 1;
  }
  // candidates: value and key position * 512 + original index (positions win ties)
  double cv = -INFINITY;
  int ck = 0x7fffffff;
  if (R >= 0 && R == C) {
#pragma unroll
    for (int a = 0; a < TB; ++a) {
      const int i = i0 + a;
      if (i < r && v[a][a] > cv) { cv = v[a][a]; ck = i * 512 + i; }
    }
  }
  wave_argmax(cv, ck);
  if (lane == 0) { cand[0][wave] = cv; candi[0][wave] = ck; }
  __syncthreads();
  double mx;
  {
    double m = lane < NW ? cand[0][lane] : -INFINITY;
    int mi = lane < NW ? candi[0][lane] : 0x7fffffff;
    group_argmax<NW>(m, mi);
    mx = read_first_lane(m);
  }
  const double thr = tol * mx;
  const bool zero = !(mx > 0.0);
  // the Gram buffer receives the columns of L in original row order
  auto* Lo = to_global(const_cast<double*>(t.G));
  unsigned dead = 0;   // this thread's diagonal entries already eliminated (bit a)
  // the rows i0 + a and columns k0 + c of this thread's tile eliminated by
  // earlier pivots (bit a / c): the pivot column is formed without reading
  // the shared flags
  unsigned rdead = 0, cdead = 0;
  int rank = 0;
  // columns j0 .. j0 + n - 1 of the LDS buffer to global memory
  auto flush = [&](int j0, int n) {
    for (int e = threadIdx.x; e < n * r; e += NT) {
      const int c = e / r, x = e - c * r;
      Lo[x + (int64_t)(j0 + c) * r] = lbuf[x + (int64_t)c * r];
    }
  };
  for (int j = 0; j < r && !zero; ++j) {
    if (j > 0 && j % kPcholChunk == 0) flush(j - kPcholChunk, kPcholChunk);
    double b = lane < NW ? cand[j & 1][lane] : -INFINITY;
    int bk = lane < NW ? candi[j & 1][lane] : 0x7fffffff;
    group_argmax<NW>(b, bk);
    b = read_first_lane(b);
    bk = __builtin_amdgcn_readfirstlane(bk);
    if (!(b > thr)) break;
    const int p = bk & 511, pb = p / TB;
    const double inv = 1.0 / sqrt(b);   // as 1 / l_pp in the swap-based kernels
    if (R >= 0 && C == pb) {
      // column p in the tiles of block column pb (rows at and below the block)
#pragma unroll
      for (int a = 0; a < TB; ++a) {
        const int i = i0 + a;
        double x = 0.0;
#pragma unroll
        for (int c = 0; c < TB; ++c) x = k0 + c == p ? v[a][c] : x;
        if (i < r) lv[i] = (i == p || !((rdead >> a) & 1u)) ? x * inv : 0.0;
      }
    }
    if (R >= 0 && R == pb && C < R) {
      // row p in the tiles left of the diagonal block: columns of the blocks before pb
#pragma unroll
      for (int c = 0; c < TB; ++c) {
        const int k = k0 + c;
        double x = 0.0;
#pragma unroll
        for (int a = 0; a < TB; ++a) x = i0 + a == p ? v[a][c] : x;
        if (k < r) lv[k] = !((cdead >> c) & 1u) ? x * inv : 0.0;
      }
    }
    if (p >= i0 && p < i0 + TB) rdead |= 1u << (p - i0);
    if (p >= k0 && p < k0 + TB) cdead |= 1u << (p - k0);
    if (threadIdx.x == 0) {
      dpiv[p] = b;
      const int q = posof[p], pj = perm[j];
      perm[j] = p;
      perm[q] = pj;
      posof[p] = j;
      posof[pj] = q;
      alive[p] = 0;
    }
    __syncthreads();
    // (the pivot's own entry is l_pp = sqrt(S(p, p)), not S(p, p) / l_pp)
    const double lpp = sqrt(b);
    double* lc = lbuf + (int64_t)(j % kPcholChunk) * r;
    for (int x = threadIdx.x; x < r; x += NT) lc[x] = x == p ? lpp : lv[x];
    cv = -INFINITY;
    ck = 0x7fffffff;
    if (R >= 0) {
      double li[TB], lk[TB];
#pragma unroll
      for (int a = 0; a < TB; ++a) {
        li[a] = i0 + a < r ? lv[i0 + a] : 0.0;
        lk[a] = k0 + a < r ? lv[k0 + a] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < TB; ++a)
#pragma unroll
        for (int c = 0; c < TB; ++c) v[a][c] -= li[a] * lk[c];
      if (R == C) {
#pragma unroll
        for (int a = 0; a < TB; ++a) {
          const int i = i0 + a;
          if (i == p) dead |= 1u << a;
          if (i < r && !((dead >> a) & 1u)) {
            const int key = posof[i] * 512 + i;
            if (v[a][a] > cv || (v[a][a] == cv && key < ck)) { cv = v[a][a]; ck = key; }
          }
        }
      }
    }
    wave_argmax(cv, ck);
    if (lane == 0) { cand[(j + 1) & 1][wave] = cv; candi[(j + 1) & 1][wave] = ck; }
    __syncthreads();
    rank = j + 1;
  }
  // the columns of the last, partial chunk
  if (rank > 0) flush((rank - 1) / kPcholChunk * kPcholChunk, rank - (rank - 1) / kPcholChunk * kPcholChunk);
  __syncthreads();
  auto* L = to_global(t.L);
  if (R >= 0 && R == C) {
#pragma unroll
    for (int a = 0; a < TB; ++a) {
      const int i = i0 + a;
      if (i < r) t.d[i] = alive[i] ? v[a][a] : dpiv[i];
    }
  }
  for (int x = threadIdx.x; x < r; x += NT) t.perm[x] = perm[x];
  for (int e = threadIdx.x; e < rank * r; e += NT) {
    const int a = e / r, q = e - a * r;
    if (q >= a) L[q + (int64_t)a * r] = Lo[perm[q] + (int64_t)a * r];
  }
  if (threadIdx.x == 0) *t.rank_out = rank;
}

__global__ __launch_bounds__(256) void k_materialize_r(const PcholTask* __restrict__ tasks) {
  __shared__ double tile[32][33];
  const PcholTask t = tasks[blockIdx.x];
  const int r = t.r, r1 = t.r1;
  const int nba = (r1 + 31) / 32, nbi = (r + 31) / 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // 32 x 32 tiles of R (rows a, pivot positions i): L read with consecutive
  // lanes on consecutive i, R written with consecutive lanes on consecutive a
  for (int tt = blockIdx.y; tt < nba * nbi; tt += gridDim.y) {
    const int ba = tt % nba, bi = tt / nba;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = bi * 32 + tx, a = ba * 32 + ty + 8 * k;
      tile[ty + 8 * k][tx] = (i < r && a < r1 && i >= a) ? t.L[i + (int64_t)a * r] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int a = ba * 32 + tx, i = bi * 32 + ty + 8 * k;
      if (a < r1 && i < r) t.R[a + (int64_t)t.perm[i] * r1] = tile[tx][ty + 8 * k];
    }
    __syncthreads();
  }
}

// W = P1 L11^{-T} Z scattered into r x k (precision T): blocked back
// substitution, one workgroup per (task, chunk of kc right-hand sides) with
// the chunk of Z in LDS.  Each 32-row diagonal block is staged in LDS (with
// the reciprocals of its diagonal) and solved by the first wavefront, one lane
// per right-hand side with the block's 32 entries in registers, right-looking,
// then subtracted from the rows above it by the whole workgroup.  LDS:
// r1 * kc + 32 * 32 doubles.
template <class T>
__global__ __launch_bounds__(256) void k_wtilde(const WtTask* __restrict__ tasks, int kc) {
  extern __shared__ double zs[];
  const WtTask t = tasks[blockIdx.x];
  const int r = t.r, r1 = t.r1, k = t.k;
  const int c0 = blockIdx.y * kc;
  if (c0 >= k) return;
  const int nc = k - c0 < kc ? k - c0 : kc;
  const double* L = t.L;
  staged_copy<256>(
      (int64_t)r1 * nc, [&](int64_t e) { return t.Z[(int)e % r1 + (int64_t)(c0 + (int)e / r1) * t.ldz]; },
      [&](int64_t e, double v) { zs[e] = v; });
  __syncthreads();
  double* Ld = zs + (int64_t)r1 * kc;   // diagonal block: Ld[i + c * 32] = L(lo + i, lo + c)
  __shared__ double rd[32];             // 1 / L(lo + i, lo + i)
  for (int hi = r1; hi > 0; hi -= 32) {
    const int lo = hi - 32 > 0 ? hi - 32 : 0;
    const int h = hi - lo;
    for (int e = threadIdx.x; e < h * h; e += 256) {
      const int i = e % h, c = e / h;
      if (i >= c) {
        const double v = L[(lo + i) + (int64_t)(lo + c) * r];
        Ld[i + c * 32] = v;
        if (i == c) rd[i] = 1.0 / v;
      }
    }
    __syncthreads();
    if (threadIdx.x < nc) {
      // right-looking: once z[a] is final, its term L(a, b) z[a] leaves every
      // row b < a of the block at once (independent updates of the block's z
      // held in registers, instead of a dependent dot product per row)
      double* z = zs + threadIdx.x * r1 + lo;
      double zr[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) zr[u] = u < h ? z[u] : 0.0;
#pragma unroll
      for (int a = 31; a >= 0; --a) {
        if (a < h) {
          const double za = zr[a] * rd[a];
          zr[a] = za;
#pragma unroll
          for (int b = 0; b < a; ++b) zr[b] = fma(-Ld[a + b * 32], za, zr[b]);
        }
      }
#pragma unroll
      for (int u = 0; u < 32; ++u)
        if (u < h) z[u] = zr[u];
    }
    __syncthreads();
    // z[b, c] -= sum over a in [lo, hi) of L(a, b) z[a, c] for b < lo: a thread
    // per (b, group of kWtCols columns) reads L(lo..hi, b) once into registers
    // for the whole group (one read per column before)
    {
      constexpr int kWtCols = 4;
      const int ng = (nc + kWtCols - 1) / kWtCols;
      for (int e = threadIdx.x; e < lo * ng; e += 256) {
        const int b = e % lo, g = e / lo;
        const double* lb = L + (int64_t)b * r + lo;   // lb[u] = L(lo + u, b)
        double lv[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) lv[u] = u < h ? lb[u] : 0.0;
        const int cend = nc < (g + 1) * kWtCols ? nc : (g + 1) * kWtCols;
        for (int c = g * kWtCols; c < cend; ++c) {
          const double* z = zs + c * r1 + lo;
          double s = 0.0;
#pragma unroll
          for (int u = 0; u < 32; ++u)
            if (u < h) s += lv[u] * z[u];
          zs[b + c * r1] -= s;
        }
      }
    }
    __syncthreads();
  }
  T* W = static_cast<T*>(t.W);
  for (int e = threadIdx.x; e < r * nc; e += 256) {
    const int a = e % r, c = e / r;
    W[t.perm[a] + (int64_t)(c0 + c) * r] = a < r1 ? T(zs[a + c * r1]) : T(0);
  }
}

}  // namespace

template <class T>
void launch_gram(const GramTask* d_tasks, int ntasks, const int* d_tile_task, const int* d_first_tile, int ntiles,
                 int reduce_wgs, hipStream_t s) {
  if (ntasks <= 0) return;
  launch_gram_mfma<T>(d_tasks, d_tile_task, d_first_tile, ntiles, s);
  hipLaunchKernelGGL(k_gram_reduce, dim3(ntasks, reduce_wgs), dim3(256), 0, s, d_tasks);
}

void launch_pchol(const PcholTask* d_tasks, int ntasks, int max_r, double tol, size_t lds_packed, hipStream_t s) {
  if (ntasks <= 0) return;
  if (lds_packed > 0) {
    // small Gram matrices in 256-thread workgroups (several per compute unit)
    if (lds_packed <= kSmallLds) {
      hipLaunchKernelGGL(k_pchol_lds<256>, dim3(ntasks), dim3(256), lds_packed, s, d_tasks, tol);
      return;
    }
    if (lds_packed > 64 * 1024)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_pchol_lds<1024>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_packed);
    hipLaunchKernelGGL(k_pchol_lds<1024>, dim3(ntasks), dim3(1024), lds_packed, s, d_tasks, tol);
    return;
  }
  const size_t lds = (size_t)max_r * (sizeof(double) + sizeof(int));
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_pchol<1024>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_pchol<1024>, dim3(ntasks), dim3(1024), lds, s, d_tasks, tol);
}

void launch_pchol_reg(const PcholTask* d_tasks, int ntasks, int max_r, double tol, int kind, hipStream_t s) {
  if (ntasks <= 0) return;
  const size_t lds = lds_bytes_pchol_reg(max_r);
  if (lds > 64 * 1024) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_pchol_reg<256, 4>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_pchol_reg<512, 8>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_pchol_reg<512, 5>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_pchol_reg<1024, 5>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  }
  if (kind == 0)
    hipLaunchKernelGGL((k_pchol_reg<256, 4>), dim3(ntasks), dim3(256), lds, s, d_tasks, tol);
  else if (kind == 1)
    hipLaunchKernelGGL((k_pchol_reg<512, 8>), dim3(ntasks), dim3(512), lds, s, d_tasks, tol);
  else if (kind == 3)
    hipLaunchKernelGGL((k_pchol_reg<512, 5>), dim3(ntasks), dim3(512), lds, s, d_tasks, tol);
  else
    hipLaunchKernelGGL((k_pchol_reg<1024, 5>), dim3(ntasks), dim3(1024), lds, s, d_tasks, tol);
}

void launch_materialize_r(const PcholTask* d_tasks, int ntasks, int wgs, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_materialize_r, dim3(ntasks, wgs), dim3(256), 0, s, d_tasks);
}

template <class T>
void launch_wtilde(const WtTask* d_tasks, int ntasks, int kc, int nchunks, size_t lds, hipStream_t s) {
  if (ntasks <= 0 || nchunks <= 0) return;
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_wtilde<T>), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  hipLaunchKernelGGL(k_wtilde<T>, dim3(ntasks, nchunks), dim3(256), lds, s, d_tasks, kc);
}

template void launch_gram<float>(const GramTask*, int, const int*, const int*, int, int, hipStream_t);
template void launch_gram<double>(const GramTask*, int, const int*, const int*, int, int, hipStream_t);
template void launch_wtilde<float>(const WtTask*, int, int, int, size_t, hipStream_t);
template void launch_wtilde<double>(const WtTask*, int, int, int, size_t, hipStream_t);

}  // namespace acr
