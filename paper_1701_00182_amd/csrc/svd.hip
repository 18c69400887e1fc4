// Truncated SVD of the compression core C = Ru Rv^T (FP64).
//
// Stage 1: Householder QR with column pivoting of C, stopped when the
// Frobenius norm of the remaining block drops below delta times the largest
// initial column norm; C P ~= Q R with R = [R11 R12] (t x q).  Stage 2: one-sided Jacobi on the t
// rows of R, whose singular values are those of C up to the dropped tail.  QR
// with column pivoting both removes the directions far below the truncation
// level and preconditions the Jacobi iteration, which then converges in a few
// sweeps.  The right singular vectors are the normalised rotated rows (mapped
// back through P); the left factor is recomputed as C Zv = U Sigma by
// k_core_left, all kept columns at once.
//
// Cores whose C is small run both stages in one workgroup with R rotated in
// place (k_svd_wave: one wavefront, lane per column, for p, q, r <= 64;
// k_svd_block up to kFusedLds bytes); larger ones take the pivoted QR (C in
// LDS when it fits, else in global memory) and then k_jacobi on the smaller
// W^T = P R^T (q x t), in LDS when it fits.

#include <cmath>

#include "kern.h"
#include "wave.h"

namespace acr {

namespace {

using dbl4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;

__device__ inline double gsum2(double v, int G) {
  for (int off = G >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

// 1 / sqrt(x) for x > 0 from the hardware estimate and two Newton steps
// (each squares the relative error).
__device__ inline double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x * r, r, 1.5);
  r = r * fma(-0.5 * x * r, r, 1.5);
  return r;
}

// 1 / x from the hardware estimate and two Newton steps.
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

__device__ inline double wsum(double v) { return gsum_dpp(v, 64); }

__device__ inline double wmax(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// wavefront argmax of (v, i); ties go to the smaller index
__device__ inline void wargmax(double& v, int& i) { wave_argmax(v, i); }

// workgroup reductions: shuffles inside each wavefront, then one slot per
// wavefront in LDS read back by every thread (all threads must call them)
template <int NT> __device__ inline double block_sum(double v, double* red) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const int l = threadIdx.x & 63;
  return wsum(l < NT / 64 ? red[l] : 0.0);
}

template <int NT> __device__ inline void block_argmax(double& v, int& i, double* red, int* redi) {
  wargmax(v, i);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) { red[threadIdx.x >> 6] = v; redi[threadIdx.x >> 6] = i; }
  __syncthreads();
  // every wavefront combines the per-wavefront results in parallel
  const int l = threadIdx.x & 63;
  v = l < NT / 64 ? red[l] : -INFINITY;
  i = l < NT / 64 ? redi[l] : 0x7fffffff;
  wargmax(v, i);
}

// Lanes per column group for one step of a Householder sweep over `cols`
// trailing columns of `rows` live rows with nt threads: enough groups to take
// every column at once (short shuffle reductions, no column queue per group),
// and enough lanes that a column slice fits `cap` registers.
__device__ inline int step_lanes(int rows, int cols, int nt, int cap) {
  int G = 4;
  while (G < 64 && 2 * G * cols <= nt) G <<= 1;
  while (G < 64 && rows > G * cap) G <<= 1;
  return G;
}

// The core C = Ru Rv^T (p x q, column stride lc) on the FP64 matrix cores:
// the wavefronts take 16 x 16 tiles; lane l feeds Ru[i0 + l%16][k] and
// Rv[j0 + l%16][k] for k = k0 + l/16 (T widened to FP64, so the products are
// exact and the sums FP64) and receives C[i0 + l/16 + 4v][j0 + l%16].  Mode 0
// panels are upper trapezoidal: entries below their diagonal (which hold
// other data) load as zero, and a tile's sum starts at k = max(i0, j0).
template <class T, int NT>
__device__ __forceinline__ void core_product_mfma(const SvdTask& t, double* C, int64_t lc) {
  const int p = t.p, q = t.q, r = t.r;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ti = (p + 15) / 16, tj = (q + 15) / 16;
  for (int tile = wave; tile < ti * tj; tile += NT / 64) {
    const int i0 = (tile % ti) * 16, j0 = (tile / ti) * 16;
    const int a = i0 + li, b = j0 + li;
    const int ac = a < p ? a : p - 1, bc = b < q ? b : q - 1;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    const int kstart = t.mode == 0 ? ((i0 > j0 ? i0 : j0) & ~3) : 0;
    for (int k0 = kstart; k0 < r; k0 += 16) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + 4 * u + lk;
        const int kc = k < r ? k : r - 1;
        double x, y;
        if (t.mode == 0) {
          x = (double)static_cast<const T*>(t.Ru)[ac + (int64_t)kc * t.ldu];
          y = (double)static_cast<const T*>(t.Rv)[bc + (int64_t)kc * t.ldv];
        } else {
          x = static_cast<const double*>(t.Ru)[ac + (int64_t)kc * t.ldu];
          y = static_cast<const double*>(t.Rv)[bc + (int64_t)kc * t.ldv];
        }
        av[u] = (a < p && k < r && (t.mode != 0 || a <= k)) ? x : 0.0;
        bv[u] = (b < q && k < r && (t.mode != 0 || b <= k)) ? y : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = i0 + lk + 4 * v, col = j0 + li;
      if (row < p && col < q) C[row + (int64_t)col * lc] = acc[v];
    }
  }
}

// Reflector j of the pivoted QR, v = (1, x_{j+1..} * scale) with factor tj,
// applied to the columns in pivot positions j+1.. (column colp[c] of C, with
// this step's exchange of positions j and pc applied; groups of G lanes, one
// column per group at a time), and the squared norms of their rows j+1..
// written to nrm by position.  With NU > 0 each lane holds NU = ceil((p - j) / G) rows of v and of
// the column in registers and the loops unroll without branches: rows of
// lanes before the last are full, the last one loads through a clamped index
// and stores under a mask.  NU = 0 streams the rows.
template <int NT, int NU>
__device__ __forceinline__ void qrcp_update(double* C, int64_t lc, int p, int q, int j, const double* col,
                                            double scale, double tj, int G, double* nrm, const int* colp, int pc) {
  const int groups = NT / G, gi = threadIdx.x / G, gl = threadIdx.x % G;
  // column at position c > j: the map before this step's pivot exchange
  auto column = [&](int c) { return C + (int64_t)(c == pc ? colp[j] : colp[c]) * lc; };
  if (NU == 0) {
    for (int c = j + 1 + gi; c < q; c += groups) {
      double* ac = column(c);
      if (tj != 0.0) {
        double w = 0.0;
        for (int i = j + gl; i < p; i += G) w += (i == j ? 1.0 : col[i] * scale) * ac[i];
        w = gsum_dpp(w, G) * tj;
        for (int i = j + gl; i < p; i += G) ac[i] -= w * (i == j ? 1.0 : col[i] * scale);
      }
      double s = 0.0;
      for (int i = j + 1 + gl; i < p; i += G) s += ac[i] * ac[i];
      s = gsum_dpp(s, G);
      if (gl == 0) nrm[c] = s;
    }
    return;
  }
  constexpr int R = NU > 0 ? NU : 1;
  const int il = j + gl + (R - 1) * G;
  const bool tail_ok = il < p;
  const int ic = tail_ok ? il : j;
  double v[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const double x = u + 1 < R ? col[j + gl + u * G] : col[ic];
    const double vv = (u == 0 && gl == 0) ? 1.0 : x * scale;
    v[u] = (u + 1 < R || tail_ok) ? vv : 0.0;
  }
  for (int c = j + 1 + gi; c < q; c += groups) {
    double* ac = column(c);
    double a[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const double x = u + 1 < R ? ac[j + gl + u * G] : ac[ic];
      a[u] = (u + 1 < R || tail_ok) ? x : 0.0;
    }
    if (tj != 0.0) {
      double w = 0.0;
#pragma unroll
      for (int u = 0; u < R; ++u) w = fma(v[u], a[u], w);
      w = gsum_dpp(w, G) * tj;
#pragma unroll
      for (int u = 0; u < R; ++u) a[u] = fma(-w, v[u], a[u]);
#pragma unroll
      for (int u = 0; u + 1 < R; ++u) ac[j + gl + u * G] = a[u];
      if (tail_ok) ac[il] = a[R - 1];
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < R; ++u) s = (u == 0 && gl == 0) ? s : fma(a[u], a[u], s);
    s = gsum_dpp(s, G);
    if (gl == 0) nrm[c] = s;
  }
}

// Householder QR with column pivoting of C (p x q, column stride lc), stopped
// before step j once the trailing block (rows and columns j..) has Frobenius
// norm at most delta times the largest column norm of C; returns the number of
// reflectors t.  The columns are not moved: the column of R in pivot position
// c is column colp[c] of C (rows a <= c of it, for a < t; the entries below
// are left unspecified), and perm[c] is its original index.  All threads call
// it.  Column slices of up to CAP rows per lane are held in
// registers.
template <int NT, int CAP>
__device__ __forceinline__ int qrcp_body(double* C, int64_t lc, int p, int q, double* nrm, int* perm, int* colp,
                                         double delta, double* red, int* redi) {
  const int mn = p < q ? p : q;
  double mx = 0.0;
  {
    const int G = step_lanes(p, q, NT, CAP), groups = NT / G;
    const int gi = threadIdx.x / G, gl = threadIdx.x % G;
    for (int c = gi; c < q; c += groups) {
      double s = 0.0;
      for (int i = gl; i < p; i += G) s += C[i + c * lc] * C[i + c * lc];
      s = gsum2(s, G);
      if (gl == 0) { nrm[c] = s; perm[c] = c; colp[c] = c; }
      mx = fmax(mx, s);
    }
  }
  {
    int dummy = 0;
    block_argmax<NT>(mx, dummy, red, redi);
  }
  // stop when the Frobenius norm of the remaining block (rows and columns j..)
  // is at most delta * (largest column norm): nrm holds its column norms
  const double thr2 = delta * delta * mx;
  // per-wavefront pivot candidates and partial sums, double buffered by step
  // parity: a buffer is written again two steps later, after barriers that
  // every reader of it has passed, so no barrier is needed before the writes
  constexpr int NW = NT / 64;
  __shared__ double cv[2][NW], cs[2][NW];
  __shared__ int ci[2][NW];
  const int lane = threadIdx.x & 63;
  int tcount = 0;
  for (int j = 0; j < mn; ++j) {
    double best = -1.0, rest = 0.0;
    int bc = j;
    for (int c = j + threadIdx.x; c < q; c += NT) {
      rest += nrm[c];
      if (nrm[c] > best) { best = nrm[c]; bc = c; }
    }
    wargmax(best, bc);
    rest = wsum(rest);
    if (lane == 0) { cv[j & 1][threadIdx.x >> 6] = best; ci[j & 1][threadIdx.x >> 6] = bc; cs[j & 1][threadIdx.x >> 6] = rest; }
    __syncthreads();
    // the NW candidates combined in log2(NW) steps, read from the first lane
    best = lane < NW ? cv[j & 1][lane] : -INFINITY;
    bc = lane < NW ? ci[j & 1][lane] : 0x7fffffff;
    rest = lane < NW ? cs[j & 1][lane] : 0.0;
    group_argmax<NW>(best, bc);
    rest = gsum_dpp(rest, NW);
    best = read_first_lane(best);
    bc = __builtin_amdgcn_readfirstlane(bc);
    rest = read_first_lane(rest);
    if (!(rest > thr2) || !(best > 0.0)) break;
    // the pivot takes position j without moving data: the columns stay where
    // they are and positions j and pc exchange their entries of the map colp
    // (and of perm) after this step's last barrier; until then every thread
    // reads the old map with the exchange applied.  The norms need no
    // exchange: position pc's entry is rewritten by this step's update (its
    // column is then the one that was at position j) and position j's is not
    // read again.
    const int pc = bc;
    // Householder reflector of the pivot column from its stored norm (best):
    // the squared norm of rows j.. (recomputed exactly after the previous
    // step), so the part below the diagonal is best - x0^2 without another
    // reduction.  The reflector v = (1, x_{j+1..} * scale) is applied on the
    // fly and not stored: only R is used afterwards.
    double* col = C + (int64_t)colp[pc] * lc;
    const double x0 = col[j];
    const double sigma = fmax(best - x0 * x0, 0.0);
    double tj = 0.0, scale = 0.0, beta = x0;
    if (sigma > 0.0) {
      const double nr = sqrt(x0 * x0 + sigma);
      beta = x0 >= 0.0 ? -nr : nr;
      tj = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    // trailing columns: group size for this step, each lane's slice of the
    // reflector and of the column held in registers when it fits
    const int G = step_lanes(p - j, q - j - 1, NT, CAP);
    const int nu = (p - j + G - 1) / G;
    switch (nu <= CAP ? nu : 0) {
#define ACR_QRCP_NU(k) \
  case k: qrcp_update<NT, (k <= CAP ? k : 0)>(C, lc, p, q, j, col, scale, tj, G, nrm, colp, pc); break;
      ACR_QRCP_NU(1) ACR_QRCP_NU(2) ACR_QRCP_NU(3) ACR_QRCP_NU(4) ACR_QRCP_NU(5) ACR_QRCP_NU(6)
      ACR_QRCP_NU(7) ACR_QRCP_NU(8) ACR_QRCP_NU(9) ACR_QRCP_NU(10) ACR_QRCP_NU(11) ACR_QRCP_NU(12)
      ACR_QRCP_NU(13) ACR_QRCP_NU(14) ACR_QRCP_NU(15) ACR_QRCP_NU(16)
#undef ACR_QRCP_NU
      default: qrcp_update<NT, 0>(C, lc, p, q, j, col, scale, tj, G, nrm, colp, pc); break;
    }
    __syncthreads();
    // every thread has read x0, the column and the map: the diagonal of R can
    // be stored and the exchange committed (the next reads of colp and perm
    // follow the next step's first barrier)
    if (threadIdx.x == 0) {
      col[j] = beta;
      if (pc != j) {
        const int b = perm[j];
        perm[j] = perm[pc];
        perm[pc] = b;
        const int d = colp[j];
        colp[j] = colp[pc];
        colp[pc] = d;
      }
    }
    tcount = j + 1;
  }
  __syncthreads();
  return tcount;
}

// Pivoted QR of cores that do not take the one-workgroup path, with C in LDS
// (ld p|1, then q norms and q pivots) or in the global workspace; writes
// W^T = P R^T (q x t) to Y for k_jacobi.
template <class T, bool LDS, int NT>
__global__ __launch_bounds__(NT) void k_qrcp(const SvdTask* __restrict__ tasks, double delta) {
  extern __shared__ double smc[];
  const SvdTask t = tasks[blockIdx.x];
  const int p = t.p, q = t.q;
  if (p == 0 || q == 0) {
    if (threadIdx.x == 0) *t.t_out = 0;
    return;
  }
  const int lc = LDS ? (p | 1) : p;
  double* C = LDS ? smc : t.C;
  double* nrm = LDS ? smc + (int64_t)lc * q : t.sig;
  int* perm = LDS ? reinterpret_cast<int*>(nrm + q) : t.perm;
  // position -> column map: after perm in LDS, else all of the dynamic LDS
  int* colp = LDS ? perm + q : reinterpret_cast<int*>(smc);
  __shared__ double red[NT / 64];
  __shared__ int redi[NT / 64];
  core_product_mfma<T, NT>(t, C, lc);
  __syncthreads();
  const int tcount = qrcp_body<NT, LDS ? 12 : 8>(C, lc, p, q, nrm, perm, colp, delta, red, redi);
  double* Wt = t.Y;
  for (int64_t e = threadIdx.x; e < (int64_t)q * tcount; e += NT) {
    const int c = (int)(e % q), a = (int)(e / q);
    Wt[perm[c] + (int64_t)a * q] = c >= a ? C[a + (int64_t)colp[c] * lc] : 0.0;
  }
  if (threadIdx.x == 0) *t.t_out = tcount;
}

// Jacobi rotation of the vector pair (x, y) with squared norms al, be and
// inner product ga that zeroes the inner product; false when the pair is
// already orthogonal to the tolerance, |ga| <= tol sqrt(al be).  The tangent
// of the smaller angle, t = sign(z) / (|z| + sqrt(1 + z^2)) with
// z = (be - al) / (2 ga), is t = s w / (|d| + h) with d = be - al, w = 2 |ga|,
// h = sqrt(d^2 + w^2) and s = sign(z); so cos = c' / r and sin = s w / r with
// c' = |d| + h and r = sqrt(c'^2 + w^2).  d and w are first scaled by a power
// of two that brings the larger to [0.5, 1), which keeps every square in range
// and both roots away from zero.
__device__ inline bool jacobi_rotation(double al, double be, double ga, double tol, double& cs, double& sn) {
  if (ga == 0.0 || !(ga * ga > tol * tol * (al * be))) return false;
  const double dd = be - al, w0 = 2.0 * fabs(ga);
  int e;
  (void)frexp(fmax(fabs(dd), w0), &e);
  const double d = ldexp(fabs(dd), -e), w = ldexp(w0, -e);
  const double h2 = fma(d, d, w * w);
  const double cp = d + h2 * rsqrt_nr(h2);
  const double r = rsqrt_nr(fma(cp, cp, w * w));
  // sign(z) = sign(d) sign(ga), and +1 for d = 0
  const bool neg = (dd < 0.0) != (ga < 0.0) && dd != 0.0;
  cs = cp * r;
  sn = neg ? -(w * r) : w * r;
  return true;
}

// Indices of pair pi in round `round` of the cyclic tournament over ne (even)
// vectors: vector 0 stays at position 0, position p >= 1 holds vector
// ((p - 1 + round) mod (ne - 1)) + 1; the sum is below 2 (ne - 1), so the
// modulo is one conditional subtraction.
__device__ inline void tournament_pair(int pi, int round, int ne, int& ia, int& ib) {
  const int m = ne - 1;
  int xa = pi - 1 + round, xb = ne - 2 - pi + round;
  xa -= xa >= m ? m : 0;
  xb -= xb >= m ? m : 0;
  const int a = pi == 0 ? 0 : xa + 1, b = xb + 1;
  ia = a < b ? a : b;
  ib = a < b ? b : a;
}

// Squared |cos| of a pair (its normalised inner product), for the stopping rule.
__device__ inline double pair_cos2(double al, double be, double ga) {
  const double ab = al * be;
  return ab > 0.0 ? ga * ga * rcp_nr(ab) : 0.0;
}

// 1 when a pair's squared |cos| exceeds tol (the stopping rule of the scalar
// sweeps only asks whether any pair does), else 0: no division per pair.
__device__ inline double pair_over(double al, double be, double ga, double tol) {
  const double ab = al * be;
  return ab > 0.0 && ga * ga > tol * ab ? 1.0 : 0.0;
}

// One Jacobi step on the vector pair (xa, xb) of length len (element i at
// index i * st), handled by the G lanes of a group (gl = lane in group): the
// three inner products, the rotation and its application.  With NU > 0 every
// lane holds NU = ceil(len / G) elements of each vector in registers between
// the products and the update, and the loops unroll without branches: rows of
// lanes before the last are full, the last one loads through a clamped index
// and stores under a mask.  NU = 0 streams the vectors twice.  Returns whether
// a rotation was applied; cmax2 becomes 1 when the pair's squared |cos| before
// it exceeds tol.
template <int NU>
__device__ __forceinline__ bool jacobi_pair(double* xa, double* xb, int st, int len, int G, int gl, double tol,
                                   double& cmax2) {
  double al = 0.0, be = 0.0, ga = 0.0;
  if (NU == 0) {
    for (int i = gl; i < len; i += G) {
      const double x = xa[i * st], y = xb[i * st];
      al += x * x;
      be += y * y;
      ga += x * y;
    }
    gsum3_dpp(al, be, ga, G);
    cmax2 = fmax(cmax2, pair_over(al, be, ga, tol));
    double cs, sn;
    if (!jacobi_rotation(al, be, ga, tol, cs, sn)) return false;
    for (int i = gl; i < len; i += G) {
      const double x = xa[i * st], y = xb[i * st];
      xa[i * st] = cs * x - sn * y;
      xb[i * st] = sn * x + cs * y;
    }
    return true;
  }
  constexpr int R = NU > 0 ? NU : 1;
  double xr[R], yr[R];
  const int il = gl + (R - 1) * G;
  const bool tail_ok = il < len;
#pragma unroll
  for (int u = 0; u < R; ++u) {
    if (u + 1 < R) {
      xr[u] = xa[(gl + u * G) * st];
      yr[u] = xb[(gl + u * G) * st];
    } else {
      const int ic = tail_ok ? il : len - 1;
      const double x = xa[ic * st], y = xb[ic * st];
      xr[u] = tail_ok ? x : 0.0;
      yr[u] = tail_ok ? y : 0.0;
    }
  }
#pragma unroll
  for (int u = 0; u < R; ++u) {
    al = fma(xr[u], xr[u], al);
    be = fma(yr[u], yr[u], be);
    ga = fma(xr[u], yr[u], ga);
  }
  gsum3_dpp(al, be, ga, G);
  cmax2 = fmax(cmax2, pair_over(al, be, ga, tol));
  double cs, sn;
  if (!jacobi_rotation(al, be, ga, tol, cs, sn)) return false;
#pragma unroll
  for (int u = 0; u + 1 < R; ++u) {
    xa[(gl + u * G) * st] = cs * xr[u] - sn * yr[u];
    xb[(gl + u * G) * st] = sn * xr[u] + cs * yr[u];
  }
  if (tail_ok) {
    xa[il * st] = cs * xr[R - 1] - sn * yr[R - 1];
    xb[il * st] = sn * xr[R - 1] + cs * yr[R - 1];
  }
  return true;
}

// The sweeps of jacobi_svd for NU elements per lane (0: streamed); returns
// the number of sweeps run and adds the flops done to `work`: the three inner
// products of every pair visit (6 len) and the rotation of the pairs that
// were rotated (6 len).
template <int NT, int NU>
__device__ __forceinline__ int jacobi_sweeps(double* V, int64_t vs, int64_t es, int n, int len, int G, double tol, double* red,
                             int* redi, double& work) {
  const int ne = n + (n & 1), npairs = ne / 2;
  const int groups = NT / G;
  const int gi = threadIdx.x / G, gl = threadIdx.x % G;
  int sweeps = 0;
  double nrot = 0.0;
  // Sweeps end when one applies no rotation, or when its largest |cos| was at
  // most sqrt(tol): convergence is quadratic there, so the pairs are left
  // orthogonal to about tol and the confirming sweep is skipped.
  for (int sweep = 0; sweep < 60 && n > 1; ++sweep) {
    ++sweeps;
    int rot = 0;
    double cmax2 = 0.0;
    for (int round = 0; round < ne - 1; ++round) {
      for (int pi = gi; pi < npairs; pi += groups) {
        int ia, ib;
        tournament_pair(pi, round, ne, ia, ib);
        if (ib >= n) continue;
        if (jacobi_pair<NU>(V + ia * vs, V + ib * vs, (int)es, len, G, gl, tol, cmax2)) {
          rot = 1;
          nrot += gl == 0 ? 1.0 : 0.0;
        }
      }
      __syncthreads();
    }
    if (!__syncthreads_or(rot)) break;
    // no pair of this sweep had squared |cos| above tol: quadratic convergence
    // leaves every pair within about tol of orthogonal
    if (!__syncthreads_or(cmax2 > 0.0)) break;
  }
  const double rots = block_sum<NT>(nrot, red);
  work += 6.0 * (double)len * ((double)sweeps * 0.5 * (double)n * (double)(n - 1) + rots);
  return sweeps;
}

// Block bounds [lo, hi) of block k at level l of the recursive halving of
// [0, n) (first half = ceil): the bits of k, most significant first, pick the
// half at each of the l splits.
__device__ inline void rec_block(int n, int l, int k, int& lo, int& hi) {
  lo = 0;
  hi = n;
  for (int d = l - 1; d >= 0; --d) {
    const int mid = lo + (hi - lo + 1) / 2;
    if ((k >> d) & 1) lo = mid;
    else hi = mid;
  }
}

// The sweeps of jacobi_svd for NU > 0 elements per lane in the recursive
// pairing order: at level l = 0, 1, ... the columns are cut into 2^l blocks
// by repeated halving, and in every block the first half S1 meets every
// vector of the second half S2 in |S1| rounds (round r pairs S1[g] with
// S2[(g + r) mod |S1|]).  Every pair is visited once per sweep, in n - 1 to
// about n + log2(n) rounds.  While a level's groups fit the workgroup, each
// group keeps its S1 vector in registers for the whole level and only the S2
// vectors go through memory: one vector loaded and stored per pair and round
// instead of two.  (Measured on pivoted-QR-preconditioned cores the order
// also converges in fewer sweeps than the round-robin tournament.)  Returns
// the number of sweeps and adds the flops to `work` as jacobi_sweeps does.
template <int NT, int NU>
__device__ __forceinline__ int jacobi_sweeps_rec(double* V, int64_t vs, int64_t es, int n, int len, int G,
                                                 double tol, double* red, int* redi, double& work) {
  const int groups = NT / G;
  const int gi0 = threadIdx.x / G, gl = threadIdx.x % G;
  const int st = (int)es;
  const int il = gl + (NU - 1) * G;
  const bool tail_ok = il < len;
  auto load = [&](const double* x, double (&r)[NU]) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      if (u + 1 < NU) {
        r[u] = x[(gl + u * G) * st];
      } else {
        const double v = x[(tail_ok ? il : len - 1) * st];
        r[u] = tail_ok ? v : 0.0;
      }
    }
  };
  auto store = [&](double* x, const double (&r)[NU]) {
#pragma unroll
    for (int u = 0; u + 1 < NU; ++u) x[(gl + u * G) * st] = r[u];
    if (tail_ok) x[il * st] = r[NU - 1];
  };
  // one pair step on register slices xr, yr; true when rotated
  auto step = [&](double (&xr)[NU], double (&yr)[NU], double& cmax2) {
    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      al = fma(xr[u], xr[u], al);
      be = fma(yr[u], yr[u], be);
      ga = fma(xr[u], yr[u], ga);
    }
    gsum3_dpp(al, be, ga, G);
    cmax2 = fmax(cmax2, pair_over(al, be, ga, tol));
    double cs, sn;
    if (!jacobi_rotation(al, be, ga, tol, cs, sn)) return false;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const double x = xr[u], y = yr[u];
      xr[u] = cs * x - sn * y;
      yr[u] = sn * x + cs * y;
    }
    return true;
  };
  int sweeps = 0;
  double nrot = 0.0;
  double xr[NU], yr[NU];
  for (int sweep = 0; sweep < 60 && n > 1; ++sweep) {
    ++sweeps;
    int rot = 0;
    double cmax2 = 0.0;
    for (int l = 0;; ++l) {
      const int smax = (n + (1 << l) - 1) >> l;   // largest block at level l
      if (smax <= 1) break;
      const int m = (smax + 1) / 2, ng = (1 << l) * m;
      if (ng <= groups) {
        int lo = 0, hi = 0, g = gi0 % m;
        bool act = gi0 < ng;
        if (act) rec_block(n, l, gi0 / m, lo, hi);
        const int mid = lo + (hi - lo + 1) / 2;
        act = act && hi - lo > 1 && lo + g < mid;
        if (act) load(V + (lo + g) * vs, xr);
        for (int r = 0; r < m; ++r) {
          if (act && r < mid - lo) {
            const int j = (g + r) % (mid - lo);
            if (mid + j < hi) {
              double* yb = V + (mid + j) * vs;
              load(yb, yr);
              if (step(xr, yr, cmax2)) {
                store(yb, yr);
                rot = 1;
                nrot += gl == 0 ? 1.0 : 0.0;
              }
            }
          }
          __syncthreads();
        }
        if (act) store(V + (lo + g) * vs, xr);
        __syncthreads();
      } else {
        // more groups than the workgroup holds (the last levels, a round or
        // two each): both vectors of a pair through memory
        for (int r = 0; r < m; ++r) {
          for (int gi = gi0; gi < ng; gi += groups) {
            int lo, hi;
            const int g = gi % m;
            rec_block(n, l, gi / m, lo, hi);
            const int mid = lo + (hi - lo + 1) / 2;
            if (hi - lo <= 1 || lo + g >= mid || r >= mid - lo) continue;
            const int j = (g + r) % (mid - lo);
            if (mid + j >= hi) continue;
            double* xb = V + (lo + g) * vs;
            double* yb = V + (mid + j) * vs;
            load(xb, xr);
            load(yb, yr);
            if (step(xr, yr, cmax2)) {
              store(xb, xr);
              store(yb, yr);
              rot = 1;
              nrot += gl == 0 ? 1.0 : 0.0;
            }
          }
          __syncthreads();
        }
      }
    }
    if (!__syncthreads_or(rot)) break;
    // no pair of this sweep had squared |cos| above tol: quadratic convergence
    // leaves every pair within about tol of orthogonal
    if (!__syncthreads_or(cmax2 > 0.0)) break;
  }
  const double rots = block_sum<NT>(nrot, red);
  work += 6.0 * (double)len * ((double)sweeps * 0.5 * (double)n * (double)(n - 1) + rots);
  return sweeps;
}

// ---- Blocked one-sided Jacobi for vectors in global memory ----------------
//
// The n columns are cut into blocks of kJB; each round of a cyclic tournament
// over the blocks pairs them up, and one wavefront takes a block pair (16
// columns Y): it forms the Gram matrix Y^T Y with FP64 matrix-core products,
// diagonalises it by cyclic two-sided Jacobi in LDS while accumulating the
// rotations in V (the same rotations one-sided Jacobi would apply to the pairs
// of Y), and applies Y <- Y V with matrix-core products.  Every column is read
// and written once per round instead of once per column pair.  The stopping
// rule is the scalar one, evaluated on the fresh Gram matrices.
constexpr int kJB = 8;
// doubles of LDS per wavefront: G, V, rotation table, two 16 x 16 transpose tiles
constexpr int kJBScratch = 16 * 16 * 2 + 16 * 3 + 2 * 256;
constexpr int kJBInner = 1;                        // inner sweeps per block-pair visit

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The Gram matrix of a block pair from its accumulators (v holds
// G[kr + 4v][kc]) into LDS, V = I, and the pair's largest squared |cos| into
// cmax2.
__device__ inline void block_gram_store(double* g, const dbl4& acc0, const dbl4& acc1, double& cmax2) {
  const int lane = threadIdx.x & 63;
  const int kc = lane & 15, kr = lane >> 4;
  double* vm = g + 256;
#pragma unroll
  for (int v = 0; v < 4; ++v) g[(kr + 4 * v) * 16 + kc] = acc0[v] + acc1[v];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int e = lane + 64 * v;
    vm[e] = (e >> 4) == (e & 15) ? 1.0 : 0.0;
  }
  wave_sync();
  double c2 = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int a = kr + 4 * v;
    if (a < kc) c2 = fmax(c2, pair_cos2(g[a * 17], g[kc * 17], g[a * 16 + kc]));
  }
  for (int off = 32; off > 0; off >>= 1) c2 = fmax(c2, __shfl_xor(c2, off, 64));
  cmax2 = fmax(cmax2, c2);
}

// Inner cyclic Jacobi on the 16 x 16 Gram matrix G in LDS, rotations
// accumulated in V; returns whether any rotation was applied.
__device__ inline bool block_inner_jacobi(double* g, double tol) {
  const int lane = threadIdx.x & 63;
  double* vm = g + 256;
  double* cself = vm + 256;
  double* cpart = cself + 16;
  int* part = reinterpret_cast<int*>(cpart + 16);
  bool changed = false;
  const int a = lane >> 2, b0 = (lane & 3) * 4;
  for (int is = 0; is < kJBInner; ++is) {
    bool swept = false;
    for (int ir = 0; ir < 15; ++ir) {
      bool r = false;
      if (lane < 8) {
        int p, q;
        tournament_pair(lane, ir, 16, p, q);
        double c = 1.0, sn = 0.0;
        r = jacobi_rotation(g[p * 17], g[q * 17], g[p * 16 + q], tol, c, sn);
        if (!r) { c = 1.0; sn = 0.0; }
        cself[p] = c;
        cpart[p] = -sn;
        part[p] = q;
        cself[q] = c;
        cpart[q] = sn;
        part[q] = p;
      }
      const bool any = __ballot(r) != 0;
      wave_sync();
      if (!any) continue;
      swept = true;
      // G <- J^T G J and V <- V J; J has column x = cself[x] e_x + cpart[x] e_part[x]
      const double sa = cself[a], ca = cpart[a];
      const int pa = part[a];
      double gn[4], vn[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int b = b0 + u;
        const double sb = cself[b], cb = cpart[b];
        const int pb = part[b];
        const double t1 = sb * g[a * 16 + b] + cb * g[a * 16 + pb];
        const double t2 = sb * g[pa * 16 + b] + cb * g[pa * 16 + pb];
        gn[u] = sa * t1 + ca * t2;
        vn[u] = sb * vm[a * 16 + b] + cb * vm[a * 16 + pb];
      }
      wave_sync();
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        g[a * 16 + b0 + u] = gn[u];
        vm[a * 16 + b0 + u] = vn[u];
      }
      wave_sync();
    }
    if (!swept) break;
    changed = true;
  }
  return changed;
}

// One block pair: columns cb[0..7] = bi*kJB.., cb[8..15] = bj*kJB.. (those >= n
// are zero).  Returns whether Y changed; cmax2 takes the largest squared |cos|
// of its column pairs before the step.  The vectors are streamed twice (Gram,
// then update), 32 rows at a time.
__device__ inline bool jacobi_block_pair(double* X, int64_t vs, int n, int len, int bi, int bj, double tol,
                                         double* g, double& cmax2) {
  const int lane = threadIdx.x & 63;
  double* vm = g + 256;
  auto colof = [&](int k) { return k < kJB ? bi * kJB + k : bj * kJB + (k - kJB); };
  // Gram matrix: lane l feeds Y[r0 + l/16][slot l%16] as both operands; rows
  // come in batches of 32 (8 loads per lane, issued together), the next batch
  // loaded while the current one is multiplied; rows past len load a clamped
  // address and contribute zero
  {
    const int kc = lane & 15, kr = lane >> 4;
    const int col = colof(kc);
    const bool ok = col < n;
    const double* xc = X + (int64_t)(ok ? col : 0) * vs;
    auto batch = [&](double (&y)[8], int r0) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int row = r0 + 4 * i + kr;
        const double v = xc[row < len ? row : len - 1];
        y[i] = (ok && row < len) ? v : 0.0;
      }
    };
    dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    double ya[8], yb[8];
    batch(ya, 0);
    for (int r0 = 0; r0 < len; r0 += 64) {
      batch(yb, r0 + 32);
#pragma unroll
      for (int i = 0; i < 8; i += 2) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[i], ya[i], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[i + 1], ya[i + 1], acc1, 0, 0, 0);
      }
      batch(ya, r0 + 64);
#pragma unroll
      for (int i = 0; i < 8; i += 2) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(yb[i], yb[i], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(yb[i + 1], yb[i + 1], acc1, 0, 0, 0);
      }
    }
    block_gram_store(g, acc0, acc1, cmax2);
  }
  if (!block_inner_jacobi(g, tol)) return false;
  // Y <- Y V, 16 rows at a time: lane l feeds Y[r0 + l%16][slot 4kk + l/16] and
  // V[4kk + l/16][l%16]; accumulator v is the new Y[r0 + l/16 + 4v][slot l%16]
  const int ir = lane & 15, ik = lane >> 4;
  const int ocol = colof(ir);
  double bv[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) bv[kk] = vm[(kk * 4 + ik) * 16 + ir];
  // column offsets fit 32 bits: a core has fewer than 2^15 rows and columns
  int aoff[4];
  bool aok[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int c = colof(kk * 4 + ik);
    aok[kk] = c < n;
    aoff[kk] = (aok[kk] ? c : 0) * (int)vs;
  }
  // two 16-row chunks per batch (8 loads per lane), the next batch loaded
  // before the current one is multiplied and stored (other rows)
  auto batch = [&](double (&a)[8], int r0) {
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int row = r0 + 16 * c + ir;
        const double v = X[aoff[kk] + (row < len ? row : len - 1)];
        a[c * 4 + kk] = (aok[kk] && row < len) ? v : 0.0;
      }
  };
  auto emit = [&](const double (&a)[8], int r0) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      dbl4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) d = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c * 4 + kk], bv[kk], d, 0, 0, 0);
      if (ocol < n) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int orow = r0 + 16 * c + ik + 4 * v;
          if (orow < len) X[ocol * (int)vs + orow] = d[v];
        }
      }
    }
  };
  double aa[8], ab[8];
  batch(aa, 0);
  for (int r0 = 0; r0 < len; r0 += 64) {
    batch(ab, r0 + 32);
    emit(aa, r0);
    batch(aa, r0 + 64);
    emit(ab, r0 + 32);
  }
  return true;
}

// The same visit for vectors of at most 32 NB elements with the block pair
// held in registers: every lane loads its share of the 16 columns in one burst
// (lane l: rows 4i + l/16 of column slot l%16), the Gram matrix and, after the
// inner sweep, the rotated columns come from the same registers, so each
// column is read once and written once per visit.  The update needs the rows
// of each 16-row chunk across the lanes (the transposed layout): the chunk
// goes through one of two 16 x 16 LDS tiles of the wavefront.
template <int NB>
__device__ inline bool jacobi_block_pair_reg(double* X, int64_t vs, int n, int len, int bi, int bj, double tol,
                                             double* g, double& cmax2) {
  const int lane = threadIdx.x & 63;
  const int kc = lane & 15, kr = lane >> 4;
  double* vm = g + 256;
  double* tile = g + 16 * 16 * 2 + 16 * 3;
  auto colof = [&](int k) { return k < kJB ? bi * kJB + k : bj * kJB + (k - kJB); };
  const int col = colof(kc);
  const bool ok = col < n;
  // one base address per lane and constant offsets; rows past len are not read
  const double* xc = X + (int64_t)(ok ? col : 0) * vs + kr;
  double y[NB][8];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int i = 0; i < 8; ++i) y[b][i] = (ok && 32 * b + 4 * i + kr < len) ? xc[32 * b + 4 * i] : 0.0;
  {
    dbl4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int i = 0; i < 8; i += 2) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(y[b][i], y[b][i], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(y[b][i + 1], y[b][i + 1], acc1, 0, 0, 0);
      }
    block_gram_store(g, acc0, acc1, cmax2);
  }
  if (!block_inner_jacobi(g, tol)) return false;
  // chunk (b, c): rows 32 b + 16 c + 4 i' + kr of slot kc in y[b][4 c + i'];
  // transposed, lane l holds rows 16 (2 b + c) + l%16 of slots 4 kk + l/16
  double bv[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) bv[kk] = vm[(kk * 4 + kr) * 16 + kc];
  double* xo = X + (int64_t)(ok ? col : 0) * vs + kr;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (32 * b + 16 * c >= len) continue;
      double* tl = tile + 256 * c;
#pragma unroll
      for (int u = 0; u < 4; ++u) tl[(4 * u + kr) * 16 + kc] = y[b][4 * c + u];
      wave_sync();
      double a[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) a[kk] = tl[kc * 16 + 4 * kk + kr];
      dbl4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) d = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], bv[kk], d, 0, 0, 0);
      if (ok) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (32 * b + 16 * c + kr + 4 * v < len) xo[32 * b + 16 * c + 4 * v] = d[v];
      }
    }
  return true;
}

// Sweeps of the blocked one-sided Jacobi over n columns of length len (column
// stride vs, element stride 1); scratch holds kJBScratch doubles of LDS per
// wavefront.  Returns the number of sweeps run and adds the flops done to
// `work`: the 16 x 16 Gram matrix of every block-pair visit (512 len) and the
// update Y V of the pairs that changed (512 len).
template <int NT, int NB = 0>
__device__ __forceinline__ int jacobi_block_sweeps(double* X, int64_t vs, int n, int len, double tol,
                                                   double* scratch, double* red, int* redi, double& work) {
  const int nblk = (n + kJB - 1) / kJB;
  const int nb = nblk + (nblk & 1);
  const int npairs = nb / 2;
  const int wave = threadIdx.x >> 6;
  double* g = scratch + wave * kJBScratch;
  int sweeps = 0;
  double visits = 0.0;
  const double lead = (threadIdx.x & 63) == 0 ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    ++sweeps;
    int rot = 0;
    double cmax2 = 0.0;
    for (int round = 0; round < nb - 1; ++round) {
      for (int pi = wave; pi < npairs; pi += NT / 64) {
        int bi, bj;
        tournament_pair(pi, round, nb, bi, bj);
        visits += lead;
        bool ch;
        if constexpr (NB > 0)
          ch = jacobi_block_pair_reg<NB>(X, vs, n, len, bi, bj, tol, g, cmax2);
        else
          ch = jacobi_block_pair(X, vs, n, len, bi, bj, tol, g, cmax2);
        if (ch) {
          rot = 1;
          visits += lead;
        }
      }
      __threadfence_block();
      __syncthreads();
    }
    if (!__syncthreads_or(rot)) break;
    int dummy = 0;
    block_argmax<NT>(cmax2, dummy, red, redi);
    if (cmax2 <= tol) break;
  }
  work += 512.0 * (double)len * block_sum<NT>(visits, red);
  return sweeps;
}

// One-sided Jacobi SVD of n vectors of length len: vector i starts at V + i * vs
// and has element stride es.  Then the singular values (vector norms, written
// to sig and t.sig), the rank k = #{sigma > eps sigma_max} (capped at
// max_rank, with a flag), and the right vectors in decreasing-sigma order:
// Zv[map(e) + ps * q] = x_i[e] / sigma_i, map(e) = perm ? perm[e] : e.  `ord`
// is n ints of scratch, red / redi one slot per wavefront.  Groups have at
// least min_g lanes (16 keeps global-memory vectors coalesced).  Returns k;
// all threads call it.
template <int NT, int min_g = 1, bool BLOCKED = false, int CAP = 0>
__device__ __forceinline__ int jacobi_svd(double* V, int64_t vs, int64_t es, int n, int len, const int* perm,
                                          double* sig, int* ord, double eps, const SvdTask& t, int* flags,
                                          double* red, int* redi, int& sweeps, double& work,
                                          double* bscratch = nullptr) {
  const int ne = n + (n & 1), npairs = ne / 2;
  // lanes per pair: up to one row of 16 (sums through DPP), fewer when that
  // takes every pair of a round in one pass; min_g keeps global-memory
  // vectors coalesced
  int G = min_g > 16 ? min_g : 16;
  while (G > min_g && G * npairs > NT) G >>= 1;
  while (G > 1 && G > 2 * len) G >>= 1;
  // a pair counts as orthogonal once |<x, y>| <= tol |x| |y|: rounding level
  // for exact factorisations, else 1e-4 eps (at most 1e-6) -- the vectors then
  // carry errors of order tol and the values of order tol^2, four orders of
  // magnitude or more below the truncation at eps sigma_1, and the last
  // sweeps of the quadratic convergence are not needed (at eps = 1e-2 the
  // headline's ranks and GMRES iterations are the same as with 1e-8)
  const double tol = fmax(fmax(1e-15, 2.3e-16 * (double)len), eps > 0.0 ? fmin(1e-6, 1e-4 * eps) : 0.0);
  // register-resident slices of up to 12 elements per lane in workgroups of
  // 256 or more threads (at most 128 registers, so that several workgroups
  // share a compute unit), 16 in a single wavefront; wider groups (a second
  // pass per round) rather than streamed vectors when a slice would exceed it
  constexpr int kCap = CAP > 0 ? CAP : NT >= 256 ? 12 : 16;
  while (G < 16 && (len + G - 1) / G > kCap) G <<= 1;
  const int groups = NT / G;
  const int gi = threadIdx.x / G, gl = threadIdx.x % G;
  const int nu = (len + G - 1) / G;
  if constexpr (BLOCKED) {
    // contiguous vectors (es == 1) and kJBScratch doubles per wavefront; block
    // pairs of vectors up to kJBRegRows long stay in registers during a visit
    // (workgroups of at most 512 threads leave them the registers)
    const int nbr = NT > 512 ? 0 : len <= 64 ? 2 : len <= 128 ? 4 : len <= 192 ? 6 : len <= kJBRegRows ? 8 : 0;
    switch (nbr) {
      case 2: sweeps = jacobi_block_sweeps<NT, 2>(V, vs, n, len, tol, bscratch, red, redi, work); break;
      case 4: sweeps = jacobi_block_sweeps<NT, 4>(V, vs, n, len, tol, bscratch, red, redi, work); break;
      case 6: sweeps = jacobi_block_sweeps<NT, 6>(V, vs, n, len, tol, bscratch, red, redi, work); break;
      case 8: sweeps = jacobi_block_sweeps<NT, 8>(V, vs, n, len, tol, bscratch, red, redi, work); break;
      default: sweeps = jacobi_block_sweeps<NT, 0>(V, vs, n, len, tol, bscratch, red, redi, work); break;
    }
  } else switch (nu <= kCap ? nu : 0) {
#define ACR_JAC_NU(k) \
  case k: sweeps = jacobi_sweeps_rec<NT, (k <= kCap ? k : 1)>(V, vs, es, n, len, G, tol, red, redi, work); break;
    ACR_JAC_NU(1) ACR_JAC_NU(2) ACR_JAC_NU(3) ACR_JAC_NU(4) ACR_JAC_NU(5) ACR_JAC_NU(6) ACR_JAC_NU(7)
    ACR_JAC_NU(8) ACR_JAC_NU(9) ACR_JAC_NU(10) ACR_JAC_NU(11) ACR_JAC_NU(12) ACR_JAC_NU(13) ACR_JAC_NU(14)
    ACR_JAC_NU(15) ACR_JAC_NU(16) ACR_JAC_NU(17) ACR_JAC_NU(18) ACR_JAC_NU(19) ACR_JAC_NU(20) ACR_JAC_NU(21)
    ACR_JAC_NU(22) ACR_JAC_NU(23) ACR_JAC_NU(24) ACR_JAC_NU(25) ACR_JAC_NU(26) ACR_JAC_NU(27) ACR_JAC_NU(28)
    ACR_JAC_NU(29) ACR_JAC_NU(30) ACR_JAC_NU(31) ACR_JAC_NU(32)
#undef ACR_JAC_NU
    default: sweeps = jacobi_sweeps<NT, 0>(V, vs, es, n, len, G, tol, red, redi, work); break;
  }
  for (int i = gi; i < n; i += groups) {
    const double* x = V + i * vs;
    double ss = 0.0;
    for (int e = gl; e < len; e += G) ss += x[e * es] * x[e * es];
    ss = gsum2(ss, G);
    if (gl == 0) {
      sig[i] = sqrt(ss);
      t.sig[i] = sqrt(ss);
    }
  }
  __syncthreads();
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) mx = fmax(mx, sig[i]);
  {
    int dummy = 0;
    block_argmax<NT>(mx, dummy, red, redi);
  }
  const double smax = mx;
  const double thr = eps > 0.0 ? eps * smax : 0.0;
  double cnt = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) cnt += (smax > 0.0 && sig[i] > thr) ? 1.0 : 0.0;
  int k = (int)block_sum<NT>(cnt, red);
  if (t.max_rank > 0 && k > t.max_rank) {
    if (threadIdx.x == 0) atomicOr(&flags[FLAG_RANK], 1);
    k = t.max_rank;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) {
    const double si = sig[i];
    int ps = 0;
    for (int j = 0; j < n; ++j) {
      const double sj = sig[j];
      ps += (sj > si || (sj == si && j < i)) ? 1 : 0;
    }
    ord[i] = ps;
  }
  __syncthreads();
  const int q = t.q;
  double* Zv = t.Y + (int64_t)q * q;
  for (int i = gi; i < n; i += groups) {
    const int ps = ord[i];
    if (ps >= k) continue;
    const double inv = 1.0 / sig[i];
    const double* x = V + i * vs;
    for (int e = gl; e < len; e += G) Zv[(perm ? perm[e] : e) + (int64_t)ps * q] = x[e * es] * inv;
  }
  return k;
}

// Jacobi stage of the cores whose pivoted QR ran in global memory: W^T
// (q x t, from k_qrcp) in LDS when it fits (scalar sweeps), else in place in
// global memory (blocked sweeps).
template <class T, bool LDS, int NT, int CAP = 0>
__global__ __launch_bounds__(NT) void k_jacobi(const SvdTask* __restrict__ tasks, double eps, int* flags) {
  extern __shared__ double smj[];
  const SvdTask t = tasks[blockIdx.x];
  const int rows = t.q;
  const int n = *t.t_out;
  if (n == 0 || rows == 0) {
    if (threadIdx.x == 0) *t.rank_out = 0;
    return;
  }
  double* A = LDS ? smj : t.Y;
  __shared__ double red[NT / 64];
  __shared__ int redi[NT / 64];
  const int ld = LDS ? jacobi_ld(rows, n) : rows;
  if (LDS)
    staged_copy<NT>((int64_t)rows * n, [&](int64_t e) { return t.Y[e]; },
                    [&](int64_t e, double v) { A[(e / rows) * ld + e % rows] = v; });
  __syncthreads();
  int sweeps = 0;
  double work = 0.0;
  // the pivot order is no longer needed: its workspace holds the sigma ranks.
  // Vectors in global memory take the blocked sweeps (LDS holds their
  // per-wavefront Gram and rotation matrices); the counters record the flops
  // the sweeps did.
  const int k = jacobi_svd<NT, LDS ? 1 : 16, !LDS, CAP>(A, ld, 1, n, rows, nullptr, t.sig, t.perm, eps, t, flags,
                                                        red, redi, sweeps, work, LDS ? nullptr : smj);
  if (threadIdx.x == 0) {
    *t.rank_out = k;
    const unsigned long long f = (unsigned long long)work;
    if (t.sweep_ctr) atomicAdd(t.sweep_ctr, f);
    if (t.flop_ctr) atomicAdd(t.flop_ctr, f);
  }
}

// flops of one core: its product (macs multiply-adds), the pivoted QR stopped
// at n, and the flops the sweeps did
__device__ inline void count_core_flops(const SvdTask& t, double macs, int n, double sweep_work) {
  const double dp = t.p, dq = t.q, dn = n;
  const double fl = 2.0 * macs + 4.0 * dp * dq * dn - 2.0 * dn * dn * (dp + dq) + 4.0 / 3.0 * dn * dn * dn +
                    sweep_work;
  const unsigned long long f = (unsigned long long)(fl > 0.0 ? fl : 0.0);
  if (t.sweep_ctr) atomicAdd(t.sweep_ctr, f);
  if (t.flop_ctr) atomicAdd(t.flop_ctr, f);
}

// multiply-adds of the core product: sum over (a, b) of r - max(a, b) for
// triangular panels
__device__ inline double core_macs(const SvdTask& t) {
  if (t.mode != 0) return (double)t.p * t.q * t.r;
  const double r = t.r;
  double m = 0.0;
  for (int a = 0; a < t.p; ++a) {
    const double lo = (a + 1 < t.q ? a + 1 : t.q);            // b <= a
    const double hi = (double)(t.q - a - 1 > 0 ? t.q - a - 1 : 0);  // b = a+1 .. q-1
    m += lo * (r - a) + hi * r - hi * ((double)a + 1.0 + (double)t.q - 1.0) / 2.0;
  }
  return m;
}

// Zero the strictly lower part of the first n rows of R (the reflectors).
__device__ inline void clear_below(double* C, int lc, int n, int nt) {
  for (int e = threadIdx.x; e < n * n; e += nt) {
    const int a = e % n, c = e / n;
    if (c < a) C[a + c * lc] = 0.0;
  }
}

// Cores whose C fits in LDS: core product, pivoted QR, then the sweeps on the
// columns of W^T = P R^T (q x t, copied into the C region), in one workgroup.
// LDS: C (p x q, ld p|1), q norms, q pivots, q ints of scratch.
template <class T, int NT>
__global__ __launch_bounds__(NT) void k_svd_block(const SvdTask* __restrict__ tasks, double delta, double eps,
                                                  int* flags) {
  extern __shared__ double smb[];
  const SvdTask t = tasks[blockIdx.x];
  const int p = t.p, q = t.q;
  if (p == 0 || q == 0) {
    if (threadIdx.x == 0) { *t.t_out = 0; *t.rank_out = 0; }
    return;
  }
  const int lc = p | 1;
  double* C = smb;
  double* nrm = C + lc * q;
  int* perm = reinterpret_cast<int*>(nrm + q);
  int* ord = perm + q;
  __shared__ double red[NT / 64];
  __shared__ int redi[NT / 64];
  core_product_mfma<T, NT>(t, C, lc);
  __syncthreads();
  // the pivot map of the QR in the sweeps' scratch
  const int n = qrcp_body<NT, 12>(C, lc, p, q, nrm, perm, ord, delta, red, redi);
  // W^T = P R^T (q x n) through the global workspace back into the C region:
  // the sweeps then run on contiguous columns
  double* Wt = t.Y;
  for (int e = threadIdx.x; e < q * n; e += NT) {
    const int c = e % q, a = e / q;
    Wt[perm[c] + a * q] = c >= a ? C[a + ord[c] * lc] : 0.0;
  }
  __threadfence();
  __syncthreads();
  for (int e = threadIdx.x; e < q * n; e += NT) C[e] = Wt[e];
  __syncthreads();
  int sweeps = 0;
  double work = 0.0;
  const int k = n > 0 ? jacobi_svd<NT>(C, q, 1, n, q, nullptr, nrm, ord, eps, t, flags, red, redi, sweeps, work)
                      : 0;
  if (threadIdx.x == 0) {
    *t.t_out = n;
    *t.rank_out = k;
    count_core_flops(t, core_macs(t), n, work);
  }
}

// The whole truncated SVD of one small core (p, q, r <= 64, triangular panels)
// in one wavefront: C from FP64 matrix-core tiles, the pivoted QR with one
// lane per column and wavefront shuffles, the sweeps on the rows of R.  LDS: C
// (p x q, ld p|1), q norms, q pivots, q ints.
template <class T>
__global__ __launch_bounds__(64) void k_svd_wave(const SvdTask* __restrict__ tasks, double delta, double eps,
                                                 int* flags) {
  extern __shared__ double sw[];
  const SvdTask t = tasks[blockIdx.x];
  const int p = t.p, q = t.q, r = t.r, lane = threadIdx.x;
  if (p == 0 || q == 0) {
    if (lane == 0) { *t.t_out = 0; *t.rank_out = 0; }
    return;
  }
  const int lc = p | 1;
  double* C = sw;
  double* nrm = C + lc * q;
  int* perm = reinterpret_cast<int*>(nrm + q);
  int* ord = perm + q;
  __shared__ double red[1];
  __shared__ int redi[1];
  core_product_mfma<T, 64>(t, C, lc);
  __syncthreads();
  // pivoted QR, lane c owns column c
  double nc = 0.0;
  if (lane < q) {
    for (int a = 0; a < p; ++a) nc += C[a + lane * lc] * C[a + lane * lc];
    nrm[lane] = nc;
    perm[lane] = lane;
  }
  // stop when the remaining block's Frobenius norm is at most delta times the
  // largest column norm (nrm holds its column norms)
  const double thr2 = delta * delta * wmax(nc);
  __syncthreads();
  const int mn = p < q ? p : q;
  int tcount = 0;
  for (int j = 0; j < mn; ++j) {
    const bool live = lane >= j && lane < q;
    double best = live ? nrm[lane] : -1.0;
    const double rest = wsum(live ? nrm[lane] : 0.0);
    int bi = lane;
    wargmax(best, bi);
    if (!(rest > thr2) || !(best > 0.0)) break;
    if (bi != j) {
      if (lane < p) {
        const double a = C[lane + j * lc];
        C[lane + j * lc] = C[lane + bi * lc];
        C[lane + bi * lc] = a;
      }
      if (lane == 0) {
        const double a = nrm[j];
        nrm[j] = nrm[bi];
        nrm[bi] = a;
        const int b = perm[j];
        perm[j] = perm[bi];
        perm[bi] = b;
      }
    }
    __syncthreads();
    // Householder vector of column j below the diagonal
    const double x = lane < p ? C[lane + j * lc] : 0.0;
    const double sigma = wsum(lane > j && lane < p ? x * x : 0.0);
    const double x0 = __shfl(x, j, 64);
    double tau = 0.0, scale = 0.0, beta = x0;
    if (sigma != 0.0) {
      const double nr = sqrt(x0 * x0 + sigma);
      beta = x0 >= 0.0 ? -nr : nr;
      tau = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    if (lane < p && lane >= j) C[lane + j * lc] = lane == j ? beta : (tau != 0.0 ? x * scale : x);
    __syncthreads();
    if (lane > j && lane < q) {
      double* ac = C + lane * lc;
      const double* v = C + j * lc;
      if (tau != 0.0) {
        double w = ac[j];
        for (int i = j + 1; i < p; ++i) w += v[i] * ac[i];
        w *= tau;
        ac[j] -= w;
        for (int i = j + 1; i < p; ++i) ac[i] -= w * v[i];
      }
      double s = 0.0;
      for (int i = j + 1; i < p; ++i) s += ac[i] * ac[i];
      nrm[lane] = s;
    }
    __syncthreads();
    tcount = j + 1;
  }
  const int n = tcount;
  clear_below(C, lc, n, 64);
  __syncthreads();
  int sweeps = 0;
  double work = 0.0;
  const int k = n > 0 ? jacobi_svd<64>(C, 1, lc, n, q, perm, nrm, ord, eps, t, flags, red, redi, sweeps, work) : 0;
  // multiply-adds of the core product
  double macs = 0.0;
  if (lane < q)
    for (int a = 0; a < p; ++a) macs += (double)(r - (a > lane ? a : lane));
  macs = wsum(macs);
  if (lane == 0) {
    *t.t_out = n;
    *t.rank_out = k;
    count_core_flops(t, macs, n, work);
  }
}

// Left factor of the core, Zu = C Zv = Ru (Rv^T Zv), for the k kept columns:
// one workgroup per (core, chunk of kc columns); the chunk of Zv and of the
// intermediate Rv^T Zv sit in LDS, both products run on the FP64 matrix cores.
template <class T>
__global__ __launch_bounds__(256) void k_core_left(const SvdTask* __restrict__ tasks, int kc,
                                                   unsigned long long* ctr) {
  extern __shared__ double sl[];
  const SvdTask t = tasks[blockIdx.x];
  const int k = *t.rank_out;
  const int c0 = blockIdx.y * kc;
  if (c0 >= k) return;
  const int nc = k - c0 < kc ? k - c0 : kc;
  const int p = t.p, q = t.q, r = t.r;
  const double* Zv = t.Y + (int64_t)q * q + (int64_t)c0 * q;
  double* Zu = t.C + (int64_t)p * q + (int64_t)c0 * p;
  double* zs = sl;               // q x nc
  double* t1 = sl + q * kc;      // r x nc
  for (int e = threadIdx.x; e < q * nc; e += 256) zs[e] = Zv[e];
  __syncthreads();
  // both products on the FP64 matrix cores, 16 x 16 tiles over the four
  // wavefronts: lane l feeds A[i0 + l%16][k0 + l/16] and B[k0 + l/16][j0 + l%16]
  // and receives D[i0 + l/16 + 4v][j0 + l%16]; mode 0 panels are upper
  // trapezoidal (entries below their diagonal load as zero)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tc = (nc + 15) / 16;
  // t1 = Rv^T Zv (r x nc): A[l][b] = Rv(b, l), B[b][c] = Zv(b, c)
  {
    const int tr = (r + 15) / 16;
    for (int tile = wave; tile < tr * tc; tile += 4) {
      const int i0 = (tile % tr) * 16, j0 = (tile / tr) * 16;
      const int l = i0 + li, c = j0 + li;
      const int lcl = l < r ? l : r - 1;
      dbl4 acc = {0.0, 0.0, 0.0, 0.0};
      const int kend = t.mode == 0 ? (i0 + 16 < q ? i0 + 16 : q) : q;
      for (int k0 = 0; k0 < kend; k0 += 4) {
        const int b = k0 + lk;
        const int bcl = b < q ? b : q - 1;
        double av;
        if (t.mode == 0) av = (double)static_cast<const T*>(t.Rv)[bcl + (int64_t)lcl * t.ldv];
        else av = static_cast<const double*>(t.Rv)[bcl + (int64_t)lcl * t.ldv];
        av = (l < r && b < q && (t.mode != 0 || b <= l)) ? av : 0.0;
        const double bv = (b < q && c < nc) ? zs[bcl + (c < nc ? c : 0) * q] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = i0 + lk + 4 * v, col = j0 + li;
        if (row < r && col < nc) t1[row + col * r] = acc[v];
      }
    }
  }
  __syncthreads();
  // Zu = Ru t1 (p x nc): A[a][l] = Ru(a, l), B[l][c] = t1(l, c)
  {
    const int tp = (p + 15) / 16;
    for (int tile = wave; tile < tp * tc; tile += 4) {
      const int i0 = (tile % tp) * 16, j0 = (tile / tp) * 16;
      const int a = i0 + li, c = j0 + li;
      const int acl = a < p ? a : p - 1;
      dbl4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int k0 = t.mode == 0 ? (i0 & ~3) : 0; k0 < r; k0 += 4) {
        const int l = k0 + lk;
        const int lcl = l < r ? l : r - 1;
        double av;
        if (t.mode == 0) av = (double)static_cast<const T*>(t.Ru)[acl + (int64_t)lcl * t.ldu];
        else av = static_cast<const double*>(t.Ru)[acl + (int64_t)lcl * t.ldu];
        av = (a < p && l < r && (t.mode != 0 || a <= l)) ? av : 0.0;
        const double bv = (l < r && c < nc) ? t1[lcl + (c < nc ? c : 0) * r] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = i0 + lk + 4 * v, col = j0 + li;
        if (row < p && col < nc) Zu[row + (int64_t)col * p] = acc[v];
      }
    }
  }
  if ((ctr || t.flop_ctr) && threadIdx.x == 0) {
    // multiply-adds of this chunk
    unsigned long long m = 0;
    if (t.mode == 0) {
      for (int l = 0; l < r; ++l) m += (unsigned long long)(l < q - 1 ? l + 1 : q);
      m += (unsigned long long)p * r - (unsigned long long)p * (p - 1) / 2;
    } else {
      m = (unsigned long long)r * (p + q);
    }
    if (ctr) atomicAdd(ctr, m * (unsigned long long)nc);
    if (t.flop_ctr) atomicAdd(t.flop_ctr, 2ull * m * (unsigned long long)nc);
  }
}

__global__ __launch_bounds__(256) void k_tri_copy(const TriCopyTask* __restrict__ tasks) {
  const TriCopyTask t = tasks[blockIdx.x];
  const int n = t.n;
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = threadIdx.x + (int64_t)blockIdx.y * 256; e < 2 * nn; e += 256 * (int64_t)gridDim.y) {
    double v = 0.0;
    if (e < nn) {
      const int i = (int)(e % n), j = (int)(e / n);
      if (i <= j) v = t.src[i + (int64_t)j * t.lds];
    }
    t.dst[e] = v;
  }
}

template <class K> void allow(K kernel, size_t bytes) {
  if (bytes > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

}  // namespace

// The pivoted QR of large cores runs with 1024 threads when its LDS working
// set exceeds kSmallLds (it already limits them to one or two workgroups per
// compute unit; the extra wavefronts hide latency and shorten each core's
// critical path), with 256 threads otherwise.
template <class T>
void launch_qrcp(const SvdTask* d_tasks, int ntasks, double delta, size_t lds, int max_q, hipStream_t s) {
  if (ntasks <= 0) return;
  if (lds == 0) {
    // C in global memory, the position -> column map in LDS
    const size_t map = (size_t)max_q * sizeof(int);
    allow(k_qrcp<T, false, 1024>, map);
    hipLaunchKernelGGL((k_qrcp<T, false, 1024>), dim3(ntasks), dim3(1024), map, s, d_tasks, delta);
    return;
  }
  if (lds <= kSmallLds) {
    allow(k_qrcp<T, true, 256>, lds);
    hipLaunchKernelGGL((k_qrcp<T, true, 256>), dim3(ntasks), dim3(256), lds, s, d_tasks, delta);
    return;
  }
  if (lds <= kMidLds) {
    allow(k_qrcp<T, true, 512>, lds);
    hipLaunchKernelGGL((k_qrcp<T, true, 512>), dim3(ntasks), dim3(512), lds, s, d_tasks, delta);
    return;
  }
  allow(k_qrcp<T, true, 1024>, lds);
  hipLaunchKernelGGL((k_qrcp<T, true, 1024>), dim3(ntasks), dim3(1024), lds, s, d_tasks, delta);
}

template <class T>
void launch_jacobi(const SvdTask* d_tasks, int ntasks, double eps, int* d_flags, size_t lds, int threads,
                   hipStream_t s) {
  if (ntasks <= 0) return;
  if (lds == 0) {
    // blocked sweeps: 512 threads leave a wavefront the registers to hold a
    // block pair of vectors up to kJBRegRows long; launches with longer
    // vectors stream them, with a block pair per wavefront of 1024 threads
    if (threads > 512) {
      const size_t scratch = (size_t)(1024 / 64) * kJBScratch * sizeof(double);
      allow(k_jacobi<T, false, 1024>, scratch);
      hipLaunchKernelGGL((k_jacobi<T, false, 1024>), dim3(ntasks), dim3(1024), scratch, s, d_tasks, eps, d_flags);
      return;
    }
    const size_t scratch = (size_t)(512 / 64) * kJBScratch * sizeof(double);
    allow(k_jacobi<T, false, 512>, scratch);
    hipLaunchKernelGGL((k_jacobi<T, false, 512>), dim3(ntasks), dim3(512), scratch, s, d_tasks, eps, d_flags);
    return;
  }
  if (lds <= kSmallLds) {
    allow(k_jacobi<T, true, 256>, lds);
    hipLaunchKernelGGL((k_jacobi<T, true, 256>), dim3(ntasks), dim3(256), lds, s, d_tasks, eps, d_flags);
    return;
  }
  // larger cores: the smallest workgroup that takes every column pair of a
  // round at once, with 8 lanes per pair for vectors up to 128 long (16
  // elements per lane) so that the per-pair work (sums across the lanes, the
  // rotation) is shared by 8 pairs per wavefront; 1024 threads allow at most
  // 12 elements per lane
  if (threads <= 256) {
    allow(k_jacobi<T, true, 256, 16>, lds);
    hipLaunchKernelGGL((k_jacobi<T, true, 256, 16>), dim3(ntasks), dim3(256), lds, s, d_tasks, eps, d_flags);
  } else if (threads <= 512) {
    allow(k_jacobi<T, true, 512, 16>, lds);
    hipLaunchKernelGGL((k_jacobi<T, true, 512, 16>), dim3(ntasks), dim3(512), lds, s, d_tasks, eps, d_flags);
  } else {
    allow(k_jacobi<T, true, 1024>, lds);
    hipLaunchKernelGGL((k_jacobi<T, true, 1024>), dim3(ntasks), dim3(1024), lds, s, d_tasks, eps, d_flags);
  }
}

// Cores whose LDS working set exceeds kSmallLds use 1024 threads (their LDS
// footprint already limits them to one or two workgroups per compute unit and
// the extra wavefronts hide LDS latency), smaller ones 256.
template <class T>
void launch_svd_block(const SvdTask* d_tasks, int ntasks, double delta, double eps, int* d_flags, size_t lds,
                      hipStream_t s) {
  if (ntasks <= 0) return;
  if (lds <= kSmallLds) {
    allow(k_svd_block<T, 256>, lds);
    hipLaunchKernelGGL((k_svd_block<T, 256>), dim3(ntasks), dim3(256), lds, s, d_tasks, delta, eps, d_flags);
    return;
  }
  allow(k_svd_block<T, 1024>, lds);
  hipLaunchKernelGGL((k_svd_block<T, 1024>), dim3(ntasks), dim3(1024), lds, s, d_tasks, delta, eps, d_flags);
}

template <class T>
void launch_svd_wave(const SvdTask* d_tasks, int ntasks, double delta, double eps, int* d_flags, size_t lds,
                     hipStream_t s) {
  if (ntasks <= 0) return;
  allow(k_svd_wave<T>, lds);
  hipLaunchKernelGGL(k_svd_wave<T>, dim3(ntasks), dim3(64), lds, s, d_tasks, delta, eps, d_flags);
}

template <class T>
void launch_core_left(const SvdTask* d_tasks, int ntasks, int kc, int nchunks, size_t lds, unsigned long long* ctr,
                      hipStream_t s) {
  if (ntasks <= 0 || nchunks <= 0) return;
  allow(k_core_left<T>, lds);
  hipLaunchKernelGGL(k_core_left<T>, dim3(ntasks, nchunks), dim3(256), lds, s, d_tasks, kc, ctr);
}

void launch_tri_copy(const TriCopyTask* d_tasks, int ntasks, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_tri_copy, dim3(ntasks, 8), dim3(256), 0, s, d_tasks);
}

#define ACR_SVD_INST(T)                                                                                     \
  template void launch_qrcp<T>(const SvdTask*, int, double, size_t, int, hipStream_t);                           \
  template void launch_jacobi<T>(const SvdTask*, int, double, int*, size_t, int, hipStream_t);                   \
  template void launch_svd_block<T>(const SvdTask*, int, double, double, int*, size_t, hipStream_t);        \
  template void launch_svd_wave<T>(const SvdTask*, int, double, double, int*, size_t, hipStream_t);         \
  template void launch_core_left<T>(const SvdTask*, int, int, int, size_t, unsigned long long*, hipStream_t);
ACR_SVD_INST(float)
ACR_SVD_INST(double)
#undef ACR_SVD_INST

}  // namespace acr
