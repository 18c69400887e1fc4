// Lane-group reductions inside a 64-lane CDNA wavefront.
#pragma once

#include <hip/hip_runtime.h>

namespace acr {

// Lane exchange inside a row of 16 lanes through the DPP operand modifier
// (no trip through the LDS crossbar): CTRL 0xB1 / 0x4E swap lanes 1 / 2 apart
// within a quad, 0x141 mirrors each half row, 0x140 the whole row.
template <int CTRL> __device__ inline double dpp_mov(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over aligned groups of G lanes (a power of two up to 64); every lane of
// a group ends with the same bits (each step adds a lane's partial to its
// partner's, which is commutative).
__device__ inline double gsum_dpp(double v, int G) {
  if (G >= 2) v += dpp_mov<0xB1>(v);
  if (G >= 4) v += dpp_mov<0x4E>(v);
  if (G >= 8) v += dpp_mov<0x141>(v);
  if (G >= 16) v += dpp_mov<0x140>(v);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  if (G >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// Three group sums at once: every exchange step is taken for all three values
// inside one (uniform) branch, so the three dependency chains overlap.
__device__ inline void gsum3_dpp(double& a, double& b, double& c, int G) {
  if (G >= 2) {
    const double x = dpp_mov<0xB1>(a), y = dpp_mov<0xB1>(b), z = dpp_mov<0xB1>(c);
    a += x; b += y; c += z;
  }
  if (G >= 4) {
    const double x = dpp_mov<0x4E>(a), y = dpp_mov<0x4E>(b), z = dpp_mov<0x4E>(c);
    a += x; b += y; c += z;
  }
  if (G >= 8) {
    const double x = dpp_mov<0x141>(a), y = dpp_mov<0x141>(b), z = dpp_mov<0x141>(c);
    a += x; b += y; c += z;
  }
  if (G >= 16) {
    const double x = dpp_mov<0x140>(a), y = dpp_mov<0x140>(b), z = dpp_mov<0x140>(c);
    a += x; b += y; c += z;
  }
  if (G >= 32) {
    const double x = __shfl_xor(a, 16, 64), y = __shfl_xor(b, 16, 64), z = __shfl_xor(c, 16, 64);
    a += x; b += y; c += z;
  }
  if (G >= 64) {
    const double x = __shfl_xor(a, 32, 64), y = __shfl_xor(b, 32, 64), z = __shfl_xor(c, 32, 64);
    a += x; b += y; c += z;
  }
}

template <int CTRL> __device__ inline int dpp_mov_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}

// One exchange step of a wavefront argmax: keep the larger value, the smaller
// index on ties (both partners end with the same pair).
__device__ inline void argmax_step(double& v, int& i, double o, int oi) {
  if (o > v || (o == v && oi < i)) {
    v = o;
    i = oi;
  }
}

// Argmax of (v, i) over the 64 lanes of a wavefront: DPP exchanges inside
// rows of 16 lanes, then two cross-row shuffles.
__device__ inline void wave_argmax(double& v, int& i) {
  argmax_step(v, i, dpp_mov<0xB1>(v), dpp_mov_i<0xB1>(i));
  argmax_step(v, i, dpp_mov<0x4E>(v), dpp_mov_i<0x4E>(i));
  argmax_step(v, i, dpp_mov<0x141>(v), dpp_mov_i<0x141>(i));
  argmax_step(v, i, dpp_mov<0x140>(v), dpp_mov_i<0x140>(i));
  argmax_step(v, i, __shfl_xor(v, 16, 64), __shfl_xor(i, 16, 64));
  argmax_step(v, i, __shfl_xor(v, 32, 64), __shfl_xor(i, 32, 64));
}

// Argmax over aligned groups of G lanes (G a power of two up to 16), with the
// same tie rule: the DPP steps of wave_argmax that stay inside the group.
template <int G> __device__ inline void group_argmax(double& v, int& i) {
  static_assert(G >= 1 && G <= 16 && (G & (G - 1)) == 0, "group of 1 to 16 lanes");
  if (G >= 2) argmax_step(v, i, dpp_mov<0xB1>(v), dpp_mov_i<0xB1>(i));
  if (G >= 4) argmax_step(v, i, dpp_mov<0x4E>(v), dpp_mov_i<0x4E>(i));
  if (G >= 8) argmax_step(v, i, dpp_mov<0x141>(v), dpp_mov_i<0x141>(i));
  if (G >= 16) argmax_step(v, i, dpp_mov<0x140>(v), dpp_mov_i<0x140>(i));
}

// The value of the first active lane, on every lane (a wavefront-uniform value).
__device__ inline double read_first_lane(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(unsigned)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// A generic pointer taken as one into global memory.  Generic (flat) accesses
// count against the LDS wait counter too, so an LDS read after a generic store
// waits for that store to reach memory; global accesses do not.
template <class T> __device__ inline __attribute__((address_space(1))) T* to_global(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Copy of count elements by a workgroup of NT threads, element e read by
// load(e) and written by store(e, v): each thread issues B reads before its
// writes.  A loop of single read-then-write steps waits for every read in
// turn, since a generic-pointer read may alias the LDS written before it.
template <int NT, int B = 8, class Load, class Store>
__device__ inline void staged_copy(int64_t count, Load load, Store store) {
  for (int64_t e0 = 0; e0 < count; e0 += (int64_t)B * NT) {
    decltype(load(int64_t(0))) v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int64_t e = e0 + b * NT + threadIdx.x;
      if (e < count) v[b] = load(e);
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int64_t e = e0 + b * NT + threadIdx.x;
      if (e < count) store(e, v[b]);
    }
  }
}

}  // namespace acr
