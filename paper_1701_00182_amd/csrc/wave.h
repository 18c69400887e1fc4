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

}  // namespace acr
