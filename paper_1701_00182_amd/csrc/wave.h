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

}  // namespace acr
