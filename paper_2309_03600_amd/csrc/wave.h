// Wavefront reductions with DPP lane rotations (no LDS traffic), for 64-wide wavefronts.
#pragma once
#include <hip/hip_runtime.h>

namespace ib {

// Four DPP row rotations leave every lane of a 16-lane row holding the row's sum; the four
// row sums are then read as scalars.
template <int C>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), C, 0xF, 0xF, false));
}
template <int C>
__device__ __forceinline__ double dpp_mov(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), C, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), C, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// row broadcast (lanes outside ``RM`` rows read zero)
template <int C, int RM>
__device__ __forceinline__ float dpp_bcast(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), C, RM, 0xF, false));
}
template <int C, int RM>
__device__ __forceinline__ double dpp_bcast(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), C, RM, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), C, RM, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float read_lane(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double read_lane(double v, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// full-wavefront sum (every lane active), returned in every lane
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp_mov<0x128>(v);   // row_ror:8
  v += dpp_mov<0x124>(v);   // row_ror:4
  v += dpp_mov<0x122>(v);   // row_ror:2
  v += dpp_mov<0x121>(v);   // row_ror:1
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// sum over each 16-lane row, returned in every lane of the row
template <typename T>
__device__ __forceinline__ T row_sum16(T v) {
  v += dpp_mov<0x128>(v);
  v += dpp_mov<0x124>(v);
  v += dpp_mov<0x122>(v);
  v += dpp_mov<0x121>(v);
  return v;
}

// sum over each 8-lane group (lanes 8k .. 8k+7), returned in every lane of the group:
// half-row mirror pairs lane i with 7 - i, then two quad permutations combine the pairs
template <typename T>
__device__ __forceinline__ T row_sum8(T v) {
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_mov<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  return v;
}

// full-wavefront sum (every lane active) returned as a scalar: row rotations leave each
// 16-lane row's sum in all its lanes, the row broadcasts carry rows 0-2 into lane 63
template <typename T>
__device__ __forceinline__ T wave_total(T v) {
  v += dpp_mov<0x128>(v);   // row_ror:8
  v += dpp_mov<0x124>(v);   // row_ror:4
  v += dpp_mov<0x122>(v);   // row_ror:2
  v += dpp_mov<0x121>(v);   // row_ror:1
  v += dpp_bcast<0x142, 0xA>(v);   // row_bcast:15 into rows 1, 3
  v += dpp_bcast<0x143, 0xC>(v);   // row_bcast:31 into rows 2, 3
  return read_lane(v, 63);
}

// inclusive prefix sum over the 64 lanes (every lane active): Hillis-Steele inside each
// 16-lane row by DPP row shifts (lanes shifted in from outside the row read zero), then the
// row totals carried forward by the row broadcasts of lanes 15 and 31
__device__ __forceinline__ int wave_incl_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);   // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);   // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
  return v;
}

}  // namespace ib
