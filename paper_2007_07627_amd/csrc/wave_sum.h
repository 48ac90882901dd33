// Fixed-order sum over a wavefront of 32 FP64 values per lane, by recursive
// halving through lane permutations (v_permlane32_swap, v_permlane16_swap,
// DPP); shared by the reduction kernel and the solver's merge of its partials.
#pragma once
#include <hip/hip_runtime.h>

namespace icp {

// The lane's value moved through a DPP lane permutation (both 32-bit halves).
template <int kCtrl>
__device__ __forceinline__ double dpp_f64(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, kCtrl, 0xf, 0xf, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), kCtrl, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One halving level over lane bit 5: lanes 0..31 return x summed with x of
// lane + 32, lanes 32..63 y summed with y of lane - 32
// (v_permlane32_swap exchanges the upper half of its first operand with the
// lower half of its second).
__device__ __forceinline__ double halve_bit5(double x, double y) {
  const unsigned long long bx = (unsigned long long)__double_as_longlong(x);
  const unsigned long long by = (unsigned long long)__double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)bx, (unsigned)by, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false, false);
  const double a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  const double b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
  return a + b;
}

// Over lane bit 4 (v_permlane16_swap: odd 16-lane rows of the first operand
// with even rows of the second): lanes with bit 4 clear sum x, the others y.
__device__ __forceinline__ double halve_bit4(double x, double y) {
  const unsigned long long bx = (unsigned long long)__double_as_longlong(x);
  const unsigned long long by = (unsigned long long)__double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)bx, (unsigned)by, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false, false);
  const double a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  const double b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
  return a + b;
}

// A halving level through a DPP permutation that pairs every lane with a lane
// whose bit differs (and whose higher bits agree): the lane keeps y when its
// bit is set, x otherwise, and adds its partner's copy of the same value.
template <int kCtrl>
__device__ __forceinline__ double halve_dpp(double x, double y, bool bit) {
  const double keep = bit ? y : x, send = bit ? x : y;
  return keep + dpp_f64<kCtrl>(send);
}

// Sum over the wavefront of v[0..31] by recursive halving (five levels, over
// lane bits 5, 4, 3, 2, 1, each keeping half of the values), then one
// exchange over bit 0: lanes 2j and 2j + 1 return the total of v[j], with the
// same bits. About four instructions per value instead of the 18 of a
// butterfly per value.
__device__ __forceinline__ double wave_sum32(const double (&v)[32]) {
  const int lane = (int)(threadIdx.x & 63);
  double a[16], b[8], c[4], d[2];
#pragma unroll
  for (int i = 0; i < 16; ++i) a[i] = halve_bit5(v[i], v[i + 16]);
#pragma unroll
  for (int i = 0; i < 8; ++i) b[i] = halve_bit4(a[i], a[i + 8]);
  // bit 3: row_ror:8 pairs lane l with l ^ 8 inside its 16-lane row
#pragma unroll
  for (int i = 0; i < 4; ++i) c[i] = halve_dpp<0x128>(b[i], b[i + 4], (lane & 8) != 0);
  // bit 2: row_half_mirror pairs lane l with l ^ 7 inside its 8 lanes
#pragma unroll
  for (int i = 0; i < 2; ++i) d[i] = halve_dpp<0x141>(c[i], c[i + 2], (lane & 4) != 0);
  // bit 1: quad_perm [2, 3, 0, 1] pairs l with l ^ 2
  const double e = halve_dpp<0x4e>(d[0], d[1], (lane & 2) != 0);
  // bit 0: quad_perm [1, 0, 3, 2]
  return e + dpp_f64<0xb1>(e);
}

// The value of lane `src` (wave-uniform) in every lane.
__device__ __forceinline__ double readlane_f64(double x, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

}  // namespace icp
