// Device-side helpers shared by the gfx950 kernels (included by .hip files
// only).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fdtd {

// Loads and stores at a 32-bit byte offset from a wave-uniform base: all
// accesses of a row can share one vector offset (base and row step in
// scalar registers), with no 64-bit address arithmetic per access.
template <typename T>
__device__ __forceinline__ T ld(const T* base, uint32_t off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
template <typename T>
__device__ __forceinline__ void st(T* base, uint32_t off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off) = v;
}

// Whole-wave lane shifts by one (DPP wave_shr:1 / wave_shl:1, no LDS
// traffic): lane_prev gives lane l the value of lane l-1 (lane 0 gets 0),
// lane_next the value of lane l+1 (lane 63 gets 0).
__device__ __forceinline__ int dpp_prev(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_next(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false); }

__device__ __forceinline__ float lane_prev(float v) { return __builtin_bit_cast(float, dpp_prev(__builtin_bit_cast(int, v))); }
__device__ __forceinline__ float lane_next(float v) { return __builtin_bit_cast(float, dpp_next(__builtin_bit_cast(int, v))); }
__device__ __forceinline__ double lane_prev(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)dpp_prev((int)(uint32_t)u), hi = (uint32_t)dpp_prev((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double lane_next(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)dpp_next((int)(uint32_t)u), hi = (uint32_t)dpp_next((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Workgroup barrier that publishes LDS writes only: global loads still in
// flight (row prefetches) are not waited for, unlike __syncthreads().
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// acc[k] += sum over this lane's columns c = lane + 64 i (c < ld, ld a
// multiple of 64) of rows[k * ld + c] * z[c], for kRows consecutive rows of
// a row-major matrix.  Loads go in groups of 4 column slices (4 * kRows per
// lane in flight, one register buffer; larger groups raise the register
// count of every kernel that contains this code, stencil waves included):
// the first group is issued before stage() - which fills z and ends with a
// barrier - so it overlaps the staging loads.  Each lane accumulates its
// columns in increasing order.
template <typename T, int kRows, typename Stage>
__device__ __forceinline__ void lane_row_dots(const T* __restrict__ rows, int ld, const T* z, int lane,
                                              T (&acc)[kRows], Stage&& stage) {
  constexpr int U = 4;
  const int nit = ld / 64;
  T g[U][kRows];
  auto fetch = [&](int it) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (it + u < nit) {
        const int c = lane + (it + u) * 64;
#pragma unroll
        for (int k = 0; k < kRows; ++k) g[u][k] = rows[(size_t)k * ld + c];
      }
  };
  fetch(0);
  stage();
  for (int it = 0; it < nit; it += U) {
    if (it > 0) fetch(it);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (it + u < nit) {
        const T zc = z[lane + (it + u) * 64];
#pragma unroll
        for (int k = 0; k < kRows; ++k) acc[k] += g[u][k] * zc;
      }
  }
}

}  // namespace fdtd
