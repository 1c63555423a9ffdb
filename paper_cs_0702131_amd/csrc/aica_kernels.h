// Device-side helpers shared by the HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aica {

constexpr int kRow = 16;        // lanes per rotation row (a DPP row)
constexpr int kRotFlag = 64;     // added to an entry's image code when its referring transform rotates
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = 64 * kWavesPerBlock;

// Error-free transformation a + b = s + e (Knuth's TwoSum).
template <typename T>
__device__ __forceinline__ void two_sum(T a, T b, T &s, T &e) {
  s = a + b;
  T bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous range of
// logical blocks so that neighbouring groups (which share j-data) meet in the same L2.
__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nblocks_padded) {
  const int64_t per = nblocks_padded >> 3;
  return (bid & 7) * per + (bid >> 3);
}

// Order this wave's LDS accesses across this point.  The LDS performs one wave's operations in issue
// order, so a later read (by any lane) sees an earlier write; only the compiler must not move memory
// accesses across.  (A memory fence here would also wait for outstanding global stores.)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

}  // namespace aica
