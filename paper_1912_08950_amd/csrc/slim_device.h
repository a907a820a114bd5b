// Device-side building blocks shared by the libslim kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slim {

constexpr int kWave = 64;
constexpr int kBlock = 256;                   // threads per block: 4 waves
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kItems = 16;                    // CSR entries per thread per tile
constexpr int kTile = kBlock * kItems;        // 4096 CSR entries per tile
constexpr int kChunks = kTile / kWave;        // 64 wave-sized chunks per tile

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  return (uint64_t(1) << lane_id()) - 1;  // lane 0 -> 0
}

// Inclusive max-scan across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t o = __shfl_up(v, d, kWave);
    if ((int)lane_id() >= d) v = v > o ? v : o;
  }
  return v;
}

// Inclusive sum-scan across the 64 lanes of a wave (64-bit values).
__device__ __forceinline__ uint64_t wave_incl_sum64(uint64_t v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint64_t o = __shfl_up(v, d, kWave);
    if ((int)lane_id() >= d) v += o;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Counter-based random source: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// SC'11).  A round sends (x0,x1,x2,x3) under key (k0,k1) to
// (hi(B*x2)^x1^k0, lo(B*x2), hi(A*x0)^x3^k1, lo(A*x0)) with A = 0xD2511F53,
// B = 0xCD9E8D57; the key then moves on by (0x9E3779B9, 0xBB67AE85).
__device__ __forceinline__ uint4 philox4(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 product each (a single multiply-add instruction on gfx950)
    const uint64_t a = (uint64_t)0xD2511F53u * x0;
    const uint64_t b = (uint64_t)0xCD9E8D57u * x2;
    // three-input exclusive or (truth table 0x96) in one instruction
    x0 = __builtin_amdgcn_bitop3_b32((uint32_t)(b >> 32), x1, k0, 0x96);
    x1 = (uint32_t)b;
    x2 = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), x3, k1, 0x96);
    x3 = (uint32_t)a;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(x0, x1, x2, x3);
}

// Output words 0 and 1 (selection and edge choice).
__device__ __forceinline__ void philox_w01(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                           uint32_t k0, uint32_t k1, uint32_t& w0,
                                           uint32_t& w1) {
  const uint4 r = philox4(x0, x1, x2, x3, k0, k1);
  w0 = r.x;
  w1 = r.y;
}

// Sort three distinct vertex ids ascending.
__device__ __forceinline__ void sort3(uint32_t& a, uint32_t& b, uint32_t& c) {
  uint32_t t;
  if (a > b) { t = a; a = b; b = t; }
  if (b > c) { t = b; b = c; c = t; }
  if (a > b) { t = a; a = b; b = t; }
}

__device__ __forceinline__ void bit_set(uint32_t* bits, uint32_t idx) {
  __hip_atomic_fetch_or(bits + (idx >> 5), 1u << (idx & 31u), __ATOMIC_RELAXED,
                        __HIP_MEMORY_SCOPE_AGENT);
}

// Deletion mark of DAG edge idx: one byte per edge, set by a plain byte
// store.  Every store writes the same value 1 and nothing reads the bytes
// before the marking kernels have ended, so concurrent stores to one byte
// leave 1 in any order; stores to other bytes of the same line, from other
// XCDs, are kept because the L2 writes back only the bytes written.  Unlike
// an atomic OR on a bitmap word (executed past the L2, a memory transaction
// per mark), the stores merge in the L2.
__device__ __forceinline__ void mark_set(uint8_t* marks, uint32_t idx) { marks[idx] = 1u; }

__device__ __forceinline__ bool bit_get(const uint32_t* bits, uint32_t idx) {
  return (bits[idx >> 5] >> (idx & 31u)) & 1u;
}

}  // namespace slim
