// Device helpers shared by the librsm kernels: wavefront reductions, the subset
// generator (Philox4x64-10 + Floyd sampling) and small dense routines.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rsm {

// ---------------------------------------------------------------- wavefront reductions

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(static_cast<uint64_t>(v) >> 32));
  return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

// 8 bytes -> 8 bits: bit k set iff byte k is nonzero.
__device__ __forceinline__ uint32_t nonzero_bytes_to_bits(uint64_t x) {
  const uint64_t lo7 = 0x7F7F7F7F7F7F7F7Full;
  uint64_t t = ((x & lo7) + lo7) | x;          // high bit of each byte = (byte != 0)
  t = (t >> 7) & 0x0101010101010101ull;        // one bit per byte, at bit 8k
  return static_cast<uint32_t>((t * 0x0102040810204080ull) >> 56);  // gather to bits 0..7
}

// ---------------------------------------------------------------- subset generator
// Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): per round the counter
// words 0 and 2 are multiplied (64 x 64 -> 128 bits) by two fixed odd constants and the
// halves are mixed with words 1 and 3 and the round key; the key advances by two Weyl
// constants between rounds.

struct Philox4x64 {
  static constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
  static constexpr uint64_t kM1 = 0xCA5A826395121157ull;
  static constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
  static constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;

  __device__ static void block(uint64_t c[4], uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
      if (rnd) {
        k0 += kW0;
        k1 += kW1;
      }
      const uint64_t lo0 = kM0 * c[0];
      const uint64_t hi0 = __umul64hi(kM0, c[0]);
      const uint64_t lo1 = kM1 * c[2];
      const uint64_t hi1 = __umul64hi(kM1, c[2]);
      const uint64_t n0 = hi1 ^ c[1] ^ k0;
      const uint64_t n2 = hi0 ^ c[3] ^ k1;
      c[0] = n0;
      c[1] = lo1;
      c[2] = n2;
      c[3] = lo0;
    }
  }
};

// Uniform l-subset of [0, n) for trial t by Floyd's algorithm (Bentley & Floyd, CACM
// 1987), word i of the trial's Philox stream drawing x in [0, j], j = n - l + i.
// Output sorted ascending in out[0..l).  MAXL is the compile-time capacity.
template <int MAXL>
__device__ void draw_subset(uint64_t seed, uint64_t t, int n, int l, int out[MAXL]) {
  constexpr int kBlocks = (MAXL + 3) / 4;
  uint64_t u[kBlocks * 4];
#pragma unroll
  for (int b = 0; b < kBlocks; ++b) {
    uint64_t c[4] = {static_cast<uint64_t>(b), t, 0ull, 0ull};
    if (b * 4 < l) Philox4x64::block(c, seed, 0ull);
    u[4 * b + 0] = c[0];
    u[4 * b + 1] = c[1];
    u[4 * b + 2] = c[2];
    u[4 * b + 3] = c[3];
  }
#pragma unroll
  for (int i = 0; i < MAXL; ++i) {
    if (i < l) {
      const int j = n - l + i;
      const int x = static_cast<int>(__umul64hi(u[i], static_cast<uint64_t>(j) + 1ull));
      bool seen = false;
#pragma unroll
      for (int k = 0; k < MAXL; ++k) seen |= (k < i) && (out[k] == x);
      out[i] = seen ? j : x;
    }
  }
  // odd-even transposition sort with static indices (keeps `out` in registers); unused
  // slots hold INT32_MAX and stay at the end
#pragma unroll
  for (int i = 0; i < MAXL; ++i)
    if (i >= l) out[i] = 0x7fffffff;
#pragma unroll
  for (int pass = 0; pass < MAXL; ++pass) {
#pragma unroll
    for (int k = pass & 1; k + 1 < MAXL; k += 2) {
      const int a = out[k], b = out[k + 1];
      out[k] = a < b ? a : b;
      out[k + 1] = a < b ? b : a;
    }
  }
}

// ---------------------------------------------------------------- FP64 atomics

__device__ __forceinline__ void atomic_add_f64(double* p, double v) {
  unsafeAtomicAdd(p, v);  // hardware global_atomic_add_f64 on gfx950
}

}  // namespace rsm
