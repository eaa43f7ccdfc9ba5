// Device helpers shared by the gfx950 kernels of the SamBaTen update:
// counter-based random numbers, the basic-operation logarithm used by the
// sampler, bfloat16 conversion and wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sbt {

constexpr int kWave = 64;  // CDNA wavefront width

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Ten rounds of the 4x32
// S-box; multipliers 0xD2511F53 / 0xCD9E8D57, key increments 0x9E3779B9 /
// 0xBB67AE85 applied before every round after the first.
// ---------------------------------------------------------------------------
struct Philox4 {
  uint32_t v[4];
};

__host__ __device__ inline Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  Philox4 r;
  r.v[0] = c0;
  r.v[1] = c1;
  r.v[2] = c2;
  r.v[3] = c3;
  return r;
}

// Streams of random numbers the update draws; packed into counter word 2 as
// stream << 24 | mode << 20 | repetition.
enum : uint32_t { kStreamSample = 1, kStreamAlsInit = 2, kStreamInit = 3, kStreamGetRank = 4 };

__host__ __device__ inline uint32_t rng_tag(uint32_t stream, uint32_t mode, uint32_t rep) {
  return (stream << 24) | ((mode & 0xFu) << 20) | (rep & 0xFFFFFu);
}

struct RngKey {
  uint32_t k0, k1;
};

__host__ __device__ inline RngKey rng_key(uint64_t seed, uint32_t tensor_id) {
  RngKey k;
  k.k0 = (uint32_t)seed;
  k.k1 = (uint32_t)(seed >> 32) ^ tensor_id;
  return k;
}

// 64-bit word (out1 << 32) | out0 of the block at counter (c0, c1, tag, t).
__host__ __device__ inline uint64_t rng_bits(RngKey key, uint32_t c0, uint32_t c1, uint32_t tag,
                                             uint32_t t) {
  const Philox4 o = philox4x32_10(c0, c1, tag, t, key.k0, key.k1);
  return ((uint64_t)o.v[1] << 32) | o.v[0];
}

// (2*(u >> 12) + 1) * 2^-53 : exact, strictly inside (0, 1).
__host__ __device__ inline double uniform_open(uint64_t u) {
  return (double)(((u >> 12) << 1) | 1ull) * 0x1p-53;
}

// (u >> 11) * 2^-53 : exact, in [0, 1).
__host__ __device__ inline double uniform_closed0(uint64_t u) {
  return (double)(u >> 11) * 0x1p-53;
}

// Natural logarithm of a positive normal double from IEEE basic operations
// only (so that every compliant implementation returns the same bits):
//   U = m 2^e, m in [1,2) by bit extraction; if m > sqrt(2): m /= 2, e += 1;
//   t = (m-1)/(m+1); p = Horner of sum_{n=0..11} t^(2n)/(2n+1) in t^2 with
//   coefficients 1.0/(2n+1); ln m = (2t) p;  ln U = e*LN2 + ln m.
// Contraction into fused multiply-adds would change the bits: it is off here.
__device__ inline double ln_basic(double U) {
#pragma clang fp contract(off)
  const uint64_t b = __double_as_longlong(U);
  int e = (int)((b >> 52) & 0x7FF) - 1023;
  double m = __longlong_as_double((long long)((b & 0x000FFFFFFFFFFFFFull) | (1023ull << 52)));
  const double kSqrt2 = 1.4142135623730951;
  const double kLn2 = 0.6931471805599453;
  if (m > kSqrt2) {
    m = m / 2.0;
    e += 1;
  }
  const double t = (m - 1.0) / (m + 1.0);
  const double t2 = t * t;
  double p = 1.0 / 23.0;
  p = p * t2; p = p + 1.0 / 21.0;
  p = p * t2; p = p + 1.0 / 19.0;
  p = p * t2; p = p + 1.0 / 17.0;
  p = p * t2; p = p + 1.0 / 15.0;
  p = p * t2; p = p + 1.0 / 13.0;
  p = p * t2; p = p + 1.0 / 11.0;
  p = p * t2; p = p + 1.0 / 9.0;
  p = p * t2; p = p + 1.0 / 7.0;
  p = p * t2; p = p + 1.0 / 5.0;
  p = p * t2; p = p + 1.0 / 3.0;
  p = p * t2; p = p + 1.0;
  const double lnm = (2.0 * t) * p;
  const double el = (double)e * kLn2;
  return el + lnm;
}

// ---------------------------------------------------------------------------
// bfloat16: 16-bit storage, round to nearest even from float.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint16_t f32_to_bf16_rne(float x) {
  uint32_t u;
  __builtin_memcpy(&u, &x, 4);
  if ((u & 0x7F800000u) == 0x7F800000u) {  // inf / nan: keep, quiet the nan
    return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  }
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_to_f32(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float x;
  __builtin_memcpy(&x, &u, 4);
  return x;
}

// ---------------------------------------------------------------------------
// Wavefront reductions (64 lanes).
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ inline int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

}  // namespace sbt
