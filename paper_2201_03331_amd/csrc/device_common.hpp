// device_common.hpp -- small device helpers shared by the libfiuncho kernels.
#pragma once

#include "internal.hpp"

namespace fiuncho {

typedef unsigned long long u64;

// Address-space qualified views.  Data that no kernel writes while the scan
// runs (bitsets, tables) is read through the constant address space, so that
// wave-uniform addresses become scalar loads into scalar registers; per-lane
// data is read through the global address space (no flat-address checks).
#define FI_CONST __attribute__((address_space(4)))
#define FI_GLOBAL __attribute__((address_space(1)))
#define FI_LDS __attribute__((address_space(3)))
typedef const FI_CONST u64 *cu64p;
typedef const FI_CONST uint32_t *cu32p;
typedef const FI_GLOBAL u64 *gu64p;

template <typename T>
__device__ __forceinline__ const FI_CONST T *as_const(const T *p) {
  return (const FI_CONST T *)p;
}
template <typename T>
__device__ __forceinline__ const FI_GLOBAL T *as_global(const T *p) {
  return (const FI_GLOBAL T *)p;
}

__device__ __forceinline__ uint32_t uni(uint32_t v) {
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ u64 uni64(u64 v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((u64)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ u64 ballot(bool p) { return __ballot(p); }

// The value x holds in lane l ^ 1, by a DPP quad permutation [1, 0, 3, 2]:
// one VALU move, no round trip through the LDS crossbar
__device__ __forceinline__ uint32_t xor1(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);
}

__device__ __forceinline__ uint32_t popc64(u64 x) { return (uint32_t)__popcll(x); }

// acc + popcount(x) as two v_bcnt_u32_b32, each taking the running count as
// its addend (the compiler otherwise reassociates into bcnt, bcnt, add3)
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
  return r;
}
__device__ __forceinline__ uint32_t add_popc64(uint32_t acc, u64 x) {
  return bcnt_acc((uint32_t)(x >> 32), bcnt_acc((uint32_t)x, acc));
}

// C(a, r) from the host-built table; 0 when a < r
__device__ __forceinline__ u64 binom(const Globals &g, uint32_t a, uint32_t r) {
  return g.binom[(size_t)a * kBinomStride + r];
}

// C(a, r) for r <= 3 from its closed form in registers, else from the table:
// the binary searches of the tile decoders and of the rank conversions then
// wait on no memory for subsets of up to 3 variants.  Each product is exact
// in 64 bits for a < 2^21 and vanishes for a < r; larger a read the table.
__device__ __forceinline__ u64 binom_small(const Globals &g, uint32_t a, uint32_t r) {
  if (r == 0) return 1;
  if (r == 1) return a;
  if (r == 2) return (u64)a * (a - 1u) / 2;
  if (r == 3 && a < (1u << 21)) return (u64)a * (a - 1u) * (a - 2u) / 6;
  return binom(g, a, r);
}

// Colex unrank of the (R)-subset of [0, hi) with index q into pre[0 .. R-1]
// (ascending): the largest element is the largest v with C(v, R) <= q, and
// so on down; the last element is the remaining index itself.
template <int R>
__device__ __forceinline__ void colex_unrank(const Globals &g, uint32_t hi, u64 q, uint32_t *pre) {
#pragma unroll
  for (int r = R; r >= 1; --r) {
    uint32_t lo;
    if (r == 1) {
      lo = (uint32_t)q;
    } else {
      lo = (uint32_t)(r - 1);
      uint32_t top = hi - 1;
      while (lo < top) {
        const uint32_t mid = (lo + top + 1) >> 1;
        if (binom_small(g, mid, r) <= q) lo = mid;
        else top = mid - 1;
      }
      q -= binom_small(g, lo, r);
    }
    pre[r - 1] = uni(lo);
    hi = lo;
  }
}

// The matrix-core kernels feed 32 samples of one class to a lane as 32 FP4
// (E2M1) operand values in four registers: register d holds sample 4p + d of
// the 32-bit half word in nibble p.  A set sample's nibble holds one of the
// values 0.5, 1, 2 (nibble bits 0, 1, 2; bit 3 is the sign); the two operands
// of the one-hot contraction use reciprocal values per register, so every
// product of two set samples is exactly 1:
//   register      0     1     2     3
//   A operand    0.5   1.0   2.0   1.0
//   B operand    2.0   1.0   0.5   1.0
// fp4_b_operand is the B form of a half word.
__device__ __forceinline__ uint4 fp4_b_operand(uint32_t b) {
  const uint32_t t = b >> 2;
  return make_uint4((b << 2) & 0x44444444u, b & 0x22222222u, t & 0x11111111u, t & 0x22222222u);
}

// relaxed loads that read the device-coherent copy (other workgroups update it)
__device__ __forceinline__ uint32_t load_relaxed(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lexicographic rank -> ascending combination (same numbering as the header
// describes): position i takes the value v whose block of combinations
// contains the remaining rank; the blocks before v hold
// C(n - prev - 1, r + 1) - C(n - v, r + 1) combinations (hockey-stick sum).
__device__ inline void lex_unrank(const Globals &g, uint32_t n, uint32_t k, u64 rank,
                                  uint32_t *c) {
  int64_t prev = -1;
  for (uint32_t i = 0; i < k; ++i) {
    uint32_t r = k - 1 - i;
    u64 top = binom_small(g, (uint32_t)(n - prev - 1), r + 1);
    // largest v in [prev+1, n-1-r] with top - C(n - v, r + 1) <= rank
    uint32_t lo = (uint32_t)(prev + 1), hi = n - 1 - r;
    while (lo < hi) {
      uint32_t mid = (lo + hi + 1) >> 1;
      if (top - binom_small(g, n - mid, r + 1) <= rank) lo = mid;
      else hi = mid - 1;
    }
    rank -= top - binom_small(g, n - lo, r + 1);
    c[i] = lo;
    prev = lo;
  }
}

// Lexicographic rank of the part contributed by the first k-1 elements of a
// combination whose (k-1)-prefix is p[0..k-2]; the full rank is this plus
// (j - p[k-2] - 1) for last element j.
__device__ inline u64 lex_rank_prefix(const Globals &g, uint32_t n, uint32_t k,
                                      const uint32_t *p) {
  u64 r = 0;
  int64_t prev = -1;
  for (uint32_t i = 0; i + 1 < k; ++i) {
    r += binom_small(g, (uint32_t)(n - prev - 1), k - i) - binom_small(g, n - p[i], k - i);
    prev = p[i];
  }
  return r;
}

// Compensated single-precision accumulation (Knuth's TwoSum): s + e carries
// the running sum with the rounding error of every addition kept in e.
__device__ __forceinline__ void two_sum_add(float &s, float &e, float v) {
  float t = s + v;
  float bp = t - s;
  e += (s - (t - bp)) + (v - bp);
  s = t;
}

}  // namespace fiuncho
