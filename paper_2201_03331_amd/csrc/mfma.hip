// mfma.hip -- orders 2 and 3 on the matrix cores.
//
// For a pair (a, j) the scan needs the four cells g_a, g_j in {0, 1} per class
// (the cells with a 2 follow from the class counts, section 3.2).  Written
// with one-hot rows X[(v, g)][s] = 1 iff sample s of the class has genotype g
// at variant v, those cells are the entries of the Gram matrix X X^T: an
// exact 0/1 contraction over the samples of the class, with int32
// accumulation (counts stay below 2^24).  Here it runs on the int8 matrix
// instruction v_mfma_i32_32x32x32_i8: fragment g of either operand holds
// genotype row g of 32 consecutive variants, so block (g_a, g_j) holds cell
// (g_a, g_j) of 32 x 32 pairs, and the four blocks give each lane (one column,
// a last variant) all four cells of its pairs.
//
// A workgroup owns 64 first variants x 64 last variants (tile of the upper
// triangle of 64-variant blocks); each of its 4 waves owns 32 x 32 of them
// (2 x 2 blocks) and accumulates both classes (class 0 words, then class 1
// words).  Operands are not stored as bytes: each lane reads the 64-bit word
// of its row from the packed bitsets and expands the 16 samples it feeds to
// 16 bytes in registers (A operands through an LDS table, B operands by
// arithmetic), so the cache traffic is that of the bitsets.
//
// The same contraction also runs with FP4 (E2M1) operands on the scaled
// matrix instruction v_mfma_scale_f32_32x32x64_f8f6f4 (scales 1): 0 and 1 are
// exact E2M1 values, every product is 0 or 1 and the FP32 accumulators hold
// integers below 2^24 exactly, so the counts are the same; one instruction
// takes 64 samples per row instead of 32, and a lane's 32 operand values come
// from its 32-bit half word by one or two bit operations per register.
//
// Order 3 uses the same contraction with prefix pairs as rows: row 2p + g_a
// of A fragment g_b is the AND of genotype row g_a of a_p and row g_b of b
// (16 prefix pairs (a_p, b) per fragment, b fixed for the tile), so the four
// blocks hold the {0,1}^3 cells of 16 prefixes x 32 last variants; the other
// cells come from the pair tables by inclusion-exclusion, as in the popcount
// kernel.
#include "filter.hpp"

namespace fiuncho {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// operand format code of E2M1 in the scaled instruction's format fields, and
// the E8M0 scale exponent of 1.0
constexpr int kFmtFp4 = 4;
constexpr int kScaleOne = 127;

constexpr int kMfmaWaves = 4;
static_assert(kMfmaWaves == kScanWaves, "pilot slots and tile decoding assume equal waves per tile");

// 8 sample bits -> 8 bytes 0/1 (byte i = bit i) by table lookup in LDS.
// A nibble times 1 + 2^7 + 2^14 + 2^21 puts bit b at bit 8b (no carries);
// the table holds that for every byte value, in kLutCopies interleaved copies
// so that the 16 lanes an LDS cycle serves always hit distinct banks.
constexpr int kLutCopies = 16;

// A wave reads the bound again within a tile after an emit in which this many
// lanes appended (a flood: the bound it holds is far below the current one);
// otherwise once per tile.
constexpr uint32_t kRefreshAppends = 16;

// Operand formats of the matrix-core kernels: int8; FP4; FP4 for jobs whose
// f table fits in LDS ("narrow": their class counts fit 16 bits, so class-0
// counts wait as 16-bit pairs while class 1 accumulates, and both classes of
// a cell share one register afterwards: half the registers for finished
// counts, and one exchange between partner lanes instead of two where the
// counts of a combination sit in two lanes).
constexpr int kMfmaI8 = 0, kMfmaF4 = 1, kMfmaF4Narrow = 2;
// FP4 for jobs whose two class sizes fit 24 bits together (bit length of m0
// plus bit length of m1 at most 24, e.g. both below 4,096): class-1 products
// carry the scale 2^bitlength(m0), so one FP32 accumulator holds c0 + 2^s c1
// exactly and the kernel runs 3 waves per SIMD ("dual").  The same launch
// group also runs the narrow kernel, each kernel skipping the other's jobs.
constexpr int kMfmaF4Dual = 3;

// Entries of the f table a matrix-core workgroup keeps in LDS (dynamic LDS;
// jobs with more samples read the table from global memory).  Two
// workgroups share a compute unit's 160 KB, 80 KB each with their static
// LDS: up to 12,280 entries next to the 32 KB byte table with int8 operands,
// 20,448 with FP4 operands (every job of a narrow launch has at most 20,447
// samples); the dual kernels run 3 workgroups per compute unit, 8,192
// entries each (jobs of at most 8,191 samples).
__host__ __device__ constexpr uint32_t mfma_f_entries(int fmt) {
  return fmt == kMfmaI8 ? 12280u : fmt == kMfmaF4Dual ? 8192u : 20448u;
}

// Dynamic LDS of a workgroup: the f table of E entries, then the 8-byte slot
// of its current tile.
__host__ __device__ constexpr size_t f_lds_bytes(uint32_t entries) {
  return (size_t)entries * sizeof(float) + sizeof(u64);
}
template <uint32_t E>
__device__ __forceinline__ FI_LDS u64 &tile_slot(FI_LDS float *f) {
  static_assert(E % 2 == 0, "the tile slot needs 8-byte alignment");
  return *reinterpret_cast<FI_LDS u64 *>(f + E);
}

// The dynamic LDS of the FP4 kernels, addressed from 0.  They declare no
// static LDS (the build checks that each reports an LDS size of 0 bytes), so
// their dynamic block starts at LDS address 0, and an f-table entry is read at
// the count's byte offset alone: through the extern array's symbol, resolved
// only when the code object is linked, every read would first add the base.
__device__ __forceinline__ FI_LDS float *lds_window() { return (FI_LDS float *)(uintptr_t)0; }

// Whether a matrix-core workgroup keeps the fixed-point table Fq in LDS (and
// scores in fixed point) or the single-precision one: fixed point where it
// measured faster, the order-3 FP4 kernels and the order-4/5 table kernels;
// the order-2 FP4 kernels ran a few per cent slower with it.
template <int ORDER, int FMT>
constexpr bool lds_fixed() { return ORDER >= 3 && FMT != kMfmaI8; }

// The f table a matrix-core workgroup keeps in LDS, as its scoring reads it
template <int ORDER, int FMT>
__device__ __forceinline__ auto lds_table(const FI_LDS float *Fl) {
  if constexpr (lds_fixed<ORDER, FMT>()) return (const FI_LDS uint32_t *)Fl;
  else return Fl;
}

__device__ __forceinline__ u64 spread8(uint32_t e) {
  const uint32_t lo = ((e & 0xFu) * 0x00204081u) & 0x01010101u;
  const uint32_t hi = (((e >> 4) & 0xFu) * 0x00204081u) & 0x01010101u;
  return (u64)lo | ((u64)hi << 32);
}

// 16 sample bits -> 16 bytes by arithmetic: each nibble times 1 + 2^7 + 2^14
// + 2^21, masked (no table; VALU only)
__device__ __forceinline__ v4i expand16_alu(uint32_t b) {
  v4i r;
  r[0] = (int)(((b & 0xFu) * 0x00204081u) & 0x01010101u);
  r[1] = (int)((((b >> 4) & 0xFu) * 0x00204081u) & 0x01010101u);
  r[2] = (int)((((b >> 8) & 0xFu) * 0x00204081u) & 0x01010101u);
  r[3] = (int)((((b >> 12) & 0xFu) * 0x00204081u) & 0x01010101u);
  return r;
}

// 16 sample bits -> the 16 int8 operand bytes of one lane
__device__ __forceinline__ v4i expand16(const u64 *lut, uint32_t b) {
  const u64 lo = lut[__builtin_amdgcn_ubfe(b, 0, 8) * kLutCopies];
  const u64 hi = lut[__builtin_amdgcn_ubfe(b, 8, 8) * kLutCopies];
  v4i r;
  r[0] = (int)(uint32_t)lo;
  r[1] = (int)(uint32_t)(lo >> 32);
  r[2] = (int)(uint32_t)hi;
  r[3] = (int)(uint32_t)(hi >> 32);
  return r;
}

// Counts of one class: words [wbeg, wend) of the bitsets.  Lane l feeds row
// r = l mod 32 of every fragment (variant base + r / 2, genotype r mod 2) and
// the 16 samples [16 (l / 32), 16 (l / 32) + 16) of each 32-sample step; the
// matrix instruction pairs the same lane half and byte of both operands, so
// any fixed sample order inside a lane is exact.
template <int kDepth, int kRaw, typename Load, typename Prep>
__device__ __forceinline__ void mfma_class(Load &&load_words, Prep &&prep, uint32_t wbeg,
                                           uint32_t wend, uint32_t h, const u64 *lut,
                                           v16i (&acc)[2][2]) {
  if (wbeg >= wend) return;
  // the loads of the next kDepth words are in flight in a register ring (the
  // depth is what the kernel's register budget allows): load_words(w, x)
  // fills x with the kRaw words the lane loads for word w, and prep(x, o)
  // makes the lane's words of both A and both B fragments from them when the
  // word is used (so no load is waited for early)
  const uint32_t wlast = wend - 1;
  u64 X[kDepth][kRaw];
#pragma unroll
  for (int u = 0; u < kDepth; ++u) load_words(min(wbeg + u, wlast), X[u]);
  auto step = [&](int slot) {
    u64 O[4];
    prep(X[slot], O);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      // 16 samples of this lane half: bits [16 h, 16 h + 16) of the 32-bit half s
      // the A fragments through the LDS table, the B fragments by arithmetic:
      // the two expansions load different units (LDS, VALU), so neither
      // alone has to keep up with the matrix instructions
      v4i E[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const uint32_t half = s ? (uint32_t)(O[f] >> 32) : (uint32_t)O[f];
        const uint32_t bits = __builtin_amdgcn_ubfe(half, 16 * h, 16);
        E[f] = f < 2 ? expand16(lut, bits) : expand16_alu(bits);
      }
      acc[0][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(E[0], E[2], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(E[0], E[3], acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(E[1], E[2], acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(E[1], E[3], acc[1][1], 0, 0, 0);
    }
  };
  uint32_t w = wbeg;
  for (; w + kDepth <= wend; w += kDepth) {
#pragma unroll
    for (int u = 0; u < kDepth; ++u) {
      step(u);
      load_words(min(w + u + kDepth, wlast), X[u]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int u = 0; u < kDepth - 1; ++u)
    if (w + u < wend) step(u);
}

// 32-bit load at a wave-uniform base plus a lane offset, as a raw buffer
// load: the base becomes a buffer descriptor in scalar registers (built by
// scalar arithmetic for every word) and the lane offset stays one 32-bit
// vector register, so no per-lane 64-bit address arithmetic is needed
constexpr int kBufferWord3 = 0x00020000;  // raw 32-bit buffer of gfx9-class GPUs
__device__ __forceinline__ uint32_t ld32(const FI_GLOBAL char *base, uint32_t off) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, 0x7fffffff, kBufferWord3);
  return __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0);
}
// the same for 16 bytes
__device__ __forceinline__ v4u ld128(const FI_GLOBAL char *base, uint32_t off) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, 0x7fffffff, kBufferWord3);
  return __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
}
// the same for a whole 64-bit word
typedef uint32_t v2u32 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u64 ld64(const FI_GLOBAL char *base, uint32_t off) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, 0x7fffffff, kBufferWord3);
  const v2u32 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
  return (u64)v.x | ((u64)v.y << 32);
}


// 32 sample bits -> the 32 FP4 operand values of one lane.  Register d takes
// bit 4p + d of b into nibble p, so both operands pair the same samples; the
// nibble bit it lands on sets the E2M1 value (bit 0: 0.5, bit 1: 1.0, bit 2:
// 2.0), and the two operands use reciprocal values per register, so every
// product of two set bits is exactly 1:
//   register      0     1     2     3
//   A operand    0.5   1.0   2.0   1.0   (no shift for registers 0-2)
//   B operand    2.0   1.0   0.5   1.0   (registers 2 and 3 share one shift)
// Only the low four registers are read for FP4 operands.
__device__ __forceinline__ v8i expand32_fp4_a(uint32_t b) {
  v8i r;
  r[0] = (int)(b & 0x11111111u);
  r[1] = (int)(b & 0x22222222u);
  r[2] = (int)(b & 0x44444444u);
  r[3] = (int)((b >> 2) & 0x22222222u);
  r[4] = r[5] = r[6] = r[7] = 0;
  return r;
}
// The A form of x AND y: each register one 3-input AND (x, y, the register's
// nibble mask), register 3 masked before its shift
__device__ __forceinline__ v8i expand32_fp4_and(uint32_t x, uint32_t y) {
  constexpr uint32_t kAnd3 = 0x80;  // truth table of a & b & c
  v8i r;
  r[0] = __builtin_amdgcn_bitop3_b32(x, y, 0x11111111u, kAnd3);
  r[1] = __builtin_amdgcn_bitop3_b32(x, y, 0x22222222u, kAnd3);
  r[2] = __builtin_amdgcn_bitop3_b32(x, y, 0x44444444u, kAnd3);
  r[3] = (int)((uint32_t)__builtin_amdgcn_bitop3_b32(x, y, 0x88888888u, kAnd3) >> 2);
  r[4] = r[5] = r[6] = r[7] = 0;
  return r;
}
__device__ __forceinline__ v8i fp4_operand(uint4 q) {
  v8i r;
  r[0] = (int)q.x;
  r[1] = (int)q.y;
  r[2] = (int)q.z;
  r[3] = (int)q.w;
  r[4] = r[5] = r[6] = r[7] = 0;
  return r;
}
__device__ __forceinline__ v8i expand32_fp4_b(uint32_t b) { return fp4_operand(fp4_b_operand(b)); }

// Counts of one class with FP4 operands: words [wbeg, wend), two at a time.
// Lane l feeds row l mod 32 of every fragment; lane half h = l / 32 loads word
// w + h whole (one 64-bit load per row), and the two instructions of a step
// take the low, then the high 32-bit halves: each covers 32 samples of word w
// (lanes 0-31) and 32 of word w + 1 (lanes 32-63), the same samples for both
// operands, since the instruction pairs the same lane half and nibble of A
// and B.  load_words(w, tail, x) fills the kRaw 64-bit words of the step at
// word w (tail: std::true_type for the last step of an odd count, whose lanes
// of half 1 must load operands with vanishing products, else
// std::false_type); ops(x, half, E) expands the given 32-bit half into the A
// fragments (FA of them) and the two B fragments.  The next kDepth steps'
// loads stay in flight in a register ring.
template <int kDepth, int kRaw, int FA = 2, typename Load, typename Ops>
__device__ __forceinline__ void mfma_class_fp4(Load &&load_words, Ops &&ops, uint32_t wbeg,
                                               uint32_t wend, v16f (&acc)[FA][2],
                                               int scale_a = kScaleOne) {
  if (wbeg >= wend) return;
  auto step = [&](const u64 (&x)[kRaw]) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      v8i E[FA + 2];
      ops(x, half, E);
#pragma unroll
      for (int i = 0; i < FA; ++i)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[i][y] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
              E[i], E[FA + y], acc[i][y], kFmtFp4, kFmtFp4, 0, scale_a, 0, kScaleOne);
    }
  };
  const uint32_t nfull = (wend - wbeg) / 2;  // steps of two words
  if (nfull > 0) {
    const uint32_t plast = nfull - 1;
    u64 X[kDepth][kRaw];
#pragma unroll
    for (int u = 0; u < kDepth; ++u) load_words(wbeg + 2 * min((uint32_t)u, plast), std::false_type{}, X[u]);
    uint32_t p = 0;
    for (; p + kDepth <= nfull; p += kDepth) {
#pragma unroll
      for (int u = 0; u < kDepth; ++u) {
        step(X[u]);
        load_words(wbeg + 2 * min(p + u + kDepth, plast), std::false_type{}, X[u]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int u = 0; u < kDepth - 1; ++u)
      if (p + u < nfull) step(X[u]);
  }
  if ((wend - wbeg) & 1) {
    u64 x[kRaw];
    load_words(wend - 1, std::true_type{}, x);
    step(x);
  }
}

__device__ __forceinline__ void zero_acc(v16i (&acc0)[2][2], v16i (&acc1)[2][2]) {
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc0[x][y][e] = acc1[x][y][e] = 0;
}

// Both classes with FP4 operands (class 0: words [0, W0), class 1: the next
// W1), counts returned as integers: the FP32 sums are integers below 2^24
template <int kDepth, int kRaw, int FA = 2, typename Load, typename Ops>
__device__ __forceinline__ void contract_fp4(Load &&load_words, Ops &&ops, uint32_t W0, uint32_t W1,
                                             v16i (&acc0)[2][2], v16i (&acc1)[2][2]) {
  v16f f0[2][2], f1[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) f0[x][y][e] = f1[x][y][e] = 0.f;
  mfma_class_fp4<kDepth, kRaw, 2>(load_words, ops, 0, W0, f0);
  mfma_class_fp4<kDepth, kRaw, 2>(load_words, ops, W0, W0 + W1, f1);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        acc0[x][y][e] = (int)(uint32_t)f0[x][y][e];
        acc1[x][y][e] = (int)(uint32_t)f1[x][y][e];
      }
}

// Both classes with FP4 operands for the narrow kernels: counts of at most 16
// bits.  Class 0's counts wait as 16-bit pairs while class 1 accumulates;
// the result Q holds class 0 in the low and class 1 in the high 16 bits of
// each output element (register e of block (x, y)).
template <int kDepth, int kRaw, int FA = 2, typename Load, typename Ops>
__device__ __forceinline__ void contract_fp4_narrow(Load &&load_words, Ops &&ops, uint32_t W0,
                                                    uint32_t W1, uint32_t (&Q)[FA][2][16]) {
  v16f f[FA][2];
#pragma unroll
  for (int x = 0; x < FA; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) f[x][y][e] = 0.f;
  mfma_class_fp4<kDepth, kRaw, FA>(load_words, ops, 0, W0, f);
  uint32_t P0[FA][2][8];
#pragma unroll
  for (int x = 0; x < FA; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        P0[x][y][i] = (uint32_t)f[x][y][2 * i] | ((uint32_t)f[x][y][2 * i + 1] << 16);
        f[x][y][2 * i] = f[x][y][2 * i + 1] = 0.f;
      }
  mfma_class_fp4<kDepth, kRaw, FA>(load_words, ops, W0, W0 + W1, f);
#pragma unroll
  for (int x = 0; x < FA; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e)
        Q[x][y][e] = ((P0[x][y][e >> 1] >> (16 * (e & 1))) & 0xFFFFu) | ((uint32_t)f[x][y][e] << 16);
}

// Both classes with FP4 operands for the dual kernels: class-0 products are
// scaled by 2^2 and class-1 products by 2^(s+2) (s = bit length of m0, given
// by the caller), so the single FP32 accumulator holds u = 4 (c0 + 2^s c1), a
// multiple of 4 below 2^26 and so an exact integer like c0 + 2^s c1 < 2^24.
// Q holds 4 c0 | 4 c1 << 16 (the scoring's byte offsets; c0, c1 < 2^13):
// u >> (s + 2) = c1 since 4 c0 < 2^(s+2), and u + c1 (2^18 - 2^(s+2)) moves
// 4 c1 to bit 16.
template <int kDepth, int kRaw, int FA = 2, typename Load, typename Ops>
__device__ __forceinline__ void contract_fp4_dual(Load &&load_words, Ops &&ops, uint32_t W0,
                                                  uint32_t W1, uint32_t s,
                                                  uint32_t (&Q)[FA][2][16]) {
  v16f f[FA][2];
#pragma unroll
  for (int x = 0; x < FA; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) f[x][y][e] = 0.f;
  mfma_class_fp4<kDepth, kRaw, FA>(load_words, ops, 0, W0, f, kScaleOne + 2);
  mfma_class_fp4<kDepth, kRaw, FA>(load_words, ops, W0, W0 + W1, f, kScaleOne + 2 + (int)s);
  const uint32_t k = (1u << 18) - (1u << (s + 2));
#pragma unroll
  for (int x = 0; x < FA; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const uint32_t u = (uint32_t)f[x][y][e];
        Q[x][y][e] = u + (u >> (s + 2)) * k;
      }
}

// A count register of the packed contractions as 4 c0 | 4 c1 << 16: the dual
// kernels' registers already are, the narrow kernels' hold c0 | c1 << 16
template <bool kDual>
__device__ __forceinline__ uint32_t packed_x4(uint32_t q) {
  return kDual ? q : q << 2;
}

// bit length of x (0 for 0)
__device__ __forceinline__ uint32_t bit_len(uint32_t x) { return x ? 32u - __clz(x) : 0u; }

// Counts of both classes of output register e of block (x, y), the lane's own
// column: from the packed registers (narrow, dual) or the per-class ones
template <int FMT>
__device__ __forceinline__ void own_counts(const v16i (&acc0)[2][2], const v16i (&acc1)[2][2],
                                           const uint32_t (&Q)[2][2][16], int x, int y, int e,
                                           uint32_t (&o)[2]) {
  if constexpr (FMT == kMfmaF4Dual) {
    o[0] = (Q[x][y][e] & 0xFFFFu) >> 2;
    o[1] = Q[x][y][e] >> 18;
  } else if constexpr (FMT == kMfmaF4Narrow) {
    o[0] = Q[x][y][e] & 0xFFFFu;
    o[1] = Q[x][y][e] >> 16;
  } else {
    o[0] = (uint32_t)acc0[x][y][e];
    o[1] = (uint32_t)acc1[x][y][e];
  }
}

// The order-2 FP4 contraction of one wave: pairs (a0 + [0, 32)) x (j0 +
// [0, 32)), fragment g of either operand genotype row g of 32 variants.  A
// lane loads both rows of its variant on each side in one 16-byte load per
// word pair (lane half h: word w + h).  Counts in Q (narrow, dual: both
// classes per register) or acc0, acc1 (per class).
template <int FMT>
__device__ __forceinline__ void pairs_contract_fp4(const JV &v, uint32_t a0, uint32_t j0, uint32_t lane,
                                                   v16i (&acc0)[2][2], v16i (&acc1)[2][2],
                                                   uint32_t (&Q)[2][2][16]) {
  const uint32_t n = v.n;
  const uint32_t r = lane & 31, h = lane >> 5;
  const FI_GLOBAL char *Bvc = reinterpret_cast<const FI_GLOBAL char *>(as_global(v.Bv));
  const size_t word_bytes = (size_t)v.n_pad * 16;  // one word of every variant
  // words in pairs: lane half h reads word w + h whole
  const uint32_t hw = h * (uint32_t)word_bytes;
  const uint32_t ol = r * 16 + hw;
  // the last step of an odd word count: lanes of half 1 read word w itself,
  // their A rows from the zero rows of padding variant n
  const uint32_t oat = h ? (n - a0) * 16 : r * 16;
  auto load_words = [&](uint32_t w, auto tail, u64 (&x)[4]) {
    const FI_GLOBAL char *sa = Bvc + (size_t)w * word_bytes + (size_t)a0 * 16;
    const FI_GLOBAL char *sj = Bvc + (size_t)w * word_bytes + (size_t)j0 * 16;
    constexpr bool kTail = decltype(tail)::value;
    const v4u qa = ld128(sa, kTail ? oat : ol);  // both rows of the lane's variants
    const v4u qj = ld128(sj, kTail ? ol - hw : ol);
    x[0] = (u64)qa[0] | ((u64)qa[1] << 32);
    x[1] = (u64)qa[2] | ((u64)qa[3] << 32);
    x[2] = (u64)qj[0] | ((u64)qj[1] << 32);
    x[3] = (u64)qj[2] | ((u64)qj[3] << 32);
  };
  const auto ops = [](const u64 (&x)[4], int half, v8i (&E)[4]) {
    const int sh = 32 * half;
    E[0] = expand32_fp4_a((uint32_t)(x[0] >> sh));
    E[1] = expand32_fp4_a((uint32_t)(x[1] >> sh));
    E[2] = expand32_fp4_b((uint32_t)(x[2] >> sh));
    E[3] = expand32_fp4_b((uint32_t)(x[3] >> sh));
  };
  if constexpr (FMT == kMfmaF4Narrow) contract_fp4_narrow<2, 4>(load_words, ops, v.W0, v.W1, Q);
  else if constexpr (FMT == kMfmaF4Dual)
    contract_fp4_dual<2, 4>(load_words, ops, v.W0, v.W1, bit_len(v.m0), Q);
  else contract_fp4<2, 4>(load_words, ops, v.W0, v.W1, acc0, acc1);
}

// One wave: pairs (a0 + [0, 32)) x (j0 + [0, 32)).
template <int FMT, bool LDS_F>
__device__ __forceinline__ void wave_pairs(const JV &v, uint32_t a0, uint32_t j0, uint32_t lane,
                                           const u64 *lut, const FI_LDS float *Fl) {
  const uint32_t n = v.n;
  const uint32_t r = lane & 31, h = lane >> 5;
  const size_t word_stride = (size_t)v.n_pad * 2;
  const FI_GLOBAL u64 *Bv = as_global(v.Bv);
  // lane r of fragment f: variant a0 + r (A) and j0 + r (B) at genotype f
  const FI_GLOBAL u64 *pa = Bv + (size_t)(a0 + r) * 2;
  const FI_GLOBAL u64 *pj = Bv + (size_t)(j0 + r) * 2;
  v16i acc0[2][2], acc1[2][2];  // int8, FP4: counts per class
  uint32_t Q[2][2][16];         // narrow FP4: both classes per register
  if constexpr (FMT != kMfmaI8) {
    pairs_contract_fp4<FMT>(v, a0, j0, lane, acc0, acc1, Q);
  } else {
    zero_acc(acc0, acc1);
    auto load_words = [&](uint32_t w, u64 (&x)[4]) {
      const size_t o = (size_t)w * word_stride;
      x[0] = pa[o];
      x[1] = pa[o + 1];
      x[2] = pj[o];
      x[3] = pj[o + 1];
    };
    auto prep = [](const u64 (&x)[4], u64 (&o)[4]) {
#pragma unroll
      for (int f = 0; f < 4; ++f) o[f] = x[f];
    };
    mfma_class<3, 4>(load_words, prep, 0, v.W0, h, lut, acc0);
    mfma_class<3, 4>(load_words, prep, v.W0, v.W0 + v.W1, h, lut, acc1);
  }

  // Output block (fa, fb): lane l holds column l mod 32, variant j0 + (l mod
  // 32) at genotype g_j = fb; register e = 4 q + i holds row 8 q + 4 h + i,
  // variant a0 + 8 q + 4 h + i at genotype g_a = fa.  So each lane holds the
  // four {0,1}^2 counts of its 16 pairs (q = 0..3, i = 0..3) and scores them.
  const MiConst mc = mi_const(v);
  const FI_GLOBAL uint32_t *marg = as_global(v.marg);
  const uint32_t mcls[2] = {v.m0, v.m1};
  // the scoring on packed byte offsets (both class sizes below 16,384; the
  // dual kernel's always are), with the table in LDS
  constexpr bool kPackable = (FMT == kMfmaF4Dual || FMT == kMfmaF4Narrow) && LDS_F;
  const bool packed = FMT == kMfmaF4Dual || (v.m0 < 16384u && v.m1 < 16384u);
  const uint32_t m4 = pack_x4(v.m0, v.m1);
  // the scoring reads the f table from the workgroup's LDS copy (LDS_F:
  // it holds this job's table) or from global memory
  float thr = current_threshold(v);
  // class counts (rows 0 and 1 of a variant) in one 16-byte read
  auto marg2 = [&](uint32_t var, uint32_t (&M)[2][2]) {
    const FI_GLOBAL v2u32 *p = reinterpret_cast<const FI_GLOBAL v2u32 *>(marg + (size_t)var * 6);  // 8-byte aligned
    const v2u32 u0 = p[0], u1 = p[1];
    M[0][0] = u0.x;
    M[0][1] = u0.y;
    M[1][0] = u1.x;
    M[1][1] = u1.y;
  };
  auto score = [&](auto F) {
    // the class counts of the lane's last variant, then per first variant
    const uint32_t j = j0 + r, jj = j < n ? j : n - 1;
    uint32_t Mj[2][2];  // [g][class]
    marg2(jj, Mj);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t a = a0 + 8 * q + 4 * h + i;
        const uint32_t aa = a < n ? a : n - 1;
        uint32_t Ma[2][2];  // [g][class]
        marg2(aa, Ma);
        {
          if (kPackable && packed) {
            // the 9 cells as packed byte offsets, 4 x count per class half,
            // as in the order-3 walk
            uint32_t C4[2][2];  // [g_a][g_j]
#pragma unroll
            for (int fa = 0; fa < 2; ++fa)
#pragma unroll
              for (int fb = 0; fb < 2; ++fb) C4[fa][fb] = packed_x4<FMT == kMfmaF4Dual>(Q[fa][fb][4 * q + i]);
            const bool active = a < j && j < n;
            float fs = mc.c;
            if (active) {
              uint32_t Ma4[2], Mj4[2];
#pragma unroll
              for (int gg = 0; gg < 2; ++gg) {
                Ma4[gg] = pack_x4(Ma[gg][0], Ma[gg][1]);
                Mj4[gg] = pack_x4(Mj[gg][0], Mj[gg][1]);
              }
              const uint32_t t9[9] = {C4[0][0], C4[0][1], Ma4[0] - C4[0][0] - C4[0][1],
                                      C4[1][0], C4[1][1], Ma4[1] - C4[1][0] - C4[1][1],
                                      Mj4[0] - C4[0][0] - C4[1][0], Mj4[1] - C4[0][1] - C4[1][1],
                                      m4 - Ma4[0] - Ma4[1] - Mj4[0] - Mj4[1] + C4[0][0] + C4[0][1] +
                                          C4[1][0] + C4[1][1]};
              const FI_LDS char *Fb = (const FI_LDS char *)Fl;
              float f0[9], f1[9], f01[9];
#pragma unroll
              for (int x = 0; x < 9; ++x) {
                const uint32_t o0 = t9[x] & 0xFFFFu, o1 = t9[x] >> 16;
                f0[x] = *(const FI_LDS float *)(Fb + o0);
                f1[x] = *(const FI_LDS float *)(Fb + o1);
                f01[x] = *(const FI_LDS float *)(Fb + o0 + o1);
              }
#pragma unroll
              for (int x = 0; x < 9; ++x) fs += (f0[x] + f1[x]) - f01[x];
            }
            if (emit_with(v, active, fs * mc.inv_m,
                          [&] { return (u64)a * (n - 1) - (u64)a * (a - 1) / 2 + (j - a - 1); }, thr,
                          lane) >= kRefreshAppends)
              thr = current_threshold_lanes(v);
            continue;
          }
          uint32_t cnt[2][2][2];  // [g_a][g_j][class]
#pragma unroll
          for (int fa = 0; fa < 2; ++fa)
#pragma unroll
            for (int fb = 0; fb < 2; ++fb) {
              uint32_t o[2];
              own_counts<FMT>(acc0, acc1, Q, fa, fb, 4 * q + i, o);
              cnt[fa][fb][0] = o[0];
              cnt[fa][fb][1] = o[1];
            }
          const bool active = a < j && j < n;
          using E = decltype(+F[0]);  // the table's element type, without its address space
          E fs = mi_start<E>(mc);
          if (active) {
            uint32_t t9[9][2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              const uint32_t (&C)[2][2][2] = cnt;
              t9[0][c] = C[0][0][c];
              t9[1][c] = C[0][1][c];
              t9[2][c] = Ma[0][c] - C[0][0][c] - C[0][1][c];
              t9[3][c] = C[1][0][c];
              t9[4][c] = C[1][1][c];
              t9[5][c] = Ma[1][c] - C[1][0][c] - C[1][1][c];
              t9[6][c] = Mj[0][c] - C[0][0][c] - C[1][0][c];
              t9[7][c] = Mj[1][c] - C[0][1][c] - C[1][1][c];
              t9[8][c] = mcls[c] - Ma[0][c] - Ma[1][c] - Mj[0][c] - Mj[1][c] + C[0][0][c] +
                         C[0][1][c] + C[1][0][c] + C[1][1][c];
              // every count is at most the class size; in global memory the
              // clamp keeps the reads inside [0, m] whatever the counts hold
              // (LDS reads cannot fault)
              if (!LDS_F) {
#pragma unroll
                for (int x = 0; x < 9; ++x) t9[x][c] = min(t9[x][c], mcls[c]);
              }
            }
            // the 27 table reads issued together
            E f0[9], f1[9], f01[9];
#pragma unroll
            for (int x = 0; x < 9; ++x) {
              f0[x] = F[t9[x][0]];
              f1[x] = F[t9[x][1]];
              f01[x] = F[t9[x][0] + t9[x][1]];
            }
#pragma unroll
            for (int x = 0; x < 9; ++x) fs += (f0[x] + f1[x]) - f01[x];
          }
          // the rank is computed by appending lanes only: lexicographic rank of
          // (a, j) = sum over a' < a of (n - 1 - a'), plus j - a - 1
          if (emit_with(v, active, mi_finish(fs, mc),
                        [&] { return (u64)a * (n - 1) - (u64)a * (a - 1) / 2 + (j - a - 1); }, thr,
                        lane) >= kRefreshAppends)
            thr = current_threshold_lanes(v);
        }
      }
    }
  };
  if constexpr (LDS_F) score(lds_table<2, FMT>(Fl));
  else score(as_global(v.Fh));
}

// One wave: prefixes (a_first + [0, 16), b) x last variants (j0 + [0, 32)).
template <int FMT, bool LDS_F>
__device__ __forceinline__ void wave_prefix3(const Globals &g, const JV &v, uint32_t b,
                                             uint32_t a_first, uint32_t j0, uint32_t lane,
                                             const u64 *lut, const FI_LDS float *Fl) {
  const uint32_t n = v.n;
  const uint32_t r = lane & 31, h = lane >> 5;
  const size_t word_stride = (size_t)v.n_pad * 2;
  const FI_GLOBAL u64 *Bv = as_global(v.Bv);
  const FI_GLOBAL u64 *Bs = as_global(v.Bs);
  // A rows: lane r of fragment f is prefix a_first + r / 2 with its genotype
  // row g_a = r & 1, AND-ed with row g_b = f of b (a fragment fixes g_b, so a
  // lane's prefix row serves both fragments); prefixes a >= b count nothing:
  // their lanes read a zero word
  const uint32_t ga = r & 1, ar = a_first + (r >> 1);
  const FI_GLOBAL u64 *pb = Bs + (size_t)b * 4 * v.wcap;
  const FI_GLOBAL u64 *pa = Bs + (size_t)min(ar, b - 1) * 4 * v.wcap + (ar < b ? ga : 3);
  // B rows: lane r of fragment f is last variant j0 + r at genotype g_j = f
  const FI_GLOBAL u64 *pj = Bv + (size_t)(j0 + r) * 2;
  v16i acc0[2][2], acc1[2][2];  // int8, FP4: counts per class
  uint32_t Q[2][2][16];         // narrow FP4: both classes per register
  if constexpr (FMT != kMfmaI8) {
    // the lane's 32-bit half of each word, every operand from the
    // variant-fastest rows (Bv): a wave-uniform base per word (scalar
    // arithmetic) plus 32-bit lane offsets.  A fragment's 8 prefixes are
    // consecutive variants, so each load of the wave reads contiguous bytes;
    // prefixes a >= b read variant n, a padding variant whose words are zero.
    const FI_GLOBAL char *Bvc = reinterpret_cast<const FI_GLOBAL char *>(Bv);
    const size_t word_bytes = (size_t)v.n_pad * 16;  // Bv bytes of one word
    // words in pairs: lane half h reads word w + h whole
    const uint32_t hw = h * (uint32_t)word_bytes;
    const uint32_t oa = (ar < b ? ar : n) * 16 + ga * 8 + hw;
    const uint32_t ob = b * 16 + hw, ol = (j0 + r) * 16 + hw;
    // the last step of an odd word count: lanes of half 1 read word w itself,
    // with the rows of b replaced by the zero rows of padding variant n, so that
    // their A operands (a row AND a row of b) vanish
    const uint32_t obt = h ? n * 16 : ob;
    auto load_words = [&](uint32_t w, auto tail, u64 (&x)[5]) {
      const FI_GLOBAL char *sw = Bvc + (size_t)w * word_bytes;
      constexpr bool kTail = decltype(tail)::value;
      const uint32_t d = kTail ? hw : 0u;
      x[0] = ld64(sw, oa - d);
      const v4u qj = ld128(sw, ol - d);  // both rows of the lane's last variant
      x[1] = (u64)qj[0] | ((u64)qj[1] << 32);
      x[2] = (u64)qj[2] | ((u64)qj[3] << 32);
      const v4u q = ld128(sw, kTail ? obt : ob);  // both rows of b
      x[3] = (u64)q[0] | ((u64)q[1] << 32);
      x[4] = (u64)q[2] | ((u64)q[3] << 32);
    };
    // A fragment f: row of a AND row f of b; B fragment f: row f of the last
    // variants
    const auto ops = [](const u64 (&x)[5], int half, v8i (&E)[4]) {
      const int sh = 32 * half;
      E[0] = expand32_fp4_and((uint32_t)(x[0] >> sh), (uint32_t)(x[3] >> sh));
      E[1] = expand32_fp4_and((uint32_t)(x[0] >> sh), (uint32_t)(x[4] >> sh));
      E[2] = expand32_fp4_b((uint32_t)(x[1] >> sh));
      E[3] = expand32_fp4_b((uint32_t)(x[2] >> sh));
    };
    if constexpr (FMT == kMfmaF4Narrow) contract_fp4_narrow<2, 5>(load_words, ops, v.W0, v.W1, Q);
    else if constexpr (FMT == kMfmaF4Dual)
      contract_fp4_dual<2, 5>(load_words, ops, v.W0, v.W1, bit_len(v.m0), Q);
    else contract_fp4<2, 5>(load_words, ops, v.W0, v.W1, acc0, acc1);
  } else {
    zero_acc(acc0, acc1);
    auto load_words = [&](uint32_t w, u64 (&x)[5]) {
      x[0] = pa[(size_t)w * 4];
      const size_t o = (size_t)w * word_stride;
      x[1] = pj[o];
      x[2] = pj[o + 1];
      x[3] = pb[(size_t)w * 4];
      x[4] = pb[(size_t)w * 4 + 1];
    };
    auto prep = [](const u64 (&x)[5], u64 (&o)[4]) {
      o[0] = x[0] & x[3];
      o[1] = x[0] & x[4];
      o[2] = x[1];
      o[3] = x[2];
    };
    mfma_class<3, 5>(load_words, prep, 0, v.W0, h, lut, acc0);
    mfma_class<3, 5>(load_words, prep, v.W0, v.W0 + v.W1, h, lut, acc1);
  }

  // Output block (f, fb): lane l holds column l mod 32, last variant j0 + (l
  // mod 32) at genotype g_j = fb; register e = 4 q + 2 s + g_a holds row 8 q +
  // 4 h + 2 s + g_a, i.e. prefix a_first + 4 q + 2 h + s at genotypes g_a and
  // g_b = f.  So each lane holds all eight {0,1}^3 counts of its last variant
  // with 8 prefixes (q = 0..3, s = 0, 1) and scores those combinations.
  const MiConst mc = mi_const(v);
  const FI_GLOBAL uint32_t *marg = as_global(v.marg);
  const FI_GLOBAL uint32_t *PT = as_global(v.pairs);
  const uint32_t mcls[2] = {v.m0, v.m1};
  uint32_t Mb[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int c = 0; c < 2; ++c) Mb[x][c] = marg[(size_t)b * 6 + 2 * x + c];
  // the scoring reads the f table from the workgroup's LDS copy (LDS_F:
  // it holds this job's table) or from global memory
  float thr = current_threshold(v);
  // the walk on packed counts, 4 x count per class half (byte offsets into
  // the LDS table: both class sizes below 16,384; the dual kernel's always
  // are)
  constexpr bool kPackable = (FMT == kMfmaF4Dual || FMT == kMfmaF4Narrow) && LDS_F;
  // packed pair tables exist for jobs of fewer than 16,384 samples (every job
  // of the dual kernel)
  const bool packed = FMT == kMfmaF4Dual || v.pairs4 != nullptr;
  uint32_t Mb4[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) Mb4[x] = pack_x4(Mb[x][0], Mb[x][1]);
  const uint32_t m4 = pack_x4(v.m0, v.m1);
  // the lane's last variant j: its class counts and (b, j) pair table are
  // read once for the lane's 8 prefixes
  const uint32_t j = j0 + r, jj = j < n ? j : n - 1;
  auto prefix_of = [&](int q, int s) { return a_first + 4 * q + 2 * h + s; };
  auto score_packed = [&]() {
    const FI_GLOBAL v4u *PT4 = reinterpret_cast<const FI_GLOBAL v4u *>(as_global(v.pairs4));
    uint32_t Mj4[2], bj4[2][2];
    {
      const v4u qb = PT4[(size_t)b * v.n_pad + jj];
      bj4[0][0] = qb[0];
      bj4[0][1] = qb[1];
      bj4[1][0] = qb[2];
      bj4[1][1] = qb[3];
#pragma unroll
      for (int x = 0; x < 2; ++x) Mj4[x] = pack_x4(marg[(size_t)jj * 6 + 2 * x], marg[(size_t)jj * 6 + 2 * x + 1]);
    }
    const FI_LDS char *Fb = (const FI_LDS char *)Fl;
    // a prefix's (a, j) and (a, b) pair-table entries are loaded one prefix
    // ahead of its scoring, so that their latency overlaps the previous
    // prefix's
    auto entry = [&](int i, uint32_t col) {
      const uint32_t a = prefix_of(i >> 1, i & 1);
      return PT4[(size_t)(a < b ? a : b - 1) * v.n_pad + col];
    };
    v4u qj_next = entry(0, jj), qb_next = entry(0, b);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const v4u qj = qj_next, qb = qb_next;
        if (2 * q + s < 7) {
          qj_next = entry(2 * q + s + 1, jj);
          qb_next = entry(2 * q + s + 1, b);
        }
        const uint32_t a = prefix_of(q, s);
        const uint32_t aa = a < b ? a : b - 1;
        uint32_t ab4[2][2], Ma4[2], aj4[2][2];
        {
          ab4[0][0] = qb[0];
          ab4[0][1] = qb[1];
          ab4[1][0] = qb[2];
          ab4[1][1] = qb[3];
          aj4[0][0] = qj[0];
          aj4[0][1] = qj[1];
          aj4[1][0] = qj[2];
          aj4[1][1] = qj[3];
        }
#pragma unroll
        for (int x = 0; x < 2; ++x) Ma4[x] = pack_x4(marg[(size_t)aa * 6 + 2 * x], marg[(size_t)aa * 6 + 2 * x + 1]);
        const uint32_t pre[2] = {aa, b};
        {
          uint32_t D4[2][2][2];  // [g_a][g_b][g_j], packed x 4
#pragma unroll
          for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int fb = 0; fb < 2; ++fb)
#pragma unroll
              for (int g = 0; g < 2; ++g) D4[g][f][fb] = packed_x4<FMT == kMfmaF4Dual>(Q[f][fb][4 * q + 2 * s + g]);
          const bool active = a < b && j < n;
          // fixed point (the LDS table holds Fq): the class terms f(n0) + f(n1)
          // added to fs, the f(n0 + n1) terms to fm (three-input adds take two
          // terms at a time), the score is fs - fm
          uint32_t fs = mc.q0, fm = 0;
          if (active) {
            constexpr int kGroup = 3;
            uint32_t o0[kGroup], o1[kGroup];
            int nc = 0;
            walk_order3_packed(D4, ab4, aj4, bj4, Ma4, Mb4, Mj4, m4, [&](uint32_t p) {
              o0[nc] = p & 0xFFFFu;
              o1[nc] = p >> 16;
              if (++nc == kGroup) {
                uint32_t f0[kGroup], f1[kGroup], f01[kGroup];
#pragma unroll
                for (int x = 0; x < kGroup; ++x) {
                  f0[x] = *(const FI_LDS uint32_t *)(Fb + o0[x]);
                  f1[x] = *(const FI_LDS uint32_t *)(Fb + o1[x]);
                  f01[x] = *(const FI_LDS uint32_t *)(Fb + o0[x] + o1[x]);
                }
#pragma unroll
                for (int x = 0; x < kGroup; ++x) fs += f0[x] + f1[x];
#pragma unroll
                for (int x = 0; x < kGroup; ++x) fm += f01[x];
                // fs is kept in order (pin_sum); fm's additions are left to
                // the compiler, which here saves instructions without spilling
                pin_sum(fs);
                nc = 0;
              }
            });
          }
          if (emit_with(v, active, mi_fixed(fs - fm, mc),
                        [&] { return lex_rank_prefix(g, n, 3, pre) + (u64)(j - b - 1); }, thr,
                        lane) >= kRefreshAppends)
            thr = current_threshold_lanes(v);
        }
      }
    }
  };
  // the per-class walk (counts of 16 bits or more per class)
  auto score = [&](auto F) {
    {
      uint32_t Mj[2][2], bj[8];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int c = 0; c < 2; ++c) Mj[x][c] = marg[(size_t)jj * 6 + 2 * x + c];
      load_pair(PT + ((size_t)b * v.n_pad + jj) * 8, bj);
      // the narrow kernel (registers to spare at 2 waves per SIMD) loads each
      // prefix's (a, j) pair entry one prefix ahead, as the packed walk does
      constexpr bool kAhead = FMT == kMfmaF4Narrow;
      auto load_aj = [&](int i, uint32_t (&o)[8]) {
        const uint32_t a = prefix_of(i >> 1, i & 1);
        load_pair(PT + ((size_t)(a < b ? a : b - 1) * v.n_pad + jj) * 8, o);
      };
      uint32_t aj_next[8];
      if constexpr (kAhead) load_aj(0, aj_next);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const uint32_t a = prefix_of(q, s);
          uint32_t D[2][2][2][2];  // [class][g_a][g_b][g_j]
#pragma unroll
          for (int f = 0; f < 2; ++f)
#pragma unroll
            for (int fb = 0; fb < 2; ++fb)
#pragma unroll
              for (int g = 0; g < 2; ++g) {
                uint32_t o[2];
                own_counts<FMT>(acc0, acc1, Q, f, fb, 4 * q + 2 * s + g, o);
                D[0][g][f][fb] = o[0];
                D[1][g][f][fb] = o[1];
              }
          const bool active = a < b && j < n;
          const uint32_t aa = a < b ? a : b - 1;
          uint32_t ab[8], aj[8], Ma[2][2];
          load_pair(PT + ((size_t)aa * v.n_pad + b) * 8, ab);
          if constexpr (kAhead) {
#pragma unroll
            for (int x = 0; x < 8; ++x) aj[x] = aj_next[x];
            if (2 * q + s < 7) load_aj(2 * q + s + 1, aj_next);
          } else {
            load_pair(PT + ((size_t)aa * v.n_pad + jj) * 8, aj);
          }
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int c = 0; c < 2; ++c) Ma[x][c] = marg[(size_t)aa * 6 + 2 * x + c];
          const Order3Parts parts = {D, ab, aj, bj, Ma, Mb, Mj, mcls};
          using E = decltype(+F[0]);  // the table's element type, without its address space
          E fs = mi_start<E>(mc);
          if (active) {
            // the cells in groups of 3, each group's 9 table reads issued
            // together rather than one cell at a time
            constexpr int kGroup = 3;
            uint32_t c0[kGroup], c1[kGroup];
            int nc = 0;
            walk_order3(parts, [&](uint32_t n0, uint32_t n1) {
              // every count is at most its class size; in global memory the
              // clamps keep the reads inside [0, m] whatever the counts hold
              // (LDS reads cannot fault)
              c0[nc] = LDS_F ? n0 : min(n0, mcls[0]);
              c1[nc] = LDS_F ? n1 : min(n1, mcls[1]);
              if (++nc == kGroup) {
                E f0[kGroup], f1[kGroup], f01[kGroup];
#pragma unroll
                for (int x = 0; x < kGroup; ++x) {
                  f0[x] = F[c0[x]];
                  f1[x] = F[c1[x]];
                  f01[x] = F[c0[x] + c1[x]];
                }
#pragma unroll
                for (int x = 0; x < kGroup; ++x) fs += (f0[x] + f1[x]) - f01[x];
                if constexpr (std::is_same_v<E, uint32_t>) pin_sum(fs);
                nc = 0;
              }
            });
          }
          const uint32_t pre[2] = {aa, b};
          if (emit_with(v, active, mi_finish(fs, mc),
                        [&] { return lex_rank_prefix(g, n, 3, pre) + (u64)(j - b - 1); }, thr,
                        lane) >= kRefreshAppends)
            thr = current_threshold_lanes(v);
        }
      }
    }
  };
  if constexpr (kPackable) {
    if (packed) {
      score_packed();
      return;
    }
  }
  if constexpr (LDS_F) score(lds_table<3, FMT>(Fl));
  else score(as_global(v.Fh));
}

// ---------------------------------------------------------------------------
// Orders 4 and 5: every genotype row of the prefix on the matrix cores
// ---------------------------------------------------------------------------
//
// For a prefix P of k - 1 variants and a last variant j the table has 3^k
// cells.  Rows 0 .. 3^(k-1) - 1 of the A operand are the prefix's genotype
// rows (the AND of one row of each prefix variant, first variant most
// significant), the B operand holds rows g = 0, 1 of the last variants, so
// the matrix cores give every cell with g_j in {0, 1}; the cells with g_j = 2
// are the prefix row's count (its popcount, taken while the A operand is
// formed) minus those two.  No lower-order tables are needed.  A wave owns one
// prefix and 64 last variants: at order 4 the 27 prefix rows fill one
// fragment (1 x 4 blocks of 32 x 32 outputs), at order 5 the 81 rows fill
// three (3 x 2 blocks, the 64 last variants in two passes of 32; measured:
// 21 % faster than 3 x 1 blocks in four passes despite a few register
// spills, with a 2-word ring).  FP4
// operands, counts kept in 16 bits (jobs of at most 20,447 samples), f table
// in LDS.

constexpr uint32_t pow3(int e) { return e == 0 ? 1u : 3u * pow3(e - 1); }

template <int K>
struct RowsShape {
  static constexpr uint32_t R = pow3(K - 1);                // prefix rows
  static constexpr int FA = (int)((R + 31) / 32);           // A fragments
  static constexpr int JB = FA == 1 ? 4 : 2;                // B fragments per pass
  static constexpr int NSB = 4 / JB;                        // passes over 64 last variants
  static constexpr int kRaw = FA * (K - 1) + JB;            // words a lane loads per word index
  static constexpr int kDepth = FA == 1 ? 4 : 2;            // register ring depth
};

// One class: words [wbeg, wend) into acc; np[fa] accumulates the popcount of
// the lane's A word of fragment fa (its prefix row's count over the lane's
// half of the samples)
template <int kDepth, int kRaw, int FA, int JB, typename Load, typename Prep>
__device__ __forceinline__ void mfma_rows_class(Load &&load_words, Prep &&prep, uint32_t wbeg,
                                                uint32_t wend, v16f (&acc)[FA][JB],
                                                uint32_t (&np)[FA], int scale_a = kScaleOne) {
  if (wbeg >= wend) return;
  const uint32_t wlast = wend - 1;
  uint32_t X[kDepth][kRaw];
#pragma unroll
  for (int u = 0; u < kDepth; ++u) load_words(min(wbeg + u, wlast), X[u]);
  auto step = [&](int slot) {
    uint32_t O[FA + JB];
    prep(X[slot], O);
    v8i E[FA + JB];
#pragma unroll
    for (int f = 0; f < FA + JB; ++f) E[f] = f < FA ? expand32_fp4_a(O[f]) : expand32_fp4_b(O[f]);
#pragma unroll
    for (int fa = 0; fa < FA; ++fa) np[fa] += __builtin_popcount(O[fa]);
#pragma unroll
    for (int fa = 0; fa < FA; ++fa)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)
        acc[fa][jb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
            E[fa], E[FA + jb], acc[fa][jb], kFmtFp4, kFmtFp4, 0, scale_a, 0, kScaleOne);
  };
  uint32_t w = wbeg;
  for (; w + kDepth <= wend; w += kDepth) {
#pragma unroll
    for (int u = 0; u < kDepth; ++u) {
      step(u);
      load_words(min(w + u + kDepth, wlast), X[u]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int u = 0; u < kDepth - 1; ++u)
    if (w + u < wend) step(u);
}

// Words of the prefix variants' rows a wave stages in LDS at a time: the
// rows of one class of a job of up to 2,048 samples, or a part of them
constexpr uint32_t kRowsChunk = 32;
template <int K>
constexpr uint32_t rows_stage_bytes() { return (uint32_t)(K - 1) * kRowsChunk * 32; }  // per wave

// One wave: prefix pre[0 .. K-2] x last variants j0 + [0, 64).  DUAL: both
// classes in one accumulator, class 1 scaled by 2^bitlen(m0) (exact while
// bitlen(m0) + bitlen(m1) <= 24), as in the dual order-2/3 kernels.
// The prefix variants' rows (wave-uniform: every lane needs one of the three
// genotype rows, or the zero word, of each variant) are copied to the wave's
// LDS region `stage` kRowsChunk words at a time by 16-byte loads, and the A
// operands are read from there: a load per variant and word instead of one
// per variant, word, fragment and pass.
template <int K, bool DUAL>
__device__ __forceinline__ void wave_rows(const Globals &g, const JV &v, const uint32_t (&pre)[K - 1],
                                          uint32_t j0, uint32_t lane, const FI_LDS float *F,
                                          FI_LDS char *stage) {
  typedef RowsShape<K> S;
  constexpr int FA = S::FA, JB = S::JB;
  const uint32_t n = v.n, b = pre[K - 2];
  const uint32_t r = lane & 31, h = lane >> 5, gl = lane & 1;
  const FI_GLOBAL char *Bsc = reinterpret_cast<const FI_GLOBAL char *>(as_global(v.Bs));
  const FI_GLOBAL char *Bvc = reinterpret_cast<const FI_GLOBAL char *>(as_global(v.Bv));
  const size_t vrow = (size_t)v.wcap * 32;         // Bs bytes of one variant
  const size_t word_bytes = (size_t)v.n_pad * 16;  // Bv bytes of one word
  // lane r of A fragment fa forms prefix row rho = 32 fa + r: genotype digit
  // i (base 3, first variant most significant) selects row g_i of variant
  // pre[i]; rows past 3^(K-1) read the zero word that follows the three
  // genotype words
  // (byte offsets of the lane's dword in a staged variant-word of 32 bytes,
  // variant i's rows at i * kRowsChunk * 32)
  uint32_t oa[FA][K - 1];
#pragma unroll
  for (int fa = 0; fa < FA; ++fa) {
    const uint32_t rho = 32 * fa + r;
    uint32_t t = rho;
#pragma unroll
    for (int i = K - 2; i >= 0; --i) {
      const uint32_t gi = rho < S::R ? t % 3 : 3;
      t /= 3;
      oa[fa][i] = (uint32_t)i * kRowsChunk * 32 + gi * 8 + 4 * h;
    }
  }
  // words [c0, c1) of every prefix variant's rows into the stage (c1 - c0 <=
  // kRowsChunk): 2 x 16 bytes per variant and word
  uint32_t c_first = 0;  // first word of the staged chunk
  auto stage_words = [&](uint32_t c0, uint32_t c1) {
    const uint32_t pieces = 2 * (c1 - c0);
#pragma unroll
    for (int i = 0; i < K - 1; ++i) {
      const FI_GLOBAL v4u *src =
          reinterpret_cast<const FI_GLOBAL v4u *>(Bsc + (size_t)pre[i] * vrow + (size_t)c0 * 32);
      FI_LDS v4u *dst = reinterpret_cast<FI_LDS v4u *>(stage + (uint32_t)i * kRowsChunk * 32);
      if (lane < pieces) dst[lane] = src[lane];
    }
    c_first = c0;
  };
  const uint32_t ol = r * 8 + 4 * h;
  const MiConst mc = mi_const(v);
  float thr = current_threshold(v);
#pragma unroll 1
  for (int sb = 0; sb < S::NSB; ++sb) {
    const uint32_t jbase = j0 + 16 * JB * sb;
    if (jbase >= n) break;
    auto load_words = [&](uint32_t w, uint32_t (&x)[S::kRaw]) {
      const FI_LDS char *sw = stage + (w - c_first) * 32;
#pragma unroll
      for (int i = 0; i < K - 1; ++i)
#pragma unroll
        for (int fa = 0; fa < FA; ++fa) x[fa * (K - 1) + i] = *(const FI_LDS uint32_t *)(sw + oa[fa][i]);
      const FI_GLOBAL char *sj = Bvc + (size_t)w * word_bytes + (size_t)jbase * 16;
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) x[FA * (K - 1) + jb] = ld32(sj, ol + 256 * jb);
    };
    // A word = AND of the prefix variants' rows
    auto prep = [](const uint32_t (&x)[S::kRaw], uint32_t (&o)[FA + JB]) {
#pragma unroll
      for (int fa = 0; fa < FA; ++fa) {
        uint32_t a = x[fa * (K - 1)];
#pragma unroll
        for (int i = 1; i < K - 1; ++i) a &= x[fa * (K - 1) + i];
        o[fa] = a;
      }
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) o[FA + jb] = x[FA * (K - 1) + jb];
    };
    // class 0, then class 1; counts as 16-bit pairs (class 0 low)
    v16f f[FA][JB];
    uint32_t np0[FA], np1[FA];
#pragma unroll
    for (int fa = 0; fa < FA; ++fa) {
      np0[fa] = np1[fa] = 0;
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int e = 0; e < 16; ++e) f[fa][jb][e] = 0.f;
    }
    // words [wb, we) of one class, kRowsChunk at a time through the stage
    auto class_words = [&](uint32_t wb, uint32_t we, uint32_t (&np)[FA], int scale_a) {
      for (uint32_t c0 = wb; c0 < we; c0 += kRowsChunk) {
        const uint32_t c1 = min(c0 + kRowsChunk, we);
        stage_words(c0, c1);
        mfma_rows_class<S::kDepth, S::kRaw, FA, JB>(load_words, prep, c0, c1, f, np, scale_a);
      }
    };
    class_words(0, v.W0, np0, kScaleOne);
    uint32_t P0[FA][JB][8];
    const uint32_t sh = bit_len(v.m0), low = (1u << sh) - 1u;
    if constexpr (DUAL) {
      class_words(v.W0, v.W0 + v.W1, np1, kScaleOne + (int)sh);
    } else {
#pragma unroll
      for (int fa = 0; fa < FA; ++fa)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            P0[fa][jb][i] = (uint32_t)f[fa][jb][2 * i] | ((uint32_t)f[fa][jb][2 * i + 1] << 16);
            f[fa][jb][2 * i] = f[fa][jb][2 * i + 1] = 0.f;
          }
      class_words(v.W0, v.W0 + v.W1, np1, kScaleOne);
    }
    // prefix row counts of both lane halves, both classes in one register
    uint32_t Np[FA];
#pragma unroll
    for (int fa = 0; fa < FA; ++fa) {
      const uint32_t c0 = np0[fa] + (uint32_t)__shfl_xor((int)np0[fa], 32);
      const uint32_t c1 = np1[fa] + (uint32_t)__shfl_xor((int)np1[fa], 32);
      Np[fa] = c0 | (c1 << 16);
    }
    // Output block (fa, jb): lane l holds column l mod 32 (last variant jbase
    // + 16 jb + (l mod 32) / 2, genotype l mod 2); register e holds prefix row
    // 32 fa + 8 (e / 4) + 4 h + e mod 4.  Each lane scores the cells of its
    // rows at its own g_j, and half of the rows' g_j = 2 cells (count = row
    // count - partner's - own, both classes at once: every part is a count);
    // MI is a sum over cells, so the four lanes of a combination (g_j, h)
    // add their parts and the lane with g_j = 0, h = 0 appends.
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) {
      float s = 0.f;
#pragma unroll
      for (int fa = 0; fa < FA; ++fa)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const uint32_t row = 8 * (e / 4) + 4 * h + (e % 4);
          const uint32_t rho = 32 * fa + row;
          uint32_t own;
          if constexpr (DUAL) {
            const uint32_t u = (uint32_t)f[fa][jb][e];
            own = (u & low) | ((u >> sh) << 16);
          } else {
            own = ((P0[fa][jb][e >> 1] >> (16 * (e & 1))) & 0xFFFFu) | ((uint32_t)f[fa][jb][e] << 16);
          }
          const uint32_t partner = xor1(own);
          const uint32_t nr = (uint32_t)__shfl((int)Np[fa], (int)row);
          if (rho < S::R) {
            const uint32_t a0 = own & 0xFFFFu, a1 = own >> 16;
            s += (F[a0] + F[a1]) - F[a0 + a1];
            if (gl == (uint32_t)(e & 1)) {
              const uint32_t c2 = nr - own - partner;
              const uint32_t b0 = c2 & 0xFFFFu, b1 = c2 >> 16;
              s += (F[b0] + F[b1]) - F[b0 + b1];
            }
          }
        }
      const float s2 = s + __uint_as_float(xor1(__float_as_uint(s)));
      const float s4 = s2 + __shfl_xor(s2, 32);
      const uint32_t j = jbase + 16 * jb + (r >> 1);
      const bool owner = gl == 0 && h == 0 && j < n;
      if (emit_with(v, owner, (mc.c + s4) * mc.inv_m,
                    [&] { return lex_rank_prefix(g, n, K, pre) + (u64)(j - b - 1); }, thr,
                    lane) >= kRefreshAppends)
        thr = current_threshold_lanes(v);
    }
  }
}

// Orders 4 and 5 on the matrix cores: the popcount kernel's tiles (a row per
// last prefix variant b, 4 prefixes x 64 last variants per tile, one prefix
// per wave).  The DUAL and the two-accumulator kernels run over the same
// tiles, each skipping the other's jobs.
template <int K, bool DUAL>
constexpr int rows_waves() { return DUAL && K == 4 ? 3 : 2; }
// the most f-table entries a launch of the kernel keeps in LDS (a launch
// sizes its LDS to the largest job of its group, up to this)
template <int K, bool DUAL>
constexpr int rows_f_entries() { return rows_waves<K, DUAL>() == 3 ? mfma_f_entries(kMfmaF4Dual) : mfma_f_entries(kMfmaF4Narrow); }
// dynamic LDS of a launch: the f table (rounded to 16 bytes), then each
// wave's stage
template <int K>
__host__ __device__ constexpr uint32_t rows_lds_bytes(uint32_t f_entries) {
  return (f_entries * 4 + 15) / 16 * 16 + kMfmaWaves * rows_stage_bytes<K>();
}

template <int K, bool DUAL>
__global__ __launch_bounds__(kMfmaWaves * 64, (rows_waves<K, DUAL>())) void mfma_rows_kernel(Globals g) {
  __shared__ u64 s_tile;
  extern __shared__ float s_f[];
  const uint32_t lane = lane_id();
  const uint32_t wave = uni(threadIdx.x >> 6);
  const FI_LDS float *Fl = (const FI_LDS float *)s_f;
  uint32_t f_job = ~0u;
  RowHint hint;  // the row of the workgroup's last tile
  if (!any_job(g, [](uint32_t m0, uint32_t m1, uint32_t m) {
        return (bit_len(m0) + bit_len(m1) <= 24 && m + 1 <= rows_f_entries<K, true>()) == DUAL;
      }))
    return;
  for (;;) {
    if (threadIdx.x == 0) s_tile = g.tile_base + atomicAdd(g.tile_counter, 1ull);
    __syncthreads();
    const u64 t = uni64(s_tile);
    __syncthreads();
    if (t >= g.total_tiles) break;
    JV v;
    const FI_CONST JobDesc *jd;
    u64 lt;
    if (!locate_tile(g, t, wave, kMfmaPilotEmits, v, jd, lt)) continue;
    // the host gives this kernel only such jobs
    if (v.path != kPathMfmaRows || v.k != (uint32_t)K) continue;
    {
      const bool dual = bit_len(v.m0) + bit_len(v.m1) <= 24 && v.m + 1 <= rows_f_entries<K, true>();
      if (dual != DUAL) {
        if (threadIdx.x == 0) {
          const u64 end = as_const(g.job_tile_start)[job_of_tile(g, t) + 1];
          atomicMax(g.tile_counter, end - g.tile_base);
        }
        continue;
      }
    }
    if (v.m + 1 > g.lds_f_entries) continue;
    {
      // the job's table, once the tile is known to be this kernel's (every
      // wave has finished the previous tile: the barriers above)
      const uint32_t jx = (uint32_t)(jd - as_const(g.jobs));
      if (jx != f_job) {
        const FI_GLOBAL float *Fh = as_global(uni_ptr(jd->Fh));
        for (uint32_t i = threadIdx.x; i <= v.m; i += blockDim.x) s_f[i] = Fh[i];
        f_job = jx;
        __syncthreads();
      }
    }
    cu64p rows = as_const(uni_ptr(jd->row_start));
    const uint32_t rl = hint.find(jd, lt);
    const u64 local = uni64(lt - rows[rl]);
    const uint32_t n = v.n;
    const uint32_t b = rl + (K - 2);
    const uint32_t nj = (n - 1 - b + 63) / 64;
    const u64 grp = local / nj;
    const uint32_t jb = (uint32_t)(local - grp * nj);
    u64 q = grp * kMfmaWaves + wave;
    if (q >= binom_small(g, b, K - 2)) continue;
    uint32_t pre[K - 1];
    pre[K - 2] = b;
    // colex unrank of the (K-2)-subset of [0, b) with index q
    colex_unrank<K - 2>(g, b, q, pre);
    FI_LDS char *stage = (FI_LDS char *)s_f + (g.lds_f_entries * 4 + 15) / 16 * 16 + wave * rows_stage_bytes<K>();
    wave_rows<K, DUAL>(g, v, pre, b + 1 + jb * 64, lane, Fl, stage);
  }
}

template <int K, bool DUAL>
int mfma_rows_grid(uint32_t f_entries) {
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, mfma_rows_kernel<K, DUAL>, kMfmaWaves * 64,
                                                     rows_lds_bytes<K>(f_entries));
  if (cus <= 0) cus = 256;
  if (per <= 0) per = 1;
  return cus * per;
}

uint32_t mfma_dual_max_samples(int order) {
  return order == 5 ? rows_f_entries<5, true>() - 1
         : order == 4 ? rows_f_entries<4, true>() - 1 : mfma_f_entries(kMfmaF4Dual) - 1;
}

uint32_t mfma_rows_max_entries(int order, bool dual) {
  if (order == 5) return dual ? rows_f_entries<5, true>() : rows_f_entries<5, false>();
  return dual ? rows_f_entries<4, true>() : rows_f_entries<4, false>();
}

int mfma_rows_grid_size(int order, bool dual, uint32_t f_entries) {
  if (order == 5) return dual ? mfma_rows_grid<5, true>(f_entries) : mfma_rows_grid<5, false>(f_entries);
  return dual ? mfma_rows_grid<4, true>(f_entries) : mfma_rows_grid<4, false>(f_entries);
}

void launch_mfma_rows(const Globals &g, int order, bool dual, int grid, hipStream_t s) {
  const dim3 gd(grid), bd(kMfmaWaves * 64);
  const size_t lds = order == 5 ? rows_lds_bytes<5>(g.lds_f_entries) : rows_lds_bytes<4>(g.lds_f_entries);
  if (order == 5) {
    if (dual) hipLaunchKernelGGL((mfma_rows_kernel<5, true>), gd, bd, lds, s, g);
    else hipLaunchKernelGGL((mfma_rows_kernel<5, false>), gd, bd, lds, s, g);
  } else {
    if (dual) hipLaunchKernelGGL((mfma_rows_kernel<4, true>), gd, bd, lds, s, g);
    else hipLaunchKernelGGL((mfma_rows_kernel<4, false>), gd, bd, lds, s, g);
  }
}

// ---------------------------------------------------------------------------
// Order 4 on the matrix cores with stored triple tables
// ---------------------------------------------------------------------------
//
// Only the {0,1}^4 cells of each combination (x, y, b, j) are counted here
// (16 per combination instead of the 54 of every prefix row); the other 65
// follow by inclusion-exclusion from the triple tables of (x, y, j),
// (x, b, j), (y, b, j) and (x, y, b), the pair tables and the class counts.
// The A rows are the {0,1}^3 genotype rows of prefixes (x, y, b): row r =
// 8 k + 4 s + i of a fragment is prefix 2 s + k / 2 of the fragment's four,
// with g_x = k mod 2, g_y = i / 2, g_b = i mod 2; the B rows are rows 0, 1 of
// the last variants.  In the output (register e of lane l holds row
// 8 (e / 4) + 4 (l / 32) + e mod 4) lane half s then holds every {0,1}^3 row
// of prefixes 2 s and 2 s + 1 at its column's g_j: registers 0-7 the first,
// 8-15 the second.  Lanes l and l ^ 1 hold the two g_j of the same j; the
// lane of g_j = t scores prefix 2 s + t after taking its partner's 8 counts
// of that prefix.
//
// Tiles: rows b = 2 .. n - 2; a tile is 16 prefixes (x, y) of [0, b),
// consecutive in colex order, by 64 last variants; wave w takes prefixes
// 8 (w / 2) + [0, 8) (4 per fragment) and last variants 32 (w mod 2) + [0, 32).
// The pair (x, y), x < y, of colex index q = C(y, 2) + x (per lane)
__device__ __forceinline__ void colex_pair(u64 q, uint32_t &x, uint32_t &y) {
  u64 t = (u64)((1.0 + __dsqrt_rn(1.0 + 8.0 * (double)q)) * 0.5);
  while (t * (t - 1) / 2 > q) --t;
  while ((t + 1) * t / 2 <= q) ++t;
  y = (uint32_t)t;
  x = (uint32_t)(q - t * (t - 1) / 2);
}

// An order-3 table's inputs, both classes in one register as 4 c0 | 4 c1 << 16
// (byte offsets into a table of floats: counts below 16,384)
struct Tab3P {
  uint32_t D[2][2][2];  // [x][y][z] over {0,1}^3
  uint32_t xy[2][2], xz[2][2], yz[2][2];
  uint32_t Mx[2], My[2], Mz[2];
  uint32_t m;
};

// The order-3 walk (walk_order3_packed's cell order) over NT packed tables at
// once: visit(cells) sees the same cell of every table.  Every result is a
// count, so the packed differences never borrow across the halves.
template <int NT, typename Visit>
__device__ __forceinline__ void walk3_zip_packed(const Tab3P (&q)[NT], Visit &&visit) {
  uint32_t sum[NT], x2z[NT][2][2], t2yz[NT][2][2], cell[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) sum[t] = 0;
  auto emit_cell = [&]() {
#pragma unroll
    for (int t = 0; t < NT; ++t) sum[t] += cell[t];
    visit(cell);
  };
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int z = 0; z < 2; ++z) {
#pragma unroll
        for (int t = 0; t < NT; ++t) cell[t] = q[t].D[x][y][z];
        emit_cell();
      }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
#pragma unroll
      for (int t = 0; t < NT; ++t) cell[t] = q[t].xy[x][y] - q[t].D[x][y][0] - q[t].D[x][y][1];
      emit_cell();  // (x, y, 2)
    }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int z = 0; z < 2; ++z) {
#pragma unroll
      for (int t = 0; t < NT; ++t) cell[t] = x2z[t][x][z] = q[t].xz[x][z] - q[t].D[x][0][z] - q[t].D[x][1][z];
      emit_cell();  // (x, 2, z)
    }
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int z = 0; z < 2; ++z) {
#pragma unroll
      for (int t = 0; t < NT; ++t) cell[t] = t2yz[t][y][z] = q[t].yz[y][z] - q[t].D[0][y][z] - q[t].D[1][y][z];
      emit_cell();  // (2, y, z)
    }
#pragma unroll
  for (int x = 0; x < 2; ++x) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
      cell[t] = q[t].Mx[x] - q[t].xy[x][0] - q[t].xy[x][1] - x2z[t][x][0] - x2z[t][x][1];
    emit_cell();  // (x, 2, 2)
  }
#pragma unroll
  for (int y = 0; y < 2; ++y) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
      cell[t] = q[t].My[y] - q[t].xy[0][y] - q[t].xy[1][y] - t2yz[t][y][0] - t2yz[t][y][1];
    emit_cell();  // (2, y, 2)
  }
#pragma unroll
  for (int z = 0; z < 2; ++z) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
      cell[t] = q[t].Mz[z] - q[t].xz[0][z] - q[t].xz[1][z] - t2yz[t][0][z] - t2yz[t][1][z];
    emit_cell();  // (2, 2, z)
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) cell[t] = q[t].m - sum[t];
  visit(cell);  // (2, 2, 2)
}

// C(t, 3) (0 for t < 3)
__device__ __forceinline__ u64 binom3(u64 t) { return t < 3 ? 0 : t * (t - 1) * (t - 2) / 6; }

// Entry of the 4-set (a, b, c, j), a < b < c < j, in the packed quad tables:
// the triples in colex order (index c3 = C(c, 3) + C(b, 2) + a), each with
// its entries for j = c + 1 .. n - 1.  The triples whose largest variant is
// below c hold sum over c' < c of C(c', 2) (n - 1 - c') = (n - 3) C(c, 3) -
// 3 C(c, 4) entries.
__device__ __forceinline__ u64 quad_entry(uint32_t n, u64 c3, uint32_t c, uint32_t j) {
  const u64 C3 = binom3(c), C4 = c < 4 ? 0 : C3 * (c - 3) / 4;
  return ((u64)n - 3) * C3 - 3 * C4 + (c3 - C3) * (n - 1 - c) + (j - c - 1);
}

// The triple (w, x, y), w < x < y, of colex index q = C(y, 3) + C(x, 2) + w
// (per lane)
__device__ __forceinline__ void colex_triple(u64 q, uint32_t &w, uint32_t &x, uint32_t &y) {
  u64 t = (u64)cbrt(6.0 * (double)q);
  while (t > 0 && binom3(t) > q) --t;
  while (binom3(t + 1) <= q) ++t;
  y = (uint32_t)t;
  colex_pair(q - binom3(t), w, x);
}

// The {0,1}^(K-1) x {0,1} counts of one wave: prefixes of K - 1 variants
// ending in b (K = 4: pairs (x, y) below b, colex indices q0 + [0, 8), four
// per fragment; K = 5: triples (w, x, y) below b, q0 + [0, 4), two per
// fragment; indices from nq on are past the last prefix) x last variants
// j0 + [0, 32).  A row r = 8 k + 4 s + i of fragment f: K = 4: prefix
// q0 + 4 f + 2 s + k / 2 with (g_x, g_y, g_b) = (k mod 2, i / 2, i mod 2);
// K = 5: prefix q0 + 2 f + s with (g_w, g_x, g_y, g_b) = (k / 2, k mod 2,
// i / 2, i mod 2).  So in the output (register e of lane l holds row
// 8 (e / 4) + 4 (l / 32) + e mod 4) lane half s holds at its column's g_j:
// K = 4: every {0,1}^3 row of prefixes 2 s (registers 0-7) and 2 s + 1
// (8-15), register 8 t + 4 g_x + 2 g_y + g_b; K = 5: every {0,1}^4 row of
// prefix s, register 8 g_w + 4 g_x + 2 g_y + g_b.  Both classes per
// register, class 0 in the low 16 bits.  DUAL: one accumulator for both
// classes (class sizes of at most 24 bits together); else class 0 first.
template <int K, bool DUAL, int FA = 2>
__device__ __forceinline__ void sub_contract(const JV &v, uint32_t b, u64 q0, u64 nq, uint32_t j0,
                                             uint32_t lane, uint32_t (&Q)[FA][2][16], int f0 = 0) {
  constexpr int NP = K - 2;           // prefix variants that vary by lane (b does not)
  constexpr int kRaw = FA * NP + 3;   // words a lane loads per word index
  const uint32_t n = v.n;
  const uint32_t r = lane & 31, h = lane >> 5;
  const FI_GLOBAL char *Bvc = reinterpret_cast<const FI_GLOBAL char *>(as_global(v.Bv));
  const size_t word_bytes = (size_t)v.n_pad * 16;  // Bv bytes of one word
  const uint32_t hw = h * (uint32_t)word_bytes;     // words in pairs: lane half h reads word w + h
  const uint32_t k = r >> 3, s = (r >> 2) & 1, i = r & 3;
  uint32_t gv[NP];  // genotype row of each lane-varying prefix variant
  if constexpr (K == 4) {
    gv[0] = k & 1;
    gv[1] = i >> 1;
  } else {
    gv[0] = k >> 1;
    gv[1] = k & 1;
    gv[2] = i >> 1;
  }
  // byte offsets of the lane's rows in a word (fragments f0 .. f0 + FA - 1);
  // prefixes past the last read variant n, a padding variant whose words
  // are zero
  uint32_t oa[FA][NP];
#pragma unroll
  for (int fa = 0; fa < FA; ++fa) {
    const int f = f0 + fa;
    const u64 q = q0 + (K == 4 ? 4 * f + 2 * s + (k >> 1) : 2 * f + s);
    uint32_t pv[NP];
#pragma unroll
    for (int t = 0; t < NP; ++t) pv[t] = n;
    if (q < nq) {
      if constexpr (K == 4) colex_pair(q, pv[0], pv[1]);
      else colex_triple(q, pv[0], pv[1], pv[2]);
    }
#pragma unroll
    for (int t = 0; t < NP; ++t) oa[fa][t] = pv[t] * 16 + gv[t] * 8 + hw;
  }
  const uint32_t ob = b * 16 + (i & 1) * 8 + hw, ol = j0 * 16 + r * 8 + hw;
  // the last step of an odd word count: lanes of half 1 read word w itself,
  // with the row of b replaced by the zero row of padding variant n, so that
  // their A operands vanish
  const uint32_t obt = h ? n * 16 : ob;
  auto load_words = [&](uint32_t w, auto tail, u64 (&xw)[kRaw]) {
    const FI_GLOBAL char *sw = Bvc + (size_t)w * word_bytes;
    constexpr bool kTail = decltype(tail)::value;
    const uint32_t d = kTail ? hw : 0u;
#pragma unroll
    for (int fa = 0; fa < FA; ++fa)
#pragma unroll
      for (int t = 0; t < NP; ++t) xw[fa * NP + t] = ld64(sw, oa[fa][t] - d);
    xw[FA * NP] = ld64(sw, kTail ? obt : ob);
    xw[FA * NP + 1] = ld64(sw, ol - d);
    xw[FA * NP + 2] = ld64(sw, ol + 256 - d);
  };
  // A row = AND of the rows of the prefix variants (the row of b last)
  const auto ops = [](const u64 (&xw)[kRaw], int half, v8i (&E)[FA + 2]) {
    const int sh = 32 * half;
#pragma unroll
    for (int fa = 0; fa < FA; ++fa) {
      uint32_t a = (uint32_t)(xw[fa * NP] >> sh);
#pragma unroll
      for (int t = 1; t < NP; ++t) a &= (uint32_t)(xw[fa * NP + t] >> sh);
      E[fa] = expand32_fp4_and(a, (uint32_t)(xw[FA * NP] >> sh));
    }
    E[FA] = expand32_fp4_b((uint32_t)(xw[FA * NP + 1] >> sh));
    E[FA + 1] = expand32_fp4_b((uint32_t)(xw[FA * NP + 2] >> sh));
  };
  if constexpr (DUAL)
    contract_fp4_dual<2, kRaw, FA>(load_words, ops, v.W0, v.W1, bit_len(v.m0), Q);
  else
    contract_fp4_narrow<2, kRaw, FA>(load_words, ops, v.W0, v.W1, Q);
}

// One wave of order 4: prefixes (x, y, b), (x, y) of colex indices q0 + [0, 8),
// x last variants j0 + [0, 32).  The lane of g_j = t in lane half s scores
// prefix 2 s + t of each fragment after taking its partner's 8 counts of it.
template <bool DUAL>
__device__ __forceinline__ void wave_t4(const Globals &g, const JV &v, uint32_t b, u64 q0, uint32_t j0,
                                        uint32_t lane, const FI_LDS float *Fl) {
  const uint32_t n = v.n, np = v.n_pad;
  const uint32_t r = lane & 31, h = lane >> 5, gl = lane & 1;
  const u64 nq = (u64)b * (b - 1) / 2;  // prefixes (x, y) below b
  uint32_t Q[2][2][16];
  sub_contract<4, DUAL>(v, b, q0, nq, j0, lane, Q);

  // scoring from the packed tables (every count times 4, class 0 in the low
  // half: byte offsets into the LDS f table)
  const MiConst mc = mi_const(v);
  float thr = current_threshold(v);
  const FI_GLOBAL v4u *TT4 = reinterpret_cast<const FI_GLOBAL v4u *>(as_global(v.triples4));
  const FI_GLOBAL v4u *PT4 = reinterpret_cast<const FI_GLOBAL v4u *>(as_global(v.pairs4));
  const FI_GLOBAL uint32_t *marg = as_global(v.marg);
  const FI_LDS char *Fb = (const FI_LDS char *)Fl;
  // one cell's term of the fixed-point sum (the LDS table holds Fq)
  auto term = [&](uint32_t p) {
    const uint32_t o0 = p & 0xFFFFu, o1 = p >> 16;
    const uint32_t f0 = *(const FI_LDS uint32_t *)(Fb + o0);
    const uint32_t f1 = *(const FI_LDS uint32_t *)(Fb + o1);
    const uint32_t f01 = *(const FI_LDS uint32_t *)(Fb + o0 + o1);
    return f0 + f1 - f01;
  };
  auto marg4 = [&](uint32_t var, int g4) { return pack_x4(marg[(size_t)var * 6 + 2 * g4], marg[(size_t)var * 6 + 2 * g4 + 1]); };
  // the lane's two last variants j (fb = 0, 1) and their class counts
  uint32_t jv[2], jj[2], Mj4[2][2];
#pragma unroll
  for (int fb = 0; fb < 2; ++fb) {
    jv[fb] = j0 + 16 * fb + (r >> 1);
    jj[fb] = jv[fb] < n ? jv[fb] : n - 1;
#pragma unroll
    for (int gj = 0; gj < 2; ++gj) Mj4[fb][gj] = marg4(jj[fb], gj);
  }
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    // the prefix this lane scores in fragment f and its own order-3 table
    const u64 q = q0 + 4 * f + 2 * h + gl;
    const bool valid = q < nq;
    uint32_t x = 0, y = 1;
    if (valid) colex_pair(q, x, y);
    const u64 pxy = pair_index(n, x, y);
    Tab3P t3[3];  // [0]: (x, y, b); [1], [2]: the cells with g_j = 0, 1
    {
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const v4u e = TT4[(pxy * np + b) * 2 + a];
#pragma unroll
        for (int c = 0; c < 4; ++c) t3[0].D[a][c >> 1][c & 1] = e[c];
      }
      const v4u exy = PT4[(size_t)x * np + y], exb = PT4[(size_t)x * np + b], eyb = PT4[(size_t)y * np + b];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        t3[0].xy[c >> 1][c & 1] = exy[c];
        t3[0].xz[c >> 1][c & 1] = exb[c];
        t3[0].yz[c >> 1][c & 1] = eyb[c];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        t3[0].Mx[a] = marg4(x, a);
        t3[0].My[a] = marg4(y, a);
        t3[0].Mz[a] = marg4(b, a);
      }
      t3[0].m = pack_x4(v.m0, v.m1);
    }
    const u64 pxb = pair_index(n, x, b), pyb = pair_index(n, y, b);
#pragma unroll
    for (int fb = 0; fb < 2; ++fb) {
      // the {0,1}^3 counts of the prefix at both g_j: own registers 8 gl +
      // [0, 8) at g_j = gl, the partner's at 1 - gl
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const uint32_t lo = Q[f][fb][a], hi = Q[f][fb][8 + a];
        const uint32_t own = gl ? hi : lo;
        const uint32_t recv = xor1(gl ? lo : hi);
        t3[1].D[a >> 2][(a >> 1) & 1][a & 1] = packed_x4<DUAL>(gl ? recv : own);
        t3[2].D[a >> 2][(a >> 1) & 1][a & 1] = packed_x4<DUAL>(gl ? own : recv);
      }
      {
        const uint32_t J = jj[fb];
        v4u txy[2], txb[2], tyb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          txy[a] = TT4[(pxy * np + J) * 2 + a];
          txb[a] = TT4[(pxb * np + J) * 2 + a];
          tyb[a] = TT4[(pyb * np + J) * 2 + a];
        }
        const v4u pxj = PT4[(size_t)x * np + J], pyj = PT4[(size_t)y * np + J], pbj = PT4[(size_t)b * np + J];
#pragma unroll
        for (int gj = 0; gj < 2; ++gj) {
          Tab3P &t = t3[1 + gj];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              t.xy[a][c] = txy[a][c * 2 + gj];
              t.xz[a][c] = txb[a][c * 2 + gj];
              t.yz[a][c] = tyb[a][c * 2 + gj];
            }
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            t.Mx[a] = pxj[a * 2 + gj];
            t.My[a] = pyj[a * 2 + gj];
            t.Mz[a] = pbj[a * 2 + gj];
          }
          t.m = Mj4[fb][gj];
        }
      }
      const uint32_t j = jv[fb];
      const bool active = valid && j < n;
      // the f(n0) + f(n1) terms to fs, the f(n0 + n1) terms to fm, three at
      // a time: the score is fs - fm
      uint32_t fs = mc.q0, fm = 0;
      if (active)
        walk3_zip_packed<3>(t3, [&](const uint32_t (&cell)[3]) {
          const uint32_t p[3] = {cell[1], cell[2], cell[0] - cell[1] - cell[2]};
          uint32_t f01[3];
#pragma unroll
          for (int x = 0; x < 3; ++x) {
            const uint32_t o0 = p[x] & 0xFFFFu, o1 = p[x] >> 16;
            fs += *(const FI_LDS uint32_t *)(Fb + o0) + *(const FI_LDS uint32_t *)(Fb + o1);
            f01[x] = *(const FI_LDS uint32_t *)(Fb + o0 + o1);
          }
          fm += f01[0] + f01[1] + f01[2];
          pin_sum(fs);
          pin_sum(fm);
        });
      const uint32_t pre[3] = {x, y, b};
      if (emit_with(v, active, mi_fixed(fs - fm, mc),
                    [&] { return lex_rank_prefix(g, n, 4, pre) + (u64)(j - b - 1); }, thr,
                    lane) >= kRefreshAppends)
        thr = current_threshold_lanes(v);
    }
  }
}

// One wave of order 5: prefixes (w, x, y, b), (w, x, y) of colex indices
// q0 + [0, 4), x last variants j0 + [0, 32).  Fixing g_w and g_j leaves an
// order-3 table over (x, y, b) whose inputs (walk_order3_packed) are {0,1}^5
// counts and the quad, triple and pair tables restricted to them; the walk
// is linear in its inputs, so the table at a 2 of g_w or g_j is the walk of
// (inputs with that variant marginalised) - (inputs at 0) - (inputs at 1).
// Each lane scores one combination, all 9 tables (243 cells): both output
// blocks of a fragment are taken at once, the lane of g_j = t taking block t
// with its partner's counts of the other g_j.
template <bool DUAL>
__device__ __forceinline__ void wave_t5(const Globals &g, const JV &v, uint32_t b, u64 q0, uint32_t j0,
                                        uint32_t lane, const FI_LDS float *Fl) {
  const uint32_t n = v.n, np = v.n_pad;
  const uint32_t r = lane & 31, h = lane >> 5, gl = lane & 1;
  const u64 nq = binom3(b);  // prefixes (w, x, y) below b

  const MiConst mc = mi_const(v);
  float thr = current_threshold(v);
  const FI_GLOBAL v4u *QT4 = reinterpret_cast<const FI_GLOBAL v4u *>(as_global(v.quads4));
  const FI_GLOBAL v4u *TT4 = reinterpret_cast<const FI_GLOBAL v4u *>(as_global(v.triples4));
  const FI_GLOBAL v4u *PT4 = reinterpret_cast<const FI_GLOBAL v4u *>(as_global(v.pairs4));
  const FI_GLOBAL uint32_t *marg = as_global(v.marg);
  const FI_LDS char *Fb = (const FI_LDS char *)Fl;
  // one cell's term of the fixed-point sum (the LDS table holds Fq)
  auto term = [&](uint32_t p) {
    const uint32_t o0 = p & 0xFFFFu, o1 = p >> 16;
    const uint32_t f0 = *(const FI_LDS uint32_t *)(Fb + o0);
    const uint32_t f1 = *(const FI_LDS uint32_t *)(Fb + o1);
    const uint32_t f01 = *(const FI_LDS uint32_t *)(Fb + o0 + o1);
    return f0 + f1 - f01;
  };
  auto marg4 = [&](uint32_t var, uint32_t g4) {
    return pack_x4(marg[(size_t)var * 6 + 2 * g4], marg[(size_t)var * 6 + 2 * g4 + 1]);
  };
  // entries of the packed tables: quad (a, b, c, j) (colex index c3 of
  // (a, b, c)): 4 v4u [g_a][g_b] of [g_c][g_j] at quad_entry; triple (a, b, j): 2 v4u [g_a]
  // of [g_b][g_j]; pair (a, j): v4u [g_a][g_j]
  // (each load through a base the compiler cannot see through: a table entry
  // is read again where it is used rather than kept in registers between
  // its uses)
  auto fresh = [](auto p) {
    asm volatile("" : "+s"(p));
    return p;
  };
  auto quad = [&](u64 c3, uint32_t c, uint32_t j, uint32_t i) { return fresh(QT4)[quad_entry(n, c3, c, j) * 4 + i]; };
  auto triple = [&](uint32_t a, uint32_t bb, uint32_t j, uint32_t i) {
    return fresh(TT4)[(pair_index(n, a, bb) * np + j) * 2 + i];
  };
  auto pair = [&](uint32_t a, uint32_t j) { return fresh(PT4)[(size_t)a * np + j]; };
  // every input register of a table, of two tables side by side
  auto each2 = [](Tab3P &t, const Tab3P &u, auto &&fn) {
#pragma unroll
    for (int a = 0; a < 8; ++a) fn(t.D[a >> 2][(a >> 1) & 1][a & 1], u.D[a >> 2][(a >> 1) & 1][a & 1]);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      fn(t.xy[a >> 1][a & 1], u.xy[a >> 1][a & 1]);
      fn(t.xz[a >> 1][a & 1], u.xz[a >> 1][a & 1]);
      fn(t.yz[a >> 1][a & 1], u.yz[a >> 1][a & 1]);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      fn(t.Mx[a], u.Mx[a]);
      fn(t.My[a], u.My[a]);
      fn(t.Mz[a], u.Mz[a]);
    }
    fn(t.m, u.m);
  };
  auto walk = [&](const Tab3P &t, auto &&visit) {
    walk_order3_packed(t.D, t.xy, t.xz, t.yz, t.Mx, t.My, t.Mz, t.m, visit);
  };
  const uint32_t hb = binom3(b);  // colex index of (a, c, b) = C(b, 3) + colex index of (a, c)
  // one A fragment at a time: its counts, then both its output blocks at
  // once, one combination per lane: the lane of g_j = t in lane half s takes
  // prefix s and the last variant of block fb = t, with its partner's counts
  // of that block at the other g_j
#pragma unroll 1
  for (int f = 0; f < 2; ++f) {
    uint32_t cells[2][2][8];  // [g_w][g_j][4 g_x + 2 g_y + g_b], packed x 4
    {
      uint32_t Q[1][2][16];
      sub_contract<5, DUAL, 1>(v, b, q0, nq, j0, lane, Q, f);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const uint32_t own = gl ? Q[0][1][e] : Q[0][0][e];
        const uint32_t recv = xor1(gl ? Q[0][0][e] : Q[0][1][e]);
        cells[e >> 3][0][e & 7] = packed_x4<DUAL>(gl ? recv : own);
        cells[e >> 3][1][e & 7] = packed_x4<DUAL>(gl ? own : recv);
      }
    }
    // (a lane past the last prefix scores nothing; it reads the tables of
    // (0, 1, 2, b), colex index 0, so that every read stays in the tables)
    const u64 qp = q0 + 2 * f + h;
    const bool valid = qp < nq;
    const u64 q = valid ? qp : 0;
    uint32_t w = 0, x = 1, y = 2;
    if (valid) colex_triple(q, w, x, y);
    const u64 cwxb = hb + (u64)x * (x - 1) / 2 + w, cwyb = hb + (u64)y * (y - 1) / 2 + w,
              cxyb = hb + (u64)y * (y - 1) / 2 + x;
    const uint32_t j = j0 + 16 * gl + (r >> 1);
    const uint32_t J = j < n ? j : n - 1;
    const bool active = valid && j < n;
    uint32_t fs = mc.q0;
    auto score = [&](const Tab3P &t) {
      if (active)
        walk(t, [&](uint32_t p) {
          fs += term(p);
          pin_sum(fs);
        });
    };
    // X(gw, sj): the inputs of the order-3 table over (x, y, b) with w at
    // genotype gw and j at sj, 2 meaning the variant marginalised (left out);
    // sj = 3: the sum of sj = 0 and 1.  t = X (sign +1) or t -= X (-1).
    auto X = [&](int gw, int sj, Tab3P &t, int sign) {
      auto put = [&](uint32_t &u, uint32_t val) { u = sign > 0 ? val : u - val; };
      auto pick = [&](const v4u &e, int c) { return sj < 2 ? e[c * 2 + sj] : e[c * 2] + e[c * 2 + 1]; };
      if (gw < 2 && sj != 2) {
#pragma unroll
        for (int a = 0; a < 8; ++a)
          put(t.D[a >> 2][(a >> 1) & 1][a & 1], sj < 2 ? cells[gw][sj][a] : cells[gw][0][a] + cells[gw][1][a]);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const v4u exy = quad(q, y, J, gw * 2 + a), exb = quad(cwxb, b, J, gw * 2 + a),
                    eyb = quad(cwyb, b, J, gw * 2 + a);
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            put(t.xy[a][c], pick(exy, c));
            put(t.xz[a][c], pick(exb, c));
            put(t.yz[a][c], pick(eyb, c));
          }
        }
        const v4u mx = triple(w, x, J, gw), my = triple(w, y, J, gw), mb = triple(w, b, J, gw);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          put(t.Mx[a], pick(mx, a));
          put(t.My[a], pick(my, a));
          put(t.Mz[a], pick(mb, a));
        }
        const v4u pj = pair(w, J);
        put(t.m, sj < 2 ? pj[gw * 2 + sj] : pj[gw * 2] + pj[gw * 2 + 1]);
      } else if (gw < 2) {  // j marginalised: the prefix's tables at g_w
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const v4u e = quad(q, y, b, gw * 2 + a);
#pragma unroll
          for (int c = 0; c < 4; ++c) put(t.D[a][c >> 1][c & 1], e[c]);
        }
        const v4u exy = triple(w, x, y, gw), exb = triple(w, x, b, gw), eyb = triple(w, y, b, gw);
        const v4u px = pair(w, x), py = pair(w, y), pb = pair(w, b);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          put(t.xy[c >> 1][c & 1], exy[c]);
          put(t.xz[c >> 1][c & 1], exb[c]);
          put(t.yz[c >> 1][c & 1], eyb[c]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          put(t.Mx[a], px[gw * 2 + a]);
          put(t.My[a], py[gw * 2 + a]);
          put(t.Mz[a], pb[gw * 2 + a]);
        }
        put(t.m, marg4(w, gw));
      } else if (sj != 2) {  // w marginalised: the tables of (x, y, b, j)
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const v4u e = quad(cxyb, b, J, a);
#pragma unroll
          for (int c = 0; c < 2; ++c) put(t.D[a >> 1][a & 1][c], pick(e, c));
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const v4u exy = triple(x, y, J, a), exb = triple(x, b, J, a), eyb = triple(y, b, J, a);
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            put(t.xy[a][c], pick(exy, c));
            put(t.xz[a][c], pick(exb, c));
            put(t.yz[a][c], pick(eyb, c));
          }
        }
        const v4u px = pair(x, J), py = pair(y, J), pb = pair(b, J);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          put(t.Mx[a], pick(px, a));
          put(t.My[a], pick(py, a));
          put(t.Mz[a], pick(pb, a));
        }
        put(t.m, sj < 2 ? marg4(J, sj) : marg4(J, 0) + marg4(J, 1));
      } else {  // both marginalised: the table of (x, y, b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const v4u e = triple(x, y, b, a);
#pragma unroll
          for (int c = 0; c < 4; ++c) put(t.D[a][c >> 1][c & 1], e[c]);
        }
        const v4u exy = pair(x, y), exb = pair(x, b), eyb = pair(y, b);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          put(t.xy[c >> 1][c & 1], exy[c]);
          put(t.xz[c >> 1][c & 1], exb[c]);
          put(t.yz[c >> 1][c & 1], eyb[c]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          put(t.Mx[a], marg4(x, a));
          put(t.My[a], marg4(y, a));
          put(t.Mz[a], marg4(b, a));
        }
        put(t.m, pack_x4(v.m0, v.m1));
      }
    };
    // the table at (G, S), G, S in {0, 1, 2}: X(G, S) for G, S < 2; a 2
    // takes that variant's marginal less its two other genotypes (one sum of
    // inputs kept in registers, the others read again: measured fastest)
    Tab3P R0;  // X(0, 0) + X(1, 0)
#pragma unroll
    for (int gw = 0; gw < 2; ++gw) {
      Tab3P t;
      X(gw, 0, t, +1);
      score(t);
      if (gw == 0) R0 = t;
      else each2(R0, t, [](uint32_t &u, uint32_t tv) { u += tv; });
      X(gw, 1, t, +1);
      score(t);
      X(gw, 2, t, +1);  // (gw, 2)
      X(gw, 3, t, -1);
      score(t);
    }
    {
      Tab3P t;
      X(2, 0, t, +1);  // (2, 0)
      each2(t, R0, [](uint32_t &u, uint32_t rv) { u -= rv; });
      score(t);
      R0 = t;  // from here on the (2, 0) and (2, 1) inputs, summed
      X(2, 1, t, +1);  // (2, 1)
      X(0, 1, t, -1);
      X(1, 1, t, -1);
      score(t);
      each2(R0, t, [](uint32_t &u, uint32_t tv) { u += tv; });
      X(2, 2, t, +1);  // (2, 2) = X(2, 2) - X(0, 2) - X(1, 2) - (2, 0) - (2, 1)
      X(0, 2, t, -1);
      X(1, 2, t, -1);
      each2(t, R0, [](uint32_t &u, uint32_t rv) { u -= rv; });
      score(t);
    }
    const uint32_t pre[4] = {w, x, y, b};
    if (emit_with(v, active, mi_fixed(fs, mc),
                  [&] { return lex_rank_prefix(g, n, 5, pre) + (u64)(j - b - 1); }, thr,
                  lane) >= kRefreshAppends)
      thr = current_threshold_lanes(v);
  }
}

// The f table entries the order-4/5 table kernels keep in LDS: 8,192 (dual)
// or 16,384 (two accumulators; the packed tables hold counts below 16,384);
// the host gives them only jobs whose table fits
template <bool DUAL>
constexpr uint32_t t4_f_entries() { return DUAL ? mfma_f_entries(kMfmaF4Dual) : 16384u; }

// Orders 4 (K = 4, path kPathMfma4t) and 5 (K = 5, kPathMfma5q) with stored
// lower-order tables.  Tiles: rows b = K - 2 .. n - 2 (the last prefix
// variant); a tile is 16 (K = 4) or 8 (K = 5) prefixes of [0, b), consecutive
// in colex order, by 64 last variants; wave w takes half the prefixes
// (w / 2) and last variants 32 (w mod 2) + [0, 32).
template <int K>
constexpr uint32_t sub_tile_prefixes() { return K == 4 ? 16u : 8u; }

// (2 waves per SIMD; at order 5 a few registers spill, measured faster than
// one wave per SIMD without spills)
template <int K, bool DUAL>
__global__ __launch_bounds__(kMfmaWaves * 64, 2) void mfma_sub_kernel(Globals g) {
  FI_LDS float *s_f = lds_window();
  FI_LDS u64 &s_tile = tile_slot<t4_f_entries<DUAL>()>(s_f);
  const uint32_t lane = lane_id();
  const uint32_t wave = uni(threadIdx.x >> 6);
  const FI_LDS float *Fl = s_f;
  uint32_t f_job = ~0u;
  RowHint hint;  // the row of the workgroup's last tile
  if (!any_job(g, [](uint32_t m0, uint32_t m1, uint32_t m) {
        return (bit_len(m0) + bit_len(m1) <= 24 && m + 1 <= t4_f_entries<true>()) == DUAL;
      }))
    return;
  for (;;) {
    if (threadIdx.x == 0) s_tile = g.tile_base + atomicAdd(g.tile_counter, 1ull);
    __syncthreads();
    const u64 t = uni64(s_tile);
    __syncthreads();
    if (t >= g.total_tiles) break;
    JV v;
    const FI_CONST JobDesc *jd;
    u64 lt;
    if (!locate_tile(g, t, wave, kMfmaPilotEmits, v, jd, lt)) continue;
    // the host gives this kernel only such jobs
    if (v.path != (K == 4 ? kPathMfma4t : kPathMfma5q) || v.m + 1 > t4_f_entries<false>()) continue;
    {
      // the dual and the two-accumulator kernels run over the same tiles,
      // each skipping the other's jobs
      const bool dual = bit_len(v.m0) + bit_len(v.m1) <= 24 && v.m + 1 <= t4_f_entries<true>();
      if (dual != DUAL) {
        if (threadIdx.x == 0) {
          const u64 end = as_const(g.job_tile_start)[job_of_tile(g, t) + 1];
          atomicMax(g.tile_counter, end - g.tile_base);
        }
        continue;
      }
    }
    {
      // the job's table, once the tile is known to be this kernel's (every
      // wave has finished the previous tile: the barriers above)
      const uint32_t jx = (uint32_t)(jd - as_const(g.jobs));
      if (jx != f_job) {
        const FI_GLOBAL uint32_t *Fq = as_global(uni_ptr(jd->Fq));
        FI_LDS uint32_t *q = (FI_LDS uint32_t *)s_f;
        for (uint32_t i = threadIdx.x; i <= v.m; i += blockDim.x) q[i] = Fq[i];
        f_job = jx;
        __syncthreads();
      }
    }
    cu64p rows = as_const(uni_ptr(jd->row_start));
    const uint32_t rl = hint.find(jd, lt);
    const u64 local = uni64(lt - rows[rl]);
    const uint32_t b = rl + (K - 2);
    const uint32_t nj = (v.n - 1 - b + 63) / 64;
    const u64 grp = local / nj;
    const uint32_t jb = (uint32_t)(local - grp * nj);
    const u64 q0 = grp * sub_tile_prefixes<K>() + (sub_tile_prefixes<K>() / 2) * (wave >> 1);
    const uint32_t j0 = b + 1 + 64 * jb + 32 * (wave & 1);
    const u64 nq = K == 4 ? (u64)b * (b - 1) / 2 : binom3(b);
    // a wave without a prefix or a last variant has nothing to count; its
    // pilot slots stay zero
    if (q0 >= nq || j0 >= v.n) continue;
    if constexpr (K == 4) wave_t4<DUAL>(g, v, b, q0, j0, lane, Fl);
    else wave_t5<DUAL>(g, v, b, q0, j0, lane, Fl);
  }
}

// The quad tables of the order-5 jobs: for every 4-set a < b < c < j its
// {0,1}^4 counts, packed, at entry quad_entry (4 v4u: [g_a][g_b] of
// [g_c][g_j]).  Grid: x = group of 16 pairs (a, b) below c in
// colex order, y = c - 2, z = job; the workgroup walks the blocks of 64 last
// variants (the order-4 kernel's tiles, counts stored instead of scored).
// (2 waves per SIMD: both contraction forms in one kernel would otherwise
// take more than 256 registers and run one wave per SIMD)
__global__ __launch_bounds__(kMfmaWaves * 64, 2) void quads_kernel(Globals g) {
  const JobDesc *jd = g.jobs + blockIdx.z;
  JV v = load_view(jd);
  v4u *QT = reinterpret_cast<v4u *>(uni_ptr(as_const(jd)->quads4));
  if (QT == nullptr) return;
  const JobState *st = v.st;
  if (uni((uint32_t)st->status) != 0) return;
  v.W0 = uni(st->W0);
  v.W1 = uni(st->W1);
  v.m0 = uni(st->m0);
  v.m1 = uni(st->m1);
  const uint32_t n = v.n;
  const uint32_t c = blockIdx.y + 2;
  if (c + 1 >= n) return;
  const u64 nq = (u64)c * (c - 1) / 2;
  const uint32_t wave = uni(threadIdx.x >> 6), lane = lane_id();
  const uint32_t r = lane & 31, h = lane >> 5, gl = lane & 1;
  const u64 q0 = (u64)blockIdx.x * 16 + 8 * (wave >> 1);
  if (q0 >= nq) return;
  const bool dual = bit_len(v.m0) + bit_len(v.m1) <= 24;
  const u64 hc = binom3(c);
  for (uint32_t j0 = c + 1 + 32 * (wave & 1); j0 < n; j0 += 64) {
    uint32_t Q[2][2][16];
    if (dual) sub_contract<4, true>(v, c, q0, nq, j0, lane, Q);
    else sub_contract<4, false>(v, c, q0, nq, j0, lane, Q);
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      // the lane of g_j = t in lane half s stores prefix 2 s + t
      const u64 q = q0 + 4 * f + 2 * h + gl;
#pragma unroll
      for (int fb = 0; fb < 2; ++fb) {
        const uint32_t j = j0 + 16 * fb + (r >> 1);
        uint32_t cell[8][2];  // [4 g_a + 2 g_b + g_c][g_j], packed x 4
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const uint32_t lo = Q[f][fb][a], hi = Q[f][fb][8 + a];
          const uint32_t own = gl ? hi : lo;
          const uint32_t recv = xor1(gl ? lo : hi);
          cell[a][0] = dual ? packed_x4<true>(gl ? recv : own) : packed_x4<false>(gl ? recv : own);
          cell[a][1] = dual ? packed_x4<true>(gl ? own : recv) : packed_x4<false>(gl ? own : recv);
        }
        if (q < nq && j < n) {
          v4u *dst = QT + quad_entry(n, hc + q, c, j) * 4;
#pragma unroll
          for (int ab = 0; ab < 4; ++ab) {
            v4u o;
            o[0] = cell[2 * ab][0];
            o[1] = cell[2 * ab][1];
            o[2] = cell[2 * ab + 1][0];
            o[3] = cell[2 * ab + 1][1];
            dst[ab] = o;
          }
        }
      }
    }
  }
}

void launch_quads(const Globals &g, uint32_t max_n, hipStream_t s) {
  if (max_n < 5) return;
  const u64 groups = ((u64)(max_n - 2) * (max_n - 3) / 2 + 15) / 16;
  hipLaunchKernelGGL(quads_kernel, dim3((uint32_t)groups, max_n - 3, g.n_jobs), dim3(kMfmaWaves * 64), 0, s,
                     g);
}

template <int K, bool DUAL>
int mfma_sub_grid() {
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, mfma_sub_kernel<K, DUAL>, kMfmaWaves * 64,
                                                     f_lds_bytes(t4_f_entries<DUAL>()));
  if (cus <= 0) cus = 256;
  if (per <= 0) per = 1;
  return cus * per;
}

int mfma_sub_grid_size(int order, bool dual) {
  if (order == 5) return dual ? mfma_sub_grid<5, true>() : mfma_sub_grid<5, false>();
  return dual ? mfma_sub_grid<4, true>() : mfma_sub_grid<4, false>();
}
uint32_t mfma_sub_dual_max_samples() { return t4_f_entries<true>() - 1; }

void launch_mfma_sub(const Globals &g, int order, bool dual, int grid, hipStream_t s) {
  const dim3 gd(grid), bd(kMfmaWaves * 64);
  const size_t lds = f_lds_bytes(dual ? t4_f_entries<true>() : t4_f_entries<false>());
  if (order == 5) {
    if (dual) hipLaunchKernelGGL((mfma_sub_kernel<5, true>), gd, bd, lds, s, g);
    else hipLaunchKernelGGL((mfma_sub_kernel<5, false>), gd, bd, lds, s, g);
  } else {
    if (dual) hipLaunchKernelGGL((mfma_sub_kernel<4, true>), gd, bd, lds, s, g);
    else hipLaunchKernelGGL((mfma_sub_kernel<4, false>), gd, bd, lds, s, g);
  }
}

// ORDER 2 or 3, FMT: operand format (kMfmaI8, kMfmaF4, kMfmaF4Narrow); the
// kernel serves the jobs of that order and format (a batch with several
// launches it once per group, each over the group's tiles).  Waves per SIMD:
// 2, the dual kernels 3 (the order-3 dual kernel at 4 spills 10 registers:
// 0.6 % faster, but its scratch traffic doubles the bytes it moves)
template <int ORDER, int FMT>
__global__ __launch_bounds__(kMfmaWaves * 64, FMT == kMfmaF4Dual ? 3 : 2) void mfma_kernel(Globals g) {
  constexpr bool F4 = FMT != kMfmaI8;
  __shared__ u64 s_lut[F4 ? 1 : 256 * kLutCopies];
  // the f table of the current job, when it has at most mfma_f_entries(FMT)
  // entries (dynamic LDS of that size), then the tile slot
  extern __shared__ float s_dyn[];
  FI_LDS float *s_f = F4 ? lds_window() : (FI_LDS float *)s_dyn;
  FI_LDS u64 &s_tile = tile_slot<mfma_f_entries(FMT)>(s_f);
  const uint32_t lane = lane_id();
  const uint32_t wave = uni(threadIdx.x >> 6);
  if (!F4)
    for (uint32_t i = threadIdx.x; i < 256 * kLutCopies; i += blockDim.x) s_lut[i] = spread8(i / kLutCopies);
  const u64 *lut = s_lut + (F4 ? 0 : lane % kLutCopies);
  const FI_LDS float *Fl = s_f;
  uint32_t f_job = ~0u;  // job whose table s_f holds (same in every thread)
  bool f_lds = false;
  RowHint hint;  // the row of the workgroup's last tile
  // order 3: the block of last variants of the workgroup's last tile, and its job
  const FI_CONST JobDesc *jb_job = nullptr;
  uint32_t jb_hint = 0;
  if (FMT == kMfmaF4Narrow || FMT == kMfmaF4Dual) {
    if (!any_job(g, [](uint32_t m0, uint32_t m1, uint32_t m) {
          return (bit_len(m0) + bit_len(m1) <= 24 && m + 1 <= mfma_f_entries(kMfmaF4Dual)) ==
                 (FMT == kMfmaF4Dual);
        }))
      return;
  }
  for (;;) {
    if (threadIdx.x == 0) s_tile = g.tile_base + atomicAdd(g.tile_counter, 1ull);
    __syncthreads();
    const u64 t = uni64(s_tile);
    __syncthreads();
    if (t >= g.total_tiles) break;
    JV v;
    const FI_CONST JobDesc *jd;
    u64 lt;
    if (!locate_tile(g, t, wave, kMfmaPilotEmits, v, jd, lt)) continue;
    if (v.fp4 != (F4 ? 1u : 0u)) continue;
    const bool fits = v.m + 1 <= mfma_f_entries(FMT);
    // the narrow kernel needs the table in LDS (and so counts below 2^16);
    // the host gives it no other job
    if (FMT == kMfmaF4Narrow && !fits) continue;
    if (FMT == kMfmaF4Narrow || FMT == kMfmaF4Dual) {
      // the narrow and dual kernels run over the same tiles: each skips the
      // other's jobs, jumping its tile counter past the job's last tile (the
      // counter only grows, so no tile of a later job is lost)
      const bool dual = bit_len(v.m0) + bit_len(v.m1) <= 24 && v.m + 1 <= mfma_f_entries(kMfmaF4Dual);
      if (dual != (FMT == kMfmaF4Dual)) {
        if (threadIdx.x == 0) {
          const u64 end = as_const(g.job_tile_start)[job_of_tile(g, t) + 1];
          atomicMax(g.tile_counter, end - g.tile_base);
        }
        continue;
      }
    }
    {
      // the job's table, once the tile is known to be this kernel's: every
      // wave of the workgroup has finished the previous tile (the barriers
      // above), so the table can be replaced
      const uint32_t jx = (uint32_t)(jd - as_const(g.jobs));
      if (jx != f_job) {
        f_lds = fits;
        if (f_lds) {
          if constexpr (lds_fixed<ORDER, FMT>()) {
            const FI_GLOBAL uint32_t *Fq = as_global(uni_ptr(jd->Fq));
            FI_LDS uint32_t *q = (FI_LDS uint32_t *)s_f;
            for (uint32_t i = threadIdx.x; i <= v.m; i += blockDim.x) q[i] = Fq[i];
          } else {
            const FI_GLOBAL float *Fh = as_global(uni_ptr(jd->Fh));
            for (uint32_t i = threadIdx.x; i <= v.m; i += blockDim.x) s_f[i] = Fh[i];
          }
        }
        f_job = jx;
        __syncthreads();
      }
    }
    cu64p rows = as_const(uni_ptr(jd->row_start));
    const uint32_t rl = hint.find(jd, lt);
    const u64 local = uni64(lt - rows[rl]);
    if (ORDER == 3) {
      if (v.path != kPathMfma3) continue;
      // rows (jb, b), jb-major: jb's rows are b = 1 .. n - 2 - 64 jb, so the
      // rows before jb number C(jb) = jb (n - 2) - 32 jb (jb - 1) = (n + 30)
      // jb - 32 jb^2; the row's tiles are its groups of 32 first variants
      // jb is searched from the workgroup's last one (its tiles mostly come
      // in increasing order)
      const uint32_t n = v.n;
      auto rows_before = [&](uint32_t x) { return (u64)x * (n + 30) - 32 * (u64)x * x; };
      if (jd != jb_job) {
        jb_job = jd;
        jb_hint = 0;
      }
      uint32_t jb = jb_hint;
      while (jb > 0 && rows_before(jb) > rl) --jb;
      while (64 * (jb + 1) + 3 <= n && rows_before(jb + 1) <= rl) ++jb;
      jb = uni(jb);
      jb_hint = jb;
      const uint32_t b = uni(rl - (uint32_t)rows_before(jb) + 1);
      // (never taken: the decode above keeps b in [1, n - 2 - 64 jb])
      if (b + 2 + 64 * jb > n) continue;
      const u64 grp = local;
      const uint32_t a_first = (uint32_t)grp * 32 + 16 * (wave >> 1);
      const uint32_t j0 = b + 1 + 64 * jb + 32 * (wave & 1);
      // a wave without a prefix a < b or a last variant j < n has nothing to
      // count; its pilot slots stay zero
      if (a_first >= b || j0 >= v.n) continue;
      if (FMT >= kMfmaF4Narrow || f_lds) wave_prefix3<FMT, true>(g, v, b, a_first, j0, lane, lut, Fl);
      else wave_prefix3<FMT, false>(g, v, b, a_first, j0, lane, lut, Fl);
      continue;
    }
    // order 2: tile (A, B) of the upper triangle of 64-variant blocks, row A first
    if (v.path != kPathMfma2) continue;
    const uint32_t B = rl + (uint32_t)local;
    const uint32_t a0 = 64 * rl + 32 * (wave >> 1);
    const uint32_t j0 = 64 * B + 32 * (wave & 1);
    // a wave with no pair a < j < n has nothing to count; its pilot slots
    // stay zero
    if (a0 + 1 >= v.n || j0 >= v.n || j0 + 31 <= a0) continue;
    if (FMT >= kMfmaF4Narrow || f_lds) wave_pairs<FMT, true>(v, a0, j0, lane, lut, Fl);
    else wave_pairs<FMT, false>(v, a0, j0, lane, lut, Fl);
  }
}

template <int ORDER, int FMT>
int mfma_grid() {
  int dev = 0, cus = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, mfma_kernel<ORDER, FMT>, kMfmaWaves * 64,
                                                     f_lds_bytes(mfma_f_entries(FMT)));
  if (cus <= 0) cus = 256;
  if (per <= 0) per = 1;
  return cus * per;
}

int mfma_grid_size(int order, int fmt) {
  if (order == 3)
    return fmt == kMfmaI8 ? mfma_grid<3, kMfmaI8>() : fmt == kMfmaF4 ? mfma_grid<3, kMfmaF4>()
           : fmt == kMfmaF4Narrow ? mfma_grid<3, kMfmaF4Narrow>() : mfma_grid<3, kMfmaF4Dual>();
  return fmt == kMfmaI8 ? mfma_grid<2, kMfmaI8>() : fmt == kMfmaF4 ? mfma_grid<2, kMfmaF4>()
         : fmt == kMfmaF4Narrow ? mfma_grid<2, kMfmaF4Narrow>() : mfma_grid<2, kMfmaF4Dual>();
}

uint32_t mfma_narrow_max_samples() { return mfma_f_entries(kMfmaF4Narrow) - 1; }

void launch_mfma(const Globals &g, int order, int fmt, int grid, hipStream_t s) {
  const dim3 gd(grid), bd(kMfmaWaves * 64);
  const size_t lds = f_lds_bytes(mfma_f_entries(fmt));
  if (order == 3) {
    if (fmt == kMfmaI8) hipLaunchKernelGGL((mfma_kernel<3, kMfmaI8>), gd, bd, lds, s, g);
    else if (fmt == kMfmaF4) hipLaunchKernelGGL((mfma_kernel<3, kMfmaF4>), gd, bd, lds, s, g);
    else if (fmt == kMfmaF4Narrow) hipLaunchKernelGGL((mfma_kernel<3, kMfmaF4Narrow>), gd, bd, lds, s, g);
    else hipLaunchKernelGGL((mfma_kernel<3, kMfmaF4Dual>), gd, bd, lds, s, g);
  } else {
    if (fmt == kMfmaI8) hipLaunchKernelGGL((mfma_kernel<2, kMfmaI8>), gd, bd, lds, s, g);
    else if (fmt == kMfmaF4) hipLaunchKernelGGL((mfma_kernel<2, kMfmaF4>), gd, bd, lds, s, g);
    else if (fmt == kMfmaF4Narrow) hipLaunchKernelGGL((mfma_kernel<2, kMfmaF4Narrow>), gd, bd, lds, s, g);
    else hipLaunchKernelGGL((mfma_kernel<2, kMfmaF4Dual>), gd, bd, lds, s, g);
  }
}

// The packed pair tables (orders 3-5 on the matrix cores, jobs of fewer than
// 16,384 samples) by the order-2 contraction: for every pair a < j, its four
// {0,1}^2 counts of both classes, 4 c0 | 4 c1 << 16 each, at pairs4[a][j] as
// [g_a][g_j].  Grid: x = tile of the upper triangle of 64-variant blocks
// (row A, column B >= A, row by row), z = job; a wave takes 32 x 32 pairs.
// Two-accumulator contraction for every job (counts below 2^14 per class).
__global__ __launch_bounds__(kMfmaWaves * 64, 2) void pairs4_kernel(Globals g) {
  const JobDesc *jd = g.jobs + blockIdx.z;
  JV v = load_view(jd);
  uint4 *PT4 = uni_ptr(as_const(jd)->pairs4);
  if (PT4 == nullptr) return;
  const JobState *st = v.st;
  if (uni((uint32_t)st->status) != 0) return;
  v.W0 = uni(st->W0);
  v.W1 = uni(st->W1);
  const uint32_t n = v.n, nb = (n + 63) / 64;
  uint32_t t = blockIdx.x, A = 0;
  while (A < nb && t >= nb - A) {
    t -= nb - A;
    ++A;
  }
  if (A >= nb) return;
  const uint32_t B = A + t;
  const uint32_t wave = uni(threadIdx.x >> 6), lane = lane_id();
  const uint32_t a0 = 64 * A + 32 * (wave >> 1), j0 = 64 * B + 32 * (wave & 1);
  // a wave without a pair a < j < n has nothing to store
  if (a0 + 1 >= n || j0 >= n || j0 + 31 <= a0) return;
  v16i acc0[2][2], acc1[2][2];
  uint32_t Q[2][2][16];
  pairs_contract_fp4<kMfmaF4Narrow>(v, a0, j0, lane, acc0, acc1, Q);
  // lane: column j = j0 + (lane mod 32); register e = 4 q + i: row a = a0 +
  // 8 q + 4 h + i; block (g_a, g_j)
  const uint32_t r = lane & 31, h = lane >> 5, j = j0 + r;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t a = a0 + 8 * q + 4 * h + i;
      const int e = 4 * q + i;
      if (a < j && j < n)
        PT4[(size_t)a * v.n_pad + j] =
            make_uint4(Q[0][0][e] << 2, Q[0][1][e] << 2, Q[1][0][e] << 2, Q[1][1][e] << 2);
    }
}

void launch_pairs4(const Globals &g, uint32_t max_n, hipStream_t s) {
  const uint32_t nb = (max_n + 63) / 64;
  hipLaunchKernelGGL(pairs4_kernel, dim3(nb * (nb + 1) / 2, 1, g.n_jobs), dim3(kMfmaWaves * 64), 0, s, g);
}

}  // namespace fiuncho
