// Shared device-side definitions for the CABS library (gfx950 / CDNA4).
//
// * element types and conversions for the four compute precisions
// * Philox-4x64-10 and Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011)
//   and the integer / unit-interval / normal maps used by every random draw
// * MFMA fragment helpers for 16x16 output tiles with FP64, FP32, BF16 and
//   FP16 operands (FP32 accumulation for the 16-bit types)
// * wave64 reductions
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cabs {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) double f64x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;

typedef __bf16 bf16;
typedef _Float16 f16;

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Conversions
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ double to_f64(T v) { return (double)v; }
template <> __device__ __forceinline__ double to_f64<bf16>(bf16 v) { return (double)(float)v; }
template <> __device__ __forceinline__ double to_f64<f16>(f16 v) { return (double)(float)v; }

template <typename T> __device__ __forceinline__ float to_f32(T v) { return (float)v; }

template <typename T> __device__ __forceinline__ T from_f64(double v) { return (T)v; }
template <> __device__ __forceinline__ bf16 from_f64<bf16>(double v) { return (bf16)(float)v; }
template <> __device__ __forceinline__ f16 from_f64<f16>(double v) { return (f16)(float)v; }

template <typename T> __device__ __forceinline__ T from_f32(float v) { return (T)v; }

// Accumulator type of a compute precision: FP64 for FP64, FP32 otherwise.
template <typename T> struct Acc { typedef float type; };
template <> struct Acc<double> { typedef double type; };

// ---------------------------------------------------------------------------
// Philox-4x64-10
// ---------------------------------------------------------------------------
struct u64x4 { uint64_t v[4]; };

__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  lo = a * b;
  hi = __umul64hi(a, b);
}

__device__ __forceinline__ u64x4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                            uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, hi0, lo0);
    mulhilo64(M1, c2, hi1, lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  u64x4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// floor(x * bound / 2^64): an integer in [0, bound).
__device__ __forceinline__ uint64_t mulhi_bound(uint64_t x, uint64_t bound) { return __umul64hi(x, bound); }

// (0, 1] and [0, 1) from the top 53 bits.
__device__ __forceinline__ double unit_open0(uint64_t x) { return ((double)(x >> 11) + 1.0) * 0x1.0p-53; }
__device__ __forceinline__ double unit_open1(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

enum : uint64_t {
  STREAM_PILOT_ROWS = 0, STREAM_PILOT_COLS = 1, STREAM_INIT_ROWS = 2, STREAM_INIT_COLS = 3,
  STREAM_ERROR = 4, STREAM_LEVERAGE_ROWS = 5, STREAM_LEVERAGE_COLS = 6
};

// Philox-4x32-10: the same round structure on 32-bit words, one 32x32->64
// product per multiplier and round.  It draws the noise of the low-rank
// generator, one block per entry of A, where the 64-bit variant's products
// (built from several 32-bit multiplies each) dominated entry evaluation.
struct u32x4 { uint32_t v[4]; };

__device__ __forceinline__ u32x4 philox4x32(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
    k0 += W0; k1 += W1;
  }
  u32x4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// The two 64-bit words of the noise block of entry (i, j): Philox-4x32-10 at
// counter (lo i, hi i, lo j, hi j), key (lo seed, hi seed); words 1:0 and 3:2.
__device__ __forceinline__ void noise_words(uint64_t seed, uint64_t i, uint64_t j, uint64_t& a, uint64_t& b) {
  const u32x4 w = philox4x32((uint32_t)i, (uint32_t)(i >> 32), (uint32_t)j, (uint32_t)(j >> 32), (uint32_t)seed,
                             (uint32_t)(seed >> 32));
  a = ((uint64_t)w.v[1] << 32) | w.v[0];
  b = ((uint64_t)w.v[3] << 32) | w.v[2];
}

// Standard normal of entry (i, j) by Box-Muller on those words.
__device__ __forceinline__ double noise_f64(uint64_t seed, uint64_t i, uint64_t j) {
  uint64_t a, b;
  noise_words(seed, i, j, a, b);
  return sqrt(-2.0 * log(unit_open0(a))) * cospi(2.0 * unit_open1(b));
}
// The FP32 form (entries computed in FP32 or narrower).  u1 is the 53-bit
// value rounded to float (relative error 2^-24: the radius sqrt(-2 ln u1)
// would magnify an absolute error of 2^-24 for small u1) and goes through the
// accurate logf; the hardware square root and cos(2 pi x) take the radius and
// the top 24 bits of the second word (already in revolutions, so no range
// reduction), both with errors of a few ulp that nothing magnifies.
__device__ __forceinline__ float noise_f32(uint64_t seed, uint64_t i, uint64_t j) {
  uint64_t a, b;
  noise_words(seed, i, j, a, b);
  const float u1 = (float)unit_open0(a);
  const float u2 = (float)(uint32_t)(b >> 40) * 0x1.0p-24f;
  return __builtin_amdgcn_sqrtf(-2.0f * logf(u1)) * __builtin_amdgcn_cosf(u2);
}

// ---------------------------------------------------------------------------
// Wave reductions (wave64)
// ---------------------------------------------------------------------------
// Order between the LDS accesses of the lanes of one wave (a wavefront-scope
// fence around a wave barrier).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exchange between partner lanes within a row of 16 lanes, in four steps
// that together connect the whole row: pairs, quads, half rows (lane i with
// 7 - i), rows (lane i with 15 - i).
__device__ __forceinline__ int dpp_xchg(int v, int ctrl_id) {
  switch (ctrl_id) {
    case 0: return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    case 1: return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    case 2: return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    default: return __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false); // row_mirror
  }
}

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}
template <typename T> __device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) { T o = __shfl_xor(v, off, WAVE); v = o > v ? o : v; }
  return v;
}
template <typename T> __device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) { T o = __shfl_xor(v, off, WAVE); v = o < v ? o : v; }
  return v;
}

// ---------------------------------------------------------------------------
// MFMA fragments.  A 16x16 output tile D = A_tile (16 x K) * B_tile (K x 16)
// is built from steps of KSTEP along K.  Lane l owns row (l % 16) of A and
// column (l % 16) of B, and the KPL = KSTEP/4 contraction indices of group
// g = l / 16.  Because the contraction only sums over k, any assignment of k
// values to (group, slot) works as long as A and B use the same one; every
// kernel here hands lane l the KPL consecutive elements starting at 4-group
// offset g * KPL of the current K block.  The output holds 4 accumulators per
// lane, in column l % 16; their rows differ by instruction: the FP32-output
// instructions give rows 4 * (l / 16) + i, the FP64 one gives rows l / 16 + 4 i
// (out_row below).
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ int out_row(int g, int i) { return 4 * g + i; }
template <> __device__ __forceinline__ int out_row<double>(int g, int i) { return g + 4 * i; }

template <typename T> struct Mfma;

template <> struct Mfma<double> {
  static constexpr int KPL = 1;             // elements per lane per step
  typedef double frag;
  typedef f64x4 acc;
  __device__ static __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  __device__ static __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  static constexpr int KPL = 1;
  typedef float frag;
  typedef f32x4 acc;
  __device__ static __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<bf16> {
  static constexpr int KPL = 8;
  typedef bf16x8 frag;
  typedef f32x4 acc;
  __device__ static __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<f16> {
  static constexpr int KPL = 8;
  typedef f16x8 frag;
  typedef f32x4 acc;
  __device__ static __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static __forceinline__ acc mma(frag a, frag b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

__host__ __device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace cabs
