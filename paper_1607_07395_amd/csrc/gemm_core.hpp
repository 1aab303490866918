// Wave-level MFMA tile core: one wave computes a 16-row x (NT*16)-column block
//   D[r][c] = sum_k X[row0 + r][k] * Y[yrow(col0 + c)][k] * ys[k]
// where X and Y are row-major with rows contiguous along k (so both operands
// are read as 16-byte runs), yrow() optionally gathers Y rows through an index
// list (sampled columns / rows of A), and ys is an optional per-k scale.
//
// Lane l owns X row (l % 16) and, per n-tile, Y row (l % 16); the k range of a
// K block is split in 4 groups of LK consecutive elements, group g = l / 16.
#pragma once

#include "common.hpp"

namespace cabs {

template <typename TC> struct TileK;
template <> struct TileK<double> { static constexpr int LK = 4; };
template <> struct TileK<float> { static constexpr int LK = 4; };
template <> struct TileK<bf16> { static constexpr int LK = 8; };
template <> struct TileK<f16> { static constexpr int LK = 8; };

template <typename TC, int LK> struct FragPack;
template <int LK> struct FragPack<double, LK> {
  __device__ static __forceinline__ double get(const double (&v)[LK], int s) { return v[s]; }
};
template <int LK> struct FragPack<float, LK> {
  __device__ static __forceinline__ float get(const float (&v)[LK], int s) { return v[s]; }
};
template <> struct FragPack<bf16, 8> {
  __device__ static __forceinline__ bf16x8 get(const bf16 (&v)[8], int) {
    bf16x8 f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = v[e];
    return f;
  }
};
template <> struct FragPack<f16, 8> {
  __device__ static __forceinline__ f16x8 get(const f16 (&v)[8], int) {
    f16x8 f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = v[e];
    return f;
  }
};

// Convert a value of the table type to the compute type (through float for the 16-bit types).
template <typename TC, typename TIn> __device__ __forceinline__ TC cvt(TIn v) { return (TC)(float)v; }
template <> __device__ __forceinline__ double cvt<double, double>(double v) { return v; }
template <> __device__ __forceinline__ float cvt<float, float>(float v) { return v; }
template <> __device__ __forceinline__ bf16 cvt<bf16, bf16>(bf16 v) { return v; }
template <> __device__ __forceinline__ f16 cvt<f16, f16>(f16 v) { return v; }
template <typename T> __device__ __forceinline__ T zero_of() { return (T)0.0f; }
template <> __device__ __forceinline__ double zero_of<double>() { return 0.0; }

// Norm accumulation in FP64 when the tables are FP64, FP32 otherwise.
template <typename TIn> struct NormT { typedef float type; };
template <> struct NormT<double> { typedef double type; };
template <typename T> __device__ __forceinline__ float widen(T v) { return (float)v; }
__device__ __forceinline__ double widen(double v) { return v; }

// Sixty-four zero bytes that out-of-range loads are pointed at, so that the
// loads need no branches (internal to each code object; never written).
static __device__ double4 kTileZero[2] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};

// A raw buffer resource over [base, base + bytes) for direct-to-LDS loads:
// offsets at or past the end (kBufOob) read zeros.  Buffer loads are not FLAT
// instructions; a FLAT load into LDS (global_load_lds) that is in flight makes
// the compiler wait for every outstanding LDS read at each use (lgkmcnt(0)),
// which undoes the read-ahead of B fragments in the MFMA loops.
constexpr uint32_t kBufOob = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t lds_src_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)bytes, 0x00020000);
}

// One 16-byte run of MFMA fragments: element s of the run as the fragment of
// MFMA step s (FP32, FP64: one element per step; 16-bit types: the whole run).
template <typename TC> struct Vec16;
template <> struct Vec16<float> {
  __device__ static __forceinline__ float frag(const uint4& v, int s) { return __uint_as_float((&v.x)[s]); }
};
template <> struct Vec16<double> {
  __device__ static __forceinline__ double frag(const uint4& v, int s) {
    return __hiloint2double((int)(&v.x)[2 * s + 1], (int)(&v.x)[2 * s]);
  }
};
template <> struct Vec16<bf16> {
  __device__ static __forceinline__ bf16x8 frag(const uint4& v, int) { return __builtin_bit_cast(bf16x8, v); }
};
template <> struct Vec16<f16> {
  __device__ static __forceinline__ f16x8 frag(const uint4& v, int) { return __builtin_bit_cast(f16x8, v); }
};

// 16-byte run of 16 / sizeof(TC) elements of row `row` from column k0 (zero
// outside the nrows x ld matrix).
template <typename TC>
__device__ __forceinline__ uint4 load_run(const TC* __restrict__ X, int64_t nrows, int ld, int64_t row, int k0,
                                          bool aligned) {
  constexpr int VE = 16 / sizeof(TC);
  uint4 v = {0u, 0u, 0u, 0u};
  if (row >= nrows || k0 >= ld) return v;
  const TC* src = X + row * ld + k0;
  if (aligned && k0 + VE <= ld) return *(const uint4*)src;
  TC tmp[VE];
#pragma unroll
  for (int e = 0; e < VE; ++e) tmp[e] = k0 + e < ld ? src[e] : zero_of<TC>();
  return __builtin_bit_cast(uint4, tmp);
}

// The same run of a matrix whose rows are whole 16-byte runs (ld a multiple
// of 16 / sizeof(TC), 16-byte aligned base): a run is either inside or wholly
// outside (then it reads zeros), so the load needs no branch.
template <typename TC>
__device__ __forceinline__ uint4 load_run_al(const TC* __restrict__ X, int64_t nrows, int ld, int64_t row, int k0,
                                             bool in) {
  const bool ok = in && row < nrows && k0 < ld;
  return *(ok ? (const uint4*)(X + row * ld + k0) : (const uint4*)kTileZero);
}

// LK consecutive elements p[k .. k+LK-1] of one row.  Whole runs are vector
// loads (16-byte pieces); `ok` false reads zeros.  All loads of a k block are
// issued before any of them is used, with no branch in between.
template <typename TIn, int LK>
__device__ __forceinline__ void tile_run_vec(const TIn* p, int k, bool ok, TIn (&v)[LK]) {
  static_assert((LK * sizeof(TIn)) % 16 == 0, "vector runs are whole 16-byte pieces");
  constexpr int NP = LK * sizeof(TIn) / 16;
  const uint4* src = (const uint4*)(ok ? p + k : (const TIn*)kTileZero);
  uint4 w[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) w[q] = src[q];
  const TIn* e = (const TIn*)w;
#pragma unroll
  for (int q = 0; q < LK; ++q) v[q] = e[q];
}
// 16-bit elements in 8-byte pieces of four, for rows whose leading dimension
// and K are multiples of 4 (8-byte aligned bases): each piece lies wholly
// inside K or wholly outside (then it reads zeros), with the same values as
// tile_run_elem and a quarter of its loads.
template <typename TIn, int LK>
__device__ __forceinline__ void tile_run_h8(const TIn* p, int k, int K, bool ok, TIn (&v)[LK]) {
  static_assert(sizeof(TIn) == 2 && LK % 4 == 0, "8-byte pieces of four 16-bit elements");
  uint2 w[LK / 4];
#pragma unroll
  for (int q = 0; q < LK / 4; ++q)
    w[q] = *(const uint2*)((ok && k + 4 * q < K) ? p + k + 4 * q : (const TIn*)kTileZero);
  const TIn* e = (const TIn*)w;
#pragma unroll
  for (int q = 0; q < LK; ++q) v[q] = e[q];
}
template <typename TIn, int LK>
__device__ __forceinline__ void tile_run_elem(const TIn* p, int k, int K, bool ok, TIn (&v)[LK]) {
#pragma unroll
  for (int q = 0; q < LK; ++q) v[q] = *((ok && k + q < K) ? p + k + q : (const TIn*)kTileZero);
}

// The tile core.  xsq / ysq receive the per-lane partial sums of squares of
// the X row and of each Y row (over this lane's k-group) when WANT_SQ.
// K blocks that lie wholly inside K use vector loads when the rows allow it
// (leading dimensions a multiple of LK, 16-byte aligned bases); the last,
// partial block uses element loads.  For tables of at most 4-byte elements
// the next block's loads are issued before the current block's MFMAs.  The
// MFMA sequence per output element is the same on every path.
template <typename TIn, typename TC, int NT, bool WANT_SQ>
__device__ __forceinline__ void gemm_tile(const TIn* __restrict__ X, int64_t ldx, int64_t M, int64_t row0,
                                          const TIn* __restrict__ Y, int64_t ldy, const int64_t* __restrict__ yidx,
                                          int64_t N, int64_t col0, const TIn* __restrict__ ys, int K,
                                          typename Mfma<TC>::acc (&acc)[NT],
                                          typename NormT<TIn>::type& xsq,
                                          typename NormT<TIn>::type (&ysq)[NT]) {
  typedef typename NormT<TIn>::type NT_t;
  constexpr int LK = TileK<TC>::LK;
  constexpr int KPL = Mfma<TC>::KPL;
  constexpr int STEPS = LK / KPL;
  constexpr bool VEC_OK = (LK * sizeof(TIn)) % 16 == 0;
  constexpr bool PREFETCH = sizeof(TIn) <= 4;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;
  const int g = lane >> 4;
  const int64_t xrow = row0 + r;
  const bool xok = xrow < M;
  const TIn* xp = X + (xok ? xrow : 0) * ldx;
  const TIn* yp[NT];
  bool yok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    int64_t c = col0 + t * 16 + r;
    yok[t] = c < N;
    int64_t yr = yok[t] ? (yidx ? yidx[c] : c) : 0;
    yp[t] = Y + yr * ldy;
    acc[t] = Mfma<TC>::zero();
    if (WANT_SQ) ysq[t] = 0;
  }
  if (WANT_SQ) xsq = 0;
  const bool vec = VEC_OK && (ldx % LK) == 0 && (ldy % LK) == 0 && (((uintptr_t)X | (uintptr_t)Y) & 15) == 0 &&
                   (ys == nullptr || ((uintptr_t)ys & 15) == 0);
  constexpr bool H8_OK = sizeof(TIn) == 2 && LK % 4 == 0;
  const bool h8 = H8_OK && (ldx % 4) == 0 && (ldy % 4) == 0 && (K % 4) == 0 &&
                  (((uintptr_t)X | (uintptr_t)Y) & 7) == 0 && (ys == nullptr || ((uintptr_t)ys & 7) == 0);
  auto fetch = [&](int kb, TIn (&xv)[LK], TIn (&yv)[NT][LK], TIn (&sv)[LK]) {
    const int k = kb + g * LK;
    if (vec && kb + 4 * LK <= K) {
      if constexpr (VEC_OK) {
        tile_run_vec<TIn, LK>(xp, k, xok, xv);
#pragma unroll
        for (int t = 0; t < NT; ++t) tile_run_vec<TIn, LK>(yp[t], k, yok[t], yv[t]);
        if (ys != nullptr) tile_run_vec<TIn, LK>(ys, k, true, sv);
      }
    } else if (h8) {
      if constexpr (H8_OK) {
        tile_run_h8<TIn, LK>(xp, k, K, xok, xv);
#pragma unroll
        for (int t = 0; t < NT; ++t) tile_run_h8<TIn, LK>(yp[t], k, K, yok[t], yv[t]);
        if (ys != nullptr) tile_run_h8<TIn, LK>(ys, k, K, true, sv);
      }
    } else {
      tile_run_elem<TIn, LK>(xp, k, K, xok, xv);
#pragma unroll
      for (int t = 0; t < NT; ++t) tile_run_elem<TIn, LK>(yp[t], k, K, yok[t], yv[t]);
      if (ys != nullptr) tile_run_elem<TIn, LK>(ys, k, K, true, sv);
    }
  };
  auto compute = [&](const TIn (&xv)[LK], const TIn (&yv)[NT][LK], const TIn (&sv)[LK]) {
    TC av[LK];
#pragma unroll
    for (int e = 0; e < LK; ++e) {
      if (WANT_SQ) xsq += (NT_t)widen(xv[e]) * (NT_t)widen(xv[e]);
      av[e] = cvt<TC, TIn>(xv[e]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      TC bv[LK];
#pragma unroll
      for (int e = 0; e < LK; ++e) {
        TIn y = yv[t][e];
        if (WANT_SQ) ysq[t] += (NT_t)widen(y) * (NT_t)widen(y);
        if (ys != nullptr) y = (TIn)(y * sv[e]);
        bv[e] = cvt<TC, TIn>(y);
      }
#pragma unroll
      for (int s = 0; s < STEPS; ++s) {
        TC as_[KPL], bs_[KPL];
#pragma unroll
        for (int e = 0; e < KPL; ++e) { as_[e] = av[s * KPL + e]; bs_[e] = bv[s * KPL + e]; }
        acc[t] = Mfma<TC>::mma(FragPack<TC, KPL>::get(as_, 0), FragPack<TC, KPL>::get(bs_, 0), acc[t]);
      }
    }
  };
  TIn xv[LK], yv[NT][LK], sv[LK];
#pragma unroll
  for (int e = 0; e < LK; ++e) sv[e] = zero_of<TIn>();
  if constexpr (PREFETCH) {
    if (K > 0) fetch(0, xv, yv, sv);
    for (int kb = 0; kb < K; kb += 4 * LK) {
      TIn xn[LK], yn[NT][LK], sn[LK];
#pragma unroll
      for (int e = 0; e < LK; ++e) sn[e] = zero_of<TIn>();
      const bool more = kb + 4 * LK < K;
      if (more) fetch(kb + 4 * LK, xn, yn, sn);
      compute(xv, yv, sv);
      if (more) {
#pragma unroll
        for (int e = 0; e < LK; ++e) { xv[e] = xn[e]; sv[e] = sn[e]; }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int e = 0; e < LK; ++e) yv[t][e] = yn[t][e];
      }
    }
  } else {
    for (int kb = 0; kb < K; kb += 4 * LK) {
      fetch(kb, xv, yv, sv);
      compute(xv, yv, sv);
    }
  }
  if (WANT_SQ) {
    xsq += __shfl_xor(xsq, 16, 64);
    xsq += __shfl_xor(xsq, 32, 64);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      ysq[t] += __shfl_xor(ysq[t], 16, 64);
      ysq[t] += __shfl_xor(ysq[t], 32, 64);
    }
  }
}

}  // namespace cabs
