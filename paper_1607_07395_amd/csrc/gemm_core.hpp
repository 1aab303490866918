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

// The tile core.  xsq / ysq receive the per-lane partial sums of squares of
// the X row and of each Y row (over this lane's k-group) when WANT_SQ.
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
  for (int kb = 0; kb < K; kb += 4 * LK) {
    const int k = kb + g * LK;
    TC av[LK];
#pragma unroll
    for (int e = 0; e < LK; ++e) {
      bool ok = xok && (k + e < K);
      TIn x = ok ? xp[k + e] : zero_of<TIn>();
      if (WANT_SQ) xsq += (NT_t)widen(x) * (NT_t)widen(x);
      av[e] = cvt<TC, TIn>(x);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      TC bv[LK];
#pragma unroll
      for (int e = 0; e < LK; ++e) {
        bool ok = yok[t] && (k + e < K);
        TIn y = ok ? yp[t][k + e] : zero_of<TIn>();
        if (WANT_SQ) ysq[t] += (NT_t)widen(y) * (NT_t)widen(y);
        if (ys != nullptr && ok) y = (TIn)(y * ys[k + e]);
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
