// Tall-skinny products of the sketching routine and the embedding step.
//
// tsgemm: Y = X B for X (M x K, compute precision) and a small FP64 B (K x N),
//   with optional FP64 column sums of squares of Y (the norms N_c, N_r of the
//   extrapolated singular vectors, Section 4.1) and row sums of squares (the
//   row norms |P_l| that set the k-means weights, Section 3.2).  B is first
//   converted to the compute precision and transposed so that both MFMA
//   operands are read along k.  Column sums are reduced across row blocks in
//   a fixed order (deterministic).
// gram: G = X^T X in FP64 on the FP64 MFMA, lower-triangular 16 x 16 tiles,
//   per-row-block partials reduced in a fixed order.  Used by the FP64
//   orthogonalisation of supplementary Section 3.
#include "common.hpp"
#include "gemm_core.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace cabs {

constexpr int TS_NT = 8;
constexpr int TS_MAXN = 1024;

template <typename TC>
__global__ __launch_bounds__(256) void convert_bt_kernel(int K, int N, const double* __restrict__ B, TC* __restrict__ Bt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * N) return;
  const int n = e / K, k = e % K;
  Bt[e] = from_f64<TC>(B[(int64_t)k * N + n]);
}

template <typename TC>
__global__ __launch_bounds__(256) void tsgemm_kernel(int64_t M, int K, int N, const TC* __restrict__ X,
                                                     const TC* __restrict__ Bt, TC* __restrict__ Y,
                                                     double* __restrict__ colpart, double* __restrict__ rowsq) {
  typedef typename Mfma<TC>::acc AccV;
  typedef typename NormT<TC>::type NrmT;
  __shared__ double cp[4][TS_MAXN];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  const bool active = row0 < M;
  double rs[4] = {0.0, 0.0, 0.0, 0.0};
  for (int col0 = 0; col0 < N; col0 += TS_NT * 16) {
    AccV acc[TS_NT];
    NrmT xs, ysq[TS_NT];
    if (active) {
      gemm_tile<TC, TC, TS_NT, false>(X, K, M, row0, Bt, K, nullptr, N, col0, nullptr, K, acc, xs, ysq);
    } else {
#pragma unroll
      for (int t = 0; t < TS_NT; ++t) acc[t] = Mfma<TC>::zero();
    }
#pragma unroll
    for (int t = 0; t < TS_NT; ++t) {
      const int col = col0 + t * 16 + c16;
      double cs = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + out_row<TC>(g, i);
        const bool ok = active && row < M && col < N;
        const double v = ok ? (double)acc[t][i] : 0.0;
        if (ok && Y != nullptr) Y[row * N + col] = from_f64<TC>(v);
        rs[i] += v * v;
        cs += v * v;
      }
      cs += __shfl_xor(cs, 16, 64);
      cs += __shfl_xor(cs, 32, 64);
      if (colpart != nullptr && g == 0 && col < N) cp[wave][col] = cs;
    }
  }
  if (rowsq != nullptr && active) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double v = rs[i];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      const int64_t row = row0 + out_row<TC>(g, i);
      if (c16 == 0 && row < M) rowsq[row] = v;
    }
  }
  if (colpart != nullptr) {
    __syncthreads();
    for (int col = threadIdx.x; col < N; col += blockDim.x)
      colpart[(int64_t)blockIdx.x * N + col] = ((cp[0][col] + cp[1][col]) + cp[2][col]) + cp[3][col];
  }
}

// out[c] = sum over b of part[b * N + c], in a fixed order: 16 interleaved
// segments per column, then the 16 segment sums in order.
__global__ __launch_bounds__(256) void colreduce_kernel(int64_t nb, int N, const double* __restrict__ part,
                                                        double* __restrict__ out) {
  __shared__ double seg[16][17];
  const int cl = threadIdx.x & 15, s = threadIdx.x >> 4;
  const int col = blockIdx.x * 16 + cl;
  double acc = 0.0;
  if (col < N)
    for (int64_t b = s; b < nb; b += 16) acc += part[b * N + col];
  seg[s][cl] = acc;
  __syncthreads();
  if (s == 0 && col < N) {
    double t = 0.0;
    for (int q = 0; q < 16; ++q) t += seg[q][cl];
    out[col] = t;
  }
}

static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t tsgemm_ws_bytes(int64_t M, int K, int N, int compute) {
  const size_t nb = (size_t)ceil_div(M, 64);
  return align256((size_t)K * N * prec_bytes(compute)) + align256(nb * N * sizeof(double));
}

template <typename TC>
static hipError_t tsgemm_t(int64_t M, int K, int N, const void* X, const double* B, void* Y, double* colsq,
                           double* rowsq, void* ws, hipStream_t st) {
  TC* Bt = (TC*)ws;
  double* part = (double*)((char*)ws + align256((size_t)K * N * sizeof(TC)));
  hipLaunchKernelGGL(convert_bt_kernel<TC>, dim3((unsigned)ceil_div((int64_t)K * N, 256)), dim3(256), 0, st, K, N, B, Bt);
  const int64_t nb = ceil_div(M, 64);
  hipLaunchKernelGGL(tsgemm_kernel<TC>, dim3((unsigned)nb), dim3(256), 0, st, M, K, N, (const TC*)X, Bt, (TC*)Y,
                     colsq ? part : nullptr, rowsq);
  if (colsq) hipLaunchKernelGGL(colreduce_kernel, dim3((unsigned)ceil_div(N, 16)), dim3(256), 0, st, nb, N, part, colsq);
  return hipGetLastError();
}

hipError_t launch_tsgemm(int64_t M, int K, int N, int compute, const void* X, const double* B, void* Y,
                         double* colsq, double* rowsq, void* ws, hipStream_t st) {
  if (M <= 0 || K <= 0 || N <= 0 || N > TS_MAXN) return hipErrorInvalidValue;
  TimerScope ts(T_TSGEMM, st);
  switch (compute) {
    case P_F64: return tsgemm_t<double>(M, K, N, X, B, Y, colsq, rowsq, ws, st);
    case P_F32: return tsgemm_t<float>(M, K, N, X, B, Y, colsq, rowsq, ws, st);
    case P_BF16: return tsgemm_t<bf16>(M, K, N, X, B, Y, colsq, rowsq, ws, st);
    case P_F16: return tsgemm_t<f16>(M, K, N, X, B, Y, colsq, rowsq, ws, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Gram
// ---------------------------------------------------------------------------
constexpr int GRAM_TPW = 8;          // 16x16 tiles per wave
constexpr int GRAM_TPB = 4 * GRAM_TPW;
constexpr int GRAM_MAX_NB = 128;

static inline int gram_nb(int64_t M) {
  int64_t nb = ceil_div(M, 512);
  return (int)(nb < 1 ? 1 : nb > GRAM_MAX_NB ? GRAM_MAX_NB : nb);
}

template <typename TC>
__global__ __launch_bounds__(256) void gram_kernel(int64_t M, int K, const TC* __restrict__ X, int ntiles,
                                                   double* __restrict__ part) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int64_t nb = gridDim.x;
  const int64_t rows_per = ceil_div(M, nb);
  const int64_t rbeg = blockIdx.x * rows_per;
  const int64_t rend = rbeg + rows_per < M ? rbeg + rows_per : M;
  // Tiles of the lower triangle, enumerated row by row: tile t -> (ti, tj), tj <= ti.
  int ti[GRAM_TPW], tj[GRAM_TPW];
  bool ok[GRAM_TPW];
  f64x4 acc[GRAM_TPW];
#pragma unroll
  for (int q = 0; q < GRAM_TPW; ++q) {
    const int t = blockIdx.y * GRAM_TPB + wave * GRAM_TPW + q;
    ok[q] = t < ntiles;
    int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((a + 1) * (a + 2) / 2 <= t) ++a;
    while (a * (a + 1) / 2 > t) --a;
    ti[q] = a;
    tj[q] = t - a * (a + 1) / 2;
    acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  for (int64_t r0 = rbeg; r0 < rend; r0 += 4) {
    const int64_t row = r0 + g;
    const bool rok = row < rend;
    const TC* xr = X + (rok ? row : 0) * K;
#pragma unroll
    for (int q = 0; q < GRAM_TPW; ++q) {
      if (!ok[q]) continue;
      const int ca = ti[q] * 16 + r, cb = tj[q] * 16 + r;
      const double av = (rok && ca < K) ? to_f64(xr[ca]) : 0.0;
      const double bv = (rok && cb < K) ? to_f64(xr[cb]) : 0.0;
      acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
    }
  }
  // part layout: [tile][block][256]
#pragma unroll
  for (int q = 0; q < GRAM_TPW; ++q) {
    if (!ok[q]) continue;
    const int t = blockIdx.y * GRAM_TPB + wave * GRAM_TPW + q;
    double* dst = part + ((int64_t)t * nb + blockIdx.x) * 256;
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[out_row<double>(g, i) * 16 + r] = acc[q][i];
  }
}

__global__ __launch_bounds__(256) void gram_reduce_kernel(int K, int nb, const double* __restrict__ part,
                                                          double* __restrict__ G) {
  const int t = blockIdx.x;
  int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  const int ti = a, tj = t - a * (a + 1) / 2;
  const int e = threadIdx.x;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[((int64_t)t * nb + b) * 256 + e];
  const int i = ti * 16 + e / 16, j = tj * 16 + e % 16;
  if (i < K && j < K) {
    G[(int64_t)i * K + j] = s;
    G[(int64_t)j * K + i] = s;
  }
}

size_t gram_ws_bytes(int64_t M, int K) {
  const int nt = (K + 15) / 16;
  const int64_t ntiles = (int64_t)nt * (nt + 1) / 2;
  return align256((size_t)ntiles * gram_nb(M) * 256 * sizeof(double));
}

hipError_t launch_gram(int64_t M, int K, int compute, const void* X, double* G, void* ws, hipStream_t st) {
  if (M <= 0 || K <= 0) return hipErrorInvalidValue;
  TimerScope ts(T_GRAM, st);
  const int nt = (K + 15) / 16;
  const int ntiles = nt * (nt + 1) / 2;
  const int nb = gram_nb(M);
  dim3 grid(nb, (unsigned)ceil_div(ntiles, GRAM_TPB));
  double* part = (double*)ws;
  switch (compute) {
    case P_F64: hipLaunchKernelGGL(gram_kernel<double>, grid, dim3(256), 0, st, M, K, (const double*)X, ntiles, part); break;
    case P_F32: hipLaunchKernelGGL(gram_kernel<float>, grid, dim3(256), 0, st, M, K, (const float*)X, ntiles, part); break;
    case P_BF16: hipLaunchKernelGGL(gram_kernel<bf16>, grid, dim3(256), 0, st, M, K, (const bf16*)X, ntiles, part); break;
    case P_F16: hipLaunchKernelGGL(gram_kernel<f16>, grid, dim3(256), 0, st, M, K, (const f16*)X, ntiles, part); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(ntiles), dim3(256), 0, st, K, nb, part, G);
  return hipGetLastError();
}

}  // namespace cabs
