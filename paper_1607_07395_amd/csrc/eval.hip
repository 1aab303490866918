// Pilot / follow-up sampling and entry evaluation (Algorithm 2, steps 1 and 3).
//
// * sample_floyd: k distinct uniform indices by Floyd's algorithm on
//   Philox-4x64-10, sorted ascending (one workgroup).
// * eval (LOWRANK, RBF): the sampled columns C = A(:, J) or rows R^T =
//   A(I, :)^T of a generator-defined matrix.  Both are one MFMA contraction
//   with an epilogue: X (m x r) diag(s) Y[J]^T plus the counter-based noise for
//   the low-rank source; |x|^2 + |y|^2 - 2 x.y then exp(-d/(2 sigma^2)) for the
//   RBF source.  The factor / point tables are read once per 64-row tile.
// * dense gathers: C = A(:, J) row by row (coalesced output rows); R^T =
//   A(I, :)^T through a 64 x 64 LDS tile so that both the row reads of A and
//   the writes of R^T are coalesced.
// * sparse gathers (CSR source): zero fill, then the sampled columns (rows) of
//   the column-ordered (row-ordered) nonzeros scattered into place.
#include "common.hpp"
#include "gemm_core.hpp"
#include "kernels.hpp"
#include "timing.hpp"

#include <algorithm>

namespace cabs {

// ---------------------------------------------------------------------------
// Floyd sampling
// ---------------------------------------------------------------------------
constexpr int SAMPLE_MAX_K = 4096;

__global__ __launch_bounds__(256) void sample_floyd_kernel(int64_t n, int k, uint64_t seed, uint64_t stream_id,
                                                           int64_t* __restrict__ out) {
  __shared__ int64_t draw[SAMPLE_MAX_K];
  __shared__ int64_t keys[SAMPLE_MAX_K];
  __shared__ uint8_t kept[SAMPLE_MAX_K], newk[SAMPLE_MAX_K];
  __shared__ int changed;
  const int tid = threadIdx.x;
  // 1. Every draw v_t = uniform in [0, n - k + t] is independent of the others.
  for (int t = tid; t < k; t += blockDim.x) {
    uint64_t j = (uint64_t)(n - k + t);
    u64x4 w = philox4x64((uint64_t)t, 0, stream_id, 0, seed, 0);
    draw[t] = (int64_t)mulhi_bound(w.v[0], j + 1);
  }
  __syncthreads();
  // 2. Step t keeps its draw unless an earlier step chose that value: either an
  // earlier draw that was kept, or an earlier replacement n - k + t'.  kept[t]
  // depends only on kept[t' < t], so iterating "kept[t] from the current kept[]"
  // from all-true is exact for one more leading t per pass; it stops at the
  // first pass that changes nothing (duplicates are rare, so after a few).
  for (int t = tid; t < k; t += blockDim.x) kept[t] = 1;
  __syncthreads();
  for (int pass = 0; pass <= k; ++pass) {
    if (tid == 0) changed = 0;
    __syncthreads();
    for (int t = tid; t < k; t += blockDim.x) {
      const int64_t v = draw[t];
      int taken = 0;
      for (int s = 0; s < t; ++s) taken |= kept[s] ? (draw[s] == v) : (n - k + s == v);
      const int kt = !taken;
      newk[t] = kt;
      if (kt != kept[t]) changed = 1;
    }
    __syncthreads();
    const int any = changed;
    for (int t = tid; t < k; t += blockDim.x) kept[t] = newk[t];
    __syncthreads();
    if (!any) break;  // uniform
  }
  for (int t = tid; t < k; t += blockDim.x) keys[t] = kept[t] ? draw[t] : n - k + t;
  __syncthreads();
  // 3. Bitonic sort of keys[0..P) (P = next power of two >= k, padded with +inf).
  int P = 1;
  while (P < k) P <<= 1;
  for (int t = k + tid; t < P; t += blockDim.x) keys[t] = INT64_MAX;
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = tid; t < P; t += blockDim.x) {
        int partner = t ^ stride;
        if (partner > t) {
          bool up = (t & size) == 0;
          int64_t a = keys[t], b = keys[partner];
          if ((a > b) == up) { keys[t] = b; keys[partner] = a; }
        }
      }
      __syncthreads();
    }
  }
  for (int t = tid; t < k; t += blockDim.x) out[t] = keys[t];
}

hipError_t launch_sample(int64_t n, int k, uint64_t seed, int stream_id, int64_t* out, hipStream_t st) {
  if (k <= 0 || k > SAMPLE_MAX_K || k > n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sample_floyd_kernel, dim3(1), dim3(256), 0, st, n, k, seed, (uint64_t)stream_id, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Generator evaluation through the MFMA tile core
// ---------------------------------------------------------------------------
struct EvalArgs {
  const void* X;  int64_t ldx; int64_t M;   // rows of the output (table of the un-sampled side)
  const void* Y;  int64_t ldy;              // table of the sampled side, gathered through idx
  const int64_t* idx; int64_t N;            // sampled indices (N = k)
  const void* ys;                           // per-k scale (low-rank s) or null
  int K;                                    // r or d
  void* out; int64_t ldo;
  int transposed;                           // 1: output row p is A column p (R^T)
  const int64_t* ridx;                      // X rows gathered from these rows of A (null: row p is row p)
  double noise_std; uint64_t noise_seed;
  double inv2s2;                            // 1 / (2 sigma^2)
  unsigned long long* counter;              // entries evaluated (may be null)
  int64_t rb0;                              // first row block of the launch (set by eval_dispatch_src)
};

// Adds a lane's count of entries to the counter: one atomic per wavefront.
__device__ __forceinline__ void count_entries(unsigned long long* counter, int c) {
  if (!counter) return;
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(counter, (unsigned long long)c);
}

// Five 16-column tiles per wave (80 columns): about 120 registers, so four
// waves per SIMD overlap one wave's MFMAs with another's per-entry work (the
// noise draw or the exponential); 2, 4, 7, 8 and 13 tiles measured slower or
// equal on the 10^5 x 200 low-rank block.
constexpr int EVAL_NT = 5;

// Work-group b of a launch evaluates row block rb0 + rb and column group cg
// (80 columns) with b = 8 (ncg (rb / 8) + cg) + rb mod 8: work-groups are
// dealt to the XCDs in turn, so the column groups of one row block run on the
// same XCD, close in time, and its L2 serves their shared rows of X (read from
// HBM once, not once per column group).  Launches cover at most EVAL_MAX_RB
// row blocks.
constexpr int64_t EVAL_MAX_RB = (int64_t)1 << 20;

template <typename TIn, typename TC, int SRC>
__global__ __launch_bounds__(256) void eval_kernel(EvalArgs a) {
  typedef typename Mfma<TC>::acc AccV;
  typedef typename NormT<TIn>::type NrmT;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t ncg = (a.N + EVAL_NT * 16 - 1) / (EVAL_NT * 16);
  const int64_t slot = blockIdx.x >> 3;
  const int64_t rb = a.rb0 + (slot / ncg) * 8 + (blockIdx.x & 7), cg = slot % ncg;
  const int64_t row0 = (rb * 4 + wave) * 16;
  const int64_t col0 = cg * EVAL_NT * 16;
  if (row0 >= a.M) return;
  AccV acc[EVAL_NT];
  NrmT xsq, ysq[EVAL_NT];
  gemm_tile<TIn, TC, EVAL_NT, SRC == SRC_RBF>((const TIn*)a.X, a.ldx, a.M, row0, (const TIn*)a.Y, a.ldy, a.idx, a.N,
                                              col0, (const TIn*)a.ys, a.K, acc, xsq, ysq);
  const int g = lane >> 4;
  const int c16 = lane & 15;
  TC* out = (TC*)a.out;
  int written = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rr = out_row<TC>(g, i);
    const int64_t row = row0 + rr;
    NrmT xr = 0;
    if (SRC == SRC_RBF) xr = __shfl(xsq, rr, 64);
#pragma unroll
    for (int t = 0; t < EVAL_NT; ++t) {
      const int64_t col = col0 + t * 16 + c16;
      if (row < a.M && col < a.N) {
        typedef typename Acc<TC>::type AT;
        AT v = (AT)acc[t][i];
        if (SRC == SRC_LOWRANK) {
          if (a.noise_std != 0.0) {
            const int64_t sidx = a.idx[col];
            const int64_t grow = a.ridx ? a.ridx[row] : row;
            const uint64_t ai = a.transposed ? (uint64_t)sidx : (uint64_t)grow;
            const uint64_t aj = a.transposed ? (uint64_t)grow : (uint64_t)sidx;
            if (sizeof(AT) == 8) v += (AT)(a.noise_std * noise_f64(a.noise_seed, ai, aj));
            else v += (AT)((float)a.noise_std * noise_f32(a.noise_seed, ai, aj));
          }
        } else {
          AT d2 = (AT)xr + (AT)ysq[t] - (AT)2 * v;
          d2 = d2 > (AT)0 ? d2 : (AT)0;
          if (sizeof(AT) == 8) v = (AT)exp(-(double)d2 * a.inv2s2);
          else v = (AT)__expf(-(float)d2 * (float)a.inv2s2);
        }
        out[row * a.ldo + col] = from_f64<TC>((double)v);
        ++written;
      }
    }
  }
  count_entries(a.counter, written);
}

template <typename TIn, typename TC>
static hipError_t eval_dispatch_src(int src, EvalArgs a, hipStream_t st) {
  const int64_t nrb = ceil_div(a.M, 64), ncg = ceil_div(a.N, EVAL_NT * 16);
  for (int64_t rb0 = 0; rb0 < nrb; rb0 += EVAL_MAX_RB) {
    a.rb0 = rb0;
    const int64_t nb = nrb - rb0 < EVAL_MAX_RB ? nrb - rb0 : EVAL_MAX_RB;
    const dim3 grid((unsigned)(ceil_div(nb, 8) * 8 * ncg));
    if (src == SRC_LOWRANK)
      hipLaunchKernelGGL((eval_kernel<TIn, TC, SRC_LOWRANK>), grid, dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL((eval_kernel<TIn, TC, SRC_RBF>), grid, dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dense gathers
// ---------------------------------------------------------------------------
template <typename TIn, typename TC>
__global__ __launch_bounds__(256) void dense_cols_kernel(const TIn* __restrict__ A, int64_t lda, int64_t m,
                                                         const int64_t* __restrict__ idx, int k, TC* __restrict__ out,
                                                         unsigned long long* counter) {
  // 8 output rows per block; consecutive threads write consecutive columns of a row.
  const int64_t p0 = (int64_t)blockIdx.x * 8;
  int read = 0;
  for (int rr = 0; rr < 8; ++rr) {
    const int64_t p = p0 + rr;
    if (p >= m) break;
    const TIn* arow = A + p * lda;
    for (int a = threadIdx.x; a < k; a += blockDim.x) {
      out[p * k + a] = from_f64<TC>((double)arow[idx[a]]);
      ++read;
    }
  }
  count_entries(counter, read);
}

template <typename TIn, typename TC>
__global__ __launch_bounds__(256) void dense_rows_t_kernel(const TIn* __restrict__ A, int64_t lda, int64_t n,
                                                           const int64_t* __restrict__ idx, int k,
                                                           TC* __restrict__ out, unsigned long long* counter) {
  // Tile: 64 columns of A (output rows p) x 64 sampled rows (output columns a).
  __shared__ double tile[64][65];
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int a0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63;
  const int ty = threadIdx.x >> 6;  // 0..3
  int read = 0;
  for (int al = ty; al < 64; al += 4) {
    const int a = a0 + al;
    const int64_t p = p0 + tx;
    double v = 0.0;
    if (a < k && p < n) {
      v = (double)A[idx[a] * lda + p];  // coalesced along p
      ++read;
    }
    tile[al][tx] = v;
  }
  count_entries(counter, read);
  __syncthreads();
  for (int pl = ty; pl < 64; pl += 4) {
    const int64_t p = p0 + pl;
    const int a = a0 + tx;
    if (p < n && a < k) out[p * k + a] = from_f64<TC>(tile[tx][pl]);  // coalesced along a
  }
}

template <typename TIn, typename TC>
static hipError_t dense_dispatch(const MatView& mv, bool rows_t, const int64_t* idx, int k, void* out,
                                 hipStream_t st, unsigned long long* counter) {
  const TIn* A = (const TIn*)mv.a;
  if (!rows_t) {
    hipLaunchKernelGGL((dense_cols_kernel<TIn, TC>), dim3((unsigned)ceil_div(mv.m, 8)), dim3(256), 0, st, A, mv.lda,
                       mv.m, idx, k, (TC*)out, counter);
  } else {
    dim3 grid((unsigned)ceil_div(mv.n, 64), (unsigned)ceil_div(k, 64));
    hipLaunchKernelGGL((dense_rows_t_kernel<TIn, TC>), grid, dim3(256), 0, st, A, mv.lda, mv.n, idx, k, (TC*)out,
                       counter);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sparse gathers (CSR source).  C = A(:, J): the output (m x k) is zero-filled,
// then work-group t scatters the nonzeros of column J_t (contiguous in the
// column-ordered copy) to out[i k + t]; R^T = A(I, :)^T likewise from the
// row-ordered copy.  Every output entry is written by the fill and at most one
// scatter, so the result does not depend on scheduling.
// ---------------------------------------------------------------------------
template <typename TC>
__global__ __launch_bounds__(256) void sparse_fill_kernel(int64_t total, TC* __restrict__ out,
                                                          unsigned long long* counter) {
  int wrote = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    out[e] = from_f64<TC>(0.0);
    ++wrote;
  }
  count_entries(counter, wrote);
}

template <typename TIn, typename TC>
__global__ __launch_bounds__(256) void sparse_scatter_kernel(const int64_t* __restrict__ ptr,
                                                             const int32_t* __restrict__ ind,
                                                             const TIn* __restrict__ val,
                                                             const int64_t* __restrict__ idx, int k,
                                                             TC* __restrict__ out) {
  const int t = blockIdx.x;
  const int64_t c = idx[t];
  const int64_t p0 = ptr[c], p1 = ptr[c + 1];
  for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) out[(int64_t)ind[p] * k + t] = from_f64<TC>((double)val[p]);
}

template <typename TIn, typename TC>
static hipError_t sparse_dispatch(const MatView& mv, bool rows_t, const int64_t* idx, int k, void* out,
                                  hipStream_t st, unsigned long long* counter) {
  const int64_t M = rows_t ? mv.n : mv.m;
  const int64_t total = M * k;
  const unsigned g = (unsigned)std::min<int64_t>(ceil_div(total, 256), 16384);
  hipLaunchKernelGGL(sparse_fill_kernel<TC>, dim3(g > 0 ? g : 1), dim3(256), 0, st, total, (TC*)out, counter);
  if (rows_t)
    hipLaunchKernelGGL((sparse_scatter_kernel<TIn, TC>), dim3(k), dim3(256), 0, st, mv.row_ptr, mv.col_idx,
                       (const TIn*)mv.vals, idx, k, (TC*)out);
  else
    hipLaunchKernelGGL((sparse_scatter_kernel<TIn, TC>), dim3(k), dim3(256), 0, st, mv.col_ptr, mv.row_idx,
                       (const TIn*)mv.vals_t, idx, k, (TC*)out);
  return hipGetLastError();
}

hipError_t launch_eval(const MatView& mv, bool rows_t, const int64_t* idx, int k, int compute, void* out,
                       hipStream_t st, unsigned long long* counter) {
  if (k <= 0) return hipErrorInvalidValue;
  TimerScope ts(T_EVAL, st);
  if (mv.kind == SRC_CSR) {
    if (mv.storage == P_F64) {
      if (compute == P_F64) return sparse_dispatch<double, double>(mv, rows_t, idx, k, out, st, counter);
      return hipErrorInvalidValue;
    }
    switch (compute) {
      case P_F32: return sparse_dispatch<float, float>(mv, rows_t, idx, k, out, st, counter);
      case P_BF16: return sparse_dispatch<float, bf16>(mv, rows_t, idx, k, out, st, counter);
      case P_F16: return sparse_dispatch<float, f16>(mv, rows_t, idx, k, out, st, counter);
      default: return hipErrorInvalidValue;
    }
  }
  if (mv.kind == SRC_DENSE) {
    if (mv.storage == P_F64) {
      if (compute == P_F64) return dense_dispatch<double, double>(mv, rows_t, idx, k, out, st, counter);
      return hipErrorInvalidValue;
    }
    switch (compute) {
      case P_F32: return dense_dispatch<float, float>(mv, rows_t, idx, k, out, st, counter);
      case P_BF16: return dense_dispatch<float, bf16>(mv, rows_t, idx, k, out, st, counter);
      case P_F16: return dense_dispatch<float, f16>(mv, rows_t, idx, k, out, st, counter);
      default: return hipErrorInvalidValue;
    }
  }
  EvalArgs a{};
  const int64_t M = rows_t ? mv.n : mv.m;
  if (mv.kind == SRC_LOWRANK) {
    a.X = rows_t ? mv.qf : mv.pf;
    a.Y = rows_t ? mv.pf : mv.qf;
    a.ldx = a.ldy = mv.r;
    a.K = mv.r;
    a.ys = mv.s;
  } else {
    a.X = rows_t ? mv.y : mv.x;
    a.Y = rows_t ? mv.x : mv.y;
    a.ldx = a.ldy = mv.d;
    a.K = mv.d;
    a.ys = nullptr;
    a.inv2s2 = 1.0 / (2.0 * mv.sigma * mv.sigma);
  }
  a.M = M;
  a.idx = idx;
  a.N = k;
  a.out = out;
  a.ldo = k;
  a.transposed = rows_t ? 1 : 0;
  a.noise_std = mv.noise_std;
  a.noise_seed = mv.noise_seed;
  a.counter = counter;
  if (mv.storage == P_F64) {
    if (compute == P_F64) return eval_dispatch_src<double, double>(mv.kind, a, st);
    return hipErrorInvalidValue;
  }
  switch (compute) {
    case P_F32: return eval_dispatch_src<float, float>(mv.kind, a, st);
    case P_BF16: return eval_dispatch_src<float, bf16>(mv.kind, a, st);
    case P_F16: return eval_dispatch_src<float, f16>(mv.kind, a, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Target block M = A(I, J) of the resampling CUR (Algorithm 1, step 3).  The
// generator sources gather the K-wide rows of I into a compact table and run
// the column evaluation on it (the same tile arithmetic as C = A(:, J), with
// the noise keyed on the original row); the stored sources read the entries.
// ---------------------------------------------------------------------------
template <typename TIn>
__global__ __launch_bounds__(256) void gather_table_rows_kernel(const TIn* __restrict__ X, int ld,
                                                                const int64_t* __restrict__ idx, int k,
                                                                TIn* __restrict__ out) {
  const int64_t total = (int64_t)k * ld;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / ld, c = e % ld;
    out[e] = X[idx[i] * ld + c];
  }
}

template <typename TIn, typename TC>
__global__ __launch_bounds__(256) void dense_block_kernel(const TIn* __restrict__ A, int64_t lda,
                                                          const int64_t* __restrict__ ri, const int64_t* __restrict__ ci,
                                                          int kc, TC* __restrict__ out) {
  const int i = blockIdx.y;
  const TIn* arow = A + ri[i] * lda;
  for (int j = blockIdx.x * 256 + threadIdx.x; j < kc; j += gridDim.x * 256)
    out[(int64_t)i * kc + j] = from_f64<TC>((double)arow[ci[j]]);
}

template <typename TIn, typename TC>
__global__ __launch_bounds__(256) void csr_block_kernel(MatView mv, const int64_t* __restrict__ ri,
                                                        const int64_t* __restrict__ ci, int kc, TC* __restrict__ out) {
  const int i = blockIdx.y;
  const int64_t r = ri[i];
  for (int j = blockIdx.x * 256 + threadIdx.x; j < kc; j += gridDim.x * 256)
    out[(int64_t)i * kc + j] = from_f64<TC>(csr_entry<TIn>(mv, r, ci[j]));
}

size_t eval_block_ws_bytes(const MatView& mv, int kr) {
  const size_t eb = mv.storage == P_F64 ? 8 : 4;
  if (mv.kind == SRC_LOWRANK) return (size_t)kr * mv.r * eb + 256;
  if (mv.kind == SRC_RBF) return (size_t)kr * mv.d * eb + 256;
  return 256;
}

template <typename TIn, typename TC>
static hipError_t block_dispatch(const MatView& mv, const int64_t* ri, int kr, const int64_t* ci, int kc, void* out,
                                 void* ws, hipStream_t st) {
  const dim3 sgrid((unsigned)ceil_div(kc, 256), (unsigned)kr);
  if (mv.kind == SRC_DENSE) {
    hipLaunchKernelGGL((dense_block_kernel<TIn, TC>), sgrid, dim3(256), 0, st, (const TIn*)mv.a, mv.lda, ri, ci, kc,
                       (TC*)out);
    return hipGetLastError();
  }
  if (mv.kind == SRC_CSR) {
    hipLaunchKernelGGL((csr_block_kernel<TIn, TC>), sgrid, dim3(256), 0, st, mv, ri, ci, kc, (TC*)out);
    return hipGetLastError();
  }
  EvalArgs a{};
  const int K = mv.kind == SRC_LOWRANK ? mv.r : mv.d;
  const TIn* X = (const TIn*)(mv.kind == SRC_LOWRANK ? mv.pf : mv.x);
  TIn* Xg = (TIn*)ws;
  const unsigned gg = (unsigned)std::min<int64_t>(ceil_div((int64_t)kr * K, 256), 4096);
  hipLaunchKernelGGL((gather_table_rows_kernel<TIn>), dim3(gg), dim3(256), 0, st, X, K, ri, kr, Xg);
  a.X = Xg;
  a.ldx = K;
  a.M = kr;
  a.Y = mv.kind == SRC_LOWRANK ? mv.qf : mv.y;
  a.ldy = K;
  a.K = K;
  a.ys = mv.kind == SRC_LOWRANK ? mv.s : nullptr;
  a.inv2s2 = mv.kind == SRC_RBF ? 1.0 / (2.0 * mv.sigma * mv.sigma) : 0.0;
  a.idx = ci;
  a.N = kc;
  a.out = out;
  a.ldo = kc;
  a.transposed = 0;
  a.ridx = ri;
  a.noise_std = mv.kind == SRC_LOWRANK ? mv.noise_std : 0.0;
  a.noise_seed = mv.noise_seed;
  a.counter = nullptr;
  return eval_dispatch_src<TIn, TC>(mv.kind, a, st);
}

hipError_t launch_eval_block(const MatView& mv, const int64_t* ri, int kr, const int64_t* ci, int kc, int compute,
                             void* out, void* ws, hipStream_t st) {
  if (kr <= 0 || kc <= 0 || kr > 65535) return hipErrorInvalidValue;
  TimerScope ts(T_EVAL, st);
  if (mv.storage == P_F64) {
    if (compute == P_F64) return block_dispatch<double, double>(mv, ri, kr, ci, kc, out, ws, st);
    return hipErrorInvalidValue;
  }
  switch (compute) {
    case P_F32: return block_dispatch<float, float>(mv, ri, kr, ci, kc, out, ws, st);
    case P_BF16: return block_dispatch<float, bf16>(mv, ri, kr, ci, kc, out, ws, st);
    case P_F16: return block_dispatch<float, f16>(mv, ri, kr, ci, kc, out, ws, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// W = C(I, :) in FP64
// ---------------------------------------------------------------------------
template <typename TC>
__global__ __launch_bounds__(256) void gather_rows_f64_kernel(const TC* __restrict__ src, int64_t ld,
                                                              const int64_t* __restrict__ idx, int k, int ncols,
                                                              double* __restrict__ out) {
  const int i = blockIdx.x;
  if (i >= k) return;
  const TC* row = src + idx[i] * ld;
  for (int c = threadIdx.x; c < ncols; c += blockDim.x) out[(int64_t)i * ncols + c] = to_f64(row[c]);
}

hipError_t launch_gather_rows_f64(const void* src, int compute, int64_t ld, const int64_t* idx, int k, int ncols,
                                  double* out, hipStream_t st) {
  dim3 grid(k), block(256);
  switch (compute) {
    case P_F64: hipLaunchKernelGGL(gather_rows_f64_kernel<double>, grid, block, 0, st, (const double*)src, ld, idx, k, ncols, out); break;
    case P_F32: hipLaunchKernelGGL(gather_rows_f64_kernel<float>, grid, block, 0, st, (const float*)src, ld, idx, k, ncols, out); break;
    case P_BF16: hipLaunchKernelGGL(gather_rows_f64_kernel<bf16>, grid, block, 0, st, (const bf16*)src, ld, idx, k, ncols, out); break;
    case P_F16: hipLaunchKernelGGL(gather_rows_f64_kernel<f16>, grid, block, 0, st, (const f16*)src, ld, idx, k, ncols, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace cabs
