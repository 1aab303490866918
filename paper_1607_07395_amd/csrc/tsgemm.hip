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

// Bt (N x Kp, Kp >= K) = B^T in the compute precision, zeros in columns K..Kp-1.
template <typename TC>
__global__ __launch_bounds__(256) void convert_bt_kernel(int K, int Kp, int N, const double* __restrict__ B,
                                                         TC* __restrict__ Bt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Kp * N) return;
  const int n = e / Kp, k = e % Kp;
  Bt[e] = k < K ? from_f64<TC>(B[(int64_t)k * N + n]) : from_f64<TC>(0.0);
}

template <typename TC>
__global__ __launch_bounds__(256) void tsgemm_kernel(int64_t M, int K, int Kp, int N, const TC* __restrict__ X,
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
      gemm_tile<TC, TC, TS_NT, false>(X, K, M, row0, Bt, Kp, nullptr, N, col0, nullptr, K, acc, xs, ysq);
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

// Fast path for K <= 512 (FP32, 16-bit) or 256 (FP64): a workgroup (4 waves)
// keeps its rows of X as 16-byte MFMA fragment runs in registers for the
// whole kernel (RT row tiles of 16 per wave) and streams B^T through LDS in
// chunks of CT column tiles, stored in fragment order (each B read is one
// contiguous 16-byte LDS read per lane).  Chunks are double-buffered in two
// LDS arrays filled by direct global-to-LDS loads (one global_load_lds_dwordx4
// per 1 KB fragment block), so chunk c + 1 is in flight while chunk c is
// multiplied; the B fragments of k block kb + D are read while block kb is
// multiplied.  B^T is stored with its rows padded to whole runs (zeros), so
// every B load is a whole run; rows of X that are not whole runs (K not a
// multiple of 16 / sizeof(TC), or X not 16-byte aligned) are loaded once per
// kernel in 8-byte pieces or element by element, with zeros past K.  Same
// outputs as tsgemm_kernel (Y, FP64 row and per-block column sums of squares).
// Compiled shapes per type: k blocks (the smallest count >= the needed one is
// used), row tiles per wave, column tiles per chunk and waves per SIMD.  The
// chunk buffers and the column sums (4 N doubles) must leave room in the
// CU's 160 KB of LDS for that many work-groups; 16-bit rows of 512 columns
// take 128 registers, so one row tile per wave (two spill).
template <typename TC> struct TsfShape {
  static constexpr int n = 5;
  static constexpr int nkb[n] = {2, 4, 7, 8, 16};
  static constexpr int rt[n] = {2, 2, 2, 2, 1};
  static constexpr int ct[n] = {2, 2, 2, 2, 2};
  static constexpr int occ[n] = {3, 3, 3, 2, 2};
};
template <> struct TsfShape<float> {
  static constexpr int n = 6;
  static constexpr int nkb[n] = {4, 8, 13, 16, 24, 32};
  static constexpr int rt[n] = {1, 1, 1, 1, 1, 1};
  static constexpr int ct[n] = {2, 2, 1, 1, 1, 1};
  static constexpr int occ[n] = {3, 3, 3, 3, 2, 2};
};
template <> struct TsfShape<double> {  // FP64 rows of K <= 256 fill 128 registers
  static constexpr int n = 4;
  static constexpr int nkb[n] = {8, 16, 25, 32};
  static constexpr int rt[n] = {1, 1, 1, 1};
  static constexpr int ct[n] = {1, 1, 1, 1};
  static constexpr int occ[n] = {1, 1, 1, 1};
};
template <typename TC> constexpr int tsf_k_max() { return TsfShape<TC>::nkb[TsfShape<TC>::n - 1] * 4 * (16 / (int)sizeof(TC)); }

#define CABS_TS_LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))

// A run of row `row` of X from column k0: a whole 16-byte load when the rows
// are whole aligned runs (mode 0), else 8-byte pieces of four 16-bit values
// (mode 1: K a multiple of 4, 8-byte aligned rows) or single elements
// (mode 2); zeros past K or M.
template <typename TC>
__device__ __forceinline__ uint4 tsf_load_a(const TC* __restrict__ X, int64_t M, int K, int64_t row, int k0, int mode) {
  constexpr int VE = 16 / sizeof(TC);
  if (mode == 0) return load_run_al<TC>(X, M, K, row, k0, true);
  uint4 v = {0u, 0u, 0u, 0u};
  if (row >= M) return v;
  const TC* p = X + row * K;
  if (mode == 1) {
    uint2* w = (uint2*)&v;
#pragma unroll
    for (int q = 0; q < VE / 4; ++q)
      if (k0 + 4 * q < K) w[q] = *(const uint2*)(p + k0 + 4 * q);
  } else {
    TC* e = (TC*)&v;
#pragma unroll
    for (int q = 0; q < VE; ++q)
      if (k0 + q < K) e[q] = p[k0 + q];
  }
  return v;
}

// NKB (k blocks of 4 runs) is a compile-time constant, so the B loads and the
// MFMA sequence carry no run-time guards; k blocks past K read zeros.
template <typename TC, int NKB, int RT, int CT, int OCC>
__global__ __launch_bounds__(256, OCC) void tsgemm_fast_kernel(int64_t M, int K, int Kp, int N, int amode,
                                                               const TC* __restrict__ X, const TC* __restrict__ Bt,
                                                               TC* __restrict__ Y, double* __restrict__ colpart,
                                                               double* __restrict__ rowsq) {
  typedef typename Mfma<TC>::acc AccV;
  constexpr int VE = 16 / sizeof(TC);          // elements per 16-byte run
  constexpr int SPV = VE / Mfma<TC>::KPL;      // MFMA steps per run
  constexpr int KBW = 4 * VE;                  // k per block (4 lane groups)
  constexpr int NBLK = CT * NKB;               // 1 KB fragment blocks per chunk
  constexpr int BPW = (NBLK + 3) / 4;          // blocks issued per wave
  constexpr int CW = CT * 16;                  // columns per chunk
  __shared__ uint4 bb0[NBLK * 64];             // [CT][NKB][64] runs
  __shared__ uint4 bb1[NBLK * 64];
  extern __shared__ double tsf_cp[];           // [4][N] per-wave column sums
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * RT);
  uint4 a[RT][NKB];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) a[rt][kb] = tsf_load_a<TC>(X, M, K, row0 + rt * 16 + c16, kb * KBW + g * VE, amode);
  auto issue = [&](uint4* dst, int cc) {
#pragma unroll
    for (int u = 0; u < BPW; ++u) {
      const int blk = wave + 4 * u;
      if (NBLK % 4 == 0 || blk < NBLK) {
        const int t = blk / NKB, kb = blk - t * NKB;
        const int c = cc + 16 * t + c16, k0 = kb * KBW + g * VE;
        const TC* src = (c < N && k0 < Kp) ? Bt + (int64_t)c * Kp + k0 : (const TC*)kTileZero;
        __builtin_amdgcn_global_load_lds((const void*)src, CABS_TS_LDS_PTR(dst + blk * 64), 16, 0, 0);
      }
    }
  };
  double rs[RT][4];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) rs[rt][i] = 0.0;
  auto compute = [&](const uint4* bs, int cc) {
    AccV acc[RT][CT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int t = 0; t < CT; ++t) acc[rt][t] = Mfma<TC>::zero();
    auto mm = [&](auto ntc) {
      constexpr int NT = decltype(ntc)::value;
      constexpr int D = RT * SPV * NT >= 8 ? 1 : 2;
      uint4 bq[D + 1][NT];
#pragma unroll
      for (int p = 0; p < D && p < NKB; ++p)
#pragma unroll
        for (int t = 0; t < NT; ++t) bq[p][t] = bs[(t * NKB + p) * 64 + lane];
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        if (kb + D < NKB) {
#pragma unroll
          for (int t = 0; t < NT; ++t) bq[(kb + D) % (D + 1)][t] = bs[(t * NKB + kb + D) * 64 + lane];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s2 = 0; s2 < SPV; ++s2)
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
              acc[rt][t] = Mfma<TC>::mma(Vec16<TC>::frag(a[rt][kb], s2), Vec16<TC>::frag(bq[kb % (D + 1)][t], s2),
                                         acc[rt][t]);
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    static_assert(CT == 1 || CT == 2, "the partial chunk below covers CT = 1 or 2");
    if constexpr (CT == 2) {
      if (N - cc > 16) mm(std::integral_constant<int, 2>{});
      else mm(std::integral_constant<int, 1>{});
    } else {
      mm(std::integral_constant<int, 1>{});
    }
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int col = cc + t * 16 + c16;
      double cs = 0.0;
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t row = row0 + rt * 16 + out_row<TC>(g, i);
          const bool ok = row < M && col < N;
          const double v = ok ? (double)acc[rt][t][i] : 0.0;
          if (ok && Y != nullptr) Y[row * N + col] = from_f64<TC>(v);
          rs[rt][i] += v * v;
          cs += v * v;
        }
      cs += __shfl_xor(cs, 16, 64);
      cs += __shfl_xor(cs, 32, 64);
      if (colpart != nullptr && g == 0 && col < N) tsf_cp[wave * N + col] = cs;
    }
  };
  issue(bb0, 0);
  for (int cc = 0; cc < N; cc += 2 * CW) {
    __builtin_amdgcn_s_waitcnt(0x3f70);  // vmcnt(0): this wave's loads of the chunk in bb0
    __syncthreads();                     // every wave's loads landed; bb1 is no longer read
    if (cc + CW < N) issue(bb1, cc + CW);
    compute(bb0, cc);
    if (cc + CW >= N) break;
    __builtin_amdgcn_s_waitcnt(0x3f70);
    __syncthreads();
    if (cc + 2 * CW < N) issue(bb0, cc + 2 * CW);
    compute(bb1, cc + CW);
  }
  if (rowsq != nullptr) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double v = rs[rt][i];
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        const int64_t row = row0 + rt * 16 + out_row<TC>(g, i);
        if (c16 == 0 && row < M) rowsq[row] = v;
      }
  }
  if (colpart != nullptr) {
    __syncthreads();
    for (int col = tid; col < N; col += 256)
      colpart[(int64_t)blockIdx.x * N + col] =
          ((tsf_cp[col] + tsf_cp[N + col]) + tsf_cp[2 * N + col]) + tsf_cp[3 * N + col];
  }
}

template <typename TC, int I>
static int64_t tsf_launch_i(int nkb, hipStream_t st, int64_t M, int K, int Kp, int N, int amode, const TC* X,
                            const TC* Bt, TC* Y, double* colpart, double* rowsq) {
  constexpr int NKB = TsfShape<TC>::nkb[I], RT = TsfShape<TC>::rt[I], CT = TsfShape<TC>::ct[I];
  constexpr int OCC = TsfShape<TC>::occ[I];
  if constexpr (I + 1 < TsfShape<TC>::n) {
    if (nkb > NKB) return tsf_launch_i<TC, I + 1>(nkb, st, M, K, Kp, N, amode, X, Bt, Y, colpart, rowsq);
  }
  const int64_t nb = ceil_div(M, 64 * RT);
  hipLaunchKernelGGL((tsgemm_fast_kernel<TC, NKB, RT, CT, OCC>), dim3((unsigned)nb), dim3(256),
                     (size_t)4 * N * sizeof(double), st, M, K, Kp, N, amode, X, Bt, Y, colpart, rowsq);
  return nb;
}

// out[c] = sum over b of part[b * N + c], in a fixed order: 16 interleaved
// segments per column, then the 16 segment sums in order.
// Column sums of the row-block partials: 16 columns per block, the 64 row
// segments of a column summed per thread with four loads in flight (fixed
// order: per thread in row order, then the segments in order).
__global__ __launch_bounds__(1024) void colreduce_kernel(int64_t nb, int N, const double* __restrict__ part,
                                                         double* __restrict__ out) {
  __shared__ double seg[64][17];
  const int cl = threadIdx.x & 15, s = threadIdx.x >> 4;
  const int col = blockIdx.x * 16 + cl;
  double acc = 0.0;
  if (col < N) {
    int64_t b = s;
    for (; b + 192 < nb; b += 256) {
      const double x0 = part[b * N + col], x1 = part[(b + 64) * N + col];
      const double x2 = part[(b + 128) * N + col], x3 = part[(b + 192) * N + col];
      acc += x0;
      acc += x1;
      acc += x2;
      acc += x3;
    }
    for (; b < nb; b += 64) acc += part[b * N + col];
  }
  seg[s][cl] = acc;
  __syncthreads();
  if (s == 0 && col < N) {
    double t = 0.0;
    for (int q = 0; q < 64; ++q) t += seg[q][cl];
    out[col] = t;
  }
}

static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// B^T's rows padded to whole 16-byte runs.
static inline int ts_kpad(int K, int compute) {
  const int ve = (int)(16 / prec_bytes(compute));
  return (K + ve - 1) / ve * ve;
}

size_t tsgemm_ws_bytes(int64_t M, int K, int N, int compute) {
  const size_t nb = (size_t)ceil_div(M, 64);
  return align256((size_t)ts_kpad(K, compute) * N * prec_bytes(compute)) + align256(nb * N * sizeof(double));
}

template <typename TC>
static hipError_t tsgemm_t(int64_t M, int K, int N, const void* X, const double* B, void* Y, double* colsq,
                           double* rowsq, void* ws, hipStream_t st) {
  constexpr int VE = 16 / (int)sizeof(TC);
  const int Kp = (K + VE - 1) / VE * VE;  // ts_kpad
  TC* Bt = (TC*)ws;
  double* part = (double*)((char*)ws + align256((size_t)Kp * N * sizeof(TC)));
  hipLaunchKernelGGL(convert_bt_kernel<TC>, dim3((unsigned)ceil_div((int64_t)Kp * N, 256)), dim3(256), 0, st, K, Kp, N,
                     B, Bt);
  int64_t nb = ceil_div(M, 64);
  if (K <= tsf_k_max<TC>()) {
    // rows of X as whole aligned runs (0), 8-byte pieces of 16-bit values (1) or single elements (2)
    const int amode = (K % VE == 0 && ((uintptr_t)X % 16) == 0) ? 0
                      : (sizeof(TC) == 2 && K % 4 == 0 && ((uintptr_t)X % 8) == 0) ? 1 : 2;
    const int nkb = (int)ceil_div(K, 4 * VE);
    nb = tsf_launch_i<TC, 0>(nkb, st, M, K, Kp, N, amode, (const TC*)X, Bt, (TC*)Y, colsq ? part : nullptr, rowsq);
  } else {
    hipLaunchKernelGGL(tsgemm_kernel<TC>, dim3((unsigned)nb), dim3(256), 0, st, M, K, Kp, N, (const TC*)X, Bt, (TC*)Y,
                       colsq ? part : nullptr, rowsq);
  }
  if (colsq) hipLaunchKernelGGL(colreduce_kernel, dim3((unsigned)ceil_div(N, 16)), dim3(1024), 0, st, nb, N, part, colsq);
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
//
// The grid is (row block) x (tile group).  A tile group is GRAM_TPB
// consecutive tiles of the lower triangle (row-major), GRAM_TPW per wave.  A
// block streams its rows through LDS in stages of `rs` rows: the stage is
// loaded with coalesced element loads into registers while the previous one
// is consumed (one 16x16x4 FP64 MFMA per tile and row quad, both operands
// read from LDS).  Rows are added in increasing order, so each tile partial
// has a fixed rounding order; partials are then summed over row blocks in
// increasing block order by a second kernel.
// ---------------------------------------------------------------------------
constexpr int GRAM_TPW = 8;          // 16x16 tiles per wave
constexpr int GRAM_TPB = 4 * GRAM_TPW;
constexpr int GRAM_MAX_NB = 256;
constexpr int GRAM_TARGET_BLOCKS = 768;  // three 256-thread blocks per CU
constexpr int GRAM_MAX_RS = 64;

template <typename TC> struct GramEpt { static constexpr int v = 32; };
template <> struct GramEpt<double> { static constexpr int v = 16; };

struct GramPlan {
  int nt, ntiles, ng, nb;
  int64_t rows_per;
};

static inline int tri_row(int t) {
  int a = (int)((std::sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  return a;
}

static inline GramPlan gram_plan(int64_t M, int K) {
  GramPlan g;
  g.nt = (K + 15) / 16;
  g.ntiles = g.nt * (g.nt + 1) / 2;
  g.ng = (int)ceil_div(g.ntiles, GRAM_TPB);
  int64_t nb = ceil_div(GRAM_TARGET_BLOCKS, g.ng);
  nb = std::min<int64_t>(nb, ceil_div(M, 16));
  nb = std::max<int64_t>(1, std::min<int64_t>(nb, GRAM_MAX_NB));
  if (nb > 8) nb = ceil_div(nb, 8) * 8;
  g.rows_per = ceil_div(M, nb);
  g.nb = (int)ceil_div(M, g.rows_per);
  return g;
}

// Staging geometry of one tile group: kal columns are read by the fragments
// (zero beyond K), kb = min(K, kal) are loaded, rows sit `stride` bytes apart
// (16 elements of padding modulo 256 bytes, so the four rows of a fragment
// fall on different LDS banks), and `rs` rows form one stage.
struct GramStage {
  int kal, kb, stride, rs;
};
__host__ __device__ inline GramStage gram_stage(int K, int ti_max, int esz, int ept) {
  GramStage s;
  s.kal = 16 * (ti_max + 1);
  s.kb = K < s.kal ? K : s.kal;
  const int want = 16 * esz;
  s.stride = s.kal * esz + ((((want - s.kal * esz) % 256) + 256) % 256);
  int rs = ((ept * 256) / s.kb) & ~3;
  s.rs = rs < 4 ? 4 : rs > GRAM_MAX_RS ? GRAM_MAX_RS : rs;
  return s;
}

__device__ __forceinline__ int tri_row_dev(int t) {
  int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  return a;
}

template <typename TC>
__global__ __launch_bounds__(256) void gram_kernel(int64_t M, int K, const TC* __restrict__ X, int ntiles, int ng,
                                                   int nb, int64_t rows_per, double* __restrict__ part) {
  constexpr int EPT = GramEpt<TC>::v;
  constexpr int ESZ = (int)sizeof(TC);
  extern __shared__ __align__(16) unsigned char gram_lds[];
  // XCD-aware order: consecutive block ids go to different XCDs, so the
  // tile groups of one row block are given ids that share an XCD (and its L2).
  const int id = blockIdx.x, xcd = id & 7, slot = id >> 3;
  const int grp = slot % ng, rb = (slot / ng) * 8 + xcd;
  if (rb >= nb) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
  const int64_t rbeg = (int64_t)rb * rows_per;
  const int64_t rend = rbeg + rows_per < M ? rbeg + rows_per : M;

  int ti[GRAM_TPW], tj[GRAM_TPW];
  bool ok[GRAM_TPW];
  f64x4 acc[GRAM_TPW];
#pragma unroll
  for (int q = 0; q < GRAM_TPW; ++q) {
    const int t = grp * GRAM_TPB + wave * GRAM_TPW + q;
    ok[q] = t < ntiles;
    const int a = tri_row_dev(ok[q] ? t : 0);
    ti[q] = ok[q] ? a : 0;
    tj[q] = ok[q] ? t - a * (a + 1) / 2 : 0;
    acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  const int tlast = min(grp * GRAM_TPB + GRAM_TPB, ntiles) - 1;
  const GramStage sg = gram_stage(K, tri_row_dev(tlast), ESZ, EPT);
  const int rs = sg.rs, kb = sg.kb, stride = sg.stride;

  // Fragment columns in [kb, kal) stay zero for the whole kernel.
  for (int e = tid; e < rs * (sg.kal - kb); e += 256) {
    const int row = e / (sg.kal - kb), col = kb + e % (sg.kal - kb);
    *(TC*)(gram_lds + row * stride + col * ESZ) = (TC)0.0f;
  }

  // Element e = i*256 + tid of a stage is (row e / kb, column e % kb).
  const int step_r = 256 / kb, step_c = 256 % kb;
  const int row_t = tid / kb, col_t = tid % kb;
  const TC* zero = (const TC*)kTileZero;
  TC v[EPT];
  auto load = [&](int64_t r0) {
    int row = row_t, col = col_t;
    asm volatile("" : "+v"(row), "+v"(col));  // recomputed per stage, not held in registers
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const bool in = row < rs && r0 + row < rend;
      const TC* src = in ? X + (r0 + row) * (int64_t)K + col : zero;
      v[i] = *src;
      col += step_c;
      row += step_r;
      if (col >= kb) { col -= kb; ++row; }
    }
  };
  auto store = [&]() {
    int row = row_t, col = col_t;
    asm volatile("" : "+v"(row), "+v"(col));  // recomputed per stage, not held in registers
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      if (row < rs) *(TC*)(gram_lds + row * stride + col * ESZ) = v[i];
      col += step_c;
      row += step_r;
      if (col >= kb) { col -= kb; ++row; }
    }
  };

  const int64_t nrows = rend > rbeg ? rend - rbeg : 0;
  const int nst = (int)ceil_div(nrows, rs);
  if (nst > 0) load(rbeg);
  for (int s = 0; s < nst; ++s) {
    __syncthreads();
    store();
    __syncthreads();
    if (s + 1 < nst) load(rbeg + (int64_t)(s + 1) * rs);
    const unsigned char* base = gram_lds + g * stride + r * ESZ;
#pragma unroll 2
    for (int qd = 0; qd < rs / 4; ++qd) {
      const unsigned char* rowp = base + 4 * qd * stride;
#pragma unroll
      for (int q = 0; q < GRAM_TPW; ++q) {
        if (!ok[q]) continue;  // uniform over the wave
        const double av = to_f64(*(const TC*)(rowp + ti[q] * 16 * ESZ));
        const double bv = to_f64(*(const TC*)(rowp + tj[q] * 16 * ESZ));
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
      }
    }
  }
  // part layout: [tile][row block][256]
#pragma unroll
  for (int q = 0; q < GRAM_TPW; ++q) {
    if (!ok[q]) continue;
    const int t = grp * GRAM_TPB + wave * GRAM_TPW + q;
    double* dst = part + ((int64_t)t * nb + rb) * 256;
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[out_row<double>(g, i) * 16 + r] = acc[q][i];
  }
}

// One block per (tile, quarter of the tile): four groups of 64 threads sum
// four fixed ranges of row blocks in increasing order, then the four sums are
// added in a fixed order.
__global__ __launch_bounds__(256) void gram_reduce_kernel(int K, int nb, const double* __restrict__ part,
                                                          double* __restrict__ G) {
  __shared__ double red[4][64];
  const int t = blockIdx.x;
  const int a = tri_row_dev(t);
  const int ti = a, tj = t - a * (a + 1) / 2;
  const int e = blockIdx.y * 64 + (threadIdx.x & 63), c = threadIdx.x >> 6;
  const int b0 = (int)(((int64_t)nb * c) / 4), b1 = (int)(((int64_t)nb * (c + 1)) / 4);
  double s = 0.0;
  for (int b = b0; b < b1; ++b) s += part[((int64_t)t * nb + b) * 256 + e];
  red[c][threadIdx.x & 63] = s;
  __syncthreads();
  if (c != 0) return;
  const int l = threadIdx.x;
  const double tot = (red[0][l] + red[1][l]) + (red[2][l] + red[3][l]);
  const int i = ti * 16 + e / 16, j = tj * 16 + e % 16;
  if (i < K && j < K) {
    G[(int64_t)i * K + j] = tot;
    G[(int64_t)j * K + i] = tot;
  }
}

size_t gram_ws_bytes(int64_t M, int K) {
  // The call may use any K' <= K (the retained rank), and the row-block count
  // grows as the tile count falls, so take the largest product.
  size_t best = 0;
  for (int kk = 16; kk < K + 16; kk += 16) {
    const GramPlan g = gram_plan(M, kk < K ? kk : K);
    best = std::max(best, (size_t)g.ntiles * g.nb * 256 * sizeof(double));
  }
  return align256(best);
}

template <typename TC>
static size_t gram_lds_bytes(const GramPlan& g, int K) {
  size_t best = 0;
  for (int grp = 0; grp < g.ng; ++grp) {
    const int tlast = std::min(grp * GRAM_TPB + GRAM_TPB, g.ntiles) - 1;
    const GramStage s = gram_stage(K, tri_row(tlast), (int)sizeof(TC), GramEpt<TC>::v);
    best = std::max(best, (size_t)s.rs * s.stride);
  }
  return best;
}

template <typename TC>
static void gram_launch(const GramPlan& g, int64_t M, int K, const TC* X, double* part, hipStream_t st) {
  const int nblk = (int)(ceil_div(g.nb, 8) * 8 * g.ng);
  hipLaunchKernelGGL(gram_kernel<TC>, dim3(nblk), dim3(256), gram_lds_bytes<TC>(g, K), st, M, K, X, g.ntiles, g.ng,
                     g.nb, g.rows_per, part);
}

hipError_t launch_gram(int64_t M, int K, int compute, const void* X, double* G, void* ws, hipStream_t st) {
  // K <= 1024 keeps one stage within one register load per thread and element slot.
  if (M <= 0 || K <= 0 || K > 1024) return hipErrorInvalidValue;
  TimerScope ts(T_GRAM, st);
  const GramPlan g = gram_plan(M, K);
  double* part = (double*)ws;
  switch (compute) {
    case P_F64: gram_launch<double>(g, M, K, (const double*)X, part, st); break;
    case P_F32: gram_launch<float>(g, M, K, (const float*)X, part, st); break;
    case P_BF16: gram_launch<bf16>(g, M, K, (const bf16*)X, part, st); break;
    case P_F16: gram_launch<f16>(g, M, K, (const f16*)X, part, st); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(g.ntiles, 4), dim3(256), 0, st, K, g.nb, part, G);
  return hipGetLastError();
}

}  // namespace cabs
