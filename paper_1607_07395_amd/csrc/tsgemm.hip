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

// Fast path for K <= 256 (512 for 16-bit types), rows of X and B^T whole 16-byte runs (K a
// multiple of 16 / sizeof(TC), X 16-byte aligned): a workgroup (4 waves, 64 rows) keeps its rows
// of X as 16-byte MFMA fragment runs in registers for the whole kernel and
// streams B^T through LDS in chunks of CT column tiles, stored in fragment
// order (each B read is one contiguous 16-byte LDS read per lane); the next
// chunk is loaded into registers while the current one is multiplied.  Same
// outputs as tsgemm_kernel (Y, FP64 row and per-block column sums of squares).
template <typename TC> struct TsfCT { static constexpr int v = 2; };
template <> struct TsfCT<double> { static constexpr int v = 1; };

template <typename TC>
static size_t tsf_lds_bytes(int nkb, int N) {
  return (size_t)TsfCT<TC>::v * nkb * 64 * 16 + (size_t)4 * N * sizeof(double);
}

template <typename TC> struct TsfOcc { static constexpr int v = 3; };
template <> struct TsfOcc<double> { static constexpr int v = 1; };  // FP64 rows of K <= 256 fill 128 registers

// NKB (k blocks of 4 runs) is a compile-time constant, so the loads, the LDS
// stores and the MFMA sequence carry no run-time guards; k blocks past K read
// zeros.
template <typename TC, int NKB>
__global__ __launch_bounds__(256, TsfOcc<TC>::v) void tsgemm_fast_kernel(int64_t M, int K, int N,
                                                                         const TC* __restrict__ X,
                                                                         const TC* __restrict__ Bt,
                                                                         TC* __restrict__ Y,
                                                                         double* __restrict__ colpart,
                                                                         double* __restrict__ rowsq) {
  typedef typename Mfma<TC>::acc AccV;
  constexpr int CT = TsfCT<TC>::v;
  constexpr int VE = 16 / sizeof(TC);          // elements per 16-byte run
  constexpr int SPV = VE / Mfma<TC>::KPL;      // MFMA steps per run
  constexpr int KBW = 4 * VE;                  // k per block (4 lane groups)
  constexpr int PER_CHUNK = CT * NKB * 64;     // runs per chunk
  constexpr int PF = (PER_CHUNK + 255) / 256;  // prefetch runs per thread
  extern __shared__ uint4 tsf_lds[];
  uint4* bs = tsf_lds;                                  // [CT][NKB][64] runs
  double* cp = (double*)(tsf_lds + PER_CHUNK);          // [4][N] per-wave column sums
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  uint4 a[NKB];
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) a[kb] = load_run_al<TC>(X, M, K, row0 + c16, kb * KBW + g * VE, true);
  uint4 pf[PF];
  auto prefetch = [&](int cc) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int e = tid + 256 * u;
      const int t = e / (NKB * 64), rem = e - t * (NKB * 64), kb = rem >> 6, l = rem & 63;
      pf[u] = load_run_al<TC>(Bt, N, K, cc + 16 * t + (l & 15), kb * KBW + (l >> 4) * VE, e < PER_CHUNK);
    }
  };
  double rs[4] = {0.0, 0.0, 0.0, 0.0};
  prefetch(0);
  for (int cc = 0; cc < N; cc += CT * 16) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int e = tid + 256 * u;
      if ((u + 1) * 256 <= PER_CHUNK || e < PER_CHUNK) bs[e] = pf[u];
    }
    __syncthreads();
    if (cc + CT * 16 < N) prefetch(cc + CT * 16);
    AccV acc[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) acc[t] = Mfma<TC>::zero();
    // tiles of the chunk that hold columns (a compile-time count per case, so
    // a chunk with fewer than CT tiles skips the empty ones)
    auto mm = [&](auto ntc) {
      constexpr int NT = decltype(ntc)::value;
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        uint4 b[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) b[t] = bs[(t * NKB + kb) * 64 + lane];
#pragma unroll
        for (int s2 = 0; s2 < SPV; ++s2)
#pragma unroll
          for (int t = 0; t < NT; ++t)
            acc[t] = Mfma<TC>::mma(Vec16<TC>::frag(a[kb], s2), Vec16<TC>::frag(b[t], s2), acc[t]);
      }
    };
    const int ntile = (N - cc + 15) / 16;
    static_assert(CT == 1 || CT == 2 || CT == 4, "the partial chunks below cover CT = 1, 2 or 4");
    if (ntile >= CT) mm(std::integral_constant<int, CT>{});
    else if constexpr (CT == 4) {
      if (ntile == 1) mm(std::integral_constant<int, 1>{});
      else if (ntile == 2) mm(std::integral_constant<int, 2>{});
      else mm(std::integral_constant<int, 3>{});
    } else if constexpr (CT == 2) {
      mm(std::integral_constant<int, 1>{});
    }
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int col = cc + t * 16 + c16;
      double cs = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + out_row<TC>(g, i);
        const bool ok = row < M && col < N;
        const double v = ok ? (double)acc[t][i] : 0.0;
        if (ok && Y != nullptr) Y[row * N + col] = from_f64<TC>(v);
        rs[i] += v * v;
        cs += v * v;
      }
      cs += __shfl_xor(cs, 16, 64);
      cs += __shfl_xor(cs, 32, 64);
      if (colpart != nullptr && g == 0 && col < N) cp[wave * N + col] = cs;
    }
  }
  if (rowsq != nullptr) {
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
    for (int col = tid; col < N; col += 256)
      colpart[(int64_t)blockIdx.x * N + col] = ((cp[col] + cp[N + col]) + cp[2 * N + col]) + cp[3 * N + col];
  }
}

// Compiled k-block counts per type (the smallest one >= the needed count is used).
template <typename TC> struct TsfNkb;
template <> struct TsfNkb<float> { static constexpr int v[4] = {4, 8, 13, 16}; };
template <> struct TsfNkb<double> { static constexpr int v[4] = {8, 16, 25, 32}; };
template <> struct TsfNkb<bf16> { static constexpr int v[5] = {2, 4, 7, 8, 16}; };  // to K = 512
template <> struct TsfNkb<f16> { static constexpr int v[5] = {2, 4, 7, 8, 16}; };
template <typename TC> constexpr int tsf_nkb_n() { return (int)(sizeof(TsfNkb<TC>::v) / sizeof(int)); }
template <typename TC> constexpr int tsf_k_max() { return TsfNkb<TC>::v[tsf_nkb_n<TC>() - 1] * 4 * (16 / (int)sizeof(TC)); }

template <typename TC, int I>
static void tsf_launch_i(int nkb, dim3 grid, hipStream_t st, int64_t M, int K, int N, const TC* X, const TC* Bt, TC* Y,
                         double* colpart, double* rowsq) {
  constexpr int NKB = TsfNkb<TC>::v[I];
  if constexpr (I + 1 < tsf_nkb_n<TC>()) {
    if (nkb > NKB) return tsf_launch_i<TC, I + 1>(nkb, grid, st, M, K, N, X, Bt, Y, colpart, rowsq);
  }
  hipLaunchKernelGGL((tsgemm_fast_kernel<TC, NKB>), grid, dim3(256), tsf_lds_bytes<TC>(NKB, N), st, M, K, N, X, Bt, Y,
                     colpart, rowsq);
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
  if (K <= tsf_k_max<TC>() && ((size_t)K * sizeof(TC)) % 16 == 0 && ((uintptr_t)X % 16) == 0) {
    const int nkb = (int)ceil_div(K, 4 * (16 / (int)sizeof(TC)));
    tsf_launch_i<TC, 0>(nkb, dim3((unsigned)nb), st, M, K, N, (const TC*)X, Bt, (TC*)Y, colsq ? part : nullptr, rowsq);
  } else {
    hipLaunchKernelGGL(tsgemm_kernel<TC>, dim3((unsigned)nb), dim3(256), 0, st, M, K, N, (const TC*)X, Bt, (TC*)Y,
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
