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
// LDS arrays filled by direct buffer-to-LDS loads (one buffer_load_dwordx4 ...
// lds per 1 KB fragment block), so chunk c + 1 is in flight while chunk c is
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
  const __amdgpu_buffer_rsrc_t brs = lds_src_rsrc(Bt, (uint32_t)N * (uint32_t)Kp * (uint32_t)sizeof(TC));
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
        const uint32_t off = (c < N && k0 < Kp) ? ((uint32_t)c * Kp + k0) * (uint32_t)sizeof(TC) : kBufOob;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(brs, CABS_TS_LDS_PTR(dst + blk * 64), 16, off, 0, 0, 0);
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

// FP64 products with K > 256 (rows too wide for registers) and without norms
// (Y = X B only), X rows and B^T rows whole 16-byte runs (K even): 128 x 128
// output tiles, 4 waves each owning a 64 x 64 quarter (16 MFMA tiles of
// 16x16x4 FP64).  K runs in stages of 16, double-buffered in LDS (64 KB, two
// work-groups per CU, so that one's barriers and first loads hide behind the
// other's MFMAs) and filled by direct buffer-to-LDS loads; a stage holds
// pairs of consecutive k of every row, ordered [pair][row], so one 16-byte LDS
// read gives a lane its operand for two MFMA steps.  Each stage reads all of
// its operands from LDS before the next stage's loads are issued: an LDS read
// issued after a pending buffer-to-LDS load makes the compiler wait for that
// load unless it can prove the two apart, which would stall every stage on
// the global latency.  The contraction order is free: in stage s, pair group
// t and step sigma, lane group g takes k = 16 s + 8 t + 2 g + sigma, for A and
// B alike.  Row and column tiles are dealt so that the column tiles of one row
// tile share an XCD (its L2 serves the rows of X to all of them).
constexpr int TF_W = 128;   // output tile edge
constexpr int TF_KT = 16;   // k per stage
constexpr int TF_NG = TF_KT / 8;         // pair groups per stage (4 lane groups x 2 k each)
constexpr int TF_NP = TF_KT / 2 * TF_W;  // 16-byte runs per operand and stage
constexpr int TF_IPW = TF_KT / 4;        // load instructions per wave, operand and stage (TF_KT over 4 waves)
typedef double tf_d2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256, 2) void tsgemm_f64_kernel(int64_t M, int K, int Kp, int N, int ntc,
                                                            const double* __restrict__ X,
                                                            const double* __restrict__ Bt, double* __restrict__ Y) {
  __shared__ uint4 sa[2][TF_NP], sb[2][TF_NP];
  const int id = blockIdx.x, xcd = id & 7, slot = id >> 3;
  const int ct = slot % ntc;
  const int64_t rt = (int64_t)(slot / ntc) * 8 + xcd;
  const int64_t row0 = rt * TF_W;
  if (row0 >= M) return;
  const int col0 = ct * TF_W;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
  const int wr = wave >> 1, wc = wave & 1;
  // this tile's rows of X, and B^T, as buffers (offsets past them read zeros)
  const int64_t nrow = M - row0 < TF_W ? M - row0 : TF_W;
  const __amdgpu_buffer_rsrc_t xrs = lds_src_rsrc(X + row0 * K, (uint32_t)(nrow * K * (int64_t)sizeof(double)));
  const __amdgpu_buffer_rsrc_t brs = lds_src_rsrc(Bt, (uint32_t)N * (uint32_t)Kp * (uint32_t)sizeof(double));
  // stage loads: instruction i (0 .. TF_KT - 1) of an operand fills pair i / 2, rows / columns 64 (i & 1) .. + 63
  auto issue = [&](uint4* da, uint4* db, int s) {
#pragma unroll
    for (int u = 0; u < TF_IPW; ++u) {
      const int i = wave * TF_IPW + u;  // TF_KT instructions per operand over 4 waves
      const int p = i >> 1, rr = ((i & 1) << 6) + lane;
      const int k0 = s * TF_KT + 2 * p;
      const int64_t xr = row0 + rr;
      const uint32_t xo = (xr < M && k0 < K) ? ((uint32_t)rr * K + k0) * (uint32_t)sizeof(double) : kBufOob;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(xrs, CABS_TS_LDS_PTR(da + i * 64), 16, xo, 0, 0, 0);
      const int bc = col0 + rr;
      const uint32_t bo = (bc < N && k0 < Kp) ? ((uint32_t)bc * Kp + k0) * (uint32_t)sizeof(double) : kBufOob;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(brs, CABS_TS_LDS_PTR(db + i * 64), 16, bo, 0, 0, 0);
    }
  };
  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  // one stage: its operands from LDS into registers, then the next stage's loads, then the MFMAs
  auto stage = [&](const uint4* ca, const uint4* cb, uint4* na, uint4* nb, int snext) {
    const tf_d2* xa = (const tf_d2*)ca;
    const tf_d2* xb = (const tf_d2*)cb;
    tf_d2 ra[TF_NG][4], rb[TF_NG][4];
#pragma unroll
    for (int t = 0; t < TF_NG; ++t) {
#pragma unroll
      for (int a = 0; a < 4; ++a) ra[t][a] = xa[(4 * t + g) * TF_W + 64 * wr + 16 * a + r];
#pragma unroll
      for (int b = 0; b < 4; ++b) rb[t][b] = xb[(4 * t + g) * TF_W + 64 * wc + 16 * b + r];
    }
    __builtin_amdgcn_sched_barrier(0);
    if (snext >= 0) issue(na, nb, snext);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < TF_NG; ++t)
#pragma unroll
      for (int sg = 0; sg < 2; ++sg)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[t][a][sg], rb[t][b][sg], acc[a][b], 0, 0, 0);
  };
  const int nks = (K + TF_KT - 1) / TF_KT;
  issue(sa[0], sb[0], 0);
  for (int s = 0; s < nks; ++s) {
    const int cur = s & 1;
    __builtin_amdgcn_s_waitcnt(0x3f70);  // vmcnt(0): this wave's loads of stage s
    __syncthreads();                     // every wave's loads landed; the other buffers are no longer read
    stage(sa[cur], sb[cur], sa[cur ^ 1], sb[cur ^ 1], s + 1 < nks ? s + 1 : -1);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int col = col0 + 64 * wc + 16 * b + r;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + 64 * wr + 16 * a + out_row<double>(g, i);
        if (row < M && col < N) Y[row * N + col] = acc[a][b][i];
      }
    }
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
  if constexpr (sizeof(TC) == 8) {
    if (K > tsf_k_max<double>() && colsq == nullptr && rowsq == nullptr && K % 2 == 0 && ((uintptr_t)X % 16) == 0 &&
        Y != nullptr) {
      const int ntc = (int)ceil_div(N, TF_W);
      const int64_t nrt = ceil_div(ceil_div(M, TF_W), 8) * 8;
      hipLaunchKernelGGL(tsgemm_f64_kernel, dim3((unsigned)(nrt * ntc)), dim3(256), 0, st, M, K, Kp, N, ntc,
                         (const double*)X, (const double*)Bt, (double*)Y);
      return hipGetLastError();
    }
  }
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
// G = X^T X with FP64 accumulation (16x16x4 FP64 MFMAs), X (M x K) in the
// compute precision.  The lower triangle of G is covered by super-tiles of
// 128 x 128 (I >= J); the grid is (row block) x (super-tile).  A block (4
// waves, each owning a 64 x 64 quarter: 16 MFMA tiles) streams its rows of
// the two 128-column strips of X through LDS in stages of GR_RS rows, loaded
// into registers one stage ahead, and converts each fragment element to FP64
// as it is read (products of FP32 or 16-bit values are exact in FP64).  The
// MFMA's contraction runs over 4 rows of X per step (lane group g takes row
// 4s + g), rows in increasing order, so each partial has a fixed rounding
// order.  Each strip of X is read once per super-tile: 4.1 x X at K = 500
// (9.3 x for 32-column tile groups).  The partials of the row blocks are
// then summed in increasing block order by gram_reduce_kernel.  The blocks of
// one row block are given ids that share an XCD (and its L2).
// ---------------------------------------------------------------------------
constexpr int GR_W = 128;             // super-tile width (columns of G)
constexpr int GR_RS = 32;             // rows per stage (16 for FP64, so that two blocks fit a CU's LDS)
constexpr int GR_TARGET_BLOCKS = 512; // two 256-thread blocks per CU

struct GramPlan {
  int nst;        // 128-column strips
  int ns;         // super-tiles (lower triangle incl. diagonal)
  int nb;         // row blocks (a multiple of 8)
  int64_t rows_per;
};

static inline int tri_row(int t) {
  int a = (int)((std::sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  return a;
}

__device__ __forceinline__ int tri_row_dev(int t) {
  int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  return a;
}

// Row blocks: every block holds a CU slot for the time of its rows, so the
// launch takes (waves of GR_TARGET_BLOCKS blocks) x (rows per block); nb (a
// multiple of 8, at most GR_MAX_BLOCKS blocks in all) minimises that product,
// the smallest nb on ties.  (A grid just past one wave, e.g. 560 blocks for
// K = 500, would run its last 48 blocks alone for a whole block time.)
constexpr int GR_MAX_BLOCKS = 2 * GR_TARGET_BLOCKS;

static inline GramPlan gram_plan(int64_t M, int K) {
  GramPlan g;
  g.nst = (K + GR_W - 1) / GR_W;
  g.ns = g.nst * (g.nst + 1) / 2;
  const int64_t nb_rows = ceil_div(ceil_div(std::max<int64_t>(M, 1), GR_RS), 8) * 8;  // one stage per block at least
  const int64_t nb_cap = std::max<int64_t>(8, std::min<int64_t>(nb_rows, GR_MAX_BLOCKS / g.ns / 8 * 8));
  int64_t nb = 8, best = -1;
  for (int64_t b = 8; b <= nb_cap; b += 8) {
    const int64_t rows_per = ceil_div(ceil_div(M, b), GR_RS) * GR_RS;
    const int64_t cost = ceil_div(g.ns * b, GR_TARGET_BLOCKS) * rows_per;
    if (best < 0 || cost < best) {
      best = cost;
      nb = b;
    }
  }
  g.rows_per = ceil_div(ceil_div(M, nb), GR_RS) * GR_RS;
  g.nb = (int)nb;
  return g;
}

// LDS row stride of a staged strip: 128 elements plus 16 elements of padding,
// so the four rows a fragment read touches start on different banks.
template <typename TC> constexpr int gr_stride() { return GR_W + 16; }
template <typename TC> constexpr int gr_rs() { return sizeof(TC) == 8 ? GR_RS / 2 : GR_RS; }

// Elements [c0, c0 + 8) of row `row` (c0 a multiple of 8; zeros past K or rend).
// mode 0: 16-byte runs of 16-bit values; 1: 8-byte pieces; 2: single elements.
template <typename TC>
__device__ __forceinline__ void gr_load8(const TC* __restrict__ X, int64_t ldx, int64_t row, int64_t rend, int K, int c0,
                                         int mode, TC (&v)[8]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = from_f64<TC>(0.0);
  if (row >= rend || c0 >= K) return;
  const TC* p = X + row * ldx + c0;
  if (c0 + 8 <= K && mode == 0 && sizeof(TC) == 2) {
    const uint4 w = *(const uint4*)p;
    const TC* e = (const TC*)&w;
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = e[q];
  } else if (c0 + 8 <= K && mode <= 1 && sizeof(TC) <= 4) {
    constexpr int PE = 8 / sizeof(TC);  // elements per 8-byte piece
#pragma unroll
    for (int q = 0; q < 8; q += PE) {
      const uint2 w = *(const uint2*)(p + q);
      const TC* e = (const TC*)&w;
#pragma unroll
      for (int u = 0; u < PE; ++u) v[q + u] = e[u];
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (c0 + q < K) v[q] = p[q];
  }
}

template <typename TC>
__global__ __launch_bounds__(256, 2) void gram_kernel(int64_t M, int K, int64_t ldx, const TC* __restrict__ X, int ns,
                                                      int nb, int64_t rows_per, int mode, double* __restrict__ part) {
  constexpr int LS = gr_stride<TC>();
  constexpr int RS = gr_rs<TC>();
  constexpr int NV = 2 * RS * GR_W / 8 / 256;  // 8-element pieces per thread and stage (both strips)
  __shared__ TC xs[2][2][RS * LS];           // [buffer][strip i / j][row][column]
  const int id = blockIdx.x, xcd = id & 7, slot = id >> 3;
  const int st = slot % ns, rb = (slot / ns) * 8 + xcd;
  if (rb >= nb) return;
  const int I = tri_row_dev(st), J = st - I * (I + 1) / 2;
  const bool diag = I == J;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
  const int wr = wave >> 1, wc = wave & 1;
  const bool active = !(diag && wr < wc);  // strictly upper quarter of a diagonal super-tile: not needed
  const int64_t rbeg = (int64_t)rb * rows_per;
  const int64_t rend = rbeg + rows_per < M ? rbeg + rows_per : M;
  const int nstage = rend > rbeg ? (int)ceil_div(rend - rbeg, RS) : 0;

  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

  // piece e = tid + 256 u: strip (e / (GR_RS * 16)), row, 8-column piece
  TC pv[NV][8];
  auto load = [&](int s) {
    const int64_t r0 = rbeg + (int64_t)s * RS;
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int e = tid + 256 * u;
      const int sj = e / (RS * 16), rem = e - sj * (RS * 16), row = rem >> 4, pc = rem & 15;
      const int c0 = (sj ? J : I) * GR_W + 8 * pc;
      if (sj && diag) {
#pragma unroll
        for (int q = 0; q < 8; ++q) pv[u][q] = from_f64<TC>(0.0);
      } else {
        gr_load8<TC>(X, ldx, r0 + row, rend, K, c0, mode, pv[u]);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int e = tid + 256 * u;
      const int sj = e / (RS * 16), rem = e - sj * (RS * 16), row = rem >> 4, pc = rem & 15;
      TC* dst = &xs[buf][sj][row * LS + 8 * pc];
#pragma unroll
      for (int q = 0; q < 8; ++q) dst[q] = pv[u][q];
    }
  };
  if (nstage > 0) load(0);
  for (int s = 0; s < nstage; ++s) {
    const int buf = s & 1;
    store(buf);
    __syncthreads();
    if (s + 1 < nstage) load(s + 1);
    if (active) {
      const TC* xi = &xs[buf][0][64 * wr + r];
      const TC* xj = diag ? &xs[buf][0][64 * wc + r] : &xs[buf][1][64 * wc + r];
#pragma unroll 2
      for (int q = 0; q < RS / 4; ++q) {
        const int ro = (4 * q + g) * LS;
        double av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = to_f64(xi[ro + 16 * a]);
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = to_f64(xj[ro + 16 * b]);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
    // no barrier here: the next stage goes to the other buffer, and the one after it is written only
    // once every wave has passed the next barrier, i.e. finished reading this one
  }
  // part layout: [super-tile][row block][128 x 128], element (i, j) of the super-tile at i * 128 + j
  if (active) {
    double* dst = part + ((int64_t)st * nb + rb) * (GR_W * GR_W);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          dst[(64 * wr + 16 * a + out_row<double>(g, i)) * GR_W + 64 * wc + 16 * b + r] = acc[a][b][i];
  }
}

// Per super-tile element: the row-block partials summed in increasing block
// order by four groups of 64 threads over four fixed ranges, then the four
// sums added in a fixed order; written to G and mirrored.
__global__ __launch_bounds__(256) void gram_reduce_kernel(int K, int nb, const double* __restrict__ part,
                                                          double* __restrict__ G) {
  __shared__ double red[4][64];
  const int st = blockIdx.x;
  const int I = tri_row_dev(st), J = st - I * (I + 1) / 2;
  const int e = blockIdx.y * 64 + (threadIdx.x & 63), c = threadIdx.x >> 6;
  const int li = e / GR_W, lj = e % GR_W;
  const int gi = I * GR_W + li, gj = J * GR_W + lj;
  const bool need = gi < K && gj < K && gi >= gj;
  const int b0 = (int)(((int64_t)nb * c) / 4), b1 = (int)(((int64_t)nb * (c + 1)) / 4);
  double s = 0.0;
  if (need)
    for (int b = b0; b < b1; ++b) s += part[((int64_t)st * nb + b) * (GR_W * GR_W) + e];
  red[c][threadIdx.x & 63] = s;
  __syncthreads();
  if (c != 0 || !need) return;
  const int l = threadIdx.x;
  const double tot = (red[0][l] + red[1][l]) + (red[2][l] + red[3][l]);
  G[(int64_t)gi * K + gj] = tot;
  G[(int64_t)gj * K + gi] = tot;
}

size_t gram_ws_bytes(int64_t M, int K) {
  // The call may use any K' <= K (the retained rank); the partials grow with the super-tile count.
  size_t best = 0;
  for (int kk = 1; kk <= K; kk += (kk == 1 ? GR_W - 1 : GR_W)) {
    const GramPlan g = gram_plan(M, std::min(kk, K));
    best = std::max(best, (size_t)g.ns * g.nb * GR_W * GR_W * sizeof(double));
  }
  const GramPlan g = gram_plan(M, K);
  best = std::max(best, (size_t)g.ns * g.nb * GR_W * GR_W * sizeof(double));
  return align256(best);
}

template <typename TC>
static void gram_launch(const GramPlan& g, int64_t M, int K, const TC* X, double* part, hipStream_t st) {
  // rows as 16-byte runs (16-bit types), 8-byte pieces, or elements
  const size_t rowb = (size_t)K * sizeof(TC);
  const int mode = (sizeof(TC) == 2 && rowb % 16 == 0 && ((uintptr_t)X % 16) == 0) ? 0
                   : (sizeof(TC) <= 4 && rowb % 8 == 0 && ((uintptr_t)X % 8) == 0) ? 1 : 2;
  const int nblk = g.nb * g.ns;
  hipLaunchKernelGGL(gram_kernel<TC>, dim3(nblk), dim3(256), 0, st, M, K, (int64_t)K, X, g.ns, g.nb, g.rows_per, mode,
                     part);
}

hipError_t launch_gram(int64_t M, int K, int compute, const void* X, double* G, void* ws, hipStream_t st) {
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
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(g.ns, GR_W * GR_W / 64), dim3(256), 0, st, K, g.nb, part, G);
  return hipGetLastError();
}

}  // namespace cabs
