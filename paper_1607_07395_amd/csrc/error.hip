// Relative Frobenius error |A - C Umid R|_F / |A|_F of a finished sketch (the
// paper's error metric, Section 5).
//
// First CU = C Umid (m x kr) in FP64 (C converted exactly to FP64, products
// accumulated in FP64), so the approximation is A~_ij = CU_i . Rt_j.  Umid can
// have large entries when W has small singular values; its product with C and
// R then cancels heavily, so it is formed and dotted in FP64 whatever the
// compute precision: the error is that of the returned factors themselves.
// * sampled: n_s i.i.d. uniform entries from Philox stream 4; each group of 16
//   lanes evaluates one entry: the k-long dot product of two gathered rows and
//   the entry of A from its generator (r-long dot plus the Box-Muller noise, or
//   the RBF of two d-long points, or a dense read), accumulated in FP64.
// * exact: every entry, in 16 x 128 tiles per wave: the approximation (FP64
//   MFMA on CU and an FP64 copy of Rt) and the generator (FP64 MFMA on the
//   tables), squared differences reduced in FP64 per block and then in a fixed
//   order.
#include "common.hpp"
#include "gemm_core.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace cabs {

constexpr int ERR_NB = 1024;
constexpr int ERR_NT = 8;

static inline size_t al256e(size_t b) { return (b + 255) & ~(size_t)255; }

template <typename TIn>
__device__ __forceinline__ double entry_f64(const MatView& mv, int64_t i, int64_t j, int lane16) {
  // Returns the full entry in every lane of the 16-lane group.
  double s = 0.0;
  if (mv.kind == SRC_DENSE) {
    s = lane16 == 0 ? (double)((const TIn*)mv.a)[i * mv.lda + j] : 0.0;
  } else if (mv.kind == SRC_LOWRANK) {
    const TIn* p = (const TIn*)mv.pf + i * mv.r;
    const TIn* q = (const TIn*)mv.qf + j * mv.r;
    const TIn* sv = (const TIn*)mv.s;
    for (int t = lane16; t < mv.r; t += 16) s += (double)p[t] * (double)sv[t] * (double)q[t];
  } else {
    const TIn* x = (const TIn*)mv.x + i * mv.d;
    const TIn* y = (const TIn*)mv.y + j * mv.d;
    for (int t = lane16; t < mv.d; t += 16) { const double df = (double)x[t] - (double)y[t]; s += df * df; }
  }
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  s += __shfl_xor(s, 4, 64);
  s += __shfl_xor(s, 8, 64);
  if (mv.kind == SRC_LOWRANK) {
    if (mv.noise_std != 0.0) s += mv.noise_std * noise_f64(mv.noise_seed, (uint64_t)i, (uint64_t)j);
  } else if (mv.kind == SRC_RBF) {
    s = exp(-s / (2.0 * mv.sigma * mv.sigma));
  }
  return s;
}

// Sample t: Philox-4x32-10 at counter (lo t, hi t, 4, 0), key (lo seed, hi
// seed); i and j from the high words of 64x64 products of words 1:0 by m and
// words 3:2 by n (uniform over the m x n entries, with replacement).
__device__ __forceinline__ void err_sample_ij(uint64_t t, uint64_t seed, int64_t m, int64_t n, int64_t& i, int64_t& j) {
  const u32x4 w = philox4x32((uint32_t)t, (uint32_t)(t >> 32), STREAM_ERROR, 0, (uint32_t)seed, (uint32_t)(seed >> 32));
  i = (int64_t)mulhi_bound(((uint64_t)w.v[1] << 32) | w.v[0], (uint64_t)m);
  j = (int64_t)mulhi_bound(((uint64_t)w.v[3] << 32) | w.v[2], (uint64_t)n);
}

// Thirty-two zero bytes to point out-of-range loads at, so that loads need no
// branches (global memory, so that the selected pointer stays a global one).
static __device__ double4 kZeroRun[1] = {{0.0, 0.0, 0.0, 0.0}};

// Four consecutive elements p[e .. e+3] widened to FP64, zero from `lim` on.
// VEC: len is a multiple of 4 and rows are 16-byte aligned, so a run is either
// whole (one 16-byte load, two for FP64) or entirely past the end, in which
// case it reads the zero run.  Otherwise element loads, each past-the-end
// element also redirected to the zero run.  No branches either way, so every
// run of a row is in flight at once.
template <typename T, bool VEC> struct Run4;
template <> struct Run4<float, true> {
  __device__ static __forceinline__ void get(const float* p, int e, int lim, double (&o)[4]) {
    const float4 v = *(const float4*)(e < lim ? p + e : (const float*)kZeroRun);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <> struct Run4<double, true> {
  __device__ static __forceinline__ void get(const double* p, int e, int lim, double (&o)[4]) {
    const double* q = e < lim ? p + e : (const double*)kZeroRun;
    const double2 a = *(const double2*)q, b = *(const double2*)(q + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
  }
};
template <typename T> struct Run4<T, true> {  // 16-bit types: one 8-byte load
  static_assert(sizeof(T) == 2, "16-bit element type expected");
  __device__ static __forceinline__ void get(const T* p, int e, int lim, double (&o)[4]) {
    const uint2 v = *(const uint2*)(e < lim ? p + e : (const T*)kZeroRun);
    const T* h = (const T*)&v;
#pragma unroll
    for (int w = 0; w < 4; ++w) o[w] = to_f64(h[w]);
  }
};
template <typename T> struct Run4<T, false> {
  __device__ static __forceinline__ void get(const T* p, int e, int lim, double (&o)[4]) {
#pragma unroll
    for (int w = 0; w < 4; ++w) o[w] = to_f64(*(e + w < lim ? p + e + w : (const T*)kZeroRun));
  }
};

// Sum over the 16 lanes of a row (lanes 16 r .. 16 r + 15) by the four DPP
// exchanges of dpp_xchg.  Every lane of the row ends with the same bits: each
// step adds the same two values on both partners.
__device__ __forceinline__ float row16_sum(float v) {
#pragma unroll
  for (int c = 0; c < 4; ++c) v += __int_as_float(dpp_xchg(__float_as_int(v), c));
  return v;
}
__device__ __forceinline__ double row16_sum(double v) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int lo = dpp_xchg(__double2loint(v), c), hi = dpp_xchg(__double2hiint(v), c);
    v += __hiloint2double(hi, lo);
  }
  return v;
}

// Runs of four in the element type (same addressing as Run4, widened later).
template <typename T, bool VEC> struct RawRun4 {
  __device__ static __forceinline__ void get(const T* p, int e, int lim, T (&o)[4]) {
    if constexpr (VEC) {
      static_assert(sizeof(T) <= 8, "element type");
      const T* src = e < lim ? p + e : (const T*)kZeroRun;
      if constexpr (sizeof(T) == 8) {
        const double2 a = *(const double2*)src, b = *(const double2*)(src + 2);
        o[0] = __builtin_bit_cast(T, a.x); o[1] = __builtin_bit_cast(T, a.y);
        o[2] = __builtin_bit_cast(T, b.x); o[3] = __builtin_bit_cast(T, b.y);
      } else if constexpr (sizeof(T) == 4) {
        const float4 v = *(const float4*)src;
        o[0] = __builtin_bit_cast(T, v.x); o[1] = __builtin_bit_cast(T, v.y);
        o[2] = __builtin_bit_cast(T, v.z); o[3] = __builtin_bit_cast(T, v.w);
      } else {
        const uint2 v = *(const uint2*)src;
        const T* h = (const T*)&v;
#pragma unroll
        for (int w = 0; w < 4; ++w) o[w] = h[w];
      }
    } else {
#pragma unroll
      for (int w = 0; w < 4; ++w) o[w] = *(e + w < lim ? p + e + w : (const T*)kZeroRun);
    }
  }
};

// FP32 runs of four (same addressing as Run4, no widening).
template <bool VEC>
__device__ __forceinline__ void run4_f32(const float* p, int e, int lim, float (&o)[4]) {
  if constexpr (VEC) {
    const float4 v = *(const float4*)(e < lim ? p + e : (const float*)kZeroRun);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  } else {
#pragma unroll
    for (int w = 0; w < 4; ++w) o[w] = *(e + w < lim ? p + e + w : (const float*)kZeroRun);
  }
}

// The source term of a low-rank entry, pf_i . diag(s) . qf_j, accumulates in
// the table precision (FP32 tables: FP32, well inside the error estimate's
// accuracy); the CUR value and the RBF distance accumulate in FP64.
template <int SRC, typename TIn> struct SvT { typedef double type; };
template <> struct SvT<SRC_LOWRANK, float> { typedef float type; };

// The two dot products of one sample (i, j) by a 16-lane group: the CUR value
// ap = CU_i . Rt_j, and the source term sv (low rank: pf_i . diag(s) . qf_j;
// RBF: |x_i - y_j|^2; dense: the stored entry).  Lane l16 takes the runs
// starting at 4 l16 + 64 u; the runs of all operands (256 elements each) are
// loaded before any is used.
template <int SRC, bool VEC, typename TIn, typename TC>
__device__ __forceinline__ void sample_dots(const MatView& mv, int kr, const double* __restrict__ CU,
                                            const TC* __restrict__ Rt, int64_t ii, int64_t jj, int l16, double& ap,
                                            typename SvT<SRC, TIn>::type& sv) {
  typedef typename SvT<SRC, TIn>::type SV;
  const int tabn = SRC == SRC_LOWRANK ? mv.r : SRC == SRC_RBF ? mv.d : 0;
  const TIn* xr = SRC == SRC_LOWRANK ? (const TIn*)mv.pf + ii * mv.r
                                     : SRC == SRC_RBF ? (const TIn*)mv.x + ii * mv.d : nullptr;
  const TIn* yr = SRC == SRC_LOWRANK ? (const TIn*)mv.qf + jj * mv.r
                                     : SRC == SRC_RBF ? (const TIn*)mv.y + jj * mv.d : nullptr;
  const TIn* sp = (const TIn*)mv.s;
  const double* cu = CU + ii * kr;
  const TC* rt = Rt + jj * kr;
  ap = 0.0;
  sv = (SV)0;
  const int len = kr > tabn ? kr : tabn;
  for (int u0 = 0; u0 < len; u0 += 256) {
    double a[4][4], b[4][4];
    SV x[4][4], y[4][4], z[4][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int e = u0 + 64 * v + 4 * l16;
      Run4<double, VEC>::get(cu, e, kr, a[v]);
      Run4<TC, VEC>::get(rt, e, kr, b[v]);
      if constexpr (SRC == SRC_LOWRANK || SRC == SRC_RBF) {
        if constexpr (sizeof(SV) == 4) {
          run4_f32<VEC>((const float*)xr, e, tabn, x[v]);
          run4_f32<VEC>((const float*)yr, e, tabn, y[v]);
        } else {
          Run4<TIn, VEC>::get(xr, e, tabn, x[v]);
          Run4<TIn, VEC>::get(yr, e, tabn, y[v]);
        }
      }
      if constexpr (SRC == SRC_LOWRANK) {
        if constexpr (sizeof(SV) == 4) run4_f32<VEC>((const float*)sp, e, tabn, z[v]);
        else Run4<TIn, VEC>::get(sp, e, tabn, z[v]);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        ap += a[v][w] * b[v][w];
        if constexpr (SRC == SRC_LOWRANK) sv += x[v][w] * z[v][w] * y[v][w];
        if constexpr (SRC == SRC_RBF) { const SV df = x[v][w] - y[v][w]; sv += df * df; }
      }
  }
  if constexpr (SRC == SRC_DENSE) sv = l16 == 0 ? (double)((const TIn*)mv.a)[ii * mv.lda + jj] : 0.0;
}

// One sample per lane ((i, j), when `valid`).  The per-sample scalar work (the
// noise of a low-rank entry, the RBF exponential, the residual) runs once per
// lane; the sample indices and noise then go through LDS to the lane's 16-lane
// group, which works through its 16 lanes' samples in order (two dot products
// and two row sums each), and the owning lane keeps the reduced values.  VEC:
// rows of CU, Rt and the tables may be read as 16-byte runs (decided on the
// host from sizes and pointer alignment).
struct ErrRec { int64_t i, j; };

template <int SRC, typename TIn, typename TC, bool VEC>
__device__ __forceinline__ void err_batch(const MatView& mv, int kr, const double* __restrict__ CU,
                                          const TC* __restrict__ Rt, int64_t i, int64_t j, bool valid,
                                          double& num, double& den) {
  typedef typename SvT<SRC, TIn>::type SV;
  __shared__ ErrRec rec[256];
  const int lane = threadIdx.x & 63, l16 = lane & 15;
  const int gbase = threadIdx.x & ~15;
  if (!valid) { i = 0; j = 0; }
  double nz = 0.0;
  if (SRC == SRC_LOWRANK && valid && mv.noise_std != 0.0) nz = noise_f64(mv.noise_seed, (uint64_t)i, (uint64_t)j);
  if (SRC == SRC_CSR && valid) nz = csr_entry<TIn>(mv, i, j);  // the stored entry or 0, one search per lane
  rec[threadIdx.x] = ErrRec{i, j};
  wave_lds_sync();
  double my_ap = 0.0;
  SV my_s = (SV)0;
  for (int q = 0; q < 16; ++q) {
    const ErrRec r = rec[gbase + q];
    double ap;
    SV sv;
    sample_dots<SRC, VEC, TIn, TC>(mv, kr, CU, Rt, r.i, r.j, l16, ap, sv);
    ap = row16_sum(ap);
    sv = row16_sum(sv);
    if (l16 == q) { my_ap = ap; my_s = sv; }
  }
  wave_lds_sync();  // the next batch rewrites rec
  if (valid) {
    double a = (double)my_s;
    if (SRC == SRC_LOWRANK) a += mv.noise_std * nz;
    else if (SRC == SRC_RBF) a = exp(-a / (2.0 * mv.sigma * mv.sigma));
    else if (SRC == SRC_CSR) a = nz;
    num += (a - my_ap) * (a - my_ap);
    den += a * a;
  }
}

// Block partial sums in a fixed order: lanes, then the four waves.
__device__ __forceinline__ void err_block_store(double num, double den, double* __restrict__ part, int64_t slot) {
  __shared__ double rn[4], rd[4];
  num = wave_sum(num);
  den = wave_sum(den);
  if ((threadIdx.x & 63) == 0) { rn[threadIdx.x >> 6] = num; rd[threadIdx.x >> 6] = den; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * slot] = ((rn[0] + rn[1]) + rn[2]) + rn[3];
    part[2 * slot + 1] = ((rd[0] + rd[1]) + rd[2]) + rd[3];
  }
}

// Samples taken in the order they are drawn: block b evaluates batches of 256
// consecutive sample numbers b * 256, (b + nb) * 256, ...
template <int SRC, typename TIn, typename TC, bool VEC>
__global__ __launch_bounds__(256) void err_sampled_kernel(MatView mv, int kr, const double* __restrict__ CU,
                                                          const TC* __restrict__ Rt, int64_t ns, uint64_t seed,
                                                          double* __restrict__ part) {
  double num = 0.0, den = 0.0;
  for (int64_t b0 = (int64_t)blockIdx.x * 256; b0 < ns; b0 += (int64_t)gridDim.x * 256) {
    const int64_t t = b0 + threadIdx.x;
    int64_t i = 0, j = 0;
    if (t < ns) err_sample_ij((uint64_t)t, seed, mv.m, mv.n, i, j);
    err_batch<SRC, TIn, TC, VEC>(mv, kr, CU, Rt, i, j, t < ns, num, den);
  }
  err_block_store(num, den, part, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Sampled error with the samples grouped by row bucket.  Each bucket (RB
// consecutive rows) is one work-group, so the row-side data of a sample (the
// generator row and the FP64 row of CU) comes from cache after its first use
// and only the column side is gathered per sample.  The grouping is a stable
// counting sort of the sample numbers t (bucket-major, then chunk, then t), so
// every sum is taken in a fixed order.  The counting pass stores each sample's
// (i, j) by t, and the sort moves the pairs themselves, so the Philox draw of a
// sample's indices is made once.
// ---------------------------------------------------------------------------
constexpr int EB_BBITS = 13;
constexpr int EB_MAXB = 1 << EB_BBITS;   // buckets at most
constexpr int EB_G = 512;       // sample chunks of the counting sort

// Sample keys: row bucket (rb consecutive rows) times column stripe (sw
// consecutive columns), row-bucket major: key = (i / rb) * ns + j / sw.
struct EbPlan { int64_t rb; int nrb; int ns; int64_t sw; int nbk; int64_t tchunk; };

static inline EbPlan eb_plan(int64_t m, int64_t n, int64_t nsamp, int stripes) {
  EbPlan p;
  p.ns = stripes;
  p.sw = ceil_div(n, stripes);
  p.rb = ceil_div(m, EB_MAXB / stripes);
  if (p.rb < 16) p.rb = 16;  // at least a 16-row bucket per work-group
  p.nrb = (int)ceil_div(m, p.rb);
  p.nbk = p.nrb * stripes;
  p.tchunk = ceil_div(nsamp, EB_G);
  return p;
}

__device__ __forceinline__ int eb_key(const EbPlan& p, int64_t i, int64_t j) {
  return (int)(i / p.rb) * p.ns + (int)(j / p.sw);
}

// The sorted path needs n_s, m, n < 2^31 (kept as int32) and at least one
// sample per row on average (else there is nothing to reuse).
static inline bool eb_use(int64_t m, int64_t n, int64_t ns) {
  const int64_t lim = (int64_t)1 << 31;
  return ns >= m && ns < lim && m < lim && n < lim;
}

__global__ __launch_bounds__(256) void eb_count_kernel(int64_t m, int64_t n, int64_t ns, uint64_t seed, EbPlan pl,
                                                       int2* __restrict__ ij, int32_t* __restrict__ counts) {
  __shared__ int32_t hist[EB_MAXB];
  for (int b = threadIdx.x; b < pl.nbk; b += 256) hist[b] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * pl.tchunk;
  const int64_t t1 = t0 + pl.tchunk < ns ? t0 + pl.tchunk : ns;
  for (int64_t t = t0 + threadIdx.x; t < t1; t += 256) {
    int64_t i, j;
    err_sample_ij((uint64_t)t, seed, m, n, i, j);
    ij[t] = make_int2((int)i, (int)j);
    atomicAdd(&hist[eb_key(pl, i, j)], 1);
  }
  __syncthreads();
  // chunk-major (counts[g * nbk + b]): each chunk writes its histogram as one contiguous row
  for (int b = threadIdx.x; b < pl.nbk; b += 256) counts[(int64_t)blockIdx.x * pl.nbk + b] = hist[b];
}

// Per bucket (one thread each, consecutive buckets in consecutive lanes, so
// every read of a chunk's row is contiguous): the total over chunks.
__global__ __launch_bounds__(256) void eb_totals_kernel(EbPlan pl, const int32_t* __restrict__ counts,
                                                        int32_t* __restrict__ totals) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= pl.nbk) return;
  int s = 0;
#pragma unroll 8
  for (int g = 0; g < EB_G; ++g) s += counts[(int64_t)g * pl.nbk + b];
  totals[b] = s;
}

// One work-group: exclusive scan of the bucket totals.
__global__ __launch_bounds__(1024) void eb_scan_kernel(EbPlan pl, const int32_t* __restrict__ totals,
                                                       int32_t* __restrict__ starts) {
  __shared__ int32_t part[1024];
  constexpr int PER = EB_MAXB / 1024;
  const int tid = threadIdx.x;
  int v[PER], sum = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid * PER + q;
    v[q] = b < pl.nbk ? totals[b] : 0;
    sum += v[q];
  }
  part[tid] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int x = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += x;
    __syncthreads();
  }
  int run = part[tid] - sum;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid * PER + q;
    if (b < pl.nbk) starts[b] = run;
    run += v[q];
  }
  if (tid == 1023) starts[pl.nbk] = part[1023];
}

// Per bucket (one thread each, as above): offsets of each chunk's run inside
// the bucket, stored chunk-major (offs[g * nbk + b]) so that a chunk reads its
// own row.
__global__ __launch_bounds__(256) void eb_offsets_kernel(EbPlan pl, const int32_t* __restrict__ counts,
                                                         const int32_t* __restrict__ starts,
                                                         int32_t* __restrict__ offs) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= pl.nbk) return;
  int run = starts[b];
#pragma unroll 8
  for (int g = 0; g < EB_G; ++g) {
    const int64_t e = (int64_t)g * pl.nbk + b;
    const int c = counts[e];
    offs[e] = run;
    run += c;
  }
}

// Chunk g places its samples' (i, j), in increasing t within each bucket.  The
// per-bucket write positions start at the chunk's offsets (read once, as one
// row) and advance in LDS.  A round is 256 consecutive samples, 64 per wave;
// ranks among equal buckets inside a wave come from ballots, and the four waves
// place their samples in wave order.
__global__ __launch_bounds__(256) void eb_scatter_kernel(int64_t ns, EbPlan pl, const int2* __restrict__ ij,
                                                         const int32_t* __restrict__ offs,
                                                         int2* __restrict__ sorted) {
  __shared__ int32_t run[EB_MAXB];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int b = tid; b < pl.nbk; b += 256) run[b] = offs[(int64_t)blockIdx.x * pl.nbk + b];
  const int64_t t0 = (int64_t)blockIdx.x * pl.tchunk;
  const int64_t t1 = t0 + pl.tchunk < ns ? t0 + pl.tchunk : ns;
  for (int64_t base = t0; base < t1; base += 256) {
    const int64_t t = base + tid;
    const bool valid = t < t1;
    const int2 e = valid ? ij[t] : make_int2(0, 0);
    const int b = valid ? eb_key(pl, e.x, e.y) : -1;
    // lanes holding the same bucket: one ballot per bit of the bucket number
    // (invalid lanes carry -1, whose top bit no valid bucket has)
    uint64_t same = ~0ull;
#pragma unroll
    for (int bit = 0; bit < EB_BBITS + 1; ++bit) {
      const bool on = (b >> bit) & 1;
      const uint64_t bb = __ballot(on);
      same &= on ? bb : ~bb;
    }
    const int rank = __builtin_popcountll(same & ((1ull << lane) - 1ull));
    const bool last = ((same >> lane) >> 1) == 0;
    for (int w = 0; w < 4; ++w) {
      __syncthreads();
      if (wave == w && valid) {
        sorted[run[b] + rank] = e;
        if (last) run[b] += rank + 1;
      }
    }
  }
}

// One work-group per bucket, in batches of 256 of the bucket's samples.
template <int SRC, typename TIn, typename TC, bool VEC>
__global__ __launch_bounds__(256) void eb_eval_kernel(MatView mv, int kr, const double* __restrict__ CU,
                                                      const TC* __restrict__ Rt,
                                                      const int32_t* __restrict__ starts,
                                                      const int2* __restrict__ sorted,
                                                      double* __restrict__ part) {
  const int b = blockIdx.x;
  const int s0 = starts[b], s1 = starts[b + 1];
  double num = 0.0, den = 0.0;
  for (int b0 = s0; b0 < s1; b0 += 256) {
    const int s = b0 + (int)threadIdx.x;
    const bool valid = s < s1;
    const int2 e = valid ? sorted[s] : make_int2(0, 0);
    err_batch<SRC, TIn, TC, VEC>(mv, kr, CU, Rt, (int64_t)e.x, (int64_t)e.y, valid, num, den);
  }
  err_block_store(num, den, part, b);
}

// Low-rank source with FP32 tables, row buckets of at most ER_RB rows and k,
// r <= ER_KMAX.  Samples are keyed by (row bucket, column stripe) with ER_S
// stripes, one work-group per key; block ids are dealt to the XCDs in turn,
// so all work-groups of a stripe run on one XCD and the column side of their
// samples (R^T_j and qf_j) comes from that XCD's L2.  Within a work-group the
// samples are laid out by row (16-lane group g takes rows g, g + 16, ...; a
// row's samples stay in key order), every lane drawing the noise of the
// samples it places.  A group walks its samples holding the current row's
// FP64 CU run and FP32 pf o s run in registers, loads only the column side
// per sample, with the next ER_D samples' loads in flight, and lane q keeps
// the sums of every 16th sample so that residuals are formed 16 at a time.
// Sums are per lane in sample order, then lanes, groups and work-groups, in
// fixed orders.
constexpr int ER_RB = 128;
constexpr int ER_CH = 2048;
constexpr int ER_KMAX = 256;
constexpr int ER_D = 2;
constexpr int ER_S = 8;

template <typename TC, bool VEC>
__global__ __launch_bounds__(256) void eb_eval_rows_kernel(MatView mv, int kr, const double* __restrict__ CU,
                                                           const TC* __restrict__ Rt, EbPlan pl,
                                                           const int32_t* __restrict__ starts,
                                                           const int2* __restrict__ sorted,
                                                           double* __restrict__ part) {
  constexpr int SETS = ER_CH / 256;  // 64-record sets per wave and chunk
  __shared__ int32_t sj[ER_CH];
  __shared__ double snz[ER_CH];
  __shared__ uint8_t sro[ER_CH];
  __shared__ int2 tmp[ER_CH];
  __shared__ int wrun[4][ER_RB];
  __shared__ int wbase[4][ER_RB];
  __shared__ int gbeg[17];
  __shared__ double gn[16], gd[16];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l16 = lane & 15, grp = tid >> 4;
  const int key = blockIdx.x;
  const int64_t row0 = (int64_t)(key / pl.ns) * pl.rb;
  const int r = mv.r;
  // per-lane byte offsets of the four runs in a row; with whole runs (VEC) a
  // run past k or r is moved to the row's last run, whose values then meet a
  // zero run of the row side (the other case loads element by element)
  int off_rt[4], off_qf[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int c = 64 * v + 4 * l16;
    off_rt[v] = (c + 4 <= kr ? c : kr - 4) * (int)sizeof(TC);
    off_qf[v] = (c + 4 <= r ? c : r - 4) * (int)sizeof(float);
  }
  double num = 0.0, den = 0.0;  // per lane: its samples' residuals
  const int s0 = starts[key], s1 = starts[key + 1];
  for (int c0 = s0; c0 < s1; c0 += ER_CH) {
    const int n = s1 - c0 < ER_CH ? s1 - c0 : ER_CH;
    for (int e = lane; e < ER_RB; e += 64) wrun[wave][e] = 0;
    wave_lds_sync();
    // pass A: wave w takes records w * (ER_CH / 4) + 64 k + lane; rank within
    // equal layout keys (row % 16, row / 16); (key, rank, column) to LDS
#pragma unroll 1
    for (int k = 0; k < SETS; ++k) {
      const int idx = wave * (ER_CH / 4) + 64 * k + lane;
      const bool valid = idx < n;
      const int2 e = valid ? sorted[c0 + idx] : make_int2(0, 0);
      const int ro = (int)(e.x - row0);
      const int lk = valid ? ((ro & 15) << 3) | (ro >> 4) : -1;
      uint64_t same = ~0ull;
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {  // lk in [-1, 128): eight bits tell them apart
        const bool on = (lk >> bit) & 1;
        const uint64_t bb = __ballot(on);
        same &= on ? bb : ~bb;
      }
      const int rank = __builtin_popcountll(same & ((1ull << lane) - 1ull));
      const bool last = ((same >> lane) >> 1) == 0;
      const int ls = valid ? lk : 0;
      const int posl = wrun[wave][ls] + rank;
      wave_lds_sync();
      if (valid && last) wrun[wave][ls] += rank + 1;
      tmp[idx] = make_int2(valid ? (lk << 16) | posl : -1, e.y);
      wave_lds_sync();
    }
    __syncthreads();
    // layout: key lk's segment starts after all smaller keys; within a key, waves in order
    if (tid < ER_RB) {
      int tot = 0;
#pragma unroll
      for (int w = 0; w < 4; ++w) tot += wrun[w][tid];
      wbase[0][tid] = tot;  // staged for the scan below
    }
    __syncthreads();
    if (wave == 0) {  // exclusive scan of the ER_RB key totals, two per lane
      const int a0 = wbase[0][2 * lane], a1 = wbase[0][2 * lane + 1];
      int incl = a0 + a1;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int x = __shfl_up(incl, o, 64);
        if (lane >= o) incl += x;
      }
      const int ex = incl - a0 - a1;
      wave_lds_sync();
      int run0 = ex, run1 = ex + a0;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int c0w = wrun[w][2 * lane], c1w = wrun[w][2 * lane + 1];
        wbase[w][2 * lane] = run0;
        wbase[w][2 * lane + 1] = run1;
        run0 += c0w;
        run1 += c1w;
      }
      if ((lane & 3) == 0) gbeg[lane >> 2] = ex;  // key 8 g starts group g's segment
      if (lane == 63) gbeg[16] = incl;
    }
    __syncthreads();
    // pass B: samples to their segments, with their noise
#pragma unroll 1
    for (int k = 0; k < SETS; ++k) {
      const int idx = wave * (ER_CH / 4) + 64 * k + lane;
      const int2 t = tmp[idx];
      if (idx < n && t.x >= 0) {
        const int lk = t.x >> 16, pos = wbase[wave][lk] + (t.x & 0xffff);
        const int ro = ((lk & 7) << 4) | (lk >> 3);
        sj[pos] = t.y;
        sro[pos] = (uint8_t)ro;
        snz[pos] = mv.noise_std != 0.0 ? noise_f64(mv.noise_seed, (uint64_t)(row0 + ro), (uint64_t)t.y) : 0.0;
      }
    }
    __syncthreads();
    // group grp: its samples in order, ER_D of them in flight
    const int p0 = gbeg[grp], p1 = gbeg[grp + 1];
    if (p0 < p1) {
      const char* rtb = (const char*)Rt;
      const char* qfb = (const char*)mv.qf;
      TC bq[ER_D][4][4];  // raw R^T_j runs (widened at use)
      float yq[ER_D][4][4];
      auto fetch = [&](int p, TC (&bo)[4][4], float (&yo)[4][4]) {
        const int64_t j = sj[p];
        const char* rrow = rtb + j * kr * (int64_t)sizeof(TC);
        const char* qrow = qfb + j * r * (int64_t)sizeof(float);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if constexpr (VEC) {
            RawRun4<TC, true>::get((const TC*)(rrow + off_rt[v]), 0, 4, bo[v]);
            run4_f32<true>((const float*)(qrow + off_qf[v]), 0, 4, yo[v]);
          } else {
            const int c = 64 * v + 4 * l16;
            RawRun4<TC, false>::get((const TC*)rrow, c, kr, bo[v]);
            run4_f32<false>((const float*)qrow, c, r, yo[v]);
          }
        }
      };
#pragma unroll
      for (int d = 0; d < ER_D; ++d)
        if (p0 + d < p1) fetch(p0 + d, bq[d], yq[d]);
      double cu[4][4];
      float ps[4][4];
      int cur = -1;
      double my_ap = 0.0;
      float my_sv = 0.0f;
      for (int p = p0; p < p1; p += ER_D) {
#pragma unroll
        for (int d = 0; d < ER_D; ++d) {
          const int pp = p + d;
          if (pp < p1) {
            const int ro = sro[pp];
            if (ro != cur) {  // the row side of a new row (uniform in the group)
              cur = ro;
              const int64_t row = row0 + ro;
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int c = 64 * v + 4 * l16;
                Run4<double, VEC>::get(CU + row * kr, c, kr, cu[v]);
                float pv[4], sv4[4];
                run4_f32<VEC>((const float*)mv.pf + row * r, c, r, pv);
                run4_f32<VEC>((const float*)mv.s, c, r, sv4);
#pragma unroll
                for (int w = 0; w < 4; ++w) ps[v][w] = pv[w] * sv4[w];
              }
            }
            double ap = 0.0;
            float sv = 0.0f;
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
              for (int w = 0; w < 4; ++w) {
                ap += cu[v][w] * to_f64(bq[d][v][w]);
                sv += ps[v][w] * yq[d][v][w];
              }
            if (pp + ER_D < p1) fetch(pp + ER_D, bq[d], yq[d]);
            ap = row16_sum(ap);
            sv = row16_sum(sv);
            const int q = (pp - p0) & 15;
            if (l16 == q) { my_ap = ap; my_sv = sv; }
            if (q == 15 || pp + 1 == p1) {  // residuals of the last 16 samples, one per lane
              if (l16 <= q) {
                const double av = (double)my_sv + mv.noise_std * snz[pp - q + l16];
                num += (av - my_ap) * (av - my_ap);
                den += av * av;
              }
            }
          }
        }
      }
    }
    __syncthreads();  // LDS reused by the next chunk
  }
  num = row16_sum(num);
  den = row16_sum(den);
  if (l16 == 0) { gn[grp] = num; gd[grp] = den; }
  __syncthreads();
  if (tid == 0) {
    double n2 = 0.0, d2 = 0.0;
    for (int g = 0; g < 16; ++g) { n2 += gn[g]; d2 += gd[g]; }
    part[2 * (int64_t)key] = n2;
    part[2 * (int64_t)key + 1] = d2;
  }
}

static inline bool er_rows_ok(const MatView& mv, int kr, int64_t ns) {
  if (mv.kind != SRC_LOWRANK || mv.storage != P_F32) return false;
  if (!eb_use(mv.m, mv.n, ns)) return false;
  return eb_plan(mv.m, mv.n, ns, ER_S).rb <= ER_RB && kr >= 4 && kr <= ER_KMAX && mv.r >= 4 && mv.r <= ER_KMAX;
}

// The sorted path's plan: column stripes when the row kernel takes it.
static inline EbPlan eb_plan_for(const MatView& mv, int kr, int64_t ns) {
  return eb_plan(mv.m, mv.n, ns, er_rows_ok(mv, kr, ns) ? ER_S : 1);
}

template <typename TIn>
__global__ __launch_bounds__(256) void err_exact_kernel(MatView mv, int kr, const double* __restrict__ CU,
                                                        const double* __restrict__ Rt, double* __restrict__ part) {
  typedef double TC;
  typedef typename Mfma<TC>::acc AccV;
  typedef typename NormT<TC>::type NrmC;
  typedef typename NormT<TIn>::type NrmI;
  __shared__ double rn[4], rd[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  double num = 0.0, den = 0.0;
  if (row0 < mv.m) {
    for (int64_t col0 = 0; col0 < mv.n; col0 += ERR_NT * 16) {
      AccV ap[ERR_NT];
      NrmC xs, ys[ERR_NT];
      gemm_tile<TC, TC, ERR_NT, false>(CU, kr, mv.m, row0, Rt, kr, nullptr, mv.n, col0, nullptr, kr, ap, xs, ys);
      typedef typename Mfma<double>::acc AccA;
      AccA av[ERR_NT];
      NrmI xa = 0, ya[ERR_NT];
      typedef double TA;
      if (mv.kind == SRC_LOWRANK) {
        gemm_tile<TIn, TA, ERR_NT, false>((const TIn*)mv.pf, mv.r, mv.m, row0, (const TIn*)mv.qf, mv.r, nullptr, mv.n,
                                          col0, (const TIn*)mv.s, mv.r, av, xa, ya);
      } else if (mv.kind == SRC_RBF) {
        gemm_tile<TIn, TA, ERR_NT, true>((const TIn*)mv.x, mv.d, mv.m, row0, (const TIn*)mv.y, mv.d, nullptr, mv.n,
                                         col0, nullptr, mv.d, av, xa, ya);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = out_row<TC>(g, i);
        const int64_t row = row0 + rr;
        const NrmI xr = mv.kind == SRC_RBF ? __shfl(xa, rr, 64) : (NrmI)0;
#pragma unroll
        for (int t = 0; t < ERR_NT; ++t) {
          const int64_t col = col0 + t * 16 + c16;
          if (row < mv.m && col < mv.n) {
            double a;
            if (mv.kind == SRC_DENSE) {
              a = (double)((const TIn*)mv.a)[row * mv.lda + col];
            } else if (mv.kind == SRC_LOWRANK) {
              a = (double)av[t][i];
              if (mv.noise_std != 0.0) a += mv.noise_std * noise_f64(mv.noise_seed, (uint64_t)row, (uint64_t)col);
            } else {
              double d2 = (double)xr + (double)ya[t] - 2.0 * (double)av[t][i];
              d2 = d2 > 0.0 ? d2 : 0.0;
              a = exp(-d2 / (2.0 * mv.sigma * mv.sigma));
            }
            const double r = a - (double)ap[t][i];
            num += r * r;
            den += a * a;
          }
        }
      }
    }
  }
  num = wave_sum(num);
  den = wave_sum(den);
  if (lane == 0) { rn[wave] = num; rd[wave] = den; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ((rn[0] + rn[1]) + rn[2]) + rn[3];
    part[2 * blockIdx.x + 1] = ((rd[0] + rd[1]) + rd[2]) + rd[3];
  }
}

// Exact error over every entry of a CSR source: the same 16-row x 128-column
// tiles of C U R as err_exact_kernel, with the tile of A built per wave in LDS:
// zero-filled, then lane r < 16 finds the first nonzero of row row0 + r at or
// after the tile's first column (binary search) and writes the row's nonzeros
// inside the tile.  Sums in the same fixed order as err_exact_kernel.
template <typename TIn>
__global__ __launch_bounds__(256) void err_exact_csr_kernel(MatView mv, int kr, const double* __restrict__ CU,
                                                            const double* __restrict__ Rt,
                                                            double* __restrict__ part) {
  typedef double TC;
  typedef typename Mfma<TC>::acc AccV;
  typedef typename NormT<TC>::type NrmC;
  constexpr int TW = ERR_NT * 16;
  __shared__ double at[4][16 * TW];
  __shared__ double rn[4], rd[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  double* tile = at[wave];
  double num = 0.0, den = 0.0;
  if (row0 < mv.m) {
    for (int64_t col0 = 0; col0 < mv.n; col0 += TW) {
      AccV ap[ERR_NT];
      NrmC xs, ys[ERR_NT];
      gemm_tile<TC, TC, ERR_NT, false>(CU, kr, mv.m, row0, Rt, kr, nullptr, mv.n, col0, nullptr, kr, ap, xs, ys);
      for (int e = lane; e < 16 * TW; e += 64) tile[e] = 0.0;
      wave_lds_sync();
      if (lane < 16 && row0 + lane < mv.m) {
        const int64_t r = row0 + lane;
        int64_t lo = mv.row_ptr[r], hi = mv.row_ptr[r + 1];
        const int64_t end = hi;
        while (lo < hi) {
          const int64_t mid = (lo + hi) >> 1;
          if (mv.col_idx[mid] < col0) lo = mid + 1;
          else hi = mid;
        }
        for (int64_t p = lo; p < end && mv.col_idx[p] < col0 + TW; ++p)
          tile[lane * TW + (mv.col_idx[p] - col0)] = (double)((const TIn*)mv.vals)[p];
      }
      wave_lds_sync();
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = out_row<TC>(g, i);
        const int64_t row = row0 + rr;
#pragma unroll
        for (int t = 0; t < ERR_NT; ++t) {
          const int64_t col = col0 + t * 16 + c16;
          if (row < mv.m && col < mv.n) {
            const double a = tile[rr * TW + t * 16 + c16];
            const double r = a - (double)ap[t][i];
            num += r * r;
            den += a * a;
          }
        }
      }
      wave_lds_sync();  // the tile is rewritten next
    }
  }
  num = wave_sum(num);
  den = wave_sum(den);
  if (lane == 0) { rn[wave] = num; rd[wave] = den; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ((rn[0] + rn[1]) + rn[2]) + rn[3];
    part[2 * blockIdx.x + 1] = ((rd[0] + rd[1]) + rd[2]) + rd[3];
  }
}

// Sum of the block partials in a fixed order: thread t takes blocks t, t + 256, ...,
// then a fixed tree over the threads.
__global__ __launch_bounds__(256) void err_final_kernel(int nb, const double* __restrict__ part,
                                                        double* __restrict__ out3) {
  __shared__ double sn[256], sd[256];
  const int tid = threadIdx.x;
  double n = 0.0, d = 0.0;
  for (int b = tid; b < nb; b += 256) { n += part[2 * b]; d += part[2 * b + 1]; }
  sn[tid] = n;
  sd[tid] = d;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) { sn[tid] += sn[tid + h]; sd[tid] += sd[tid + h]; }
    __syncthreads();
  }
  if (tid == 0) {
    out3[0] = sn[0];
    out3[1] = sd[0];
    out3[2] = sd[0] > 0.0 ? sqrt(sn[0] / sd[0]) : 0.0;
  }
}

static inline int64_t exact_nb(const MatView& mv) { return ceil_div(mv.m, 64); }

static inline int64_t part_blocks(const MatView& mv, int kr, int64_t ns) {
  if (ns == 0) return exact_nb(mv);
  return eb_use(mv.m, mv.n, ns) ? eb_plan_for(mv, kr, ns).nbk : ERR_NB;
}

static inline size_t eb_ws_bytes(const MatView& mv, int kr, int64_t ns) {
  if (ns == 0 || !eb_use(mv.m, mv.n, ns)) return 0;
  const EbPlan pl = eb_plan_for(mv, kr, ns);
  return 2 * al256e((size_t)pl.nbk * EB_G * 4) + 2 * al256e(((size_t)pl.nbk + 1) * 4) + 2 * al256e((size_t)ns * 8);
}

size_t error_ws_bytes(const MatView& mv, int k2c, int k2r, int compute, int64_t n_samples) {
  const int64_t nb = part_blocks(mv, k2r, n_samples);
  size_t b = al256e((size_t)mv.m * k2r * sizeof(double)) + tsgemm_ws_bytes(mv.m, k2c, k2r, P_F64) +
             al256e((size_t)nb * 2 * sizeof(double)) + eb_ws_bytes(mv, k2r, n_samples) + 256;
  if (compute != P_F64) {
    b += al256e((size_t)mv.m * k2c * sizeof(double));                     // C in FP64
    if (n_samples == 0) b += al256e((size_t)mv.n * k2r * sizeof(double));  // Rt in FP64 (exact mode)
  }
  return b;
}

template <typename TC>
__global__ __launch_bounds__(256) void widen_kernel(int64_t n, const TC* __restrict__ src, double* __restrict__ dst) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) dst[e] = to_f64(src[e]);
}

template <typename TC>
static void widen(int64_t n, const void* src, double* dst, hipStream_t st) {
  const unsigned g = (unsigned)std::min<int64_t>(ceil_div(n, 256), 8192);
  hipLaunchKernelGGL(widen_kernel<TC>, dim3(g), dim3(256), 0, st, n, (const TC*)src, dst);
}

static void widen_any(int compute, int64_t n, const void* src, double* dst, hipStream_t st) {
  switch (compute) {
    case P_F32: widen<float>(n, src, dst, st); break;
    case P_BF16: widen<bf16>(n, src, dst, st); break;
    case P_F16: widen<f16>(n, src, dst, st); break;
    default: break;
  }
}

// Calls f(source kind, vec) with both as compile-time constants.
template <typename F>
static void with_src(int kind, bool vec, F&& f) {
  auto go = [&](auto src) {
    if (vec) f(src, std::integral_constant<bool, true>{});
    else f(src, std::integral_constant<bool, false>{});
  };
  if (kind == SRC_DENSE) go(std::integral_constant<int, SRC_DENSE>{});
  else if (kind == SRC_LOWRANK) go(std::integral_constant<int, SRC_LOWRANK>{});
  else if (kind == SRC_CSR) go(std::integral_constant<int, SRC_CSR>{});
  else go(std::integral_constant<int, SRC_RBF>{});
}

template <typename TIn, typename TC>
static hipError_t error_t(const MatView& mv, int kr, const double* CU, const TC* Rt, const double* Rt64, int64_t ns,
                          uint64_t seed, double* part, char* ebws, double* out3, hipStream_t st) {
  TimerScope ts(T_ERROR, st);
  // rows are read as 16-byte runs when their length is a multiple of 4 and the bases are 16-byte aligned
  const auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  const int tabn = mv.kind == SRC_LOWRANK ? mv.r : mv.kind == SRC_RBF ? mv.d : 0;
  const void* t0 = mv.kind == SRC_LOWRANK ? mv.pf : mv.x;
  const void* t1 = mv.kind == SRC_LOWRANK ? mv.qf : mv.y;
  const void* t2 = mv.kind == SRC_LOWRANK ? mv.s : mv.x;
  // vector runs need whole runs (lengths a multiple of 4) and 16-byte aligned bases
  const bool vec = kr % 4 == 0 && al16(CU) && al16(Rt) &&
                   (mv.kind == SRC_DENSE || mv.kind == SRC_CSR || (tabn % 4 == 0 && al16(t0) && al16(t1) && al16(t2)));
  int nb;
  if (ns > 0 && eb_use(mv.m, mv.n, ns)) {
    const EbPlan pl = eb_plan_for(mv, kr, ns);
    int32_t* counts = (int32_t*)ebws;
    int32_t* offs = (int32_t*)(ebws + al256e((size_t)pl.nbk * EB_G * 4));
    int32_t* totals = (int32_t*)((char*)offs + al256e((size_t)pl.nbk * EB_G * 4));
    int32_t* starts = (int32_t*)((char*)totals + al256e(((size_t)pl.nbk + 1) * 4));
    int2* ij = (int2*)((char*)starts + al256e(((size_t)pl.nbk + 1) * 4));
    int2* sorted = (int2*)((char*)ij + al256e((size_t)ns * 8));
    const unsigned gw = (unsigned)ceil_div(pl.nbk, 256);
    hipLaunchKernelGGL(eb_count_kernel, dim3(EB_G), dim3(256), 0, st, mv.m, mv.n, ns, seed, pl, ij, counts);
    hipLaunchKernelGGL(eb_totals_kernel, dim3(gw), dim3(256), 0, st, pl, counts, totals);
    hipLaunchKernelGGL(eb_scan_kernel, dim3(1), dim3(1024), 0, st, pl, totals, starts);
    hipLaunchKernelGGL(eb_offsets_kernel, dim3(gw), dim3(256), 0, st, pl, counts, starts, offs);
    hipLaunchKernelGGL(eb_scatter_kernel, dim3(EB_G), dim3(256), 0, st, ns, pl, ij, offs, sorted);
    if (er_rows_ok(mv, kr, ns)) {
      nb = pl.nbk;
      if (vec)
        hipLaunchKernelGGL((eb_eval_rows_kernel<TC, true>), dim3(nb), dim3(256), 0, st, mv, kr, CU, Rt, pl, starts,
                           sorted, part);
      else
        hipLaunchKernelGGL((eb_eval_rows_kernel<TC, false>), dim3(nb), dim3(256), 0, st, mv, kr, CU, Rt, pl, starts,
                           sorted, part);
    } else {
      nb = pl.nbk;
      with_src(mv.kind, vec, [&](auto src, auto vc) {
        hipLaunchKernelGGL((eb_eval_kernel<decltype(src)::value, TIn, TC, decltype(vc)::value>), dim3(nb), dim3(256), 0,
                           st, mv, kr, CU, Rt, starts, sorted, part);
      });
    }
  } else if (ns > 0) {
    nb = ERR_NB;
    with_src(mv.kind, vec, [&](auto src, auto vc) {
      hipLaunchKernelGGL((err_sampled_kernel<decltype(src)::value, TIn, TC, decltype(vc)::value>), dim3(nb), dim3(256),
                         0, st, mv, kr, CU, Rt, ns, seed, part);
    });
  } else if (mv.kind == SRC_CSR) {
    nb = (int)exact_nb(mv);
    hipLaunchKernelGGL((err_exact_csr_kernel<TIn>), dim3(nb), dim3(256), 0, st, mv, kr, CU, Rt64, part);
  } else {
    nb = (int)exact_nb(mv);
    hipLaunchKernelGGL((err_exact_kernel<TIn>), dim3(nb), dim3(256), 0, st, mv, kr, CU, Rt64, part);
  }
  hipLaunchKernelGGL(err_final_kernel, dim3(1), dim3(256), 0, st, nb, part, out3);
  return hipGetLastError();
}

hipError_t launch_error(const MatView& mv, int k2c, int k2r, int compute, const void* C, const double* Umid,
                        const void* Rt, int64_t n_samples, uint64_t seed, void* ws, double* out3, hipStream_t st) {
  if (mv.storage == P_F64 && compute != P_F64) return hipErrorInvalidValue;
  if (compute < P_F64 || compute > P_F16) return hipErrorInvalidValue;
  char* p = (char*)ws;
  double* CU = (double*)p;
  p += al256e((size_t)mv.m * k2r * sizeof(double));
  void* tws = p;
  p += tsgemm_ws_bytes(mv.m, k2c, k2r, P_F64);
  double* part = (double*)p;
  p += al256e((size_t)part_blocks(mv, k2r, n_samples) * 2 * sizeof(double));
  char* ebws = p;
  p += eb_ws_bytes(mv, k2r, n_samples);
  const double* C64 = (const double*)C;
  const double* Rt64 = (const double*)Rt;
  if (compute != P_F64) {
    double* c64 = (double*)p;
    p += al256e((size_t)mv.m * k2c * sizeof(double));
    widen_any(compute, (int64_t)mv.m * k2c, C, c64, st);
    C64 = c64;
    if (n_samples == 0) {
      double* r64 = (double*)p;
      widen_any(compute, (int64_t)mv.n * k2r, Rt, r64, st);
      Rt64 = r64;
    }
  }
  hipError_t e = launch_tsgemm(mv.m, k2c, k2r, P_F64, C64, Umid, CU, nullptr, nullptr, tws, st);
  if (e != hipSuccess) return e;
  if (mv.storage == P_F64)
    return error_t<double, double>(mv, k2r, CU, (const double*)Rt, Rt64, n_samples, seed, part, ebws, out3, st);
  switch (compute) {
    case P_F32: return error_t<float, float>(mv, k2r, CU, (const float*)Rt, Rt64, n_samples, seed, part, ebws, out3, st);
    case P_BF16: return error_t<float, bf16>(mv, k2r, CU, (const bf16*)Rt, Rt64, n_samples, seed, part, ebws, out3, st);
    case P_F16: return error_t<float, f16>(mv, k2r, CU, (const f16*)Rt, Rt64, n_samples, seed, part, ebws, out3, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cabs
