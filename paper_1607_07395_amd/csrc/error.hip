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

__device__ __forceinline__ void err_sample_ij(uint64_t t, uint64_t seed, int64_t m, int64_t n, int64_t& i, int64_t& j) {
  const u64x4 w = philox4x64(t, 0, STREAM_ERROR, 0, seed, 0);
  i = (int64_t)mulhi_bound(w.v[0], (uint64_t)m);
  j = (int64_t)mulhi_bound(w.v[1], (uint64_t)n);
}

// Sixteen zero bytes to point out-of-range loads at, so that loads need no branches.
__device__ const double4 kZeroRun = {0.0, 0.0, 0.0, 0.0};

// Four consecutive elements p[e .. e+3] widened to FP64, zero from `lim` on.
// VEC: len is a multiple of 4 and rows are 16-byte aligned, so a run is either
// whole (one 16-byte load, two for FP64) or entirely past the end, in which
// case it reads the zero run.  Otherwise element loads, each past-the-end
// element also redirected to the zero run.  No branches either way, so every
// run of a row is in flight at once.
template <typename T, bool VEC> struct Run4;
template <> struct Run4<float, true> {
  __device__ static __forceinline__ void get(const float* p, int e, int lim, double (&o)[4]) {
    const float4 v = *(const float4*)(e < lim ? p + e : (const float*)&kZeroRun);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
template <> struct Run4<double, true> {
  __device__ static __forceinline__ void get(const double* p, int e, int lim, double (&o)[4]) {
    const double* q = e < lim ? p + e : (const double*)&kZeroRun;
    const double2 a = *(const double2*)q, b = *(const double2*)(q + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
  }
};
template <typename T> struct Run4<T, true> {  // 16-bit types: one 8-byte load
  static_assert(sizeof(T) == 2, "16-bit element type expected");
  __device__ static __forceinline__ void get(const T* p, int e, int lim, double (&o)[4]) {
    const uint2 v = *(const uint2*)(e < lim ? p + e : (const T*)&kZeroRun);
    const T* h = (const T*)&v;
#pragma unroll
    for (int w = 0; w < 4; ++w) o[w] = to_f64(h[w]);
  }
};
template <typename T> struct Run4<T, false> {
  __device__ static __forceinline__ void get(const T* p, int e, int lim, double (&o)[4]) {
#pragma unroll
    for (int w = 0; w < 4; ++w) o[w] = to_f64(*(e + w < lim ? p + e + w : (const T*)&kZeroRun));
  }
};

// sum over e < len of f(x[e], y[e]) by a 16-lane group: lane l16 takes the runs
// starting at 4 l16 + 64 u; four runs (256 elements) of each operand are in flight.
template <int KIND, bool VEC, typename TX, typename TY>
__device__ __forceinline__ double group_dot(const TX* x, const TY* y, const TY* z, int len, int l16) {
  double acc = 0.0;
  for (int u0 = 0; u0 < len; u0 += 256) {
    double a[4][4], b[4][4], c[4][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int e = u0 + 64 * v + 4 * l16;
      Run4<TX, VEC>::get(x, e, len, a[v]);
      Run4<TY, VEC>::get(y, e, len, b[v]);
      if (KIND == 1) Run4<TY, VEC>::get(z, e, len, c[v]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        if (KIND == 0) acc += a[v][w] * b[v][w];                      // plain dot
        else if (KIND == 1) acc += a[v][w] * c[v][w] * b[v][w];       // x . diag(z) . y
        else { const double df = a[v][w] - b[v][w]; acc += df * df; }  // squared distance
      }
  }
  return acc;
}

// One sample per lane (t, when `valid`).  The per-sample scalar work (sample
// indices, the noise of a low-rank entry, the RBF exponential, the residual)
// runs once per lane; the two long dot products of each sample run on the
// lane's 16-lane group, which works through its 16 lanes' samples in order,
// and the owning lane keeps the reduced values.  vec: rows of CU, Rt and the
// tables may be read as 16-byte runs (decided on the host from sizes and
// pointer alignment).
template <typename TIn, typename TC, bool VEC>
__device__ __forceinline__ void err_batch(const MatView& mv, int kr, const double* __restrict__ CU,
                                          const TC* __restrict__ Rt, uint64_t seed, int64_t t, bool valid,
                                          double& num, double& den) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, base = lane & 48;
  int64_t i = 0, j = 0;
  double nz = 0.0;
  if (valid) {
    err_sample_ij((uint64_t)t, seed, mv.m, mv.n, i, j);
    if (mv.kind == SRC_LOWRANK && mv.noise_std != 0.0) nz = noise_f64(mv.noise_seed, (uint64_t)i, (uint64_t)j);
  }
  double my_ap = 0.0, my_s = 0.0;
  for (int q = 0; q < 16; ++q) {
    const int64_t ii = __shfl(i, base + q, 64);
    const int64_t jj = __shfl(j, base + q, 64);
    double ap = group_dot<0, VEC, double, TC>(CU + ii * kr, Rt + jj * kr, nullptr, kr, l16);
    double sv = 0.0;
    if (mv.kind == SRC_DENSE) {
      sv = l16 == 0 ? (double)((const TIn*)mv.a)[ii * mv.lda + jj] : 0.0;
    } else if (mv.kind == SRC_LOWRANK) {
      sv = group_dot<1, VEC, TIn, TIn>((const TIn*)mv.pf + ii * mv.r, (const TIn*)mv.qf + jj * mv.r, (const TIn*)mv.s,
                                       mv.r, l16);
    } else {
      sv = group_dot<2, VEC, TIn, TIn>((const TIn*)mv.x + ii * mv.d, (const TIn*)mv.y + jj * mv.d, nullptr, mv.d, l16);
    }
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      ap += __shfl_xor(ap, off, 64);
      sv += __shfl_xor(sv, off, 64);
    }
    if (l16 == q) { my_ap = ap; my_s = sv; }
  }
  if (valid) {
    double a = my_s;
    if (mv.kind == SRC_LOWRANK) a += mv.noise_std * nz;
    else if (mv.kind == SRC_RBF) a = exp(-my_s / (2.0 * mv.sigma * mv.sigma));
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
template <typename TIn, typename TC, bool VEC>
__global__ __launch_bounds__(256) void err_sampled_kernel(MatView mv, int kr, const double* __restrict__ CU,
                                                          const TC* __restrict__ Rt, int64_t ns, uint64_t seed,
                                                          double* __restrict__ part) {
  double num = 0.0, den = 0.0;
  for (int64_t b0 = (int64_t)blockIdx.x * 256; b0 < ns; b0 += (int64_t)gridDim.x * 256) {
    const int64_t t = b0 + threadIdx.x;
    err_batch<TIn, TC, VEC>(mv, kr, CU, Rt, seed, t, t < ns, num, den);
  }
  err_block_store(num, den, part, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Sampled error with the samples grouped by row bucket.  Each bucket (RB
// consecutive rows) is one work-group, so the row-side data of a sample (the
// generator row and the FP64 row of CU) comes from cache after its first use
// and only the column side is gathered per sample.  The grouping is a stable
// counting sort of the sample numbers t (bucket-major, then chunk, then t), so
// every sum is taken in a fixed order.
// ---------------------------------------------------------------------------
constexpr int EB_MAXB = 8192;   // buckets at most
constexpr int EB_G = 512;       // sample chunks of the counting sort

struct EbPlan { int64_t rb; int nbk; int64_t tchunk; };

static inline EbPlan eb_plan(int64_t m, int64_t ns) {
  EbPlan p;
  p.rb = ceil_div(m, EB_MAXB);
  p.nbk = (int)ceil_div(m, p.rb);
  p.tchunk = ceil_div(ns, EB_G);
  return p;
}

// The sorted path needs n_s < 2^31 (sample numbers kept as int32) and at least
// one sample per row on average (else there is nothing to reuse).
static inline bool eb_use(int64_t m, int64_t ns) { return ns >= m && ns < ((int64_t)1 << 31); }


__global__ __launch_bounds__(256) void eb_count_kernel(int64_t m, int64_t n, int64_t ns, uint64_t seed, EbPlan pl,
                                                       int32_t* __restrict__ counts) {
  __shared__ int32_t hist[EB_MAXB];
  for (int b = threadIdx.x; b < pl.nbk; b += 256) hist[b] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * pl.tchunk;
  const int64_t t1 = t0 + pl.tchunk < ns ? t0 + pl.tchunk : ns;
  for (int64_t t = t0 + threadIdx.x; t < t1; t += 256) {
    int64_t i, j;
    err_sample_ij((uint64_t)t, seed, m, n, i, j);
    atomicAdd(&hist[(int)(i / pl.rb)], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < pl.nbk; b += 256) counts[(int64_t)b * EB_G + blockIdx.x] = hist[b];
}

// Per bucket (one wave each): the total over chunks.
__global__ __launch_bounds__(256) void eb_totals_kernel(EbPlan pl, const int32_t* __restrict__ counts,
                                                        int32_t* __restrict__ totals) {
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (b >= pl.nbk) return;
  int s = 0;
  for (int g = lane; g < EB_G; g += 64) s += counts[(int64_t)b * EB_G + g];
  s = wave_sum(s);
  if (lane == 0) totals[b] = s;
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

// Per bucket (one wave each): offsets of each chunk's run inside the bucket.
__global__ __launch_bounds__(256) void eb_offsets_kernel(EbPlan pl, const int32_t* __restrict__ counts,
                                                         const int32_t* __restrict__ starts,
                                                         int32_t* __restrict__ offs) {
  constexpr int PER = EB_G / 64;
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (b >= pl.nbk) return;
  const int32_t* c = counts + (int64_t)b * EB_G + lane * PER;
  int v[PER], sum = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) { v[q] = c[q]; sum += v[q]; }
  int incl = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int x = __shfl_up(incl, off, 64);
    if (lane >= off) incl += x;
  }
  int run = starts[b] + incl - sum;
  int32_t* o = offs + (int64_t)b * EB_G + lane * PER;
#pragma unroll
  for (int q = 0; q < PER; ++q) { o[q] = run; run += v[q]; }
}

// Chunk g places its sample numbers, in increasing t within each bucket.  A
// round is 256 consecutive samples, 64 per wave; ranks among equal buckets
// inside a wave come from shuffles, and the four waves place their samples in
// wave order, each advancing the per-bucket run counters in LDS.
__global__ __launch_bounds__(256) void eb_scatter_kernel(int64_t m, int64_t n, int64_t ns, uint64_t seed, EbPlan pl,
                                                         const int32_t* __restrict__ offs,
                                                         int32_t* __restrict__ sorted) {
  __shared__ int32_t run[EB_MAXB];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int b = tid; b < pl.nbk; b += 256) run[b] = 0;
  const int64_t t0 = (int64_t)blockIdx.x * pl.tchunk;
  const int64_t t1 = t0 + pl.tchunk < ns ? t0 + pl.tchunk : ns;
  for (int64_t base = t0; base < t1; base += 256) {
    const int64_t t = base + tid;
    const bool valid = t < t1;
    int b = -1;
    if (valid) {
      int64_t i, j;
      err_sample_ij((uint64_t)t, seed, m, n, i, j);
      b = (int)(i / pl.rb);
    }
    int rank = 0;
    bool last = true;
    for (int q = 0; q < 64; ++q) {
      const int o = __shfl(b, q, 64);
      rank += (q < lane) & (o == b);
      last = last && !((q > lane) & (o == b));
    }
    for (int w = 0; w < 4; ++w) {
      __syncthreads();
      if (wave == w && valid) {
        sorted[offs[(int64_t)b * EB_G + blockIdx.x] + run[b] + rank] = (int32_t)t;
        if (last) run[b] += rank + 1;
      }
    }
  }
}

// One work-group per bucket, in batches of 256 of the bucket's samples.
template <typename TIn, typename TC, bool VEC>
__global__ __launch_bounds__(256) void eb_eval_kernel(MatView mv, int kr, const double* __restrict__ CU,
                                                      const TC* __restrict__ Rt, uint64_t seed,
                                                      const int32_t* __restrict__ starts,
                                                      const int32_t* __restrict__ sorted,
                                                      double* __restrict__ part) {
  const int b = blockIdx.x;
  const int s0 = starts[b], s1 = starts[b + 1];
  double num = 0.0, den = 0.0;
  for (int b0 = s0; b0 < s1; b0 += 256) {
    const int s = b0 + (int)threadIdx.x;
    const bool valid = s < s1;
    err_batch<TIn, TC, VEC>(mv, kr, CU, Rt, seed, valid ? (int64_t)sorted[s] : 0, valid, num, den);
  }
  err_block_store(num, den, part, b);
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

static inline int64_t part_blocks(const MatView& mv, int64_t ns) {
  if (ns == 0) return exact_nb(mv);
  return eb_use(mv.m, ns) ? eb_plan(mv.m, ns).nbk : ERR_NB;
}

static inline size_t eb_ws_bytes(const MatView& mv, int64_t ns) {
  if (ns == 0 || !eb_use(mv.m, ns)) return 0;
  const EbPlan pl = eb_plan(mv.m, ns);
  return 2 * al256e((size_t)pl.nbk * EB_G * 4) + 2 * al256e(((size_t)pl.nbk + 1) * 4) + al256e((size_t)ns * 4);
}

size_t error_ws_bytes(const MatView& mv, int k2c, int k2r, int compute, int64_t n_samples) {
  const int64_t nb = part_blocks(mv, n_samples);
  size_t b = al256e((size_t)mv.m * k2r * sizeof(double)) + tsgemm_ws_bytes(mv.m, k2c, k2r, P_F64) +
             al256e((size_t)nb * 2 * sizeof(double)) + eb_ws_bytes(mv, n_samples) + 256;
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
                   (mv.kind == SRC_DENSE || (tabn % 4 == 0 && al16(t0) && al16(t1) && al16(t2)));
  int nb;
  if (ns > 0 && eb_use(mv.m, ns)) {
    const EbPlan pl = eb_plan(mv.m, ns);
    int32_t* counts = (int32_t*)ebws;
    int32_t* offs = (int32_t*)(ebws + al256e((size_t)pl.nbk * EB_G * 4));
    int32_t* totals = (int32_t*)((char*)offs + al256e((size_t)pl.nbk * EB_G * 4));
    int32_t* starts = (int32_t*)((char*)totals + al256e(((size_t)pl.nbk + 1) * 4));
    int32_t* sorted = (int32_t*)((char*)starts + al256e(((size_t)pl.nbk + 1) * 4));
    const unsigned gw = (unsigned)ceil_div(pl.nbk, 4);
    hipLaunchKernelGGL(eb_count_kernel, dim3(EB_G), dim3(256), 0, st, mv.m, mv.n, ns, seed, pl, counts);
    hipLaunchKernelGGL(eb_totals_kernel, dim3(gw), dim3(256), 0, st, pl, counts, totals);
    hipLaunchKernelGGL(eb_scan_kernel, dim3(1), dim3(1024), 0, st, pl, totals, starts);
    hipLaunchKernelGGL(eb_offsets_kernel, dim3(gw), dim3(256), 0, st, pl, counts, starts, offs);
    hipLaunchKernelGGL(eb_scatter_kernel, dim3(EB_G), dim3(256), 0, st, mv.m, mv.n, ns, seed, pl, offs, sorted);
    nb = pl.nbk;
    if (vec)
      hipLaunchKernelGGL((eb_eval_kernel<TIn, TC, true>), dim3(nb), dim3(256), 0, st, mv, kr, CU, Rt, seed, starts,
                         sorted, part);
    else
      hipLaunchKernelGGL((eb_eval_kernel<TIn, TC, false>), dim3(nb), dim3(256), 0, st, mv, kr, CU, Rt, seed, starts,
                         sorted, part);
  } else if (ns > 0) {
    nb = ERR_NB;
    if (vec)
      hipLaunchKernelGGL((err_sampled_kernel<TIn, TC, true>), dim3(nb), dim3(256), 0, st, mv, kr, CU, Rt, ns, seed, part);
    else
      hipLaunchKernelGGL((err_sampled_kernel<TIn, TC, false>), dim3(nb), dim3(256), 0, st, mv, kr, CU, Rt, ns, seed,
                         part);
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
  p += al256e((size_t)part_blocks(mv, n_samples) * 2 * sizeof(double));
  char* ebws = p;
  p += eb_ws_bytes(mv, n_samples);
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
