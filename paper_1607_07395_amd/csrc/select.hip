// Hard-threshold follow-up selection (the variant of Section 5): the k rows
// with the largest weights Upsilon(|P_l|), equal weights to the lower row
// index, NaN weights after every number, returned in ascending row order.
//
// A bitonic sort of (weight, row) pairs, padded to a power of two n2 >= 2048
// with (-inf, INT32_MAX) entries that order after every row: chunks of 2048
// pairs are sorted in LDS, each merge level runs its strides >= 2048 as global
// compare-exchange passes and the rest in LDS.  The first k pairs of the
// result are the selection; one work-group sorts their rows ascending.  Every
// step is a fixed network, so the result does not depend on scheduling.
#include "common.hpp"
#include "kernels.hpp"

namespace cabs {

namespace {

constexpr int SEL_CH = 2048;  // pairs per LDS chunk: 1024 threads, one compare-exchange each

// (wa, ia) orders before (wb, ib): the larger weight, then the lower row.
__device__ __forceinline__ bool sel_before(double wa, int32_t ia, double wb, int32_t ib) {
  return wa > wb || (wa == wb && ia < ib);
}

__global__ __launch_bounds__(256) void sel_init_kernel(int64_t rows, int64_t n2, const double* __restrict__ w,
                                                       double* __restrict__ kw, int32_t* __restrict__ ki) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n2) return;
  double v = -__builtin_huge_val();
  if (i < rows) {
    const double x = w[i];
    v = x == x ? x : -__builtin_huge_val();
  }
  kw[i] = v;
  ki[i] = i < rows ? (int32_t)i : INT32_MAX;
}

// One compare-exchange of the bitonic network: positions p < q = p + j, in
// ascending 'before' order when bit k of p is clear, descending otherwise.
__device__ __forceinline__ void sel_cx(double& wp, int32_t& ip, double& wq, int32_t& iq, bool up) {
  const bool swap = up ? sel_before(wq, iq, wp, ip) : sel_before(wp, ip, wq, iq);
  if (swap) {
    const double tw = wp;
    const int32_t ti = ip;
    wp = wq; ip = iq;
    wq = tw; iq = ti;
  }
}

// kmerge == 0: sort each chunk completely (levels 2 .. SEL_CH); otherwise the
// strides SEL_CH / 2 .. 1 of merge level kmerge.  The direction of a pair
// comes from its global position, so neighbouring chunks alternate as the
// next level needs.
__global__ __launch_bounds__(1024) void sel_local_kernel(double* __restrict__ kw, int32_t* __restrict__ ki,
                                                         int64_t kmerge) {
  __shared__ double sw[SEL_CH];
  __shared__ int32_t si[SEL_CH];
  const int64_t base = (int64_t)blockIdx.x * SEL_CH;
  const int t = threadIdx.x;
  for (int e = t; e < SEL_CH; e += 1024) {
    sw[e] = kw[base + e];
    si[e] = ki[base + e];
  }
  __syncthreads();
  auto step = [&](int64_t k, int j) {
    const int p = (t / j) * 2 * j + (t % j), q = p + j;
    double wp = sw[p], wq = sw[q];
    int32_t ip = si[p], iq = si[q];
    sel_cx(wp, ip, wq, iq, ((base + p) & k) == 0);
    sw[p] = wp; si[p] = ip;
    sw[q] = wq; si[q] = iq;
    __syncthreads();
  };
  if (kmerge == 0) {
    for (int k = 2; k <= SEL_CH; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) step(k, j);
  } else {
    for (int j = SEL_CH / 2; j > 0; j >>= 1) step(kmerge, j);
  }
  for (int e = t; e < SEL_CH; e += 1024) {
    kw[base + e] = sw[e];
    ki[base + e] = si[e];
  }
}

// Stride j >= SEL_CH of merge level k over all n2 / 2 pairs.
__global__ __launch_bounds__(256) void sel_global_kernel(double* __restrict__ kw, int32_t* __restrict__ ki, int64_t n2,
                                                         int64_t k, int64_t j) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n2 / 2) return;
  const int64_t p = (t / j) * 2 * j + (t % j), q = p + j;
  double wp = kw[p], wq = kw[q];
  int32_t ip = ki[p], iq = ki[q];
  sel_cx(wp, ip, wq, iq, (p & k) == 0);
  kw[p] = wp; ki[p] = ip;
  kw[q] = wq; ki[q] = iq;
}

// The rows of the first k pairs (k <= 1024), sorted ascending.
__global__ __launch_bounds__(1024) void sel_out_kernel(const int32_t* __restrict__ ki, int k, int64_t* __restrict__ out) {
  __shared__ int32_t s[1024];
  const int t = threadIdx.x;
  s[t] = t < k ? ki[t] : INT32_MAX;
  __syncthreads();
  for (int kk = 2; kk <= 1024; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      const int l = t ^ j;
      if (l > t) {
        const int32_t a = s[t], b = s[l];
        if (((t & kk) == 0) ? a > b : a < b) {
          s[t] = b;
          s[l] = a;
        }
      }
      __syncthreads();
    }
  if (t < k) out[t] = s[t];
}

int64_t sel_n2(int64_t rows) {
  int64_t n2 = SEL_CH;
  while (n2 < rows) n2 <<= 1;
  return n2;
}

}  // namespace

size_t select_ws_bytes(int64_t rows) {
  const int64_t n2 = sel_n2(rows);
  return (size_t)n2 * sizeof(double) + (size_t)n2 * sizeof(int32_t) + 256;
}

hipError_t launch_select_topk(int64_t rows, const double* w, int k, int64_t* out, void* ws, hipStream_t st) {
  if (rows <= 0 || rows >= INT32_MAX || k < 1 || k > 1024 || k > rows) return hipErrorInvalidValue;
  const int64_t n2 = sel_n2(rows);
  double* kw = (double*)ws;
  int32_t* ki = (int32_t*)(kw + n2);
  hipLaunchKernelGGL(sel_init_kernel, dim3((unsigned)ceil_div(n2, 256)), dim3(256), 0, st, rows, n2, w, kw, ki);
  const unsigned chunks = (unsigned)(n2 / SEL_CH);
  hipLaunchKernelGGL(sel_local_kernel, dim3(chunks), dim3(1024), 0, st, kw, ki, (int64_t)0);
  for (int64_t k2 = 2 * SEL_CH; k2 <= n2; k2 <<= 1) {
    for (int64_t j = k2 >> 1; j >= SEL_CH; j >>= 1)
      hipLaunchKernelGGL(sel_global_kernel, dim3((unsigned)ceil_div(n2 / 2, 256)), dim3(256), 0, st, kw, ki, n2, k2,
                         j);
    hipLaunchKernelGGL(sel_local_kernel, dim3(chunks), dim3(1024), 0, st, kw, ki, k2);
  }
  hipLaunchKernelGGL(sel_out_kernel, dim3(1), dim3(1024), 0, st, ki, k, out);
  return hipGetLastError();
}

}  // namespace cabs
