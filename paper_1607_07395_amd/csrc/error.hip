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

template <typename TIn, typename TC>
__global__ __launch_bounds__(256) void err_sampled_kernel(MatView mv, int kr, const double* __restrict__ CU,
                                                          const TC* __restrict__ Rt, int64_t ns, uint64_t seed,
                                                          double* __restrict__ part) {
  __shared__ double rn[16], rd[16];
  const int lane = threadIdx.x & 63;
  const int l16 = lane & 15;
  const int grp = threadIdx.x >> 4;            // 16 groups per block
  const int64_t ngroups = (int64_t)gridDim.x * 16;
  double num = 0.0, den = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * 16 + grp; t < ns; t += ngroups) {
    const u64x4 w = philox4x64((uint64_t)t, 0, STREAM_ERROR, 0, seed, 0);
    const int64_t i = (int64_t)mulhi_bound(w.v[0], (uint64_t)mv.m);
    const int64_t j = (int64_t)mulhi_bound(w.v[1], (uint64_t)mv.n);
    double ap = 0.0;
    const double* cu = CU + i * kr;
    const TC* rt = Rt + j * kr;
    for (int a = l16; a < kr; a += 16) ap += cu[a] * to_f64(rt[a]);
    ap += __shfl_xor(ap, 1, 64);
    ap += __shfl_xor(ap, 2, 64);
    ap += __shfl_xor(ap, 4, 64);
    ap += __shfl_xor(ap, 8, 64);
    const double a = entry_f64<TIn>(mv, i, j, l16);
    if (l16 == 0) { num += (a - ap) * (a - ap); den += a * a; }
  }
  // fixed-order block reduction: lanes -> waves -> block
  num = wave_sum(num);
  den = wave_sum(den);
  if (lane == 0) { rn[threadIdx.x >> 6] = num; rd[threadIdx.x >> 6] = den; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ((rn[0] + rn[1]) + rn[2]) + rn[3];
    part[2 * blockIdx.x + 1] = ((rd[0] + rd[1]) + rd[2]) + rd[3];
  }
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

__global__ void err_final_kernel(int nb, const double* __restrict__ part, double* __restrict__ out3) {
  if (threadIdx.x != 0) return;
  double n = 0.0, d = 0.0;
  for (int b = 0; b < nb; ++b) { n += part[2 * b]; d += part[2 * b + 1]; }
  out3[0] = n;
  out3[1] = d;
  out3[2] = d > 0.0 ? sqrt(n / d) : 0.0;
}

static inline int64_t exact_nb(const MatView& mv) { return ceil_div(mv.m, 64); }

size_t error_ws_bytes(const MatView& mv, int k2c, int k2r, int compute, int64_t n_samples) {
  const int64_t nb = n_samples > 0 ? ERR_NB : exact_nb(mv);
  size_t b = al256e((size_t)mv.m * k2r * sizeof(double)) + tsgemm_ws_bytes(mv.m, k2c, k2r, P_F64) +
             al256e((size_t)nb * 2 * sizeof(double)) + 256;
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
                          uint64_t seed, double* part, double* out3, hipStream_t st) {
  TimerScope ts(T_ERROR, st);
  int nb;
  if (ns > 0) {
    nb = ERR_NB;
    hipLaunchKernelGGL((err_sampled_kernel<TIn, TC>), dim3(nb), dim3(256), 0, st, mv, kr, CU, Rt, ns, seed, part);
  } else {
    nb = (int)exact_nb(mv);
    hipLaunchKernelGGL((err_exact_kernel<TIn>), dim3(nb), dim3(256), 0, st, mv, kr, CU, Rt64, part);
  }
  hipLaunchKernelGGL(err_final_kernel, dim3(1), dim3(64), 0, st, nb, part, out3);
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
  p += al256e((size_t)(n_samples > 0 ? ERR_NB : exact_nb(mv)) * 2 * sizeof(double));
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
    return error_t<double, double>(mv, k2r, CU, (const double*)Rt, Rt64, n_samples, seed, part, out3, st);
  switch (compute) {
    case P_F32: return error_t<float, float>(mv, k2r, CU, (const float*)Rt, Rt64, n_samples, seed, part, out3, st);
    case P_BF16: return error_t<float, bf16>(mv, k2r, CU, (const bf16*)Rt, Rt64, n_samples, seed, part, out3, st);
    case P_F16: return error_t<float, f16>(mv, k2r, CU, (const f16*)Rt, Rt64, n_samples, seed, part, out3, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cabs
