// libcabs host runtime: argument checking, workspace planning and the stage
// sequence of one CABS sketch (Algorithm 2), behind the C ABI of cabs.h.
//
// Stage order of cabs_sketch (all enqueued on the caller's stream, no host
// synchronisation):
//   1  pilot indices I^r, I^c (Floyd on Philox streams 0 / 1)
//   2  C = A(:, I^c), R^T = A(I^r, :)^T; W = C(I^r, :) in FP64
//   3  SVD W = U_w S_w V_w^T (FP64 Jacobi)
//   4  C^ = C V_w, R^ = R^T U_w with FP64 column norms N_c, N_r; kept components,
//      S (stabilised: S_w sqrt(mn/(kr kc)); pseudo-skeleton: N_c N_r / S_w)
//   5  orthogonalisation (supplementary Section 3) in FP64: Grams of C^ N_c^-1 and
//      R^ N_r^-1, their pivoted Cholesky factors R_u, R_v, the SVD of
//      K = R_u S R_v^T; the embedding maps M_u, M_v (k x k) such that
//      P = C^ M_u, Q = R^ M_v hold U_o S_o^(1/2) and V_o S_o^(1/2)
//   6  P, Q with row norms -> weights Upsilon(|P_l|)
//   7  weighted k-means + snapping on P (rows) and Q (columns)
//   8  C_bar, R_bar^T, W_bar; SVD; norms; Umid = V_w diag(S / (N_c N_r)) U_w^T
//   9  optional factor form (Uf, S, Vf) by the same orthogonalisation
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cabs.h"
#include "common.hpp"
#include "group.hpp"
#include "kernels.hpp"

using namespace cabs;

// ---------------------------------------------------------------------------
// Error reporting
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static cabs_status fail(cabs_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return fail(CABS_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

extern "C" const char* cabs_last_error(void) { return g_last_error.c_str(); }

void cabs::set_last_error(const char* msg) { g_last_error = msg; }
extern "C" const char* cabs_version(void) { return "libcabs 0.1 (gfx950)"; }

// ---------------------------------------------------------------------------
// Small device kernels for the k x k bookkeeping
// ---------------------------------------------------------------------------
namespace {

// Kept components and the scalings of the sketching routine (Section 4.1).
__global__ void sketch_vec_kernel(int p, int kr, int kc, double m, double n, const double* __restrict__ sw,
                                  const double* __restrict__ nc2, const double* __restrict__ nr2, double rtol, int kind,
                                  double* __restrict__ invc, double* __restrict__ invr, double* __restrict__ sk,
                                  double* __restrict__ dk, double* __restrict__ diag, int diag_rank, int diag_sig) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  const double s1 = sw[0];
  const double tol = (rtol > 0.0 ? rtol : (double)(kr > kc ? kr : kc) * eps) * s1;
  const double scale = sqrt(m * n / ((double)kr * (double)kc));
  for (int i = threadIdx.x; i < p; i += blockDim.x) {
    const double nc = sqrt(nc2[i]), nr = sqrt(nr2[i]), s = sw[i];
    const bool keep = s1 > 0.0 && s > tol && nc > 0.0 && nr > 0.0;
    double S = 0.0, D = 0.0;
    if (keep) {
      if (kind == CABS_SK_STABILIZED) { S = s * scale; D = S / (nc * nr); }
      else { S = nc * nr / s; D = 1.0 / s; }
      atomicAdd(&cnt, 1);
    }
    invc[i] = keep ? 1.0 / nc : 0.0;
    invr[i] = keep ? 1.0 / nr : 0.0;
    sk[i] = S;
    dk[i] = D;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    diag[diag_rank] = (double)cnt;
    diag[diag_sig] = s1;
    if (cnt == 0) diag[CABS_DIAG_STATUS] = (double)CABS_ERANK;
  }
}

// out[i][j] = dl[i] * G[i][j] * dr[j]   (batched: item b uses G + b*p*p)
__global__ void scale2_kernel(int p, const double* __restrict__ G, const double* __restrict__ dl,
                              const double* __restrict__ dr, double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p * p) return;
  const int i = e / p, j = e % p;
  out[e] = dl[i] * G[e] * dr[j];
}

// w[j] = s[j]^(-1/2) for s[j] > p eps s[0] (s descending), else 0
__global__ void rsqrt_trunc_kernel(int p, const double* __restrict__ s, double* __restrict__ w) {
  const double eps = 2.220446049250313e-16;
  const double smax = s[0];
  for (int j = threadIdx.x; j < p; j += blockDim.x) {
    const bool keep = smax > 0.0 && s[j] > (double)p * eps * smax;
    w[j] = keep ? 1.0 / sqrt(s[j]) : 0.0;
  }
}

// out[j] = a[j] b[j]
__global__ void mul_vec_kernel(int p, const double* __restrict__ a, const double* __restrict__ b,
                               double* __restrict__ out) {
  for (int j = threadIdx.x; j < p; j += blockDim.x) out[j] = a[j] * b[j];
}

// B = diag(v) as a dense p x p matrix.
__global__ void diag_mat_kernel(int p, const double* __restrict__ a, const double* __restrict__ b,
                                double* __restrict__ B) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p * p) return;
  const int i = e / p, j = e % p;
  B[e] = i == j ? a[i] * (b ? (b[i] > 0.0 ? sqrt(b[i]) : 0.0) : 1.0) : 0.0;
}

// B (rows x cols) copied into Bp (rows x ldp), columns cols .. ldp - 1 zero.
__global__ void pad_cols_kernel(int rows, int cols, int ldp, const double* __restrict__ B, double* __restrict__ Bp) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * ldp) return;
  const int i = e / ldp, j = e % ldp;
  Bp[e] = j < cols ? B[(int64_t)i * cols + j] : 0.0;
}

// Weights Upsilon(|P_l|) from squared row norms (Section 3.2).
__global__ void weights_kernel(int64_t rows, const double* __restrict__ rowsq, int kind, double prm,
                               double* __restrict__ w) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const double x = sqrt(rowsq[r]);
  double v = 1.0;
  if (kind == CABS_W_POW) v = pow(x, prm);
  else if (kind == CABS_W_SIGMOID) v = 1.0 / (1.0 + exp(-prm * x));
  else if (kind == CABS_W_STEP) v = x >= prm ? 1.0 : 0.0;
  w[r] = v;
}

// Reciprocals of the embedding's singular values over the kept components
// (> p eps max), zero for the others, so that sum_t P_lt^2 inv_t is the
// squared row norm of the factor behind P = U' diag(s)^(1/2).
__global__ void lev_inv_kernel(int p, const double* __restrict__ s, double* __restrict__ inv) {
  __shared__ double smax;
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int t = 0; t < p; ++t) m = s[t] > m ? s[t] : m;
    smax = m;
  }
  __syncthreads();
  const double cut = (double)p * 2.220446049250313e-16 * smax;
  for (int t = threadIdx.x; t < p; t += blockDim.x) inv[t] = (smax > 0.0 && s[t] > cut) ? 1.0 / s[t] : 0.0;
}

// Leverage-variant keys (Section 5): score_l = sum_t P_lt^2 inv_t (FP64, one
// wave per row, lane-strided partial sums then a fixed butterfly), key_l =
// ln(u_l) / score_l with u_l in (0, 1] from Philox-4x64-10 at counter
// (l, 0, stream, 0), key (seed, 0); -inf for a zero score.  The selection of
// the k largest keys is the hard-threshold selection.
template <typename TC>
__global__ __launch_bounds__(256) void lev_keys_kernel(int64_t rows, int ld, int e, const TC* __restrict__ P,
                                                       const double* __restrict__ inv, uint64_t seed, uint64_t stream,
                                                       double* __restrict__ key) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  double s = 0.0;
  for (int t = lane; t < e; t += 64) {
    const double v = to_f64(P[row * ld + t]);
    s += v * v * inv[t];
  }
  s = wave_sum(s);
  if (lane == 0) {
    const u64x4 w = philox4x64((uint64_t)row, 0, stream, 0, seed, 0);
    const double u = unit_open0(w.v[0]);
    key[row] = s > 0.0 ? log(u) / s : -__builtin_huge_val();
  }
}

template <typename TC>
static void launch_lev_keys(int64_t rows, int ld, int e, const void* P, const double* inv, uint64_t seed,
                            uint64_t stream, double* key, hipStream_t st) {
  hipLaunchKernelGGL(lev_keys_kernel<TC>, dim3((unsigned)ceil_div(rows, 4)), dim3(256), 0, st, rows, ld, e,
                     (const TC*)P, inv, seed, stream, key);
}

static hipError_t launch_lev_keys_any(int prec, int64_t rows, int ld, int e, const void* P, const double* inv,
                                      uint64_t seed, uint64_t stream, double* key, hipStream_t st) {
  switch (prec) {
    case CABS_F64: launch_lev_keys<double>(rows, ld, e, P, inv, seed, stream, key, st); break;
    case CABS_F32: launch_lev_keys<float>(rows, ld, e, P, inv, seed, stream, key, st); break;
    case CABS_BF16: launch_lev_keys<bf16>(rows, ld, e, P, inv, seed, stream, key, st); break;
    case CABS_F16: launch_lev_keys<f16>(rows, ld, e, P, inv, seed, stream, key, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ void diag_init_kernel(double* __restrict__ diag, unsigned long long* __restrict__ counter, int counted) {
  const int i = threadIdx.x;
  if (i < CABS_DIAG_LEN) diag[i] = i == CABS_DIAG_ENTRIES ? (counted ? 0.0 : -1.0) : 0.0;
  if (i == 0) *counter = 0ull;
}

__global__ void entries_out_kernel(const unsigned long long* __restrict__ counter, double* __restrict__ diag) {
  if (threadIdx.x == 0) diag[CABS_DIAG_ENTRIES] = (double)*counter;
}

__global__ void copy_slot_kernel(const double* __restrict__ src, double* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}

__global__ void copy_vec_kernel(int n, const double* __restrict__ src, double* __restrict__ dst) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// Sign of every column of U (rows x p): the entry of largest magnitude, first on ties.
__global__ void colsign_partial_kernel(int64_t rows, int p, int64_t rows_per, const void* __restrict__ U, int prec,
                                       double* __restrict__ pmax, int64_t* __restrict__ pidx,
                                       double* __restrict__ psgn) {
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= p) return;
  const int64_t r0 = blockIdx.x * rows_per;
  const int64_t r1 = r0 + rows_per < rows ? r0 + rows_per : rows;
  double best = -1.0, sg = 1.0;
  int64_t bi = INT64_MAX;
  for (int64_t r = r0; r < r1; ++r) {
    double v;
    switch (prec) {
      case P_F64: v = ((const double*)U)[r * p + j]; break;
      case P_F32: v = ((const float*)U)[r * p + j]; break;
      case P_BF16: v = (double)(float)((const bf16*)U)[r * p + j]; break;
      default: v = (double)(float)((const f16*)U)[r * p + j]; break;
    }
    if (fabs(v) > best) { best = fabs(v); bi = r; sg = v < 0.0 ? -1.0 : 1.0; }
  }
  const int64_t o = (int64_t)blockIdx.x * p + j;
  pmax[o] = best;
  pidx[o] = bi;
  psgn[o] = sg;
}

__global__ void colsign_final_kernel(int nb, int p, const double* __restrict__ pmax, const int64_t* __restrict__ pidx,
                                     const double* __restrict__ psgn, double* __restrict__ sgn) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= p) return;
  double best = -1.0, sg = 1.0;
  int64_t bi = INT64_MAX;
  for (int b = 0; b < nb; ++b) {
    const int64_t o = (int64_t)b * p + j;
    if (pmax[o] > best || (pmax[o] == best && pidx[o] < bi)) { best = pmax[o]; bi = pidx[o]; sg = psgn[o]; }
  }
  sgn[j] = sg;
}

template <typename TC>
__global__ void colscale_kernel(int64_t rows, int p, TC* __restrict__ U, const double* __restrict__ s) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * p) return;
  const int j = (int)(e % p);
  if (s[j] < 0.0) U[e] = from_f64<TC>(-to_f64(U[e]));
}

}  // namespace

// ---------------------------------------------------------------------------
// Workspace planner
// ---------------------------------------------------------------------------
namespace {

struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <typename T> T* take(size_t count) {
    void* p = base ? base + off : nullptr;
    off += (count * sizeof(T) + 255) & ~(size_t)255;
    return (T*)p;
  }
  void* take_bytes(size_t bytes) {
    void* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  }
};

// FP64 scratch of one sketching round with p components.
struct RoundWs {
  double *W, *Uw, *Sw, *Vw, *nc2, *nr2, *invc, *invr, *sk, *dk;
  double *G2, *Gs2, *E2V, *fpos, *fneg;   // both Grams and their pivoted Cholesky factors
  void* pch_ws;                           // the factorisation's workspace (used above PCHOL_MAXP)
  double *K, *Us, *S1, *Vs, *T1, *T2, *Mu, *Mv, *sq;
  void *svd_ws, *gram_ws, *ts_ws;
  void *Ch, *Rh;                                      // extrapolated vectors (compute precision)
};

struct Plan {
  int prec, kr1, kc1, kr2, kc2, p1, p2;
  int ep;  // columns of the stored embeddings P, Q: p1, padded to whole 16-byte runs in FP32 and 16-bit compute
  int64_t m, n;
};

static void plan_round(Carve& cv, RoundWs& R, const Plan& pl, int kr, int kc, bool need_vectors, bool need_ortho) {
  const int p = std::min(kr, kc);
  const size_t eb = prec_bytes(pl.prec);
  R.W = cv.take<double>((size_t)kr * kc);
  R.Uw = cv.take<double>((size_t)kr * p);
  R.Sw = cv.take<double>(p);
  R.Vw = cv.take<double>((size_t)kc * p);
  R.nc2 = cv.take<double>(p);
  R.nr2 = cv.take<double>(p);
  R.invc = cv.take<double>(p);
  R.invr = cv.take<double>(p);
  R.sk = cv.take<double>(p);
  R.dk = cv.take<double>(p);
  size_t svd_b = std::max(svd_ws_bytes(1, kr, kc), need_ortho ? svd_ws_bytes(1, p, p) : 0);
  R.svd_ws = cv.take_bytes(svd_b);
  const int64_t mx = std::max(pl.m, pl.n);
  R.ts_ws = cv.take_bytes(std::max(tsgemm_ws_bytes(mx, std::max(kr, kc), p, pl.prec), tsgemm_ws_bytes(mx, p, p, pl.prec)));
  if (need_vectors) {
    R.Ch = cv.take_bytes((size_t)pl.m * p * eb);
    R.Rh = cv.take_bytes((size_t)pl.n * p * eb);
  } else {
    R.Ch = R.Rh = nullptr;
  }
  if (need_ortho) {
    R.G2 = cv.take<double>(2 * (size_t)p * p);
    R.Gs2 = cv.take<double>(2 * (size_t)p * p);
    R.pch_ws = cv.take_bytes(pchol_ws_bytes(2, p));
    R.E2V = cv.take<double>(2 * (size_t)p * p);
    R.fpos = cv.take<double>(2 * (size_t)p);
    R.fneg = cv.take<double>(2 * (size_t)p);
    R.K = cv.take<double>((size_t)p * p);
    R.Us = cv.take<double>((size_t)p * p);
    R.S1 = cv.take<double>(p);
    R.Vs = cv.take<double>((size_t)p * p);
    R.T1 = cv.take<double>((size_t)p * p);
    R.T2 = cv.take<double>((size_t)p * p);
    R.Mu = cv.take<double>((size_t)p * p);
    R.Mv = cv.take<double>((size_t)p * p);
    R.sq = cv.take<double>(p);
    R.gram_ws = cv.take_bytes(gram_ws_bytes(mx, p));
  } else {
    R.Mu = cv.take<double>((size_t)p * p);
    R.Mv = cv.take<double>((size_t)p * p);
    R.G2 = R.Gs2 = R.E2V = R.fpos = R.fneg = R.K = R.Us = R.S1 = R.Vs = R.T1 = R.T2 = R.sq = nullptr;
    R.pch_ws = nullptr;
    R.gram_ws = nullptr;
  }
}

struct SketchWs {
  int64_t *Ir, *Ic, *Ir0, *Ic0;
  void *C, *Rt, *P, *Q;
  double *rowsqP, *rowsqQ, *wr, *wc, *Z0r, *Z0c, *Zr, *Zc, *diag, *obj;
  unsigned long long* entries;
  double* levinv;      // leverage variant: reciprocal singular values of the kept components
  double *MuP, *MvP;  // the embedding maps with ep - p1 zero columns (16-bit compute, p1 not a multiple of 8)
  void* ts6;
  void *kmr, *kmc, *selr, *selc;
  RoundWs r1, r2;
  double* sgn_ws;
};

static size_t plan_sketch(void* ws, const Plan& pl, const cabs_params* prm, SketchWs& S) {
  Carve cv(ws);
  const size_t eb = prec_bytes(pl.prec);
  const int e = pl.p1, ep = pl.ep;
  if (prm->follow_up == CABS_FOLLOW_PILOT) {  // one round: the output buffers hold the pilot sample and sketch
    S = SketchWs{};
    S.diag = cv.take<double>(CABS_DIAG_LEN);
    S.entries = cv.take<unsigned long long>(1);
    plan_round(cv, S.r2, pl, pl.kr2, pl.kc2, prm->want_factors != 0, prm->want_factors != 0);
    S.sgn_ws = prm->want_factors ? cv.take<double>((size_t)3 * 256 * pl.p2) : nullptr;
    return cv.off + 256;
  }
  S.Ir = cv.take<int64_t>(pl.kr1);
  S.Ic = cv.take<int64_t>(pl.kc1);
  S.Ir0 = cv.take<int64_t>(std::max(pl.kr2, 1));
  S.Ic0 = cv.take<int64_t>(std::max(pl.kc2, 1));
  S.C = cv.take_bytes((size_t)pl.m * pl.kc1 * eb);
  S.Rt = cv.take_bytes((size_t)pl.n * pl.kr1 * eb);
  S.P = cv.take_bytes((size_t)pl.m * ep * eb);
  S.Q = cv.take_bytes((size_t)pl.n * ep * eb);
  S.rowsqP = cv.take<double>(pl.m);
  S.rowsqQ = cv.take<double>(pl.n);
  S.wr = cv.take<double>(pl.m);
  S.wc = cv.take<double>(pl.n);
  S.Z0r = cv.take<double>((size_t)pl.kr2 * ep);
  S.Z0c = cv.take<double>((size_t)pl.kc2 * ep);
  S.Zr = cv.take<double>((size_t)pl.kr2 * ep);
  S.Zc = cv.take<double>((size_t)pl.kc2 * ep);
  S.MuP = ep != e ? cv.take<double>((size_t)e * ep) : nullptr;
  S.MvP = ep != e ? cv.take<double>((size_t)e * ep) : nullptr;
  S.ts6 = ep != e ? cv.take_bytes(tsgemm_ws_bytes(std::max(pl.m, pl.n), e, ep, pl.prec)) : nullptr;
  S.levinv = cv.take<double>(std::max(e, 1));
  S.diag = cv.take<double>(CABS_DIAG_LEN);
  S.obj = cv.take<double>(8);
  S.entries = cv.take<unsigned long long>(1);
  if (prm->follow_up == CABS_FOLLOW_HARD || prm->follow_up == CABS_FOLLOW_LEVERAGE) {
    S.kmr = S.kmc = nullptr;
    S.selr = cv.take_bytes(select_ws_bytes(pl.m));
    S.selc = cv.take_bytes(select_ws_bytes(pl.n));
  } else {
    S.kmr = cv.take_bytes(kmeans_ws_bytes(pl.m, ep, pl.kr2, pl.prec));
    S.kmc = cv.take_bytes(kmeans_ws_bytes(pl.n, ep, pl.kc2, pl.prec));
    S.selr = S.selc = nullptr;
  }
  plan_round(cv, S.r1, pl, pl.kr1, pl.kc1, true, prm->orthogonalize != 0);
  plan_round(cv, S.r2, pl, pl.kr2, pl.kc2, prm->want_factors != 0, prm->want_factors != 0);
  S.sgn_ws = prm->want_factors ? cv.take<double>((size_t)3 * 256 * pl.p2) : nullptr;
  return cv.off + 256;
}

static bool valid_prec(int p) { return p == CABS_F64 || p == CABS_F32 || p == CABS_BF16 || p == CABS_F16; }

static cabs_status check_matrix(const cabs_matrix* mat) {
  if (!mat) return fail(CABS_EINVAL, "null matrix descriptor");
  if (mat->m <= 0 || mat->n <= 0) return fail(CABS_EINVAL, "matrix dimensions must be positive");
  if (mat->m >= (int64_t)1 << 31 || mat->n >= (int64_t)1 << 31)
    return fail(CABS_EINVAL, "matrix dimensions must be below 2^31");
  if (mat->storage != CABS_F64 && mat->storage != CABS_F32) return fail(CABS_EINVAL, "storage must be F64 or F32");
  switch (mat->kind) {
    case CABS_SRC_DENSE:
      if (!mat->a) return fail(CABS_EINVAL, "dense source needs a");
      if (mat->lda < mat->n) return fail(CABS_EINVAL, "lda must be >= n");
      break;
    case CABS_SRC_LOWRANK:
      if (!mat->pf || !mat->qf || !mat->s) return fail(CABS_EINVAL, "low-rank source needs pf, qf, s");
      if (mat->r <= 0) return fail(CABS_EINVAL, "rank r must be positive");
      if (!(mat->noise_std >= 0.0)) return fail(CABS_EINVAL, "noise_std must be >= 0");
      break;
    case CABS_SRC_RBF:
      if (!mat->x || !mat->y) return fail(CABS_EINVAL, "RBF source needs x and y");
      if (mat->d <= 0) return fail(CABS_EINVAL, "dimension d must be positive");
      if (!(mat->sigma > 0.0)) return fail(CABS_EINVAL, "sigma must be positive");
      break;
    case CABS_SRC_CSR:
      if (!mat->row_ptr || !mat->col_ptr || (mat->nnz > 0 && (!mat->col_idx || !mat->vals || !mat->row_idx ||
                                                               !mat->vals_t)))
        return fail(CABS_EINVAL, "CSR source needs row_ptr, col_idx, vals, col_ptr, row_idx, vals_t");
      if (mat->nnz < 0) return fail(CABS_EINVAL, "nnz must be >= 0");
      if (mat->m >= INT32_MAX || mat->n >= INT32_MAX) return fail(CABS_EINVAL, "CSR source needs m, n < 2^31 - 1");
      break;
    default:
      return fail(CABS_EINVAL, "unknown source kind %d", mat->kind);
  }
  return CABS_OK;
}

static cabs_status check_compute(const cabs_matrix* mat, int compute) {
  if (!valid_prec(compute)) return fail(CABS_EINVAL, "unknown compute precision %d", compute);
  if (mat->storage == CABS_F64 && compute != CABS_F64)
    return fail(CABS_EINVAL, "FP64 tables need FP64 compute");
  if (mat->storage == CABS_F32 && compute == CABS_F64)
    return fail(CABS_EINVAL, "FP64 compute needs FP64 tables");
  return CABS_OK;
}

static cabs_status check_params(const cabs_matrix* mat, const cabs_params* prm) {
  cabs_status s = check_matrix(mat);
  if (s != CABS_OK) return s;
  if (!prm) return fail(CABS_EINVAL, "null parameters");
  s = check_compute(mat, prm->compute);
  if (s != CABS_OK) return s;
  const int ks[4] = {prm->k1_rows, prm->k1_cols, prm->k2_rows, prm->k2_cols};
  for (int i = 0; i < 4; ++i)
    if (ks[i] < 1 || ks[i] > 1024) return fail(CABS_EINVAL, "sample sizes must be in [1, 1024]");
  if (prm->k1_rows > mat->m || prm->k2_rows > mat->m) return fail(CABS_EINVAL, "row sample size exceeds m");
  if (prm->k1_cols > mat->n || prm->k2_cols > mat->n) return fail(CABS_EINVAL, "column sample size exceeds n");
  if (prm->kmeans_iters < 0 || prm->kmeans_iters > 10000) return fail(CABS_EINVAL, "kmeans_iters out of range");
  if (prm->weight_kind < CABS_W_CONST || prm->weight_kind > CABS_W_STEP) return fail(CABS_EINVAL, "unknown weight kind");
  if (prm->sketch_kind != CABS_SK_STABILIZED && prm->sketch_kind != CABS_SK_PSEUDO_SKELETON)
    return fail(CABS_EINVAL, "unknown sketch kind");
  if (prm->follow_up != CABS_FOLLOW_KMEANS && prm->follow_up != CABS_FOLLOW_HARD &&
      prm->follow_up != CABS_FOLLOW_LEVERAGE && prm->follow_up != CABS_FOLLOW_PILOT)
    return fail(CABS_EINVAL, "unknown follow-up kind");
  if (prm->follow_up == CABS_FOLLOW_PILOT && (prm->k2_rows != prm->k1_rows || prm->k2_cols != prm->k1_cols))
    return fail(CABS_EINVAL, "the pilot sketch alone needs k2 = k1 on both sides");
  if (prm->flags & ~CABS_FLAG_COUNT_ENTRIES) return fail(CABS_EINVAL, "unknown flag bits");
  if ((prm->follow_up == CABS_FOLLOW_HARD || prm->follow_up == CABS_FOLLOW_LEVERAGE) &&
      (mat->m >= INT32_MAX || mat->n >= INT32_MAX))
    return fail(CABS_EINVAL, "the hard-threshold and leverage selections need m, n < 2^31 - 1");
  return CABS_OK;
}

static Plan make_plan(const cabs_matrix* mat, const cabs_params* prm) {
  Plan pl;
  pl.prec = prm->compute;
  pl.kr1 = prm->k1_rows;
  pl.kc1 = prm->k1_cols;
  pl.kr2 = prm->k2_rows;
  pl.kc2 = prm->k2_cols;
  pl.p1 = std::min(pl.kr1, pl.kc1);
  pl.p2 = std::min(pl.kr2, pl.kc2);
  pl.ep = (pl.prec == CABS_BF16 || pl.prec == CABS_F16) ? (pl.p1 + 7) / 8 * 8
          : pl.prec == CABS_F32                          ? (pl.p1 + 3) / 4 * 4
                                                         : pl.p1;
  pl.m = mat->m;
  pl.n = mat->n;
  return pl;
}

static MatView view_of(const cabs_matrix* mat) {
  MatView v;
  v.kind = mat->kind;
  v.storage = mat->storage;
  v.m = mat->m;
  v.n = mat->n;
  v.a = mat->a;
  v.lda = mat->lda;
  v.pf = mat->pf;
  v.qf = mat->qf;
  v.s = mat->s;
  v.r = mat->r;
  v.noise_std = mat->noise_std;
  v.noise_seed = mat->noise_seed;
  v.x = mat->x;
  v.y = mat->y;
  v.d = mat->d;
  v.sigma = mat->sigma;
  v.row_ptr = mat->row_ptr;
  v.col_idx = mat->col_idx;
  v.vals = mat->vals;
  v.col_ptr = mat->col_ptr;
  v.row_idx = mat->row_idx;
  v.vals_t = mat->vals_t;
  v.nnz = mat->nnz;
  return v;
}

// ---------------------------------------------------------------------------
// The sketch as a sequence of phases between its FP64 SVDs.  advance() runs a
// request's kernels up to its next SVD and describes that SVD (SvdJob); the
// caller runs it (cabs_sketch: at once; a server group: one batched launch
// for several same-shape requests, each item in its own workspace, so the
// results are the same bits either way) and calls advance() again.
//
// One sketching round on sampled C (m x kc), R^T (n x kr), W (kr x kc, FP64):
//   SVD of W | norms and scalings (sketch_vec); with `ortho` the Grams, their
//   pivoted Cholesky factors and K | the SVD of K | the embedding maps.
// ---------------------------------------------------------------------------
struct SvdJob {
  int n = 0, rows = 0, cols = 0;  // n items (0: no SVD, the sketch has finished)
  const double* A[1];
  double *U[1], *S[1], *V[1], *W[1];
};

enum Phase {
  PH_START = 0,
  PH_R1_AFTER_W,     // round 1: after the SVD of W
  PH_R1_AFTER_K,     // round 1: after the SVD of K
  PH_R2_AFTER_W,
  PH_R2_AFTER_K,
  PH_DONE
};

struct SketchRun {
  const cabs_matrix* mat;
  const cabs_params* prm;
  cabs_result* out;
  Plan pl;
  SketchWs S;
  MatView mv;
  double* diag;
  hipStream_t st;
  bool counted;
  unsigned long long* ecnt;
  int phase;
};

static void svd_job_one(SvdJob& j, int rows, int cols, const double* A, double* U, double* S, double* V, void* ws) {
  j.n = 1;
  j.rows = rows;
  j.cols = cols;
  j.A[0] = A;
  j.U[0] = U;
  j.S[0] = S;
  j.V[0] = V;
  j.W[0] = (double*)ws;
}

// Round part after the SVD of W: C^ = C V_w, R^ = R^T U_w with norms, the
// kept components and scalings; with `ortho` the Grams, their pivoted
// Cholesky factors and K (next: the SVD of K).  `next` receives the following SVD.
static cabs_status round_after_w(const SketchRun& c, RoundWs& R, int kr, int kc, const void* C, const void* Rt,
                                 bool vectors, bool ortho, int slot_rank, int slot_sig, SvdJob& next) {
  const Plan& pl = c.pl;
  hipStream_t st = c.st;
  const int p = std::min(kr, kc);
  next.n = 0;
  HIP_TRY(launch_tsgemm(pl.m, kc, p, pl.prec, C, R.Vw, vectors ? R.Ch : nullptr, R.nc2, nullptr, R.ts_ws, st));
  HIP_TRY(launch_tsgemm(pl.n, kr, p, pl.prec, Rt, R.Uw, vectors ? R.Rh : nullptr, R.nr2, nullptr, R.ts_ws, st));
  hipLaunchKernelGGL(sketch_vec_kernel, dim3(1), dim3(1024), 0, st, p, kr, kc, (double)pl.m, (double)pl.n, R.Sw, R.nc2,
                     R.nr2, c.prm->pinv_rtol, c.prm->sketch_kind, R.invc, R.invr, R.sk, R.dk, c.diag, slot_rank,
                     slot_sig);
  HIP_TRY(hipGetLastError());
  if (!vectors) return CABS_OK;
  if (!ortho) {
    // P = U S^(1/2) = C^ diag(invc sqrt(S)), Q = R^ diag(invr sqrt(S))
    const unsigned gb = (unsigned)ceil_div((int64_t)p * p, 256);
    hipLaunchKernelGGL(diag_mat_kernel, dim3(gb), dim3(256), 0, st, p, R.invc, R.sk, R.Mu);
    hipLaunchKernelGGL(diag_mat_kernel, dim3(gb), dim3(256), 0, st, p, R.invr, R.sk, R.Mv);
    HIP_TRY(hipGetLastError());
    return CABS_OK;
  }
  const size_t pp = (size_t)p * p;
  // Grams of the unit-norm factors U = C^ N_c^-1, V = R^ N_r^-1 (FP64).
  HIP_TRY(launch_gram(pl.m, p, pl.prec, R.Ch, R.Gs2, R.gram_ws, st));
  HIP_TRY(launch_gram(pl.n, p, pl.prec, R.Rh, R.Gs2 + pp, R.gram_ws, st));
  const unsigned gb = (unsigned)ceil_div((int64_t)pp, 256);
  hipLaunchKernelGGL(scale2_kernel, dim3(gb), dim3(256), 0, st, p, R.Gs2, R.invc, R.invc, R.G2);
  hipLaunchKernelGGL(scale2_kernel, dim3(gb), dim3(256), 0, st, p, R.Gs2 + pp, R.invr, R.invr, R.G2 + pp);
  // Pivoted Cholesky G = R^T R of both Grams (rank-revealing: pivots <= p eps of the unit diagonal
  // stop it), K = R_u diag(S) R_v^T, then the SVD of K (next).
  const double eps = 2.220446049250313e-16;
  HIP_TRY(launch_pchol(2, p, R.G2, pp, (double)p * eps, R.E2V, pp, R.pch_ws, st));
  HIP_TRY(launch_small_gemm(p, p, p, R.E2V, p, false, R.E2V + pp, p, true, nullptr, R.sk, nullptr, R.K, p, st));
  svd_job_one(next, p, p, R.K, R.Us, R.S1, R.Vs, R.svd_ws);
  return CABS_OK;
}

// After the SVD of K: the embedding maps M_u, M_v.
static cabs_status round_after_k(const SketchRun& c, RoundWs& R, int p) {
  hipStream_t st = c.st;
  const size_t pp = (size_t)p * p;
  // Since K V_s = U_s S_1, R_u^-1 U_s = diag(S) R_v^T V_s S_1^-1, so without any triangular solve
  //   M_u = diag(invc S) R_v^T V_s S_1^(-1/2),  M_v = diag(invr S) R_u^T U_s S_1^(-1/2)
  // map C^ and R^ to P = U' S_1^(1/2), Q = V' S_1^(1/2) (components with S_1 <= p eps S_1[0] dropped).
  hipLaunchKernelGGL(rsqrt_trunc_kernel, dim3(1), dim3(1024), 0, st, p, R.S1, R.sq);
  hipLaunchKernelGGL(mul_vec_kernel, dim3(1), dim3(1024), 0, st, p, R.invc, R.sk, R.fpos);
  hipLaunchKernelGGL(mul_vec_kernel, dim3(1), dim3(1024), 0, st, p, R.invr, R.sk, R.fpos + p);
  HIP_TRY(launch_small_gemm(p, p, p, R.E2V + pp, p, true, R.Vs, p, false, R.fpos, nullptr, R.sq, R.Mu, p, st));
  HIP_TRY(launch_small_gemm(p, p, p, R.E2V, p, true, R.Us, p, false, R.fpos + p, nullptr, R.sq, R.Mv, p, st));
  HIP_TRY(hipGetLastError());
  return CABS_OK;
}

static cabs_status sketch_begin(SketchRun& c, const cabs_matrix* mat, const cabs_params* prm, void* ws,
                                size_t ws_bytes, cabs_result* out, hipStream_t st) {
  cabs_status s = check_params(mat, prm);
  if (s != CABS_OK) return s;
  if (!out || !out->idx_r || !out->idx_c || !out->C || !out->Rt || !out->Umid)
    return fail(CABS_EINVAL, "result buffers idx_r, idx_c, C, Rt, Umid are required");
  if (prm->want_factors && (!out->Uf || !out->S || !out->Vf))
    return fail(CABS_EINVAL, "want_factors needs Uf, S, Vf");
  if (!ws || ((uintptr_t)ws & 255)) return fail(CABS_EINVAL, "workspace must be non-null and 256-byte aligned");
  c.mat = mat;
  c.prm = prm;
  c.out = out;
  c.pl = make_plan(mat, prm);
  const size_t need = plan_sketch(nullptr, c.pl, prm, c.S);
  if (ws_bytes < need) return fail(CABS_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  plan_sketch(ws, c.pl, prm, c.S);
  c.st = st;
  c.mv = view_of(mat);
  c.diag = out->diag ? out->diag : c.S.diag;
  c.counted = (prm->flags & CABS_FLAG_COUNT_ENTRIES) != 0;
  c.ecnt = c.counted ? c.S.entries : nullptr;
  c.phase = PH_START;
  return CABS_OK;
}

// Steps 6-7 (embeddings, weights, follow-up sampling) after the pilot round.
static cabs_status sketch_middle(SketchRun& c) {
  const Plan& pl = c.pl;
  SketchWs& S = c.S;
  const cabs_params* prm = c.prm;
  cabs_result* out = c.out;
  hipStream_t st = c.st;
  double* diag = c.diag;
  const int e = pl.p1, ep = pl.ep;
  int64_t* Ir = out->pilot_r ? out->pilot_r : S.Ir;
  int64_t* Ic = out->pilot_c ? out->pilot_c : S.Ic;
  // 6: embeddings and weights
  // When p1 elements are not a whole number of 16-byte runs (FP32: p1 not a multiple of 4, 16-bit:
  // of 8) the embeddings get ep - p1 zero columns, so that their rows are whole runs for the k-means
  // kernels; zero columns add exact zeros to every distance, norm and centre.
  const double* Mu = S.r1.Mu;
  const double* Mv = S.r1.Mv;
  void* ts6 = S.r1.ts_ws;
  if (ep != e) {
    const unsigned gp = (unsigned)ceil_div((int64_t)e * ep, 256);
    hipLaunchKernelGGL(pad_cols_kernel, dim3(gp), dim3(256), 0, st, e, e, ep, S.r1.Mu, S.MuP);
    hipLaunchKernelGGL(pad_cols_kernel, dim3(gp), dim3(256), 0, st, e, e, ep, S.r1.Mv, S.MvP);
    Mu = S.MuP;
    Mv = S.MvP;
    ts6 = S.ts6;
  }
  HIP_TRY(launch_tsgemm(pl.m, e, ep, pl.prec, S.r1.Ch, Mu, S.P, nullptr, S.rowsqP, ts6, st));
  HIP_TRY(launch_tsgemm(pl.n, e, ep, pl.prec, S.r1.Rh, Mv, S.Q, nullptr, S.rowsqQ, ts6, st));
  hipLaunchKernelGGL(weights_kernel, dim3((unsigned)ceil_div(pl.m, 256)), dim3(256), 0, st, pl.m, S.rowsqP,
                     prm->weight_kind, prm->weight_param, S.wr);
  hipLaunchKernelGGL(weights_kernel, dim3((unsigned)ceil_div(pl.n, 256)), dim3(256), 0, st, pl.n, S.rowsqQ,
                     prm->weight_kind, prm->weight_param, S.wc);
  HIP_TRY(hipGetLastError());

  // 7: follow-up sampling.  Hard-threshold variant (Section 5): the rows and
  // columns with the largest weights.
  if (prm->follow_up == CABS_FOLLOW_HARD) {
    HIP_TRY(launch_select_topk(pl.m, S.wr, pl.kr2, out->idx_r, S.selr, st));
    HIP_TRY(launch_select_topk(pl.n, S.wc, pl.kc2, out->idx_c, S.selc, st));
  } else if (prm->follow_up == CABS_FOLLOW_LEVERAGE) {
    // Leverage variant (Section 5): keys from the squared row norms of the factors behind P and Q
    // (P = U' diag(s)^(1/2), s = the orthogonalised singular values, or the sketch's S without
    // orthogonalisation), then the k largest keys.  The weights buffers hold the keys.
    const double* sv = prm->orthogonalize ? S.r1.S1 : S.r1.sk;
    hipLaunchKernelGGL(lev_inv_kernel, dim3(1), dim3(256), 0, st, e, sv, S.levinv);
    HIP_TRY(hipGetLastError());
    HIP_TRY(launch_lev_keys_any(pl.prec, pl.m, ep, e, S.P, S.levinv, prm->seed, STREAM_LEVERAGE_ROWS, S.wr, st));
    HIP_TRY(launch_lev_keys_any(pl.prec, pl.n, ep, e, S.Q, S.levinv, prm->seed, STREAM_LEVERAGE_COLS, S.wc, st));
    HIP_TRY(launch_select_topk(pl.m, S.wr, pl.kr2, out->idx_r, S.selr, st));
    HIP_TRY(launch_select_topk(pl.n, S.wc, pl.kc2, out->idx_c, S.selc, st));
  } else {
    // Weighted k-means from the pilot sample, then snapping.
    const int64_t* I0r = Ir;
    const int64_t* I0c = Ic;
    if (pl.kr2 > pl.kr1) {
      HIP_TRY(launch_sample(pl.m, pl.kr2, prm->seed, STREAM_INIT_ROWS, S.Ir0, st));
      I0r = S.Ir0;
    }
    if (pl.kc2 > pl.kc1) {
      HIP_TRY(launch_sample(pl.n, pl.kc2, prm->seed, STREAM_INIT_COLS, S.Ic0, st));
      I0c = S.Ic0;
    }
    HIP_TRY(launch_gather_rows_f64(S.P, pl.prec, ep, I0r, pl.kr2, ep, S.Z0r, st));
    HIP_TRY(launch_gather_rows_f64(S.Q, pl.prec, ep, I0c, pl.kc2, ep, S.Z0c, st));
    KMeansOut kr{S.Zr, nullptr, S.obj, diag + CABS_DIAG_TMAX_R, diag + CABS_DIAG_GAP_R, out->idx_r,
                 diag + CABS_DIAG_SNAP_SCANS_R};
    HIP_TRY(launch_kmeans(pl.m, ep, pl.kr2, pl.prec, S.P, S.wr, S.Z0r, prm->kmeans_iters, kr, S.kmr, st));
    KMeansOut kc{S.Zc, nullptr, S.obj + 2, diag + CABS_DIAG_TMAX_C, diag + CABS_DIAG_GAP_C, out->idx_c,
                 diag + CABS_DIAG_SNAP_SCANS_C};
    HIP_TRY(launch_kmeans(pl.n, ep, pl.kc2, pl.prec, S.Q, S.wc, S.Z0c, prm->kmeans_iters, kc, S.kmc, st));
    hipLaunchKernelGGL(copy_slot_kernel, dim3(1), dim3(64), 0, st, S.obj + 0, diag + CABS_DIAG_ENC_R_PILOT);
    hipLaunchKernelGGL(copy_slot_kernel, dim3(1), dim3(64), 0, st, S.obj + 1, diag + CABS_DIAG_ENC_R_FINAL);
    hipLaunchKernelGGL(copy_slot_kernel, dim3(1), dim3(64), 0, st, S.obj + 2, diag + CABS_DIAG_ENC_C_PILOT);
    hipLaunchKernelGGL(copy_slot_kernel, dim3(1), dim3(64), 0, st, S.obj + 3, diag + CABS_DIAG_ENC_C_FINAL);
    HIP_TRY(hipGetLastError());
  }
  return CABS_OK;
}

// Follow-up evaluation (step 8) up to W-bar: C-bar, R-bar^T and W-bar = C-bar(I-bar^r, :).
static cabs_status sketch_followup_eval(SketchRun& c, SvdJob& next) {
  const Plan& pl = c.pl;
  cabs_result* out = c.out;
  hipStream_t st = c.st;
  HIP_TRY(launch_eval(c.mv, false, out->idx_c, pl.kc2, pl.prec, out->C, st, c.ecnt));
  HIP_TRY(launch_eval(c.mv, true, out->idx_r, pl.kr2, pl.prec, out->Rt, st, c.ecnt));
  if (c.counted) hipLaunchKernelGGL(entries_out_kernel, dim3(1), dim3(64), 0, st, c.S.entries, c.diag);
  HIP_TRY(launch_gather_rows_f64(out->C, pl.prec, pl.kc2, out->idx_r, pl.kr2, pl.kc2, c.S.r2.W, st));
  RoundWs& R = c.S.r2;
  svd_job_one(next, pl.kr2, pl.kc2, R.W, R.Uw, R.Sw, R.Vw, R.svd_ws);
  return CABS_OK;
}

// After the follow-up round: U_mid, the pilot-only diagnostics and the optional factor form (step 9).
static cabs_status sketch_final(SketchRun& c) {
  const Plan& pl = c.pl;
  SketchWs& S = c.S;
  const cabs_params* prm = c.prm;
  cabs_result* out = c.out;
  hipStream_t st = c.st;
  double* diag = c.diag;
  const bool fac = prm->want_factors != 0;
  // Umid = V_w diag(D) U_w^T  (kc2 x kr2)
  HIP_TRY(launch_small_gemm(pl.kc2, pl.kr2, pl.p2, S.r2.Vw, pl.p2, false, S.r2.Uw, pl.p2, true, nullptr, S.r2.dk,
                            nullptr, out->Umid, pl.kr2, st));
  if (prm->follow_up == CABS_FOLLOW_PILOT) {
    hipLaunchKernelGGL(copy_slot_kernel, dim3(1), dim3(64), 0, st, diag + CABS_DIAG_RANK_FINAL, diag + CABS_DIAG_RANK_PILOT);
    hipLaunchKernelGGL(copy_slot_kernel, dim3(1), dim3(64), 0, st, diag + CABS_DIAG_SIGMA1_FINAL,
                       diag + CABS_DIAG_SIGMA1_PILOT);
    HIP_TRY(hipGetLastError());
  }

  // 9: optional factor form: Uf = U' (orthonormal), S = S_1, Vf = V', mapped from C^ and R^.
  if (fac) {
    const int p = pl.p2;
    RoundWs& R = S.r2;
    // M_u = diag(invc S) R_v^T V_s S_1^-1, M_v likewise
    hipLaunchKernelGGL(mul_vec_kernel, dim3(1), dim3(1024), 0, st, p, R.sq, R.sq, R.fneg);
    HIP_TRY(launch_small_gemm(p, p, p, R.E2V + (size_t)p * p, p, true, R.Vs, p, false, R.fpos, nullptr, R.fneg,
                              R.Mu, p, st));
    HIP_TRY(launch_small_gemm(p, p, p, R.E2V, p, true, R.Us, p, false, R.fpos + p, nullptr, R.fneg, R.Mv, p, st));
    HIP_TRY(launch_tsgemm(pl.m, p, p, pl.prec, R.Ch, R.Mu, out->Uf, nullptr, nullptr, R.ts_ws, st));
    HIP_TRY(launch_tsgemm(pl.n, p, p, pl.prec, R.Rh, R.Mv, out->Vf, nullptr, nullptr, R.ts_ws, st));
    // signs: largest-magnitude entry of each Uf column positive
    const int nb = (int)std::min<int64_t>(256, ceil_div(pl.m, 256));
    const int64_t rows_per = ceil_div(pl.m, nb);
    double* pm = S.sgn_ws;
    int64_t* pi = (int64_t*)(S.sgn_ws + (size_t)256 * p);
    double* ps = S.sgn_ws + 2 * (size_t)256 * p;
    hipLaunchKernelGGL(colsign_partial_kernel, dim3(nb, (unsigned)ceil_div(p, 256)), dim3(256), 0, st, pl.m, p,
                       rows_per, out->Uf, pl.prec, pm, pi, ps);
    hipLaunchKernelGGL(colsign_final_kernel, dim3((unsigned)ceil_div(p, 256)), dim3(256), 0, st, nb, p, pm, pi, ps,
                       R.sq);
    const unsigned gu = (unsigned)ceil_div(pl.m * p, 256), gv = (unsigned)ceil_div(pl.n * p, 256);
    switch (pl.prec) {
      case P_F64:
        hipLaunchKernelGGL(colscale_kernel<double>, dim3(gu), dim3(256), 0, st, pl.m, p, (double*)out->Uf, R.sq);
        hipLaunchKernelGGL(colscale_kernel<double>, dim3(gv), dim3(256), 0, st, pl.n, p, (double*)out->Vf, R.sq);
        break;
      case P_F32:
        hipLaunchKernelGGL(colscale_kernel<float>, dim3(gu), dim3(256), 0, st, pl.m, p, (float*)out->Uf, R.sq);
        hipLaunchKernelGGL(colscale_kernel<float>, dim3(gv), dim3(256), 0, st, pl.n, p, (float*)out->Vf, R.sq);
        break;
      case P_BF16:
        hipLaunchKernelGGL(colscale_kernel<bf16>, dim3(gu), dim3(256), 0, st, pl.m, p, (bf16*)out->Uf, R.sq);
        hipLaunchKernelGGL(colscale_kernel<bf16>, dim3(gv), dim3(256), 0, st, pl.n, p, (bf16*)out->Vf, R.sq);
        break;
      default:
        hipLaunchKernelGGL(colscale_kernel<f16>, dim3(gu), dim3(256), 0, st, pl.m, p, (f16*)out->Uf, R.sq);
        hipLaunchKernelGGL(colscale_kernel<f16>, dim3(gv), dim3(256), 0, st, pl.n, p, (f16*)out->Vf, R.sq);
        break;
    }
    hipLaunchKernelGGL(copy_vec_kernel, dim3(1), dim3(1024), 0, st, p, R.S1, out->S);
  }
  HIP_TRY(hipGetLastError());
  return CABS_OK;
}

// Runs the sketch up to its next SVD (described in `job`) or to its end (job.n = 0).
static cabs_status sketch_advance(SketchRun& c, SvdJob& job) {
  const Plan& pl = c.pl;
  SketchWs& S = c.S;
  const cabs_params* prm = c.prm;
  cabs_result* out = c.out;
  hipStream_t st = c.st;
  const bool ortho = prm->orthogonalize != 0, fac = prm->want_factors != 0;
  job.n = 0;
  cabs_status s = CABS_OK;
  switch (c.phase) {
    case PH_START: {
      hipLaunchKernelGGL(diag_init_kernel, dim3(1), dim3(64), 0, st, c.diag, S.entries, c.counted ? 1 : 0);
      HIP_TRY(hipGetLastError());
      if (prm->follow_up == CABS_FOLLOW_PILOT) {
        // The pilot sketch alone: the pilot sample is the output sample, and the follow-up
        // round below is the pilot round (steps 1-3 of Algorithm 2).
        HIP_TRY(launch_sample(pl.m, pl.kr1, prm->seed, STREAM_PILOT_ROWS, out->idx_r, st));
        HIP_TRY(launch_sample(pl.n, pl.kc1, prm->seed, STREAM_PILOT_COLS, out->idx_c, st));
        if (out->pilot_r) HIP_TRY(launch_sample(pl.m, pl.kr1, prm->seed, STREAM_PILOT_ROWS, out->pilot_r, st));
        if (out->pilot_c) HIP_TRY(launch_sample(pl.n, pl.kc1, prm->seed, STREAM_PILOT_COLS, out->pilot_c, st));
        c.phase = PH_R2_AFTER_W;
        return sketch_followup_eval(c, job);
      }
      // 1-2: pilot sampling and evaluation
      int64_t* Ir = out->pilot_r ? out->pilot_r : S.Ir;
      int64_t* Ic = out->pilot_c ? out->pilot_c : S.Ic;
      HIP_TRY(launch_sample(pl.m, pl.kr1, prm->seed, STREAM_PILOT_ROWS, Ir, st));
      HIP_TRY(launch_sample(pl.n, pl.kc1, prm->seed, STREAM_PILOT_COLS, Ic, st));
      HIP_TRY(launch_eval(c.mv, false, Ic, pl.kc1, pl.prec, S.C, st, c.ecnt));
      HIP_TRY(launch_eval(c.mv, true, Ir, pl.kr1, pl.prec, S.Rt, st, c.ecnt));
      HIP_TRY(launch_gather_rows_f64(S.C, pl.prec, pl.kc1, Ir, pl.kr1, pl.kc1, S.r1.W, st));
      // 3: the SVD of W (next)
      svd_job_one(job, pl.kr1, pl.kc1, S.r1.W, S.r1.Uw, S.r1.Sw, S.r1.Vw, S.r1.svd_ws);
      c.phase = PH_R1_AFTER_W;
      return CABS_OK;
    }
    case PH_R1_AFTER_W:
      // 4-5: pilot sketch and embedding maps
      s = round_after_w(c, S.r1, pl.kr1, pl.kc1, S.C, S.Rt, true, ortho, CABS_DIAG_RANK_PILOT, CABS_DIAG_SIGMA1_PILOT,
                        job);
      if (s != CABS_OK) return s;
      if (job.n) {
        c.phase = PH_R1_AFTER_K;
        return CABS_OK;
      }
      s = sketch_middle(c);
      if (s != CABS_OK) return s;
      c.phase = PH_R2_AFTER_W;
      return sketch_followup_eval(c, job);
    case PH_R1_AFTER_K:
      s = round_after_k(c, S.r1, pl.p1);
      if (s != CABS_OK) return s;
      s = sketch_middle(c);
      if (s != CABS_OK) return s;
      c.phase = PH_R2_AFTER_W;
      return sketch_followup_eval(c, job);
    case PH_R2_AFTER_W:
      s = round_after_w(c, S.r2, pl.kr2, pl.kc2, out->C, out->Rt, fac, fac, CABS_DIAG_RANK_FINAL,
                        CABS_DIAG_SIGMA1_FINAL, job);
      if (s != CABS_OK) return s;
      if (job.n) {
        c.phase = PH_R2_AFTER_K;
        return CABS_OK;
      }
      c.phase = PH_DONE;
      return sketch_final(c);
    case PH_R2_AFTER_K:
      s = round_after_k(c, S.r2, pl.p2);
      if (s != CABS_OK) return s;
      c.phase = PH_DONE;
      return sketch_final(c);
    default:
      return fail(CABS_EINVAL, "sketch already finished");
  }
}

static hipError_t run_svd_job(const SvdJob* const* jobs, int njobs, hipStream_t st) {
  SvdItems it{};
  int n = 0;
  for (int q = 0; q < njobs; ++q)
    for (int i = 0; i < jobs[q]->n; ++i) {
      if (n >= SVD_MAX_PTR) return hipErrorInvalidValue;
      it.Ap[n] = jobs[q]->A[i];
      it.Up[n] = jobs[q]->U[i];
      it.Sp[n] = jobs[q]->S[i];
      it.Vp[n] = jobs[q]->V[i];
      it.Wp[n] = jobs[q]->W[i];
      ++n;
    }
  it.n_ptr = n;
  return launch_svd_items(n, jobs[0]->rows, jobs[0]->cols, it, st);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" size_t cabs_workspace_bytes(const cabs_matrix* mat, const cabs_params* prm) {
  if (check_params(mat, prm) != CABS_OK) return 0;
  SketchWs S;
  return plan_sketch(nullptr, make_plan(mat, prm), prm, S);
}

extern "C" cabs_status cabs_sketch(const cabs_matrix* mat, const cabs_params* prm, void* ws, size_t ws_bytes,
                                   cabs_result* out, void* stream) {
  SketchRun c;
  cabs_status s = sketch_begin(c, mat, prm, ws, ws_bytes, out, (hipStream_t)stream);
  if (s != CABS_OK) return s;
  for (;;) {
    SvdJob job;
    s = sketch_advance(c, job);
    if (s != CABS_OK) return s;
    if (job.n == 0) return CABS_OK;
    const SvdJob* jp = &job;
    HIP_TRY(run_svd_job(&jp, 1, c.st));
  }
}

// Same-shape requests run phase by phase, each on its own stream, with each
// SVD of the sketch batched into one launch on the first stream (the other
// streams join it before and wait for it after, through the caller's events).
namespace cabs {
bool sketch_groupable(const cabs_params* a, const cabs_params* b) {
  return a->k1_rows == b->k1_rows && a->k1_cols == b->k1_cols && a->k2_rows == b->k2_rows &&
         a->k2_cols == b->k2_cols && a->compute == b->compute && a->orthogonalize == b->orthogonalize &&
         a->want_factors == b->want_factors && a->follow_up == b->follow_up && a->want_factors == 0;
}

cabs_status sketch_group(int G, const cabs_matrix* const* mats, const cabs_params* const* prms,
                         cabs_result* const* outs, void* const* ws, const size_t* ws_bytes, const hipStream_t* streams,
                         const hipEvent_t* join_ev, hipEvent_t fork_ev, cabs_status* status) {
  if (G < 1 || G > 4) return fail(CABS_EINVAL, "group size must be in [1, 4]");
  std::vector<SketchRun> c(G);
  for (int g = 0; g < G; ++g) {
    status[g] = sketch_begin(c[g], mats[g], prms[g], ws[g], ws_bytes[g], outs[g], streams[g]);
    if (status[g] != CABS_OK) return status[g];
    if (g > 0 && !sketch_groupable(prms[0], prms[g])) return fail(CABS_EINVAL, "requests of different shapes");
  }
  for (;;) {
    SvdJob job[4];
    const SvdJob* jp[4];
    for (int g = 0; g < G; ++g) {
      status[g] = sketch_advance(c[g], job[g]);
      if (status[g] != CABS_OK) return status[g];
      jp[g] = &job[g];
    }
    if (job[0].n == 0) return CABS_OK;  // same phases for every member
    bool other = false;
    for (int g = 1; g < G; ++g) {
      if (streams[g] == streams[0]) continue;  // already ordered
      other = true;
      HIP_TRY(hipEventRecord(join_ev[g], streams[g]));
      HIP_TRY(hipStreamWaitEvent(streams[0], join_ev[g], 0));
    }
    HIP_TRY(run_svd_job(jp, G, streams[0]));
    if (other) {
      HIP_TRY(hipEventRecord(fork_ev, streams[0]));
      for (int g = 1; g < G; ++g)
        if (streams[g] != streams[0]) HIP_TRY(hipStreamWaitEvent(streams[g], fork_ev, 0));
    }
  }
}
}  // namespace cabs

extern "C" cabs_status cabs_sketch_batch(int32_t count, const cabs_matrix* mats, const cabs_params* prms,
                                         void* const* ws, const size_t* ws_bytes, cabs_result* outs, void* stream) {
  if (count < 1 || count > 4 || !mats || !prms || !ws || !ws_bytes || !outs)
    return fail(CABS_EINVAL, "need 1 <= count <= 4 and non-null arrays");
  for (int g = 1; g < count; ++g)
    if (!cabs::sketch_groupable(&prms[0], &prms[g]))
      return fail(CABS_EINVAL, "request %d differs in shape from request 0 (or wants the factor form)", g);
  if (count > 1 && prms[0].want_factors) return fail(CABS_EINVAL, "the factor form is not batched");
  const cabs_matrix* mp[4];
  const cabs_params* pp[4];
  cabs_result* op[4];
  hipStream_t sts[4];
  hipEvent_t evs[4] = {nullptr, nullptr, nullptr, nullptr};
  cabs_status gst[4];
  for (int g = 0; g < count; ++g) {
    mp[g] = &mats[g];
    pp[g] = &prms[g];
    op[g] = &outs[g];
    sts[g] = (hipStream_t)stream;
  }
  return cabs::sketch_group(count, mp, pp, op, ws, ws_bytes, sts, evs, nullptr, gst);
}

// ---------------------------------------------------------------------------
// Error metric
// ---------------------------------------------------------------------------
extern "C" size_t cabs_error_workspace_bytes(const cabs_matrix* mat, const cabs_params* prm, int64_t n_samples) {
  if (check_params(mat, prm) != CABS_OK || n_samples < 0) return 0;
  return error_ws_bytes(view_of(mat), prm->k2_cols, prm->k2_rows, prm->compute, n_samples);
}

extern "C" cabs_status cabs_error(const cabs_matrix* mat, const cabs_params* prm, const cabs_result* res,
                                  int64_t n_samples, uint64_t seed, void* ws, size_t ws_bytes, double* out3,
                                  void* stream) {
  cabs_status s = check_params(mat, prm);
  if (s != CABS_OK) return s;
  if (!res || !res->C || !res->Rt || !res->Umid || !out3) return fail(CABS_EINVAL, "null result buffers");
  if (n_samples < 0) return fail(CABS_EINVAL, "n_samples must be >= 0");
  if (!ws || ((uintptr_t)ws & 255)) return fail(CABS_EINVAL, "workspace must be non-null and 256-byte aligned");
  const MatView mv = view_of(mat);
  const size_t need = error_ws_bytes(mv, prm->k2_cols, prm->k2_rows, prm->compute, n_samples);
  if (ws_bytes < need) return fail(CABS_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  HIP_TRY(launch_error(mv, prm->k2_cols, prm->k2_rows, prm->compute, res->C, res->Umid, res->Rt, n_samples, seed, ws,
                       out3, (hipStream_t)stream));
  return CABS_OK;
}

// ---------------------------------------------------------------------------
// Bilateral resampling CUR (Algorithm 1): Umid = Cbar^+ M Rbar^+, or W^+ when
// the target sample is the base sample (Eq. W).
// ---------------------------------------------------------------------------
namespace {

__global__ void brcur_diag_init_kernel(double* __restrict__ diag) {
  if (threadIdx.x < CABS_BRCUR_DIAG_LEN) diag[threadIdx.x] = 0.0;
}

// Reciprocals of the kept singular values (descending S of a rows x cols
// matrix): sigma_i > tol and i < cap (cap > 0); 0 for the dropped ones.
__global__ void pinv_scale_kernel(int p, int rows, int cols, const double* __restrict__ S, double rtol, int cap,
                                  double* __restrict__ inv, double* __restrict__ diag, int slot_rank, int slot_sig,
                                  int slot_rank2, int slot_sig2) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  const double s1 = S[0];
  const double tol = (rtol > 0.0 ? rtol : (double)(rows > cols ? rows : cols) * eps) * s1;
  for (int i = threadIdx.x; i < p; i += blockDim.x) {
    const bool keep = s1 > 0.0 && S[i] > tol && (cap <= 0 || i < cap);
    inv[i] = keep ? 1.0 / S[i] : 0.0;
    if (keep) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    diag[slot_rank] = (double)cnt;
    diag[slot_sig] = s1;
    if (slot_rank2 >= 0) diag[slot_rank2] = (double)cnt;
    if (slot_sig2 >= 0) diag[slot_sig2] = s1;
    if (cnt == 0) diag[CABS_BRCUR_DIAG_STATUS] = (double)CABS_ERANK;
  }
}

template <typename TC>
__global__ __launch_bounds__(256) void widen_f64_kernel(int64_t n, const TC* __restrict__ in, double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) out[e] = to_f64(in[e]);
}

static hipError_t launch_widen_f64(int prec, int64_t n, const void* in, double* out, hipStream_t st) {
  const dim3 g((unsigned)std::min<int64_t>(ceil_div(n, 256), 4096)), b(256);
  switch (prec) {
    case P_F32: hipLaunchKernelGGL(widen_f64_kernel<float>, g, b, 0, st, n, (const float*)in, out); break;
    case P_BF16: hipLaunchKernelGGL(widen_f64_kernel<bf16>, g, b, 0, st, n, (const bf16*)in, out); break;
    case P_F16: hipLaunchKernelGGL(widen_f64_kernel<f16>, g, b, 0, st, n, (const f16*)in, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

struct BrWs {
  double *Cb, *U1, *S1, *V1, *inv1;            // Cbar (W when the samples coincide) and its SVD
  double *Rb, *U2, *S2, *V2, *inv2;            // Rbar^T and its SVD
  double *M64, *T1, *T2, *T3, *diag;
  void *Mtc, *blk_ws, *svd_ws;
};

static size_t plan_brcur(void* ws, const MatView& mv, const cabs_brcur_params* prm, bool same, BrWs& B) {
  Carve cv(ws);
  B = BrWs{};
  const int kbr = prm->kb_rows, kbc = prm->kb_cols;
  const int ktr = same ? kbr : prm->kt_rows, ktc = same ? kbc : prm->kt_cols;
  const int p1 = std::min(ktr, kbc), p2 = std::min(ktc, kbr);
  B.Cb = cv.take<double>((size_t)ktr * kbc);
  B.U1 = cv.take<double>((size_t)ktr * p1);
  B.S1 = cv.take<double>(p1);
  B.V1 = cv.take<double>((size_t)kbc * p1);
  B.inv1 = cv.take<double>(p1);
  B.diag = cv.take<double>(CABS_BRCUR_DIAG_LEN);
  size_t svd_b = svd_ws_bytes(1, ktr, kbc);
  if (!same) {
    B.Rb = cv.take<double>((size_t)ktc * kbr);
    B.U2 = cv.take<double>((size_t)ktc * p2);
    B.S2 = cv.take<double>(p2);
    B.V2 = cv.take<double>((size_t)kbr * p2);
    B.inv2 = cv.take<double>(p2);
    B.M64 = cv.take<double>((size_t)ktr * ktc);
    B.Mtc = prm->compute == CABS_F64 ? (void*)B.M64 : cv.take_bytes((size_t)ktr * ktc * prec_bytes(prm->compute));
    B.T1 = cv.take<double>((size_t)p1 * ktc);
    B.T2 = cv.take<double>((size_t)p1 * p2);
    B.T3 = cv.take<double>((size_t)kbc * p2);
    B.blk_ws = cv.take_bytes(eval_block_ws_bytes(mv, ktr));
    svd_b = std::max(svd_b, svd_ws_bytes(1, ktc, kbr));
  }
  B.svd_ws = cv.take_bytes(svd_b);
  return cv.off + 256;
}

static cabs_status check_brcur(const cabs_matrix* mat, const cabs_brcur_params* prm, bool same) {
  cabs_status s = check_matrix(mat);
  if (s != CABS_OK) return s;
  if (!prm) return fail(CABS_EINVAL, "null parameters");
  s = check_compute(mat, prm->compute);
  if (s != CABS_OK) return s;
  if (prm->kb_rows < 1 || prm->kb_rows > 1024 || prm->kb_cols < 1 || prm->kb_cols > 1024)
    return fail(CABS_EINVAL, "base sample sizes must be in [1, 1024]");
  if (prm->kb_rows > mat->m || prm->kb_cols > mat->n) return fail(CABS_EINVAL, "base sample size exceeds the dimension");
  if (!same) {
    if (prm->kt_rows < 1 || prm->kt_rows > 4096 || prm->kt_cols < 1 || prm->kt_cols > 4096)
      return fail(CABS_EINVAL, "target sample sizes must be in [1, 4096]");
    if (prm->kt_rows > mat->m || prm->kt_cols > mat->n)
      return fail(CABS_EINVAL, "target sample size exceeds the dimension");
  }
  if (prm->rank_cap < 0) return fail(CABS_EINVAL, "rank_cap must be >= 0");
  if (prm->flags != 0) return fail(CABS_EINVAL, "unknown flag bits");
  return CABS_OK;
}

}  // namespace

extern "C" size_t cabs_brcur_workspace_bytes(const cabs_matrix* mat, const cabs_brcur_params* prm,
                                             int32_t same_sample) {
  if (check_brcur(mat, prm, same_sample != 0) != CABS_OK) return 0;
  BrWs B;
  return plan_brcur(nullptr, view_of(mat), prm, same_sample != 0, B);
}

extern "C" cabs_status cabs_brcur(const cabs_matrix* mat, const cabs_brcur_params* prm, const int64_t* base_r,
                                  const int64_t* base_c, const int64_t* tgt_r, const int64_t* tgt_c, void* ws,
                                  size_t ws_bytes, void* C, void* Rt, double* Umid, double* diag, void* stream) {
  if ((tgt_r == nullptr) != (tgt_c == nullptr)) return fail(CABS_EINVAL, "give both target samples or neither");
  const bool same = tgt_r == nullptr;
  cabs_status s = check_brcur(mat, prm, same);
  if (s != CABS_OK) return s;
  if (!base_r || !base_c || !C || !Rt || !Umid) return fail(CABS_EINVAL, "base samples, C, Rt and Umid are required");
  if (!ws || ((uintptr_t)ws & 255)) return fail(CABS_EINVAL, "workspace must be non-null and 256-byte aligned");
  const MatView mv = view_of(mat);
  BrWs B;
  const size_t need = plan_brcur(nullptr, mv, prm, same, B);
  if (ws_bytes < need) return fail(CABS_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  plan_brcur(ws, mv, prm, same, B);
  hipStream_t st = (hipStream_t)stream;
  double* dg = diag ? diag : B.diag;
  const int prec = prm->compute;
  const int kbr = prm->kb_rows, kbc = prm->kb_cols;
  hipLaunchKernelGGL(brcur_diag_init_kernel, dim3(1), dim3(64), 0, st, dg);
  HIP_TRY(hipGetLastError());
  // step 1: the bases C = A(:, Ib_c), R^T = A(Ib_r, :)^T
  HIP_TRY(launch_eval(mv, false, base_c, kbc, prec, C, st));
  HIP_TRY(launch_eval(mv, true, base_r, kbr, prec, Rt, st));
  if (same) {
    // Eq. (W): W = C(Ib_r, :), Umid = V_w diag(1 / sigma) U_w^T over the kept components
    const int p = std::min(kbr, kbc);
    HIP_TRY(launch_gather_rows_f64(C, prec, kbc, base_r, kbr, kbc, B.Cb, st));
    HIP_TRY(launch_svd(1, kbr, kbc, B.Cb, 0, B.U1, 0, B.S1, 0, B.V1, 0, B.svd_ws, st));
    hipLaunchKernelGGL(pinv_scale_kernel, dim3(1), dim3(1024), 0, st, p, kbr, kbc, B.S1, prm->pinv_rtol,
                       prm->rank_cap, B.inv1, dg, (int)CABS_BRCUR_DIAG_RANK_C, (int)CABS_BRCUR_DIAG_SIGMA1_C,
                       (int)CABS_BRCUR_DIAG_RANK_R, (int)CABS_BRCUR_DIAG_SIGMA1_R);
    HIP_TRY(hipGetLastError());
    HIP_TRY(launch_small_gemm(kbc, kbr, p, B.V1, p, false, B.U1, p, true, nullptr, B.inv1, nullptr, Umid, kbr, st));
    return CABS_OK;
  }
  const int ktr = prm->kt_rows, ktc = prm->kt_cols;
  const int p1 = std::min(ktr, kbc), p2 = std::min(ktc, kbr);
  // step 2: the bases on the target sample, Cbar (kt_r x kb_c) and Rbar^T (kt_c x kb_r), in FP64
  HIP_TRY(launch_gather_rows_f64(C, prec, kbc, tgt_r, ktr, kbc, B.Cb, st));
  HIP_TRY(launch_gather_rows_f64(Rt, prec, kbr, tgt_c, ktc, kbr, B.Rb, st));
  // step 3: the target block M = A(It_r, It_c)
  HIP_TRY(launch_eval_block(mv, tgt_r, ktr, tgt_c, ktc, prec, B.Mtc, B.blk_ws, st));
  if (prec != CABS_F64) HIP_TRY(launch_widen_f64(prec, (int64_t)ktr * ktc, B.Mtc, B.M64, st));
  // step 4: Cbar = U1 S1 V1^T, Rbar^T = U2 S2 V2^T (so Rbar^+ = U2 S2^-1 V2^T);
  //   Umid = V1 S1^-1 (U1^T M U2) S2^-1 V2^T
  HIP_TRY(launch_svd(1, ktr, kbc, B.Cb, 0, B.U1, 0, B.S1, 0, B.V1, 0, B.svd_ws, st));
  hipLaunchKernelGGL(pinv_scale_kernel, dim3(1), dim3(1024), 0, st, p1, ktr, kbc, B.S1, prm->pinv_rtol,
                     prm->rank_cap, B.inv1, dg, (int)CABS_BRCUR_DIAG_RANK_C, (int)CABS_BRCUR_DIAG_SIGMA1_C, -1, -1);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_svd(1, ktc, kbr, B.Rb, 0, B.U2, 0, B.S2, 0, B.V2, 0, B.svd_ws, st));
  hipLaunchKernelGGL(pinv_scale_kernel, dim3(1), dim3(1024), 0, st, p2, ktc, kbr, B.S2, prm->pinv_rtol,
                     prm->rank_cap, B.inv2, dg, (int)CABS_BRCUR_DIAG_RANK_R, (int)CABS_BRCUR_DIAG_SIGMA1_R, -1, -1);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_small_gemm(p1, ktc, ktr, B.U1, p1, true, B.M64, ktc, false, B.inv1, nullptr, nullptr, B.T1, ktc, st));
  HIP_TRY(launch_small_gemm(p1, p2, ktc, B.T1, ktc, false, B.U2, p2, false, nullptr, nullptr, B.inv2, B.T2, p2, st));
  HIP_TRY(launch_small_gemm(kbc, p2, p1, B.V1, p1, false, B.T2, p2, false, nullptr, nullptr, nullptr, B.T3, p2, st));
  HIP_TRY(launch_small_gemm(kbc, kbr, p2, B.T3, p2, false, B.V2, p2, true, nullptr, nullptr, nullptr, Umid, kbr, st));
  return CABS_OK;
}

// ---------------------------------------------------------------------------
// Stage entry points
// ---------------------------------------------------------------------------
extern "C" cabs_status cabs_sample(int64_t n, int32_t k, uint64_t seed, int32_t stream_id, int64_t* out, void* stream) {
  if (!out) return fail(CABS_EINVAL, "null output");
  if (k <= 0 || k > 4096 || (int64_t)k > n) return fail(CABS_EINVAL, "need 0 < k <= min(n, 4096)");
  if (stream_id < 0) return fail(CABS_EINVAL, "stream id must be >= 0");
  HIP_TRY(launch_sample(n, k, seed, stream_id, out, (hipStream_t)stream));
  return CABS_OK;
}

static cabs_status eval_common(const cabs_matrix* mat, const int64_t* idx, int32_t k, int32_t compute, void* out,
                               void* stream, bool rows_t) {
  cabs_status s = check_matrix(mat);
  if (s != CABS_OK) return s;
  s = check_compute(mat, compute);
  if (s != CABS_OK) return s;
  if (!idx || !out) return fail(CABS_EINVAL, "null index or output");
  const int64_t lim = rows_t ? mat->m : mat->n;
  if (k <= 0 || k > lim) return fail(CABS_EINVAL, "k out of range");
  HIP_TRY(launch_eval(view_of(mat), rows_t, idx, k, compute, out, (hipStream_t)stream));
  return CABS_OK;
}

extern "C" cabs_status cabs_eval_cols(const cabs_matrix* mat, const int64_t* idx, int32_t k, int32_t compute, void* out,
                                      void* stream) {
  return eval_common(mat, idx, k, compute, out, stream, false);
}

extern "C" cabs_status cabs_eval_rows_t(const cabs_matrix* mat, const int64_t* idx, int32_t k, int32_t compute,
                                        void* out, void* stream) {
  return eval_common(mat, idx, k, compute, out, stream, true);
}

static bool svd_shape_ok(int32_t batch, int32_t rows, int32_t cols) {
  return batch > 0 && rows > 0 && cols > 0 && std::min(rows, cols) <= 1024 && std::max(rows, cols) <= 4096;
}

extern "C" size_t cabs_svd_workspace_bytes(int32_t batch, int32_t rows, int32_t cols) {
  if (!svd_shape_ok(batch, rows, cols)) return 0;
  return svd_ws_bytes(batch, rows, cols);
}

extern "C" cabs_status cabs_svd_ex(int32_t batch, int32_t rows, int32_t cols, const double* A, double* U, double* S,
                                   double* V, void* ws, size_t ws_bytes, int32_t fast_sweeps, void* stream) {
  if (!svd_shape_ok(batch, rows, cols))
    return fail(CABS_EINVAL, "need batch > 0, 0 < min(rows, cols) <= 1024 and max(rows, cols) <= 4096");
  if (fast_sweeps < 0 || fast_sweeps > 24) return fail(CABS_EINVAL, "need 0 <= fast_sweeps <= 24");
  if (!A || !U || !S || !V || !ws) return fail(CABS_EINVAL, "null pointer");
  if (ws_bytes < svd_ws_bytes(batch, rows, cols)) return fail(CABS_ENOMEM, "workspace too small");
  const int64_t p = rows < cols ? rows : cols;
  HIP_TRY(launch_svd(batch, rows, cols, A, (int64_t)rows * cols, U, (int64_t)rows * p, S, p, V, (int64_t)cols * p, ws,
                     (hipStream_t)stream, fast_sweeps));
  return CABS_OK;
}

extern "C" cabs_status cabs_svd(int32_t batch, int32_t rows, int32_t cols, const double* A, double* U, double* S,
                                double* V, void* ws, size_t ws_bytes, void* stream) {
  return cabs_svd_ex(batch, rows, cols, A, U, S, V, ws, ws_bytes, 0, stream);
}

extern "C" size_t cabs_kmeans_workspace_bytes(int64_t rows, int32_t dim, int32_t k, int32_t compute) {
  if (rows <= 0 || dim <= 0 || dim > 1024 || k <= 0 || k > 1024 || k > rows || !valid_prec(compute)) return 0;
  return kmeans_ws_bytes(rows, dim, k, compute);
}

extern "C" cabs_status cabs_kmeans(int64_t rows, int32_t dim, int32_t k, int32_t compute, const void* P, const double* w,
                                   const double* Z0, int32_t iters, double* Z, int32_t* labels, double* obj2,
                                   int64_t* snap_out, void* ws, size_t ws_bytes, void* stream) {
  if (rows <= 0 || rows >= (int64_t)1 << 31 || dim <= 0 || dim > 1024 || k <= 0 || k > 1024 || k > rows)
    return fail(CABS_EINVAL, "need 0 < k <= min(rows, 1024), 0 < dim <= 1024");
  if (!valid_prec(compute)) return fail(CABS_EINVAL, "unknown precision");
  if (!P || !w || !Z0 || !Z || !ws) return fail(CABS_EINVAL, "null pointer");
  if (iters < 0) return fail(CABS_EINVAL, "iters must be >= 0");
  if (ws_bytes < kmeans_ws_bytes(rows, dim, k, compute)) return fail(CABS_ENOMEM, "workspace too small");
  KMeansOut o{Z, labels, obj2, nullptr, nullptr, snap_out, nullptr};
  HIP_TRY(launch_kmeans(rows, dim, k, compute, P, w, Z0, iters, o, ws, (hipStream_t)stream));
  return CABS_OK;
}

// ---------------------------------------------------------------------------
// cabs_kmeans_noalloc: cabs_kmeans with its scratch in a fixed device array
// ---------------------------------------------------------------------------
// The array lives in the library's code object, one copy per device, for the
// life of the process.  Host code never passes its name to a kernel (in host
// code the name is only a stand-in): the device address of each device's copy
// is looked up once, with that device current, and kept.  Nothing in the
// k-means kernels needs the scratch to start at zero (every buffer they read is
// written earlier in the same call), so consecutive calls need no clearing.
static __device__ __align__(256) unsigned char scratch[CABS_KMEANS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static cabs_status scratch_on_current_device(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(CABS_EDEVICE, "device index %d out of range", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(CABS_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CABS_OK;
}

extern "C" cabs_status cabs_kmeans_noalloc(int64_t rows, int32_t dim, int32_t k, int32_t compute, const void* P,
                                           const double* w, const double* Z0, int32_t iters, double* Z,
                                           int32_t* labels, double* obj2, int64_t* snap_out, void* stream) {
  if (rows <= 0 || rows >= (int64_t)1 << 31 || dim <= 0 || dim > 1024 || k <= 0 || k > 1024 || k > rows)
    return fail(CABS_EINVAL, "need 0 < k <= min(rows, 1024), 0 < dim <= 1024");
  if (!valid_prec(compute)) return fail(CABS_EINVAL, "unknown precision");
  if (!P || !w || !Z0 || !Z) return fail(CABS_EINVAL, "null pointer");
  if (iters < 0) return fail(CABS_EINVAL, "iters must be >= 0");
  const size_t need = kmeans_ws_bytes(rows, dim, k, compute, true);
  if (need > (size_t)CABS_KMEANS_NOALLOC_SCRATCH_BYTES)
    return fail(CABS_ENOMEM, "cabs_kmeans_noalloc: needs %zu bytes of scratch, the fixed array holds %zu", need,
                (size_t)CABS_KMEANS_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  const cabs_status s = scratch_on_current_device(&ws);
  if (s != CABS_OK) return s;
  KMeansOut o{Z, labels, obj2, nullptr, nullptr, snap_out, nullptr};
  HIP_TRY(launch_kmeans(rows, dim, k, compute, P, w, Z0, iters, o, ws, (hipStream_t)stream, true));
  return CABS_OK;
}
