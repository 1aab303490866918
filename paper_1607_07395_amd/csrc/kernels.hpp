// Host-side launchers of the CABS device kernels (internal to libcabs).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cabs {

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_F16 = 3 };
enum Src { SRC_DENSE = 0, SRC_LOWRANK = 1, SRC_RBF = 2, SRC_CSR = 3 };

inline size_t prec_bytes(int p) { return p == P_F64 ? 8 : p == P_F32 ? 4 : 2; }

// Matrix descriptor as the kernels see it.
struct MatView {
  int kind;
  int storage;
  int64_t m, n;
  const void* a;
  int64_t lda;
  const void* pf;
  const void* qf;
  const void* s;
  int r;
  double noise_std;
  uint64_t noise_seed;
  const void* x;
  const void* y;
  int d;
  double sigma;
  const int64_t* row_ptr;  // CSR: the nonzeros in row order and in column order
  const int32_t* col_idx;
  const void* vals;
  const int64_t* col_ptr;
  const int32_t* row_idx;
  const void* vals_t;
  int64_t nnz;
};

// Entry (i, j) of a CSR source: a binary search of row i's ascending columns.
template <typename TIn>
__device__ __forceinline__ double csr_entry(const MatView& mv, int64_t i, int64_t j) {
  int64_t lo = mv.row_ptr[i], hi = mv.row_ptr[i + 1];  // search [lo, hi)
  const int32_t jj = (int32_t)j;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (mv.col_idx[mid] < jj) lo = mid + 1;
    else hi = mid;
  }
  return (lo < mv.row_ptr[i + 1] && mv.col_idx[lo] == jj) ? (double)((const TIn*)mv.vals)[lo] : 0.0;
}

// --- sampling / entry evaluation (eval.hip) ---
hipError_t launch_sample(int64_t n, int k, uint64_t seed, int stream_id, int64_t* out, hipStream_t st);
// rows_t = false: out (m x k) = A(:, idx); rows_t = true: out (n x k) = A(idx, :)^T.
// counter (may be null): every entry evaluated or read is added to it on the device.
hipError_t launch_eval(const MatView& mv, bool rows_t, const int64_t* idx, int k, int compute, void* out,
                       hipStream_t st, unsigned long long* counter = nullptr);
// out (kr x kc, row-major, compute precision) = A(ri, ci): the target block of the resampling CUR.
// ws: eval_block_ws_bytes(mv, kr) bytes (the generator rows of ri, for the low-rank and RBF sources).
size_t eval_block_ws_bytes(const MatView& mv, int kr);
hipError_t launch_eval_block(const MatView& mv, const int64_t* ri, int kr, const int64_t* ci, int kc, int compute,
                             void* out, void* ws, hipStream_t st);
// out (k x ncols, FP64) = src[idx[i], :] for a compute-precision row-major src with row stride ld.
hipError_t launch_gather_rows_f64(const void* src, int compute, int64_t ld, const int64_t* idx, int k, int ncols,
                                  double* out, hipStream_t st);

// --- hard-threshold follow-up selection (select.hip) ---
// The k (1..1024) rows with the largest weights w (ties to the lower row, NaN last), written
// ascending to out (device int64); rows < 2^31 - 1.
size_t select_ws_bytes(int64_t rows);
hipError_t launch_select_topk(int64_t rows, const double* w, int k, int64_t* out, void* ws, hipStream_t st);

// --- FP64 small dense algebra (svd.hip, small.hip) ---
size_t svd_ws_bytes(int batch, int rows, int cols);
size_t svd_ws_item_doubles(int rows, int cols);  // one item's share of svd_ws_bytes, in doubles
// Batched one-sided Jacobi SVD; A_b rows x cols row-major, strides in elements between batch items.
// fast_sweeps (1 .. 24): sweeps launched round by round before the single-workgroup finisher;
// 0: 12 up to min(rows, cols) = 256, 24 above.
// Item b of a batched SVD: A_b, U_b, S_b, V_b and its workspace (svd_ws_doubles
// per item) at fixed strides from the base pointers, or, with n_ptr = batch
// (at most SVD_MAX_PTR), from the pointer lists.
constexpr int SVD_MAX_PTR = 8;
struct SvdItems {
  const double* A;
  double *U, *S, *V, *W;
  int64_t sA, sU, sS, sV, sW;
  int n_ptr;
  const double* Ap[SVD_MAX_PTR];
  double* Up[SVD_MAX_PTR];
  double* Sp[SVD_MAX_PTR];
  double* Vp[SVD_MAX_PTR];
  double* Wp[SVD_MAX_PTR];
};
hipError_t launch_svd_items(int batch, int rows, int cols, const SvdItems& it, hipStream_t st, int fast_sweeps = 0);
hipError_t launch_svd(int batch, int rows, int cols, const double* A, int64_t strideA, double* U, int64_t strideU,
                      double* S, int64_t strideS, double* V, int64_t strideV, void* ws, hipStream_t st,
                      int fast_sweeps = 0);

// C (M x N) = alpha * op(A) diag(dl) ... : general small FP64 product
//   C = diag(dl) * op(A) * diag(dm) * op(B) * diag(dr)   (any diag pointer may be null)
// op(A) is M x K: A row-major (lda) or its transpose; same for B (K x N).
hipError_t launch_small_gemm(int M, int N, int K, const double* A, int lda, bool transA, const double* B, int ldb,
                             bool transB, const double* dl, const double* dm, const double* dr, double* C, int ldc,
                             hipStream_t st);

// Pivoted Cholesky of `batch` PSD p x p matrices (p <= 1024): Rf row k = R's row k with columns in the
// original order, rows from the numerical rank on zero (pivots <= tol stop the factorisation).  Up to
// PCHOL_MAXP one work-group per matrix holds it in registers; above, one launch per step over many
// work-groups, in ws (pchol_ws_bytes(batch, p) bytes).
size_t pchol_ws_bytes(int batch, int p);
hipError_t launch_pchol(int batch, int p, const double* G, int64_t strideG, double tol, double* Rf, int64_t strideR,
                        void* ws, hipStream_t st);
constexpr int PCHOL_MAXP = 204;

// --- tall-skinny products, Grams, norms (tsgemm.hip) ---
// Y (M x N, compute) = X (M x K, compute) * B (K x N, FP64); B is converted to the compute
// precision into bt_ws (N x K).  colsq (N, FP64) receives column sums of squares of Y when
// non-null (partials in part_ws: ceil(M/64) x N doubles); rowsq (M, FP64) row sums of squares.
// Y may be null (norms only).
size_t tsgemm_ws_bytes(int64_t M, int K, int N, int compute);
hipError_t launch_tsgemm(int64_t M, int K, int N, int compute, const void* X, const double* B, void* Y,
                         double* colsq, double* rowsq, void* ws, hipStream_t st);
// G (K x K, FP64) = X^T X for X (M x K, compute precision); deterministic two-stage reduction.
size_t gram_ws_bytes(int64_t M, int K);
hipError_t launch_gram(int64_t M, int K, int compute, const void* X, double* G, void* ws, hipStream_t st);

// --- weighted k-means and snapping (kmeans.hip) ---
// lean: the layout without the final assignment's stored dot products, from
// which the snap otherwise takes its distances (its top-T pass then forms them).
size_t kmeans_ws_bytes(int64_t rows, int dim, int k, int compute, bool lean = false);
struct KMeansOut {
  double* Z;         // k x dim FP64 (in: Z0 if z0 == nullptr)
  int32_t* labels;   // rows (may be null)
  double* obj2;      // {objective at Z0, objective at final Z} (may be null)
  double* tmax;      // largest cluster of the final assignment (may be null)
  double* gap;       // smallest best/second-best gap of the final assignment (may be null)
  int64_t* snap;     // k snapped rows, ascending (may be null)
  double* fallbacks; // number of centres resolved by a full scan (may be null)
};
hipError_t launch_kmeans(int64_t rows, int dim, int k, int compute, const void* P, const double* w,
                         const double* Z0, int iters, const KMeansOut& out, void* ws, hipStream_t st,
                         bool lean = false);

// --- error metric (error.hip) ---
size_t error_ws_bytes(const MatView& mv, int k2c, int k2r, int compute, int64_t n_samples);
hipError_t launch_error(const MatView& mv, int k2c, int k2r, int compute, const void* C, const double* Umid,
                        const void* Rt, int64_t n_samples, uint64_t seed, void* ws, double* out3, hipStream_t st);

}  // namespace cabs
