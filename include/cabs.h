/*
 * cabs.h -- C ABI of libcabs, a GPU (AMD MI355X, gfx950) implementation of the
 * data-parallel hot path of cascaded bilateral sampling (CABS): Zhang, Liu,
 * Zhang, Xiong, Xing, Ye, "Seeing the forest from the trees in two looks:
 * matrix sketching by cascaded bilateral sampling", arXiv:1607.07395.
 *
 * The problem (paper, Section 1): approximate an m x n matrix A that is only
 * accessible through the rows and columns one asks for, in O(m + n) time and
 * memory, by a small set of its own rows and columns.  The method (Algorithm 2):
 * a uniformly sampled pilot sketch gives row and column embeddings P, Q; a
 * weighted k-means on each (Section 3.2) picks representative rows and columns;
 * the sketching routine of Section 4.1 turns them into A ~ C Umid R.
 *
 * Conventions for every call below
 *   - Array arguments are DEVICE pointers unless the comment says "host".
 *     The caller owns every buffer; the library allocates nothing inside a call
 *     (scratch comes from the caller's workspace).
 *   - Matrices are row-major.  Sampled rows are stored transposed: R^T is n x k.
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL =
 *     the default stream).  Outputs are valid once the stream has reached the
 *     end of the call's work.  The host-side return value only reports argument
 *     and launch errors; conditions found on the device (rank loss) are written
 *     to the result's `diag` array.
 *   - Every call is deterministic: the same arguments give bitwise the same
 *     outputs (all reductions run in a fixed order; no floating-point atomics).
 *   - On error no work is enqueued and cabs_last_error() describes the problem.
 */
#ifndef CABS_H
#define CABS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CABS_OK = 0,
  CABS_EINVAL = -1,     /* bad argument: null pointer, size out of range, unsupported combination */
  CABS_ENOMEM = -2,     /* workspace (or serving memory budget) too small */
  CABS_ERANK = -3,      /* W has no singular value above the threshold (reported in diag[0]) */
  CABS_EDEVICE = -4,    /* a HIP call failed */
  CABS_EBUSY = -5,      /* serving: request not finished yet */
  CABS_ECANCELED = -6   /* serving: request was cancelled */
} cabs_status;

/* Arithmetic precisions.  SVDs, pivoted Cholesky factorisations, Grams for the
 * orthogonalisation and all k x k algebra always run in FP64. */
typedef enum { CABS_F64 = 0, CABS_F32 = 1, CABS_BF16 = 2, CABS_F16 = 3 } cabs_prec;

/* How entries of A are obtained. */
typedef enum {
  CABS_SRC_DENSE = 0,   /* A stored row-major with leading dimension lda; sampled rows are
                           gathered with coalesced row reads, sampled columns through LDS tiles */
  CABS_SRC_LOWRANK = 1, /* A_ij = sum_t pf[i,t] s[t] qf[j,t] + noise_std * g(noise_seed, i, j),
                           g a standard normal by Box-Muller on Philox-4x32-10 at counter
                           (lo i, hi i, lo j, hi j), key (lo noise_seed, hi noise_seed): words
                           1:0 give u1 in (0, 1], words 3:2 u2 in [0, 1); E is never stored */
  CABS_SRC_RBF = 2,     /* A_ij = exp(-|x_i - y_j|^2 / (2 sigma^2)) */
  CABS_SRC_CSR = 3      /* sparse A, its nonzeros in both CSR and CSC order */
} cabs_src;

/* The monotone weight Upsilon(|P_l|) of the weighted k-means objective
 * (Section 3.2): 1, |p|^param, 1/(1+exp(-param |p|)), or [|p| >= param]. */
typedef enum { CABS_W_CONST = 0, CABS_W_POW = 1, CABS_W_SIGMOID = 2, CABS_W_STEP = 3 } cabs_weight;

/* Follow-up sampling (Algorithm 2, step 3).  KMEANS: weighted k-means on the
 * pilot embeddings from the pilot sample, then each centre snapped to its
 * nearest untaken row (Section 3.2).  HARD: the hard-threshold variant of
 * Section 5: the k2 rows (columns) with the largest weights Upsilon(|P_l|),
 * equal weights to the lower index, NaN weights last.  LEVERAGE: the
 * leverage variant of Section 5: k2 distinct rows (columns) drawn with
 * probabilities proportional to approximate leverage scores, the squared row
 * norms of the pilot sketch's left (right) factor (orthonormal when
 * `orthogonalize` is set, as the supplementary orthogonalisation section
 * intends) over the components whose singular value exceeds
 * p eps max (p = min(k1_rows, k1_cols)); drawn without replacement by
 * exponential races: row i gets the key ln(u_i) / score_i (-inf for score 0),
 * u_i in (0, 1] from word 0 of Philox-4x64-10 at counter (i, 0, 5, 0) for rows
 * and (i, 0, 6, 0) for columns, key (seed, 0), and the k2 largest keys are
 * taken, equal keys to the lower index.  HARD and LEVERAGE run no k-means and
 * leave the encoding-error diagnostics at 0; both need m, n < 2^31 - 1.
 * PILOT: no follow-up round; the output is the pilot sketch itself (step 2 of
 * Algorithm 2, the "pilot-sketch" method of Section 5's comparison): idx_r,
 * idx_c are the pilot sample, C, Rt, Umid its sketch; needs k2 = k1 on both
 * sides; only the FINAL rank and sigma diagnostics (copied to the PILOT slots)
 * are written. */
typedef enum {
  CABS_FOLLOW_KMEANS = 0,
  CABS_FOLLOW_HARD = 1,
  CABS_FOLLOW_LEVERAGE = 2,
  CABS_FOLLOW_PILOT = 3
} cabs_follow_up;

/* The sketching routine: the stabilised form of Section 4.1 (default), or the
 * pseudo-skeleton A ~ C W^+ R of Eq. (W), Section 2.2. */
typedef enum { CABS_SK_STABILIZED = 0, CABS_SK_PSEUDO_SKELETON = 1 } cabs_sketch_kind;

/* Descriptor of the input matrix (an entry generator or a dense array).
 * Table arrays (a, pf, qf, s, x, y) use precision `storage` (F64 or F32).
 * The compute precision must be F64 when storage is F64. */
typedef struct {
  int32_t kind;          /* cabs_src */
  int32_t storage;       /* cabs_prec of the table arrays: CABS_F64 or CABS_F32 */
  int64_t m, n;
  /* DENSE */
  const void* a;         /* m x n, row stride lda elements */
  int64_t lda;
  /* LOWRANK */
  const void* pf;        /* m x r */
  const void* qf;        /* n x r */
  const void* s;         /* r */
  int32_t r;
  int32_t reserved0;
  double noise_std;
  uint64_t noise_seed;
  /* RBF */
  const void* x;         /* m x d */
  const void* y;         /* n x d (may equal x) */
  int32_t d;
  int32_t reserved1;
  double sigma;
  /* CSR (the sparse matrices of Section 5, Table 1): the nonzeros of A twice,
   * so that sampled rows and sampled columns are both contiguous gathers.
   * row_ptr (m + 1, int64, row_ptr[0] = 0, row_ptr[m] = nnz), col_idx (nnz,
   * int32, strictly ascending within a row), vals (nnz, `storage`); col_ptr
   * (n + 1), row_idx (nnz, strictly ascending within a column), vals_t (nnz)
   * the same nonzeros in column order.  Entries not listed are 0.  The
   * library does not check that the two orders hold the same matrix. */
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const void* vals;
  const int64_t* col_ptr;
  const int32_t* row_idx;
  const void* vals_t;
  int64_t nnz;
} cabs_matrix;

/* Parameters of one sketch.  Sample sizes: pilot k1_rows x k1_cols (Algorithm 2,
 * pilot sampling), follow-up k2_rows x k2_cols (follow-up sampling); the output
 * rank is at most min(k2_rows, k2_cols). */
typedef struct {
  int32_t k1_rows, k1_cols, k2_rows, k2_cols;
  int32_t kmeans_iters;  /* c, Lloyd iterations per side (the paper uses 5) */
  int32_t weight_kind;   /* cabs_weight */
  double weight_param;
  int32_t sketch_kind;   /* cabs_sketch_kind */
  int32_t orthogonalize; /* 1: orthogonalise the pilot factors before embedding
                            (supplementary Section 3), in FP64 */
  double pinv_rtol;      /* components with sigma_i <= rtol * sigma_1 are dropped;
                            <= 0 selects max(kr, kc) * eps(FP64) */
  int32_t compute;       /* cabs_prec of entry evaluation, embeddings, distance GEMMs */
  int32_t want_factors;  /* 1: also produce the orthogonalised factor form (Uf, S, Vf) */
  int32_t follow_up;     /* cabs_follow_up: how the follow-up rows and columns are chosen */
  int32_t flags;         /* CABS_FLAG_* bits; all others must be 0 */
  uint64_t seed;         /* Philox key for every draw of the method */
} cabs_params;

/* cabs_params.flags.  COUNT_ENTRIES: the entry-evaluation kernels count, on
 * the device, every entry of A they evaluate or read (one integer atomic per
 * wavefront; a debugging aid, off by default) into CABS_DIAG_ENTRIES. */
enum { CABS_FLAG_COUNT_ENTRIES = 1 };

/* Diagnostic slots written to cabs_result.diag (doubles). */
enum {
  CABS_DIAG_STATUS = 0,        /* 0 or CABS_ERANK */
  CABS_DIAG_ENC_R_PILOT = 1,   /* weighted encoding error of the rows, pilot representatives (Section 3.1) */
  CABS_DIAG_ENC_C_PILOT = 2,
  CABS_DIAG_ENC_R_FINAL = 3,   /* ... after the last k-means iteration (before snapping) */
  CABS_DIAG_ENC_C_FINAL = 4,
  CABS_DIAG_TMAX_R = 5,        /* largest cluster size T (Section 3.1) */
  CABS_DIAG_TMAX_C = 6,
  CABS_DIAG_RANK_PILOT = 7,    /* kept components of the pilot sketch */
  CABS_DIAG_RANK_FINAL = 8,
  CABS_DIAG_ENTRIES = 9,       /* with CABS_FLAG_COUNT_ENTRIES: entries of A evaluated over both rounds,
                                  counted on the device (m k_c + n k_r per round; the k_r x k_c entries
                                  of W are evaluated twice, once in C and once in R^T, so the distinct
                                  entries touched are this minus k1_rows k1_cols + k2_rows k2_cols);
                                  -1 when not counted */
  CABS_DIAG_GAP_R = 10,        /* smallest nearest/second-nearest centre gap, final assignment */
  CABS_DIAG_GAP_C = 11,
  CABS_DIAG_SIGMA1_PILOT = 12, /* largest singular value of W, pilot and follow-up */
  CABS_DIAG_SIGMA1_FINAL = 13,
  CABS_DIAG_SNAP_SCANS_R = 14, /* centres whose snap needed a scan of every row (candidate lists exhausted) */
  CABS_DIAG_SNAP_SCANS_C = 15,
  CABS_DIAG_LEN = 16
};

/* Outputs of cabs_sketch.  All buffers are caller-owned device memory.
 * Element type of C, Rt, Uf, Vf is the compute precision. */
typedef struct {
  int64_t* idx_r;        /* [k2_rows] follow-up row indices, ascending */
  int64_t* idx_c;        /* [k2_cols] follow-up column indices, ascending */
  int64_t* pilot_r;      /* [k1_rows] pilot row indices, ascending (NULL: not returned) */
  int64_t* pilot_c;      /* [k1_cols] */
  void* C;               /* m x k2_cols: A(:, idx_c) */
  void* Rt;              /* n x k2_rows: A(idx_r, :)^T */
  double* Umid;          /* k2_cols x k2_rows: A ~ C Umid Rt^T */
  void* Uf;              /* m x kf (kf = min(k2_rows, k2_cols)), orthonormal columns; NULL unless want_factors */
  double* S;             /* kf singular values, descending */
  void* Vf;              /* n x kf */
  double* diag;          /* CABS_DIAG_LEN doubles (may be NULL) */
} cabs_result;

/* Library version string and the last error message of the calling thread. */
const char* cabs_version(void);
const char* cabs_last_error(void);

/* Bytes of workspace cabs_sketch needs for this matrix and these parameters
 * (0 on invalid arguments; see cabs_last_error). */
size_t cabs_workspace_bytes(const cabs_matrix* mat, const cabs_params* prm);

/* One CABS sketch (Algorithm 2): pilot sampling (Floyd on Philox, streams 0/1),
 * pilot evaluation of C = A(:, I^c) and R^T, W = C(I^r, :); the sketching
 * routine (Section 4.1) with an FP64 SVD of W; optional FP64 orthogonalisation
 * (supplementary Section 3); embeddings P = U S^(1/2), Q = V S^(1/2) with
 * weights Upsilon(|P_l|); c iterations of weighted k-means per side from the
 * pilot sample; snapping of every centre to the nearest untaken row; follow-up
 * evaluation and sketch.  ws must hold cabs_workspace_bytes() bytes, 256-byte
 * aligned.  Returns CABS_EINVAL for k > dimension, null required pointers or an
 * unsupported precision/source pair; CABS_ENOMEM if ws_bytes is too small. */
cabs_status cabs_sketch(const cabs_matrix* mat, const cabs_params* prm, void* ws, size_t ws_bytes,
                        cabs_result* out, void* stream);

/* cabs_sketch on `count` (1..4) requests of the same shape at once: equal
 * sample sizes, compute precision, orthogonalize and follow_up, and (for
 * count > 1) no factor form.  The requests' kernels run one after another on
 * `stream`, except that each FP64 SVD of the sketch (Section 4.1's W and the
 * orthogonalisation's) is one launch for all of them.  Request g has its own
 * matrix mats[g], parameters prms[g] (seeds may differ), workspace ws[g] of
 * ws_bytes[g] (cabs_workspace_bytes of that request) and outputs outs[g]; the
 * results are bitwise those of cabs_sketch.  CABS_EINVAL for a count outside
 * 1..4 or requests of different shapes; otherwise as cabs_sketch. */
cabs_status cabs_sketch_batch(int32_t count, const cabs_matrix* mats, const cabs_params* prms, void* const* ws,
                              const size_t* ws_bytes, cabs_result* outs, void* stream);

/* Relative Frobenius error |A - C Umid R|_F / |A|_F (the paper's error metric,
 * Section 5) of a finished sketch.  n_samples = 0: exact, over all m*n entries;
 * otherwise over n_samples i.i.d. uniform entries drawn with replacement from
 * Philox-4x32-10 at counter (lo t, hi t, 4, 0), key (lo seed, hi seed): sample t is
 * (mulhi(w, m), mulhi(w', n)) with w = words 1:0 and w' = words 3:2 as 64-bit integers.
 * out3 (device) receives {sum of squared residuals, sum of squared entries,
 * ratio}.  ws must hold cabs_error_workspace_bytes() bytes. */
size_t cabs_error_workspace_bytes(const cabs_matrix* mat, const cabs_params* prm, int64_t n_samples);
cabs_status cabs_error(const cabs_matrix* mat, const cabs_params* prm, const cabs_result* res,
                       int64_t n_samples, uint64_t seed, void* ws, size_t ws_bytes, double* out3,
                       void* stream);

/* ---- Bilateral resampling CUR (Algorithm 1, Section 2.2) ----
 *
 * The family of linear-cost sketches that the paper compares CABS with: a base
 * sample gives C = A(:, Ib_c) (m x kb_cols) and R^T = A(Ib_r, :)^T (n x kb_rows);
 * a target sample selects Cbar = C(It_r, :) (kt_rows x kb_cols), Rbar =
 * R(:, It_c) (kb_rows x kt_cols) and the block M = A(It_r, It_c); the middle
 * factor is the minimum-norm minimiser of |M - Cbar U Rbar|_F,
 *   Umid = Cbar^+ M Rbar^+   (kb_cols x kb_rows),  A ~ C Umid Rt^T.
 * Each pseudo-inverse comes from an FP64 SVD (cabs_svd) and drops the singular
 * values <= tol = (pinv_rtol > 0 ? pinv_rtol : max(rows, cols) eps) sigma_1,
 * and, if rank_cap > 0, all but the rank_cap largest.
 * tgt_r = tgt_c = NULL means the target sample IS the base sample: the
 * pseudo-skeleton Eq. (W), Umid = W^+ with W = A(Ib_r, Ib_c) read out of C
 * (one SVD, no block evaluation); with base_r = base_c on a square symmetric
 * positive semi-definite A this is the Nystrom method.  Sketch-CUR is the
 * general case with independently drawn samples (cabs_sample; the library's
 * convention: base from streams 0 / 1, target from streams 7 / 8, with a
 * target size three times the base size as in Section 5).
 * The C, Rt and Umid outputs have the layout of cabs_result, so cabs_error
 * takes them with k2_rows = kb_rows, k2_cols = kb_cols.
 * Indices are device int64 arrays (any order, repeats allowed) that must lie in
 * range: the call does not read them on the host.  Sizes: 1 <= kb <= 1024,
 * 1 <= kt <= 4096, kb and kt at most the dimension they sample.
 * diag (device, CABS_BRCUR_DIAG_LEN doubles, may be NULL): status (0 or
 * CABS_ERANK when a pseudo-inverse keeps nothing; Umid is then zero), kept
 * components and sigma_1 of Cbar and Rbar (of W twice when the samples
 * coincide). */
typedef struct {
  int32_t kb_rows, kb_cols;  /* base sample sizes: rows of R, columns of C */
  int32_t kt_rows, kt_cols;  /* target sample sizes (ignored when the target is the base) */
  int32_t compute;           /* cabs_prec of C, Rt and the block M; the solve is FP64 */
  int32_t rank_cap;          /* 0: every component above tol */
  double pinv_rtol;          /* <= 0: max(rows, cols) eps */
  int32_t flags;             /* must be 0 */
  int32_t reserved;
} cabs_brcur_params;

enum {
  CABS_BRCUR_DIAG_STATUS = 0,
  CABS_BRCUR_DIAG_RANK_C = 1,
  CABS_BRCUR_DIAG_RANK_R = 2,
  CABS_BRCUR_DIAG_SIGMA1_C = 3,
  CABS_BRCUR_DIAG_SIGMA1_R = 4,
  CABS_BRCUR_DIAG_LEN = 8
};

/* Workspace bytes of cabs_brcur (same_sample: 1 when the target is the base);
 * 0 on invalid arguments. */
size_t cabs_brcur_workspace_bytes(const cabs_matrix* mat, const cabs_brcur_params* prm, int32_t same_sample);
cabs_status cabs_brcur(const cabs_matrix* mat, const cabs_brcur_params* prm, const int64_t* base_r,
                       const int64_t* base_c, const int64_t* tgt_r, const int64_t* tgt_c, void* ws, size_t ws_bytes,
                       void* C, void* Rt, double* Umid, double* diag, void* stream);

/* ---- Stage entry points (the same kernels cabs_sketch runs, one at a time) ---- */

/* k distinct indices from [0, n), uniform, ascending (Floyd's algorithm on
 * Philox-4x64-10: draw t uses word 0 at counter (t, 0, stream_id, 0), key
 * (seed, 0)).  Pilot sampling of Algorithm 2.  Requires 0 < k <= n, k <= 4096. */
cabs_status cabs_sample(int64_t n, int32_t k, uint64_t seed, int32_t stream_id, int64_t* out, void* stream);

/* C = A(:, idx) (m x k) or R^T = A(idx, :)^T (n x k) in precision `compute`:
 * the sampled columns / rows of Algorithm 2.  idx: k device int64 in range. */
cabs_status cabs_eval_cols(const cabs_matrix* mat, const int64_t* idx, int32_t k, int32_t compute, void* out,
                           void* stream);
cabs_status cabs_eval_rows_t(const cabs_matrix* mat, const int64_t* idx, int32_t k, int32_t compute, void* out,
                             void* stream);

/* Batched FP64 SVD by one-sided Jacobi: A_b (rows x cols, row-major) =
 * U_b diag(S_b) V_b^T with p = min(rows, cols), U_b rows x p, V_b cols x p,
 * S_b descending, the largest-magnitude entry of every column of U_b positive.
 * Used on W in the sketching routine (Section 4.1) and on the target rows and
 * columns of the resampling CUR (Algorithm 1).  min(rows, cols) <= 1024,
 * max(rows, cols) <= 4096.
 * ws: cabs_svd_workspace_bytes() bytes. */
size_t cabs_svd_workspace_bytes(int32_t batch, int32_t rows, int32_t cols);
cabs_status cabs_svd(int32_t batch, int32_t rows, int32_t cols, const double* A, double* U, double* S, double* V,
                     void* ws, size_t ws_bytes, void* stream);
/* cabs_svd with the split of the Jacobi sweeps chosen by the caller: the first
 * fast_sweeps (1 .. 24) run as one launch per round over many work-groups, the
 * rest, if the iteration has not ended, in one work-group.  fast_sweeps = 0 is
 * cabs_svd's choice: 12 up to min(rows, cols) = 256, 24 above.  Every split
 * meets the same convergence test and accuracy (the single work-group applies
 * its rotations in another grouping, so factors can differ at the rounding
 * level); a small value saves launches on matrices known to converge in few
 * sweeps.  Out-of-range fast_sweeps: CABS_EINVAL. */
cabs_status cabs_svd_ex(int32_t batch, int32_t rows, int32_t cols, const double* A, double* U, double* S, double* V,
                        void* ws, size_t ws_bytes, int32_t fast_sweeps, void* stream);

/* Weighted k-means (Section 3.2) on the rows of P (rows x dim, precision
 * `compute`) with weights w (rows, FP64), from the k initial centres Z0
 * (k x dim, FP64), for `iters` Lloyd iterations; then, if snap_out is not
 * NULL, every centre (in index order) takes the nearest row not taken before
 * it, written ascending to snap_out[k].  Z (k x dim FP64), labels (rows,
 * int32, assignment to Z) and obj2 ({objective at Z0, objective at Z}) are
 * outputs (obj2 and labels may be NULL).  Ties go to the lowest index.
 * ws: cabs_kmeans_workspace_bytes() bytes. */
size_t cabs_kmeans_workspace_bytes(int64_t rows, int32_t dim, int32_t k, int32_t compute);
cabs_status cabs_kmeans(int64_t rows, int32_t dim, int32_t k, int32_t compute, const void* P, const double* w,
                        const double* Z0, int32_t iters, double* Z, int32_t* labels, double* obj2,
                        int64_t* snap_out, void* ws, size_t ws_bytes, void* stream);

/* cabs_kmeans without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results as cabs_kmeans;
 * the scratch cabs_kmeans would carve from `ws` comes from a fixed array of
 * CABS_KMEANS_NOALLOC_SCRATCH_BYTES in the library, one per device, held until
 * the process ends.  The call allocates nothing; the first call on a device
 * looks up that device's array.  Problems whose cabs_kmeans_workspace_bytes()
 * exceeds the array (about 1e5 rows x 200 dimensions x 200 centres in FP32
 * fits) return CABS_ENOMEM before anything is enqueued.  All calls on one
 * device share its array: calls that overlap in time on that device (on
 * different streams, or from different threads) race and must be serialised
 * by the caller. */
#define CABS_KMEANS_NOALLOC_SCRATCH_BYTES (64u << 20)
cabs_status cabs_kmeans_noalloc(int64_t rows, int32_t dim, int32_t k, int32_t compute, const void* P,
                                const double* w, const double* Z0, int32_t iters, double* Z, int32_t* labels,
                                double* obj2, int64_t* snap_out, void* stream);

/* ---- Kernel timing (diagnostics) ----
 * When enabled, every launch of a kernel family is bracketed by two HIP events
 * recorded on the stream it is launched on.  Families: "assign" (fused
 * distance GEMM + argmin of the k-means), "eval" (entry evaluation / gathers),
 * "tsgemm" (tall-skinny products), "gram", "svd", "snap" (top-T candidate
 * pass), "centroid" (centroid partial sums), "error".  cabs_timing_read waits
 * for the recorded events and returns the summed duration (milliseconds) and
 * the number of launches since the last reset; CABS_EINVAL for an unknown
 * family.  Timing adds two event records per launch. */
cabs_status cabs_timing_enable(int32_t on);
cabs_status cabs_timing_read(const char* family, double* total_ms, int64_t* launches);
void cabs_timing_reset(void);

/* ---- Continuous-batching server ---- */

typedef struct cabs_server cabs_server;

/* A server owns `max_slots` concurrent request slots on `device` (each with
 * its own stream) and a device memory pool of hbm_budget_bytes from which
 * request workspaces are carved.  Returns NULL on failure (see cabs_last_error). */
cabs_server* cabs_server_create(int32_t device, size_t hbm_budget_bytes, int32_t max_slots);

/* Queue a sketch, optionally followed by its relative Frobenius error
 * (cabs_error with err_samples and err_seed, result {num, den, ratio} into the
 * device array err_out3; err_out3 = NULL requests no error estimate).  `mat`
 * and `prm` are copied; the device buffers they and `out` name, and err_out3,
 * must stay valid until the request completes or is cancelled.
 * Ordering: an event is recorded on `stream` (the caller's stream; NULL = the
 * default stream) during this call, and the request's first kernel waits for
 * it, so everything the caller enqueued on `stream` before submitting (writing
 * the tables, clearing err_out3, reusing freed memory) is complete before the
 * request touches those buffers.  Work the caller enqueues later is not
 * ordered with the request: read the outputs only after cabs_poll reports it
 * finished.
 * Admission: a request is admitted when a slot is free and its workspace (the
 * larger of the sketch's and the error's; the error runs after the sketch on
 * the same stream and reuses it) fits in the pool.  Requests are considered
 * in arrival order, but one that does not fit yet may be passed by later
 * requests, at most 4 * max_slots times; after that nothing behind it is
 * admitted until it fits.  A request that can never fit is rejected here with
 * CABS_ENOMEM, a negative err_samples with CABS_EINVAL.  *ticket identifies it.
 * If a launch fails after some of the request's kernels were enqueued, its
 * workspace stays reserved until those kernels have finished, and cabs_poll
 * then returns the error. */
cabs_status cabs_submit(cabs_server* srv, const cabs_matrix* mat, const cabs_params* prm, const cabs_result* out,
                        int64_t err_samples, uint64_t err_seed, double* err_out3, void* stream, uint64_t* ticket);

/* CABS_OK when finished (latency_s, host, may be NULL: submit-to-completion
 * seconds), CABS_EBUSY while queued or running, CABS_ECANCELED if cancelled,
 * CABS_EINVAL for an unknown ticket.  A finished ticket is forgotten after it is
 * reported once. */
cabs_status cabs_poll(cabs_server* srv, uint64_t ticket, double* latency_s);

/* Cancel a request that has not been admitted yet (CABS_EBUSY if it already runs). */
cabs_status cabs_cancel(cabs_server* srv, uint64_t ticket);

/* Requests admitted together whose sketches have the same shape (equal sample
 * sizes, compute precision, orthogonalize and follow_up, no factor form) run
 * as a group of up to group_max (1..4; default 1 = never): each request on
 * its own slot stream, with each FP64 SVD of the sketch (Section 4.1's W, and
 * the orthogonalisation's) batched into one launch for the whole group, the
 * members' streams joining before it and waiting for it after.  Results are
 * bitwise those of the requests run alone.  Off by default because the
 * separate SVD chains of concurrent slots already overlap on the device and
 * the joins make each member wait for the slowest (measured: 4 % fewer
 * sketches/s on the uneven request stream).  CABS_EINVAL for a size outside
 * 1..4. */
cabs_status cabs_server_set_group(cabs_server* srv, int32_t group_max);

/* Block until every submitted request has completed. */
cabs_status cabs_server_drain(cabs_server* srv);

/* Waits for running requests, then frees the pool and streams. */
void cabs_server_destroy(cabs_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* CABS_H */
