// Batched FP64 SVD of small matrices by one-sided (Hestenes) Jacobi.
//
// The sketching routine (Section 4.1) needs the SVD of the k_r x k_c
// intersection W in FP64; the orthogonalisation (supplementary Section 3) needs
// two more small symmetric decompositions and one SVD.  One workgroup owns one
// matrix.  Its p = min(rows, cols) working columns (of length q = max(rows,
// cols)) are orthogonalised pairwise, the rotations accumulating in V; p/2
// disjoint pairs are handled per round by the 16 waves, with a round-robin
// ("circle") schedule so that every pair meets once per sweep.  Working
// columns live in LDS when they fit and in the caller's workspace otherwise.
// The output is sorted by singular value, descending, and the sign of each
// pair is fixed so that the largest-magnitude entry of every left singular
// vector is positive (first such entry on ties).
#include <algorithm>

#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace cabs {

constexpr int SVD_THREADS = 1024;
constexpr int SVD_MAX_SWEEPS = 40;
constexpr int SVD_LDS_BYTES = 60 * 1024;

__host__ __device__ static inline int even_up(int p) { return p + (p & 1); }

constexpr int BJ_B = 8;               // columns per block of the block-Jacobi path
constexpr int BJ_QS1 = 256;           // rows of X a round kernel with NU = 1 keeps in LDS (NU = 2: 512)
constexpr int BJ_SPLIT = 4;           // workgroups per pair of blocks in a round
constexpr int BJ_MAX_SWEEPS = 40;
constexpr int BJ_INNER_SWEEPS = 1;   // inner sweeps per pair and round in the finishing kernel
                                      // (one: more outer sweeps, each cheaper; 2 was slower)

// Number of column blocks (even) and padded column count of the block-Jacobi path.
__host__ __device__ static inline int bj_blocks(int p) { int nb = (p + BJ_B - 1) / BJ_B; return nb + (nb & 1); }

// Per-matrix scratch of the block-Jacobi path in doubles: X (q x P), V (P x P)
// with P >= p the padded column count, sigma (p), rank / sign (p each), and 64
// words of flags.
__host__ __device__ static inline size_t bj_ws_doubles(int rows, int cols) {
  const size_t p = rows < cols ? rows : cols, q = rows < cols ? cols : rows;
  const size_t P = (size_t)bj_blocks((int)p) * BJ_B;
  return 2 * q * P + P * P + 3 * p + 64;
}

// The QR-preconditioned path (below) for matrices with 384 <= min and max <=
// 1024 at the default sweep count: the working matrix A (q x p, q >= p; A^T
// when rows < cols) is factored A Pi = Q R by Householder QR with column
// pivoting, and the block-Jacobi SVD runs on R^T, whose columns are far closer
// to orthogonal (on 500 x 500 RBF kernel blocks about 11 sweeps instead of 24).
constexpr int QRP_MINP = 384;  // below this the plain path takes fewer launches
constexpr int QRP_MAXQ = 1024;
__host__ __device__ static inline bool qrp_applies(int rows, int cols) {
  const int p = rows < cols ? rows : cols, q = rows < cols ? cols : rows;
  return p >= QRP_MINP && q <= QRP_MAXQ;
}
// Its scratch in doubles: Ac (q x p, column-major), Q (q x q, row-major),
// R, R^T in pivot order and the two factors of its SVD (p x p each), the
// column norms (two buffers of p), the taken flags (two of p ints) and the
// pivots (p ints), then the block-Jacobi scratch of the p x p problem.
__host__ __device__ static inline size_t qrp_ws_doubles(int rows, int cols) {
  const size_t p = rows < cols ? rows : cols, q = rows < cols ? cols : rows;
  return q * p + q * q + 4 * p * p + 2 * p + (3 * p + 1) / 2 + 8 + bj_ws_doubles((int)p, (int)p);
}

__host__ __device__ static inline size_t svd_ws_doubles(int rows, int cols) {
  const size_t bj = bj_ws_doubles(rows, cols);
  if (!qrp_applies(rows, cols)) return bj;
  const size_t qr = qrp_ws_doubles(rows, cols);
  return qr > bj ? qr : bj;
}

size_t svd_ws_item_doubles(int rows, int cols) { return svd_ws_doubles(rows, cols); }

size_t svd_ws_bytes(int batch, int rows, int cols) {
  return (size_t)batch * svd_ws_doubles(rows, cols) * sizeof(double) + 256;
}

// Item b of a batch: its input, outputs and scratch, at fixed strides from
// base pointers, or from per-item pointer lists (n_ptr > 0: same-shape
// matrices that live in different requests' workspaces).
__device__ __forceinline__ const double* item_a(const SvdItems& it, int b) {
  return it.n_ptr ? it.Ap[b] : it.A + b * it.sA;
}
__device__ __forceinline__ double* item_u(const SvdItems& it, int b) { return it.n_ptr ? it.Up[b] : it.U + b * it.sU; }
__device__ __forceinline__ double* item_s(const SvdItems& it, int b) { return it.n_ptr ? it.Sp[b] : it.S + b * it.sS; }
__device__ __forceinline__ double* item_v(const SvdItems& it, int b) { return it.n_ptr ? it.Vp[b] : it.V + b * it.sV; }
__device__ __forceinline__ double* item_w(const SvdItems& it, int b) { return it.n_ptr ? it.Wp[b] : it.W + b * it.sW; }

// Singular values (column norms of the converged X), descending order, signs,
// and the outputs in row-major U (rows x p), S (p), V (cols x p).  X is q x p
// column-major with column stride ldx, V (p x p, rotations) with stride ldv.
__device__ void svd_finalize(const double* X, int64_t xrs, int64_t xcs, const double* V, int64_t vrs, int64_t vcs, int q,
                             int p, bool trans, double* sig, int* rank, double* sgn, double* Ub, double* Sb,
                             double* Vb) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int nwaves = nthr >> 6;
  // Singular values = column norms (one wave per column).
  for (int j = wave; j < p; j += nwaves) {
    double s2 = 0.0;
    for (int i = lane; i < q; i += 64) s2 += X[i * xrs + j * xcs] * X[i * xrs + j * xcs];
    s2 = wave_sum(s2);
    if (lane == 0) sig[j] = sqrt(s2);
  }
  __syncthreads();
  // Descending order, lower column index first on ties.
  // NaN (from non-finite input) ranks below every number so that ranks stay a permutation.
  for (int j = tid; j < p; j += nthr) {
    const double sj = sig[j] == sig[j] ? sig[j] : -1.0;
    int r = 0;
    for (int i = 0; i < p; ++i) {
      const double si = sig[i] == sig[i] ? sig[i] : -1.0;
      r += (si > sj) || (si == sj && i < j);
    }
    rank[j] = r;
  }
  __syncthreads();
  // Sign: the left singular vector of A is X[:, j] / sigma (not transposed) or V[:, j]
  // (transposed); make its largest-magnitude entry positive.
  for (int j = wave; j < p; j += nwaves) {
    const double* lv = trans ? V + j * vcs : X + j * xcs;
    const int64_t st = trans ? vrs : xrs;
    const int len = trans ? p : q;
    double best = -1.0;
    int bi = 0x7fffffff;
    double bval = 0.0;
    for (int i = lane; i < len; i += 64) {
      const double v = lv[i * st];
      if (fabs(v) > best) { best = fabs(v); bi = i; bval = v; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      const double ov = __shfl_xor(bval, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; bval = ov; }
    }
    if (lane == 0) sgn[j] = bval < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  for (int j = tid; j < p; j += nthr) Sb[rank[j]] = sig[j];
  // Left factor of the working problem: X / sigma (q x p); right: V (p x p).
  for (int e = tid; e < q * p; e += nthr) {
    const int j = e / q, i = e % q;
    const double sj = sig[j];
    const double v = sj > 0.0 ? sgn[j] * X[i * xrs + j * xcs] / sj : 0.0;
    if (!trans) Ub[(int64_t)i * p + rank[j]] = v;   // U: rows x p
    else Vb[(int64_t)i * p + rank[j]] = v;          // V: cols x p
  }
  for (int e = tid; e < p * p; e += nthr) {
    const int j = e / p, i = e % p;
    const double v = sgn[j] * V[i * vrs + j * vcs];
    if (!trans) Vb[(int64_t)i * p + rank[j]] = v;   // V: cols x p
    else Ub[(int64_t)i * p + rank[j]] = v;          // U: rows x p
  }
}

__global__ __launch_bounds__(SVD_THREADS) void svd_jacobi_kernel(int rows, int cols, SvdItems it, int use_lds) {
  extern __shared__ double lds[];
  __shared__ int rotated;
  const int b = blockIdx.x;
  const bool trans = rows < cols;
  const int p = trans ? rows : cols;
  const int q = trans ? cols : rows;
  const int pe = even_up(p);
  double* base = item_w(it, b);
  double* X = use_lds ? lds : base;              // column-major q x p
  double* V = use_lds ? lds + (size_t)q * p : base + (size_t)q * p;  // column-major p x p
  const size_t Pb = (size_t)bj_blocks(p) * BJ_B;
  double* sig = base + (size_t)q * Pb + Pb * Pb;
  int* rank = (int*)(sig + p);
  double* sgn = sig + 2 * p;
  const double* Ab = item_a(it, b);
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int nwaves = SVD_THREADS / 64;

  // Load: X[:, j] = A[:, j] (or A[j, :] when transposed); V = I.
  for (int e = tid; e < q * p; e += SVD_THREADS) {
    const int j = e / q, i = e % q;
    X[e] = trans ? Ab[(int64_t)j * cols + i] : Ab[(int64_t)i * cols + j];
  }
  for (int e = tid; e < p * p; e += SVD_THREADS) V[e] = (e / p == e % p) ? 1.0 : 0.0;
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  const double tol = eps * (q > 16 ? (double)q : 16.0);

  for (int sweep = 0; sweep < SVD_MAX_SWEEPS; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < pe - 1; ++round) {
      for (int pr = wave; pr < pe / 2; pr += nwaves) {
        // circle schedule: position 0 fixed, the others rotate by `round`
        const int pa = pr, pb = pe - 1 - pr;
        const int ca = pa == 0 ? 0 : 1 + (pa - 1 + round) % (pe - 1);
        const int cb = pb == 0 ? 0 : 1 + (pb - 1 + round) % (pe - 1);
        if (ca >= p || cb >= p) continue;
        const int a = ca < cb ? ca : cb;
        const int c = ca < cb ? cb : ca;
        double* xa = X + (size_t)a * q;
        double* xc = X + (size_t)c * q;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < q; i += 64) {
          const double u = xa[i], v = xc[i];
          al += u * u;
          be += v * v;
          ga += u * v;
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        const double nrm = sqrt(al) * sqrt(be);
        if (!(nrm > 0.0) || !(fabs(ga) > tol * nrm)) continue;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t);
        const double sn = cs * t;
        for (int i = lane; i < q; i += 64) {
          const double u = xa[i], v = xc[i];
          xa[i] = cs * u - sn * v;
          xc[i] = sn * u + cs * v;
        }
        double* va = V + (size_t)a * p;
        double* vc = V + (size_t)c * p;
        for (int i = lane; i < p; i += 64) {
          const double u = va[i], v = vc[i];
          va[i] = cs * u - sn * v;
          vc[i] = sn * u + cs * v;
        }
        if (lane == 0) rotated = 1;
      }
      __syncthreads();
    }
    const int done = rotated == 0;
    __syncthreads();
    if (done) break;
  }

  svd_finalize(X, 1, q, V, 1, p, q, p, trans, sig, rank, sgn, item_u(it, b), item_s(it, b), item_v(it, b));
}

// ---------------------------------------------------------------------------
// Block one-sided Jacobi for larger matrices.
//
// The p working columns are split into blocks of 8 and every round pairs the
// blocks (circle schedule).  For one pair of blocks: form the 16 x 16 FP64 Gram
// of its columns on the MFMA, skip the pair if it is already orthogonal, else
// diagonalise the Gram by cyclic two-sided Jacobi (relatively accurate on
// positive definite matrices; one sweep per round in the fast phase,
// BJ_INNER_SWEEPS in the finishing kernel) while accumulating the rotation J, and replace
// the 16 columns of X and V by X J and V J (MFMA again).  A sweep with no
// rotation ends the iteration.  Columns below eps |X|_F are at the rounding
// level of the block updates and are neither tested nor rotated.
//
// The first sweeps (at most BJ_FAST_SWEEPS, fewer where the caller expects
// fast convergence) run as one launch per round with BJ_SPLIT workgroups per
// block pair, spreading a round over many CUs; rounds after convergence return
// at once but still cost a launch.  A single-workgroup kernel then finishes
// the matrices that need more sweeps (it skips that step when the matrix has
// converged) and writes the outputs.
// X (q x P) and V (P x P) are row-major in the workspace.
// ---------------------------------------------------------------------------
constexpr int BJ_FAST_SWEEPS = 24;  // most sweeps launched round by round
// The default split: 12 sweeps up to p = 256 (where the finisher's sweeps cost about twice the
// round-by-round ones), 24 above (where a finisher sweep on one work-group costs several times a
// round-by-round sweep, and a round that only finds the converged flag costs one launch).
static inline int bj_default_fast_sweeps(int p) { return p > 256 ? 24 : 12; }

__device__ __forceinline__ int circle_pos(int pos, int round, int n) {
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (n - 1);
}

// Round-robin schedule of 16 indices in 15 rounds of 8 disjoint pairs: index
// 0 stays at position 0, the others rotate one position per round, and pair k
// of round r joins positions k and 15 - k.
__device__ __forceinline__ int s16_elem(int pos, int r) { return pos == 0 ? 0 : 1 + (pos - 1 + r) % 15; }
__device__ __forceinline__ int s16_pos(int c, int r) { return c == 0 ? 0 : 1 + (c + 14 - r) % 15; }

struct BjView {
  double* X; double* X1; double* V; double* sig; int* rank; double* sgn; int* flags; double* fro2;
  int q, p, P, nb;
  bool trans;
};

__device__ __forceinline__ BjView bj_view(double* base, int rows, int cols) {
  BjView v;
  v.trans = rows < cols;
  v.p = v.trans ? rows : cols;
  v.q = v.trans ? cols : rows;
  v.nb = bj_blocks(v.p);
  v.P = v.nb * BJ_B;
  v.X = base;
  v.V = base + (size_t)v.q * v.P;
  v.sig = v.V + (size_t)v.P * v.P;
  v.rank = (int*)(v.sig + v.p);
  v.sgn = v.sig + 2 * (size_t)v.p;
  v.flags = (int*)(v.sig + 3 * (size_t)v.p);  // [2 + s]: sweep s rotated
  v.fro2 = (double*)(v.flags + 64);
  v.X1 = v.sig + 3 * (size_t)v.p + 64;  // second copy of X (the rounds alternate between the two)
  return v;
}

__global__ __launch_bounds__(256) void bj_init_kernel(int rows, int cols, SvdItems it) {
  BjView v = bj_view(item_w(it, blockIdx.y), rows, cols);
  const double* Ab = item_a(it, blockIdx.y);
  const int64_t nx = (int64_t)v.q * v.P, nv = (int64_t)v.P * v.P;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nx + nv; e += (int64_t)gridDim.x * 256) {
    if (e < nx) {
      const int i = (int)(e / v.P), j = (int)(e % v.P);
      double x = 0.0;
      if (j < v.p) x = v.trans ? Ab[(int64_t)j * cols + i] : Ab[(int64_t)i * cols + j];
      v.X[e] = x;
    } else {
      const int64_t f = e - nx;
      v.V[f] = (f / v.P == f % v.P) ? 1.0 : 0.0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < 64) v.flags[threadIdx.x] = 0;
}

// |X|_F^2, invariant under the rotations, for the negligible-column floor
// (fixed summation order: per thread, then per wave, then the waves in order).
__global__ __launch_bounds__(1024) void bj_norm_kernel(int rows, int cols, SvdItems it) {
  __shared__ double red[16];
  BjView v = bj_view(item_w(it, blockIdx.x), rows, cols);
  const double* Ab = item_a(it, blockIdx.x);
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)rows * cols; e += 1024) s += Ab[e] * Ab[e];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    v.fro2[0] = t;
  }
}

// A zero that out-of-range loads are pointed at (global memory, never written),
// so that the loads need no branch.
static __device__ double kBjZero[2] = {0.0, 0.0};

// Gram of the 16 columns cols(c) = block ba (c < 8) / bb (c >= 8), rows [r0, r1), by one wave;
// 8 row quads are loaded before their MFMAs.
__device__ __forceinline__ f64x4 pair_gram(const BjView& v, int ba, int bb, int r0, int r1) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
  const int mycol = c16 < 8 ? ba * BJ_B + c16 : bb * BJ_B + c16 - 8;
  const double* xc = v.X + mycol;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int r = r0; r < r1; r += 32) {
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int rr = r + 4 * u + g;
      x[u] = *(rr < r1 ? xc + (size_t)rr * v.P : (const double*)kBjZero);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u], x[u], acc, 0, 0, 0);
  }
  return acc;
}

// The same Gram for at most 4 NQ rows [r0, r1): the NQ row quads are loaded by
// pair_x_load in one batch, then multiplied and kept in the LDS stash.
template <int NQ>
__device__ __forceinline__ void pair_x_load(const BjView& v, int ba, int bb, int r0, int r1, double (&x)[NQ]) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
  const int mycol = c16 < 8 ? ba * BJ_B + c16 : bb * BJ_B + c16 - 8;
  const double* xc = v.X + mycol;
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    const int rr = r0 + 4 * u + g;
    x[u] = *(rr < r1 ? xc + (size_t)rr * v.P : (const double*)kBjZero);
  }
}

// Rows of the tiles workgroup `share` rotates go to its stash (BJ_SPLIT tiles
// apart: stash row 16 (t / BJ_SPLIT) + i for row i of tile t).
template <int NQ>
__device__ __forceinline__ f64x4 pair_gram_regs(const double (&x)[NQ], int r0, int r1, int share,
                                                double (*xs)[17]) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < NQ; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u], x[u], acc, 0, 0, 0);
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    const int rr = r0 + 4 * u + g, t = rr >> 4;
    if (rr < r1 && t % BJ_SPLIT == share) xs[(t / BJ_SPLIT) * 16 + (rr & 15)][c16] = x[u];
  }
  return acc;
}

// X <- X J, V <- V J on the pair's 16 columns for the 16-row tiles t = t0, t0 + dt, ...,
// TB tiles' loads in flight at a time.  jb[st] = J[4 st + g][c16].
template <int TB>
__device__ __forceinline__ void pair_apply(const BjView& v, double* xo, int ba, int bb, const double (&jb)[4], int t0,
                                           int dt) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
  const int qt = (v.q + 15) >> 4, ntiles = qt + (v.P >> 4);
  const int outcol = c16 < 8 ? ba * BJ_B + c16 : bb * BJ_B + c16 - 8;
  int colk[4];
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int kc = 4 * st + g;
    colk[st] = kc < 8 ? ba * BJ_B + kc : bb * BJ_B + kc - 8;
  }
  for (int tb = t0; tb < ntiles; tb += TB * dt) {
    double a[TB][4];
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int t = tb + u * dt;
      const double* mat = t < qt ? v.X : v.V;
      const int r0 = t < qt ? t * 16 : (t - qt) * 16, nr = t < qt ? v.q : v.P;
      const int rr = r0 + c16;
      const bool in = t < ntiles && rr < nr;
#pragma unroll
      for (int st = 0; st < 4; ++st) a[u][st] = *(in ? mat + (size_t)rr * v.P + colk[st] : (const double*)kBjZero);
    }
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int t = tb + u * dt;
      if (t >= ntiles) break;
      double* mat = t < qt ? xo : v.V;
      const int r0 = t < qt ? t * 16 : (t - qt) * 16, nr = t < qt ? v.q : v.P;
      f64x4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < 4; ++st) d = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][st], jb[st], d, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = r0 + out_row<double>(g, i);
        if (rr < nr) mat[(size_t)rr * v.P + outcol] = d[i];
      }
    }
  }
}

// Hardware reciprocal and reciprocal square root, each refined by one Newton step.
__device__ __forceinline__ double rsq_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = __builtin_fma(-x * y, y, 1.0);
  return __builtin_fma(0.5 * y, e, y);
}

// Rotation zeroing G[ia][ib] of the positive semidefinite G (one-sided Jacobi
// formulas).  The angle only steers convergence; c = (1 + t^2)^(-1/2) and
// s = c t make the rotation orthogonal to rounding, which is what the accuracy
// of X J and V J rests on.  Branch-free, so that the two rotations a lane
// needs per step run as interleaved chains: the skip test (squares, no roots)
// selects the identity at the end.  When it passes, |zeta| <= 1 / (2 eps tol),
// so zeta^2 cannot overflow; when it fails the temporaries are discarded.
__device__ __forceinline__ bool jacobi_rot(double al, double be, double ga, double tol, double floor2, double& c,
                                           double& sn) {
  const bool rot = al > floor2 && be > floor2 && ga * ga > (tol * tol) * (al * be);
  const double gs = rot ? ga : 1.0;
  // t only steers the angle: the hardware reciprocal and root estimates are
  // enough there; c gets a refined root, so that c^2 (1 + t^2) = 1 to rounding
  const double zeta = (be - al) * (0.5 * __builtin_amdgcn_rcp(gs));
  const double z2 = __builtin_fma(zeta, zeta, 1.0);
  const double t = __builtin_copysign(__builtin_amdgcn_rcp(fabs(zeta) + z2 * __builtin_amdgcn_rsq(z2)), zeta);
  const double cr = rsq_nr(__builtin_fma(t, t, 1.0));
  c = rot ? cr : 1.0;
  sn = rot ? cr * t : 0.0;
  return rot;
}

// Rotation of the pair's columns when the X rows sit in the LDS stash (q <=
// 256 NU): wave w rotates its X tiles from LDS and its V tiles from vv, which
// it loaded before the inner solve.  jb[st] = J[4 st + g][c16].  Matrices with
// more than 512 rows read X from global memory twice.
//
// With the stash, the 16-row tiles of X and of V are split between the
// BJ_SPLIT workgroups of a pair: workgroup s, wave w rotates tiles
// s + BJ_SPLIT (w + 4 u), u < NU, of each (q, P <= 256 NU = 16 NU tiles), and
// its stash holds only those X tiles (64 NU rows, stash row 16 (w + 4 u) + i
// for row i of tile s + BJ_SPLIT (w + 4 u)), so that the kernel's LDS stays
// small enough to share a CU with other kernels' work-groups.

__device__ __forceinline__ int pair_tile(int s, int wave, int u) { return s + BJ_SPLIT * (wave + 4 * u); }

template <int NU>
__device__ __forceinline__ void pair_v_load(const BjView& v, int ba, int bb, int s, int wave, double (&vv)[NU][4]) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
  const int vt = v.P >> 4;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int t = pair_tile(s, wave, u), rr = t * 16 + c16;
    const bool in = t < vt && rr < v.P;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int kc = 4 * st + g;
      const int col = kc < 8 ? ba * BJ_B + kc : bb * BJ_B + kc - 8;
      vv[u][st] = *(in ? v.V + (size_t)rr * v.P + col : (const double*)kBjZero);
    }
  }
}

template <int NU>
__device__ __forceinline__ void pair_apply_stash(const BjView& v, double* xo, int ba, int bb, const double (&jb)[4],
                                                 int s, int wave, const double (*xs)[17], const double (&vv)[NU][4]) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
  const int qt = (v.q + 15) >> 4, vt = v.P >> 4;
  const int outcol = c16 < 8 ? ba * BJ_B + c16 : bb * BJ_B + c16 - 8;
  f64x4 dx[NU], dv[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int t = pair_tile(s, wave, u), rr = t * 16 + c16;
    double a[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) a[st] = (t < qt && rr < v.q) ? xs[(wave + 4 * u) * 16 + c16][4 * st + g] : 0.0;
    dx[u] = f64x4{0.0, 0.0, 0.0, 0.0};
    dv[u] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      dx[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], jb[st], dx[u], 0, 0, 0);
      dv[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(vv[u][st], jb[st], dv[u], 0, 0, 0);
    }
  }
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int t = pair_tile(s, wave, u);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = t * 16 + out_row<double>(g, i);
      if (t < qt && r < v.q) xo[(size_t)r * v.P + outcol] = dx[u][i];
      if (t < vt && r < v.P) v.V[(size_t)r * v.P + outcol] = dv[u][i];
    }
  }
}

// A pair that does not rotate carries its columns of X over to the other copy.
template <int NU>
__device__ __forceinline__ void pair_copy_stash(const BjView& v, double* xo, int ba, int bb, int s, int wave,
                                                const double (*xs)[17]) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
  const int qt = (v.q + 15) >> 4;
  const int outcol = c16 < 8 ? ba * BJ_B + c16 : bb * BJ_B + c16 - 8;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int t = pair_tile(s, wave, u);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = t * 16 + out_row<double>(g, i);
      if (t < qt && r < v.q) xo[(size_t)r * v.P + outcol] = xs[(wave + 4 * u) * 16 + out_row<double>(g, i)][c16];
    }
  }
}

__device__ __forceinline__ void pair_copy(const BjView& v, double* xo, int ba, int bb, int t0, int dt) {
  const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
  const int qt = (v.q + 15) >> 4;
  const int outcol = c16 < 8 ? ba * BJ_B + c16 : bb * BJ_B + c16 - 8;
  for (int t = t0; t < qt; t += dt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = t * 16 + out_row<double>(g, i);
      if (r < v.q) xo[(size_t)r * v.P + outcol] = v.X[(size_t)r * v.P + outcol];
    }
  }
}

// One round of the fast phase: BJ_SPLIT workgroups (4 waves each) per pair of
// blocks.  Each forms the pair's Gram and J itself (the same code on the same
// data, so the same J bit for bit) and rotates its share of the row tiles.
// Since a workgroup may rotate its tiles while another one still reads the
// pair's columns, round g (counted over the sweeps) reads copy g mod 2 of X
// and writes copy (g + 1) mod 2, every pair writing all of its columns.  The
// 16 x 16 Gram is diagonalised by one Jacobi sweep in wave 0: lane (kp, kq)
// owns the 2 x 2 block of G at row pair kp and column pair kq of the current
// step (and the matching block of J), computes both rotations itself, and
// writes the rotated block to the other half of a double buffer.

template <int NU>
__global__ __launch_bounds__(256) void bj_round_kernel(int rows, int cols, int round, int sweep, SvdItems it) {
  __shared__ double gp[4][16][17];
  __shared__ double Gb[2][16][17];
  __shared__ double Jb[2][16][17];
  __shared__ double xs[BJ_QS1 * NU / BJ_SPLIT][17];
  __shared__ int any_off;
  BjView v = bj_view(item_w(it, blockIdx.y), rows, cols);
  const int gr = sweep * (v.nb - 1) + round;
  double* const xo = (gr & 1) ? v.X : v.X1;
  if (gr & 1) v.X = v.X1;  // v.X: the copy this round reads
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, c16 = lane & 15, g = lane >> 4;
  const int pr = blockIdx.x / BJ_SPLIT, share = blockIdx.x % BJ_SPLIT;
  const int ba = circle_pos(pr, round, v.nb), bb = circle_pos(v.nb - 1 - pr, round, v.nb);
  const bool stash = v.q <= BJ_QS1 * NU;  // uniform
  // A sweep without rotations leaves X as it was (copied to the other copy),
  // so every later sweep would find none either: the matrix has converged,
  // and the rounds still launched return at once.
  if (sweep > 0 && v.flags[2 + sweep - 1] == 0) return;  // uniform over the grid
  double vv[NU][4];
  {
    const int r0 = (int)(((int64_t)v.q * wave) / 4), r1 = (int)(((int64_t)v.q * (wave + 1)) / 4);
    f64x4 acc;
    if (stash) {  // r1 - r0 <= 64 NU rows: one batch of loads
      double x[16 * NU];
      pair_x_load(v, ba, bb, r0, r1, x);
      pair_v_load(v, ba, bb, share, wave, vv);  // in flight during the inner solve
      acc = pair_gram_regs(x, r0, r1, share, xs);
    } else {
      acc = pair_gram(v, ba, bb, r0, r1);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) gp[wave][out_row<double>(g, i)][c16] = acc[i];
  }
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  const double tol = eps * (v.q > 16 ? (double)v.q : 16.0);
  const double floor2 = eps * eps * v.fro2[0];
  // Round 0 of a sweep runs a full cyclic Jacobi sweep of the pair's 16 x 16
  // Gram (15 steps, every pair of its columns); the other rounds only the 8
  // steps that pair a column of block ba with one of block bb (step s: i with
  // 8 + (i + s) mod 8).  Each pair of the matrix's columns is still visited
  // once per sweep: pairs inside a block in round 0, pairs across blocks in
  // the round where the blocks meet.
  const bool full = round == 0;  // uniform
  // Schedule positions: in the full sweep position p holds element
  // s16_elem(p, r) at step r (start: the identity); in the cross steps the
  // first block stays put and position 15 - k holds element 8 + (k + s) mod 8
  // (start: e0(p) = p for p < 8, 23 - p for p >= 8, an involution).
  const auto e0 = [full](int p) { return full || p < 8 ? p : 23 - p; };
  if (wave == 0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = lane + 64 * t, i = e >> 4, j = e & 15;
      const int pi = e0(i), pj = e0(j);
      Gb[0][i][j] = ((gp[0][pi][pj] + gp[1][pi][pj]) + gp[2][pi][pj]) + gp[3][pi][pj];
      Jb[0][i][j] = i == pj ? 1.0 : 0.0;  // row: element, column: position
    }
    wave_lds_sync();
    bool off = false;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = lane + 64 * t, i = e >> 4, j = e & 15;
      const double gi = Gb[0][i][i], gj = Gb[0][j][j], gij = Gb[0][i][j];
      if (i < j && gi > floor2 && gj > floor2 && gij * gij > (tol * tol) * (gi * gj)) off = true;
    }
    const bool anyo = __ballot(off) != 0;
    int cur = 0;
    if (anyo) {
      // G and the columns of J are kept in schedule-position order, so the
      // lane's positions (kp, 15 - kp) x (kq, 15 - kq) are the same at every
      // step, and each rotated entry is written where its element sits at the
      // next step: full sweep p -> p - 1, 1 -> 15, 0 stays; cross steps
      // p -> p + 1 for 8 <= p < 15, 15 -> 8, the first block stays.  After
      // the 15 (8) steps every element is back at its start position.
      const int kp = lane >> 3, kq = lane & 7;
      const int A = kp, B = 15 - kp, C = kq, D = 15 - kq;
      const int j0 = 2 * kp, j1 = 2 * kp + 1;
      auto sweep_steps = [&](auto nsteps, auto nxt) {
        constexpr int NS = decltype(nsteps)::value;
        const int nA = nxt(A), nB = nxt(B), nC = nxt(C), nD = nxt(D);
#pragma unroll
        for (int r = 0; r < NS; ++r) {
          const double (*G)[17] = Gb[r & 1];
          const double (*J)[17] = Jb[r & 1];
          const double paa = G[A][A], pbb = G[B][B], pab = G[A][B];
          const double qaa = G[C][C], qbb = G[D][D], qab = G[C][D];
          const double b00 = G[A][C], b01 = G[A][D], b10 = G[B][C], b11 = G[B][D];
          const double j00 = J[j0][C], j01 = J[j0][D], j10 = J[j1][C], j11 = J[j1][D];
          double cp, sp, cq, sq;
          jacobi_rot(paa, pbb, pab, tol, floor2, cp, sp);
          jacobi_rot(qaa, qbb, qab, tol, floor2, cq, sq);
          // columns (right rotation by pair kq), then rows (left rotation by pair kp)
          const double c00 = cq * b00 - sq * b01, c01 = sq * b00 + cq * b01;
          const double c10 = cq * b10 - sq * b11, c11 = sq * b10 + cq * b11;
          double (*Gn)[17] = Gb[(r & 1) ^ 1];
          double (*Jn)[17] = Jb[(r & 1) ^ 1];
          Gn[nA][nC] = cp * c00 - sp * c10;
          Gn[nB][nC] = sp * c00 + cp * c10;
          Gn[nA][nD] = cp * c01 - sp * c11;
          Gn[nB][nD] = sp * c01 + cp * c11;
          Jn[j0][nC] = cq * j00 - sq * j01;
          Jn[j0][nD] = sq * j00 + cq * j01;
          Jn[j1][nC] = cq * j10 - sq * j11;
          Jn[j1][nD] = sq * j10 + cq * j11;
          wave_lds_sync();
        }
      };
      if (full) {
        sweep_steps(std::integral_constant<int, 15>{}, [](int p) { return p == 0 ? 0 : (p == 1 ? 15 : p - 1); });
        cur = 1;  // 15 steps: the result is in buffer 1
      } else {
        sweep_steps(std::integral_constant<int, 8>{}, [](int p) { return p < 8 ? p : (p < 15 ? p + 1 : 8); });
        cur = 0;  // 8 steps: buffer 0
      }
    }
    if (lane == 0) any_off = anyo ? cur + 1 : 0;
  }
  __syncthreads();
  const int ao = any_off;
  if (!ao) {  // uniform
    if (stash) pair_copy_stash<NU>(v, xo, ba, bb, share, wave, xs);
    else pair_copy(v, xo, ba, bb, share + BJ_SPLIT * wave, 4 * BJ_SPLIT);
    return;
  }
  if (tid == 0) v.flags[2 + sweep] = 1;
  double jb[4];  // J[4 st + g][c16]: its column c16 sits at position e0(c16)
#pragma unroll
  for (int st = 0; st < 4; ++st) jb[st] = Jb[ao - 1][4 * st + g][e0(c16)];
  if (stash) pair_apply_stash(v, xo, ba, bb, jb, share, wave, xs, vv);
  else pair_apply<8>(v, xo, ba, bb, jb, share + BJ_SPLIT * wave, 4 * BJ_SPLIT);
}

// The outputs from row-major X (q x P) and V (P x P) by the 1024 threads of
// one workgroup (the same results as svd_finalize).  Thread t works on column
// t mod p over the rows of group t / p (up to 4 groups of contiguous rows, so
// that loads along a row are contiguous across lanes); the groups' partial
// sums and maxima are combined in group order, which for the maxima (largest
// magnitude, lowest index on ties) gives the same entry as one scan.
constexpr int BJF_MAXP = 1024;
struct BjFinalLds {
  double part2[BJF_MAXP];   // partial sums of squares
  double pbest[BJF_MAXP];   // partial largest magnitude
  double pval[BJF_MAXP];    // ... its value
  int pidx[BJF_MAXP];       // ... its row
  double sig[BJF_MAXP];
  double sgn[BJF_MAXP];
  int rank[BJF_MAXP];
};

__device__ void svd_finalize_rm(const BjView& v, BjFinalLds& L, double* Ub, double* Sb, double* Vb) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int p = v.p, q = v.q, P = v.P;
  const int ng = p >= 1024 ? 1 : (1024 / p < 4 ? 1024 / p : 4);
  const int j = tid % p, grp = tid / p;
  if (grp < ng) {
    double s2 = 0.0;
    for (int i = (int)((int64_t)q * grp / ng), i1 = (int)((int64_t)q * (grp + 1) / ng); i < i1; ++i) {
      const double x = v.X[(size_t)i * P + j];
      s2 += x * x;
    }
    // left singular vector of A: X[:, j] / sigma (not transposed) or V[:, j] (transposed)
    const double* lv = v.trans ? v.V : v.X;
    const int len = v.trans ? p : q;
    double best = -1.0, bval = 0.0;
    int bi = 0x7fffffff;
    for (int i = (int)((int64_t)len * grp / ng), i1 = (int)((int64_t)len * (grp + 1) / ng); i < i1; ++i) {
      const double x = lv[(size_t)i * P + j];
      if (fabs(x) > best) { best = fabs(x); bi = i; bval = x; }
    }
    L.part2[tid] = s2;
    L.pbest[tid] = best;
    L.pval[tid] = bval;
    L.pidx[tid] = bi;
  }
  __syncthreads();
  if (tid < p) {
    double s2 = L.part2[tid], best = L.pbest[tid], bval = L.pval[tid];
    int bi = L.pidx[tid];
    for (int gi = 1; gi < ng; ++gi) {
      const int t = gi * p + tid;
      s2 += L.part2[t];
      if (L.pbest[t] > best || (L.pbest[t] == best && L.pidx[t] < bi)) { best = L.pbest[t]; bi = L.pidx[t]; bval = L.pval[t]; }
    }
    L.sig[tid] = sqrt(s2);
    L.sgn[tid] = bval < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  // descending order, lower column index first on ties; NaN ranks below every number
  if (tid < p) {
    const double sj = L.sig[tid] == L.sig[tid] ? L.sig[tid] : -1.0;
    int r = 0;
    for (int i = 0; i < p; ++i) {
      const double si = L.sig[i] == L.sig[i] ? L.sig[i] : -1.0;
      r += (si > sj) || (si == sj && i < tid);
    }
    L.rank[tid] = r;
    Sb[r] = L.sig[tid];
  }
  __syncthreads();
  // left factor of the working problem X / sigma (q x p), right factor V (p x p)
  double* const xo = v.trans ? Vb : Ub;
  double* const vo = v.trans ? Ub : Vb;
  for (int i = wave; i < q; i += 16)
    for (int c = lane; c < p; c += 64) {
      const double sc = L.sig[c];
      xo[(int64_t)i * p + L.rank[c]] = sc > 0.0 ? L.sgn[c] * v.X[(size_t)i * P + c] / sc : 0.0;
    }
  for (int i = wave; i < p; i += 16)
    for (int c = lane; c < p; c += 64) vo[(int64_t)i * p + L.rank[c]] = L.sgn[c] * v.V[(size_t)i * P + c];
}

// Remaining sweeps (if any) in one workgroup, one wave per pair; then the outputs.
__global__ __launch_bounds__(1024) void bj_finish_kernel(int rows, int cols, int first_sweep, SvdItems it) {
  __shared__ double Gs[16][16][17];
  __shared__ double cs[16][8][2];
  __shared__ int rotated;
  __shared__ BjFinalLds fin;
  const int b = blockIdx.x;
  BjView v = bj_view(item_w(it, b), rows, cols);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, c16 = lane & 15, g = lane >> 4;
  const double eps = 2.220446049250313e-16;
  const double tol = eps * (v.q > 16 ? (double)v.q : 16.0);
  const double floor2 = eps * eps * v.fro2[0];
  double (*G)[17] = Gs[wave];
  // the copy of X the fast phase ended on (its sweeps have nb - 1 rounds, an odd number);
  // the sweeps here work on it in place
  int used = first_sweep;  // sweeps run by the fast phase: through the first without rotations
  for (int sw = 0; sw < first_sweep; ++sw)
    if (v.flags[2 + sw] == 0) { used = sw + 1; break; }
  if (used & 1) v.X = v.X1;
  const bool converged = v.flags[2 + used - 1] == 0;
  for (int sweep = first_sweep; !converged && sweep < BJ_MAX_SWEEPS; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < v.nb - 1; ++round) {
      for (int pr = wave; pr < v.nb / 2; pr += 16) {
        const int ba = circle_pos(pr, round, v.nb), bb = circle_pos(v.nb - 1 - pr, round, v.nb);
        const f64x4 acc = pair_gram(v, ba, bb, 0, v.q);
#pragma unroll
        for (int i = 0; i < 4; ++i) G[out_row<double>(g, i)][c16] = acc[i];
        wave_lds_sync();
        bool off = false;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int e = lane + 64 * t, i = e >> 4, j = e & 15;
          if (i < j && G[i][i] > floor2 && G[j][j] > floor2 && fabs(G[i][j]) > tol * sqrt(G[i][i]) * sqrt(G[j][j]))
            off = true;
        }
        if (__ballot(off) == 0) continue;
        if (lane == 0) rotated = 1;
        double jr[4];  // J[4g + i][c16]
#pragma unroll
        for (int i = 0; i < 4; ++i) jr[i] = (4 * g + i == c16) ? 1.0 : 0.0;
        for (int is = 0; is < BJ_INNER_SWEEPS; ++is) {
          bool any = false;
          for (int r = 0; r < 15; ++r) {
            if (lane < 8) {
              const int ia = s16_elem(lane, r), ib = s16_elem(15 - lane, r);
              double c, sn;
              any |= jacobi_rot(G[ia][ia], G[ib][ib], G[ia][ib], tol, floor2, c, sn);
              cs[wave][lane][0] = c;
              cs[wave][lane][1] = sn;
            }
            wave_lds_sync();
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              const int e = lane + 64 * t, k = e >> 4, i = e & 15, ia = s16_elem(k, r), ib = s16_elem(15 - k, r);
              const double c = cs[wave][k][0], sn = cs[wave][k][1], u = G[i][ia], w = G[i][ib];
              G[i][ia] = c * u - sn * w;
              G[i][ib] = sn * u + c * w;
            }
            wave_lds_sync();
#pragma unroll
            for (int t = 0; t < 2; ++t) {
              const int e = lane + 64 * t, k = e >> 4, j = e & 15, ia = s16_elem(k, r), ib = s16_elem(15 - k, r);
              const double c = cs[wave][k][0], sn = cs[wave][k][1], u = G[ia][j], w = G[ib][j];
              G[ia][j] = c * u - sn * w;
              G[ib][j] = sn * u + c * w;
            }
            {
              const int pos = s16_pos(c16, r), k = pos < 15 - pos ? pos : 15 - pos, ia = s16_elem(k, r),
                        partner = s16_elem(15 - pos, r);
              const double c = cs[wave][k][0], sn = cs[wave][k][1];
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const double other = __shfl(jr[i], (lane & 48) | partner, 64);
                jr[i] = c16 == ia ? c * jr[i] - sn * other : sn * other + c * jr[i];
              }
            }
            wave_lds_sync();
          }
          if (__ballot(any) == 0) break;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) G[4 * g + i][c16] = jr[i];
        wave_lds_sync();
        double jb[4];
#pragma unroll
        for (int st = 0; st < 4; ++st) jb[st] = G[4 * st + g][c16];
        pair_apply<4>(v, v.X, ba, bb, jb, 0, 1);
        wave_lds_sync();
      }
      __syncthreads();
    }
    const int done = rotated == 0;
    __syncthreads();
    if (done) break;
  }
  __syncthreads();
  svd_finalize_rm(v, fin, item_u(it, b), item_s(it, b), item_v(it, b));
}

static hipError_t launch_svd_qrp(int batch, int rows, int cols, const SvdItems& it, hipStream_t st);

// The Jacobi SVD itself (no QR preconditioning).
static hipError_t launch_svd_jacobi(int batch, int rows, int cols, const SvdItems& it, hipStream_t st,
                                    int fast_sweeps) {
  const size_t p = rows < cols ? rows : cols, q = rows < cols ? cols : rows;
  const size_t lds_bytes = (q * p + p * p) * sizeof(double);
  const int use_lds = lds_bytes <= (size_t)SVD_LDS_BYTES ? 1 : 0;
  if (p < 24) {
    hipLaunchKernelGGL(svd_jacobi_kernel, dim3(batch), dim3(SVD_THREADS), use_lds ? lds_bytes : 0, st, rows, cols, it,
                       use_lds);
    return hipGetLastError();
  }
  const int nb = bj_blocks((int)p);
  const int64_t elems = (int64_t)q * nb * BJ_B + (int64_t)nb * BJ_B * nb * BJ_B;
  hipLaunchKernelGGL(bj_init_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(elems, 256), 1024), batch), dim3(256), 0,
                     st, rows, cols, it);
  hipLaunchKernelGGL(bj_norm_kernel, dim3(batch), dim3(1024), 0, st, rows, cols, it);
  for (int sweep = 0; sweep < fast_sweeps; ++sweep) {
    for (int round = 0; round < nb - 1; ++round) {
      if (q > BJ_QS1 && q <= 2 * BJ_QS1)
        hipLaunchKernelGGL(bj_round_kernel<2>, dim3(nb / 2 * BJ_SPLIT, batch), dim3(256), 0, st, rows, cols, round,
                           sweep, it);
      else
        hipLaunchKernelGGL(bj_round_kernel<1>, dim3(nb / 2 * BJ_SPLIT, batch), dim3(256), 0, st, rows, cols, round,
                           sweep, it);
    }
  }
  hipLaunchKernelGGL(bj_finish_kernel, dim3(batch), dim3(1024), 0, st, rows, cols, fast_sweeps, it);
  return hipGetLastError();
}

hipError_t launch_svd_items(int batch, int rows, int cols, const SvdItems& it, hipStream_t st, int fast_sweeps) {
  if (batch <= 0 || rows <= 0 || cols <= 0 || std::min(rows, cols) > 1024 || std::max(rows, cols) > 4096)
    return hipErrorInvalidValue;
  if (it.n_ptr && (it.n_ptr != batch || batch > SVD_MAX_PTR)) return hipErrorInvalidValue;
  if (fast_sweeps < 0 || fast_sweeps > BJ_FAST_SWEEPS) return hipErrorInvalidValue;
  TimerScope ts(T_SVD, st);
  if (fast_sweeps == 0 && qrp_applies(rows, cols)) return launch_svd_qrp(batch, rows, cols, it, st);
  if (fast_sweeps == 0) fast_sweeps = bj_default_fast_sweeps(rows < cols ? rows : cols);
  return launch_svd_jacobi(batch, rows, cols, it, st, fast_sweeps);
}

// ---------------------------------------------------------------------------
// QR-preconditioned SVD.  A Pi = Q R (Householder, column pivoting: each step
// takes the remaining column of largest norm, lowest index on ties), then the
// block-Jacobi SVD of M = R^T in pivot order, M = U' S V'^T.  Since
// A Pi = Q V' S U'^T, the working matrix has left factor Q V' and right factor
// Pi U' (row pi_i of it is row i of U'); for rows < cols the working matrix is
// A^T and the two swap.  The signs are then set as on the plain path (the
// largest-magnitude entry of each left singular vector, lowest row on ties,
// positive).
//
// Step j is one launch of QRP_WG work-groups per matrix.  Every work-group
// finds the pivot and forms the reflector from the pivot column itself (the
// same code on the same data, so the same values), then each wave updates its
// columns (v^T a, a -= tau (v^T a) v, and the exact squared norm of rows
// j + 1.. as the next step's pivot key) and its rows of Q (Q <- Q H_j).  The
// pivot column is only read in its step, and the norms and taken flags are
// double-buffered between steps, so no work-group reads what another writes
// in the same launch.
// ---------------------------------------------------------------------------
constexpr int QRP_WG = 128;  // work-groups per matrix and step (one column and one row of Q per wave at q <= 512)

struct QrpView {
  double *Ac, *Q, *R, *M, *Up, *Vp, *nrm;
  int *tk, *piv;
  double* jw;
  int q, p;
  bool trans;
};

__host__ __device__ inline QrpView qrp_view(double* base, int rows, int cols) {
  QrpView v;
  v.trans = rows < cols;
  v.p = v.trans ? rows : cols;
  v.q = v.trans ? cols : rows;
  const size_t p = v.p, q = v.q;
  v.Ac = base;
  v.Q = v.Ac + q * p;
  v.R = v.Q + q * q;
  v.M = v.R + p * p;
  v.Up = v.M + p * p;
  v.Vp = v.Up + p * p;
  v.nrm = v.Vp + p * p;
  v.tk = (int*)(v.nrm + 2 * p);
  v.piv = v.tk + 2 * p;
  v.jw = v.nrm + 2 * p + (3 * p + 1) / 2 + 8;
  return v;
}

// Ac = the working matrix column-major, Q = I, R = 0, no column taken.
__global__ __launch_bounds__(256) void qrp_init_kernel(int rows, int cols, SvdItems it) {
  const QrpView v = qrp_view(item_w(it, blockIdx.y), rows, cols);
  const double* A = item_a(it, blockIdx.y);
  const int64_t q = v.q, p = v.p;
  const int64_t n1 = q * p, n2 = n1 + q * q, n3 = n2 + p * p, n4 = n3 + 2 * p;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n4; e += (int64_t)gridDim.x * 256) {
    if (e < n1) {
      const int64_t c = e / q, i = e - c * q;  // Ac[c q + i] = working A[i][c]
      v.Ac[e] = v.trans ? A[c * cols + i] : A[i * cols + c];
    } else if (e < n2) {
      const int64_t f = e - n1;
      v.Q[f] = (f / q == f % q) ? 1.0 : 0.0;
    } else if (e < n3) {
      v.R[e - n2] = 0.0;
    } else {
      v.tk[e - n3] = 0;
    }
  }
}

// Squared column norms of Ac, one wave per column (fixed order), into buffer 0.
__global__ __launch_bounds__(256) void qrp_norm_kernel(int rows, int cols, SvdItems it) {
  const QrpView v = qrp_view(item_w(it, blockIdx.y), rows, cols);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = blockIdx.x * 4 + wave; c < v.p; c += gridDim.x * 4) {
    const double* col = v.Ac + (size_t)c * v.q;
    double s2 = 0.0;
    for (int i = lane; i < v.q; i += 64) s2 += col[i] * col[i];
    s2 = wave_sum(s2);
    if (lane == 0) v.nrm[c] = s2;
  }
}

__global__ __launch_bounds__(256) void qrp_step_kernel(int rows, int cols, int j, SvdItems it) {
  __shared__ double xv[QRP_MAXQ];  // the reflector v (rows j .. q - 1)
  __shared__ double rd[4];
  __shared__ int ri[4];
  const QrpView v = qrp_view(item_w(it, blockIdx.y), rows, cols);
  const int q = v.q, p = v.p, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int sb = j & 1;
  const double* nin = v.nrm + sb * p;
  double* nout = v.nrm + (sb ^ 1) * p;
  const int* tin = v.tk + sb * p;
  int* tout = v.tk + (sb ^ 1) * p;
  const int len = q - j;
  // pivot: the untaken column of largest norm, lowest index on ties (NaN below
  // every number); the maximum is order-independent, so a butterfly does
  double bv = -2.0;
  int bi = 0x7fffffff;
  for (int c = tid; c < p; c += 256) {
    if (tin[c]) continue;
    const double x = nin[c] == nin[c] ? nin[c] : -1.0;
    if (x > bv) { bv = x; bi = c; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(bv, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
  }
  if (lane == 0) { rd[wave] = bv; ri[wave] = bi; }
  __syncthreads();
  int piv = ri[0];
  {
    double m = rd[0];
    for (int w = 1; w < 4; ++w)
      if (rd[w] > m || (rd[w] == m && ri[w] < piv)) { m = rd[w]; piv = ri[w]; }
  }
  __syncthreads();
  // the pivot column's rows j .. q - 1 and their squared norm (the same fixed
  // order in every work-group)
  const double* pc = v.Ac + (size_t)piv * q + j;
  double ss = 0.0;
  for (int i = tid; i < len; i += 256) {
    const double x = pc[i];
    xv[i] = x;
    ss += x * x;
  }
  ss = wave_sum(ss);
  if (lane == 0) rd[wave] = ss;
  __syncthreads();
  const double sig2 = ((rd[0] + rd[1]) + rd[2]) + rd[3], x0 = xv[0];
  const double sigma = sqrt(sig2);
  const double alpha = x0 >= 0.0 ? -sigma : sigma;  // H x = alpha e_0
  const double v0 = x0 - alpha;
  const double vtv = sig2 - x0 * x0 + v0 * v0;
  const double tau = vtv > 0.0 ? 2.0 / vtv : 0.0;
  __syncthreads();
  if (tid == 0) xv[0] = v0;
  __syncthreads();
  if (blockIdx.x == 0 && tid == 0) {
    v.piv[j] = piv;
    v.R[(size_t)j * p + piv] = alpha;
  }
  // wave g (over the grid) updates column g and row g of Q (then g + 4 QRP_WG,
  // ...); the two are independent, so their loads are in flight together
  const int gw = blockIdx.x * 4 + wave, stride = 4 * gridDim.x;
  const int n = p > q ? p : q;
  for (int g = gw; g < n; g += stride) {
    const bool hc = g < p;
    const bool live = hc && tin[g] == 0 && g != piv;
    const bool hr = g < q;
    double* col = v.Ac + (size_t)(hc ? g : 0) * q + j;
    double* qr = v.Q + (size_t)(hr ? g : 0) * q + j;
    double dc = 0.0, dr = 0.0;
    for (int i = lane; i < len; i += 64) {
      const double x = xv[i];
      if (live) dc += x * col[i];
      if (hr) dr += x * qr[i];
    }
    dc = wave_sum(dc);
    dr = wave_sum(dr);
    const double fc = tau * dc, fr = tau * dr;
    double s2 = 0.0, head = 0.0;
    for (int i = lane; i < len; i += 64) {
      const double x = xv[i];
      if (live) {
        const double y = col[i] - fc * x;
        col[i] = y;
        if (i == 0) head = y;
        else s2 += y * y;
      }
      if (hr) qr[i] -= fr * x;
    }
    if (hc) {
      s2 = wave_sum(s2);
      if (lane == 0) {
        tout[g] = live ? 0 : 1;
        nout[g] = live ? s2 : 0.0;
        if (live) v.R[(size_t)j * p + g] = head;
      }
    }
  }
}

// M = R^T in pivot order: M[i][k] = R[k][pi_i] (lower triangular).
__global__ __launch_bounds__(256) void qrp_form_kernel(int rows, int cols, SvdItems it) {
  const QrpView v = qrp_view(item_w(it, blockIdx.y), rows, cols);
  const int64_t p = v.p;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < p * p; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / p, k = e - i * p;
    v.M[e] = v.R[k * p + v.piv[i]];
  }
}

// The permuted factor: row pi_i of Pi U' is row i of U' (into U for rows <
// cols, else into V; both p x p there).
__global__ __launch_bounds__(256) void qrp_perm_kernel(int rows, int cols, SvdItems it) {
  const QrpView v = qrp_view(item_w(it, blockIdx.y), rows, cols);
  double* out = v.trans ? item_u(it, blockIdx.y) : item_v(it, blockIdx.y);
  const int64_t p = v.p;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < p * p; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / p, c = e - i * p;
    out[(int64_t)v.piv[i] * p + c] = v.Up[e];
  }
}

// Signs: per singular vector (one wave each), the largest-magnitude entry of
// the left vector (lowest row on ties) made positive, flipping both vectors.
__global__ __launch_bounds__(256) void qrp_sign_kernel(int rows, int cols, SvdItems it) {
  const int b = blockIdx.y;
  double* U = item_u(it, b);
  double* V = item_v(it, b);
  const int p = rows < cols ? rows : cols;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = blockIdx.x * 4 + wave; c < p; c += gridDim.x * 4) {
    double best = -1.0, bval = 0.0;
    int bi = 0x7fffffff;
    for (int i = lane; i < rows; i += 64) {
      const double x = U[(int64_t)i * p + c];
      if (fabs(x) > best) { best = fabs(x); bval = x; bi = i; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64), ov = __shfl_xor(bval, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bval = ov; bi = oi; }
    }
    if (bval < 0.0) {
      for (int i = lane; i < rows; i += 64) U[(int64_t)i * p + c] = -U[(int64_t)i * p + c];
      for (int i = lane; i < cols; i += 64) V[(int64_t)i * p + c] = -V[(int64_t)i * p + c];
    }
  }
}

// Host views of an item's pointers.
static double* h_item_u(const SvdItems& it, int b) { return it.n_ptr ? it.Up[b] : it.U + b * it.sU; }
static double* h_item_s(const SvdItems& it, int b) { return it.n_ptr ? it.Sp[b] : it.S + b * it.sS; }
static double* h_item_v(const SvdItems& it, int b) { return it.n_ptr ? it.Vp[b] : it.V + b * it.sV; }
static double* h_item_w(const SvdItems& it, int b) { return it.n_ptr ? it.Wp[b] : it.W + b * it.sW; }

static hipError_t launch_svd_qrp(int batch, int rows, int cols, const SvdItems& it, hipStream_t st) {
  const int p = rows < cols ? rows : cols, q = rows < cols ? cols : rows;
  const int64_t elems = (int64_t)q * p + (int64_t)q * q + (int64_t)p * p + 2 * p;
  hipLaunchKernelGGL(qrp_init_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(elems, 256), 1024), batch), dim3(256),
                     0, st, rows, cols, it);
  hipLaunchKernelGGL(qrp_norm_kernel, dim3((unsigned)ceil_div(p, 4), batch), dim3(256), 0, st, rows, cols, it);
  for (int j = 0; j < p; ++j)
    hipLaunchKernelGGL(qrp_step_kernel, dim3(QRP_WG, batch), dim3(256), 0, st, rows, cols, j, it);
  hipLaunchKernelGGL(qrp_form_kernel, dim3((unsigned)ceil_div((int64_t)p * p, 256), batch), dim3(256), 0, st, rows,
                     cols, it);
  // the Jacobi SVD of M (p x p) into U', the item's S, V'
  SvdItems in{};
  if (it.n_ptr) {
    in.n_ptr = batch;
    for (int b = 0; b < batch; ++b) {
      const QrpView v = qrp_view(h_item_w(it, b), rows, cols);
      in.Ap[b] = v.M;
      in.Up[b] = v.Up;
      in.Sp[b] = h_item_s(it, b);
      in.Vp[b] = v.Vp;
      in.Wp[b] = v.jw;
    }
  } else {
    const QrpView v = qrp_view(it.W, rows, cols);
    in.A = v.M;
    in.U = v.Up;
    in.S = it.S;
    in.V = v.Vp;
    in.W = v.jw;
    in.sA = in.sU = in.sV = in.sW = it.sW;
    in.sS = it.sS;
  }
  hipError_t e = launch_svd_jacobi(batch, p, p, in, st, 16);
  if (e != hipSuccess) return e;
  // left factor of the working matrix Q V' (q x p); right factor Pi U'
  for (int b = 0; b < batch; ++b) {
    const QrpView v = qrp_view(h_item_w(it, b), rows, cols);
    double* lo = v.trans ? h_item_v(it, b) : h_item_u(it, b);
    e = launch_small_gemm(q, p, p, v.Q, q, false, v.Vp, p, false, nullptr, nullptr, nullptr, lo, p, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(qrp_perm_kernel, dim3((unsigned)ceil_div((int64_t)p * p, 256), batch), dim3(256), 0, st, rows,
                     cols, it);
  hipLaunchKernelGGL(qrp_sign_kernel, dim3((unsigned)ceil_div(p, 4), batch), dim3(256), 0, st, rows, cols, it);
  return hipGetLastError();
}

hipError_t launch_svd(int batch, int rows, int cols, const double* A, int64_t strideA, double* U, int64_t strideU,
                      double* S, int64_t strideS, double* V, int64_t strideV, void* ws, hipStream_t st,
                      int fast_sweeps) {
  SvdItems it{};
  it.A = A;
  it.U = U;
  it.S = S;
  it.V = V;
  it.W = (double*)ws;
  it.sA = strideA;
  it.sU = strideU;
  it.sS = strideS;
  it.sV = strideV;
  it.sW = (int64_t)svd_ws_doubles(rows, cols);
  return launch_svd_items(batch, rows, cols, it, st, fast_sweeps);
}

}  // namespace cabs
