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
#include "common.hpp"
#include "kernels.hpp"

namespace cabs {

constexpr int SVD_THREADS = 1024;
constexpr int SVD_MAX_SWEEPS = 40;
constexpr int SVD_LDS_BYTES = 60 * 1024;

__host__ __device__ static inline int even_up(int p) { return p + (p & 1); }

// Per-matrix scratch in doubles: X (q*p), V (p*p), sigma (p), plus rank/sign (p ints each).
__host__ __device__ static inline size_t svd_ws_doubles(int rows, int cols) {
  const size_t p = rows < cols ? rows : cols, q = rows < cols ? cols : rows;
  return q * p + p * p + 3 * p + 64;
}

size_t svd_ws_bytes(int batch, int rows, int cols) {
  return (size_t)batch * svd_ws_doubles(rows, cols) * sizeof(double) + 256;
}

__global__ __launch_bounds__(SVD_THREADS) void svd_jacobi_kernel(int rows, int cols, const double* __restrict__ A,
                                                                  int64_t strideA, double* __restrict__ U,
                                                                  int64_t strideU, double* __restrict__ S,
                                                                  int64_t strideS, double* __restrict__ Vout,
                                                                  int64_t strideV, double* __restrict__ ws,
                                                                  int use_lds) {
  extern __shared__ double lds[];
  __shared__ int rotated;
  const int b = blockIdx.x;
  const bool trans = rows < cols;
  const int p = trans ? rows : cols;
  const int q = trans ? cols : rows;
  const int pe = even_up(p);
  double* base = ws + (size_t)b * svd_ws_doubles(rows, cols);
  double* X = use_lds ? lds : base;              // column-major q x p
  double* V = use_lds ? lds + (size_t)q * p : base + (size_t)q * p;  // column-major p x p
  double* sig = base + (size_t)q * p + (size_t)p * p;
  int* rank = (int*)(sig + p);
  double* sgn = sig + 2 * p;
  const double* Ab = A + b * strideA;
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

  // Singular values = column norms (one wave per column).
  for (int j = wave; j < p; j += nwaves) {
    double s2 = 0.0;
    for (int i = lane; i < q; i += 64) s2 += X[(size_t)j * q + i] * X[(size_t)j * q + i];
    s2 = wave_sum(s2);
    if (lane == 0) sig[j] = sqrt(s2);
  }
  __syncthreads();
  // Descending order, lower column index first on ties.
  // NaN (from non-finite input) ranks below every number so that ranks stay a permutation.
  for (int j = tid; j < p; j += SVD_THREADS) {
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
    const double* lv = trans ? V + (size_t)j * p : X + (size_t)j * q;
    const int len = trans ? p : q;
    double best = -1.0;
    int bi = 0x7fffffff;
    double bval = 0.0;
    for (int i = lane; i < len; i += 64) {
      const double v = lv[i];
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
  double* Ub = U + b * strideU;
  double* Vb = Vout + b * strideV;
  double* Sb = S + b * strideS;
  for (int j = tid; j < p; j += SVD_THREADS) Sb[rank[j]] = sig[j];
  // Left factor of the working problem: X / sigma (q x p); right: V (p x p).
  for (int e = tid; e < q * p; e += SVD_THREADS) {
    const int j = e / q, i = e % q;
    const double sj = sig[j];
    const double v = sj > 0.0 ? sgn[j] * X[e] / sj : 0.0;
    if (!trans) Ub[(int64_t)i * p + rank[j]] = v;   // U: rows x p
    else Vb[(int64_t)i * p + rank[j]] = v;          // V: cols x p
  }
  for (int e = tid; e < p * p; e += SVD_THREADS) {
    const int j = e / p, i = e % p;
    const double v = sgn[j] * V[e];
    if (!trans) Vb[(int64_t)i * p + rank[j]] = v;   // V: cols x p
    else Ub[(int64_t)i * p + rank[j]] = v;          // U: rows x p
  }
}

hipError_t launch_svd(int batch, int rows, int cols, const double* A, int64_t strideA, double* U, int64_t strideU,
                      double* S, int64_t strideS, double* V, int64_t strideV, void* ws, hipStream_t st) {
  if (batch <= 0 || rows <= 0 || cols <= 0 || rows > 1024 || cols > 1024) return hipErrorInvalidValue;
  const size_t p = rows < cols ? rows : cols, q = rows < cols ? cols : rows;
  const size_t lds_bytes = (q * p + p * p) * sizeof(double);
  const int use_lds = lds_bytes <= (size_t)SVD_LDS_BYTES ? 1 : 0;
  hipLaunchKernelGGL(svd_jacobi_kernel, dim3(batch), dim3(SVD_THREADS), use_lds ? lds_bytes : 0, st, rows, cols, A,
                     strideA, U, strideU, S, strideS, V, strideV, (double*)ws, use_lds);
  return hipGetLastError();
}

}  // namespace cabs
