// Small FP64 products for the k x k algebra of the sketching routine and the
// orthogonalisation: C = diag(dl) op(A) diag(dm) op(B) diag(dr), one 16 x 16
// output tile per wave on the FP64 MFMA (v_mfma_f64_16x16x4f64).
#include "common.hpp"
#include "kernels.hpp"

namespace cabs {

struct SmallGemmArgs {
  int M, N, K;
  const double* A; int lda; int transA;
  const double* B; int ldb; int transB;
  const double* dl; const double* dm; const double* dr;
  double* C; int ldc;
};

__global__ __launch_bounds__(256) void small_gemm_kernel(SmallGemmArgs g) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int tilesN = (g.N + 15) / 16;
  const int tile = blockIdx.x * 4 + wave;
  const int tm = tile / tilesN, tn = tile % tilesN;
  if (tm * 16 >= g.M) return;
  const int r = lane & 15, grp = lane >> 4;
  const int row = tm * 16 + r;   // A row owned for the A fragment
  const int col = tn * 16 + r;   // B column owned for the B fragment
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int kb = 0; kb < g.K; kb += 4) {
    const int k = kb + grp;
    double av = 0.0, bv = 0.0;
    if (k < g.K) {
      if (row < g.M) av = g.transA ? g.A[(int64_t)k * g.lda + row] : g.A[(int64_t)row * g.lda + k];
      if (col < g.N) bv = g.transB ? g.B[(int64_t)col * g.ldb + k] : g.B[(int64_t)k * g.ldb + col];
      if (g.dm) av *= g.dm[k];
    }
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
  const int oc = tn * 16 + r;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int orow = tm * 16 + out_row<double>(grp, i);
    if (orow < g.M && oc < g.N) {
      double v = acc[i];
      if (g.dl) v *= g.dl[orow];
      if (g.dr) v *= g.dr[oc];
      g.C[(int64_t)orow * g.ldc + oc] = v;
    }
  }
}

hipError_t launch_small_gemm(int M, int N, int K, const double* A, int lda, bool transA, const double* B, int ldb,
                             bool transB, const double* dl, const double* dm, const double* dr, double* C, int ldc,
                             hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
  SmallGemmArgs g{M, N, K, A, lda, transA ? 1 : 0, B, ldb, transB ? 1 : 0, dl, dm, dr, C, ldc};
  const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
  hipLaunchKernelGGL(small_gemm_kernel, dim3((tiles + 3) / 4), dim3(256), 0, st, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pivoted Cholesky of a batch of positive semidefinite p x p matrices (FP64),
// one work-group each: G[order, order] ~ R^T R, R upper trapezoidal in pivot
// order.  Output Rf (p x p, row-major): row k is R's row k with its columns in
// the ORIGINAL index order (zero at indices pivoted earlier), rows from the
// rank on are zero.  Step k takes the largest remaining diagonal (lowest index
// on ties) and stops once it is <= tol (rank = k).
//
// The upper triangle of the symmetric matrix stays in registers: the 6 x 6
// tiles (TR, TC), TR <= TC, of a 34 x 34 tile grid (p <= 204) are numbered row
// by row and thread t < 595 of the 640 owns tile t.  A step broadcasts the pivot row
// through LDS; each thread updates its tile by the outer product of 6 + 6
// entries of that row; the diagonal is kept in LDS.
constexpr int PC_T = 6;                   // tile edge
constexpr int PC_G = 34;                  // tiles per dimension
constexpr int PC_NT = PC_G * (PC_G + 1) / 2;
constexpr int PC_MAXP = PC_G * PC_T;      // 204
constexpr int PC_THREADS = 640;           // 10 waves: >= PC_NT tile owners

__global__ __launch_bounds__(PC_THREADS) void pchol_kernel(int p, const double* __restrict__ G, int64_t strideG, double tol,
                                                     double* __restrict__ Rf, int64_t strideR) {
  __shared__ double rowk[PC_MAXP];
  __shared__ double wbest[2][16];
  __shared__ int wbi[2][16];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  constexpr int NW = PC_THREADS / 64;
  const double* Gb = G + blockIdx.x * strideG;
  double* Rb = Rf + blockIdx.x * strideR;
  // tile of this thread: row-major over the upper triangle of the tile grid
  int tr = 0, rem = tid;
  while (tr < PC_G && rem >= PC_G - tr) { rem -= PC_G - tr; ++tr; }
  const bool owner = tid < PC_NT;
  const int r0 = owner ? PC_T * tr : PC_MAXP, c0 = owner ? PC_T * (tr + rem) : PC_MAXP;
  double val[PC_T][PC_T];
#pragma unroll
  for (int a = 0; a < PC_T; ++a)
#pragma unroll
    for (int b = 0; b < PC_T; ++b)
      val[a][b] = (r0 + a < p && c0 + b < p) ? Gb[(int64_t)(r0 + a) * p + c0 + b] : 0.0;
  // index c = tid (p <= PC_MAXP < PC_THREADS): its remaining diagonal and whether it was pivoted
  const bool mine = tid < p;
  double diag = mine ? Gb[(int64_t)tid * p + tid] : 0.0;
  bool done = !mine;
  // candidate for the next pivot: largest remaining diagonal, lowest index on ties
  auto propose = [&](int slot) {
    double bd = done ? -1.0 : diag;
    int bi = done ? 0x7fffffff : tid;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double od = __shfl_xor(bd, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (od > bd || (od == bd && oi < bi)) { bd = od; bi = oi; }
    }
    if (lane == 0) { wbest[slot][wave] = bd; wbi[slot][wave] = bi; }
  };
  propose(0);
  __syncthreads();
  int k = 0;
  for (; k < p; ++k) {
    const int slot = k & 1;
    // every thread reduces the wave candidates the same way
    double d = wbest[slot][0];
    int piv = wbi[slot][0];
#pragma unroll
    for (int w = 1; w < NW; ++w)
      if (wbest[slot][w] > d || (wbest[slot][w] == d && wbi[slot][w] < piv)) { d = wbest[slot][w]; piv = wbi[slot][w]; }
    if (!(d > tol)) break;  // uniform: nothing left above the threshold
    const double rkk = sqrt(d);
    // the pivot row of R over all indices, written in full (zero at pivoted
    // indices): entries (piv, j > piv) sit in the tile row of piv, entries
    // (i < piv, piv) in its tile column, r_kk itself at piv
    if (piv >= r0 && piv < r0 + PC_T) {
#pragma unroll
      for (int a = 0; a < PC_T; ++a)
        if (r0 + a == piv) {
#pragma unroll
          for (int b = 0; b < PC_T; ++b) {
            const int c = c0 + b;
            if (c < p && c > piv) rowk[c] = val[a][b] / rkk;
          }
        }
    }
    if (piv >= c0 && piv < c0 + PC_T) {
#pragma unroll
      for (int b = 0; b < PC_T; ++b)
        if (c0 + b == piv) {
#pragma unroll
          for (int a = 0; a < PC_T; ++a) {
            const int c = r0 + a;
            if (c < piv) rowk[c] = val[a][b] / rkk;
          }
        }
    }
    if (tid == piv) rowk[piv] = rkk;
    if (tid >= p && tid < PC_MAXP) rowk[tid] = 0.0;  // padding read by the edge tiles
    __syncthreads();
    // entries at pivoted indices are exact zeros of the Schur complement, so
    // the row may carry the (zero-valued) stored entries there; mask them
    double rmine = mine && !done ? rowk[tid] : 0.0;
    if (tid == piv) rmine = rkk;
    // Schur complement of the upper triangle; the pivot's own row and column
    // change but are never read again
    double rj[PC_T];
#pragma unroll
    for (int b = 0; b < PC_T; ++b) rj[b] = c0 + b < PC_MAXP ? rowk[c0 + b] : 0.0;
#pragma unroll
    for (int a = 0; a < PC_T; ++a) {
      const double ra = r0 + a < PC_MAXP ? rowk[r0 + a] : 0.0;
#pragma unroll
      for (int b = 0; b < PC_T; ++b) val[a][b] -= ra * rj[b];
    }
    if (mine) {
      Rb[(int64_t)k * p + tid] = rmine;
      if (!done) diag -= rmine * rmine;
      if (tid == piv) done = true;
    }
    propose(slot ^ 1);
    __syncthreads();
  }
  for (int e = tid; e < (p - k) * p; e += PC_THREADS) Rb[(int64_t)k * p + e] = 0.0;
}

hipError_t launch_pchol(int batch, int p, const double* G, int64_t strideG, double tol, double* Rf, int64_t strideR,
                        hipStream_t st) {
  if (batch <= 0 || p <= 0 || p > PC_MAXP) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pchol_kernel, dim3(batch), dim3(PC_THREADS), 0, st, p, G, strideG, tol, Rf, strideR);
  return hipGetLastError();
}

}  // namespace cabs
