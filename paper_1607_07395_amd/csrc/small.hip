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

}  // namespace cabs
