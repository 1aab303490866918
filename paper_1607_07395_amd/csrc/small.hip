// Small FP64 products for the k x k algebra of the sketching routine and the
// orthogonalisation: C = diag(dl) op(A) diag(dm) op(B) diag(dr), one 16 x 16
// output tile per wave on the FP64 MFMA (v_mfma_f64_16x16x4f64).
#include <type_traits>

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
  // The loads of SG_U k-steps are issued together (from clamped, always valid
  // addresses; out-of-range entries are replaced by zeros), then their MFMAs.
  constexpr int SG_U = 8;
  const int rowc = row < g.M ? row : 0, colc = col < g.N ? col : 0;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int kb = 0; kb < g.K; kb += 4 * SG_U) {
    double av[SG_U], bv[SG_U];
#pragma unroll
    for (int u = 0; u < SG_U; ++u) {
      const int k = kb + 4 * u + grp;
      const bool kin = k < g.K;
      const int kc = kin ? k : 0;
      double a = g.transA ? g.A[(int64_t)kc * g.lda + rowc] : g.A[(int64_t)rowc * g.lda + kc];
      const double b = g.transB ? g.B[(int64_t)colc * g.ldb + kc] : g.B[(int64_t)kc * g.ldb + colc];
      if (g.dm) a *= g.dm[kc];
      av[u] = kin && row < g.M ? a : 0.0;
      bv[u] = kin && col < g.N ? b : 0.0;
    }
#pragma unroll
    for (int u = 0; u < SG_U; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
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
// The upper triangle of the symmetric matrix stays in registers: the 8 x 8
// tiles (TR, TC), TR <= TC, of a 26 x 26 tile grid (p <= 208) are numbered row
// by row and thread t < 351 of the 384 owns tile t.  A step broadcasts the
// pivot row of R through LDS (written by the owners of the pivot's tile row
// and tile column, already divided by r_kk); each owner updates its tile by the
// outer product of 8 + 8 entries of that row.  Thread c < p keeps the
// remaining diagonal entry c, so only the first PC_CW waves hold pivot
// candidates.
constexpr int PC_T = 8;                   // tile edge
constexpr int PC_G = 26;                  // tiles per dimension
constexpr int PC_NT = PC_G * (PC_G + 1) / 2;
constexpr int PC_MAXP = PC_G * PC_T;      // 208
constexpr int PC_THREADS = 384;           // 6 waves: >= PC_NT tile owners, >= PC_MAXP diagonal keepers
constexpr int PC_CW = (PC_MAXP + 63) / 64;  // waves with candidates

__global__ __launch_bounds__(PC_THREADS) void pchol_kernel(int p, const double* __restrict__ G, int64_t strideG, double tol,
                                                     double* __restrict__ Rf, int64_t strideR) {
  __shared__ double rowk[PC_MAXP];  // row k of R
  __shared__ double wbest[2][PC_CW];
  __shared__ int wbi[2][PC_CW];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
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
  // index c = tid (p <= PC_MAXP <= PC_THREADS): its remaining diagonal and whether it was pivoted
  const bool mine = tid < p;
  double diag = mine ? Gb[(int64_t)tid * p + tid] : 0.0;
  bool done = !mine;
  // candidate for the next pivot: largest remaining diagonal, lowest index on
  // ties (a commutative choice, so any reduction order gives the same one):
  // DPP exchanges within rows of 16 lanes, then across the four rows
  auto better = [](double od, int oi, double& bd, int& bi) {
    if (od > bd || (od == bd && oi < bi)) { bd = od; bi = oi; }
  };
  auto propose = [&](int slot) {
    double bd = done ? -1.0 : diag;
    int bi = done ? 0x7fffffff : tid;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double od = __hiloint2double(dpp_xchg(__double2hiint(bd), c), dpp_xchg(__double2loint(bd), c));
      const int oi = dpp_xchg(bi, c);
      better(od, oi, bd, bi);
    }
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
      const double od = __shfl_xor(bd, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      better(od, oi, bd, bi);
    }
    if (lane == 0) { wbest[slot][wave] = bd; wbi[slot][wave] = bi; }
  };
  for (int e = tid; e < PC_MAXP; e += PC_THREADS) rowk[e] = 0.0;
  if (wave < PC_CW) propose(0);  // uniform per wave
  __syncthreads();
  int k = 0;
  for (; k < p; ++k) {
    const int slot = k & 1;
    // every thread reduces the wave candidates the same way (all loaded first;
    // the empty asm keeps the loads together ahead of their uses)
    double wd[PC_CW];
    int wi[PC_CW];
#pragma unroll
    for (int w = 0; w < PC_CW; ++w) {
      wd[w] = wbest[slot][w];
      wi[w] = wbi[slot][w];
    }
#pragma unroll
    for (int w = 0; w < PC_CW; ++w) asm volatile("" : "+v"(wd[w]), "+v"(wi[w]));
    double d = wd[0];
    int piv = wi[0];
#pragma unroll
    for (int w = 1; w < PC_CW; ++w) better(wd[w], wi[w], d, piv);
    if (!(d > tol)) break;  // uniform: nothing left above the threshold
    const double rkk = sqrt(d);
    const double inv = 1.0 / rkk;
    // Row k of R over all indices c: (pivot row of the Schur complement)[c] /
    // r_kk, and r_kk at piv.  Entries (piv, c > piv) sit in the tile row of
    // piv, entries (c <= piv, piv) in its tile column: the owners there write
    // those indices of rowk.  The lanes of a wave that take part share one tile row
    // (one r0) or one tile column (one c0), so the row (column) of the tile is
    // a wave-uniform index: a scalar switch picks it with constant register
    // indices.
    auto emit_row = [&](auto A) {
      constexpr int a = decltype(A)::value;
#pragma unroll
      for (int b = 0; b < PC_T; ++b)
        if (c0 + b > piv) rowk[c0 + b] = val[a][b] * inv;
    };
    auto emit_col = [&](auto B) {
      constexpr int b = decltype(B)::value;
#pragma unroll
      for (int a = 0; a < PC_T; ++a)
        if (r0 + a <= piv) rowk[r0 + a] = r0 + a == piv ? rkk : val[a][b] * inv;
    };
    static_assert(PC_T == 8, "the switches below list 8 cases");
    const int ai = piv - r0, bi = piv - c0;
    if ((unsigned)ai < (unsigned)PC_T) {
      switch (__builtin_amdgcn_readfirstlane(ai)) {
        case 0: emit_row(std::integral_constant<int, 0>{}); break;
        case 1: emit_row(std::integral_constant<int, 1>{}); break;
        case 2: emit_row(std::integral_constant<int, 2>{}); break;
        case 3: emit_row(std::integral_constant<int, 3>{}); break;
        case 4: emit_row(std::integral_constant<int, 4>{}); break;
        case 5: emit_row(std::integral_constant<int, 5>{}); break;
        case 6: emit_row(std::integral_constant<int, 6>{}); break;
        default: emit_row(std::integral_constant<int, 7>{}); break;
      }
    }
    if ((unsigned)bi < (unsigned)PC_T) {
      switch (__builtin_amdgcn_readfirstlane(bi)) {
        case 0: emit_col(std::integral_constant<int, 0>{}); break;
        case 1: emit_col(std::integral_constant<int, 1>{}); break;
        case 2: emit_col(std::integral_constant<int, 2>{}); break;
        case 3: emit_col(std::integral_constant<int, 3>{}); break;
        case 4: emit_col(std::integral_constant<int, 4>{}); break;
        case 5: emit_col(std::integral_constant<int, 5>{}); break;
        case 6: emit_col(std::integral_constant<int, 6>{}); break;
        default: emit_col(std::integral_constant<int, 7>{}); break;
      }
    }
    __syncthreads();
    // Entries of rowk at indices pivoted earlier are zeros of the Schur
    // complement up to rounding: they only update entries that are never read
    // again, and R gets exact zeros there.
    auto rk = [&](int c) { return rowk[c]; };
    if (owner) {
      // all loads first (the empty asm keeps the compiler from sinking a load
      // into a branch of its own), then the outer product
      double x[2 * PC_T];
#pragma unroll
      for (int a = 0; a < PC_T; ++a) x[a] = rk(r0 + a);
#pragma unroll
      for (int b = 0; b < PC_T; ++b) x[PC_T + b] = rk(c0 + b);
#pragma unroll
      for (int i = 0; i < 2 * PC_T; ++i) asm volatile("" : "+v"(x[i]));
      // Schur complement of the upper triangle; the pivot's own row and
      // column change but are never read again
#pragma unroll
      for (int a = 0; a < PC_T; ++a)
#pragma unroll
        for (int b = 0; b < PC_T; ++b) val[a][b] -= x[a] * x[PC_T + b];
    }
    if (mine) {
      const double rmine = done ? 0.0 : rk(tid);
      Rb[(int64_t)k * p + tid] = rmine;
      if (!done) diag -= rmine * rmine;
      if (tid == piv) done = true;
    }
    if (wave < PC_CW) propose(slot ^ 1);  // uniform per wave
    __syncthreads();
  }
  for (int e = tid; e < (p - k) * p; e += PC_THREADS) Rb[(int64_t)k * p + e] = 0.0;
}

// The same factorisation for p > PC_MAXP, one launch per step over many
// work-groups, in a workspace per matrix: the Schur complement S (upper
// triangle, row-major p x p), the remaining diagonal and the pivoted flags
// (each double-buffered, so that a step reads the previous step's values while
// it writes its own), and a stop word.  Step k: every work-group finds the
// pivot the same way (largest remaining diagonal, lowest index on ties; stop
// once it is <= tol), forms row k of R in LDS from the pivot's row and column
// of S, work-group 0 writes it, and the work-groups update their rows of S
// (rows dealt cyclically) and of the diagonal.  The pivot's row and column,
// which the row is read from, are never updated, so the reads and the updates
// of one step do not overlap.  Entries of R at indices pivoted earlier are
// exact zeros, as in pchol_kernel.
constexpr int PCG_WG = 128;  // work-groups per matrix (about four rows of the update each at p = 500)

struct PcgView {
  double *S, *dg0, *dg1;
  int *tk0, *tk1, *ctl;
};
__host__ __device__ inline size_t pcg_ws_doubles(int p) { return (size_t)p * p + 4 * (size_t)p + 8; }
__device__ __forceinline__ PcgView pcg_view(void* ws, int p, int b) {
  double* base = (double*)ws + (size_t)b * pcg_ws_doubles(p);
  PcgView v;
  v.S = base;
  v.dg0 = base + (size_t)p * p;
  v.dg1 = v.dg0 + p;
  v.tk0 = (int*)(v.dg1 + p);
  v.tk1 = v.tk0 + p;
  v.ctl = v.tk1 + p;
  return v;
}

size_t pchol_ws_bytes(int batch, int p) {
  return p > PC_MAXP ? (size_t)batch * pcg_ws_doubles(p) * sizeof(double) + 256 : 256;
}

__global__ __launch_bounds__(256) void pcg_init_kernel(int p, const double* __restrict__ G, int64_t strideG,
                                                       double* __restrict__ Rf, int64_t strideR, void* ws) {
  const int b = blockIdx.y;
  const PcgView v = pcg_view(ws, p, b);
  const double* Gb = G + b * strideG;
  double* Rb = Rf + b * strideR;
  const int64_t pp = (int64_t)p * p;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < pp; e += (int64_t)gridDim.x * 256) {
    v.S[e] = Gb[e];
    Rb[e] = 0.0;
  }
  for (int c = blockIdx.x * 256 + threadIdx.x; c < p; c += gridDim.x * 256) {
    v.dg0[c] = Gb[(int64_t)c * p + c];
    v.tk0[c] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) v.ctl[0] = 0;
}

__global__ __launch_bounds__(256) void pcg_step_kernel(int p, int k, double tol, double* __restrict__ Rf,
                                                       int64_t strideR, void* ws) {
  __shared__ double rowk[1024];
  __shared__ double wbd[4];
  __shared__ int wbi[4];
  const int b = blockIdx.y, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const PcgView v = pcg_view(ws, p, b);
  if (v.ctl[0]) return;  // stopped at an earlier step
  const double* dgc = (k & 1) ? v.dg1 : v.dg0;
  double* dgn = (k & 1) ? v.dg0 : v.dg1;
  const int* tkc = (k & 1) ? v.tk1 : v.tk0;
  int* tkn = (k & 1) ? v.tk0 : v.tk1;
  // pivot: largest remaining diagonal, lowest index on ties (commutative, so any order gives it)
  double bd = -1.0;
  int bi = 0x7fffffff;
  for (int c = tid; c < p; c += 256)
    if (!tkc[c]) {
      const double d = dgc[c];
      if (d > bd || (d == bd && c < bi)) { bd = d; bi = c; }
    }
  for (int off = 1; off < 64; off <<= 1) {
    const double od = __shfl_xor(bd, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (od > bd || (od == bd && oi < bi)) { bd = od; bi = oi; }
  }
  if (lane == 0) { wbd[wave] = bd; wbi[wave] = bi; }
  __syncthreads();
  double d = wbd[0];
  int piv = wbi[0];
  for (int w = 1; w < 4; ++w)
    if (wbd[w] > d || (wbd[w] == d && wbi[w] < piv)) { d = wbd[w]; piv = wbi[w]; }
  if (!(d > tol)) {  // uniform: nothing left above the threshold; rows k.. of R stay zero
    if (blockIdx.x == 0 && tid == 0) v.ctl[0] = 1;
    return;
  }
  const double rkk = sqrt(d);
  const double inv = 1.0 / rkk;
  // row k of R: the pivot's row of S (upper triangle: S[piv][c] for c > piv, S[c][piv] for c < piv)
  for (int c = tid; c < p; c += 256) {
    double r = 0.0;
    if (!tkc[c]) r = c == piv ? rkk : (c > piv ? v.S[(int64_t)piv * p + c] : v.S[(int64_t)c * p + piv]) * inv;
    rowk[c] = r;
  }
  __syncthreads();
  if (blockIdx.x == 0)
    for (int c = tid; c < p; c += 256) Rf[b * strideR + (int64_t)k * p + c] = rowk[c];
  // this work-group's rows: the flags and diagonal for the next step, and the Schur update
  for (int i = blockIdx.x; i < p; i += gridDim.x) {
    const bool live = !tkc[i] && i != piv;
    if (tid == 0) {
      tkn[i] = live ? 0 : 1;
      dgn[i] = live ? dgc[i] - rowk[i] * rowk[i] : dgc[i];
    }
    if (!live) continue;  // uniform
    const double ri = rowk[i];
    double* Si = v.S + (int64_t)i * p;
    for (int j = i + tid; j < p; j += 256)
      if (!tkc[j] && j != piv) Si[j] -= ri * rowk[j];
  }
}

hipError_t launch_pchol(int batch, int p, const double* G, int64_t strideG, double tol, double* Rf, int64_t strideR,
                        void* ws, hipStream_t st) {
  if (batch <= 0 || p <= 0 || p > 1024) return hipErrorInvalidValue;
  if (p <= PC_MAXP) {
    hipLaunchKernelGGL(pchol_kernel, dim3(batch), dim3(PC_THREADS), 0, st, p, G, strideG, tol, Rf, strideR);
    return hipGetLastError();
  }
  if (!ws) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pcg_init_kernel, dim3(64, batch), dim3(256), 0, st, p, G, strideG, Rf, strideR, ws);
  for (int k = 0; k < p; ++k)
    hipLaunchKernelGGL(pcg_step_kernel, dim3(PCG_WG, batch), dim3(256), 0, st, p, k, tol, Rf, strideR, ws);
  return hipGetLastError();
}

}  // namespace cabs
