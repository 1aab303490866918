// Follow-up sampling (Algorithm 2, step 3): weighted k-means on the rows of an
// embedding P (rows x dim) with weights w, then snapping of every centre to an
// in-sample row (Section 3.2).
//
// Per Lloyd iteration:
//   assign     fused MFMA distance GEMM  |Z_j|^2 - 2 P_l . Z_j  with a running
//              (best, index, second) per row in registers and a 16-lane
//              butterfly merge; ties go to the lowest centre index.  Writes
//              the label, |P_l - Z_s(l)|^2 and the best/second gap.
//   label_hist per 512-row block: rank of every row among the rows of the same
//              label before it (wave ballots + per-wave counts in LDS) and the
//              block's label histogram.
//   scan       one workgroup: exclusive scan of the (label, block) histogram ->
//              stable positions of every row in label order, label ranges,
//              cluster sizes and a table of fixed-size row chunks per label.
//   scatter    rows into label order (ascending row index within a label).
//   centroid   per chunk: FP64 sums of w_l P_l in row order; per label: the
//              chunk sums in chunk order, divided by the weight (empty or
//              zero-weight clusters keep their centre).
// Nothing uses floating-point atomics, so every run is bitwise reproducible.
//
// Snapping: per 4096-row block, the 16 nearest rows of every centre (MFMA
// distance tiles staged in LDS); a per-centre merge of the block lists; then
// one workgroup visits the centres in order and gives each the nearest row
// not yet taken, falling back to a full scan of all rows when all 16
// candidates are taken.
#include "common.hpp"
#include "gemm_core.hpp"
#include "kernels.hpp"
#include "timing.hpp"

namespace cabs {

constexpr int KM_NT = 8;          // centres per wave pass = 128
constexpr int KM_MAXK = 1024;
constexpr int HIST_SB = 512;      // rows per histogram block (8 waves)
constexpr int CENT_CH = 256;      // rows per centroid chunk
constexpr int SNAP_T = 16;        // candidates kept per centre and block
constexpr int SNAP_CC = 64;       // centres per LDS chunk in the top-T pass
constexpr int SNAP_NT = SNAP_CC / 16;
constexpr int SNAP_SUB = 64;      // rows per distance sub-tile

static inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
template <typename TC>
__global__ __launch_bounds__(256) void rownorm2_kernel(int64_t rows, int dim, const TC* __restrict__ P,
                                                       double* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= rows) return;
  double s = 0.0;
  for (int c = lane; c < dim; c += 64) { const double v = to_f64(P[row * dim + c]); s += v * v; }
  s = wave_sum(s);
  if (lane == 0) out[row] = s;
}

// Zc = round(Z) in the compute precision; znorm_j = |Zc_j|^2 (FP64, fixed order).
template <typename TC>
__global__ __launch_bounds__(256) void zprep_kernel(int k, int dim, const double* __restrict__ Z, TC* __restrict__ Zc,
                                                    double* __restrict__ znorm) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int c = threadIdx.x; c < dim; c += 256) {
    const TC v = from_f64<TC>(Z[(int64_t)j * dim + c]);
    Zc[(int64_t)j * dim + c] = v;
    const double dv = to_f64(v);
    s += dv * dv;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) znorm[j] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void copy_f64_kernel(int64_t n, const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) dst[e] = src[e];
}

__global__ __launch_bounds__(256) void fill_u32_kernel(int64_t n, uint32_t* __restrict__ dst, uint32_t v) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) dst[e] = v;
}

// ---------------------------------------------------------------------------
// assign: fused distance GEMM + argmin
// ---------------------------------------------------------------------------
template <typename AT>
__device__ __forceinline__ void merge_best(AT& b, int& bi, AT& s, AT ob, int obi, AT os) {
  const bool take = ob < b || (ob == b && obi < bi);
  const AT loser = take ? b : ob;
  if (take) { b = ob; bi = obi; }
  AT ns = s < os ? s : os;
  s = ns < loser ? ns : loser;
}

template <typename TC>
__global__ __launch_bounds__(256) void assign_kernel(int64_t rows, int dim, int k, const TC* __restrict__ P,
                                                     const TC* __restrict__ Zc, const double* __restrict__ znorm,
                                                     const double* __restrict__ pnorm, int32_t* __restrict__ labels,
                                                     double* __restrict__ dmin, double* __restrict__ gap) {
  typedef typename Mfma<TC>::acc AccV;
  typedef typename Acc<TC>::type AT;
  typedef typename NormT<TC>::type NrmT;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (row0 >= rows) return;
  AT best[4], second[4];
  int bidx[4];
  const AT INF = (AT)__builtin_huge_val();
#pragma unroll
  for (int i = 0; i < 4; ++i) { best[i] = INF; second[i] = INF; bidx[i] = 0x7fffffff; }
  for (int col0 = 0; col0 < k; col0 += KM_NT * 16) {
    AccV acc[KM_NT];
    NrmT xs, ys[KM_NT];
    gemm_tile<TC, TC, KM_NT, false>(P, dim, rows, row0, Zc, dim, nullptr, k, col0, nullptr, dim, acc, xs, ys);
#pragma unroll
    for (int t = 0; t < KM_NT; ++t) {
      const int col = col0 + t * 16 + c16;
      if (col < k) {
        const AT zn = (AT)znorm[col];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const AT d = zn - (AT)2 * (AT)acc[t][i];
          if (d < best[i]) { second[i] = best[i]; best[i] = d; bidx[i] = col; }
          else if (d < second[i]) second[i] = d;
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const AT ob = __shfl_xor(best[i], off, 64);
      const int obi = __shfl_xor(bidx[i], off, 64);
      const AT os = __shfl_xor(second[i], off, 64);
      merge_best(best[i], bidx[i], second[i], ob, obi, os);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = row0 + out_row<TC>(g, i);
    if (c16 == i && row < rows) {
      labels[row] = bidx[i] < k ? bidx[i] : 0;  // all-NaN rows fall back to centre 0
      const double dd = pnorm[row] + (double)best[i];
      dmin[row] = dd > 0.0 ? dd : 0.0;
      if (gap) gap[row] = (double)second[i] - (double)best[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Stable counting sort of rows by label
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(HIST_SB) void label_hist_kernel(int64_t rows, int k, const int32_t* __restrict__ labels,
                                                             int32_t* __restrict__ hist, int32_t* __restrict__ rank_blk,
                                                             int64_t nsb) {
  __shared__ int32_t wh[HIST_SB / 64][KM_MAXK];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = HIST_SB / 64;
  for (int e = threadIdx.x; e < nw * k; e += HIST_SB) wh[e / k][e % k] = 0;
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * HIST_SB + threadIdx.x;
  const bool valid = row < rows;
  const int lab = valid ? labels[row] : -1;
  // rank among equal labels of lower lanes of this wave
  uint64_t remaining = __ballot(valid);
  int rin = 0;
  while (remaining) {
    const int leader = __builtin_ctzll(remaining);
    const int llab = __shfl(lab, leader, 64);
    const uint64_t same = __ballot(lab == llab) & remaining;
    if (lab == llab) rin = __builtin_popcountll(same & ((1ull << lane) - 1ull));
    if (lane == leader) wh[wave][llab] = __builtin_popcountll(same);
    remaining &= ~same;
  }
  __syncthreads();
  // per label: exclusive prefix over waves (in place), block total to hist
  for (int j = threadIdx.x; j < k; j += HIST_SB) {
    int run = 0;
    for (int w = 0; w < nw; ++w) { const int c = wh[w][j]; wh[w][j] = run; run += c; }
    hist[(int64_t)j * nsb + blockIdx.x] = run;
  }
  __syncthreads();
  if (valid) rank_blk[row] = wh[wave][lab] + rin;
}

// One workgroup.  offs = exclusive scan of hist (label-major); label ranges;
// chunk table; cluster-size maximum.
__global__ __launch_bounds__(1024) void scan_kernel(int k, int64_t nsb, const int32_t* __restrict__ hist,
                                                    int32_t* __restrict__ offs, int32_t* __restrict__ lstart,
                                                    int32_t* __restrict__ chunk_lab, int32_t* __restrict__ chunk_beg,
                                                    int32_t* __restrict__ chunk_end, int32_t* __restrict__ lchunk,
                                                    int32_t* __restrict__ nchunks_out, double* __restrict__ tmax_out) {
  __shared__ int64_t part[1024];
  __shared__ int32_t cnt[KM_MAXK + 1];
  const int tid = threadIdx.x;
  const int64_t L = (int64_t)k * nsb;
  const int64_t per = ceil_div(L, 1024);
  const int64_t b0 = tid * per, b1 = b0 + per < L ? b0 + per : L;
  int64_t s = 0;
  for (int64_t e = b0; e < b1; ++e) s += hist[e];
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    int64_t run = 0;
    for (int t = 0; t < 1024; ++t) { const int64_t c = part[t]; part[t] = run; run += c; }
  }
  __syncthreads();
  int64_t run = part[tid];
  for (int64_t e = b0; e < b1; ++e) { const int32_t c = hist[e]; offs[e] = (int32_t)run; run += c; }
  __syncthreads();
  // label starts and counts
  for (int j = tid; j < k; j += 1024) {
    const int32_t st = offs[(int64_t)j * nsb];
    lstart[j] = st;
    int64_t c = 0;
    for (int64_t b = 0; b < nsb; ++b) c += hist[(int64_t)j * nsb + b];
    cnt[j] = (int32_t)c;
  }
  __syncthreads();
  if (tid == 0) {
    int32_t mx = 0, run_ch = 0;
    for (int j = 0; j < k; ++j) {
      mx = cnt[j] > mx ? cnt[j] : mx;
      const int32_t nch = (cnt[j] + CENT_CH - 1) / CENT_CH;
      lchunk[j] = run_ch;
      run_ch += nch;
    }
    lchunk[k] = run_ch;
    *nchunks_out = run_ch;
    if (tmax_out) *tmax_out = (double)mx;
  }
  __syncthreads();
  for (int j = tid; j < k; j += 1024) {
    const int32_t st = lstart[j], en = st + cnt[j];
    int32_t c = lchunk[j];
    for (int32_t b = st; b < en; b += CENT_CH, ++c) {
      chunk_lab[c] = j;
      chunk_beg[c] = b;
      chunk_end[c] = b + CENT_CH < en ? b + CENT_CH : en;
    }
  }
}

__global__ __launch_bounds__(256) void scatter_kernel(int64_t rows, int64_t nsb, const int32_t* __restrict__ labels,
                                                      const int32_t* __restrict__ rank_blk,
                                                      const int32_t* __restrict__ offs, int32_t* __restrict__ sorted) {
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= rows) return;
  const int64_t sb = row / HIST_SB;
  sorted[offs[(int64_t)labels[row] * nsb + sb] + rank_blk[row]] = (int32_t)row;
}

template <typename TC>
__global__ __launch_bounds__(256) void centroid_partial_kernel(int dim, const TC* __restrict__ P,
                                                               const double* __restrict__ w,
                                                               const int32_t* __restrict__ sorted,
                                                               const int32_t* __restrict__ chunk_beg,
                                                               const int32_t* __restrict__ chunk_end,
                                                               const int32_t* __restrict__ nchunks,
                                                               double* __restrict__ part, double* __restrict__ partw) {
  const int c = blockIdx.x;
  if (c >= *nchunks) return;
  const int32_t b = chunk_beg[c], e = chunk_end[c];
  for (int col = threadIdx.x; col < dim; col += 256) {
    double acc = 0.0;
    for (int32_t pos = b; pos < e; ++pos) {
      const int64_t row = sorted[pos];
      acc += w[row] * to_f64(P[row * dim + col]);
    }
    part[(int64_t)c * dim + col] = acc;
  }
  if (threadIdx.x == 0) {
    double ws = 0.0;
    for (int32_t pos = b; pos < e; ++pos) ws += w[sorted[pos]];
    partw[c] = ws;
  }
}

template <typename TC>
__global__ __launch_bounds__(256) void centroid_final_kernel(int k, int dim, const int32_t* __restrict__ lchunk,
                                                             const double* __restrict__ part,
                                                             const double* __restrict__ partw, double* __restrict__ Z,
                                                             TC* __restrict__ Zc, double* __restrict__ znorm) {
  __shared__ double red[4];
  const int j = blockIdx.x;
  const int c0 = lchunk[j], c1 = lchunk[j + 1];
  double W = 0.0;
  for (int c = c0; c < c1; ++c) W += partw[c];
  double s2 = 0.0;
  for (int col = threadIdx.x; col < dim; col += 256) {
    double z = Z[(int64_t)j * dim + col];
    if (W > 0.0) {
      double s = 0.0;
      for (int c = c0; c < c1; ++c) s += part[(int64_t)c * dim + col];
      z = s / W;
      Z[(int64_t)j * dim + col] = z;
    }
    const TC zc = from_f64<TC>(z);
    Zc[(int64_t)j * dim + col] = zc;
    const double dz = to_f64(zc);
    s2 += dz * dz;
  }
  s2 = wave_sum(s2);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s2;
  __syncthreads();
  if (threadIdx.x == 0) znorm[j] = ((red[0] + red[1]) + red[2]) + red[3];
}

// ---------------------------------------------------------------------------
// Fixed-order reductions: sum_l w_l dmin_l, min_l gap_l
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void wsum_partial_kernel(int64_t rows, const double* __restrict__ w,
                                                           const double* __restrict__ d, const double* __restrict__ gap,
                                                           double* __restrict__ part_s, double* __restrict__ part_g) {
  __shared__ double rs[4], rg[4];
  const int64_t per = ceil_div(rows, (int64_t)gridDim.x);
  const int64_t b0 = blockIdx.x * per, b1 = b0 + per < rows ? b0 + per : rows;
  double s = 0.0, gm = __builtin_huge_val();
  for (int64_t r = b0 + threadIdx.x; r < b1; r += 256) {
    s += w[r] * d[r];
    if (gap) gm = gap[r] < gm ? gap[r] : gm;
  }
  s = wave_sum(s);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) { const double o = __shfl_xor(gm, off, 64); gm = o < gm ? o : gm; }
  if ((threadIdx.x & 63) == 0) { rs[threadIdx.x >> 6] = s; rg[threadIdx.x >> 6] = gm; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part_s[blockIdx.x] = ((rs[0] + rs[1]) + rs[2]) + rs[3];
    double m = rg[0];
    for (int q = 1; q < 4; ++q) m = rg[q] < m ? rg[q] : m;
    part_g[blockIdx.x] = m;
  }
}

__global__ void wsum_final_kernel(int nb, const double* __restrict__ part_s, const double* __restrict__ part_g,
                                  double* __restrict__ out_s, double* __restrict__ out_g) {
  if (threadIdx.x != 0) return;
  double s = 0.0, g = __builtin_huge_val();
  for (int b = 0; b < nb; ++b) { s += part_s[b]; g = part_g[b] < g ? part_g[b] : g; }
  if (out_s) *out_s = s;
  if (out_g) *out_g = g;
}

// ---------------------------------------------------------------------------
// Snapping
// ---------------------------------------------------------------------------
template <typename AT>
__device__ __forceinline__ void topt_insert(AT (&d)[SNAP_T], int (&r)[SNAP_T], AT nd, int nr) {
  // rows arrive in increasing order, so a new equal distance goes after the old ones
  if (!(nd < d[SNAP_T - 1])) return;
#pragma unroll
  for (int q = SNAP_T - 1; q > 0; --q) {
    const bool shift = nd < d[q - 1];
    const bool place = !shift && nd < d[q];
    if (shift) { d[q] = d[q - 1]; r[q] = r[q - 1]; }
    else if (place) { d[q] = nd; r[q] = nr; }
  }
  if (nd < d[0]) { d[0] = nd; r[0] = nr; }
}

template <typename TC>
__global__ __launch_bounds__(256) void snap_topt_kernel(int64_t rows, int dim, int k, int64_t rows_per_block,
                                                        const TC* __restrict__ P, const TC* __restrict__ Zc,
                                                        const double* __restrict__ znorm,
                                                        const double* __restrict__ pnorm, double* __restrict__ cand_d,
                                                        int32_t* __restrict__ cand_r) {
  typedef typename Mfma<TC>::acc AccV;
  typedef typename NormT<TC>::type NrmT;
  __shared__ double dist[SNAP_SUB][SNAP_CC + 1];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t rbeg = (int64_t)blockIdx.x * rows_per_block;
  const int64_t rend = rbeg + rows_per_block < rows ? rbeg + rows_per_block : rows;
  const int nblk = gridDim.x;
  for (int cc = 0; cc < k; cc += SNAP_CC) {
    double td[SNAP_T];
    int tr[SNAP_T];
#pragma unroll
    for (int q = 0; q < SNAP_T; ++q) { td[q] = __builtin_huge_val(); tr[q] = 0x7fffffff; }
    const int myc = cc + threadIdx.x;  // centre tracked by this thread (threads < SNAP_CC)
    for (int64_t s0 = rbeg; s0 < rend; s0 += SNAP_SUB) {
      const int64_t row0 = s0 + wave * 16;
      AccV acc[SNAP_NT];
      NrmT xs, ys[SNAP_NT];
      if (row0 < rend) {
        gemm_tile<TC, TC, SNAP_NT, false>(P, dim, rend, row0, Zc, dim, nullptr, k, cc, nullptr, dim, acc, xs, ys);
      }
#pragma unroll
      for (int t = 0; t < SNAP_NT; ++t) {
        const int cl = t * 16 + c16;
        const int col = cc + cl;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int rl = wave * 16 + out_row<TC>(g, i);
          const int64_t row = s0 + rl;
          double d = __builtin_huge_val();
          if (row0 < rend && row < rend && col < k) {
            d = pnorm[row] + znorm[col] - 2.0 * (double)acc[t][i];
            d = d > 0.0 ? d : 0.0;
          }
          dist[rl][cl] = d;
        }
      }
      __syncthreads();
      if (threadIdx.x < SNAP_CC && myc < k) {
        for (int rl = 0; rl < SNAP_SUB; ++rl) {
          const int64_t row = s0 + rl;
          if (row >= rend) break;
          topt_insert<double>(td, tr, dist[rl][threadIdx.x], (int)row);
        }
      }
      __syncthreads();
    }
    if (threadIdx.x < SNAP_CC && myc < k) {
      const int64_t base = ((int64_t)myc * nblk + blockIdx.x) * SNAP_T;
#pragma unroll
      for (int q = 0; q < SNAP_T; ++q) { cand_d[base + q] = td[q]; cand_r[base + q] = tr[q]; }
    }
  }
}

// Per centre: sort the nblk * SNAP_T candidates by (distance, row); keep SNAP_T.
__global__ __launch_bounds__(256) void snap_merge_kernel(int nblk, const double* __restrict__ cand_d,
                                                         const int32_t* __restrict__ cand_r, double* __restrict__ top_d,
                                                         int32_t* __restrict__ top_r) {
  __shared__ double sd[4096];
  __shared__ int32_t sr[4096];
  const int j = blockIdx.x;
  const int n = nblk * SNAP_T;
  int P2 = 1;
  while (P2 < n) P2 <<= 1;
  for (int e = threadIdx.x; e < P2; e += 256) {
    if (e < n) { sd[e] = cand_d[(int64_t)j * n + e]; sr[e] = cand_r[(int64_t)j * n + e]; }
    else { sd[e] = __builtin_huge_val(); sr[e] = 0x7fffffff; }
  }
  __syncthreads();
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P2; t += 256) {
        const int p = t ^ stride;
        if (p > t) {
          const bool up = (t & size) == 0;
          const double a = sd[t], b = sd[p];
          const int ra = sr[t], rb = sr[p];
          const bool gt = a > b || (a == b && ra > rb);
          if (gt == up) { sd[t] = b; sd[p] = a; sr[t] = rb; sr[p] = ra; }
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x < SNAP_T) {
    top_d[(int64_t)j * SNAP_T + threadIdx.x] = sd[threadIdx.x];
    top_r[(int64_t)j * SNAP_T + threadIdx.x] = sr[threadIdx.x];
  }
}

// Distances within tie_rtol * (|Z_j| + sqrt(d_min))^2 of the nearest untaken row
// count as ties and go to the lowest row index (the centre of a two-row cluster
// is equidistant from both rows).  Wave 0 walks the centres in order using
// candidate lists staged in LDS; the whole block joins only when a centre's
// list cannot decide (every candidate taken, or the tie window reaches past
// the list), and then scans every untaken row.
constexpr int RES_CHUNK = 256;

template <typename TC>
__global__ __launch_bounds__(1024) void snap_resolve_kernel(int64_t rows, int dim, int k, const TC* __restrict__ P,
                                                            const TC* __restrict__ Zc, const double* __restrict__ znorm,
                                                            const double* __restrict__ pnorm,
                                                            const double* __restrict__ top_d,
                                                            const int32_t* __restrict__ top_r, double tie_rtol,
                                                            uint32_t* __restrict__ taken_bits,
                                                            int64_t* __restrict__ out) {
  __shared__ int64_t chosen[KM_MAXK];
  __shared__ double ld[RES_CHUNK * SNAP_T];
  __shared__ int32_t lr[RES_CHUNK * SNAP_T];
  __shared__ double lz[RES_CHUNK];
  __shared__ double bd[16];
  __shared__ int64_t br[16];
  __shared__ int sh_next, sh_marked;
  __shared__ double sh_dmin;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const double INF = __builtin_huge_val();
  int j = 0;
  int chunk0 = -RES_CHUNK;
  int marked = 0;  // chosen[0 .. marked) are already in taken_bits
  while (j < k) {
    if (j >= chunk0 + RES_CHUNK) {  // stage the lists of centres [j, j + RES_CHUNK)
      chunk0 = j;
      const int n = (k - j < RES_CHUNK ? k - j : RES_CHUNK);
      for (int e = tid; e < n * SNAP_T; e += 1024) {
        ld[e] = top_d[(int64_t)j * SNAP_T + e];
        lr[e] = top_r[(int64_t)j * SNAP_T + e];
      }
      for (int e = tid; e < n; e += 1024) lz[e] = sqrt(znorm[j + e]);
      __syncthreads();
    }
    if (wave == 0) {
      int jj = j;
      const int lim = (chunk0 + RES_CHUNK < k ? chunk0 + RES_CHUNK : k);
      for (; jj < lim; ++jj) {
        const double zn = lz[jj - chunk0];
        int64_t found = -1;
        double dmin = INF, tol = 0.0, last_d = INF;
        int q = 0;
        for (; q < SNAP_T; ++q) {
          const int32_t r = lr[(jj - chunk0) * SNAP_T + q];
          const double d = ld[(jj - chunk0) * SNAP_T + q];
          if (r == 0x7fffffff) break;
          if (found >= 0 && d > dmin + tol) break;
          last_d = d;
          bool hit = false;
          for (int s = lane; s < jj; s += 64) hit |= chosen[s] == (int64_t)r;
          if (__ballot(hit) != 0) continue;
          if (found < 0) {
            dmin = d;
            const double rr = zn + sqrt(d);
            tol = tie_rtol * rr * rr;
            found = r;
          } else if (r < found) {
            found = r;
          }
        }
        const bool undecided = found < 0 || (q == SNAP_T && last_d <= dmin + tol);
        if (undecided) break;
        if (lane == 0) chosen[jj] = found;
        __builtin_amdgcn_wave_barrier();
      }
      if (lane == 0) sh_next = jj;
    }
    __syncthreads();
    j = sh_next;
    if (j >= k) break;
    if (j >= chunk0 + RES_CHUNK) continue;  // next chunk
    // Centre j needs a full scan: mark the rows chosen so far, then nearest
    // distance over the untaken rows, then the lowest row in its tie window.
    for (int s = marked + tid; s < j; s += 1024) atomicOr(&taken_bits[chosen[s] >> 5], 1u << (chosen[s] & 31));
    marked = j;
    __syncthreads();
    const double zn = lz[j - chunk0];
    double best = INF;
    for (int64_t row = tid; row < rows; row += 1024) {
      if (taken_bits[row >> 5] & (1u << (row & 31))) continue;
      double dot = 0.0;
      for (int c = 0; c < dim; ++c) dot += to_f64(P[row * dim + c]) * to_f64(Zc[(int64_t)j * dim + c]);
      double d = pnorm[row] + znorm[j] - 2.0 * dot;
      d = d > 0.0 ? d : 0.0;
      if (d != d) d = INF;
      best = d < best ? d : best;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) { const double ob = __shfl_xor(best, off, 64); best = ob < best ? ob : best; }
    if (lane == 0) bd[wave] = best;
    __syncthreads();
    if (tid == 0) {
      double b = bd[0];
      for (int w = 1; w < 16; ++w) b = bd[w] < b ? bd[w] : b;
      sh_dmin = b;
    }
    __syncthreads();
    const double dmin = sh_dmin;
    const double rr = zn + sqrt(dmin < INF ? dmin : 0.0);
    const double lim = dmin < INF ? dmin + tie_rtol * rr * rr : INF;
    int64_t brow = INT64_MAX;
    for (int64_t row = tid; row < rows && brow == INT64_MAX; row += 1024) {
      if (taken_bits[row >> 5] & (1u << (row & 31))) continue;
      double dot = 0.0;
      for (int c = 0; c < dim; ++c) dot += to_f64(P[row * dim + c]) * to_f64(Zc[(int64_t)j * dim + c]);
      double d = pnorm[row] + znorm[j] - 2.0 * dot;
      d = d > 0.0 ? d : 0.0;
      if (d != d) d = INF;
      if (d <= lim) brow = row;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const int64_t orow = __shfl_xor(brow, off, 64);
      brow = orow < brow ? orow : brow;
    }
    if (lane == 0) br[wave] = brow;
    __syncthreads();
    if (tid == 0) {
      int64_t r = br[0];
      for (int w = 1; w < 16; ++w) r = br[w] < r ? br[w] : r;
      if (r == INT64_MAX) {  // every untaken distance is NaN: lowest untaken row
        for (int64_t row = 0; row < rows; ++row)
          if (!(taken_bits[row >> 5] & (1u << (row & 31)))) { r = row; break; }
      }
      chosen[j] = r;
      sh_marked = 0;
    }
    __syncthreads();
    j += 1;
  }
  __syncthreads();
  // ascending order (reuses the candidate area as sort keys)
  int64_t* keys = (int64_t*)ld;
  int P2 = 1;
  while (P2 < k) P2 <<= 1;
  for (int e = tid; e < P2; e += 1024) keys[e] = e < k ? chosen[e] : INT64_MAX;
  __syncthreads();
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = tid; t < P2; t += 1024) {
        const int p = t ^ stride;
        if (p > t) {
          const bool up = (t & size) == 0;
          const int64_t a = keys[t], b = keys[p];
          if ((a > b) == up) { keys[t] = b; keys[p] = a; }
        }
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < k; e += 1024) out[e] = keys[e];
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
struct KmWs {
  void* Zc; double* znorm; double* pnorm; int32_t* labels; double* dmin; double* gap;
  int32_t* hist; int32_t* offs; int32_t* rank_blk; int32_t* sorted; int32_t* lstart;
  int32_t* chunk_lab; int32_t* chunk_beg; int32_t* chunk_end; int32_t* lchunk; int32_t* nchunks;
  double* part; double* partw; double* red_s; double* red_g; double* obj_tmp; double* tmax_tmp; double* gap_tmp;
  double* cand_d; int32_t* cand_r; double* top_d; int32_t* top_r; uint32_t* bits;
  size_t total;
};

static inline int snap_nblk(int64_t rows) {
  int64_t nb = ceil_div(rows, 512);
  if (nb > 256) nb = 256;
  return (int)(nb < 1 ? 1 : nb);
}
constexpr int RED_NB = 256;

static KmWs km_layout(void* base, int64_t rows, int dim, int k, int compute) {
  KmWs w{};
  char* p = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) { void* q = p ? p + off : nullptr; off += al256(bytes); return q; };
  const int64_t nsb = ceil_div(rows, HIST_SB);
  const int64_t maxch = ceil_div(rows, CENT_CH) + k;
  const int nblk = snap_nblk(rows);
  w.Zc = take((size_t)k * dim * prec_bytes(compute));
  w.znorm = (double*)take(k * 8);
  w.pnorm = (double*)take(rows * 8);
  w.labels = (int32_t*)take(rows * 4);
  w.dmin = (double*)take(rows * 8);
  w.gap = (double*)take(rows * 8);
  w.hist = (int32_t*)take((size_t)k * nsb * 4);
  w.offs = (int32_t*)take((size_t)k * nsb * 4);
  w.rank_blk = (int32_t*)take(rows * 4);
  w.sorted = (int32_t*)take(rows * 4);
  w.lstart = (int32_t*)take((k + 1) * 4);
  w.chunk_lab = (int32_t*)take(maxch * 4);
  w.chunk_beg = (int32_t*)take(maxch * 4);
  w.chunk_end = (int32_t*)take(maxch * 4);
  w.lchunk = (int32_t*)take((k + 1) * 4);
  w.nchunks = (int32_t*)take(4);
  w.part = (double*)take((size_t)maxch * dim * 8);
  w.partw = (double*)take(maxch * 8);
  w.red_s = (double*)take(RED_NB * 8);
  w.red_g = (double*)take(RED_NB * 8);
  w.obj_tmp = (double*)take(2 * 8);
  w.tmax_tmp = (double*)take(8);
  w.gap_tmp = (double*)take(8);
  w.cand_d = (double*)take((size_t)k * nblk * SNAP_T * 8);
  w.cand_r = (int32_t*)take((size_t)k * nblk * SNAP_T * 4);
  w.top_d = (double*)take((size_t)k * SNAP_T * 8);
  w.top_r = (int32_t*)take((size_t)k * SNAP_T * 4);
  w.bits = (uint32_t*)take((size_t)ceil_div(rows, 32) * 4);
  w.total = off;
  return w;
}

size_t kmeans_ws_bytes(int64_t rows, int dim, int k, int compute) {
  return km_layout(nullptr, rows, dim, k, compute).total + 256;
}

template <typename TC>
static hipError_t kmeans_t(int compute, int64_t rows, int dim, int k, const void* Pv, const double* w, const double* Z0,
                           int iters, const KMeansOut& out, void* ws, hipStream_t st) {
  const TC* P = (const TC*)Pv;
  KmWs W = km_layout(ws, rows, dim, k, compute);
  TC* Zc = (TC*)W.Zc;
  const int64_t nsb = ceil_div(rows, HIST_SB);
  const unsigned gA = (unsigned)ceil_div(rows, 64);
  const unsigned gR = (unsigned)ceil_div(rows, 4);
  const int64_t maxch = ceil_div(rows, CENT_CH) + k;
  int32_t* labels = out.labels ? out.labels : W.labels;
  const int red_nb = (int)(rows < RED_NB * 256 ? ceil_div(rows, 256) : RED_NB);

  if (Z0 != out.Z)
    hipLaunchKernelGGL(copy_f64_kernel, dim3((unsigned)ceil_div((int64_t)k * dim, 256)), dim3(256), 0, st,
                       (int64_t)k * dim, Z0, out.Z);
  hipLaunchKernelGGL(zprep_kernel<TC>, dim3(k), dim3(256), 0, st, k, dim, out.Z, Zc, W.znorm);
  hipLaunchKernelGGL(rownorm2_kernel<TC>, dim3(gR), dim3(256), 0, st, rows, dim, P, W.pnorm);

  for (int it = 0; it <= iters; ++it) {
    const bool last = it == iters;
    {
      TimerScope ts(T_ASSIGN, st);
      hipLaunchKernelGGL(assign_kernel<TC>, dim3(gA), dim3(256), 0, st, rows, dim, k, P, (const TC*)Zc, W.znorm,
                         W.pnorm, labels, W.dmin, last ? W.gap : nullptr);
    }
    if (it == 0 || last) {
      hipLaunchKernelGGL(wsum_partial_kernel, dim3(red_nb), dim3(256), 0, st, rows, w, W.dmin,
                         last ? W.gap : nullptr, W.red_s, W.red_g);
      double* dst = out.obj2 ? out.obj2 + (last ? 1 : 0) : W.obj_tmp + (last ? 1 : 0);
      hipLaunchKernelGGL(wsum_final_kernel, dim3(1), dim3(64), 0, st, red_nb, W.red_s, W.red_g, dst,
                         last ? (out.gap ? out.gap : W.gap_tmp) : nullptr);
      if (it == 0 && last && out.obj2)  // no iterations: both objectives are the initial one
        hipLaunchKernelGGL(copy_f64_kernel, dim3(1), dim3(256), 0, st, (int64_t)1, out.obj2 + 1, out.obj2);
    }
    hipLaunchKernelGGL(label_hist_kernel, dim3((unsigned)nsb), dim3(HIST_SB), 0, st, rows, k, labels, W.hist,
                       W.rank_blk, nsb);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, k, nsb, W.hist, W.offs, W.lstart, W.chunk_lab,
                       W.chunk_beg, W.chunk_end, W.lchunk, W.nchunks, last ? (out.tmax ? out.tmax : W.tmax_tmp) : nullptr);
    if (last) break;
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)ceil_div(rows, 256)), dim3(256), 0, st, rows, nsb, labels,
                       W.rank_blk, W.offs, W.sorted);
    {
      TimerScope ts(T_CENTROID, st);
      hipLaunchKernelGGL(centroid_partial_kernel<TC>, dim3((unsigned)maxch), dim3(256), 0, st, dim, P, w, W.sorted,
                         W.chunk_beg, W.chunk_end, W.nchunks, W.part, W.partw);
    }
    hipLaunchKernelGGL(centroid_final_kernel<TC>, dim3(k), dim3(256), 0, st, k, dim, W.lchunk, W.part, W.partw, out.Z,
                       Zc, W.znorm);
  }
  if (out.snap) {
    const int nblk = snap_nblk(rows);
    const int64_t rpb = ceil_div(ceil_div(rows, nblk), SNAP_SUB) * SNAP_SUB;
    const int nblk_eff = (int)ceil_div(rows, rpb);
    TimerScope ts(T_SNAP, st);
    hipLaunchKernelGGL(snap_topt_kernel<TC>, dim3(nblk_eff), dim3(256), 0, st, rows, dim, k, rpb, P, (const TC*)Zc,
                       W.znorm, W.pnorm, W.cand_d, W.cand_r);
    hipLaunchKernelGGL(snap_merge_kernel, dim3(k), dim3(256), 0, st, nblk_eff, W.cand_d, W.cand_r, W.top_d, W.top_r);
    const int64_t nbits = ceil_div(rows, 32);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)ceil_div(nbits, 256)), dim3(256), 0, st, nbits, W.bits, 0u);
    // FP64: a relative tie window makes the choice independent of rounding order
    // (and equal to the FP64 reference); other precisions compare exactly.
    const double tie_rtol = sizeof(TC) == 8 ? 1e-11 : 0.0;
    hipLaunchKernelGGL(snap_resolve_kernel<TC>, dim3(1), dim3(1024), 0, st, rows, dim, k, P, (const TC*)Zc, W.znorm,
                       W.pnorm, W.top_d, W.top_r, tie_rtol, W.bits, out.snap);
  }
  return hipGetLastError();
}

hipError_t launch_kmeans(int64_t rows, int dim, int k, int compute, const void* P, const double* w, const double* Z0,
                         int iters, const KMeansOut& out, void* ws, hipStream_t st) {
  if (rows <= 0 || dim <= 0 || k <= 0 || k > KM_MAXK || k > rows || iters < 0 || out.Z == nullptr)
    return hipErrorInvalidValue;
  switch (compute) {
    case P_F64: return kmeans_t<double>(compute, rows, dim, k, P, w, Z0, iters, out, ws, st);
    case P_F32: return kmeans_t<float>(compute, rows, dim, k, P, w, Z0, iters, out, ws, st);
    case P_BF16: return kmeans_t<bf16>(compute, rows, dim, k, P, w, Z0, iters, out, ws, st);
    case P_F16: return kmeans_t<f16>(compute, rows, dim, k, P, w, Z0, iters, out, ws, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cabs
