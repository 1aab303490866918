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
// Snapping: per block of about 128 rows, the 16 nearest rows of every centre (MFMA
// distance tiles staged in LDS); a per-centre merge of the block lists; then
// one workgroup visits the centres in order and gives each the nearest row
// not yet taken, falling back to the per-block lists (and exact rescans of
// the blocks whose lists may be incomplete) when the merged 16 cannot decide.
#include "common.hpp"
#include "gemm_core.hpp"
#include "kernels.hpp"
#include "timing.hpp"

#include <algorithm>
#include <atomic>
#include <cstdlib>

namespace cabs {

constexpr int KM_NT = 8;          // centres per wave pass = 128
constexpr int KM_MAXK = 1024;
constexpr int HIST_SB = 512;      // rows per histogram block (8 waves)
constexpr int CENT_CH = 256;      // rows per centroid chunk
constexpr int SNAP_T = 16;        // candidates kept per centre and block
constexpr int SNAP_CC = 64;       // centres per LDS chunk in the top-T pass
constexpr int SNAP_NT = SNAP_CC / 16;
constexpr int SNAP_SUB = 64;      // rows per distance sub-tile
constexpr int SNAP_ROWS = 128;    // rows per block of the top-T pass (a multiple of SNAP_SUB)
constexpr int SNAP_MAXBLK = 2048; // row blocks at most
constexpr int64_t SNAP_MAXCAND = (int64_t)1 << 19;  // k * blocks at most
constexpr int AF_MAXG = 4;        // centre groups of the fast assignment at most

static inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Compute units of the current device (looked up once per device).
static int device_cus() {
  static std::atomic<int> cus[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int v = cus[dev].load(std::memory_order_relaxed);
  if (v <= 0) {
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    cus[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}

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

// Fast assignment for FP32 / BF16 / FP16, dim <= 512 and rows that are whole
// 16-byte runs (dim a multiple of 16 / sizeof(TC), P and Zc 16-byte aligned).
// A workgroup has 4 waves; each wave keeps RT row tiles of 16 rows as 16-byte
// MFMA fragments in registers for the whole kernel and streams its centre
// group through LDS in chunks of CT x 16 centres, stored in fragment order so
// that every B read is one contiguous ds_read_b128 per wave (no bank
// conflicts).  Each B fragment read from LDS feeds RT MFMAs: 16-bit types use
// RT = 2, since one 16x16x32 MFMA per 1 KB LDS read would leave the CU's LDS
// port, not the matrix cores, as the bound; FP32 MFMAs are 8x slower per byte
// of B, so RT = 1 suffices there.
//
// Chunks are double-buffered in two LDS arrays and filled by direct
// buffer-to-LDS loads (buffer_load_dwordx4 ... lds: lane l's 16 bytes land at
// 16 l past the wave's LDS address, so one instruction fills one 1 KB
// fragment block; offsets past the centres read zeros).  Chunk c + 1 is in flight while chunk c is multiplied, and
// no registers hold it.  The two arrays are distinct objects, so the compiler
// knows that reads of one do not wait for loads into the other; the explicit
// vmcnt(0) + barrier before a chunk is used is the only wait.  NKB (k blocks)
// is a compile-time constant, so no load, store or MFMA needs a run-time
// guard (runs past dim or k come from a zero buffer and add exact zeros).
//
// blockIdx.y selects a group of gsize consecutive centres (a multiple of
// CT x 16).  With one group the kernel writes labels, distances and gaps; with
// several (rows too few to fill the chip in whole row tiles) every group
// writes its (best, index, second) per row to pb/pi/ps and
// assign_merge_kernel combines the groups.  The summary of a set of centres
// (lexicographic minimum of (distance, index), second-smallest distance) is
// merged exactly, so any grouping gives the same labels, distances and gaps.
// Per output element the k blocks and MFMA steps come in the same order as in
// assign_kernel, so distances, labels and gaps are bit-identical to it.
#define CABS_LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))

// SD: the pass also stores every row's dot products with the centres
// (sacc[row k + centre], the MFMA sums before the epilogue) for the top-T pass
// of the snap, which then needs no second distance GEMM.
template <typename TC, int NKB, int RT, int CT, int OCC, bool SD>
__global__ __launch_bounds__(256, OCC) void assign_fast_kernel(int64_t rows, int dim, int k, int gsize,
                                                               const TC* __restrict__ P, const TC* __restrict__ Zc,
                                                               const double* __restrict__ znorm,
                                                               const double* __restrict__ pnorm,
                                                               int32_t* __restrict__ labels, double* __restrict__ dmin,
                                                               double* __restrict__ gap, float* __restrict__ pb,
                                                               int32_t* __restrict__ pi, float* __restrict__ ps,
                                                               float* __restrict__ sacc) {
  typedef typename Mfma<TC>::acc AccV;
  constexpr int VE = 16 / sizeof(TC);           // elements per 16-byte run
  constexpr int SPV = VE / Mfma<TC>::KPL;       // MFMA steps per run
  constexpr int KBW = 4 * VE;                   // k per block (4 lane groups)
  constexpr int NBLK = CT * NKB;                // 1 KB fragment blocks per chunk
  constexpr int BPW = (NBLK + 3) / 4;           // blocks issued per wave
  constexpr int CW = CT * 16;                   // centres per chunk
  __shared__ uint4 zb0[NBLK * 64];              // [CT][NKB][64] runs
  __shared__ uint4 zb1[NBLK * 64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * RT);
  const int cbeg = (int)blockIdx.y * gsize;
  const int cend = cbeg + gsize < k ? cbeg + gsize : k;
  const __amdgpu_buffer_rsrc_t zrs = lds_src_rsrc(Zc, (uint32_t)k * (uint32_t)dim * (uint32_t)sizeof(TC));
  uint4 a[RT][NKB];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb)
      a[rt][kb] = load_run_al<TC>(P, rows, dim, row0 + rt * 16 + c16, kb * KBW + g * VE, true);
  // Chunk loads: wave w fills fragment blocks w, w + 4, ...; the norms of this
  // lane's centres come with them.
  auto issue = [&](uint4* dst, int cc, double (&znf)[CT]) {
#pragma unroll
    for (int u = 0; u < BPW; ++u) {
      const int blk = wave + 4 * u;
      if (NBLK % 4 == 0 || blk < NBLK) {
        const int t = blk / NKB, kb = blk - t * NKB;
        const int c = cc + 16 * t + c16, k0 = kb * KBW + g * VE;
        const uint32_t off = (c < k && k0 < dim) ? ((uint32_t)c * dim + k0) * (uint32_t)sizeof(TC) : kBufOob;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(zrs, CABS_LDS_PTR(dst + blk * 64), 16, off, 0, 0, 0);
      }
    }
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int col = cc + t * 16 + c16;
      znf[t] = znorm[col < k ? col : k - 1];
    }
  };
  float best[RT][4], second[RT][4];
  int bidx[RT][4];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      best[rt][i] = __builtin_huge_valf();
      second[rt][i] = __builtin_huge_valf();
      bidx[rt][i] = 0x7fffffff;
    }
  auto compute = [&](const uint4* zs, int cc, const double (&znf)[CT]) {
    AccV acc[RT][CT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int t = 0; t < CT; ++t) acc[rt][t] = Mfma<TC>::zero();
    // tiles of the chunk that hold centres of the group (a compile-time count
    // per case, so a chunk with fewer than CT tiles skips the empty ones)
    // The B fragments of k block kb + D are read while block kb is multiplied
    // (D = 2 when a block has fewer than 8 MFMAs per read, so that the LDS
    // latency stays covered); scheduling barriers keep the compiler from
    // moving the reads next to their use.
    auto mm = [&](auto ntc) {
      constexpr int NT = decltype(ntc)::value;
      constexpr int D = RT * SPV * NT >= 8 ? 1 : 2;
      uint4 bq[D + 1][NT];
#pragma unroll
      for (int p = 0; p < D && p < NKB; ++p)
#pragma unroll
        for (int t = 0; t < NT; ++t) bq[p][t] = zs[(t * NKB + p) * 64 + lane];
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        if (kb + D < NKB) {
#pragma unroll
          for (int t = 0; t < NT; ++t) bq[(kb + D) % (D + 1)][t] = zs[(t * NKB + kb + D) * 64 + lane];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s2 = 0; s2 < SPV; ++s2)
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
              acc[rt][t] = Mfma<TC>::mma(Vec16<TC>::frag(a[rt][kb], s2), Vec16<TC>::frag(bq[kb % (D + 1)][t], s2),
                                         acc[rt][t]);
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    static_assert(CT == 1 || CT == 2, "the partial chunk below covers CT = 1 or 2");
    if constexpr (CT == 2) {
      if (cend - cc > 16) mm(std::integral_constant<int, 2>{});
      else mm(std::integral_constant<int, 1>{});
    } else {
      mm(std::integral_constant<int, 1>{});
    }
    // Branch-free running (best, index, second): a new strict minimum pushes the
    // old best to second; otherwise the distance may still lower the second.
    // Columns past the group are skipped through an infinite distance.
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int col = cc + t * 16 + c16;
      const bool in = col < cend;
      const float zn = (float)znf[t];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if constexpr (SD) {
            const int64_t row = row0 + rt * 16 + out_row<TC>(g, i);
            if (in && row < rows) sacc[row * k + col] = acc[rt][t][i];
          }
          const float d0 = zn - 2.0f * acc[rt][t][i];
          const float d = in ? d0 : __builtin_huge_valf();
          const bool lt = d < best[rt][i];
          const float s2 = d < second[rt][i] ? d : second[rt][i];
          second[rt][i] = lt ? best[rt][i] : s2;
          best[rt][i] = lt ? d : best[rt][i];
          bidx[rt][i] = lt ? col : bidx[rt][i];
        }
    }
  };
  double zn0[CT], zn1[CT];
  issue(zb0, cbeg, zn0);
  for (int cc = cbeg; cc < cend; cc += 2 * CW) {
    __builtin_amdgcn_s_waitcnt(0x3f70);  // vmcnt(0): this wave's loads of the chunk in zb0
    __syncthreads();                     // every wave's loads landed; zb1 is no longer read
    if (cc + CW < cend) issue(zb1, cc + CW, zn1);
    compute(zb0, cc, zn0);
    if (cc + CW >= cend) break;
    __builtin_amdgcn_s_waitcnt(0x3f70);
    __syncthreads();
    if (cc + 2 * CW < cend) issue(zb0, cc + 2 * CW, zn0);
    compute(zb1, cc + CW, zn1);
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        const float ob = __shfl_xor(best[rt][i], off, 64);
        const int obi = __shfl_xor(bidx[rt][i], off, 64);
        const float os = __shfl_xor(second[rt][i], off, 64);
        merge_best(best[rt][i], bidx[rt][i], second[rt][i], ob, obi, os);
      }
    }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = row0 + rt * 16 + out_row<TC>(g, i);
      if (c16 == i && row < rows) {
        if (pb) {
          const int64_t o = (int64_t)blockIdx.y * rows + row;
          pb[o] = best[rt][i];
          pi[o] = bidx[rt][i];
          ps[o] = second[rt][i];
        } else {
          labels[row] = bidx[rt][i] < k ? bidx[rt][i] : 0;  // all-NaN rows fall back to centre 0
          const double dd = pnorm[row] + (double)best[rt][i];
          dmin[row] = dd > 0.0 ? dd : 0.0;
          if (gap) gap[row] = (double)second[rt][i] - (double)best[rt][i];
        }
      }
    }
}

// Combines the G centre groups of assign_fast_kernel in group order.
__global__ __launch_bounds__(256) void assign_merge_kernel(int64_t rows, int G, int k, const float* __restrict__ pb,
                                                           const int32_t* __restrict__ pi, const float* __restrict__ ps,
                                                           const double* __restrict__ pnorm,
                                                           int32_t* __restrict__ labels, double* __restrict__ dmin,
                                                           double* __restrict__ gap) {
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= rows) return;
  float b = pb[row], s = ps[row];
  int bi = pi[row];
  for (int q = 1; q < G; ++q) {
    const int64_t o = (int64_t)q * rows + row;
    merge_best(b, bi, s, pb[o], pi[o], ps[o]);
  }
  labels[row] = bi < k ? bi : 0;
  const double dd = pnorm[row] + (double)b;
  dmin[row] = dd > 0.0 ? dd : 0.0;
  if (gap) gap[row] = (double)s - (double)b;
}

// Compiled shapes per type: k blocks (the smallest count >= the needed one is
// used), row tiles per wave, centre tiles per chunk and waves per SIMD.  The
// two chunk buffers (2 x CT x NKB KB) must leave room in the CU's 160 KB of
// LDS for that many work-groups: FP32 streams 16-centre chunks from 193
// dimensions on.
template <typename TC> struct AfShape {
  static constexpr int n = 5;
  static constexpr int nkb[n] = {2, 4, 7, 8, 16};
  static constexpr int rt[n] = {2, 2, 2, 2, 2};
  static constexpr int ct[n] = {2, 2, 2, 2, 2};
  static constexpr int occ[n] = {3, 3, 3, 3, 2};
};
template <> struct AfShape<float> {
  static constexpr int n = 6;
  static constexpr int nkb[n] = {4, 8, 13, 16, 24, 32};
  static constexpr int rt[n] = {1, 1, 1, 1, 1, 1};
  static constexpr int ct[n] = {2, 2, 2, 1, 1, 1};
  static constexpr int occ[n] = {3, 3, 3, 3, 2, 2};
};
template <typename TC> constexpr int af_dim_max() { return AfShape<TC>::nkb[AfShape<TC>::n - 1] * 4 * (16 / (int)sizeof(TC)); }

// Number of centre groups for a launch: whole rounds of resident work-groups
// times (chunks per group + about one chunk's worth of row loading and
// epilogue), plus half a chunk for the merge when groups are used.
static int af_groups(int64_t wgs, int nchunk, int64_t slots) {
  static const int forced = [] {
    const char* e = getenv("CABS_ASSIGN_GROUPS");  // a fixed group count, for measurements
    return e ? std::max(0, atoi(e)) : 0;
  }();
  if (forced > 0) return std::min(forced, std::min(nchunk, AF_MAXG));
  int bestG = 1;
  double bestc = (double)ceil_div(wgs, slots) * (nchunk + 1.0);
  for (int G = 2; G <= std::min(nchunk, AF_MAXG); ++G) {
    const int per = (int)ceil_div(nchunk, G);
    const int Ge = (int)ceil_div(nchunk, per);
    if (Ge != G) continue;
    const double c = (double)ceil_div(wgs * G, slots) * (per + 1.0) + 0.5;
    if (c < bestc) { bestc = c; bestG = G; }
  }
  return bestG;
}

template <typename TC, int I>
static void assign_fast_launch(int nkb, int64_t rows, int dim, int k, const TC* P, const TC* Zc, const double* znorm,
                               const double* pnorm, int32_t* labels, double* dmin, double* gap, float* pb, int32_t* pi,
                               float* ps, float* sacc, hipStream_t st) {
  constexpr int NKB = AfShape<TC>::nkb[I], RT = AfShape<TC>::rt[I], CT = AfShape<TC>::ct[I];
  constexpr int OCC = AfShape<TC>::occ[I];
  if constexpr (I + 1 < AfShape<TC>::n) {
    if (nkb > NKB)
      return assign_fast_launch<TC, I + 1>(nkb, rows, dim, k, P, Zc, znorm, pnorm, labels, dmin, gap, pb, pi, ps, sacc,
                                           st);
  }
  const int64_t wgs = ceil_div(rows, 64 * RT);
  const int nchunk = (int)ceil_div(k, CT * 16);
  const int G = pb ? af_groups(wgs, nchunk, (int64_t)device_cus() * OCC) : 1;
  const int gsize = (int)ceil_div(nchunk, G) * CT * 16;
  if (sacc)
    hipLaunchKernelGGL((assign_fast_kernel<TC, NKB, RT, CT, OCC, true>), dim3((unsigned)wgs, (unsigned)G), dim3(256), 0,
                       st, rows, dim, k, gsize, P, Zc, znorm, pnorm, labels, dmin, gap, G > 1 ? pb : nullptr, pi, ps,
                       sacc);
  else
    hipLaunchKernelGGL((assign_fast_kernel<TC, NKB, RT, CT, OCC, false>), dim3((unsigned)wgs, (unsigned)G), dim3(256),
                       0, st, rows, dim, k, gsize, P, Zc, znorm, pnorm, labels, dmin, gap, G > 1 ? pb : nullptr, pi,
                       ps, nullptr);
  if (G > 1)
    hipLaunchKernelGGL(assign_merge_kernel, dim3((unsigned)ceil_div(rows, 256)), dim3(256), 0, st, rows, G, k, pb, pi,
                       ps, pnorm, labels, dmin, gap);
}

template <typename TC> struct AssignFast { static constexpr bool ok = true; };
template <> struct AssignFast<double> { static constexpr bool ok = false; };

// Whether the fast assignment kernel takes these rows: its dimension limit,
// whole 16-byte runs per row, 16-byte aligned P and centres.
template <typename TC>
static bool assign_fast_ok(int dim, const void* P, const void* Zc) {
  if constexpr (AssignFast<TC>::ok) {
    constexpr int VE = 16 / (int)sizeof(TC);
    return dim <= af_dim_max<TC>() && dim % VE == 0 && ((uintptr_t)P % 16) == 0 && ((uintptr_t)Zc % 16) == 0;
  }
  return false;
}

// pb / pi / ps: AF_MAXG x rows partials for centre groups (null: one group).
// sacc (may be null): the fast kernel stores the dot products there.
template <typename TC>
static void launch_assign(int64_t rows, int dim, int k, const TC* P, const TC* Zc, const double* znorm,
                          const double* pnorm, int32_t* labels, double* dmin, double* gap, float* pb, int32_t* pi,
                          float* ps, float* sacc, hipStream_t st) {
  if constexpr (AssignFast<TC>::ok) {
    if (assign_fast_ok<TC>(dim, P, Zc)) {
      constexpr int VE = 16 / (int)sizeof(TC);
      const int nkb = (dim + 4 * VE - 1) / (4 * VE);
      assign_fast_launch<TC, 0>(nkb, rows, dim, k, P, Zc, znorm, pnorm, labels, dmin, gap, pb, pi, ps, sacc, st);
      return;
    }
  }
  hipLaunchKernelGGL(assign_kernel<TC>, dim3((unsigned)ceil_div(rows, 64)), dim3(256), 0, st, rows, dim, k, P, Zc,
                     znorm, pnorm, labels, dmin, gap);
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

// Exclusive scan over the 1024 threads of a block (16 waves): wave scans by
// shuffles, then the wave totals.
template <typename T>
__device__ __forceinline__ T block_excl_scan_1024(T v, T* wtot, T& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T x = __shfl_up(incl, o, 64);
    if (lane >= o) incl += x;
  }
  if (lane == 63) wtot[wave] = incl;
  __syncthreads();
  T base = 0, tot = 0;
  for (int w = 0; w < 16; ++w) {
    const T t = wtot[w];
    base += w < wave ? t : (T)0;
    tot += t;
  }
  __syncthreads();  // wtot may be reused
  total = tot;
  return base + incl - v;
}

// The exclusive scan of hist (label-major, k x nsb entries) runs over tiles of
// SC_TILE entries, one work-group each: scan_tile_sum_kernel sums every tile,
// scan_kernel adds the sums of the earlier tiles (in tile order) to its own
// block scan and writes the offsets and the start of every label whose first
// entry lies in the tile; label_chunks_kernel then forms cluster sizes, the
// chunk table and the largest cluster from the label starts.
constexpr int SC_R = 16;               // entries per thread
constexpr int SC_TILE = 1024 * SC_R;   // entries per tile

// Entries [e0, e0 + SC_R) of hist (16-byte loads when whole; hist is 16-byte
// aligned and e0 a multiple of SC_R).
__device__ __forceinline__ void scan_load(const int32_t* __restrict__ hist, int64_t L, int64_t e0, int32_t (&c)[SC_R]) {
  if (e0 + SC_R <= L) {
#pragma unroll
    for (int i = 0; i < SC_R; i += 4) {
      const int4 q = *(const int4*)(hist + e0 + i);
      c[i] = q.x; c[i + 1] = q.y; c[i + 2] = q.z; c[i + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < SC_R; ++i) c[i] = e0 + i < L ? hist[e0 + i] : 0;
  }
}

__global__ __launch_bounds__(1024) void scan_tile_sum_kernel(int64_t L, const int32_t* __restrict__ hist,
                                                             int32_t* __restrict__ tsum) {
  __shared__ int32_t wtot[16];
  const int64_t e0 = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_R;
  int32_t c[SC_R];
  scan_load(hist, L, e0, c);
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < SC_R; ++i) s += c[i];
  int32_t total;
  block_excl_scan_1024<int32_t>(s, wtot, total);
  if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void scan_kernel(int k, int64_t nsb, const int32_t* __restrict__ hist,
                                                    const int32_t* __restrict__ tsum, int32_t* __restrict__ offs,
                                                    int32_t* __restrict__ lstart) {
  __shared__ int32_t wtot[16];
  const int tid = threadIdx.x;
  const int64_t L = (int64_t)k * nsb;
  const int t = blockIdx.x;
  // carry = sum of the earlier tiles' totals (integers: any order is exact)
  int32_t part = 0;
  for (int q = tid; q < t; q += 1024) part += tsum[q];
  int32_t carry;
  block_excl_scan_1024<int32_t>(part, wtot, carry);
  const int64_t e0 = (int64_t)t * SC_TILE + (int64_t)tid * SC_R;
  int32_t c[SC_R];
  scan_load(hist, L, e0, c);
  int32_t sum = 0;
#pragma unroll
  for (int i = 0; i < SC_R; ++i) sum += c[i];
  int32_t tile_total;
  int32_t run = block_excl_scan_1024<int32_t>(sum, wtot, tile_total) + carry;
  int32_t lab = (int32_t)(e0 / nsb), rem = (int32_t)(e0 - (int64_t)lab * nsb);
#pragma unroll
  for (int i = 0; i < SC_R; ++i) {
    const int64_t e = e0 + i;
    if (e < L) {
      offs[e] = run;
      if (rem == 0) lstart[lab] = run;
    }
    run += c[i];
    if (++rem == nsb) { rem = 0; ++lab; }
  }
  if (t == (int)gridDim.x - 1 && tid == 0) lstart[k] = carry + tile_total;
}

// One workgroup: cluster sizes from the label starts, the chunk table (an
// exclusive scan of the chunk counts) and the largest cluster.
__global__ __launch_bounds__(1024) void label_chunks_kernel(int k, const int32_t* __restrict__ lstart,
                                                            int32_t* __restrict__ chunk_lab,
                                                            int32_t* __restrict__ chunk_beg,
                                                            int32_t* __restrict__ chunk_end,
                                                            int32_t* __restrict__ lchunk,
                                                            int32_t* __restrict__ nchunks_out,
                                                            double* __restrict__ tmax_out) {
  __shared__ int32_t wtot32[16];
  __shared__ int32_t lst[KM_MAXK + 1];
  __shared__ int32_t lch[KM_MAXK + 1];
  const int tid = threadIdx.x;
  for (int j = tid; j <= k; j += 1024) lst[j] = lstart[j];
  __syncthreads();
  int32_t cnt = 0, nch = 0;
  if (tid < k) {
    cnt = lst[tid + 1] - lst[tid];
    nch = (cnt + CENT_CH - 1) / CENT_CH;
  }
  int32_t nch_total;
  const int32_t ch0 = block_excl_scan_1024<int32_t>(nch, wtot32, nch_total);
  int32_t mx = cnt;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) { const int32_t x = __shfl_xor(mx, o, 64); mx = x > mx ? x : mx; }
  if ((tid & 63) == 0) wtot32[tid >> 6] = mx;
  __syncthreads();
  if (tid < k) { lchunk[tid] = ch0; lch[tid] = ch0; }
  if (tid == 0) {
    int32_t m = 0;
    for (int w = 0; w < 16; ++w) m = wtot32[w] > m ? wtot32[w] : m;
    lchunk[k] = nch_total;
    *nchunks_out = nch_total;
    if (tmax_out) *tmax_out = (double)m;
    lch[k] = nch_total;
  }
  __syncthreads();
  // chunk table: chunk c belongs to the label j with lch[j] <= c < lch[j + 1]
  // (labels without rows have lch[j] == lch[j + 1] and never match)
  for (int32_t c = tid; c < nch_total; c += 1024) {
    int lo = 0, hi = k;  // lch[lo] <= c < lch[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (lch[mid] <= c) lo = mid;
      else hi = mid;
    }
    const int32_t b = lst[lo] + (c - lch[lo]) * CENT_CH, en = lst[lo + 1];
    chunk_lab[c] = lo;
    chunk_beg[c] = b;
    chunk_end[c] = b + CENT_CH < en ? b + CENT_CH : en;
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

// One block per chunk (at most CENT_CH rows of one label).  The chunk's row
// indices and weights are staged in LDS; thread (row lane rl, column piece cv)
// sums rows rl, rl + RL, ... of the chunk in increasing order, with the loads
// of eight rows issued before any is used (rows past the chunk read a zero
// buffer with weight 0); the RL lane sums are then added in lane order.  A
// column piece is VW columns (one 16-byte load) when rows are 16-byte
// aligned, else one column.
template <typename TC, bool VEC>
__global__ __launch_bounds__(256) void centroid_partial_kernel(int dim, const TC* __restrict__ P,
                                                               const double* __restrict__ w,
                                                               const int32_t* __restrict__ sorted,
                                                               const int32_t* __restrict__ chunk_beg,
                                                               const int32_t* __restrict__ chunk_end,
                                                               const int32_t* __restrict__ nchunks,
                                                               double* __restrict__ part, double* __restrict__ partw) {
  constexpr int VW = VEC ? 16 / (int)sizeof(TC) : 1;
  constexpr int B = 8;
  __shared__ int32_t srow[CENT_CH];
  __shared__ double swt[CENT_CH];
  __shared__ double red[256 * VW];
  const int c = blockIdx.x;
  if (c >= *nchunks) return;
  const int tid = threadIdx.x;
  const int32_t b = chunk_beg[c];
  const int n = chunk_end[c] - b;
  if (tid < n) {
    const int32_t r = sorted[b + tid];
    srow[tid] = r;
    swt[tid] = w[r];
  }
  __syncthreads();
  if (tid < 64) {  // chunk weight: four consecutive weights per lane, then a fixed butterfly
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < CENT_CH / 64; ++i) {
      const int q = tid * (CENT_CH / 64) + i;
      s += q < n ? swt[q] : 0.0;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (tid == 0) partw[c] = s;
  }
  const int ncv = (dim + VW - 1) / VW;
  const int ncvp = ncv < 256 ? ncv : 256;
  const int RL = 256 / ncvp;
  const int rl = tid / ncvp, cvo = tid % ncvp;
  const TC* zero = (const TC*)kTileZero;
  for (int cv0 = 0; cv0 < ncv; cv0 += ncvp) {
    const int cv = cv0 + cvo;
    const bool act = rl < RL && cv < ncv;
    double acc[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] = 0.0;
    for (int p0 = act ? rl : n; p0 < n; p0 += B * RL) {
      TC x[B][VW];
      double wu[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int q = p0 + u * RL;
        const bool ok = q < n;
        const int qq = ok ? q : 0;
        wu[u] = ok ? swt[qq] : 0.0;
        const TC* src = ok ? P + (int64_t)srow[qq] * dim + cv * VW : zero;
        if constexpr (VEC) {
          const uint4 v4 = *(const uint4*)src;
          const TC* e = (const TC*)&v4;
#pragma unroll
          for (int i = 0; i < VW; ++i) x[u][i] = e[i];
        } else {
          x[u][0] = *src;
        }
      }
#pragma unroll
      for (int u = 0; u < B; ++u)
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] = fma(wu[u], to_f64(x[u][e]), acc[e]);
    }
    if (cv0 > 0) __syncthreads();  // previous pass has read red
    if (act) {
#pragma unroll
      for (int e = 0; e < VW; ++e) red[(rl * ncvp + cvo) * VW + e] = acc[e];
    }
    __syncthreads();
    for (int j = tid; j < ncvp * VW; j += 256) {
      const int col = cv0 * VW + j;
      if (col >= dim) continue;
      double s = red[j];
      for (int l = 1; l < RL; ++l) s += red[l * ncvp * VW + j];
      part[(int64_t)c * dim + col] = s;
    }
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

// One wave: lane t sums partials t, t + 64, ... in order, then the lanes are
// added in the fixed order of wave_sum.
__global__ void wsum_final_kernel(int nb, const double* __restrict__ part_s, const double* __restrict__ part_g,
                                  double* __restrict__ out_s, double* __restrict__ out_g) {
  double s = 0.0, g = __builtin_huge_val();
  for (int b = threadIdx.x; b < nb; b += 64) { s += part_s[b]; g = part_g[b] < g ? part_g[b] : g; }
  s = wave_sum(s);
  g = wave_min(g);
  if (threadIdx.x == 0) {
    if (out_s) *out_s = s;
    if (out_g) *out_g = g;
  }
}

// ---------------------------------------------------------------------------
// Snapping
// ---------------------------------------------------------------------------
// Squared distance of a row to a centre from the norms and the MFMA dot
// product.  Written with an explicit fma so that every kernel that needs it
// rounds identically; NaN counts as +inf (never the nearest).
__device__ __forceinline__ double snap_dist(double pn, double zn, double dot) {
  const double d = __builtin_fma(-2.0, dot, pn + zn);
  return d > 0.0 ? d : (d == d ? 0.0 : __builtin_huge_val());
}

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

// The distances of RT 16-row tiles x SNAP_NT 16-centre tiles at once, with
// gemm_tile's loads and MFMA sequence (k blocks of 4 LK elements, lane group g
// holding elements g LK .. g LK + LK - 1 of a block, STEPS MFMAs per block in
// element order) but each centre fragment loaded once for the RT row tiles
// instead of once per tile.  Per output element the MFMA sequence is
// gemm_tile's, so the values are bit-identical to a one-tile gemm_tile call at
// the same row and column offsets (the resolver's rescans rely on that).
template <typename TC, int RT>
__device__ __forceinline__ void snap_tile_rt(const TC* __restrict__ P, int dim, int64_t M, int64_t row0,
                                             const TC* __restrict__ Zc, int k, int col0,
                                             typename Mfma<TC>::acc (&acc)[RT][SNAP_NT]) {
  constexpr int LK = TileK<TC>::LK;
  constexpr int KPL = Mfma<TC>::KPL;
  constexpr int STEPS = LK / KPL;
  constexpr int NT = SNAP_NT;
  constexpr bool PREFETCH = false;  // two waves per SIMD hide the load latency instead
  const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
  const TC* xp[RT];
  bool xok[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t row = row0 + 16 * rt + r;
    xok[rt] = row < M;
    xp[rt] = P + (xok[rt] ? row : 0) * dim;
  }
  const TC* yp[NT];
  bool yok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int c = col0 + 16 * t + r;
    yok[t] = c < k;
    yp[t] = Zc + (int64_t)(yok[t] ? c : 0) * dim;
  }
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[rt][t] = Mfma<TC>::zero();
  const bool vec = (dim % LK) == 0 && (((uintptr_t)P | (uintptr_t)Zc) & 15) == 0;
  auto fetch = [&](int kb, TC (&xv)[RT][LK], TC (&yv)[NT][LK]) {
    const int kk = kb + g * LK;
    if (vec && kb + 4 * LK <= dim) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) tile_run_vec<TC, LK>(xp[rt], kk, xok[rt], xv[rt]);
#pragma unroll
      for (int t = 0; t < NT; ++t) tile_run_vec<TC, LK>(yp[t], kk, yok[t], yv[t]);
    } else {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) tile_run_elem<TC, LK>(xp[rt], kk, dim, xok[rt], xv[rt]);
#pragma unroll
      for (int t = 0; t < NT; ++t) tile_run_elem<TC, LK>(yp[t], kk, dim, yok[t], yv[t]);
    }
  };
  auto compute = [&](const TC (&xv)[RT][LK], const TC (&yv)[NT][LK]) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int s2 = 0; s2 < STEPS; ++s2) {
          TC as_[KPL], bs_[KPL];
#pragma unroll
          for (int e = 0; e < KPL; ++e) { as_[e] = xv[rt][s2 * KPL + e]; bs_[e] = yv[t][s2 * KPL + e]; }
          acc[rt][t] = Mfma<TC>::mma(FragPack<TC, KPL>::get(as_, 0), FragPack<TC, KPL>::get(bs_, 0), acc[rt][t]);
        }
  };
  TC xv[RT][LK], yv[NT][LK];
  if constexpr (PREFETCH) {
    if (dim > 0) fetch(0, xv, yv);
    for (int kb = 0; kb < dim; kb += 4 * LK) {
      TC xn[RT][LK], yn[NT][LK];
      const bool more = kb + 4 * LK < dim;
      if (more) fetch(kb + 4 * LK, xn, yn);
      compute(xv, yv);
      if (more) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int e = 0; e < LK; ++e) xv[rt][e] = xn[rt][e];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int e = 0; e < LK; ++e) yv[t][e] = yn[t][e];
      }
    }
  } else {
    for (int kb = 0; kb < dim; kb += 4 * LK) {
      fetch(kb, xv, yv);
      compute(xv, yv);
    }
  }
}

// Per block of rows_per_block consecutive rows and per centre: the SNAP_T
// nearest rows, sorted by (distance, row).  Wave w takes the 64-centre chunks
// w, w + 4, ... (lane = centre) and walks the block's rows in groups of SRT
// 16-row tiles: it forms the group's distances (snap_tile_rt over the chunk's
// 4 column tiles, each centre fragment loaded once per group), then, tile by
// tile through its own LDS tile, each lane inserts its centre's 16 distances
// in row order.  One list per (block, centre), so each list fills once; no
// barrier across waves.  A list holding fewer than SNAP_T rows means every
// other row of the block is at +inf.  Rows of norm 0 are left out (+inf): they
// form one class of equal distance to every centre, which the resolver handles
// as a single candidate (its lowest untaken row).  Each 16-centre column tile of gemm_tile
// is an independent MFMA chain and every row tile starts 16-aligned from the
// block start, so snap_resolve_kernel recomputes these distances bit-exactly
// from a one-tile call at the same row and column offsets.
template <typename TC>
__global__ __launch_bounds__(256) void snap_topt_kernel(int64_t rows, int dim, int k, int64_t rows_per_block,
                                                        const TC* __restrict__ P, const TC* __restrict__ Zc,
                                                        const double* __restrict__ znorm,
                                                        const double* __restrict__ pnorm, double* __restrict__ cand_d,
                                                        int32_t* __restrict__ cand_r) {
  typedef typename Mfma<TC>::acc AccV;
  constexpr int SRT = 2;  // row tiles sharing each centre fragment load
  constexpr int LDD = SNAP_CC + 1;
  __shared__ double sm_d[4][16 * SRT * LDD];  // per wave: 16 SRT rows x 64 centres
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t rbeg = (int64_t)blockIdx.x * rows_per_block;
  const int64_t rend = rbeg + rows_per_block < rows ? rbeg + rows_per_block : rows;
  const int nblk = gridDim.x;
  double* sd = sm_d[wave];
  for (int cw = wave * SNAP_CC; cw < k; cw += 4 * SNAP_CC) {
    double td[SNAP_T];
    int tr[SNAP_T];
#pragma unroll
    for (int q = 0; q < SNAP_T; ++q) { td[q] = __builtin_huge_val(); tr[q] = 0x7fffffff; }
    const int myc = cw + lane;  // centre tracked by this lane
    for (int64_t row0 = rbeg; row0 < rend; row0 += 16 * SRT) {
      {
        AccV acc[SRT][SNAP_NT];
        snap_tile_rt<TC, SRT>(P, dim, rend, row0, Zc, k, cw, acc);
#pragma unroll
        for (int rt = 0; rt < SRT; ++rt)
#pragma unroll
          for (int t = 0; t < SNAP_NT; ++t) {
            const int cl = t * 16 + c16;
            const int col = cw + cl;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int rl = 16 * rt + out_row<TC>(g, i);
              const int64_t row = row0 + rl;
              double d = __builtin_huge_val();
              if (row < rend && col < k && pnorm[row] != 0.0)
                d = snap_dist(pnorm[row], znorm[col], (double)acc[rt][t][i]);
              sd[rl * LDD + cl] = d;
            }
          }
      }
      wave_lds_sync();
      if (myc < k) {
        for (int q = 0; q < 16 * SRT; ++q) {
          const int64_t row = row0 + q;
          if (row >= rend) break;
          topt_insert<double>(td, tr, sd[q * LDD + lane], (int)row);
        }
      }
      wave_lds_sync();  // the tile is rewritten next
    }
    if (myc < k) {
      const int64_t base = ((int64_t)myc * nblk + blockIdx.x) * SNAP_T;
#pragma unroll
      for (int q = 0; q < SNAP_T; ++q) {
        cand_d[base + q] = td[q];
        cand_r[base + q] = tr[q];
      }
    }
  }
}

// The same per-block lists from the dot products the final assignment stored
// (sacc[row k + centre]): that kernel's MFMA sequence per element is the tile
// core's, so each distance snap_dist(|p|^2, |z|^2, dot) is bit for bit the one
// snap_topt_kernel forms, and the rows are inserted in the same order.  Wave w
// takes the 64-centre chunks w, w + 4, ... (lane = centre) and reads the block's
// rows eight at a time (one coalesced 256-byte run per row).
__global__ __launch_bounds__(256) void snap_select_kernel(int64_t rows, int k, int64_t rows_per_block,
                                                          const float* __restrict__ sacc,
                                                          const double* __restrict__ znorm,
                                                          const double* __restrict__ pnorm, double* __restrict__ cand_d,
                                                          int32_t* __restrict__ cand_r) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t rbeg = (int64_t)blockIdx.x * rows_per_block;
  const int64_t rend = rbeg + rows_per_block < rows ? rbeg + rows_per_block : rows;
  const int nblk = gridDim.x;
  constexpr int U = 8;
  for (int cw = wave * SNAP_CC; cw < k; cw += 4 * SNAP_CC) {
    const int myc = cw + lane;
    if (myc >= k) continue;
    double td[SNAP_T];
    int tr[SNAP_T];
#pragma unroll
    for (int q = 0; q < SNAP_T; ++q) { td[q] = __builtin_huge_val(); tr[q] = 0x7fffffff; }
    const double zn = znorm[myc];
    for (int64_t r0 = rbeg; r0 < rend; r0 += U) {
      float a[U];
      double pn[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t row = r0 + u < rend ? r0 + u : rend - 1;
        a[u] = sacc[row * k + myc];
        pn[u] = pnorm[row];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (r0 + u >= rend) break;
        const double d = pn[u] != 0.0 ? snap_dist(pn[u], zn, (double)a[u]) : __builtin_huge_val();
        topt_insert<double>(td, tr, d, (int)(r0 + u));
      }
    }
    const int64_t base = ((int64_t)myc * nblk + blockIdx.x) * SNAP_T;
#pragma unroll
    for (int q = 0; q < SNAP_T; ++q) {
      cand_d[base + q] = td[q];
      cand_r[base + q] = tr[q];
    }
  }
}

// Per centre: the SNAP_T smallest (distance, row) pairs over the per-block
// lists, each of which is sorted.  Rows are distinct, so exactly SNAP_T list
// heads are no greater than tau, the SNAP_T-th smallest head; every pair of
// the result is no greater than tau, and only those SNAP_T lists hold such
// pairs.  So the heads are sorted to find tau, the pairs no greater than tau
// (at most SNAP_T * SNAP_T) are gathered, and those are sorted.
__device__ __forceinline__ bool pair_gt(double a, int32_t ra, double b, int32_t rb) {
  return a > b || (a == b && ra > rb);
}

template <int N, int NT>
__device__ __forceinline__ void bitonic_pairs(double* sd, int32_t* sr, int P2) {
  for (int size = 2; size <= P2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P2; t += NT) {
        const int p = t ^ stride;
        if (p > t) {
          const bool up = (t & size) == 0;
          const double a = sd[t], b = sd[p];
          const int32_t ra = sr[t], rb = sr[p];
          if (pair_gt(a, ra, b, rb) == up) { sd[t] = b; sd[p] = a; sr[t] = rb; sr[p] = ra; }
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(256) void snap_merge_kernel(int nblk, const double* __restrict__ cand_d,
                                                         const int32_t* __restrict__ cand_r, double* __restrict__ top_d,
                                                         int32_t* __restrict__ top_r) {
  constexpr int32_t SENT = 0x7fffffff;
  constexpr int NC = SNAP_T * SNAP_T;
  __shared__ double hd[SNAP_MAXBLK];
  __shared__ int32_t hr[SNAP_MAXBLK];
  __shared__ double sd[NC];
  __shared__ int32_t sr[NC];
  __shared__ int cnt;
  const int j = blockIdx.x, tid = threadIdx.x;
  const int64_t base = (int64_t)j * nblk * SNAP_T;
  const double INF = __builtin_huge_val();
  int P2 = 1;
  while (P2 < nblk) P2 <<= 1;
  for (int e = tid; e < P2; e += 256) {
    hd[e] = e < nblk ? cand_d[base + (int64_t)e * SNAP_T] : INF;
    hr[e] = e < nblk ? cand_r[base + (int64_t)e * SNAP_T] : SENT;
  }
  for (int e = tid; e < NC; e += 256) { sd[e] = INF; sr[e] = SENT; }
  if (tid == 0) cnt = 0;
  __syncthreads();
  bitonic_pairs<SNAP_MAXBLK, 256>(hd, hr, P2);
  const double tau = P2 >= SNAP_T ? hd[SNAP_T - 1] : INF;
  const int32_t taur = P2 >= SNAP_T ? hr[SNAP_T - 1] : SENT;
  for (int b = tid; b < nblk; b += 256) {
    const int64_t o = base + (int64_t)b * SNAP_T;
    for (int q = 0; q < SNAP_T; ++q) {
      const double d = cand_d[o + q];
      const int32_t r = cand_r[o + q];
      if (r == SENT || pair_gt(d, r, tau, taur)) break;
      const int slot = atomicAdd(&cnt, 1);
      if (slot < NC) { sd[slot] = d; sr[slot] = r; }
    }
  }
  __syncthreads();
  bitonic_pairs<NC, 256>(sd, sr, NC);
  if (tid < SNAP_T) {
    top_d[(int64_t)j * SNAP_T + tid] = sd[tid];
    top_r[(int64_t)j * SNAP_T + tid] = sr[tid];
  }
}

// Rows of FP64 squared norm 0, ascending (the all-zero rows of sparse
// embeddings): block b counts its contiguous chunk, one block turns the counts
// into offsets (zoff[ZR_NB] = the total), block b writes its chunk's rows.
constexpr int ZR_NB = 256;

__device__ __forceinline__ void zr_chunk(int64_t rows, int b, int64_t& r0, int64_t& r1) {
  const int64_t ch = (rows + ZR_NB - 1) / ZR_NB;
  r0 = (int64_t)b * ch;
  r1 = r0 + ch < rows ? r0 + ch : rows;
}

__global__ __launch_bounds__(256) void zero_rows_count_kernel(int64_t rows, const double* __restrict__ pnorm,
                                                              int32_t* __restrict__ zcnt) {
  __shared__ int wc[4];
  int64_t r0, r1;
  zr_chunk(rows, blockIdx.x, r0, r1);
  int c = 0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) c += pnorm[r] == 0.0 ? 1 : 0;
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) zcnt[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

__global__ void zero_rows_scan_kernel(const int32_t* __restrict__ zcnt, int32_t* __restrict__ zoff) {
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int b = 0; b < ZR_NB; ++b) { zoff[b] = s; s += zcnt[b]; }
    zoff[ZR_NB] = s;
  }
}

__global__ __launch_bounds__(256) void zero_rows_write_kernel(int64_t rows, const double* __restrict__ pnorm,
                                                              const int32_t* __restrict__ zoff,
                                                              int32_t* __restrict__ zrows) {
  __shared__ int wc[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int64_t r0, r1;
  zr_chunk(rows, blockIdx.x, r0, r1);
  int32_t base = zoff[blockIdx.x];
  for (int64_t t0 = r0; t0 < r1; t0 += 256) {
    const int64_t r = t0 + threadIdx.x;
    const bool z = r < r1 && pnorm[r] == 0.0;
    const uint64_t m = __ballot(z);
    if (lane == 0) wc[wave] = __builtin_popcountll(m);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wc[w];
    const int tot = wc[0] + wc[1] + wc[2] + wc[3];
    if (z) zrows[base + before + __builtin_popcountll(m & ((1ull << lane) - 1))] = (int32_t)r;
    base += tot;
    __syncthreads();  // wc is rewritten next
  }
}

// Snapping, in centre order: centre j takes the nearest row not taken by an
// earlier centre; distances within tie_rtol * (|Z_j| + sqrt(d_min))^2 of the
// nearest untaken one count as ties and go to the lowest row index (the
// centre of a two-row cluster is equidistant from both rows).
//
// Wave 0 walks the centres using their merged top-SNAP_T lists staged in LDS;
// taken rows live in an LDS hash set.  When a merged list cannot decide
// (every candidate taken, or the tie window reaching past the list) the whole
// block resolves the centre from the per-block lists: each block contributes
// its first untaken candidate, and a block whose SNAP_T-th listed distance
// lies inside the current window (so unlisted rows of that block might too) is
// rescanned.  Rescans recompute the block's distances exactly as the top-T
// pass did (same tile calls, same rounding) into dws; the window is
// recomputed and the rescan set widened until no further block qualifies.
// Rows of norm 0 are in no list and no rescan: all of them lie at the same
// distance snap_dist(0, |Z_j|^2, 0) from centre j (the value the tile pass
// gives them), so of that class only its lowest untaken row can be chosen,
// and they are taken in ascending order: one candidate per centre, read from
// the ascending list zrows at a moving position.
constexpr int RES_CHUNK = 128;
constexpr int RES_HT = 2048;  // hash slots for taken rows (k <= KM_MAXK = RES_HT / 2)

__device__ __forceinline__ int res_slot(int32_t r) { return (int)(((uint32_t)r * 2654435761u) >> 21); }
__device__ __forceinline__ bool res_has(const int32_t* ht, int32_t r) {
  for (int h = res_slot(r);; h = (h + 1) & (RES_HT - 1)) {
    const int32_t v = ht[h];
    if (v == r) return true;
    if (v < 0) return false;
  }
}
__device__ __forceinline__ void res_put(int32_t* ht, int32_t r) {
  int h = res_slot(r);
  while (ht[h] >= 0 && ht[h] != r) h = (h + 1) & (RES_HT - 1);
  ht[h] = r;
}

template <typename TC>
__global__ __launch_bounds__(1024) void snap_resolve_kernel(
    int64_t rows, int dim, int k, const TC* __restrict__ P, const TC* __restrict__ Zc,
    const double* __restrict__ znorm, const double* __restrict__ pnorm, const double* __restrict__ top_d,
    const int32_t* __restrict__ top_r, const double* __restrict__ cand_d, const int32_t* __restrict__ cand_r, int nblk,
    int64_t rows_per_block, double tie_rtol, double* __restrict__ dws, const int32_t* __restrict__ zrows,
    const int32_t* __restrict__ zoff, int64_t* __restrict__ out, double* __restrict__ nfall) {
  typedef typename Mfma<TC>::acc AccV;
  typedef typename NormT<TC>::type NrmT;
  constexpr int32_t SENT = 0x7fffffff;
  const int32_t nzero = zoff[ZR_NB];
  __shared__ int32_t sh_zp;             // zrows[sh_zp] is the lowest untaken row of norm 0
  __shared__ double lzn[RES_CHUNK];     // |Z_j|^2 of the staged centres
  __shared__ int64_t chosen[KM_MAXK];
  __shared__ int32_t ht[RES_HT];
  __shared__ double ld[RES_CHUNK * SNAP_T];
  __shared__ int32_t lr[RES_CHUNK * SNAP_T];
  __shared__ double lz[RES_CHUNK];
  __shared__ double b_fd[SNAP_MAXBLK], b_bound[SNAP_MAXBLK], b_smin[SNAP_MAXBLK];
  __shared__ int32_t b_state[SNAP_MAXBLK];  // 0 list, 1 rescanned, 2 rescan pending
  __shared__ double wred[16];
  __shared__ int64_t wrow[16];
  __shared__ int sh_next, sh_more;
  __shared__ double sh_lim;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const double INF = __builtin_huge_val();
  for (int e = tid; e < RES_HT; e += 1024) ht[e] = -1;
  if (tid == 0) sh_zp = 0;
  int j = 0;
  int chunk0 = -RES_CHUNK;
  int fallbacks = 0;
  while (j < k) {
    if (j >= chunk0 + RES_CHUNK) {  // stage the lists of centres [j, j + RES_CHUNK)
      __syncthreads();
      chunk0 = j;
      const int n = (k - j < RES_CHUNK ? k - j : RES_CHUNK);
      for (int e = tid; e < n * SNAP_T; e += 1024) {
        ld[e] = top_d[(int64_t)j * SNAP_T + e];
        lr[e] = top_r[(int64_t)j * SNAP_T + e];
      }
      for (int e = tid; e < n; e += 1024) {
        lzn[e] = znorm[j + e];
        lz[e] = sqrt(lzn[e]);
      }
    }
    __syncthreads();
    if (wave == 0) {
      int jj = j;
      const int lim = (chunk0 + RES_CHUNK < k ? chunk0 + RES_CHUNK : k);
      // One centre at a time, its list's SNAP_T candidates checked at once
      // (lane q holds candidate q), plus the zero-norm class's candidate:
      // dmin is the nearer of the first untaken listed row and that class;
      // the choice is the lowest untaken row within [dmin, dmin + tol] among
      // the listed rows and the class.  Undecided: no candidate at all, or a
      // full list whose last distance lies inside the window (then unlisted
      // rows may be inside too).
      int zp = sh_zp;
      for (; jj < lim; ++jj) {
        const double zn = lz[jj - chunk0];
        const int q = lane;
        int32_t r = SENT;
        double d = INF;
        if (q < SNAP_T) {
          r = lr[(jj - chunk0) * SNAP_T + q];
          d = ld[(jj - chunk0) * SNAP_T + q];
        }
        const bool valid = r != SENT;  // lists hold their entries first, then SENT
        const bool free_row = valid && !res_has(ht, r);
        const uint64_t m_end = __ballot(q < SNAP_T && !valid);
        const int q_end = m_end ? __builtin_ctzll(m_end) : SNAP_T;
        const uint64_t m_free = __ballot(free_row && q < q_end);
        const double dfree = m_free ? __shfl(d, __builtin_ctzll(m_free), 64) : INF;
        const bool has0 = zp < nzero;
        const double d0 = has0 ? snap_dist(0.0, lzn[jj - chunk0], 0.0) : INF;
        const double dmin = dfree < d0 ? dfree : d0;
        if (!(dmin < INF)) break;  // undecided
        const double rr = zn + sqrt(dmin);
        const double wlim = dmin + tie_rtol * rr * rr;
        const double dlast = __shfl(d, SNAP_T - 1, 64);
        if (q_end == SNAP_T && dlast <= wlim) break;  // undecided: a full list ends inside the window
        int32_t found = wave_min<int32_t>(free_row && q < q_end && d <= wlim ? r : SENT);
        const bool take0 = has0 && d0 <= wlim && zrows[zp] < found;
        if (take0) found = zrows[zp];
        if (lane == 0) {
          chosen[jj] = found;
          if (!take0) res_put(ht, found);
        }
        if (take0) ++zp;
        wave_lds_sync();  // the next centre's lookups see the new row
      }
      if (lane == 0) sh_zp = zp;
      if (lane == 0) sh_next = jj;
    }
    __syncthreads();
    j = sh_next;
    if (j >= k) break;
    if (j >= chunk0 + RES_CHUNK) continue;  // next chunk

    // ---- centre j from the per-block lists ----
    ++fallbacks;
    const double zn = lz[j - chunk0];
    const int64_t cbase = (int64_t)j * nblk * SNAP_T;
    for (int b = tid; b < nblk; b += 1024) {
      double fd = INF;
      for (int q = 0; q < SNAP_T; ++q) {
        const int32_t r = cand_r[cbase + b * SNAP_T + q];
        if (r == SENT) break;
        if (!res_has(ht, r)) { fd = cand_d[cbase + b * SNAP_T + q]; break; }
      }
      const bool full = cand_r[cbase + b * SNAP_T + SNAP_T - 1] != SENT;
      b_fd[b] = fd;
      b_bound[b] = full ? cand_d[cbase + b * SNAP_T + SNAP_T - 1] : INF;
      b_smin[b] = INF;
      b_state[b] = 0;
    }
    __syncthreads();
    const int cc = (j / SNAP_CC) * SNAP_CC;
    const int col0 = cc + ((j - cc) / 16) * 16;
    const int jc = j - col0;
    for (;;) {
      if (wave == 0) {
        double m = sh_zp < nzero ? snap_dist(0.0, lzn[j - chunk0], 0.0) : INF;
        for (int b = lane; b < nblk; b += 64) {
          const double v = b_state[b] ? b_smin[b] : b_fd[b];
          m = v < m ? v : m;
        }
        m = wave_min(m);
        const double rr = zn + sqrt(m < INF ? m : 0.0);
        const double lim = m < INF ? m + tie_rtol * rr * rr : INF;
        bool any = false;
        for (int b = lane; b < nblk; b += 64)
          if (b_state[b] == 0 && b_bound[b] <= lim) { b_state[b] = 2; any = true; }
        any = __ballot(any) != 0;
        if (lane == 0) { sh_lim = lim; sh_more = any ? 1 : 0; }
      }
      __syncthreads();
      if (!sh_more) break;
      // Rescans, one block per wave (the whole block's 16-row tiles, the same tile calls and
      // rounding as the top-T pass), then one barrier: sparse embeddings with many identical rows
      // send most centres here, and every block of such a tie class qualifies.
      for (int b = wave; b < nblk; b += 16) {
        if (b_state[b] != 2) continue;  // uniform within the wave: LDS value read after a barrier
        const int64_t rbeg = (int64_t)b * rows_per_block;
        const int64_t rend = rbeg + rows_per_block < rows ? rbeg + rows_per_block : rows;
        double mloc = INF;
        for (int64_t row0 = rbeg; row0 < rend; row0 += 16) {
          AccV acc[1];
          NrmT xs, ys[1];
          gemm_tile<TC, TC, 1, false>(P, dim, rend, row0, Zc, dim, nullptr, k, col0, nullptr, dim, acc, xs, ys);
          if ((lane & 15) == jc) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int64_t row = row0 + out_row<TC>(lane >> 4, i);
              if (row < rend) {
                double d = snap_dist(pnorm[row], znorm[j], (double)acc[0][i]);
                if (pnorm[row] == 0.0 || res_has(ht, (int32_t)row)) d = INF;
                dws[row] = d;
                mloc = d < mloc ? d : mloc;
              }
            }
          }
        }
        mloc = wave_min(mloc);
        if (lane == 0) {
          b_smin[b] = mloc;
          b_state[b] = 1;
        }
      }
      __syncthreads();
    }
    // lowest untaken row inside the window
    const double lim = sh_lim;
    int64_t best = INT64_MAX;
    for (int b = tid; b < nblk; b += 1024) {
      if (b_state[b] != 0) continue;
      for (int q = 0; q < SNAP_T; ++q) {
        const int32_t r = cand_r[cbase + b * SNAP_T + q];
        if (r == SENT || cand_d[cbase + b * SNAP_T + q] > lim) break;
        if (!res_has(ht, r) && r < best) best = r;
      }
    }
    for (int b = 0; b < nblk; ++b) {
      if (b_state[b] != 1) continue;
      const int64_t rbeg = (int64_t)b * rows_per_block;
      const int64_t rend = rbeg + rows_per_block < rows ? rbeg + rows_per_block : rows;
      for (int64_t row = rbeg + tid; row < rend && row < best; row += 1024)
        if (dws[row] <= lim) { best = row; break; }
    }
    best = wave_min<int64_t>(best);
    if (lane == 0) wrow[wave] = best;
    __syncthreads();
    if (tid == 0) {
      int64_t r = wrow[0];
      for (int w = 1; w < 16; ++w) r = wrow[w] < r ? wrow[w] : r;
      const int zp = sh_zp;
      if (zp < nzero && snap_dist(0.0, lzn[j - chunk0], 0.0) <= lim && zrows[zp] < r) {
        r = zrows[zp];
        sh_zp = zp + 1;
      } else {
        if (r == INT64_MAX)  // unreachable while k <= rows: every block was rescanned at lim = +inf
          for (r = 0; r < rows && (res_has(ht, (int32_t)r) || pnorm[r] == 0.0); ++r) {}
        res_put(ht, (int32_t)r);
      }
      chosen[j] = r;
      sh_next = j + 1;
    }
    __syncthreads();
    j = sh_next;
  }
  __syncthreads();
  // ascending order (reuses the candidate area as sort keys)
  int64_t* keys = (int64_t*)ld;
  static_assert(RES_CHUNK * SNAP_T >= KM_MAXK, "sort keys must fit the staging area");
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
  if (tid == 0 && nfall) *nfall = (double)fallbacks;
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
struct KmWs {
  void* Zc; double* znorm; double* pnorm; int32_t* labels; double* dmin; double* gap;
  int32_t* hist; int32_t* offs; int32_t* rank_blk; int32_t* sorted; int32_t* lstart;
  int32_t* chunk_lab; int32_t* chunk_beg; int32_t* chunk_end; int32_t* lchunk; int32_t* nchunks;
  double* part; double* partw; double* red_s; double* red_g; double* obj_tmp; double* tmax_tmp; double* gap_tmp;
  double* cand_d; int32_t* cand_r; double* top_d; int32_t* top_r; int32_t* zrows; int32_t* zcnt;
  float* apb; int32_t* api; float* aps; int32_t* tsum;
  float* sacc;  // rows x k dot products of the final assignment (null: the top-T pass forms its own)
  size_t total;
};

// Row blocks of the top-T pass: about SNAP_ROWS rows each, at most
// SNAP_MAXBLK, and at most SNAP_MAXCAND / k so the candidate lists stay bounded.
static inline int snap_nblk(int64_t rows, int k) {
  int64_t nb = ceil_div(rows, SNAP_ROWS);
  if (nb < 256) nb = ceil_div(rows, SNAP_SUB);  // few rows: 64-row blocks, so that more work-groups run
  const int64_t cap = std::min<int64_t>(SNAP_MAXBLK, std::max<int64_t>(1, SNAP_MAXCAND / k));
  if (nb > cap) nb = cap;
  return (int)(nb < 1 ? 1 : nb);
}
constexpr int RED_NB = 256;

// Whether the snap can take its distances from the final assignment: the
// precisions with a fast assignment kernel, at dimensions it takes.
static bool snap_from_assign(int dim, int compute) {
  switch (compute) {
    case P_F32: return dim <= af_dim_max<float>() && dim % 4 == 0;
    case P_BF16: return dim <= af_dim_max<bf16>() && dim % 8 == 0;
    case P_F16: return dim <= af_dim_max<f16>() && dim % 8 == 0;
    default: return false;
  }
}

// lean: no room for the stored dot products (the snap forms its own distances).
static KmWs km_layout(void* base, int64_t rows, int dim, int k, int compute, bool lean) {
  KmWs w{};
  char* p = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) { void* q = p ? p + off : nullptr; off += al256(bytes); return q; };
  const int64_t nsb = ceil_div(rows, HIST_SB);
  const int64_t maxch = ceil_div(rows, CENT_CH) + k;
  const int nblk = snap_nblk(rows, k);
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
  w.zrows = (int32_t*)take(rows * 4);
  w.zcnt = (int32_t*)take(2 * (ZR_NB + 1) * 4);
  w.apb = (float*)take((size_t)AF_MAXG * rows * 4);
  w.api = (int32_t*)take((size_t)AF_MAXG * rows * 4);
  w.aps = (float*)take((size_t)AF_MAXG * rows * 4);
  w.tsum = (int32_t*)take((size_t)ceil_div((int64_t)k * nsb, SC_TILE) * 4);
  w.sacc = (!lean && snap_from_assign(dim, compute)) ? (float*)take((size_t)rows * k * 4) : nullptr;
  w.total = off;
  return w;
}

size_t kmeans_ws_bytes(int64_t rows, int dim, int k, int compute, bool lean) {
  return km_layout(nullptr, rows, dim, k, compute, lean).total + 256;
}

template <typename TC>
static hipError_t kmeans_t(int compute, int64_t rows, int dim, int k, const void* Pv, const double* w, const double* Z0,
                           int iters, const KMeansOut& out, void* ws, bool lean, hipStream_t st) {
  const TC* P = (const TC*)Pv;
  KmWs W = km_layout(ws, rows, dim, k, compute, lean);
  TC* Zc = (TC*)W.Zc;
  const int64_t nsb = ceil_div(rows, HIST_SB);
  const unsigned gR = (unsigned)ceil_div(rows, 4);
  const int64_t maxch = ceil_div(rows, CENT_CH) + k;
  int32_t* labels = out.labels ? out.labels : W.labels;
  const int red_nb = (int)(rows < RED_NB * 256 ? ceil_div(rows, 256) : RED_NB);
  const unsigned ntile = (unsigned)ceil_div((int64_t)k * nsb, SC_TILE);

  if (Z0 != out.Z)
    hipLaunchKernelGGL(copy_f64_kernel, dim3((unsigned)ceil_div((int64_t)k * dim, 256)), dim3(256), 0, st,
                       (int64_t)k * dim, Z0, out.Z);
  hipLaunchKernelGGL(zprep_kernel<TC>, dim3(k), dim3(256), 0, st, k, dim, out.Z, Zc, W.znorm);
  hipLaunchKernelGGL(rownorm2_kernel<TC>, dim3(gR), dim3(256), 0, st, rows, dim, P, W.pnorm);

  // the final assignment stores its dot products for the snap when there is room and the fast kernel takes P
  const bool stored = out.snap != nullptr && W.sacc != nullptr && assign_fast_ok<TC>(dim, P, Zc);
  for (int it = 0; it <= iters; ++it) {
    const bool last = it == iters;
    {
      TimerScope ts(T_ASSIGN, st);
      launch_assign<TC>(rows, dim, k, P, (const TC*)Zc, W.znorm, W.pnorm, labels, W.dmin, last ? W.gap : nullptr,
                        W.apb, W.api, W.aps, last && stored ? W.sacc : nullptr, st);
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
    hipLaunchKernelGGL(scan_tile_sum_kernel, dim3(ntile), dim3(1024), 0, st, (int64_t)k * nsb, W.hist, W.tsum);
    hipLaunchKernelGGL(scan_kernel, dim3(ntile), dim3(1024), 0, st, k, nsb, W.hist, W.tsum, W.offs, W.lstart);
    hipLaunchKernelGGL(label_chunks_kernel, dim3(1), dim3(1024), 0, st, k, W.lstart, W.chunk_lab, W.chunk_beg,
                       W.chunk_end, W.lchunk, W.nchunks, last ? (out.tmax ? out.tmax : W.tmax_tmp) : nullptr);
    if (last) break;
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)ceil_div(rows, 256)), dim3(256), 0, st, rows, nsb, labels,
                       W.rank_blk, W.offs, W.sorted);
    {
      TimerScope ts(T_CENTROID, st);
      const bool vec = ((uintptr_t)P % 16) == 0 && ((size_t)dim * sizeof(TC)) % 16 == 0;
      if (vec)
        hipLaunchKernelGGL((centroid_partial_kernel<TC, true>), dim3((unsigned)maxch), dim3(256), 0, st, dim, P, w,
                           W.sorted, W.chunk_beg, W.chunk_end, W.nchunks, W.part, W.partw);
      else
        hipLaunchKernelGGL((centroid_partial_kernel<TC, false>), dim3((unsigned)maxch), dim3(256), 0, st, dim, P, w,
                           W.sorted, W.chunk_beg, W.chunk_end, W.nchunks, W.part, W.partw);
    }
    hipLaunchKernelGGL(centroid_final_kernel<TC>, dim3(k), dim3(256), 0, st, k, dim, W.lchunk, W.part, W.partw, out.Z,
                       Zc, W.znorm);
  }
  if (out.snap) {
    const int nblk = snap_nblk(rows, k);
    const int64_t rpb = ceil_div(ceil_div(rows, nblk), SNAP_SUB) * SNAP_SUB;
    const int nblk_eff = (int)ceil_div(rows, rpb);
    TimerScope ts(T_SNAP, st);
    if (stored)
      hipLaunchKernelGGL(snap_select_kernel, dim3(nblk_eff), dim3(256), 0, st, rows, k, rpb, (const float*)W.sacc,
                         W.znorm, W.pnorm, W.cand_d, W.cand_r);
    else
      hipLaunchKernelGGL(snap_topt_kernel<TC>, dim3(nblk_eff), dim3(256), 0, st, rows, dim, k, rpb, P, (const TC*)Zc,
                         W.znorm, W.pnorm, W.cand_d, W.cand_r);
    hipLaunchKernelGGL(snap_merge_kernel, dim3(k), dim3(256), 0, st, nblk_eff, W.cand_d, W.cand_r, W.top_d, W.top_r);
    int32_t* zoff = W.zcnt + ZR_NB + 1;
    hipLaunchKernelGGL(zero_rows_count_kernel, dim3(ZR_NB), dim3(256), 0, st, rows, W.pnorm, W.zcnt);
    hipLaunchKernelGGL(zero_rows_scan_kernel, dim3(1), dim3(64), 0, st, W.zcnt, zoff);
    hipLaunchKernelGGL(zero_rows_write_kernel, dim3(ZR_NB), dim3(256), 0, st, rows, W.pnorm, zoff, W.zrows);
    // FP64: a relative tie window makes the choice independent of rounding order
    // (and equal to the FP64 reference); other precisions compare exactly.
    const double tie_rtol = sizeof(TC) == 8 ? 1e-11 : 0.0;
    hipLaunchKernelGGL(snap_resolve_kernel<TC>, dim3(1), dim3(1024), 0, st, rows, dim, k, P, (const TC*)Zc, W.znorm,
                       W.pnorm, W.top_d, W.top_r, W.cand_d, W.cand_r, nblk_eff, rpb, tie_rtol, W.dmin, W.zrows, zoff,
                       out.snap, out.fallbacks);
  }
  return hipGetLastError();
}

hipError_t launch_kmeans(int64_t rows, int dim, int k, int compute, const void* P, const double* w, const double* Z0,
                         int iters, const KMeansOut& out, void* ws, hipStream_t st, bool lean) {
  if (rows <= 0 || rows > INT32_MAX || dim <= 0 || k <= 0 || k > KM_MAXK || k > rows || iters < 0 || out.Z == nullptr)
    return hipErrorInvalidValue;
  switch (compute) {
    case P_F64: return kmeans_t<double>(compute, rows, dim, k, P, w, Z0, iters, out, ws, lean, st);
    case P_F32: return kmeans_t<float>(compute, rows, dim, k, P, w, Z0, iters, out, ws, lean, st);
    case P_BF16: return kmeans_t<bf16>(compute, rows, dim, k, P, w, Z0, iters, out, ws, lean, st);
    case P_F16: return kmeans_t<f16>(compute, rows, dim, k, P, w, Z0, iters, out, ws, lean, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace cabs
