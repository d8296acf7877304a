// Grid-based approximate candidate search (Section 6.2.1, eqs. 4-9, and the
// GPU steps 1, 3 and 4 of Appendix A).
//
// b's features are binned once per pair into four grids of 2d x 2d cells,
// shifted by (0,0), (d,0), (0,d) and (d,d).  A query's line is cut by b's
// keypoint box at A and B; K + 1 equidistant points are taken between them
// (K the smallest integer with K d >= |AB|), and each point selects the
// centre-most of the four cells that contain it.  C' is the union of the
// features of the selected cells, made a set with a per-query bitmap in LDS;
// the two nearest of C' by exact squared L2 and the ratio test decide the
// match.  C' approximates the band of eq. (2): it can hold features up to 2d
// (per axis) from a sample point and miss band members near a cell corner.
//
// Every floating-point decision (crossings, sample points, cells, centre
// distances) is IEEE double with no contraction, in a fixed order, so the
// result is reproducible bit for bit by a plain implementation of the same
// steps.
#include <algorithm>
#include <cmath>


#include "sfm_internal.h"

#pragma clang fp contract(off)

namespace sfm {
namespace {

constexpr int kBinThreads = 256;

__device__ __forceinline__ double grid_shift(int g, double d, int axis) {
  return ((g >> axis) & 1) ? d : 0.0;
}

// Cell of (x, y) in grid g of pair P, as an index into its table; -1 outside.
// (The pair record stays in global memory: indexing its per-grid arrays
// with a run-time grid number would otherwise put a copy in scratch.)
__device__ __forceinline__ int64_t cell_of(const GridPair* P, int g, double x, double y) {
  const double two_d = 2.0 * P->d;
  const double sx = grid_shift(g, P->d, 0), sy = grid_shift(g, P->d, 1);
  const int64_t cx = int64_t(floor((x - sx) / two_d)) - P->cx0[g];
  const int64_t cy = int64_t(floor((y - sy) / two_d)) - P->cy0[g];
  if (cx < 0 || cx >= P->ncx[g] || cy < 0 || cy >= P->ncy[g]) return -1;
  return cy * P->ncx[g] + cx;
}

__device__ __forceinline__ int32_t load_count(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One workgroup per (pair, grid): count per cell, scan, scatter.  Features
// of one cell land in any order; C' is a set, so the order never matters.
// The counts live in LDS when the grid has at most v.lds_cells cells, else in
// the HBM cursor array (atomics there are many times slower).
__global__ __launch_bounds__(kBinThreads) void grid_bin_kernel(GridView v) {
  extern __shared__ int32_t lcnt[];
  __shared__ int64_t part[kBinThreads];
  const int32_t p = blockIdx.x >> 2, g = blockIdx.x & 3;
  const GridPair* P = v.pairs + p;
  const ImageDev B = v.images[P->b];
  const int32_t nb = P->nb;
  const int64_t ncell = int64_t(P->ncx[g]) * P->ncy[g];
  int32_t* start = v.cell_start + P->cell_off[g];
  int32_t* items = v.items + P->item_off + int64_t(g) * nb;
  const bool local = ncell <= v.lds_cells;
  int32_t* cur = local ? lcnt : v.cursor + P->cell_off[g];
  const int t = threadIdx.x;
  for (int64_t c = t; c < ncell; c += kBinThreads) cur[c] = 0;
  __syncthreads();
  for (int32_t j = t; j < nb; j += kBinThreads) {
    const int64_t c = cell_of(P, g, double(B.xy[2 * j]), double(B.xy[2 * j + 1]));
    if (c < 0) {
      *v.err = 1;
      continue;
    }
    atomicAdd(&cur[c], 1);
  }
  __syncthreads();
  // Exclusive scan: each thread owns a contiguous run of cells.  (HBM counts
  // are read as device-scope atomics: the adds happened in L2.)
  const int64_t chunk = (ncell + kBinThreads - 1) / kBinThreads;
  const int64_t c0 = std::min<int64_t>(ncell, chunk * t), c1 = std::min<int64_t>(ncell, c0 + chunk);
  int64_t sum = 0;
  for (int64_t c = c0; c < c1; ++c) sum += local ? cur[c] : load_count(&cur[c]);
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < kBinThreads; o <<= 1) {
    const int64_t add = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int64_t run = part[t] - sum;
  for (int64_t c = c0; c < c1; ++c) {
    const int32_t n = local ? cur[c] : load_count(&cur[c]);
    start[c] = int32_t(run);
    if (local)
      cur[c] = int32_t(run);
    else
      __hip_atomic_store(&cur[c], int32_t(run), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    run += n;
  }
  if (t == kBinThreads - 1) start[ncell] = int32_t(part[t]);
  __syncthreads();
  for (int32_t j = t; j < nb; j += kBinThreads) {
    const int64_t c = cell_of(P, g, double(B.xy[2 * j]), double(B.xy[2 * j + 1]));
    if (c < 0) continue;
    items[atomicAdd(&cur[c], 1)] = j;
  }
}

__device__ __forceinline__ unsigned long long wave_min(unsigned long long x) {
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(x, o, 64);
    x = y < x ? y : x;
  }
  return x;
}

// The line of query i of pair pr cut by b's keypoint box: crossings on the
// edges x = x0, x = x1, y = y0, y = y1 in that order; A is the first, B the
// first of those farthest from A.  False without a crossing.
__device__ __forceinline__ bool line_crossings(const GridView& v, const GridPair* P, int32_t pr,
                                               const ImageDev& A, int32_t i, double& xA,
                                               double& yA, double& xB, double& yB) {
  const double xa = double(A.xy[2 * i]), ya = double(A.xy[2 * i + 1]);
  const double* F = v.F + 9 * int64_t(pr);
  const double la = F[0] * xa + F[1] * ya + F[2];
  const double lb = F[3] * xa + F[4] * ya + F[5];
  const double lc = F[6] * xa + F[7] * ya + F[8];
  const double x0 = P->box[0], y0 = P->box[1], x1 = P->box[2], y1 = P->box[3];
  int nh = 0;
  double far = -1.0;
  auto hit = [&](double x, double y) {
    if (nh++ == 0) { xA = x; yA = y; }
    const double dx = x - xA, dy = y - yA;
    const double r = dx * dx + dy * dy;
    if (r > far) { xB = x; yB = y; far = r; }
  };
  if (lb != 0.0) {
    const double ya0 = -(la * x0 + lc) / lb;
    if (y0 <= ya0 && ya0 <= y1) hit(x0, ya0);
    const double ya1 = -(la * x1 + lc) / lb;
    if (y0 <= ya1 && ya1 <= y1) hit(x1, ya1);
  }
  if (la != 0.0) {
    const double xb0 = -(lb * y0 + lc) / la;
    if (x0 <= xb0 && xb0 <= x1) hit(xb0, y0);
    const double xb1 = -(lb * y1 + lc) / la;
    if (x0 <= xb1 && xb1 <= x1) hit(xb1, y1);
  }
  return nh > 0;
}

// Walks the cells of query i of pair pr and calls on_new(j) once for every
// feature j of C' (the bitmap, one bit per feature of b, clear on entry,
// makes C' a set).  Lanes take the sample points k = lane, lane + 64, ...
template <class OnNew>
__device__ __forceinline__ void grid_walk(const GridView& v, const GridPair* P, int32_t pr,
                                          const ImageDev& A, int32_t i, uint32_t* bitmap,
                                          OnNew&& on_new) {
  const int lane = threadIdx.x;
  double xA = 0.0, yA = 0.0, xB = 0.0, yB = 0.0;
  const bool crosses = line_crossings(v, P, pr, A, i, xA, yA, xB, yB);
  if (!crosses || P->nb == 0) return;
  {
    const double dx = xB - xA, dy = yB - yA;
    const double len2 = dx * dx + dy * dy;
    const double d2 = P->d * P->d;
    int64_t K = int64_t(ceil(sqrt(len2) / P->d));
    while (K > 0 && double((K - 1) * (K - 1)) * d2 >= len2) --K;
    while (double(K * K) * d2 < len2) ++K;
    const double two_d = 2.0 * P->d;
    for (int64_t k = lane; k <= K; k += 64) {
      double px = xA, py = yA;
      if (K > 0) {
        const double kd = double(k), rd = double(K - k), Kd = double(K);
        px = (kd * xA + rd * xB) / Kd;
        py = (kd * yA + rd * yB) / Kd;
      }
      // Centre-most of the four cells holding the point (lower grid on ties).
      int gsel = 0;
      double best = INFINITY, bcx = 0.0, bcy = 0.0;
      for (int g = 0; g < 4; ++g) {
        const double sx = grid_shift(g, P->d, 0), sy = grid_shift(g, P->d, 1);
        const double cx = floor((px - sx) / two_d), cy = floor((py - sy) / two_d);
        const double ex = px - (cx * two_d + sx + P->d);
        const double ey = py - (cy * two_d + sy + P->d);
        const double r = ex * ex + ey * ey;
        if (r < best) { best = r; gsel = g; bcx = cx; bcy = cy; }
      }
      const int64_t cx = int64_t(bcx) - P->cx0[gsel], cy = int64_t(bcy) - P->cy0[gsel];
      if (cx < 0 || cx >= P->ncx[gsel] || cy < 0 || cy >= P->ncy[gsel]) continue;
      const int32_t* start = v.cell_start + P->cell_off[gsel];
      const int32_t* items = v.items + P->item_off + int64_t(gsel) * P->nb;
      const int64_t c = cy * P->ncx[gsel] + cx;
      for (int32_t s = start[c], e = start[c + 1]; s < e; ++s) {
        const int32_t j = items[s];
        const uint32_t bit = 1u << (j & 31);
        if (atomicOr(&bitmap[j >> 5], bit) & bit) continue;
        on_new(j);
      }
    }
  }
}

// C' of query i into the LDS list `cand` (count in *ncand).
__device__ __forceinline__ void grid_collect(const GridView& v, const GridPair* P, int32_t pr,
                                             const ImageDev& A, int32_t i, uint32_t* bitmap,
                                             int32_t* cand, int32_t* ncand) {
  grid_walk(v, P, pr, A, i, bitmap, [&](int32_t j) {
    const int32_t slot = atomicAdd(ncand, 1);
    if (slot < kGridMaxCand) cand[slot] = j;
  });
}

// The query's 128 descriptor bytes as 32 words, and its exact squared
// distance to feature j of b: |q|^2 + |b_j|^2 - 2 q.b_j.
__device__ __forceinline__ void query_words(const ImageDev& A, int32_t i, uint32_t q[32]) {
  const uint4* qd = reinterpret_cast<const uint4*>(A.desc + 128 * int64_t(i));
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    const uint4 u = qd[w];
    q[4 * w] = u.x; q[4 * w + 1] = u.y; q[4 * w + 2] = u.z; q[4 * w + 3] = u.w;
  }
}

__device__ __forceinline__ unsigned long long dist_key(const uint32_t q[32], int32_t qn,
                                                       const ImageDev& B, int32_t j) {
  const uint4* bd = reinterpret_cast<const uint4*>(B.desc + 128 * int64_t(j));
  uint32_t dot = 0;
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    const uint4 u = bd[w];
    dot = __builtin_amdgcn_udot4(q[4 * w], u.x, dot, false);
    dot = __builtin_amdgcn_udot4(q[4 * w + 1], u.y, dot, false);
    dot = __builtin_amdgcn_udot4(q[4 * w + 2], u.z, dot, false);
    dot = __builtin_amdgcn_udot4(q[4 * w + 3], u.w, dot, false);
  }
  const int32_t D = qn + B.norm2[j] - 2 * int32_t(dot);
  // Packed keys (D << 32 | j) order by distance, then index.
  return (static_cast<unsigned long long>(uint32_t(D)) << 32) | uint32_t(j);
}

// Branch-free, so the two stay in registers (a conditional store to one of
// the two references made the compiler keep them in scratch).
__device__ __forceinline__ void push_two(unsigned long long key, unsigned long long& b1,
                                         unsigned long long& b2) {
  const bool lt1 = key < b1;
  const unsigned long long n2 = lt1 ? b1 : (key < b2 ? key : b2);
  b1 = lt1 ? key : b1;
  b2 = n2;
}

// Wave-wide two nearest of the lanes' pairs and the ratio test; lane 0
// writes the query's result and adds to its pair's counters.
__device__ __forceinline__ void grid_finish(const GridView& v, int64_t q_off, int32_t pr,
                                            int32_t i, unsigned long long b1,
                                            unsigned long long b2, int32_t n) {
  const unsigned long long m1 = wave_min(b1);
  const unsigned long long m2 = wave_min(b1 == m1 ? b2 : b1);
  if (threadIdx.x == 0) {
    QueryResult r;
    r.match = n > 0 ? int32_t(uint32_t(m1)) : -1;
    r.d1 = n > 0 ? int32_t(m1 >> 32) : kDistInf;
    r.d2 = n > 1 ? int32_t(m2 >> 32) : kDistInf;
    bool accept = false;
    if (n >= 2)
      accept = int64_t(v.ratio_den) * r.d1 < int64_t(v.ratio_num) * r.d2;
    else if (n == 1)
      accept = v.accept_single != 0;
    r.flags = (accept ? 1 : 0) | (v.keep_counts ? (n << 1) : 0);
    v.res[q_off + i] = r;
    atomicAdd(&v.counters[pr].comparisons, static_cast<unsigned long long>(n));
    if (accept) atomicAdd(&v.counters[pr].accepted, 1u);
  }
}

// Two nearest of the listed C' and the ratio test for query i of pair pr.
__device__ __forceinline__ void grid_decide(const GridView& v, int64_t q_off, int32_t pr,
                                            const ImageDev& A, const ImageDev& B, int32_t i,
                                            const int32_t* cand, int32_t n) {
  uint32_t q[32];
  query_words(A, i, q);
  const int32_t qn = A.norm2[i];
  unsigned long long b1 = ~0ull, b2 = ~0ull;
  for (int32_t s = threadIdx.x; s < n; s += 64) push_two(dist_key(q, qn, B, cand[s]), b1, b2);
  grid_finish(v, q_off, pr, i, b1, b2, n);
}

// One wave per workgroup, taking up to kGridQueriesPerBlock consecutive
// queries of one pair (an entry of the host's block table) one after the
// other.  LDS: a bitmap with one bit per feature of the largest b of the
// call, then kGridMaxCand candidate slots and their count.  (Computing each
// distance in the walk, by the lane that finds the candidate, needs no list
// but measured 10% slower: the walk's lanes diverge, the list pass does not.)
// The occupancy hint (6 waves per SIMD) holds it to 68 VGPRs without spills;
// with the 1,024-slot list that keeps more queries in flight (22.2 -> 19.9 ms
// on the 500-pair batch).
__global__ __launch_bounds__(64, 6) void grid_query_kernel(GridView v) {
  extern __shared__ uint32_t lds[];
  const int2 blk = v.blocks[blockIdx.x];
  const int32_t pr = blk.x;
  const GridPair* P = v.pairs + pr;
  const ImageDev A = v.images[P->a], B = v.images[P->b];
  const int64_t q_off = P->q_off;
  uint32_t* bitmap = lds;
  int32_t* cand = reinterpret_cast<int32_t*>(lds + v.bitmap_words);
  int32_t* ncand = cand + kGridMaxCand;
  const int32_t words = (P->nb + 31) >> 5;
  const int32_t i_end = min(P->na, blk.y + kGridQueriesPerBlock);
  for (int32_t i = blk.y; i < i_end; ++i) {
    for (int32_t w = threadIdx.x; w < words; w += 64) bitmap[w] = 0;
    if (threadIdx.x == 0) *ncand = 0;
    __syncthreads();
    grid_collect(v, P, pr, A, i, bitmap, cand, ncand);
    __syncthreads();
    int32_t n = *ncand;
    if (n > kGridMaxCand) {
      if (threadIdx.x == 0) *v.err = 1;
      n = kGridMaxCand;
    }
    grid_decide(v, q_off, pr, A, B, i, cand, n);
    __syncthreads();   // the next query clears the bitmap and the list
  }
}

// ---------------------------------------------------------------------------
// Query grouping: queries whose lines cross b's box within tol of the
// previous line's crossings (in sorted order) share the first line's C'.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int32_t pair_of(const int32_t* seg_begin, int32_t n_pairs, int32_t t) {
  int32_t lo = 0, hi = n_pairs - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (seg_begin[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Unsigned key with the order of the double (-0 first made +0).
__device__ __forceinline__ unsigned long long sortable(double x) {
  x = x + 0.0;
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ __launch_bounds__(256) void grid_cross_kernel(GridView v, GroupView g) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.n) return;
  const int32_t pr = pair_of(g.seg_begin, v.n_pairs, t);
  const GridPair* P = v.pairs + pr;
  const ImageDev A = v.images[P->a];
  double xA = 0.0, yA = 0.0, xB = 0.0, yB = 0.0;
  const bool crosses = line_crossings(v, P, pr, A, int32_t(t - P->q_off), xA, yA, xB, yB);
  g.cross[4 * int64_t(t)] = xA;
  g.cross[4 * int64_t(t) + 1] = yA;
  g.cross[4 * int64_t(t) + 2] = xB;
  g.cross[4 * int64_t(t) + 3] = yB;
  g.hit[t] = crosses ? 1 : 0;
  g.val[0][t] = t;
}

// ---------------------------------------------------------------------------
// Least-significant-digit radix sort of the positions by (pair, A.x, A.y,
// B.x, B.y), the crossing components as 64-bit order-preserving keys (lines
// without a crossing sort last) and the pair index as the most significant
// key: 8-bit digits, least significant first, each pass a stable counting
// sort, so equal keys keep position order.  A pass counts the digits of each
// 2048-position tile, scans the counts (digit-major, so each digit's tiles
// follow each other), then sorts every tile by the digit in LDS (eight
// stable one-bit splits) and scatters it.
// ---------------------------------------------------------------------------
constexpr int kSortThreads = 256;
constexpr int kSortPer = 8;                              // positions per thread
constexpr int kSortTile = kSortThreads * kSortPer;       // positions per tile
constexpr int kRadix = 256;

// Digit `byte` of the sort key `comp` (0..3: crossing component, 4: pair) of
// original position s.
__device__ __forceinline__ uint32_t sort_digit(const GridView& v, const GroupView& g, int32_t s,
                                               int comp, int byte) {
  unsigned long long key;
  if (comp < 4)
    key = g.hit[s] ? sortable(g.cross[4 * int64_t(s) + comp]) : ~0ull;
  else
    key = static_cast<unsigned long long>(pair_of(g.seg_begin, v.n_pairs, s));
  return uint32_t(key >> (8 * byte)) & (kRadix - 1);
}

// counts[d * ntiles + tile]: positions of the tile with digit d.
__global__ __launch_bounds__(kSortThreads) void sort_count_kernel(GridView v, GroupView g,
                                                                  const int32_t* val, int comp,
                                                                  int byte, int32_t* counts,
                                                                  int32_t ntiles) {
  __shared__ int32_t h[kRadix];
  const int t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const int32_t base = blockIdx.x * kSortTile;
  for (int k = 0; k < kSortPer; ++k) {
    const int32_t i = base + k * kSortThreads + t;
    if (i < g.n) atomicAdd(&h[sort_digit(v, g, val[i], comp, byte)], 1);
  }
  __syncthreads();
  counts[int64_t(t) * ntiles + blockIdx.x] = h[t];
}

// Exclusive scan of one value per thread over the block; returns the total.
__device__ __forceinline__ int32_t block_excl_scan(int32_t x, int32_t& total, int32_t* wsum) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int32_t inc = x;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int32_t before = 0;
  total = 0;
  for (int w = 0; w < kSortThreads / 64; ++w) {
    before += w < wv ? wsum[w] : 0;
    total += wsum[w];
  }
  __syncthreads();
  return before + inc - x;
}

// One pass: the tile sorted stably by the digit, then every position written
// at (scanned count of its digit and tile) + (its rank among the tile's
// positions with that digit).
__global__ __launch_bounds__(kSortThreads) void sort_scatter_kernel(
    GridView v, GroupView g, const int32_t* val_in, int32_t* val_out, int comp, int byte,
    const int32_t* offsets, int32_t ntiles) {
  __shared__ int32_t sval[kSortTile];
  __shared__ uint8_t sdig[kSortTile];
  __shared__ int32_t dstart[kRadix];
  __shared__ int32_t wsum[kSortThreads / 64];
  const int t = threadIdx.x;
  const int32_t base = blockIdx.x * kSortTile;
  const int32_t cnt = min(kSortTile, g.n - base);
  // Thread t holds tile positions kSortPer t .. kSortPer t + kSortPer - 1.
  // Past the end: digit 255 and last in order, so they stay behind every
  // real position and are never written.
  int32_t vals[kSortPer];
  uint32_t dig[kSortPer];
#pragma unroll
  for (int k = 0; k < kSortPer; ++k) {
    const int32_t i = kSortPer * t + k;
    vals[k] = i < cnt ? val_in[base + i] : 0;
    dig[k] = i < cnt ? sort_digit(v, g, vals[k], comp, byte) : kRadix - 1;
  }
  for (int bit = 0; bit < 8; ++bit) {
    int32_t zeros = 0;
#pragma unroll
    for (int k = 0; k < kSortPer; ++k) zeros += ((dig[k] >> bit) & 1) ? 0 : 1;
    int32_t total_zeros;
    int32_t zb = block_excl_scan(zeros, total_zeros, wsum);   // zeros before this thread
    const int32_t first = kSortPer * t;
#pragma unroll
    for (int k = 0; k < kSortPer; ++k) {
      const bool one = (dig[k] >> bit) & 1;
      const int32_t pos = one ? total_zeros + (first + k - zb) : zb;
      zb += one ? 0 : 1;
      sval[pos] = vals[k];
      sdig[pos] = uint8_t(dig[k]);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSortPer; ++k) {
      vals[k] = sval[kSortPer * t + k];
      dig[k] = sdig[kSortPer * t + k];
    }
    __syncthreads();
  }
  // First tile position of each digit among the real positions.
  dstart[t] = 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSortPer; ++k)
    if (kSortPer * t + k < cnt) atomicAdd(&dstart[dig[k]], 1);
  __syncthreads();
  int32_t total;
  const int32_t start = block_excl_scan(dstart[t], total, wsum);
  dstart[t] = start;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSortPer; ++k) {
    const int32_t i = kSortPer * t + k;
    if (i < cnt)
      val_out[offsets[int64_t(dig[k]) * ntiles + blockIdx.x] + (i - dstart[dig[k]])] = vals[k];
  }
}

__global__ __launch_bounds__(256) void copy_i32_kernel(const int32_t* src, int32_t* dst,
                                                       int32_t n) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[t];
}

__global__ __launch_bounds__(256) void grid_stencil_kernel(GridView v, GroupView g) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.n) return;
  const int32_t pr = pair_of(g.seg_begin, v.n_pairs, t);
  int32_t start = 1;
  if (t > g.seg_begin[pr]) {
    const int32_t s = g.val[0][t], q = g.val[0][t - 1];
    if (g.hit[s] && g.hit[q]) {
      const double* a = g.cross + 4 * int64_t(s);
      const double* b = g.cross + 4 * int64_t(q);
      const double dA = (a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]);
      const double dB = (a[2] - b[2]) * (a[2] - b[2]) + (a[3] - b[3]) * (a[3] - b[3]);
      start = (dA > g.tol2 || dB > g.tol2) ? 1 : 0;
    }
  }
  g.stencil[t] = start;
}

// The same decision against the group's first line: a walk along each
// pair's sorted queries.  One wave per pair loads 64 positions at a time into
// LDS; its first lane then walks them in order, carrying the leader.
__global__ __launch_bounds__(64) void grid_stencil_leader_kernel(GridView v, GroupView g) {
  __shared__ double cx[64][4];
  __shared__ int32_t hs[64], out[64];
  const int32_t pr = blockIdx.x;
  const int lane = threadIdx.x;
  const int32_t* order = g.val[0];
  const int32_t begin = g.seg_begin[pr], end = g.seg_end[pr];
  bool have_lead = false, lead_hit = false;
  double L0 = 0.0, L1 = 0.0, L2 = 0.0, L3 = 0.0;
  for (int32_t base = begin; base < end; base += 64) {
    const int32_t t = base + lane;
    if (t < end) {
      const int32_t s = order[t];
      hs[lane] = g.hit[s];
#pragma unroll
      for (int c = 0; c < 4; ++c) cx[lane][c] = g.cross[4 * int64_t(s) + c];
    }
    __syncthreads();
    if (lane == 0) {
      const int32_t cnt = min(64, end - base);
      for (int32_t k = 0; k < cnt; ++k) {
        int32_t start = 1;
        if (have_lead && hs[k] && lead_hit) {
          const double dA = (cx[k][0] - L0) * (cx[k][0] - L0) + (cx[k][1] - L1) * (cx[k][1] - L1);
          const double dB = (cx[k][2] - L2) * (cx[k][2] - L2) + (cx[k][3] - L3) * (cx[k][3] - L3);
          start = (dA > g.tol2 || dB > g.tol2) ? 1 : 0;
        }
        if (start) {
          have_lead = true;
          lead_hit = hs[k] != 0;
          L0 = cx[k][0]; L1 = cx[k][1]; L2 = cx[k][2]; L3 = cx[k][3];
        }
        out[k] = start;
      }
    }
    __syncthreads();
    if (t < end) g.stencil[t] = out[lane];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void grid_gstart_kernel(GroupView g) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < g.n && g.stencil[t]) g.gstart[g.gid[t] - 1] = t;
}

__global__ __launch_bounds__(64) void grid_group_query_kernel(GridView v, GroupView g,
                                                              int32_t n_groups) {
  extern __shared__ uint32_t lds[];
  const int32_t gi = blockIdx.x;
  const int32_t t0 = g.gstart[gi], t1 = gi + 1 < n_groups ? g.gstart[gi + 1] : g.n;
  const int32_t pr = pair_of(g.seg_begin, v.n_pairs, t0);
  const GridPair* P = v.pairs + pr;
  const ImageDev A = v.images[P->a], B = v.images[P->b];
  const int64_t q_off = P->q_off;
  const int32_t* order = g.val[0];
  uint32_t* bitmap = lds;
  int32_t* cand = reinterpret_cast<int32_t*>(lds + v.bitmap_words);
  int32_t* ncand = cand + kGridMaxCand;
  const int32_t words = (P->nb + 31) >> 5;
  for (int32_t w = threadIdx.x; w < words; w += 64) bitmap[w] = 0;
  if (threadIdx.x == 0) *ncand = 0;
  __syncthreads();
  grid_collect(v, P, pr, A, int32_t(order[t0] - q_off), bitmap, cand, ncand);
  __syncthreads();
  int32_t n = *ncand;
  if (n > kGridMaxCand) {
    if (threadIdx.x == 0) *v.err = 1;
    n = kGridMaxCand;
  }
  for (int32_t t = t0; t < t1; ++t) grid_decide(v, q_off, pr, A, B, int32_t(order[t] - q_off), cand, n);
}

int32_t blocks256(int32_t n) { return (n + 255) / 256; }

}  // namespace

// Radix-sort tile counts, then the scan's block sums (reused by the stencil
// scan).
static int32_t sort_tiles(int32_t n) { return (n + kSortTile - 1) / kSortTile; }

hipError_t grid_group_temp_bytes(int32_t n, int32_t n_pairs, size_t* bytes) {
  (void)n_pairs;
  const int64_t ncount = int64_t(kRadix) * sort_tiles(n);
  if (ncount > scan_limit() || int64_t(n) > scan_limit()) return hipErrorInvalidValue;
  *bytes = sizeof(int32_t) * size_t(ncount) + std::max(scan_temp_bytes(ncount), scan_temp_bytes(n));
  return hipSuccess;
}

hipError_t launch_grid_group_prepare(const GridView& v, const GroupView& g, hipStream_t st) {
  if (g.n <= 0) return hipSuccess;
  const int32_t ntiles = sort_tiles(g.n);
  const int64_t ncount = int64_t(kRadix) * ntiles;
  int32_t* counts = static_cast<int32_t*>(g.temp);
  int32_t* sums = counts + ncount;
  size_t need = 0;
  hipError_t e = grid_group_temp_bytes(g.n, v.n_pairs, &need);
  if (e != hipSuccess) return e;
  if (g.temp_bytes < need) return hipErrorInvalidValue;
  hipLaunchKernelGGL(grid_cross_kernel, dim3(blocks256(g.n)), dim3(256), 0, st, v, g);
  // Passes: every byte of components 3, 2, 1, 0, then the pair index's bytes.
  int pair_bytes = 0;
  while (pair_bytes < 4 && (int64_t(1) << (8 * pair_bytes)) < int64_t(v.n_pairs)) ++pair_bytes;
  int cur = 0;
  for (int comp = 3; comp >= -1; --comp) {
    const int key = comp >= 0 ? comp : 4;
    const int nbytes = comp >= 0 ? 8 : pair_bytes;
    for (int byte = 0; byte < nbytes; ++byte) {
      hipLaunchKernelGGL(sort_count_kernel, dim3(ntiles), dim3(kSortThreads), 0, st, v, g,
                         g.val[cur], key, byte, counts, ntiles);
      e = launch_scan(counts, counts, ncount, false, sums, nullptr, st);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(sort_scatter_kernel, dim3(ntiles), dim3(kSortThreads), 0, st, v, g,
                         g.val[cur], g.val[1 - cur], key, byte, counts, ntiles);
      cur = 1 - cur;
    }
  }
  if (cur != 0)
    hipLaunchKernelGGL(copy_i32_kernel, dim3(blocks256(g.n)), dim3(256), 0, st, g.val[1],
                       g.val[0], g.n);
  if (g.to_leader)
    hipLaunchKernelGGL(grid_stencil_leader_kernel, dim3(v.n_pairs), dim3(64), 0, st, v, g);
  else
    hipLaunchKernelGGL(grid_stencil_kernel, dim3(blocks256(g.n)), dim3(256), 0, st, v, g);
  e = launch_scan(g.stencil, g.gid, g.n, true, sums, nullptr, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(grid_gstart_kernel, dim3(blocks256(g.n)), dim3(256), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_grid_groups(const GridView& v, const GroupView& g, int32_t n_groups,
                              hipStream_t st) {
  if (n_groups <= 0) return hipSuccess;
  const size_t lds = sizeof(uint32_t) * (size_t(v.bitmap_words) + kGridMaxCand + 1);
  hipLaunchKernelGGL(grid_group_query_kernel, dim3(uint32_t(n_groups)), dim3(64), lds, st, v, g,
                     n_groups);
  return hipGetLastError();
}

hipError_t launch_grid(const GridView& v, int64_t n_blocks, hipStream_t st) {
  if (v.n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(grid_bin_kernel, dim3(4 * v.n_pairs), dim3(kBinThreads),
                     sizeof(int32_t) * size_t(v.lds_cells), st, v);
  if (n_blocks > 0) {
    const size_t lds = sizeof(uint32_t) * (size_t(v.bitmap_words) + kGridMaxCand + 1);
    hipLaunchKernelGGL(grid_query_kernel, dim3(uint32_t(n_blocks)), dim3(64), lds, st, v);
  }
  return hipGetLastError();
}

}  // namespace sfm
