// Ordered emission of accepted matches (a7).
//
// Per pair: a prefix over pairs gives each pair's first output row; then one
// workgroup per chunk of a pair's queries compacts its accepted queries in
// ascending query index with a ballot + mbcnt prefix inside each wave and a
// scan over waves.
#include <algorithm>

#include "sfm_internal.h"

namespace sfm {
namespace {

constexpr int kEmitThreads = 1024;

// offset[pb + k + 1] = offset[pb] + sum of accepted over pairs pb..pb+k.
__global__ __launch_bounds__(1024) void scan_pairs_kernel(BatchView v, int32_t pb, int32_t pc,
                                                          int64_t* offset, int64_t* n_cmp,
                                                          int64_t* n_bl) {
  __shared__ long long wtot[16];
  __shared__ long long carry;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (t == 0) {
    if (pb == 0) offset[0] = 0;
    carry = offset[pb];
  }
  __syncthreads();
  for (int32_t base = 0; base < pc; base += blockDim.x) {
    const int32_t k = base + t;
    long long x = k < pc ? (long long)v.counters[pb + k].accepted : 0;
    if (k < pc && n_cmp) n_cmp[pb + k] = (long long)v.counters[pb + k].comparisons;
    if (k < pc && n_bl) n_bl[pb + k] = (long long)v.counters[pb + k].borderline;
    for (int o = 1; o < 64; o <<= 1) {
      const long long y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wtot[wv] = x;
    __syncthreads();
    long long before = carry;
    for (int w = 0; w < wv; ++w) before += wtot[w];
    if (k < pc) offset[pb + k + 1] = before + x;
    __syncthreads();
    if (t == int(blockDim.x) - 1) carry = before + x;
    __syncthreads();
  }
}

// One workgroup per chunk of kEmitChunk consecutive queries of a pair (the
// last chunk of a pair takes whatever remains, in rounds of kEmitChunk).  A
// round covers kEmitPer slices of kEmitThreads consecutive queries, whose
// results are read together with coalesced loads (thread t reads query t of
// every slice).  Ranks come from a ballot + mbcnt inside each wave and one
// scan over the (slice, wave) counts of the round; the accepted queries of
// the pair's earlier chunks are counted first from their flags, so the
// chunks of a large pair are emitted side by side.  With `fused` (batches of
// at most kEmitThreads pairs) the workgroup also sums the accepted queries of
// the batch's earlier pairs for its first row, and the pair's first chunk
// writes its offset and counts, so no separate scan over pairs runs first.
constexpr int kEmitPer = 8;
constexpr int kEmitWaves = kEmitThreads / 64;
constexpr int32_t kEmitChunk = kEmitThreads * kEmitPer;

__global__ __launch_bounds__(kEmitThreads) void emit_kernel(BatchView v, int32_t pb, int32_t fused,
                                                            int64_t* offset, int64_t* n_cmp,
                                                            int64_t* n_bl, int32_t* oq,
                                                            int32_t* om, int32_t* od1,
                                                            int32_t* od2, int32_t* am,
                                                            int32_t* ad1, int32_t* ad2,
                                                            int32_t* ac) {
  __shared__ int32_t cnt[kEmitPer * kEmitWaves];   // accepted per (slice, wave), then prefix
  __shared__ int32_t run;
  __shared__ long long wtot[kEmitWaves];
  const int32_t p = pb + blockIdx.x;
  const PairDesc P = v.pairs[p];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int64_t out0;
  if (fused) {
    // Rows of the batch's pairs before this one (p - pb < kEmitThreads).
    long long a = t < p - pb ? (long long)v.counters[pb + t].accepted : 0;
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    if (lane == 0) wtot[wv] = a;
    __syncthreads();
    long long sum = 0;
    for (int w = 0; w < kEmitWaves; ++w) sum += wtot[w];
    out0 = (pb == 0 ? 0 : offset[pb]) + sum;   // offset[pb] comes from an earlier launch
    if (blockIdx.y == 0 && t == 0) {
      if (p == 0) offset[0] = 0;
      offset[p + 1] = out0 + (long long)v.counters[p].accepted;
      if (n_cmp) n_cmp[p] = (long long)v.counters[p].comparisons;
      if (n_bl) n_bl[p] = (long long)v.counters[p].borderline;
    }
  } else {
    out0 = offset[p];
  }
  const int32_t first = int32_t(blockIdx.y) * kEmitChunk;
  if (first >= P.na) return;
  const int32_t last = blockIdx.y + 1 < gridDim.y ? min(P.na, first + kEmitChunk) : P.na;
  const QueryResult* res = v.res + P.q_off;
  // Accepted queries of the chunks before this one.
  int32_t before = 0;
#pragma unroll 8
  for (int32_t i = t; i < first; i += kEmitThreads) before += res[i].flags & 1;
  for (int o = 32; o > 0; o >>= 1) before += __shfl_xor(before, o, 64);
  if (lane == 0) cnt[wv] = before;
  __syncthreads();
  if (t == 0) {
    int32_t r = 0;
    for (int w = 0; w < kEmitWaves; ++w) r += cnt[w];
    run = r;
  }
  __syncthreads();
  for (int32_t base = first; base < last; base += kEmitChunk) {
    const int32_t rbase = run;   // rows before this round (read before its first barrier)
    QueryResult r[kEmitPer];
#pragma unroll
    for (int k = 0; k < kEmitPer; ++k) {
      const int32_t i = base + k * kEmitThreads + t;
      if (i < last) {
        r[k] = res[i];
      } else {
        r[k].match = -1; r[k].d1 = r[k].d2 = kDistInf; r[k].flags = 0;
      }
    }
    // The match kernel leaves the binned position of the match; only rows
    // that are written need its index in b.
#pragma unroll
    for (int k = 0; k < kEmitPer; ++k)
      if (v.cand_j && r[k].match >= 0 && (am || (r[k].flags & 1)))
        r[k].match = v.cand_j[P.c_off + r[k].match];
    int32_t pre[kEmitPer];
#pragma unroll
    for (int k = 0; k < kEmitPer; ++k) {
      const int32_t i = base + k * kEmitThreads + t;
      if (am && i < last) {
        am[P.q_off + i] = r[k].match;
        ad1[P.q_off + i] = r[k].d1;
        ad2[P.q_off + i] = r[k].d2;
        ac[P.q_off + i] = r[k].flags >> 1;
      }
      const unsigned long long m = __ballot((r[k].flags & 1) != 0);
      pre[k] = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32),
                                         __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0));
      if (lane == 0) cnt[k * kEmitWaves + wv] = __builtin_popcountll(m);
    }
    __syncthreads();
    // Exclusive scan of the kEmitPer * kEmitWaves counts in (slice, wave)
    // order by the first wave, two entries per lane.
    if (wv == 0) {
      static_assert(kEmitPer * kEmitWaves == 128, "two counts per lane");
      const int32_t c0 = cnt[2 * lane], c1 = cnt[2 * lane + 1];
      int32_t x = c0 + c1;
      for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      const int32_t ex = x - c0 - c1;
      cnt[2 * lane] = ex;
      cnt[2 * lane + 1] = ex + c0;
      if (lane == 63) run = rbase + x;   // every thread has read rbase already
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kEmitPer; ++k) {
      if (r[k].flags & 1) {
        const int64_t row = out0 + rbase + cnt[k * kEmitWaves + wv] + pre[k];
        const int32_t i = base + k * kEmitThreads + t;
        oq[row] = i;
        om[row] = r[k].match;
        od1[row] = r[k].d1;
        od2[row] = r[k].d2;
      }
    }
    __syncthreads();   // the next round rewrites cnt
  }
}

}  // namespace

hipError_t launch_emit(const BatchView& v, int32_t pb, int32_t pc, int64_t* offset, int32_t* oq,
                       int32_t* om, int32_t* od1, int32_t* od2, int64_t* n_cmp, int64_t* n_bl,
                       int32_t* am, int32_t* ad1, int32_t* ad2, int32_t* ac, hipStream_t st) {
  if (pc <= 0) return hipSuccess;
  const int32_t fused = pc <= kEmitThreads ? 1 : 0;
  if (!fused)
    hipLaunchKernelGGL(scan_pairs_kernel, dim3(1), dim3(1024), 0, st, v, pb, pc, offset, n_cmp,
                       n_bl);
  const uint32_t chunks = uint32_t(std::max(1, (v.max_na + kEmitChunk - 1) / kEmitChunk));
  hipLaunchKernelGGL(emit_kernel, dim3(pc, chunks), dim3(kEmitThreads), 0, st, v, pb, fused,
                     offset, n_cmp, n_bl, oq, om, od1, od2, am, ad1, ad2, ac);
  return hipGetLastError();
}

}  // namespace sfm
