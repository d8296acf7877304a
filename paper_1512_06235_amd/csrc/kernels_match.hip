// Fused candidate test + distance + two-nearest kernel (a4-a6), Appendix A
// steps 3-4 redesigned for CDNA4.
//
// One wave owns a tile of 32 consecutive queries (in pencil order) and walks
// the contiguous range of b's binned features that covers their bands, 32
// candidates per step:
//   - the candidates' 128-byte descriptor rows are loaded straight into the
//     A operand of v_mfma_i32_32x32x32_i8 (16 bytes per lane per k-step), the
//     negated query rows stay resident as the B operand, so four MFMAs give
//     -q.c for a 32x32 tile with exact int32 accumulation (bytes 0..127 fit
//     int8, 128 * 127^2 < 2^31);
//   - each lane then holds one query and 16 candidates of the tile; it runs
//     the exact band test of eqs. (2)-(3) in FP32 on the candidates' centred
//     coordinates (staged through LDS) and folds in-band distances into a
//     running two-smallest pair of 32-bit keys
//         key = ((||c||^2 - 2 q.c + 2^21) << 10) | (position mod 1024),
//     so one unsigned min and one med3 keep (D1, its position) and D2;
//   - the 32 + 32 lanes of one query merge with one cross-half exchange.
// The key orders equal distances by binned position, not by index in b; when
// the two smallest keys of a chunk share the distance, an exact pass picks the
// lowest index among the tied candidates, so results equal the definition.
#include <cmath>

#include "sfm_internal.h"

namespace sfm {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kWaves = 4;

// Band test of eqs. (2)-(3) on centred FP32 coordinates: |a x + b y + c| <= d
// with (a, b) unit.  The single definition used by every pass.
__device__ __forceinline__ bool in_band(float a, float b, float c, float x, float y, float d) {
  const float e = __builtin_fmaf(a, x, __builtin_fmaf(b, y, c));
  return __builtin_fabsf(e) <= d;
}

// Per-byte negation of four bytes in 0..127 (no borrow crosses a byte).
__device__ __forceinline__ int neg_bytes(uint32_t w) {
  return int((0x80808080u - w) ^ 0x80808080u);
}

__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c) {
  return max(min(a, b), min(max(a, b), c));   // selects v_med3_u32
}

// Largest p in [lo, hi) with pairs[p].blk_off <= item.
__device__ inline int32_t find_pair(const PairDesc* pairs, int32_t lo, int32_t hi, int64_t item) {
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (pairs[mid].blk_off <= item) lo = mid; else hi = mid;
  }
  return lo;
}

// Workgroups are dealt to the 8 XCDs round-robin; renumber them so each XCD
// gets one contiguous run of work items (neighbouring query tiles of one pair
// share candidate rows, and each XCD has its own L2).
__device__ __forceinline__ int32_t xcd_contiguous(int32_t g, int32_t G) {
  const int32_t x = g & 7, k = g >> 3, q = G >> 3, r = G & 7;
  return x * q + min(x, r) + k;
}

// Exact squared L2 of two 128-byte rows with VALU dot products.
__device__ inline int32_t row_dist(const uint8_t* p, const uint8_t* q, int32_t np, int32_t nq) {
  uint32_t dot = 0;
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    const uint4 u = reinterpret_cast<const uint4*>(p)[w];
    const uint4 v = reinterpret_cast<const uint4*>(q)[w];
    dot = __builtin_amdgcn_udot4(u.x, v.x, dot, false);
    dot = __builtin_amdgcn_udot4(u.y, v.y, dot, false);
    dot = __builtin_amdgcn_udot4(u.z, v.z, dot, false);
    dot = __builtin_amdgcn_udot4(u.w, v.w, dot, false);
  }
  return np + nq - 2 * int32_t(dot);
}

template <bool kKeepCounts>
__global__ __launch_bounds__(256) void match_kernel(BatchView v, int32_t blk_begin,
                                                    int32_t blk_count, int32_t pb, int32_t pe) {
  __shared__ __attribute__((aligned(16))) float smX[kWaves][kCandTile];
  __shared__ __attribute__((aligned(16))) float smY[kWaves][kCandTile];
  __shared__ __attribute__((aligned(16))) uint32_t smN[kWaves][kCandTile];

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t item = xcd_contiguous(blockIdx.x, gridDim.x) * kWaves + wave;
  if (item >= blk_count) return;
  const int64_t gblk = int64_t(blk_begin) + item;
  const int32_t p = find_pair(v.pairs, pb, pe, gblk);
  const PairDesc P = v.pairs[p];
  const int32_t blk = int32_t(gblk - P.blk_off);
  const ImageDev A = v.images[P.a];
  const ImageDev B = v.images[P.b];
  const float band = v.geom[p].band32;
  const int col = lane & 31, half = lane >> 5;

  // This lane's query column: line, squared norm and negated descriptor
  // bytes as the MFMA B operand (k-slice 16 * half + 32 * s of the row).
  const int32_t qs = blk * kQueryTile + col;
  const bool qv = qs < P.na;
  QueryRec qr;
  if (qv) {
    qr = v.qrec[P.q_off + qs];
  } else {
    qr.a = qr.b = qr.c = NAN;
    qr.i = 0;
  }
  v4i bq[4];
  int32_t nq = 0;
  if (qv) {
    const uint4* qrow = reinterpret_cast<const uint4*>(A.desc + int64_t(qr.i) * kDescBytes + 16 * half);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const uint4 w = qrow[2 * s];
      bq[s] = v4i{neg_bytes(w.x), neg_bytes(w.y), neg_bytes(w.z), neg_bytes(w.w)};
    }
    nq = A.norm2[qr.i];
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) bq[s] = v4i{0, 0, 0, 0};
  }

  int32_t s_begin = 0, s_end = 0;
  const int2 w = v.blk_win[P.blk_off + blk];
  if (w.x <= w.y) {
    s_begin = v.bin_start[P.bin_off + w.x];
    s_end = v.bin_start[P.bin_off + w.y + 1];
  }

  int32_t d1 = kDistInf, d2 = kDistInf, j1 = -1, cnt = 0;
  unsigned long long total = 0;    // in-band comparisons of this tile (wave-uniform)
  uint32_t ties = 0;
  const CandRec* cand = v.cand + P.c_off;

  for (int32_t c0 = s_begin; c0 < s_end; c0 += kChunk) {
    const int32_t c1 = min(s_end, c0 + kChunk);
    uint32_t k1 = kKeyInf, k2 = kKeyInf;
    for (int32_t t0 = c0; t0 < c1; t0 += kCandTile) {
      const int32_t cp = t0 + col;
      const bool cv = cp < c1;
      CandRec cr;
      v4i ac[4];
      if (cv) {
        cr = cand[cp];
        const uint4* crow = reinterpret_cast<const uint4*>(B.desc + int64_t(cr.j) * kDescBytes + 16 * half);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const uint4 u = crow[2 * s];
          ac[s] = v4i{int(u.x), int(u.y), int(u.z), int(u.w)};
        }
      } else {
        cr.x = cr.y = NAN;
        cr.ncpos = 0;
        cr.j = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s) ac[s] = v4i{0, 0, 0, 0};
      }
      if (half == 0) {
        smX[wave][col] = cr.x;
        smY[wave][col] = cr.y;
        smN[wave][col] = cr.ncpos;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

      v16i acc = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(ac[s], bq[s], acc, 0, 0, 0);

      // Lane (col, half) holds rows 8g + 4*half + e of the tile, e = 0..3.
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int r0 = 8 * g + 4 * half;
        const float4 xs = *reinterpret_cast<const float4*>(&smX[wave][r0]);
        const float4 ys = *reinterpret_cast<const float4*>(&smY[wave][r0]);
        const uint4 ns = *reinterpret_cast<const uint4*>(&smN[wave][r0]);
        const float xv[4] = {xs.x, xs.y, xs.z, xs.w};
        const float yv[4] = {ys.x, ys.y, ys.z, ys.w};
        const uint32_t nv[4] = {ns.x, ns.y, ns.z, ns.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool mem = in_band(qr.a, qr.b, qr.c, xv[e], yv[e], band);
          uint32_t key = nv[e] + (uint32_t(acc[4 * g + e]) << 11);
          key = mem ? key : kKeyInf;
          k2 = umed3(k1, key, k2);
          k1 = min(k1, key);
          total += __builtin_popcountll(__ballot(mem));
          if (kKeepCounts) cnt += mem ? 1 : 0;
        }
      }
      __builtin_amdgcn_wave_barrier();
    }

    // Merge the two halves of each query column.
    {
      const uint32_t p1 = __shfl_xor(k1, 32, 64);
      const uint32_t p2 = __shfl_xor(k2, 32, 64);
      k2 = min(max(k1, p1), min(k2, p2));
      k1 = min(k1, p1);
    }
    int32_t D1c = kDistInf, D2c = kDistInf, j1c = -1;
    if (k1 != kKeyInf) {
      D1c = int32_t(k1 >> kPosBits) - int32_t(kDistBias) + nq;
      const int32_t pos = int32_t(k1 & (kChunk - 1));
      j1c = cand[c0 + ((pos - c0) & (kChunk - 1))].j;
    }
    if (k2 != kKeyInf) D2c = int32_t(k2 >> kPosBits) - int32_t(kDistBias) + nq;

    // Equal smallest distances: choose the lowest index of b exactly.
    const bool tie = k2 != kKeyInf && (k1 >> kPosBits) == (k2 >> kPosBits);
    unsigned long long tmask = __ballot(tie && half == 0);
    while (tmask) {
      const int L = __builtin_ctzll(tmask);
      tmask &= tmask - 1;
      ++ties;
      const float la = __shfl(qr.a, L, 64), lb = __shfl(qr.b, L, 64), lc = __shfl(qr.c, L, 64);
      const int32_t li = __shfl(qr.i, L, 64), lnq = __shfl(nq, L, 64), lD = __shfl(D1c, L, 64);
      const uint8_t* qrow = A.desc + int64_t(li) * kDescBytes;
      int32_t jbest = 0x7FFFFFFF;
      for (int32_t s = c0 + lane; s < c1; s += 64) {
        const CandRec r = cand[s];
        if (!in_band(la, lb, lc, r.x, r.y, band)) continue;
        const int32_t nc = int32_t(r.ncpos >> kPosBits) - int32_t(kDistBias);
        const int32_t D = row_dist(qrow, B.desc + int64_t(r.j) * kDescBytes, lnq, nc);
        if (D == lD) jbest = min(jbest, r.j);
      }
      for (int o = 32; o > 0; o >>= 1) jbest = min(jbest, __shfl_xor(jbest, o, 64));
      if (col == L) j1c = jbest;
    }

    // Fold this chunk's (D1, j1, D2) into the running result.
    if (D1c < d1 || (D1c == d1 && D1c != kDistInf && j1c < j1)) {
      d2 = min(d1, D2c);
      d1 = D1c;
      j1 = j1c;
    } else {
      d2 = min(d2, D1c);
    }
  }

  bool accept;
  if (d2 != kDistInf) {
    accept = int64_t(v.ratio_den) * d1 < int64_t(v.ratio_num) * d2;
  } else {
    accept = d1 != kDistInf && v.accept_single;
  }
  if (kKeepCounts) cnt += __shfl_xor(cnt, 32, 64);
  if (qv && half == 0) {
    QueryResult out;
    out.match = j1;
    out.d1 = d1;
    out.d2 = d2;
    out.flags = (accept ? 1 : 0) | (kKeepCounts ? (cnt << 1) : 0);
    v.res[P.q_off + qr.i] = out;
  }
  const uint32_t nacc = __builtin_popcountll(__ballot(accept && qv && half == 0));
  if (lane == 0) {
    if (total) atomicAdd(&v.counters[p].comparisons, total);
    if (nacc) atomicAdd(&v.counters[p].accepted, nacc);
    if (ties) atomicAdd(&v.counters[p].ties, ties);
  }
}

}  // namespace

hipError_t launch_match(const BatchView& v, int32_t blk_begin, int32_t blk_count, int32_t pb,
                        int32_t pe, hipStream_t st) {
  if (blk_count <= 0) return hipSuccess;
  const int32_t groups = (blk_count + kWaves - 1) / kWaves;
  if (v.keep_counts)
    hipLaunchKernelGGL(match_kernel<true>, dim3(groups), dim3(64 * kWaves), 0, st, v, blk_begin,
                       blk_count, pb, pe);
  else
    hipLaunchKernelGGL(match_kernel<false>, dim3(groups), dim3(64 * kWaves), 0, st, v, blk_begin,
                       blk_count, pb, pe);
  return hipGetLastError();
}

}  // namespace sfm
