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
// Loads are software-pipelined: the binned record of tile t+2 and the
// descriptor rows of tile t+1 are in flight while tile t is computed.
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

// Global-address-space views: loads through them compile to global_load_*,
// which only count against vmcnt (flat loads would also hold up LDS waits).
typedef unsigned int nv4u __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) nv4u g_nv4u;
typedef const __attribute__((address_space(1))) int32_t g_i32;

__device__ __forceinline__ nv4u gload16(const void* p) { return *(g_nv4u*)p; }

// Raw binned record {x, y, ncpos, j} of position min(cp, c1 - 1); the caller
// masks positions >= c1 when it stages the record (c1 > 0 is guaranteed).
__device__ __forceinline__ nv4u load_rec(const CandRec* cand, int32_t cp, int32_t c1) {
  return gload16(cand + min(cp, c1 - 1));
}

// Per-wave LDS: two stages of 32 candidate rows and their metadata.  A row is
// stored as eight 16-byte chunks with chunk c of row r at slot c ^ (r & 7), so
// that both the coalesced stores (eight lanes per row) and the MFMA operand
// reads (one row per lane) hit all 32 banks without conflicts.
struct WaveLds {
  uint8_t rows[2][kCandTile * kDescBytes];
  float x[2][kCandTile];
  float y[2][kCandTile];
  uint32_t nc[2][kCandTile];
  int32_t jt[2][8][4];       // row index of candidate 8k + m at jt[m][k]
};

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stage record r of position t0 + col into metadata slot st.  Both halves
// hold the same 32 records and store identical values (no divergent branch).
// Positions past the range get a NaN coordinate: no band test passes.
__device__ __forceinline__ void stage_meta(WaveLds& L, int st, const nv4u& r, int32_t t0,
                                           int32_t c1, int col) {
  L.x[st][col] = t0 + col < c1 ? __uint_as_float(r.x) : NAN;
  L.y[st][col] = __uint_as_float(r.y);
  L.nc[st][col] = r.z;
  L.jt[st][col & 7][col >> 3] = int32_t(r.w);
}

// Coalesced loads of the 32 rows named in slot st: lane l fetches 16-byte
// chunk (l & 7) of row 8k + (l >> 3), k = 0..3, so eight lanes read one
// contiguous 128-byte row.
__device__ __forceinline__ void load_rows_coalesced(const WaveLds& L, int st,
                                                    const uint8_t* desc, int lane, nv4u (&rw)[4]) {
  const int4 j = *reinterpret_cast<const int4*>(&L.jt[st][lane >> 3][0]);
  const int32_t jj[4] = {j.x, j.y, j.z, j.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) rw[k] = gload16(desc + int64_t(jj[k]) * kDescBytes + 16 * (lane & 7));
}

__device__ __forceinline__ void store_rows(WaveLds& L, int st, int lane, const nv4u (&rw)[4]) {
  const int m = lane >> 3, c = lane & 7;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    *reinterpret_cast<nv4u*>(&L.rows[st][(8 * k + m) * kDescBytes + ((c ^ (m & 7)) << 4)]) = rw[k];
}

// The MFMA A operand: row (lane & 31), k-slice 16 * half + 32 * s = chunk 2s + half.
__device__ __forceinline__ void read_a(const WaveLds& L, int st, int lane, v4i (&a)[4]) {
  const int r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int s = 0; s < 4; ++s)
    a[s] = *reinterpret_cast<const v4i*>(&L.rows[st][r * kDescBytes + (((2 * s + h) ^ (r & 7)) << 4)]);
}

// tile_compute: the four MFMAs on this step's rows ac, then this lane's 16
// results folded into the running two smallest keys (k1, k2), with the
// candidates' coordinates and keys read from metadata slot st.
template <bool kKeepCounts>
__device__ __forceinline__ void tile_compute(const v4i (&ac)[4], const v4i (&bq)[4],
                                             const QueryRec& qr, float band, const WaveLds& L,
                                             int st, int half, uint32_t& k1, uint32_t& k2,
                                             int32_t& cnt) {
  const float* smX = L.x[st];
  const float* smY = L.y[st];
  const uint32_t* smN = L.nc[st];
  v16i acc = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(ac[s], bq[s], acc, 0, 0, 0);

  // Lane (col, half) holds rows 8g + 4*half + e of the tile, e = 0..3.
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int r0 = 8 * g + 4 * half;
    const float4 xs = *reinterpret_cast<const float4*>(&smX[r0]);
    const float4 ys = *reinterpret_cast<const float4*>(&smY[r0]);
    const uint4 ns = *reinterpret_cast<const uint4*>(&smN[r0]);
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
      cnt += mem ? 1 : 0;   // per lane, in VALU: no VALU -> SALU hand-off per slot
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// One query tile: its 32 queries against the candidate range [s_begin, s_end).
template <bool kKeepCounts>
__device__ __forceinline__ void match_tile(const BatchView& v, const PairDesc& P, int32_t p,
                                           const ImageDev& A, const ImageDev& B, float band,
                                           int32_t blk, int32_t s_begin, int32_t s_end,
                                           WaveLds& L, int lane) {
  const int col = lane & 31, half = lane >> 5;

  // This lane's query column: line, squared norm and negated descriptor
  // bytes as the MFMA B operand.
  const int32_t qs = blk * kQueryTile + col;
  const bool qv = qs < P.na;
  QueryRec qr;
  if (qv) {
    const nv4u u = gload16(v.qrec + P.q_off + qs);
    qr.a = __uint_as_float(u.x);
    qr.b = __uint_as_float(u.y);
    qr.c = __uint_as_float(u.z);
    qr.i = int32_t(u.w);
  } else {
    qr.a = qr.b = qr.c = NAN;
    qr.i = 0;
  }
  const CandRec* cand = v.cand + P.c_off;
  // The first candidate record goes out together with the query loads.
  nv4u rc = {0u, 0u, 0u, 0u};
  if (s_end > s_begin) rc = load_rec(cand, s_begin + col, s_end);
  v4i bq[4];
  int32_t nq = 0;
  {
    // Padding columns (qv false) read query row 0; their line is NaN.
    const uint8_t* qrow = A.desc + int64_t(qr.i) * kDescBytes + 16 * half;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const nv4u u = gload16(qrow + 32 * s);
      bq[s] = v4i{neg_bytes(u.x), neg_bytes(u.y), neg_bytes(u.z), neg_bytes(u.w)};
    }
    nq = ((g_i32*)A.norm2)[qr.i];
  }

  int32_t d1 = kDistInf, d2 = kDistInf, j1 = -1, cnt = 0;
  uint32_t ties = 0;

  for (int32_t c0 = s_begin; c0 < s_end; c0 += kChunk) {
    const int32_t c1 = min(s_end, c0 + kChunk);
    uint32_t k1 = kKeyInf, k2 = kKeyInf;
    if (c0 != s_begin) rc = load_rec(cand, c0 + col, c1);
    // Step u works on positions c0 + 32u .. +31 from LDS slot u & 1.  While it
    // computes, the rows of step u+1 and the record of step u+2 are in flight;
    // rows are addressed from LDS and always read as whole 128-byte rows, eight
    // lanes per row.
    stage_meta(L, 0, rc, c0, c1, col);
    wave_sync_lds();
    nv4u rw[4];
    load_rows_coalesced(L, 0, B.desc, lane, rw);
    rc = load_rec(cand, c0 + kCandTile + col, c1);
    int st = 0;
    for (int32_t t0 = c0; t0 < c1; t0 += kCandTile, st ^= 1) {
      store_rows(L, st, lane, rw);
      stage_meta(L, st ^ 1, rc, t0 + kCandTile, c1, col);
      wave_sync_lds();
      load_rows_coalesced(L, st ^ 1, B.desc, lane, rw);
      rc = load_rec(cand, t0 + 2 * kCandTile + col, c1);
      v4i a[4];
      read_a(L, st, lane, a);
      tile_compute<kKeepCounts>(a, bq, qr, band, L, st, half, k1, k2, cnt);
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
  cnt += __shfl_xor(cnt, 32, 64);   // |C| of this lane's query
  // In-band comparisons of the tile: the sum of its queries' counts.
  int32_t tsum = (half == 0) ? cnt : 0;
  for (int o = 16; o > 0; o >>= 1) tsum += __shfl_xor(tsum, o, 64);
  const unsigned long long total = (unsigned long long)__shfl(tsum, 0, 64);
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
    const unsigned long long padded =
        (unsigned long long)((s_end - s_begin + kCandTile - 1) / kCandTile) * (kCandTile * kQueryTile);
    if (total) atomicAdd(&v.counters[p].comparisons, total);
    if (padded) atomicAdd(&v.counters[p].elements, padded);
    if (nacc) atomicAdd(&v.counters[p].accepted, nacc);
    if (ties) atomicAdd(&v.counters[p].ties, ties);
  }
}

// Each wave walks tiles_per_wave consecutive query tiles of [blk_begin, blk_end)
// (they may belong to different pairs); per-pair data is reloaded on change.
#ifndef SFM_MATCH_WAVES_PER_EU
#define SFM_MATCH_WAVES_PER_EU 3
#endif
template <bool kKeepCounts>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SFM_MATCH_WAVES_PER_EU, 8)))
void match_kernel(BatchView v, int32_t blk_begin, int32_t blk_end) {
  __shared__ __attribute__((aligned(16))) WaveLds lds[kWaves];

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t item = xcd_contiguous(blockIdx.x, gridDim.x) * kWaves + wave;
  const int64_t t_first = int64_t(blk_begin) + int64_t(item) * v.tiles_per_wave;
  const int64_t t_last = min(int64_t(blk_end), t_first + v.tiles_per_wave);
  int32_t cur = -1;
  PairDesc P;
  ImageDev A, B;
  float band = 0.0f;
  for (int64_t t = t_first; t < t_last; ++t) {
    const int4 ti = v.tiles[t];
    if (ti.x != cur) {
      cur = ti.x;
      P = v.pairs[cur];
      A = v.images[P.a];
      B = v.images[P.b];
      band = v.geom[cur].band32;
    }
    match_tile<kKeepCounts>(v, P, cur, A, B, band, ti.y, ti.z, ti.w, lds[wave], lane);
  }
}

}  // namespace

hipError_t launch_match(const BatchView& v, int32_t blk_begin, int32_t blk_count, hipStream_t st) {
  if (blk_count <= 0) return hipSuccess;
  const int32_t per_wave = v.tiles_per_wave;
  const int32_t waves = (blk_count + per_wave - 1) / per_wave;
  const int32_t groups = (waves + kWaves - 1) / kWaves;
  if (v.keep_counts)
    hipLaunchKernelGGL(match_kernel<true>, dim3(groups), dim3(64 * kWaves), 0, st, v, blk_begin,
                       blk_begin + blk_count);
  else
    hipLaunchKernelGGL(match_kernel<false>, dim3(groups), dim3(64 * kWaves), 0, st, v, blk_begin,
                       blk_begin + blk_count);
  return hipGetLastError();
}

}  // namespace sfm
