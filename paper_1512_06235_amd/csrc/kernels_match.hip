// Fused candidate test + distance + two-nearest kernel (a4-a6), Appendix A
// steps 3-4 redesigned for CDNA4.
//
// A workgroup of 1, 2 or 4 waves (default two) owns a group of consecutive query
// tiles (32 queries each, in pencil order) of one pair, one tile per wave.
// Their candidate ranges overlap heavily, so the workgroup streams the union
// range of b's binned features through LDS once, 32 candidates per step:
//   - each wave fetches its share of the 32 descriptor rows with coalesced
//     loads (eight lanes per 128-byte row) and stores them XOR-swizzled into
//     the shared stage; one barrier per step publishes the stage;
//   - each wave whose own range meets the step reads the rows back as the A
//     operand of v_mfma_i32_32x32x32_i8; its negated query rows are the
//     resident B operand, so four MFMAs give -q.c for a 32x32 tile with exact
//     int32 accumulation (bytes 0..127 fit int8, 128 * 127^2 < 2^31);
//   - each lane then holds one query and 16 candidates; it runs the exact
//     band test of eqs. (2)-(3) in FP32 on the candidates' centred
//     coordinates and folds in-band distances into a running two-smallest
//     pair of 32-bit keys
//         key = ((||c||^2 - 2 q.c + 2^21) << 10) | (position mod 1024),
//     so one unsigned min and one med3 keep (D1, its position) and D2;
//   - the two lanes of one query merge with one cross-half exchange.
// The key orders equal distances by binned position, not by index in b; when
// the two smallest keys of a chunk share the distance, an exact pass picks the
// lowest index among the tied candidates, so results equal the definition.
// Two tiles per group balance the row fetches each wave issues against the
// steps a wave idles at the barrier outside its own range (four tiles: 13%
// slower; one tile, no sharing: 17% slower, bound by the address units).
#include <algorithm>
#include <cmath>

#include "sfm_internal.h"

namespace sfm {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned int nv4u __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) nv4u g_nv4u;
typedef const __attribute__((address_space(1))) int32_t g_i32;

// A workgroup of W waves (one query tile each) shares the candidate stream:
// each wave fetches kCandTile / W rows of every step with (kCandTile / W) / 8
// loads of 16 bytes per lane.
template <int W>
struct Split {
  static constexpr int kRowsPerWave = kCandTile / W;
  static constexpr int kRowLoads = kRowsPerWave / 8;
  static_assert(kRowsPerWave % 8 == 0 && kRowsPerWave <= 64, "waves split a step by 8 rows");
};
constexpr int kMetaSlots = 3;

// Epipolar distance of eqs. (2)-(3) on centred FP32 coordinates,
// |a x + b y + c| with (a, b) unit.  The single FP32 evaluation every pass uses.
__device__ __forceinline__ float band_dist32(float a, float b, float c, float x, float y) {
  return __builtin_fabsf(__builtin_fmaf(a, x, __builtin_fmaf(b, y, c)));
}

// The epipolar distance of eqs. (2)-(3) in FP64, on the caller's F and the
// original keypoints, every operation as written (no contraction): the line
// l = F (x, y, 1)^T row by row, s = sqrt(l0^2 + l1^2), then
// |l0 x' + l1 y' + l2| / s.  NaN when s = 0 or s or l2 is not finite (such a
// line has no candidates).
__device__ __forceinline__ double band_dist64(const double* F, float xq, float yq, float xb,
                                           float yb) {
#pragma clang fp contract(off)
  const double x = xq, y = yq;
  const double a = F[0] * x + F[1] * y + F[2];
  const double b = F[3] * x + F[4] * y + F[5];
  const double c = F[6] * x + F[7] * y + F[8];
  const double s = sqrt(a * a + b * b);
  if (!(s > 0.0) || !isfinite(s) || !isfinite(c)) return NAN;
  return fabs(a * double(xb) + b * double(yb) + c) / s;
}

// The band decision in FP64.  The FP32 test is decided again by this function
// for every distance within the margin of d, so results equal an FP64
// evaluation as long as the FP32 error stays below the margin.
__device__ __forceinline__ bool band_exact(const double* F, float xq, float yq, float xb, float yb,
                                           double d) {
  return band_dist64(F, xq, yq, xb, yb) <= d;
}

// What the FP64 re-decision of one pair needs, read when a step first has a
// borderline slot.
struct ExactCtx {
  const double* F;          // the caller's F of the pair
  const float* a_xy;        // original keypoints of a and b
  const float* b_xy;
  double d;
};

__device__ __forceinline__ ExactCtx exact_ctx(const BatchView& v, int32_t pair) {
  const PairDesc P = v.pairs[pair];
  ExactCtx x;
  x.F = v.F + 9 * int64_t(pair);
  x.a_xy = v.images[P.a].xy;
  x.b_xy = v.images[P.b].xy;
  x.d = P.band;
  return x;
}

// Band membership of query i (original index in a) and target j (original
// index in b) from the FP32 distance e32: in below band_lo, out above band_hi,
// decided in FP64 in between.
__device__ __forceinline__ bool member(float e32, float lo, float hi, const ExactCtx& x, int32_t i,
                                       int32_t j) {
  if (e32 <= lo) return true;
  if (!(e32 <= hi)) return false;
  return band_exact(x.F, x.a_xy[2 * i], x.a_xy[2 * i + 1], x.b_xy[2 * j], x.b_xy[2 * j + 1], x.d);
}

// Per-byte negation of four bytes in 0..127 (no borrow crosses a byte).
__device__ __forceinline__ int neg_bytes(uint32_t w) {
  return int((0x80808080u - w) ^ 0x80808080u);
}

__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c) {
  return max(min(a, b), min(max(a, b), c));   // selects v_med3_u32
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

// The same with one pair of 16-byte loads in flight (few registers: for the
// rare FP64 re-decision inside the step loop).
__device__ inline int32_t row_dist_lean(const uint8_t* p, const uint8_t* q, int32_t np,
                                        int32_t nq) {
  uint32_t dot = 0;
#pragma unroll 1
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

// Loads through global-address-space pointers compile to global_load_*,
// which only count against vmcnt.
__device__ __forceinline__ nv4u gload16(const void* p) { return *(g_nv4u*)p; }

// Raw binned record {x, y, ncpos, j} of position min(cp, c1 - 1) (c1 > 0).
__device__ __forceinline__ nv4u load_rec(const CandRec* cand, int32_t cp, int32_t c1) {
  return gload16(cand + min(cp, c1 - 1));
}

// Workgroup LDS: two stages of 32 candidate rows and three stages of their
// metadata.  A row is stored as eight 16-byte chunks with chunk c of row r at
// slot c ^ (r & 7), so both the coalesced stores (eight lanes per row) and the
// MFMA operand reads (one row per lane) hit all 32 banks without conflicts.
struct GroupLds {
  uint8_t rows[2][kCandTile * kDescBytes];
  float x[kMetaSlots][kCandTile];
  float y[kMetaSlots][kCandTile];
  uint32_t nc[kMetaSlots][kCandTile];
  uint32_t sink[kMaxGroupTiles][3][64];   // targets of the lanes that own no record
};

// Wave w owns candidates R*w .. R*w+R-1 of every step (R = kRowsPerWave):
// lane l < R holds the record of candidate R*w + l.  Those lanes stage the
// metadata (the other lanes write to distinct sink words: no divergent
// branch, no bank conflict).  Positions past the range get a NaN coordinate,
// which no band test passes.
template <int W>
__device__ __forceinline__ void stage_meta(GroupLds& L, int st, const nv4u& r, int32_t t0,
                                           int32_t c1, int wave, int lane) {
  constexpr int R = Split<W>::kRowsPerWave;
  const int cand_i = R * wave + (lane % R);
  const bool own = lane < R;
  float* px = own ? &L.x[st][cand_i] : reinterpret_cast<float*>(&L.sink[wave][0][lane]);
  float* py = own ? &L.y[st][cand_i] : reinterpret_cast<float*>(&L.sink[wave][1][lane]);
  uint32_t* pn = own ? &L.nc[st][cand_i] : &L.sink[wave][2][lane];
  *px = t0 + cand_i < c1 ? __uint_as_float(r.x) : NAN;
  *py = __uint_as_float(r.y);
  *pn = r.z;
}

// Load k of this wave's coalesced share of a step's rows: lane l fetches
// 16-byte chunk (l & 7) of row R*w + 8k + (l >> 3), whose index in b lane
// 8k + (l >> 3) holds.
__device__ __forceinline__ nv4u load_row_share(const nv4u& r, const uint8_t* desc, int lane,
                                               int k) {
  const int32_t j = __shfl(int32_t(r.w), 8 * k + (lane >> 3), 64);
  return gload16(desc + int64_t(j) * kDescBytes + 16 * (lane & 7));
}

template <int W>
__device__ __forceinline__ void store_row_share(GroupLds& L, int st, int wave, int lane, int k,
                                                const nv4u& rw) {
  const int m = lane >> 3, c = lane & 7;
  const int row = Split<W>::kRowsPerWave * wave + 8 * k + m;   // row & 7 == m
  *reinterpret_cast<nv4u*>(&L.rows[st][row * kDescBytes + ((c ^ m) << 4)]) = rw;
}

// The MFMA A operand: row (lane & 31), k-slice 16 * half + 32 * s = chunk 2s + half.
__device__ __forceinline__ void read_a(const GroupLds& L, int st, int lane, v4i (&a)[4]) {
  const int r = lane & 31, h = lane >> 5;
#pragma unroll
  for (int s = 0; s < 4; ++s)
    a[s] = *reinterpret_cast<const v4i*>(&L.rows[st][r * kDescBytes + (((2 * s + h) ^ (r & 7)) << 4)]);
}

// The four MFMAs on one step's rows, then this lane's 16 results folded into
// the running two smallest keys (k1, k2), with the candidates' coordinates and
// keys read from metadata slot st.  A slot is folded when its FP32 distance is
// at most band_lo; when any slot of the wave lies within (band_lo, band_hi],
// those slots are decided in FP64 afterwards, one at a time, and folded with
// their distance recomputed on the VALU.  In-band slots are counted per lane
// when counts are kept, per wave (scalar) otherwise.
template <bool kKeepCounts>
__device__ __forceinline__ void tile_compute(const v4i (&ac)[4], const v4i (&bq)[4],
                                             const QueryRec& qr, int32_t nq, float lo, float hi,
                                             const GroupLds& L, int st, int half, uint32_t& k1,
                                             uint32_t& k2, int32_t& cnt, uint32_t& wcnt,
                                             uint32_t& wbl, const BatchView& v,
                                             const TileGroup& G, int32_t t0) {
  v16i acc = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(ac[s], bq[s], acc, 0, 0, 0);

  // Lane (col, half) holds rows 8g + 4*half + e of the tile, e = 0..3.
  unsigned long long border = 0;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int r0 = 8 * g + 4 * half;
    const float4 xs = *reinterpret_cast<const float4*>(&L.x[st][r0]);
    const float4 ys = *reinterpret_cast<const float4*>(&L.y[st][r0]);
    const uint4 ns = *reinterpret_cast<const uint4*>(&L.nc[st][r0]);
    const float xv[4] = {xs.x, xs.y, xs.z, xs.w};
    const float yv[4] = {ys.x, ys.y, ys.z, ys.w};
    const uint32_t nv[4] = {ns.x, ns.y, ns.z, ns.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float d32 = band_dist32(qr.a, qr.b, qr.c, xv[e], yv[e]);
      const bool mem = d32 <= lo;
      border |= __ballot(d32 <= hi) ^ __ballot(mem);   // lo <= hi: mem implies d32 <= hi
      uint32_t key = nv[e] + (uint32_t(acc[4 * g + e]) << 11);
      key = mem ? key : kKeyInf;
      k2 = umed3(k1, key, k2);
      k1 = min(k1, key);
      if (kKeepCounts)
        cnt += mem ? 1 : 0;
      else
        wcnt += __builtin_popcountll(__ballot(mem));
    }
  }
  if (border == 0) return;

  // Rare: this lane's slots within the margin of d, decided in FP64.
  uint32_t bm = 0;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 8 * g + 4 * half + e;
      const float d32 = band_dist32(qr.a, qr.b, qr.c, L.x[st][r], L.y[st][r]);
      if (d32 <= hi && !(d32 <= lo)) bm |= 1u << (4 * g + e);
    }
  }
  int32_t nbl = __builtin_popcount(bm), nin = 0;
  const ExactCtx x = exact_ctx(v, G.pair);
  const CandRec* cand = v.cand + G.c_off;
  while (bm) {
    const int sidx = __builtin_ctz(bm);
    bm &= bm - 1;
    const int r = 8 * (sidx >> 2) + 4 * half + (sidx & 3);
    const int32_t j = cand[t0 + r].j;
    if (!band_exact(x.F, x.a_xy[2 * qr.i], x.a_xy[2 * qr.i + 1], x.b_xy[2 * j],
                    x.b_xy[2 * j + 1], x.d))
      continue;
    const uint32_t nc = L.nc[st][r];
    const int32_t D = row_dist_lean(G.a_desc + int64_t(qr.i) * kDescBytes,
                               G.b_desc + int64_t(j) * kDescBytes, nq,
                               int32_t(nc >> kPosBits) - int32_t(kDistBias));
    const uint32_t key = (uint32_t(D - nq + int32_t(kDistBias)) << kPosBits) | (nc & (kChunk - 1));
    k2 = umed3(k1, key, k2);
    k1 = min(k1, key);
    ++nin;
  }
  if (kKeepCounts) cnt += nin;
  for (int o = 32; o > 0; o >>= 1) {
    nbl += __shfl_xor(nbl, o, 64);
    nin += __shfl_xor(nin, o, 64);
  }
  wbl += uint32_t(nbl);
  if (!kKeepCounts) wcnt += uint32_t(nin);
}

// Running result of one query column across chunks of 1024 positions.
struct QueryState {
  int32_t d1, d2, j1;
  uint32_t ties;
};

// End of a chunk [c0, c1): merge the halves' keys, decode (D1, position, D2),
// resolve equal smallest distances exactly, fold into the running result.
__device__ __forceinline__ void finish_chunk(const BatchView& v, const TileGroup& G,
                                             const CandRec* cand, const uint8_t* a_desc,
                                             const uint8_t* b_desc, const QueryRec& qr, int32_t nq,
                                             float lo, float hi, int32_t c0, int32_t c1, int lane,
                                             uint32_t k1, uint32_t k2, QueryState& q) {
  const int col = lane & 31, half = lane >> 5;
  {
    const uint32_t p1 = __shfl_xor(k1, 32, 64);
    const uint32_t p2 = __shfl_xor(k2, 32, 64);
    k2 = min(max(k1, p1), min(k2, p2));
    k1 = min(k1, p1);
  }
  // The index load is unconditional and consumed at once, so no load stays
  // in flight past the chunk end (a pending load into a register the loop
  // reuses would make every later step wait for all prefetches).
  const int32_t pos = int32_t(k1 & (kChunk - 1));
  const int32_t at = min(c0 + ((pos - c0) & (kChunk - 1)), c1 - 1);
  const int32_t jl = *(g_i32*)&cand[at].j;
  const int32_t D1c = k1 != kKeyInf ? int32_t(k1 >> kPosBits) - int32_t(kDistBias) + nq : kDistInf;
  const int32_t D2c = k2 != kKeyInf ? int32_t(k2 >> kPosBits) - int32_t(kDistBias) + nq : kDistInf;
  int32_t j1c = k1 != kKeyInf ? jl : -1;

  // Equal smallest distances: choose the lowest index of b exactly.
  const bool tie = k2 != kKeyInf && (k1 >> kPosBits) == (k2 >> kPosBits);
  unsigned long long tmask = __ballot(tie && half == 0);
  const ExactCtx x = tmask ? exact_ctx(v, G.pair) : ExactCtx{nullptr, nullptr, nullptr, 0.0};
  while (tmask) {
    const int Lq = __builtin_ctzll(tmask);
    tmask &= tmask - 1;
    ++q.ties;
    const float la = __shfl(qr.a, Lq, 64), lb = __shfl(qr.b, Lq, 64), lc = __shfl(qr.c, Lq, 64);
    const int32_t li = __shfl(qr.i, Lq, 64), lnq = __shfl(nq, Lq, 64), lD = __shfl(D1c, Lq, 64);
    const uint8_t* qrow = a_desc + int64_t(li) * kDescBytes;
    int32_t jbest = 0x7FFFFFFF;
    for (int32_t s = c0 + lane; s < c1; s += 64) {
      const CandRec r = cand[s];
      if (!member(band_dist32(la, lb, lc, r.x, r.y), lo, hi, x, li, r.j)) continue;
      const int32_t nc = int32_t(r.ncpos >> kPosBits) - int32_t(kDistBias);
      const int32_t D = row_dist(qrow, b_desc + int64_t(r.j) * kDescBytes, lnq, nc);
      if (D == lD) jbest = min(jbest, r.j);
    }
    for (int o = 32; o > 0; o >>= 1) jbest = min(jbest, __shfl_xor(jbest, o, 64));
    if (col == Lq) j1c = jbest;
  }

  if (D1c < q.d1 || (D1c == q.d1 && D1c != kDistInf && j1c < q.j1)) {
    q.d2 = min(q.d1, D2c);
    q.d1 = D1c;
    q.j1 = j1c;
  } else {
    q.d2 = min(q.d2, D1c);
  }
}

// Per-wave statistics of the groups of one pair, flushed when the pair changes.
struct WaveStats {
  int32_t pair;
  unsigned long long comparisons, elements, borderline;
  uint32_t accepted, ties;
};

__device__ __forceinline__ void flush_stats(const BatchView& v, WaveStats& w, int lane) {
  if (w.pair >= 0 && lane == 0) {
    if (w.comparisons) atomicAdd(&v.counters[w.pair].comparisons, w.comparisons);
    if (w.elements) atomicAdd(&v.counters[w.pair].elements, w.elements);
    if (w.borderline) atomicAdd(&v.counters[w.pair].borderline, w.borderline);
    if (w.accepted) atomicAdd(&v.counters[w.pair].accepted, w.accepted);
    if (w.ties) atomicAdd(&v.counters[w.pair].ties, w.ties);
  }
  w.comparisons = w.elements = w.borderline = 0;
  w.accepted = w.ties = 0;
}

// A group record read with scalar loads (its index is uniform).
typedef const __attribute__((address_space(4))) v4i c_v4i;
__device__ __forceinline__ TileGroup load_group(const TileGroup* groups, int32_t g) {
  union {
    v4i w[sizeof(TileGroup) / 16];
    TileGroup t;
  } u;
  c_v4i* src = (c_v4i*)(groups + g);
#pragma unroll
  for (int k = 0; k < int(sizeof(TileGroup) / 16); ++k) u.w[k] = src[k];
  return u.t;
}

// One group: up to four query tiles (one per wave) against their union
// candidate range, streamed through LDS 32 candidates per step with one
// barrier per step.
template <bool kKeepCounts, int W>
__device__ __forceinline__ void match_group(const BatchView& v, const TileGroup& G, GroupLds& L,
                                            int wave, int lane, WaveStats& ws) {
  constexpr int kRowLoads = Split<W>::kRowLoads;
  constexpr int kRowsPerWave = Split<W>::kRowsPerWave;
  const int col = lane & 31, half = lane >> 5;
  const bool wv = wave < G.ntiles;
  const int32_t blk = G.tile0 + wave;
  // Selects, not an indexed read: a dynamic index would put the record in
  // private memory.
  int32_t my_b = 0, my_e = 0;
#pragma unroll
  for (int t = 0; t < W; ++t) {
    my_b = wave == t ? G.t_begin[t] : my_b;
    my_e = wave == t ? G.t_end[t] : my_e;
  }
  if (!wv) my_b = my_e = 0;
  const float lo = G.band_lo, hi = G.band_hi;
  const uint8_t* const a_desc = G.a_desc;
  const uint8_t* const b_desc = G.b_desc;

  // This lane's query column: line, squared norm and negated descriptor bytes
  // as the MFMA B operand.  Padding columns read query row 0 with a NaN line.
  const int32_t qs = blk * kQueryTile + col;
  const bool qv = wv && qs < G.na;
  const nv4u qu = gload16(v.qrec + G.q_off + min(qs, G.na - 1));
  QueryRec qr;
  qr.a = qv ? __uint_as_float(qu.x) : NAN;
  qr.b = __uint_as_float(qu.y);
  qr.c = __uint_as_float(qu.z);
  qr.i = int32_t(qu.w);
  const int32_t S0 = G.s_begin, S1 = G.s_end;
  const CandRec* cand = v.cand + G.c_off;

  // Records of the first two steps go out with the query record; the query
  // row and the first candidate rows follow one latency later.
  const int32_t own = kRowsPerWave * wave + (lane % kRowsPerWave);
  const bool any = S1 > S0;
  nv4u re = {0, 0, 0, 0}, ro = {0, 0, 0, 0};
  if (any) {
    re = load_rec(cand, S0 + own, S1);
    ro = load_rec(cand, S0 + kCandTile + own, S1);
  }
  v4i bq[4];
  {
    const uint8_t* qrow = a_desc + int64_t(qr.i) * kDescBytes + 16 * half;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const nv4u u = gload16(qrow + 32 * s);
      bq[s] = v4i{neg_bytes(u.x), neg_bytes(u.y), neg_bytes(u.z), neg_bytes(u.w)};
    }
  }
  const int32_t nq = ((g_i32*)G.a_norm)[qr.i];

  QueryState q = {kDistInf, kDistInf, -1, 0};
  int32_t cnt = 0;       // in-band slots of this lane (counts kept)
  uint32_t wcnt = 0;     // in-band slots of this wave (counts not kept)
  uint32_t wbl = 0;      // slots decided in FP64

  if (any) {
    // Software pipeline over steps u = 0, 1, ... of 32 candidates.  Iteration
    // u stores rows u (loaded two iterations earlier) into row stage u & 1,
    // passes the barrier, issues the rows of u + 2 (their indices come from
    // the record registers, so no barrier lies on that chain), stages the
    // metadata of u + 2 into slot (u + 2) % 3, loads the record of u + 4 and
    // computes step u from row stage u & 1 and metadata slot u % 3.  The loop
    // is unrolled by two so the in-flight registers never move (a copy of a
    // register with a load in flight would wait for that load).
    const int32_t nsteps = (S1 - S0 + kCandTile - 1) / kCandTile;
    nv4u we[kRowLoads], wo[kRowLoads];
    stage_meta<W>(L, 0, re, S0, S1, wave, lane);
#pragma unroll
    for (int k = 0; k < kRowLoads; ++k) we[k] = load_row_share(re, b_desc, lane, k);
    re = load_rec(cand, S0 + 2 * kCandTile + own, S1);
    stage_meta<W>(L, 1, ro, S0 + kCandTile, S1, wave, lane);
#pragma unroll
    for (int k = 0; k < kRowLoads; ++k) wo[k] = load_row_share(ro, b_desc, lane, k);
    ro = load_rec(cand, S0 + 3 * kCandTile + own, S1);

    uint32_t k1 = kKeyInf, k2 = kKeyInf;
    int32_t c0 = S0;
    int ms = 0;   // metadata slot of step u
    // One step; `w` and `r` are this parity's row and record registers.
    auto step = [&](int32_t u, int rs, nv4u (&w)[kRowLoads], nv4u& r) {
      const int32_t t0 = S0 + u * kCandTile;
#pragma unroll
      for (int k = 0; k < kRowLoads; ++k) store_row_share<W>(L, rs, wave, lane, k, w[k]);
      __syncthreads();
      const int ms2 = ms == 0 ? 2 : ms - 1;   // (u + 2) % 3
      stage_meta<W>(L, ms2, r, t0 + 2 * kCandTile, S1, wave, lane);
#pragma unroll
      for (int k = 0; k < kRowLoads; ++k) w[k] = load_row_share(r, b_desc, lane, k);
      r = load_rec(cand, t0 + 4 * kCandTile + own, S1);
      if (t0 < my_e && t0 + kCandTile > my_b) {
        // Waves in their compute phase issue first (1-2% faster than equal
        // priority; raising the load phase instead gains nothing).
        __builtin_amdgcn_s_setprio(2);
        v4i a[4];
        read_a(L, rs, lane, a);
        tile_compute<kKeepCounts>(a, bq, qr, nq, lo, hi, L, ms, half, k1, k2, cnt, wcnt, wbl, v,
                                  G, t0);
        __builtin_amdgcn_s_setprio(0);
      }
      // Keys hold positions mod 1024: close a chunk every 1024 positions.
      const int32_t t1 = t0 + kCandTile;
      if (t1 >= S1 || t1 - c0 >= kChunk) {
        const int32_t c1 = min(S1, c0 + kChunk);
        finish_chunk(v, G, cand, a_desc, b_desc, qr, nq, lo, hi, c0, c1, lane, k1, k2, q);
        k1 = kKeyInf;
        k2 = kKeyInf;
        c0 = c1;
      }
      ms = ms == 2 ? 0 : ms + 1;
    };
    // The loop body always runs both steps, so the loads in flight at its
    // head are the same on every path (an odd last step runs after it).
    int32_t u = 0;
    for (; u + 1 < nsteps; u += 2) {
      step(u, 0, we, re);
      step(u + 1, 1, wo, ro);
    }
    if (u < nsteps) step(u, 0, we, re);
    // No wave may overwrite the stage of the next group while others read it.
    __syncthreads();
  }

  bool accept;
  if (q.d2 != kDistInf) {
    accept = int64_t(v.ratio_den) * q.d1 < int64_t(v.ratio_num) * q.d2;
  } else {
    accept = q.d1 != kDistInf && v.accept_single;
  }
  if (kKeepCounts) cnt += __shfl_xor(cnt, 32, 64);   // |C| of this lane's query
  if (qv && half == 0) {
    QueryResult out;
    out.match = q.j1;
    out.d1 = q.d1;
    out.d2 = q.d2;
    out.flags = (accept ? 1 : 0) | (kKeepCounts ? (cnt << 1) : 0);
    v.res[G.q_off + qr.i] = out;
  }
  // In-band comparisons of the tile: the sum of its queries' counts.
  int32_t tsum = int32_t(wcnt);
  if (kKeepCounts) {
    tsum = (half == 0) ? cnt : 0;
    for (int o = 16; o > 0; o >>= 1) tsum += __shfl_xor(tsum, o, 64);
    tsum = __shfl(tsum, 0, 64);
  }
  const uint32_t nacc = __builtin_popcountll(__ballot(accept && qv && half == 0));
  if (wv) {
    if (G.pair != ws.pair) {
      flush_stats(v, ws, lane);
      ws.pair = G.pair;
    }
    int32_t steps = 0;
    if (my_e > my_b) {
      const int32_t first = (max(my_b, S0) - S0) / kCandTile;
      const int32_t last = (my_e - 1 - S0) / kCandTile;
      steps = last - first + 1;
    }
    ws.comparisons += (unsigned long long)tsum;
    ws.borderline += wbl;
    ws.elements += (unsigned long long)steps * (kCandTile * kQueryTile);
    ws.accepted += nacc;
    ws.ties += q.ties;
  }
}

// One resident wave of workgroups.  Workgroups are dealt to the 8 XCDs
// round-robin (workgroup k runs on XCD k mod 8), and each XCD has its own L2.
// The preparation pass splits the groups into one contiguous share of about
// equal estimated cost per XCD; the workgroups of an XCD sweep its share
// together, workgroup i taking groups i, i + W, i + 2W, ... (W workgroups on
// the XCD).  At any moment an XCD then works on about W consecutive groups,
// one or two pairs, whose candidate and query rows stay in its L2; giving
// each workgroup a contiguous run instead spreads an XCD over dozens of
// pairs at once and its rows over HBM.
#ifndef SFM_MATCH_WAVES_PER_EU
#define SFM_MATCH_WAVES_PER_EU 3
#endif
#ifndef SFM_XCD_SWEEP
#define SFM_XCD_SWEEP 0
#endif
__device__ __forceinline__ int32_t xcd_contiguous(int32_t g, int32_t G) {
  const int32_t x = g & 7, k = g >> 3, q = G >> 3, r = G & 7;
  return x * q + min(x, r) + k;
}
template <bool kKeepCounts, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(SFM_MATCH_WAVES_PER_EU, 8)))
void match_kernel(BatchView v) {
  __shared__ __attribute__((aligned(16))) GroupLds lds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  typedef const __attribute__((address_space(4))) int32_t c_i32;
#if SFM_XCD_SWEEP
  const int32_t shares = min(8, int32_t(gridDim.x));
  const int32_t x = blockIdx.x % shares;
  const int32_t i = blockIdx.x / shares;
  const int32_t w = (int32_t(gridDim.x) - x + shares - 1) / shares;
  const int32_t g_first = ((c_i32*)v.wg_start)[x] + i;
  const int32_t g_end = ((c_i32*)v.wg_start)[x + 1];
#else
  const int32_t run = xcd_contiguous(blockIdx.x, gridDim.x);
  const int32_t w = 1;
  const int32_t g_first = ((c_i32*)v.wg_start)[run];
  const int32_t g_end = ((c_i32*)v.wg_start)[run + 1];
#endif
  WaveStats ws = {-1, 0, 0, 0, 0, 0};
  for (int32_t g = g_first; g < g_end; g += w) {
    const TileGroup G = load_group(v.groups, g);
    match_group<kKeepCounts, W>(v, G, lds, wave, lane, ws);
  }
  flush_stats(v, ws, lane);
}

// Diagnostic of the FP32 band test: over every (query, candidate) slot of
// every query tile's candidate range whose FP64 distance is at most 2d, the
// largest |FP32 distance - FP64 distance| (as the bits of a non-negative
// double, which order like the integers) and the number of such slots.  One
// wave per tile, one lane per query.
__global__ __launch_bounds__(64) void band_error_kernel(BatchView v,
                                                        unsigned long long* out) {
  const int32_t g = blockIdx.x / v.group_tiles, t = blockIdx.x % v.group_tiles;
  const TileGroup& G = v.groups[g];
  const int lane = threadIdx.x;
  if (t >= G.ntiles || lane >= kQueryTile) return;
  const int32_t qs = (G.tile0 + t) * kQueryTile + lane;
  const int32_t b = G.t_begin[t], e = G.t_end[t];
  double worst = 0.0;
  unsigned long long n = 0;
  if (qs < G.na && e > b) {
    const QueryRec qr = v.qrec[G.q_off + qs];
    const ExactCtx x = exact_ctx(v, G.pair);
    const CandRec* cand = v.cand + G.c_off;
    const double two_d = 2.0 * x.d;
    const float xq = x.a_xy[2 * qr.i], yq = x.a_xy[2 * qr.i + 1];
    for (int32_t s = b; s < e; ++s) {
      const CandRec r = cand[s];
      const double e64 = band_dist64(x.F, xq, yq, x.b_xy[2 * r.j], x.b_xy[2 * r.j + 1]);
      if (!(e64 <= two_d)) continue;
      const double e32 = band_dist32(qr.a, qr.b, qr.c, r.x, r.y);
      worst = fmax(worst, fabs(e32 - e64));
      ++n;
    }
  }
  unsigned long long bits = __double_as_longlong(worst);
  for (int o = 32; o > 0; o >>= 1) {
    bits = max(bits, (unsigned long long)__shfl_xor((long long)bits, o, 64));
    n += (unsigned long long)__shfl_xor((long long)n, o, 64);
  }
  if (lane == 0) {
    if (bits) atomicMax(&out[0], bits);
    if (n) atomicAdd(&out[1], n);
  }
}

}  // namespace

// Workgroups of the match kernel that fit on a device at once.
template <int W>
static int32_t resident_workgroups(int dev) {
  static int32_t cached[64] = {0};
  if (dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, match_kernel<false, W>, 64 * W, 0) !=
            hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        per_cu <= 0 || cus <= 0) {
      per_cu = 1;
      cus = 256;
    }
    cached[dev] = per_cu * cus;
  }
  return cached[dev];
}

int32_t match_workgroups(int32_t device, int32_t group_tiles, int64_t groups) {
  const int32_t r = group_tiles == 1   ? resident_workgroups<1>(device)
                    : group_tiles == 4 ? resident_workgroups<4>(device)
                                       : resident_workgroups<2>(device);
  return int32_t(std::max<int64_t>(1, std::min<int64_t>(groups, r)));
}

template <int W>
static void launch_match_w(const BatchView& v, int32_t wgs, hipStream_t st) {
  if (v.keep_counts)
    hipLaunchKernelGGL((match_kernel<true, W>), dim3(wgs), dim3(64 * W), 0, st, v);
  else
    hipLaunchKernelGGL((match_kernel<false, W>), dim3(wgs), dim3(64 * W), 0, st, v);
}

hipError_t launch_match(const BatchView& v, int32_t wgs, hipStream_t st) {
  if (wgs <= 0) return hipSuccess;
  if (v.group_tiles == 1)
    launch_match_w<1>(v, wgs, st);
  else if (v.group_tiles == 4)
    launch_match_w<4>(v, wgs, st);
  else
    launch_match_w<2>(v, wgs, st);
  return hipGetLastError();
}

hipError_t launch_band_error(const BatchView& v, int64_t n_groups, unsigned long long* out,
                             hipStream_t st) {
  const int64_t blocks = n_groups * v.group_tiles;
  if (blocks <= 0) return hipSuccess;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(band_error_kernel, dim3(uint32_t(blocks)), dim3(64), 0, st, v, out);
  return hipGetLastError();
}

}  // namespace sfm
