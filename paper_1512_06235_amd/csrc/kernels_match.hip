// Fused candidate test + distance + two-nearest kernel (a4-a6), Appendix A
// steps 3-4 redesigned for CDNA4.
//
// Work unit: a group of up to 4 * TPW consecutive query tiles of one pair (16
// queries each, in pencil order).  A workgroup of four waves loads the union
// of the group's candidate ranges (b's features in binned order, up to 256
// positions at a time) into one LDS buffer, then each wave runs its own tiles
// over their ranges without further synchronisation.
//   - The buffer is filled by LDS DMA (global_load_lds): wave w fetches the
//     16-position blocks w, w + 4, ... (two 16-byte loads per lane for a
//     block's 16 descriptor rows, eight lanes per 128-byte row, XOR-swizzled,
//     and 16 of its coordinates and keys).  The rows' indices in b arrive one
//     group earlier in an index buffer of their own, so no loaded value passes
//     through a register on its way to LDS.
//   - Per group: one wait and one barrier before the buffer is read, one
//     barrier before it is refilled.  The next group's row indices and query
//     records load while the current group computes.  The workgroups on one
//     XCD take the groups of one contiguous share in turn, so at any time they
//     work on one or two pairs whose rows stay in that XCD's L2.
//   - Wave w owns tiles w and 2 * 4 - 1 - w (when a group has eight), which
//     balances the waves of a group whose range lengths drift along it.
//   - Each tile walks its candidate range in steps of 16 positions aligned to
//     16.  A step's rows are the A operand of v_mfma_i32_16x16x64_i8 and the
//     tile's negated query rows the resident B operand: two MFMAs give -q.c
//     for 16 candidates x 16 queries, exact in int32 (bytes 0..127 fit int8,
//     128 * 127^2 < 2^31).  The next step's operands are read from LDS before
//     the current step's fold.
//   - Each lane then holds one query and 4 candidates.  It runs the band test
//     of eqs. (2)-(3) in FP32 on centred coordinates and folds in-band keys
//         key = ((||c||^2 - 2 q.c + 2^21) << 10) | (position mod 1024)
//     into its two smallest with one v_med3_u32 and one v_min_u32.
//   - Slots whose FP32 distance lies within the margin of d are queued in LDS
//     with their exact key and index in b, and decided in FP64 when the
//     group's tiles are done.
// The key orders equal distances by binned position, not by index in b; when
// a query's smallest distance is shared, an exact pass picks the lowest index
// among the tied candidates, so results equal the definition.  Results hold
// the binned position of the match; emission maps it to the index in b.
#include <algorithm>
#include <cmath>
#include <cstddef>

#include "sfm_internal.h"

namespace sfm {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned int nv4u __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) nv4u g_nv4u;
typedef const __attribute__((address_space(1))) int32_t g_i32;
typedef __attribute__((address_space(3))) void lds_void;

constexpr int kWaves = kMatchWaves;           // waves per workgroup
#ifndef SFM_MATCH_BUF
#define SFM_MATCH_BUF 256
#endif
constexpr int kBuf = SFM_MATCH_BUF;           // candidate positions one buffer fill holds (power of two)
constexpr int kBlock = 16;                    // positions per DMA block (one step)
constexpr int kBlocks = kBuf / kBlock;        // blocks of a buffer fill
constexpr int kBlocksPerWave = kBlocks / kWaves;
constexpr int kBorderCap = 32;                // queued FP64 decisions per wave and group
static_assert(kBlocksPerWave * kWaves == kBlocks, "blocks are dealt evenly to the waves");
static_assert(kBlocksPerWave * kBlock <= 64, "one 64-lane load fetches a wave's row indices");
static_assert((kBuf & (kBuf - 1)) == 0, "buffer offsets wrap with a mask");
static_assert(kQueryTile == kBlock, "one MFMA column block of queries per tile");
static_assert(kBuf <= kChunk, "a tile's steps in one fill fit one key chunk");
constexpr uint32_t kKeyDistInf = kKeyInf >> kPosBits;

// A global load through an address-space-1 pointer: the pointers used with
// it come from records, and the flat loads the compiler would otherwise emit
// also count against the LDS counter, so each would be waited for alone.
template <class T>
__device__ __forceinline__ T ldg(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

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
  double f[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) f[k] = ldg(F + k);
  const double a = f[0] * x + f[1] * y + f[2];
  const double b = f[3] * x + f[4] * y + f[5];
  const double c = f[6] * x + f[7] * y + f[8];
  const double s = sqrt(a * a + b * b);
  const bool line = s > 0.0 && isfinite(s) && isfinite(c);
  // Computed either way and selected, so the loads of (xb, yb) are not
  // moved into a branch behind this one's.
  const double e = fabs(a * double(xb) + b * double(yb) + c) / s;
  return line ? e : NAN;
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
#pragma unroll 2
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

__device__ __forceinline__ nv4u gload16(const void* p) { return *(g_nv4u*)p; }

// ---------------------------------------------------------------------------
// LDS of a workgroup (40 KB: four workgroups per CU): one buffer fill of
// candidates (rows XOR-swizzled: chunk c of buffer position r at
// (c ^ (r & 7)) * 16 within the row), the row indices of two groups (each
// wave's blocks together, block w + 4 k at 16 k) and the queues of FP64
// decisions.
// ---------------------------------------------------------------------------
struct MatchLds {
  uint8_t rows[kBuf * kDescBytes];
  float x[kBuf];
  float y[kBuf];
  uint32_t nc[kBuf];
  int32_t j[2][kWaves][kBlocksPerWave * kBlock];
  uint4 queue[kWaves][kBorderCap];   // {key, rel. position << 7 | tile << 6 | lane, j, -}
};
static_assert(sizeof(MatchLds) <= 40960, "four workgroups per CU");

// Keeps the compiler from moving memory accesses across a wait or barrier.
__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

// Waits until at most N of this wave's vector-memory operations are in
// flight (they complete in order); expcnt and lgkmcnt are left alone.
template <int N>
__device__ __forceinline__ void wait_loads() {
  static_assert(N >= 0 && N < 16, "vmcnt range used here");
  compiler_fence();
  __builtin_amdgcn_s_waitcnt(N | 0x0F70);
  compiler_fence();
}

// Workgroup barrier without the fence __syncthreads() adds (which would wait
// for every LDS DMA in flight, including those of segments not yet needed).
__device__ __forceinline__ void barrier() {
  compiler_fence();
  __builtin_amdgcn_s_barrier();
  compiler_fence();
}

// LDS DMA: lane l's 16 (or 4) bytes at src land at LDS offset lds_off + 16 l
// (4 l); lds_off is wave-uniform.  Written as inline asm (M0 set in the same
// statement) so that the compiler does not track these LDS writes: it would
// otherwise wait for every DMA in flight before each LDS read of the ring.
// The kernel orders them itself with wait_loads() and barrier(); the
// compiler's own waits for loads into registers stay correct (they can only
// become stricter).
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void dma16(const void* src, uint32_t lds_off) {
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off"
               :: "s"(__builtin_amdgcn_readfirstlane(lds_off)), "v"(src) : "memory", "m0");
}
__device__ __forceinline__ void dma4(const void* src, uint32_t lds_off) {
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dword %1, off"
               :: "s"(__builtin_amdgcn_readfirstlane(lds_off)), "v"(src) : "memory", "m0");
}
#pragma clang diagnostic pop

// One pair's binned candidates as one group reads them, by position
// relative to `base` (the group's first position rounded down to 16).
struct Stream {
  const float* x;
  const float* y;
  const uint32_t* nc;
  const int32_t* j;
  const uint8_t* b_desc;
  int32_t base;             // pair position of relative position 0
  int32_t last;             // last readable pair position (n_b plus padding, minus 1)
  int32_t len;              // positions to read, a multiple of 16 (0: none)
  uint32_t lds;             // LDS offset of the workgroup's MatchLds
};

__device__ __forceinline__ Stream make_stream(const BatchView& v, const TileGroup& G,
                                              const MatchLds& L) {
  Stream s;
  s.x = v.cand_x + G.c_off;
  s.y = v.cand_y + G.c_off;
  s.nc = v.cand_nc + G.c_off;
  s.j = v.cand_j + G.c_off;
  s.b_desc = G.b_desc;
  s.base = G.s_begin & ~(kBlock - 1);
  s.last = G.nb + kCandPad - 1;
  s.len = G.s_end > G.s_begin ? ((G.s_end - s.base + kBlock - 1) & ~(kBlock - 1)) : 0;
  s.lds = uint32_t(reinterpret_cast<uintptr_t>((lds_void*)&L));
  return s;
}

// The row indices of this wave's blocks of the fill starting at relative
// position f into index buffer `par`: one 4-byte load (lane l:
// block w + 4 (l >> 4), position l & 15; blocks past the stream load a
// clamped position that is never used).
__device__ __forceinline__ void issue_j(const Stream& s, int32_t f, int par, int w, int lane) {
  if (kBlocksPerWave * kBlock < 64 && lane >= kBlocksPerWave * kBlock) return;
  const int32_t p = min(s.base + f + kBlock * (w + kWaves * (lane >> 4)) + (lane & 15), s.last);
  dma4(s.j + p, s.lds + uint32_t(offsetof(MatchLds, j)) +
                    4u * uint32_t((par * kWaves + w) * kBlocksPerWave * kBlock));
}

// Rows and metadata of this wave's blocks of the fill starting at relative
// position f (nblk blocks): per block two 16-byte loads per lane (lane l: row
// 8 t + (l >> 3) of the block, chunk (l & 7) ^ (row & 7), landing at slot
// l & 7 of the row) and three 4-byte loads on 16 lanes.  The rows' indices
// come from index buffer `par` (loaded earlier by this wave and complete).
__device__ __forceinline__ void issue_rows(const Stream& s, const MatchLds& L, int32_t f,
                                           int32_t nblk, int par, int w, int lane) {
  const int32_t* jw = &L.j[par][w][0];
#pragma unroll
  for (int k = 0; k < kBlocksPerWave; ++k) {
    const int32_t b = w + kWaves * k;
    if (b >= nblk) break;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int rr = 8 * t + (lane >> 3);
      const int32_t jr = jw[kBlock * k + rr];
      const int c = (lane & 7) ^ (rr & 7);
      dma16(s.b_desc + int64_t(jr) * kDescBytes + 16 * c,
            s.lds + uint32_t(offsetof(MatchLds, rows)) +
                uint32_t((kBlock * b + 8 * t) * kDescBytes));
    }
    if (lane < kBlock) {
      const int32_t p = min(s.base + f + kBlock * b + lane, s.last);
      const uint32_t o = 4u * uint32_t(kBlock * b);
      dma4(s.x + p, s.lds + uint32_t(offsetof(MatchLds, x)) + o);
      dma4(s.y + p, s.lds + uint32_t(offsetof(MatchLds, y)) + o);
      dma4(s.nc + p, s.lds + uint32_t(offsetof(MatchLds, nc)) + o);
    }
  }
}

// A group record read with scalar loads (its index is uniform).
typedef const __attribute__((address_space(4))) v4i c_v4i;
typedef const __attribute__((address_space(4))) int32_t c_i32;
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

// Tile k of wave w in a group of 4 * TPW tiles.
template <int TPW>
__device__ __forceinline__ int32_t tile_of(int w, int k) {
  return k == 0 ? w : 2 * kWaves - 1 - w;
}

// The first stage of a group: this wave's query records (in registers) and
// the row indices of its blocks of the first fill (into index buffer par).
template <int TPW>
struct GroupStart {
  nv4u qu[TPW];
};
template <int TPW>
__device__ __forceinline__ GroupStart<TPW> start_group(const BatchView& v, const TileGroup& G,
                                                       const MatchLds& L, int par, int w,
                                                       int lane) {
  GroupStart<TPW> st;
  const int col = lane & (kQueryTile - 1);
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    const int32_t qs = (G.tile0 + tile_of<TPW>(w, k)) * kQueryTile + col;
    st.qu[k] = gload16(v.qrec + G.q_off + min(qs, G.na - 1));
  }
  const Stream s = make_stream(v, G, L);
  issue_j(s, 0, par, w, lane);
  return st;
}

// One query tile of a wave: its query column (one query per lane, four lanes
// per query), the negated query bytes as the MFMA B operand and the running
// result.  Distances are kept as key distances (D - ||q||^2 + 2^21, the top
// 22 bits of a key), so chunks merge without the query's norm.
struct Tile {
  float a, b, c;            // the query's FP32 line on centred coordinates
  int32_t i, nq;            // its index in a and ||q||^2
  v4i bq[2];
  uint32_t k1, k2;          // two smallest keys of the current chunk
  uint32_t s1, s2;          // two smallest key distances so far (kKeyDistInf: none)
  int32_t p1;               // pair position of s1's candidate
  bool tie;                 // s1 is reached by more than one candidate
  int32_t cnt;              // in-band slots of this lane (counts kept)
};

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

// What the FP64 decisions and the rare exact passes of one group read (all
// uniform).
struct GroupRefs {
  const double* F;          // the caller's F of the pair
  const float* a_xy;        // original keypoints of a and b
  const float* b_xy;
  const uint8_t* a_desc;
  const uint8_t* b_desc;
  const float* cx;          // the pair's binned targets
  const float* cy;
  const uint32_t* cnc;
  const int32_t* cj;
  double d;
  float lo, hi;
};

__device__ __forceinline__ GroupRefs group_refs(const BatchView& v, const TileGroup& G) {
  GroupRefs r;
  r.F = v.F + 9 * int64_t(G.pair);
  r.a_xy = G.a_xy;
  r.b_xy = G.b_xy;
  r.d = G.band;
  r.a_desc = G.a_desc;
  r.b_desc = G.b_desc;
  r.cx = v.cand_x + G.c_off;
  r.cy = v.cand_y + G.c_off;
  r.cnc = v.cand_nc + G.c_off;
  r.cj = v.cand_j + G.c_off;
  r.lo = G.band_lo;
  r.hi = G.band_hi;
  return r;
}

// Band membership from the FP32 distance e32: in at most lo, out above hi,
// decided in FP64 in between.
__device__ __forceinline__ bool member(const GroupRefs& r, float e32, int32_t i, int32_t j) {
  if (e32 <= r.lo) return true;
  if (!(e32 <= r.hi)) return false;
  return band_dist64(r.F, r.a_xy[2 * i], r.a_xy[2 * i + 1], r.b_xy[2 * j], r.b_xy[2 * j + 1]) <=
         r.d;
}

// Exact pass for a query whose smallest distance D1 is shared: over pair
// positions [p0, p1) the position of the lowest index in b among members at
// distance D1.
__device__ __forceinline__ int32_t lowest_tied(const GroupRefs& r, float a, float b, float c,
                                               int32_t i, int32_t nq, int32_t D1, int32_t p0,
                                               int32_t p1, int lane) {
  const uint8_t* qrow = r.a_desc + int64_t(i) * kDescBytes;
  int32_t jbest = 0x7FFFFFFF, pbest = -1;
  for (int32_t p = p0 + lane; p < p1; p += 64) {
    const int32_t j = r.cj[p];
    if (!member(r, band_dist32(a, b, c, r.cx[p], r.cy[p]), i, j)) continue;
    const int32_t nc = int32_t(r.cnc[p] >> kPosBits) - int32_t(kDistBias);
    if (row_dist(qrow, r.b_desc + int64_t(j) * kDescBytes, nq, nc) == D1 && j < jbest) {
      jbest = j;
      pbest = p;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const int32_t oj = __shfl_xor(jbest, o, 64), op = __shfl_xor(pbest, o, 64);
    if (oj < jbest) { jbest = oj; pbest = op; }
  }
  return pbest;
}

// Exact recomputation of one tile (after its wave's queue of FP64 decisions
// overflowed): lane (col, rg) takes positions p0 + rg, p0 + rg + 4, ... for
// its query, with the membership test of the stream (FP32, FP64 within the
// margin) and exact distances; the four lanes of a query merge (D1, lowest
// index at D1 and its position, D2) and the in-band count.
struct ExactResult {
  int32_t d1, j1, p1, d2, cnt;
};
__device__ __forceinline__ ExactResult exact_tile(const GroupRefs& r, const Tile& T, bool qv,
                                                  int32_t p0, int32_t p1, int lane) {
  ExactResult o = {kDistInf, 0x7FFFFFFF, -1, kDistInf, 0};
  if (qv) {
    const uint8_t* qrow = r.a_desc + int64_t(T.i) * kDescBytes;
    for (int32_t p = p0 + (lane >> 4); p < p1; p += 4) {
      const int32_t j = r.cj[p];
      if (!member(r, band_dist32(T.a, T.b, T.c, r.cx[p], r.cy[p]), T.i, j)) continue;
      ++o.cnt;
      const int32_t nc = int32_t(r.cnc[p] >> kPosBits) - int32_t(kDistBias);
      const int32_t D = row_dist(qrow, r.b_desc + int64_t(j) * kDescBytes, T.nq, nc);
      if (D < o.d1 || (D == o.d1 && j < o.j1)) {
        o.d2 = o.d1;
        o.d1 = D;
        o.j1 = j;
        o.p1 = p;
      } else {
        o.d2 = min(o.d2, D);
      }
    }
  }
#pragma unroll
  for (int off = 16; off <= 32; off <<= 1) {
    const int32_t e1 = __shfl_xor(o.d1, off, 64), k1 = __shfl_xor(o.j1, off, 64);
    const int32_t q1 = __shfl_xor(o.p1, off, 64), e2 = __shfl_xor(o.d2, off, 64);
    o.cnt += __shfl_xor(o.cnt, off, 64);
    if (e1 < o.d1 || (e1 == o.d1 && k1 < o.j1)) {
      o.d2 = min(o.d1, e2);
      o.d1 = e1;
      o.j1 = k1;
      o.p1 = q1;
    } else {
      o.d2 = min(o.d2, e1);
    }
  }
  return o;
}

// Folds one decided candidate (key distance kd, pair position pos) into a
// running result.
__device__ __forceinline__ void fold_state(Tile& T, uint32_t kd, int32_t pos) {
  if (kd < T.s1) {
    T.s2 = T.s1;
    T.s1 = kd;
    T.p1 = pos;
    T.tie = false;
  } else if (kd == T.s1) {
    T.s2 = T.s1;
    T.tie = true;
  } else {
    T.s2 = min(T.s2, kd);
  }
}

// End of a tile's chunk starting at pair position c0p: merge the four lanes
// of each query, then fold the chunk's two smallest into the running result.
// No memory access: a shared smallest distance only sets the tie flag.
__device__ __forceinline__ void close_chunk(Tile& T, int32_t c0p, int32_t c1p) {
#pragma unroll
  for (int o = 16; o <= 32; o <<= 1) {
    const uint32_t p1 = __shfl_xor(T.k1, o, 64);
    const uint32_t p2 = __shfl_xor(T.k2, o, 64);
    T.k2 = min(max(T.k1, p1), min(T.k2, p2));
    T.k1 = min(T.k1, p1);
  }
  const uint32_t kd1 = T.k1 >> kPosBits, kd2 = T.k2 >> kPosBits;
  const int32_t pf = int32_t(T.k1 & (kChunk - 1));
  const int32_t at = min(c0p + ((pf - c0p) & (kChunk - 1)), c1p - 1);
  if (kd1 < T.s1) {
    T.s2 = min(T.s1, kd2);
    T.s1 = kd1;
    T.p1 = at;
    T.tie = kd2 == kd1;
  } else if (kd1 == T.s1 && kd1 != kKeyDistInf) {
    T.s2 = T.s1;
    T.tie = true;
  } else {
    T.s2 = min(T.s2, kd1);
  }
  T.k1 = kKeyInf;
  T.k2 = kKeyInf;
}

// One group: up to 4 * TPW query tiles (TPW per wave) against their candidate
// ranges, read from the LDS buffer.  `gs` holds the group's query records and
// its first fill's row indices are in index buffer `par` (both issued by the
// previous group or the kernel's start).  The group issues the first stage of
// group gn (if gn >= 0) into the other index buffer.
template <bool kKeepCounts, int TPW>
__device__ __forceinline__ void match_group(const BatchView& v, const TileGroup& G, int32_t g,
                                            const GroupStart<TPW>& gs, int par, int32_t gn,
                                            GroupStart<TPW>& gsn, MatchLds& L, int w, int lane,
                                            WaveStats& ws) {
  const int col = lane & (kQueryTile - 1), rg = lane >> 4;
  const float lo = G.band_lo, hi = G.band_hi;
  const Stream s = make_stream(v, G, L);
  const int32_t nfill = (s.len + kBuf - 1) / kBuf;

  // Tile ranges (uniform, relative to s.base; steps start at rb + 16 i).
  Tile T[TPW];
  int32_t rb[TPW], re[TPW], c0[TPW];
  bool qv[TPW];
  // The record's tile ranges by scalar load at the uniform tile index.
  c_i32* gw = (c_i32*)(v.groups + g);
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    const int32_t tidx = tile_of<TPW>(w, k);
    const int32_t qs = (G.tile0 + tidx) * kQueryTile + col;
    qv[k] = tidx < G.ntiles && qs < G.na;
    int32_t tb = gw[offsetof(TileGroup, t_begin) / 4 + tidx];
    int32_t te = gw[offsetof(TileGroup, t_end) / 4 + tidx];
    if (tidx >= G.ntiles || te <= tb) tb = te = s.base;
    rb[k] = (tb & ~(kBlock - 1)) - s.base;
    re[k] = te - s.base;
    c0[k] = rb[k];
  }

  // This wave's own index loads (and everything before them) are complete;
  // the barrier also ends every wave's reads of the previous group's fill.
  wait_loads<0>();
  barrier();
  const int32_t nblk0 = min(s.len, kBuf) / kBlock;
  issue_rows(s, L, 0, nblk0, par, w, lane);
  nv4u qr[TPW][2];
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    T[k].a = qv[k] ? __uint_as_float(gs.qu[k].x) : NAN;
    T[k].b = __uint_as_float(gs.qu[k].y);
    T[k].c = __uint_as_float(gs.qu[k].z);
    T[k].i = int32_t(gs.qu[k].w);
    const uint8_t* qrow = G.a_desc + int64_t(T[k].i) * kDescBytes + 16 * rg;
    qr[k][0] = gload16(qrow);
    qr[k][1] = gload16(qrow + 64);
    T[k].nq = ((g_i32*)G.a_norm)[T[k].i];
  }
  // The next group's first stage: TPW query records and one index load.
  const bool next = gn >= 0;
  if (next) gsn = start_group<TPW>(v, load_group(v.groups, gn), L, par ^ 1, w, lane);
  // This wave's fill, then (after the barrier) every wave's; then the query rows.
  if (next)
    wait_loads<3 * TPW + TPW + 1>();
  else
    wait_loads<3 * TPW>();
  barrier();
  if (next)
    wait_loads<TPW + 1>();
  else
    wait_loads<0>();
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
#pragma unroll
    for (int m = 0; m < 2; ++m)
      T[k].bq[m] = v4i{neg_bytes(qr[k][m].x), neg_bytes(qr[k][m].y), neg_bytes(qr[k][m].z),
                       neg_bytes(qr[k][m].w)};
    T[k].k1 = T[k].k2 = kKeyInf;
    T[k].s1 = T[k].s2 = kKeyDistInf;
    T[k].p1 = 0;
    T[k].tie = false;
    T[k].cnt = 0;
  }

  uint32_t wcnt = 0;       // in-band slots of the wave (counts not kept per query)
  uint32_t wbl = 0;        // slots decided in FP64
  int32_t nbq = 0;         // queued FP64 decisions
  bool overflow = false;   // more than kBorderCap: the wave's tiles are recomputed exactly
  uint32_t nsteps = 0;     // 16 x 16 steps evaluated

  for (int32_t fi = 0; fi < nfill; ++fi) {
    const int32_t f = kBuf * fi;   // relative position of the fill's start
    if (fi > 0) {
      // A range longer than one fill: every wave is done with the previous
      // fill; load this one's indices, then its rows.
      barrier();
      issue_j(s, f, par, w, lane);
      wait_loads<0>();
      issue_rows(s, L, f, min(s.len - f, kBuf) / kBlock, par, w, lane);
      wait_loads<0>();
      barrier();
    }
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
      Tile& t = T[k];
      const int32_t p0 = max(rb[k], f);
      const int32_t pe = min(re[k], f + kBuf);
      if (p0 >= pe) continue;
      const int32_t n = (pe - p0 + kBlock - 1) / kBlock;
      nsteps += uint32_t(n);
      // Keys hold positions mod 1024: a chunk closes before a fill whose
      // steps would take it past 1024 positions.
      if (p0 + kBlock * n - c0[k] > kChunk) {
        close_chunk(t, s.base + c0[k], s.base + p0);
        c0[k] = p0;
      }
      // A operand: buffer row q + col of the step, k-slices rg and rg + 4
      // (chunk slots rg ^ (row & 7) and that ^ 4).  Metadata: the four
      // candidates 4 rg .. 4 rg + 3 of the step.  Both advance by 16 rows.
      const int32_t q0 = p0 - f;
      uint32_t oa = uint32_t((q0 + col) * kDescBytes + ((rg ^ ((q0 + col) & 7)) << 4));
      uint32_t om = uint32_t((q0 + 4 * rg) * 4);
      // The first step's operands; each step reads the next one's before
      // its own fold (the read after the last step wraps and is unused).
      const uint32_t oa0 = oa, om0 = om;
      v4i na0 = *reinterpret_cast<const v4i*>(&L.rows[oa]);
      v4i na1 = *reinterpret_cast<const v4i*>(&L.rows[oa ^ 64u]);
      float4 nxs = reinterpret_cast<const float4*>(L.x)[om >> 4];
      float4 nys = reinterpret_cast<const float4*>(L.y)[om >> 4];
      uint4 nns = reinterpret_cast<const uint4*>(L.nc)[om >> 4];
      // Steps of this fill (at most kBuf / 16) with a slot within the margin
      // of d: only marked here, so the loop keeps nothing live for them.
      static_assert(kBuf / kBlock <= 32, "one bit per step of a fill");
      uint32_t bsteps = 0;
      for (int32_t i = 0; i < n; ++i) {
        v4i acc = {0, 0, 0, 0};
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(na0, t.bq[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(na1, t.bq[1], acc, 0, 0, 0);
        const float xv[4] = {nxs.x, nxs.y, nxs.z, nxs.w};
        const float yv[4] = {nys.x, nys.y, nys.z, nys.w};
        const uint32_t nv[4] = {nns.x, nns.y, nns.z, nns.w};
        oa = (oa + kBlock * kDescBytes) & (kBuf * kDescBytes - 1);
        om = (om + 4 * kBlock) & (4 * kBuf - 1);
        na0 = *reinterpret_cast<const v4i*>(&L.rows[oa]);
        na1 = *reinterpret_cast<const v4i*>(&L.rows[oa ^ 64u]);
        nxs = reinterpret_cast<const float4*>(L.x)[om >> 4];
        nys = reinterpret_cast<const float4*>(L.y)[om >> 4];
        nns = reinterpret_cast<const uint4*>(L.nc)[om >> 4];
        unsigned long long border = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float d32 = band_dist32(t.a, t.b, t.c, xv[e], yv[e]);
          const bool mem = d32 <= lo;
          border |= __ballot(d32 <= hi) & ~__ballot(mem);
          const uint32_t kin = mem ? nv[e] + (uint32_t(acc[e]) << 11) : kKeyInf;
          t.k2 = umed3(t.k1, kin, t.k2);
          t.k1 = min(t.k1, kin);
          if (kKeepCounts)
            t.cnt += mem ? 1 : 0;
          else
            wcnt += __builtin_popcountll(__ballot(mem));
        }
        if (border) bsteps |= 1u << i;
      }
      // Rare: the marked steps again (the same operations, so the same keys),
      // queueing their slots within the margin of d with their exact keys and
      // indices in b for the FP64 decision after the group's tiles (the index
      // buffer holds the whole fill).
      while (bsteps) {
        const int32_t i = __builtin_ctz(bsteps);
        bsteps &= bsteps - 1;
        const uint32_t oai = (oa0 + uint32_t(i) * (kBlock * kDescBytes)) & (kBuf * kDescBytes - 1);
        const uint32_t omi = (om0 + uint32_t(i) * (4 * kBlock)) & (4 * kBuf - 1);
        const v4i a0 = *reinterpret_cast<const v4i*>(&L.rows[oai]);
        const v4i a1 = *reinterpret_cast<const v4i*>(&L.rows[oai ^ 64u]);
        const float4 xs = reinterpret_cast<const float4*>(L.x)[omi >> 4];
        const float4 ys = reinterpret_cast<const float4*>(L.y)[omi >> 4];
        const uint4 ns = reinterpret_cast<const uint4*>(L.nc)[omi >> 4];
        v4i acc = {0, 0, 0, 0};
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0, t.bq[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, t.bq[1], acc, 0, 0, 0);
        const float xv[4] = {xs.x, xs.y, xs.z, xs.w};
        const float yv[4] = {ys.x, ys.y, ys.z, ys.w};
        const uint32_t nv[4] = {ns.x, ns.y, ns.z, ns.w};
        unsigned long long bm[4];
        uint32_t keys[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float d32 = band_dist32(t.a, t.b, t.c, xv[e], yv[e]);
          bm[e] = __ballot(d32 <= hi) & ~__ballot(d32 <= lo);
          keys[e] = nv[e] + (uint32_t(acc[e]) << 11);
        }
        {
          const int32_t p = p0 + kBlock * i;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            if (!bm[e]) continue;
            const int32_t nb = __builtin_popcountll(bm[e]);
            wbl += uint32_t(nb);
            if (nbq + nb > kBorderCap) {
              overflow = true;
              continue;
            }
            const int32_t idx = nbq + int32_t(__builtin_amdgcn_mbcnt_hi(
                                          uint32_t(bm[e] >> 32),
                                          __builtin_amdgcn_mbcnt_lo(uint32_t(bm[e]), 0)));
            if ((bm[e] >> lane) & 1ull) {
              const int32_t pr = p + 4 * rg + e;        // relative position
              const int32_t bq = (pr - f) >> 4;          // block of the fill
              const int32_t jq = L.j[par][bq & (kWaves - 1)][kBlock * (bq >> 2) + (pr & 15)];
              L.queue[w][idx] = make_uint4(
                  keys[e], (uint32_t(pr) << 7) | (uint32_t(k) << 6) | uint32_t(lane),
                  uint32_t(jq), 0u);
            }
            nbq += nb;
          }
        }
      }
    }
  }

  // The last chunk of every tile, then the queued FP64 decisions (one per
  // lane), folded into the result of the lane with rg = 0 of their query.
#pragma unroll
  for (int k = 0; k < TPW; ++k)
    if (re[k] > rb[k]) close_chunk(T[k], s.base + c0[k], s.base + re[k]);
  const GroupRefs gr = group_refs(v, G);
  if (nbq > 0 && !overflow) {
    const uint4 en = L.queue[w][min(lane, nbq - 1)];
    const int owner = int(en.y & 63), ot = int((en.y >> 6) & 1);
    int32_t qi = 0;
#pragma unroll
    for (int k = 0; k < TPW; ++k) {
      const int32_t ik = __shfl(T[k].i, owner, 64);
      if (ot == k) qi = ik;
    }
    bool in = false;
    if (lane < nbq) {
      const int32_t j = int32_t(en.z);
      // The keypoints' and F's loads are independent: all are in flight together.
      const float xq = ldg(gr.a_xy + 2 * qi), yq = ldg(gr.a_xy + 2 * qi + 1);
      const float xb = ldg(gr.b_xy + 2 * j), yb = ldg(gr.b_xy + 2 * j + 1);
      in = band_dist64(gr.F, xq, yq, xb, yb) <= gr.d;
    }
    const unsigned long long inm = __ballot(in);
    if (!kKeepCounts) wcnt += __builtin_popcountll(inm);
    // Entry e is in lane e's registers: broadcast each member to its owner.
    unsigned long long todo = inm;
    while (todo) {
      const int e = __builtin_ctzll(todo);
      todo &= todo - 1;
      const uint32_t qx = __builtin_amdgcn_readlane(en.x, e);
      const uint32_t qy = __builtin_amdgcn_readlane(en.y, e);
      if (lane != int(qy & (kQueryTile - 1))) continue;
#pragma unroll
      for (int k = 0; k < TPW; ++k) {
        if (int((qy >> 6) & 1) == k) {
          fold_state(T[k], qx >> kPosBits, s.base + int32_t(qy >> 7));
          if (kKeepCounts) ++T[k].cnt;
        }
      }
    }
  }

  // Results (the binned position of the match) and statistics.
  int32_t tsum = 0;        // in-band slots of the tiles, by lane (counts kept or recomputed)
  uint32_t nacc = 0, ties = 0;
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    Tile& t = T[k];
    int32_t d1, d2, p1, qc = 0;
    if (overflow) {
      const ExactResult x = exact_tile(gr, t, qv[k], s.base + rb[k], s.base + re[k], lane);
      d1 = x.d1;
      d2 = x.d2;
      p1 = x.p1;
      qc = x.cnt;
      tsum += lane < kQueryTile && qv[k] ? qc : 0;
    } else {
      d1 = t.s1 != kKeyDistInf ? int32_t(t.s1) - int32_t(kDistBias) + t.nq : kDistInf;
      d2 = t.s2 != kKeyDistInf ? int32_t(t.s2) - int32_t(kDistBias) + t.nq : kDistInf;
      p1 = d1 != kDistInf ? t.p1 : -1;
      // Equal smallest distances: the lowest index of b, exactly.
      unsigned long long tmask = __ballot(t.tie && qv[k] && lane < kQueryTile);
      while (tmask) {
        const int Lq = __builtin_ctzll(tmask);
        tmask &= tmask - 1;
        ++ties;
        const int32_t pb = lowest_tied(gr, __shfl(t.a, Lq, 64), __shfl(t.b, Lq, 64),
                                       __shfl(t.c, Lq, 64), __shfl(t.i, Lq, 64),
                                       __shfl(t.nq, Lq, 64), __shfl(d1, Lq, 64),
                                       s.base + rb[k], s.base + re[k], lane);
        if (lane == Lq) p1 = pb;
      }
      if (kKeepCounts) {
        qc = t.cnt;
        qc += __shfl_xor(qc, 16, 64);
        qc += __shfl_xor(qc, 32, 64);
        tsum += lane < kQueryTile && qv[k] ? qc : 0;
      }
    }
    bool accept;
    if (d2 != kDistInf) {
      accept = int64_t(v.ratio_den) * d1 < int64_t(v.ratio_num) * d2;
    } else {
      accept = d1 != kDistInf && v.accept_single;
    }
    if (qv[k] && lane < kQueryTile) {
      QueryResult out;
      out.match = d1 != kDistInf ? p1 : -1;
      out.d1 = d1;
      out.d2 = d2;
      out.flags = (accept ? 1 : 0) | (kKeepCounts ? (qc << 1) : 0);
      v.res[G.q_off + t.i] = out;
    }
    nacc += __builtin_popcountll(__ballot(accept && qv[k] && lane < kQueryTile));
  }
  for (int o = 8; o > 0; o >>= 1) tsum += __shfl_xor(tsum, o, 64);
  tsum = __shfl(tsum, 0, 64);
  // Without per-query counts the wave counted in-band slots itself (unless
  // its tiles were recomputed).
  if (!kKeepCounts && !overflow) tsum = int32_t(wcnt);
  if (G.pair != ws.pair) {
    flush_stats(v, ws, lane);
    ws.pair = G.pair;
  }
  ws.comparisons += (unsigned long long)tsum;
  ws.borderline += wbl;
  ws.elements += (unsigned long long)nsteps * (kQueryTile * kQueryTile);
  ws.accepted += nacc;
  ws.ties += ties;
}

// One resident wave of workgroups.  Preparation splits the groups into
// kXcds contiguous shares of about equal estimated cost, one per XCD (each
// XCD has its own L2).
#ifndef SFM_MATCH_WAVES_PER_EU
#define SFM_MATCH_WAVES_PER_EU 4
#endif
template <bool kKeepCounts, int TPW>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(SFM_MATCH_WAVES_PER_EU, 8)))
void match_kernel(BatchView v) {
  __shared__ __attribute__((aligned(16))) MatchLds lds;
  // The wave index is uniform: readfirstlane lets the compiler keep
  // everything derived from it (tile ranges, queue counts) in SGPRs.
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  // Workgroup k runs on XCD x = k mod 8 (workgroups are dealt to the XCDs
  // round-robin) and takes every W-th group of share x, W being the number of
  // workgroups on that XCD.
  const int32_t shares = min(kXcds, int32_t(gridDim.x));
  const int32_t x = blockIdx.x % shares, i = blockIdx.x / shares;
  const int32_t W = (int32_t(gridDim.x) - x + shares - 1) / shares;
  const int32_t g_first = ((c_i32*)v.wg_start)[x] + i;
  const int32_t g_end = ((c_i32*)v.wg_start)[x + 1];
  WaveStats ws = {-1, 0, 0, 0, 0, 0};
  if (g_first < g_end) {
    GroupStart<TPW> gs = start_group<TPW>(v, load_group(v.groups, g_first), lds, 0, wave, lane);
    int par = 0;
    for (int32_t g = g_first; g < g_end; g += W) {
      const TileGroup G = load_group(v.groups, g);
      GroupStart<TPW> gsn;
      match_group<kKeepCounts, TPW>(v, G, g, gs, par, g + W < g_end ? g + W : -1, gsn, lds,
                                    wave, lane, ws);
      gs = gsn;
      par ^= 1;
    }
  }
  flush_stats(v, ws, lane);
}

// Diagnostic of the FP32 band test: over every (query, candidate) slot of
// every query tile's candidate range whose FP64 distance is at most 2d, the
// largest |FP32 distance - FP64 distance| (as the bits of a non-negative
// double, which order like the integers) and the number of such slots.  One
// wave per tile, one lane per query.
__global__ __launch_bounds__(64) void band_error_kernel(BatchView v, unsigned long long* out) {
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
    const double* F = v.F + 9 * int64_t(G.pair);
    const float* cx = v.cand_x + G.c_off;
    const float* cy = v.cand_y + G.c_off;
    const int32_t* cj = v.cand_j + G.c_off;
    const double two_d = 2.0 * G.band;
    const float xq = G.a_xy[2 * qr.i], yq = G.a_xy[2 * qr.i + 1];
    for (int32_t s = b; s < e; ++s) {
      const int32_t j = cj[s];
      const double e64 = band_dist64(F, xq, yq, G.b_xy[2 * j], G.b_xy[2 * j + 1]);
      if (!(e64 <= two_d)) continue;
      const double e32 = band_dist32(qr.a, qr.b, qr.c, cx[s], cy[s]);
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
template <int TPW>
static int32_t resident_workgroups(int dev) {
  static int32_t cached[64] = {0};
  if (dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, match_kernel<false, TPW>,
                                                     64 * kWaves, 0) != hipSuccess ||
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
  const int32_t r = group_tiles == kWaves ? resident_workgroups<1>(device)
                                          : resident_workgroups<2>(device);
  return int32_t(std::max<int64_t>(1, std::min<int64_t>(groups, r)));
}

template <int TPW>
static void launch_match_t(const BatchView& v, int32_t wgs, hipStream_t st) {
  if (v.keep_counts)
    hipLaunchKernelGGL((match_kernel<true, TPW>), dim3(wgs), dim3(64 * kWaves), 0, st, v);
  else
    hipLaunchKernelGGL((match_kernel<false, TPW>), dim3(wgs), dim3(64 * kWaves), 0, st, v);
}

hipError_t launch_match(const BatchView& v, int32_t wgs, hipStream_t st) {
  if (wgs <= 0) return hipSuccess;
  if (v.group_tiles == kWaves)
    launch_match_t<1>(v, wgs, st);
  else
    launch_match_t<2>(v, wgs, st);
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
