// Exhaustive two-nearest matching: every feature of b is a candidate of every
// query of a (the band of eqs. (2)-(3) ignored).  The comparison point of
// Section 6 and the matcher of both stages of staged coarse matching (Section 4).
//
// Work item: (pair, block of 256 queries, slice of up to 1024 targets starting
// at a multiple of 1024).  A workgroup of four waves takes one item:
//   - Wave w owns queries 64 w .. 64 w + 63 of the block as four 16-query
//     tiles; their negated rows are the resident B operands of
//     v_mfma_i32_16x16x64_i8 (two per tile: bytes 0..63 and 64..127).
//   - The slice's rows stream through two LDS buffers of 128 targets by LDS
//     DMA (rows XOR-swizzled: chunk c of row r at slot c ^ (r & 7)); the next
//     buffer loads while the current one is used, one barrier per buffer.
//     Targets past n_b read a zero row, so their products are 0.
//   - Per 16-target step: eight MFMAs give -q.c for 16 targets x 64 queries,
//     then each lane folds its four results per tile into its two smallest
//         key = ((||c||^2 - 2 q.c + 2^21) << 10) | (target mod 1024)
//     with one v_med3_u32 and one v_min_u32 (padding targets carry the key
//     0xFFFFFFFF).
// Keys are unique within a slice, and at equal distance the lower index has
// the smaller key, so a slice's smallest key names the lowest index at the
// smallest distance.  The slice's two smallest keys of every query go to a
// partial-result array; the merge kernel folds a query's slices in ascending
// order (the earlier slice keeps a shared smallest distance), adds ||q||^2
// and applies the ratio test.
#include <algorithm>

#include "sfm_internal.h"

namespace sfm {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned int nv4u __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) nv4u g_nv4u;
typedef const __attribute__((address_space(1))) int32_t g_i32;
typedef int v2i __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) v2i g_v2i;
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) v2u g_v2u;
typedef __attribute__((address_space(3))) void lds_void;

constexpr int kExWaves = 4;
constexpr int kExTiles = 4;                                    // 16-query tiles per wave
constexpr int32_t kExQueries = kExWaves * kExTiles * kQueryTile;   // queries per work item
constexpr int32_t kExSlice = kChunk;                           // targets per work item
constexpr int kExBuf = 128;                                    // targets per LDS buffer
constexpr int kExRowsPerWave = kExBuf / kExWaves;              // rows one wave fetches per buffer
constexpr int kExSteps = kExBuf / kQueryTile;                  // 16-target steps per buffer
static_assert(kExQueries == 256 && kExSlice == 1024, "the size limits of item indices");
static_assert(int64_t(kExhaustiveMaxQueries) <= int64_t(32767) * kExQueries &&
                  int64_t(kExhaustiveMaxTargets) <= int64_t(65535) * kExSlice,
              "query blocks fit 15 bits, slices 16");
static_assert(kExSlice % kExBuf == 0 && kExBuf % kQueryTile == 0, "whole steps per buffer");
static_assert(kExRowsPerWave % 8 == 0, "one DMA instruction fetches eight rows");
constexpr uint32_t kExKeyDistInf = kKeyInf >> kPosBits;

// Two buffers of rows and keys' norm words: 33 KB, four workgroups per CU.
struct ExLds {
  uint8_t rows[2][kExBuf * kDescBytes];
  uint32_t nc[2][kExBuf];
};
static_assert(sizeof(ExLds) <= 40960, "four workgroups per CU");

// The DMA source of targets past n_b.
__device__ __attribute__((aligned(16))) const uint8_t zero_row[kDescBytes] = {};

__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

// Waits for all of this wave's vector-memory operations (LDS DMA included).
__device__ __forceinline__ void wait_all_loads() {
  compiler_fence();
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt and lgkmcnt untouched
  compiler_fence();
}

__device__ __forceinline__ void barrier() {
  compiler_fence();
  __builtin_amdgcn_s_barrier();
  compiler_fence();
}

// LDS DMA of 16 bytes per lane: lane l's bytes at src land at LDS offset
// lds_off + 16 l (lds_off wave-uniform).  Inline asm with M0 set in the same
// statement; the kernel orders these writes itself (wait_all_loads, barrier).
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void dma16(const void* src, uint32_t lds_off) {
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off"
               :: "s"(__builtin_amdgcn_readfirstlane(lds_off)), "v"(src) : "memory", "m0");
}
// The same with a uniform base address in SGPRs plus a 32-bit lane offset:
// no per-lane address arithmetic.
__device__ __forceinline__ void dma16s(const void* base, uint32_t voff, uint32_t lds_off) {
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %2"
               :: "s"(__builtin_amdgcn_readfirstlane(lds_off)), "v"(voff), "s"(base)
               : "memory", "m0");
}
#pragma clang diagnostic pop

// Per-byte negation of four bytes in 0..127 (no borrow crosses a byte).
__device__ __forceinline__ int neg_bytes(uint32_t w) {
  return int((0x80808080u - w) ^ 0x80808080u);
}

__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c) {
  return max(min(a, b), min(max(a, b), c));   // selects v_med3_u32
}

// Rows of targets t .. t + kExBuf - 1 into the buffer at LDS offset
// lds_rows: wave w fetches rows
// kExRowsPerWave w .. + kExRowsPerWave - 1, eight per instruction (lane l:
// row 8 u + (l >> 3), chunk (l & 7) ^ (row & 7), landing at slot l & 7).
// A buffer wholly inside b takes the base-address form: the lane's offset
// voff = (kExRowsPerWave w + (l >> 3)) * 128 + 16 ((l & 7) ^ (l >> 3)) is the
// same for every buffer and instruction (row 8 u + (l >> 3) of the wave's
// rows: the base advances by 8 rows per instruction).
__device__ __forceinline__ void issue_rows(const uint8_t* b_desc, int32_t nb, int32_t t,
                                           uint32_t lds_rows, uint32_t voff, int w, int lane) {
  const uint32_t lw = lds_rows + uint32_t(kExRowsPerWave * w * kDescBytes);
  if (t + kExBuf <= nb) {
    const uint8_t* base = b_desc + int64_t(t) * kDescBytes;
#pragma unroll
    for (int u = 0; u < kExRowsPerWave / 8; ++u)
      dma16s(base + 8 * u * kDescBytes, voff, lw + uint32_t(8 * u * kDescBytes));
    return;
  }
#pragma unroll
  for (int u = 0; u < kExRowsPerWave / 8; ++u) {
    const int r = kExRowsPerWave * w + 8 * u + (lane >> 3);
    const int c = (lane & 7) ^ (r & 7);
    const int32_t j = t + r;
    const uint8_t* src = j < nb ? b_desc + int64_t(j) * kDescBytes + 16 * c : zero_row + 16 * c;
    dma16(src, lw + uint32_t(8 * u * kDescBytes));
  }
}

// The norm word of target j of the slice (threads 0 .. kExBuf - 1 of the
// workgroup, one target each): ((||c||^2 + 2^21) << 10) | (j mod 1024), or
// the largest key past n_b.
__device__ __forceinline__ uint32_t norm_word(const int32_t* norm2, int32_t nb, int32_t j) {
  const int32_t n = ((g_i32*)norm2)[min(j, nb - 1)];
  return j < nb ? ((uint32_t(n) + kDistBias) << kPosBits) | uint32_t(j & (kChunk - 1)) : kKeyInf;
}

// Eight MFMAs of one step: -q.c for the step's 16 targets (the lane's
// chunks of k-half 0 at a0, of k-half 1 at a1) and the wave's four query tiles.
__device__ __forceinline__ void mfma_step(const uint8_t* a0p, const uint8_t* a1p,
                                          const v4i (&bq)[kExTiles][2], v4i (&acc)[kExTiles]) {
  const v4i a0 = *reinterpret_cast<const v4i*>(a0p);
  const v4i a1 = *reinterpret_cast<const v4i*>(a1p);
#pragma unroll
  for (int k = 0; k < kExTiles; ++k) {
    acc[k] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0, bq[k][0], v4i{0, 0, 0, 0}, 0, 0, 0);
    acc[k] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, bq[k][1], acc[k], 0, 0, 0);
  }
}

// The lane's four results per tile into its two smallest keys (nw: the norm
// words of the lane's four targets).
__device__ __forceinline__ void fold_step(const uint32_t* nw, const v4i (&acc)[kExTiles],
                                          uint32_t (&k1)[kExTiles], uint32_t (&k2)[kExTiles]) {
  const uint4 nn = *reinterpret_cast<const uint4*>(nw);
  const uint32_t nv[4] = {nn.x, nn.y, nn.z, nn.w};
#pragma unroll
  for (int k = 0; k < kExTiles; ++k) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t key = nv[e] + (uint32_t(acc[k][e]) << 11);
      k2[k] = umed3(k1[k], key, k2[k]);
      k1[k] = min(k1[k], key);
    }
  }
}

__global__ __launch_bounds__(64 * kExWaves) __attribute__((amdgpu_waves_per_eu(4, 8)))
void exhaustive_kernel(BatchView v, const int2* items, int32_t n_items, uint2* part) {
  __shared__ __attribute__((aligned(128))) ExLds lds;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int tid = threadIdx.x;
  // The per-pair counters the merge kernel adds its accepted queries to:
  // workgroup k resets pairs 256 k .. 256 k + 255.
  {
    const int32_t p = int32_t(blockIdx.x) * (64 * kExWaves) + tid;
    if (p < v.n_pairs) {
      const PairDesc P = v.pairs[p];
      const int64_t nqb = (P.na + kExQueries - 1) / kExQueries;
      const int64_t tail = P.nb - int64_t(kExSlice) * ((P.nb - 1) / kExSlice);
      PairCounters c;
      c.comparisons = (unsigned long long)(int64_t(P.na) * P.nb);
      c.elements = P.nb > 0 ? (unsigned long long)(nqb * kExQueries *
                                                   (P.nb - tail + ((tail + 15) & ~int64_t(15))))
                            : 0ull;
      c.borderline = 0;
      c.accepted = 0;
      c.ties = 0;
      v.counters[p] = c;
    }
  }
  if (int32_t(blockIdx.x) >= n_items) return;
  const v2i it = ((g_v2i*)items)[blockIdx.x];
  const int32_t p = __builtin_amdgcn_readfirstlane(it.x);
  const int32_t qb = __builtin_amdgcn_readfirstlane(it.y) >> 16;
  const int32_t s = __builtin_amdgcn_readfirstlane(it.y) & 0xFFFF;
  const PairDesc P = v.pairs[p];
  const ImageDev A = v.images[P.a], B = v.images[P.b];
  const int32_t t0 = s * kExSlice;
  const int32_t cnt = min(kExSlice, P.nb - t0);
  const int32_t nfill = (cnt + kExBuf - 1) / kExBuf;
  const uint32_t lbase = uint32_t(reinterpret_cast<uintptr_t>((lds_void*)&lds));
  const uint32_t lrows = lbase + uint32_t(offsetof(ExLds, rows));

  // The first buffer, the wave's query rows and the first norm words.
  const uint32_t voff = uint32_t((kExRowsPerWave * w + (lane >> 3)) * kDescBytes +
                                 16 * ((lane & 7) ^ ((lane >> 3) & 7)));
  issue_rows(B.desc, P.nb, t0, lrows, voff, w, lane);
  const int col = lane & (kQueryTile - 1), g = lane >> 4;
  const int32_t qw = qb * kExQueries + kExTiles * kQueryTile * w;   // the wave's first query
  nv4u qr[kExTiles][2];
#pragma unroll
  for (int k = 0; k < kExTiles; ++k) {
    const int32_t i = min(qw + kQueryTile * k + col, P.na - 1);
    const uint8_t* row = A.desc + int64_t(i) * kDescBytes + 16 * g;
    qr[k][0] = *(g_nv4u*)row;
    qr[k][1] = *(g_nv4u*)(row + 64);
  }
  uint32_t nw = tid < kExBuf ? norm_word(B.norm2, P.nb, t0 + tid) : 0u;
  if (tid < kExBuf) lds.nc[0][tid] = nw;
  v4i bq[kExTiles][2];
#pragma unroll
  for (int k = 0; k < kExTiles; ++k)
#pragma unroll
    for (int h = 0; h < 2; ++h)
      bq[k][h] = v4i{neg_bytes(qr[k][h].x), neg_bytes(qr[k][h].y), neg_bytes(qr[k][h].z),
                     neg_bytes(qr[k][h].w)};
  uint32_t k1[kExTiles], k2[kExTiles];
#pragma unroll
  for (int k = 0; k < kExTiles; ++k) k1[k] = k2[k] = kKeyInf;
  wait_all_loads();
  barrier();

  for (int32_t f = 0; f < nfill; ++f) {
    const int cur = f & 1;
    const int32_t tf = t0 + kExBuf * f;   // first target of this buffer
    const bool more = f + 1 < nfill;
    // The next buffer: its rows by DMA, its norm words into a register.
    if (more) {
      issue_rows(B.desc, P.nb, tf + kExBuf, lrows + uint32_t((cur ^ 1) * kExBuf * kDescBytes),
                 voff, w, lane);
      if (tid < kExBuf) nw = norm_word(B.norm2, P.nb, tf + kExBuf + tid);
    }
    // A wave whose queries all lie past n_a only fetches its share of the
    // buffers and meets the barriers.
    const int32_t nsteps =
        qw < P.na ? (min(kExBuf, t0 + cnt - tf) + kQueryTile - 1) / kQueryTile : 0;
    // Step i: A operand from buffer row 16 i + col, k-slices g and g + 4
    // (chunk slots g ^ (row & 7) and that ^ 4); norm words of rows
    // 16 i + 4 g .. + 3.  A whole buffer runs unrolled with step i + 1's
    // MFMAs issued before step i's fold, so the matrix core's work can
    // overlap the fold; a partial buffer (the end of b) runs step by step.
    const uint8_t* r0 = lds.rows[cur] + col * kDescBytes + ((g ^ (col & 7)) << 4);
    const uint8_t* r1 = lds.rows[cur] + col * kDescBytes + (((g ^ (col & 7)) ^ 4) << 4);
    const uint32_t* nb4 = lds.nc[cur] + 4 * g;
    constexpr int kStepBytes = kQueryTile * kDescBytes;
    if (nsteps == kExSteps) {
      v4i acc[2][kExTiles];
      mfma_step(r0, r1, bq, acc[0]);
#pragma unroll
      for (int i = 0; i < kExSteps; ++i) {
        if (i + 1 < kExSteps)
          mfma_step(r0 + (i + 1) * kStepBytes, r1 + (i + 1) * kStepBytes, bq, acc[(i + 1) & 1]);
        fold_step(nb4 + i * kQueryTile, acc[i & 1], k1, k2);
      }
    } else {
      for (int32_t i = 0; i < nsteps; ++i) {
        v4i acc[kExTiles];
        mfma_step(r0 + i * kStepBytes, r1 + i * kStepBytes, bq, acc);
        fold_step(nb4 + i * kQueryTile, acc, k1, k2);
      }
    }
    if (more) {
      // Every wave is done with the other buffer (last barrier); this one's
      // reads end at the barrier below, after which the next buffer is whole.
      if (tid < kExBuf) lds.nc[cur ^ 1][tid] = nw;
      wait_all_loads();
      barrier();
    }
  }

  // The four lanes of each query merge their two smallest; lanes 0..15 write.
  uint2* pp = part + P.ex_off + int64_t(s) * P.na;
#pragma unroll
  for (int k = 0; k < kExTiles; ++k) {
#pragma unroll
    for (int o = 16; o <= 32; o <<= 1) {
      const uint32_t p1 = __shfl_xor(k1[k], o, 64), p2 = __shfl_xor(k2[k], o, 64);
      k2[k] = min(max(k1[k], p1), min(k2[k], p2));
      k1[k] = min(k1[k], p1);
    }
    const int32_t i = qw + kQueryTile * k + col;
    if (g == 0 && i < P.na) pp[i] = make_uint2(k1[k], k2[k]);
  }
}

// One thread per query: fold the pair's slices in ascending order (strictly
// smaller replaces, so the earlier slice keeps a shared smallest distance and
// the second distance becomes equal to it), then the ratio test and the
// per-query result (the index in b).
constexpr int kMergeThreads = 256;
constexpr int kMergeBatch = 8;
__global__ __launch_bounds__(kMergeThreads) void exhaustive_merge_kernel(BatchView v,
                                                                         const uint2* part) {
  const int32_t p = int32_t(blockIdx.x);
  const PairDesc P = v.pairs[p];
  const int32_t i = int32_t(blockIdx.y) * kMergeThreads + int32_t(threadIdx.x);
  bool accept = false;
  if (i < P.na) {
    const int32_t nsl = (P.nb + kExSlice - 1) / kExSlice;
    const uint2* pp = part + P.ex_off + i;
    uint32_t s1 = kExKeyDistInf, s2 = kExKeyDistInf;
    int32_t j1 = -1;
    // kMergeBatch slices' loads in flight together (clamped past the last).
    for (int32_t s0 = 0; s0 < nsl; s0 += kMergeBatch) {
      v2u kk[kMergeBatch];
#pragma unroll
      for (int b = 0; b < kMergeBatch; ++b)
        kk[b] = *(g_v2u*)(pp + int64_t(min(s0 + b, nsl - 1)) * P.na);
#pragma unroll
      for (int b = 0; b < kMergeBatch; ++b) {
        if (s0 + b >= nsl) break;
        const uint32_t kd1 = kk[b].x >> kPosBits, kd2 = kk[b].y >> kPosBits;
        if (kd1 < s1) {
          s2 = min(s1, kd2);
          s1 = kd1;
          j1 = (s0 + b) * kExSlice + int32_t(kk[b].x & (kChunk - 1));
        } else if (kd1 == s1) {
          s2 = s1;
        } else {
          s2 = min(s2, kd1);
        }
      }
    }
    const int32_t nq = v.images[P.a].norm2[i];
    const int32_t d1 = s1 != kExKeyDistInf ? int32_t(s1) - int32_t(kDistBias) + nq : kDistInf;
    const int32_t d2 = s2 != kExKeyDistInf ? int32_t(s2) - int32_t(kDistBias) + nq : kDistInf;
    if (d2 != kDistInf)
      accept = int64_t(v.ratio_den) * d1 < int64_t(v.ratio_num) * d2;
    else
      accept = d1 != kDistInf && v.accept_single;
    QueryResult r;
    r.match = d1 != kDistInf ? j1 : -1;
    r.d1 = d1;
    r.d2 = d2;
    r.flags = (accept ? 1 : 0) | (v.keep_counts ? (P.nb << 1) : 0);
    v.res[P.q_off + i] = r;
  }
  const unsigned long long m = __ballot(accept);
  if ((threadIdx.x & 63) == 0 && m)
    atomicAdd(&v.counters[p].accepted, uint32_t(__builtin_popcountll(m)));
}

}  // namespace

void exhaustive_plan(PairDesc* pd, int32_t n_pairs, int2* items, int64_t* n_items,
                     int64_t* n_part) {
  int64_t ni = 0, np = 0;
  for (int32_t k = 0; k < n_pairs; ++k) {
    PairDesc& P = pd[k];
    P.ex_off = np;
    const int32_t nqb = (P.na + kExQueries - 1) / kExQueries;
    const int32_t nsl = (P.nb + kExSlice - 1) / kExSlice;
    np += int64_t(P.na) * nsl;
    for (int32_t s = 0; s < nsl; ++s)
      for (int32_t qb = 0; qb < nqb; ++qb) {
        if (items) items[ni] = make_int2(k, (qb << 16) | s);
        ++ni;
      }
  }
  *n_items = ni;
  *n_part = np;
}

hipError_t launch_exhaustive(const BatchView& v, const int2* items, int64_t n_items, uint2* part,
                             hipStream_t st) {
  if (v.n_pairs <= 0) return hipSuccess;
  const int64_t zero_wgs = (int64_t(v.n_pairs) + 64 * kExWaves - 1) / (64 * kExWaves);
  const int64_t wgs = std::max(n_items, zero_wgs);
  if (wgs > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(exhaustive_kernel, dim3(uint32_t(wgs)), dim3(64 * kExWaves), 0, st, v, items,
                     int32_t(std::min<int64_t>(n_items, INT32_MAX)), part);
  const uint32_t chunks =
      uint32_t(std::max(1, (v.max_na + kMergeThreads - 1) / kMergeThreads));
  hipLaunchKernelGGL(exhaustive_merge_kernel, dim3(uint32_t(v.n_pairs), chunks),
                     dim3(kMergeThreads), 0, st, v, part);
  return hipGetLastError();
}

}  // namespace sfm
