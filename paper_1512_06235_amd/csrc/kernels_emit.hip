// Ordered emission of accepted matches (a7).
//
// Per pair: a prefix over pairs gives each pair's first output row; then one
// workgroup per pair compacts its accepted queries in ascending query index
// with a ballot + mbcnt prefix inside each wave and a scan over waves.
#include "sfm_internal.h"

namespace sfm {
namespace {

constexpr int kEmitThreads = 1024;

// offset[pb + k + 1] = offset[pb] + sum of accepted over pairs pb..pb+k.
__global__ __launch_bounds__(1024) void scan_pairs_kernel(BatchView v, int32_t pb, int32_t pc,
                                                          int64_t* offset, int64_t* n_cmp) {
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
    if (t == blockDim.x - 1) carry = before + x;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kEmitThreads) void emit_kernel(BatchView v, int32_t pb,
                                                            const int64_t* offset, int32_t* oq,
                                                            int32_t* om, int32_t* od1,
                                                            int32_t* od2, int32_t* am,
                                                            int32_t* ad1, int32_t* ad2,
                                                            int32_t* ac) {
  __shared__ int32_t wtot[kEmitThreads / 64];
  __shared__ int32_t run;
  const int32_t p = pb + blockIdx.x;
  const PairDesc P = v.pairs[p];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t out0 = offset[p];
  if (t == 0) run = 0;
  __syncthreads();
  for (int32_t base = 0; base < P.na; base += kEmitThreads) {
    const int32_t i = base + t;
    QueryResult r;
    r.match = -1; r.d1 = r.d2 = kDistInf; r.flags = 0;
    if (i < P.na) r = v.res[P.q_off + i];
    const bool acc = (r.flags & 1) != 0;
    if (am && i < P.na) {
      am[P.q_off + i] = r.match;
      ad1[P.q_off + i] = r.d1;
      ad2[P.q_off + i] = r.d2;
      ac[P.q_off + i] = r.flags >> 1;
    }
    const unsigned long long m = __ballot(acc);
    const int32_t pre = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32),
                                                  __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0));
    if (lane == 0) wtot[wv] = __builtin_popcountll(m);
    __syncthreads();
    int32_t before = run;
    for (int w = 0; w < wv; ++w) before += wtot[w];
    if (acc) {
      const int64_t row = out0 + before + pre;
      oq[row] = i;
      om[row] = r.match;
      od1[row] = r.d1;
      od2[row] = r.d2;
    }
    __syncthreads();
    if (t == 0) {
      int32_t s = 0;
      for (int w = 0; w < kEmitThreads / 64; ++w) s += wtot[w];
      run += s;
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_emit(const BatchView& v, int32_t pb, int32_t pc, int64_t* offset, int32_t* oq,
                       int32_t* om, int32_t* od1, int32_t* od2, int64_t* n_cmp, int32_t* am,
                       int32_t* ad1, int32_t* ad2, int32_t* ac, hipStream_t st) {
  if (pc <= 0) return hipSuccess;
  hipLaunchKernelGGL(scan_pairs_kernel, dim3(1), dim3(1024), 0, st, v, pb, pc, offset, n_cmp);
  hipLaunchKernelGGL(emit_kernel, dim3(pc), dim3(kEmitThreads), 0, st, v, pb, offset, oq, om, od1,
                     od2, am, ad1, ad2, ac);
  return hipGetLastError();
}

}  // namespace sfm
