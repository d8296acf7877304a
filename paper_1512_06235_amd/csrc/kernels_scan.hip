// Device-wide prefix sums of int32 arrays (exclusive or inclusive), shared by
// the covisibility, grid-grouping, radix-sort and track kernels: each block
// of 8192 items is scanned in registers and LDS, the block sums are scanned
// by one block, and a last pass adds each block's offset.
#include <algorithm>

#include "sfm_internal.h"

namespace sfm {
namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;                            // items per thread of one scan block
constexpr int kScanBlock = kScanThreads * kScanPer;    // items per scan block

// Scan of one block of kScanBlock items; block sums to `sums`.  In place is
// allowed (each thread reads its items before writing them).
__global__ __launch_bounds__(kScanThreads) void scan_block_kernel(const int32_t* in,
                                                                  int32_t* out, int64_t n,
                                                                  int32_t* sums, int inclusive) {
  __shared__ int32_t wtot[kScanThreads / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t base = int64_t(blockIdx.x) * kScanBlock + int64_t(t) * kScanPer;
  int32_t v[kScanPer];
  int32_t run = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    run += v[k];
  }
  int32_t x = run;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wtot[wv] = x;
  __syncthreads();
  int32_t before = 0;
  for (int w = 0; w < wv; ++w) before += wtot[w];
  int32_t acc = before + x - run;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    acc += inclusive ? v[k] : 0;
    if (base + k < n) out[base + k] = acc;
    acc += inclusive ? 0 : v[k];
  }
  if (t == kScanThreads - 1) sums[blockIdx.x] = before + x;
}

// In place exclusive scan of the block sums (one block; at most kScanBlock).
__global__ __launch_bounds__(kScanThreads) void scan_sums_kernel(int32_t* sums, int32_t nb) {
  __shared__ int32_t wtot[kScanThreads / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int32_t v[kScanPer];
  int32_t run = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int32_t i = t * kScanPer + k;
    v[k] = i < nb ? sums[i] : 0;
    run += v[k];
  }
  int32_t x = run;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wtot[wv] = x;
  __syncthreads();
  int32_t before = 0;
  for (int w = 0; w < wv; ++w) before += wtot[w];
  int32_t acc = before + x - run;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int32_t i = t * kScanPer + k;
    if (i < nb) sums[i] = acc;
    acc += v[k];
  }
}

// Adds each block's offset; also writes a copy when `copy` is not NULL.
__global__ __launch_bounds__(256) void scan_add_kernel(int32_t* out, int64_t n,
                                                       const int32_t* sums, int32_t* copy) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t v = out[i] + sums[i / kScanBlock];
    out[i] = v;
    if (copy) copy[i] = v;
  }
}

}  // namespace

int64_t scan_limit() { return int64_t(kScanBlock) * kScanBlock; }

size_t scan_temp_bytes(int64_t n) {
  return sizeof(int32_t) * size_t(std::max<int64_t>(1, (n + kScanBlock - 1) / kScanBlock));
}

hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t n, bool inclusive,
                       int32_t* sums, int32_t* copy, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > scan_limit()) return hipErrorInvalidValue;
  const int32_t nb = int32_t((n + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(scan_block_kernel, dim3(nb), dim3(kScanThreads), 0, st, in, out, n, sums,
                     inclusive ? 1 : 0);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanThreads), 0, st, sums, nb);
  const int32_t blocks = int32_t(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65535)));
  hipLaunchKernelGGL(scan_add_kernel, dim3(blocks), dim3(256), 0, st, out, n, sums, copy);
  return hipGetLastError();
}

}  // namespace sfm
