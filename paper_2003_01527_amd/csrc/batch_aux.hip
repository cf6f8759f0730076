// Helper kernels of the batched driver: per-query pair totals of a level's
// rows, and retirement of the rows of queries taken out of the shared
// launches.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gsm_internal.h"

namespace gsm {

namespace {

constexpr int kAuxWG = 256;
constexpr int kAuxRun = 64;  // consecutive rows per thread

// qpairs[q] += W[r] over rows r < *n of query q.  Rows of one query sit
// together (first frontiers are written query by query and every tile keeps
// its survivors in order), so each thread sums a run of consecutive rows and
// adds once per change of query.
__global__ __launch_bounds__(kAuxWG) void k_query_pairs(const uint32_t *W, const uint16_t *qid,
                                                        const uint64_t *n_dev, uint64_t *qpairs) {
  const uint64_t N = *n_dev;
  const uint64_t stride = (uint64_t)gridDim.x * kAuxWG * kAuxRun;
  for (uint64_t b = ((uint64_t)blockIdx.x * kAuxWG + threadIdx.x) * kAuxRun; b < N; b += stride) {
    const uint64_t e = min(N, b + kAuxRun);
    uint32_t cur = qid[b];
    uint64_t acc = 0;
    for (uint64_t r = b; r < e; ++r) {
      const uint32_t q = qid[r];
      if (q != cur) {
        if (acc) atomicAdd((unsigned long long *)(qpairs + cur), (unsigned long long)acc);
        cur = q;
        acc = 0;
      }
      acc += W[r];
    }
    if (acc) atomicAdd((unsigned long long *)(qpairs + cur), (unsigned long long)acc);
  }
}

// Rows of evicted queries keep one pair (the expansion relies on every row
// having at least one, so a tile touches at most as many rows as it has
// pairs) and move to the retired query slot, whose candidate test fails.
__global__ __launch_bounds__(kAuxWG) void k_retire_evicted(uint32_t *W, uint16_t *qid, const uint64_t *n_dev,
                                                           const uint8_t *evicted, uint16_t retired) {
  const uint64_t N = *n_dev;
  for (uint64_t r = (uint64_t)blockIdx.x * kAuxWG + threadIdx.x; r < N; r += (uint64_t)gridDim.x * kAuxWG)
    if (evicted[qid[r]]) {
      W[r] = 1;
      qid[r] = retired;
    }
}

__global__ __launch_bounds__(kAuxWG) void k_mark_evicted(const uint64_t *qpairs, int nq, uint64_t threshold,
                                                         uint8_t *evicted) {
  for (int k = blockIdx.x * kAuxWG + threadIdx.x; k < nq; k += gridDim.x * kAuxWG)
    if (qpairs[k] > threshold) evicted[k] = 1;
}

}  // namespace

void launch_mark_evicted(const uint64_t *qpairs, int nq, uint64_t threshold, uint8_t *evicted, hipStream_t s) {
  if (nq <= 0) return;
  const unsigned grid = (unsigned)std::min<int>((nq + kAuxWG - 1) / kAuxWG, 1024);
  hipLaunchKernelGGL(k_mark_evicted, dim3(grid), dim3(kAuxWG), 0, s, qpairs, nq, threshold, evicted);
  GSM_HIP(hipGetLastError());
}

void launch_query_pairs(const uint32_t *W, const uint16_t *qid, const uint64_t *n_dev, uint64_t rows_hint,
                        uint64_t *qpairs, hipStream_t s) {
  const uint64_t per = (uint64_t)kAuxWG * kAuxRun;
  const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((rows_hint + per - 1) / per, 4096));
  hipLaunchKernelGGL(k_query_pairs, dim3(grid), dim3(kAuxWG), 0, s, W, qid, n_dev, qpairs);
  GSM_HIP(hipGetLastError());
}

void launch_retire_evicted(uint32_t *W, uint16_t *qid, const uint64_t *n_dev, uint64_t rows_hint,
                           const uint8_t *evicted, uint16_t retired, hipStream_t s) {
  const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((rows_hint + kAuxWG - 1) / kAuxWG, 8192));
  hipLaunchKernelGGL(k_retire_evicted, dim3(grid), dim3(kAuxWG), 0, s, W, qid, n_dev, evicted, retired);
  GSM_HIP(hipGetLastError());
}

}  // namespace gsm
