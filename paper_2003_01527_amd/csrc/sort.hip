// Lexicographic order of embedding rows on the device (the optional sorted
// output of the result step, Alg. 1 output M).
//
// A row of q int32 ids in [0, n) is packed into one (q*b)-bit key, b the bit
// width of n-1, column 0 most significant, so the numeric order of keys is the
// lexicographic order of rows.  Keys are kept as W little-endian 64-bit words
// in structure-of-arrays form (word j of key k at keys[j*N + k]) so every pass
// reads and writes whole coalesced words.  A least-significant-digit radix
// sort with 8-bit digits orders them, every pass moving all W words of a key
// (the last step unpacks every column).  Each pass is stable: a tile's
// elements are ranked in index order (wave match on the digit, then a
// workgroup prefix per digit in LDS), and tiles take their slots from an
// exclusive scan of the per-(digit, tile) histogram laid out digit-major.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "gsm_internal.h"

namespace gsm {

namespace {

constexpr int kSortWG = 256;
constexpr int kSortRounds = 8;  // elements per thread per tile
constexpr int kSortTile = kSortWG * kSortRounds;
constexpr int kSortWaves = kSortWG / 64;
constexpr int kDigits = 256;

__device__ __forceinline__ uint32_t below_lane(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Bits [lo, lo + 64) of the concatenated key of one row, as one word.
__device__ __forceinline__ uint64_t key_word(const int32_t *row, int q, int b, int j) {
  const int lo = 64 * j;
  uint64_t w = 0;
  for (int c = 0; c < q; ++c) {
    const int off = b * (q - 1 - c);  // position of column c's lowest bit
    const uint64_t v = (uint32_t)row[c];
    if (off + b <= lo || off >= lo + 64) continue;
    const int sh = off - lo;
    w |= sh >= 0 ? (v << sh) : (v >> -sh);
  }
  return w;
}

__global__ __launch_bounds__(256) void k_sort_pack(const int32_t *rows, uint64_t N, int q, int b, int W,
                                                   uint64_t *keys) {
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (uint64_t)gridDim.x * blockDim.x) {
    int32_t r[kMaxQ];
    for (int c = 0; c < q; ++c) r[c] = rows[k * q + c];
    for (int j = 0; j < W; ++j) keys[(uint64_t)j * N + k] = key_word(r, q, b, j);
  }
}

__global__ __launch_bounds__(256) void k_sort_unpack(const uint64_t *keys, uint64_t N, int q, int b, int W,
                                                     int32_t *rows) {
  const uint64_t mask = (b >= 64) ? ~0ull : ((1ull << b) - 1);
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (uint64_t)gridDim.x * blockDim.x) {
    for (int c = 0; c < q; ++c) {
      const int off = b * (q - 1 - c);
      const int j = off >> 6, sh = off & 63;
      uint64_t v = keys[(uint64_t)j * N + k] >> sh;
      if (sh + b > 64) v |= keys[(uint64_t)(j + 1) * N + k] << (64 - sh);
      rows[k * q + c] = (int32_t)(v & mask);
    }
  }
}

// Digit histogram of each tile, stored digit-major: hist[d * tiles + tile].
__global__ __launch_bounds__(kSortWG) void k_sort_hist(const uint64_t *word, uint64_t N, int shift,
                                                       uint32_t *hist, uint64_t *hist_len) {
  __shared__ uint32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  for (int j = 0; j < kSortRounds; ++j) {
    const uint64_t e = base + (uint64_t)j * kSortWG + threadIdx.x;
    if (e < N) atomicAdd(&h[(word[e] >> shift) & 0xff], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
  if (blockIdx.x == 0 && threadIdx.x == 0) *hist_len = (uint64_t)kDigits * gridDim.x;
}

// Stable scatter of whole keys by the digit of word j at `shift`.
__global__ __launch_bounds__(kSortWG) void k_sort_scatter(const uint64_t *src, uint64_t *dst, uint64_t N, int j,
                                                          int W, int shift, const uint64_t *offs) {
  __shared__ uint64_t s_next[kDigits];   // next free slot of each digit
  __shared__ uint64_t s_start[kDigits];  // that slot at the start of the round
  __shared__ uint32_t s_cnt[kSortWaves][kDigits];
  const int wid = threadIdx.x >> 6;
  s_next[threadIdx.x] = offs[(uint64_t)threadIdx.x * gridDim.x + blockIdx.x];
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) s_cnt[w][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t e = base + (uint64_t)r * kSortWG + threadIdx.x;
    const bool valid = e < N;
    const uint64_t key = valid ? src[(uint64_t)j * N + e] : 0;
    const uint32_t d = (uint32_t)(key >> shift) & 0xff;
    // lanes of this wave that hold the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool set = (d >> bit) & 1;
      const uint64_t m = __ballot(set);
      peers &= set ? m : ~m;
    }
    const uint32_t rank = below_lane(peers);
    if (valid && rank == 0) s_cnt[wid][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    {
      // digit t: each wave's offset inside this round, waves in order
      const int t = threadIdx.x;
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < kSortWaves; ++w) {
        const uint32_t c = s_cnt[w][t];
        s_cnt[w][t] = run;
        run += c;
      }
      s_start[t] = s_next[t];
      s_next[t] += run;
    }
    __syncthreads();
    if (valid) {
      const uint64_t pos = s_start[d] + s_cnt[wid][d] + rank;
      dst[(uint64_t)j * N + pos] = key;
      for (int w = 0; w < W; ++w)
        if (w != j) dst[(uint64_t)w * N + pos] = src[(uint64_t)w * N + e];
    }
    __syncthreads();
  }
}

}  // namespace

// Sorts N rows of q int32 ids in [0, n) (device memory, row-major) into
// ascending lexicographic order in place.  Device memory taken from sb:
// two key buffers of W*N words, W = ceil(q*b/64), and 12 bytes per 256 rows
// of histogram and offsets.
void sort_rows_device(int32_t *rows, uint64_t N, int q, int64_t n, SortBuffers &sb, hipStream_t s) {
  if (N < 2 || q <= 0) return;
  int b = 1;
  while (b < 63 && (uint64_t(1) << b) < (uint64_t)n) ++b;
  const int bits = b * q;
  const int W = (bits + 63) / 64;
  const uint64_t tiles = (N + kSortTile - 1) / kSortTile;
  sb.keys[0].reserve(sizeof(uint64_t) * W * N, s);
  sb.keys[1].reserve(sizeof(uint64_t) * W * N, s);
  sb.hist.reserve(sizeof(uint32_t) * kDigits * tiles, s);
  sb.offs.reserve(sizeof(uint64_t) * (kDigits * tiles + 1), s);
  sb.len.reserve(sizeof(uint64_t), s);
  sb.scratch.reserve(sizeof(uint64_t) * 1024, s);
  uint64_t *k0 = sb.keys[0].as<uint64_t>(), *k1 = sb.keys[1].as<uint64_t>();
  const unsigned grid = (unsigned)std::min<uint64_t>((N + 255) / 256, 65536);
  hipLaunchKernelGGL(k_sort_pack, dim3(grid), dim3(256), 0, s, rows, N, q, b, W, k0);
  const int passes = (bits + 7) / 8;
  for (int p = 0; p < passes; ++p) {
    const int j = p / 8, shift = (p % 8) * 8;
    hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)tiles), dim3(kSortWG), 0, s, k0 + (uint64_t)j * N, N, shift,
                       sb.hist.as<uint32_t>(), sb.len.as<uint64_t>());
    launch_scan(sb.hist.as<uint32_t>(), sb.len.as<uint64_t>(), sb.offs.as<uint64_t>(), nullptr,
                sb.scratch.as<uint64_t>(), s);
    hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)tiles), dim3(kSortWG), 0, s, k0, k1, N, j, W, shift,
                       sb.offs.as<uint64_t>());
    std::swap(k0, k1);
  }
  hipLaunchKernelGGL(k_sort_unpack, dim3(grid), dim3(256), 0, s, k0, N, q, b, W, rows);
  GSM_HIP(hipGetLastError());
}

}  // namespace gsm
