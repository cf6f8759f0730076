// HIP kernels of the matcher, written for gfx950 (wave64, 256 CUs in 8 XCDs).
//
// Everything here is integer work that streams or gathers CSR data from HBM;
// nothing is a dense contraction, so no kernel uses the matrix cores.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gsm_internal.h"

namespace gsm {

namespace {

constexpr int kWave = 64;

// Root-slice hash: the output of one splitmix64 step (Steele, Lea, Flood,
// OOPSLA 2014) from state x, i.e. the finaliser applied to x + golden gamma.
__device__ __forceinline__ uint64_t slice_mix(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t lane_prefix(uint64_t mask) {
  // number of set bits of mask below this lane
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

// Inclusive scan of a 64-bit value across the wave.
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint64_t o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan of one value per thread across the workgroup.  `sw` holds
// one slot per wave.  Returns the prefix; *total gets the workgroup sum.
template <int WG>
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t *sw, uint64_t *total) {
  constexpr int NW = WG / kWave;
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  uint64_t inc = wave_incl_scan(v);
  if (lane == kWave - 1) sw[wid] = inc;
  __syncthreads();
  uint64_t before = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    uint64_t x = sw[w];
    if (w < wid) before += x;
    sum += x;
  }
  __syncthreads();
  *total = sum;
  return before + inc - v;
}

// Index of w in the ascending list c[0..n), or -1: the window is halved down
// to its last entry <= w, with 32-bit offsets from the list start, then one
// compare.  (Interpolation probes were measured slower on the 2^21-vertex
// R-MAT graph: lanes of a wave search nearby keys, so halving's first probes
// are shared loads, while every interpolation probe is a separate one.)
__device__ __forceinline__ int32_t find_sorted(const int32_t *c, uint32_t n, int32_t w) {
  if (n == 0) return -1;
  uint32_t b = 0, m = n;
  while (m > 1) {
    const uint32_t h = m >> 1;
    b = (c[b + h] <= w) ? b + h : b;
    m -= h;
  }
  return c[b] == w ? (int32_t)b : -1;
}

// Binary-search steps a plain search of a list of n entries takes (halving
// steps plus the final compare): the unit of the back-edge term of the
// algorithmic byte count, whatever search the kernel actually runs.
__device__ __forceinline__ uint32_t search_steps(uint32_t n) {
  return n > 1 ? 33 - __builtin_clz(n - 1) : 1;
}

__device__ __forceinline__ int64_t vd_start(const int4 &d) {
  return (int64_t)(((uint64_t)(uint32_t)d.y << 32) | (uint32_t)d.x);
}

// Is w a neighbour of x: one 16-byte record load, then one bitmap word or a
// search of the sorted list.
__device__ __forceinline__ bool has_edge(const DeviceGraph &g, int32_t x, int32_t w,
                                         uint32_t &probes) {
  const int4 d = g.vdesc[x];
  const uint32_t n = (uint32_t)d.z;
  probes += search_steps(n);
  if (d.w >= 0) return (g.hub_bits[(uint64_t)d.w * g.hub_words + ((uint32_t)w >> 5)] >> (w & 31)) & 1u;
  return find_sorted(g.col + vd_start(d), n, w) >= 0;
}

// Position of w in the sorted neighbour list of x (an index into col), or -1.
__device__ __forceinline__ int64_t edge_pos(const DeviceGraph &g, int32_t x, int32_t w, uint32_t &probes) {
  const int4 d = g.vdesc[x];
  const int64_t b = vd_start(d);
  const uint32_t n = (uint32_t)d.z;
  probes += search_steps(n);
  const int32_t k = find_sorted(g.col + b, n, w);
  return k >= 0 ? b + k : -1;
}

// ------------------------------------------------------------ graph stats --

// deg[v] and NE0[v] = sum over neighbours of (label+1); 16 lanes per vertex.
__global__ void k_graph_stats(const int64_t *rp, const int32_t *col, const int32_t *lab,
                              int64_t n, uint32_t *deg, uint64_t *ne0, uint2 *dne) {
  constexpr int G = 16;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int sub = threadIdx.x & (G - 1);
  for (int64_t v = gid / G; v < n; v += nthreads / G) {
    const int64_t b = rp[v], e = rp[v + 1];
    uint64_t s = 0;
    if (lab)
      for (int64_t k = b + sub; k < e; k += G) s += (uint64_t)lab[col[k]] + 1;
#pragma unroll
    for (int d = G / 2; d > 0; d >>= 1) s += __shfl_xor(s, d, G);
    if (sub == 0) {
      deg[v] = (uint32_t)(e - b);
      if (ne0) ne0[v] = s;
      const uint64_t ne = lab ? s : (uint64_t)(e - b);
      dne[v] = make_uint2((uint32_t)(e - b), ne > 0xffffffffull ? 0xffffffffu : (uint32_t)ne);
    }
  }
}

// Adjacency bitmap of hubs[s] (blockIdx.x = s): one bit per neighbour.
__global__ __launch_bounds__(256) void k_hub_bitmaps(const int64_t *rp, const int32_t *col, const int32_t *hubs,
                                                     int64_t nhubs, uint32_t *bits, uint64_t words) {
  for (int64_t h = blockIdx.x; h < nhubs; h += gridDim.x) {
    const int32_t v = hubs[h];
    uint32_t *bm = bits + (uint64_t)h * words;
    for (int64_t k = rp[v] + threadIdx.x; k < rp[v + 1]; k += blockDim.x) {
      const uint32_t w = (uint32_t)col[k];
      atomicOr(bm + (w >> 5), 1u << (w & 31));
    }
  }
}

// ---------------------------------------------------------------- filter --

// The id a root slice hashes: the caller's id of v.
__device__ __forceinline__ uint64_t slice_id(const DeviceGraph &g, int32_t v) {
  return (uint64_t)(uint32_t)(g.orig ? g.orig[v] : v);
}

__device__ __forceinline__ uint16_t candidate_bits(const QueryArgs &qa, int32_t lv, uint32_t d,
                                                   uint64_t ne, uint64_t v) {
  uint32_t m = 0;
  for (int u = 0; u < qa.q; ++u) {
    bool ok = (lv == qa.qlab[u]);
    ok = ok && (!qa.use_deg || d >= qa.qdeg[u]);
    ok = ok && (!qa.use_ne || ne >= qa.qne[u]);
    if (u == qa.root_bit) ok = ok && (slice_mix(v) % qa.root_mod == qa.root_rem);
    m |= (uint32_t)ok << u;
  }
  return (uint16_t)m;
}

__global__ void k_filter_init(DeviceGraph g, QueryArgs qa, uint16_t *cmask) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += stride) {
    const int32_t lv = g.lab ? g.lab[v] : 0;
    const uint32_t d = g.deg[v];
    const uint64_t ne = g.ne0 ? g.ne0[v] : (uint64_t)d;
    cmask[v] = candidate_bits(qa, lv, d, ne, slice_id(g, (int32_t)v));
  }
}

__device__ __forceinline__ uint16_t refine_bits(const QueryArgs &qa, uint16_t pm, uint32_t c,
                                                uint64_t s) {
  uint32_t m = 0;
  for (int u = 0; u < qa.q; ++u) {
    bool ok = (pm >> u) & 1;
    ok = ok && (!qa.use_deg || c >= qa.qdeg[u]);
    ok = ok && (!qa.use_ne || s >= qa.qne[u]);
    m |= (uint32_t)ok << u;
  }
  return (uint16_t)m;
}

// One refinement round for vertices of degree <= kHeavyDegree; 16 lanes per vertex.
__global__ void k_refine_light(DeviceGraph g, QueryArgs qa, const uint16_t *prev, uint16_t *next) {
  constexpr int G = 16;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int sub = threadIdx.x & (G - 1);
  for (int64_t v = gid / G; v < g.n; v += nthreads / G) {
    const uint16_t pm = prev[v];
    const int64_t b = g.rp[v], e = g.rp[v + 1];
    if (e - b > kHeavyDegree) continue;  // k_refine_heavy writes it
    if (pm == 0) {
      if (sub == 0) next[v] = 0;
      continue;
    }
    uint32_t c = 0;
    uint64_t s = 0;
    for (int64_t k = b + sub; k < e; k += G) {
      const int32_t w = g.col[k];
      if (prev[w]) {
        c += 1;
        s += g.lab ? (uint64_t)g.lab[w] + 1 : 1;
      }
    }
#pragma unroll
    for (int d = G / 2; d > 0; d >>= 1) {
      c += __shfl_xor(c, d, G);
      s += __shfl_xor(s, d, G);
    }
    if (sub == 0) next[v] = refine_bits(qa, pm, c, s);
  }
}

// One refinement round for the high-degree vertices; one workgroup per vertex.
__global__ __launch_bounds__(256) void k_refine_heavy(DeviceGraph g, QueryArgs qa,
                                                      const int32_t *heavy, int64_t nheavy,
                                                      const uint16_t *prev, uint16_t *next) {
  __shared__ uint64_t sw[256 / kWave];
  for (int64_t h = blockIdx.x; h < nheavy; h += gridDim.x) {
    const int32_t v = heavy[h];
    const uint16_t pm = prev[v];
    if (pm == 0) {  // uniform across the workgroup
      if (threadIdx.x == 0) next[v] = 0;
      continue;
    }
    const int64_t b = g.rp[v], e = g.rp[v + 1];
    uint64_t c = 0, s = 0;
    for (int64_t k = b + threadIdx.x; k < e; k += blockDim.x) {
      const int32_t w = g.col[k];
      if (prev[w]) {
        c += 1;
        s += g.lab ? (uint64_t)g.lab[w] + 1 : 1;
      }
    }
    uint64_t tc, ts;
    block_excl_scan<256>(c, sw, &tc);
    block_excl_scan<256>(s, sw, &ts);
    if (threadIdx.x == 0) next[v] = refine_bits(qa, pm, (uint32_t)tc, ts);
  }
}

// ------------------------------------------------------ first frontier --

// Column j of a packed frontier row (b-bit ids laid end to end from bit 0 of
// the row's first 32-bit word; b <= 31, so an id spans at most two words):
// the reversible packing of partial results.
__device__ __forceinline__ int32_t unpack_id(const uint32_t *row, uint32_t j, uint32_t b) {
  const uint32_t bit = j * b, wd = bit >> 5, sh = bit & 31;
  uint32_t v = row[wd] >> sh;
  if (sh + b > 32) v |= row[wd + 1] << (32 - sh);
  return (int32_t)(v & ((1u << b) - 1u));
}

// Neighbour range of x that holds label l: [base, base + size) in g.gather.
__device__ __forceinline__ uint32_t label_range(const DeviceGraph &g, int32_t x, int32_t l,
                                                int64_t &base) {
  const int4 d = g.vdesc[x];
  const int64_t b = vd_start(d);
  if (g.loff) {
    const uint32_t *o = g.loff + (int64_t)x * g.loff_stride;
    if (l + 1 >= g.loff_stride) {  // label absent from the graph
      base = b;
      return 0;
    }
    const uint32_t lo = o[l], hi = o[l + 1];
    base = b + lo;
    return hi - lo;
  }
  base = b;
  return (uint32_t)d.z;
}

// k-look-ahead (Sec. 3.3) on a new row: the ids row[0..i) already matched
// and w placed at position i.  One step: every later query neighbour of
// position i must find its own image among w's neighbours of its label:
// there must be at least la_need of them (those of the matched neighbours
// included), and, for a label group short enough to scan, one that is a
// candidate of that query vertex and not in the row.  Two steps (la2): that
// neighbour must also have, for each label the later query vertex's own
// neighbours carry, at least as many neighbours of that label.  Failing any,
// no extension of the row can be an embedding.
__device__ __forceinline__ bool lookahead_ok(const ExpandArgs &a, int32_t w, const int32_t *row) {
  for (int f = 0; f < a.L.la_n; ++f) {
    int64_t base;
    const uint32_t cnt = label_range(a.g, w, a.L.la_label[f], base);
    if (cnt < a.L.la_need[f]) return false;
    if (cnt > kLookaheadScan) continue;
    bool found = false;
    for (uint32_t t = 0; t < cnt && !found; ++t) {
      const int32_t x = a.g.gather[base + t];
      if (!((a.cmask[x] >> a.L.la_qbit[f]) & 1)) continue;
      bool used = false;
      for (int j = 0; j < a.L.i; ++j) used = used || row[j] == x;
      if (used) continue;
      // two steps: x would take the later query vertex, whose neighbours of
      // each label must then map to distinct neighbours of x of that label
      bool enough = true;
      for (int e = 0; a.L.la2 && e < a.L.la2_n[f] && enough; ++e) {
        int64_t xb;
        enough = label_range(a.g, x, a.L.la2_label[f][e], xb) >= a.L.la2_need[f][e];
      }
      found = enough;
    }
    if (!found) return false;
  }
  return true;
}

__global__ __launch_bounds__(256) void k_compact_first(DeviceGraph g, const uint16_t *cmask,
                                                       uint32_t qbit, int32_t next_label,
                                                       int32_t *rows, uint32_t *W, int64_t *abase,
                                                       uint8_t *apos, uint64_t *counter,
                                                       int32_t *emit_rows, uint64_t emit_cap) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // every lane of the wave runs the same number of iterations
  const int64_t base0 = start - (threadIdx.x & (kWave - 1));
  for (int64_t vb = base0; vb < g.n; vb += stride) {
    const int64_t v = vb + (threadIdx.x & (kWave - 1));
    bool keep = false;
    uint32_t d = 0;
    int64_t b = 0;
    if (v < g.n) {
      keep = (cmask[v] >> qbit) & 1;
      if (keep && rows) {
        d = label_range(g, (int32_t)v, next_label, b);
        keep = d > 0;  // no neighbour can take the next query vertex
      }
    }
    const uint64_t mask = wave_ballot(keep);
    if (mask == 0) continue;
    uint64_t base = 0;
    if ((threadIdx.x & (kWave - 1)) == 0)
      base = atomicAdd((unsigned long long *)counter, (unsigned long long)__popcll(mask));
    base = __shfl(base, 0, kWave);
    if (keep) {
      const uint64_t pos = base + lane_prefix(mask);
      if (rows) {
        rows[pos] = (int32_t)v;
        W[pos] = d;
        abase[pos] = b;
        apos[pos] = 0;
      }
      if (emit_rows && pos < emit_cap) emit_rows[pos] = g.orig ? g.orig[v] : (int32_t)v;  // caller's ids
    }
  }
}

// ------------------------------------------------ batched first frontier --

// Round-0 candidate test without a per-query array: one 8-byte load of
// (degree, NE) and, where neighbours were not gathered by label, the label.
// NE is stored saturated at 2^32-1 and the host clamps the query's NE to the
// same value, so the test can only accept more vertices than the exact one
// (it stays sound; every embedding is still verified edge by edge).
__device__ __forceinline__ bool inline_candidate(const DeviceGraph &g, int32_t v, int32_t qlab,
                                                 uint32_t qdeg, uint64_t qne, bool label_known) {
  const uint2 dn = g.dne[v];
  bool ok = dn.x >= qdeg && (uint64_t)dn.y >= qne;
  if (!label_known) ok = ok && (g.lab ? g.lab[v] == qlab : qlab == 0);
  return ok;
}

// rows == null: estimate only, adding each query's first-level pair total
// (the sum of its rows' range sizes) to pairs1[k] and writing nothing else.
// The candidates of position 0 of query k (blockIdx.y) among the vertices
// of its label class (vertices sorted by label, or all vertices when the
// graph has no such index): first-frontier rows, or (rows == null) only the
// query's first-level pair total, or (a one-vertex query) its count.  Each
// block aggregates its survivors before one atomic.
__global__ __launch_bounds__(256) void k_compact_first_batch(DeviceGraph g, const FirstBatch *fb_all,
                                                             int32_t *rows,
                                                             uint16_t *qid, uint32_t *W, int64_t *abase,
                                                             uint8_t *apos, uint64_t *counter,
                                                             uint64_t *counts, uint64_t *pairs1) {
  __shared__ uint64_t sw[256 / kWave];
  __shared__ uint64_t s_base;
  const int k = blockIdx.y;
  const FirstBatch fb = fb_all[k];
  const int64_t len = fb.vend - fb.vbegin;
  uint64_t tally = 0;  // single: vertices kept; estimate: pairs
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < len; i0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t idx = i0 + threadIdx.x;
    bool keep = false;
    uint32_t d = 0;
    int64_t b = 0;
    int32_t v = 0;
    if (idx < len) {
      v = g.lab_vert ? g.lab_vert[fb.vbegin + idx] : (int32_t)(fb.vbegin + idx);
      keep = inline_candidate(g, v, fb.qlab0, fb.qdeg0, fb.qne0, g.lab_vert != nullptr);
      if (keep && fb.slice_mod) keep = slice_mix(slice_id(g, v)) % fb.slice_mod == fb.slice_rem;
      if (keep && !fb.single) {
        d = label_range(g, v, fb.label1, b);
        keep = d > 0;
      }
    }
    if (fb.single || !rows) {
      tally += fb.single ? (uint64_t)keep : (keep ? d : 0);
      continue;
    }
    uint64_t total;
    const uint64_t before = block_excl_scan<256>(keep ? 1u : 0u, sw, &total);
    if (total == 0) continue;  // uniform: every thread has the same total
    if (threadIdx.x == 0) s_base = atomicAdd((unsigned long long *)counter, (unsigned long long)total);
    __syncthreads();
    const uint64_t base = s_base;
    if (keep) {
      const uint64_t pos = base + before;
      rows[pos] = v;
      qid[pos] = (uint16_t)k;
      W[pos] = d;
      abase[pos] = b;
      apos[pos] = 0;
    }
    __syncthreads();  // s_base is rewritten by the next iteration
  }
  if (fb.single || !rows) {
    uint64_t total;
    block_excl_scan<256>(tally, sw, &total);
    if (threadIdx.x == 0 && total) {
      if (fb.single && counts) atomicAdd((unsigned long long *)(counts + k), (unsigned long long)total);
      if (!fb.single && !rows) atomicAdd((unsigned long long *)(pairs1 + k), (unsigned long long)total);
    }
  }
}

// ------------------------------------------------------------------ scan --

constexpr int kScanBlocks = 512;
constexpr int kScanWG = 256;
constexpr int kScanItems = 4;

__global__ __launch_bounds__(kScanWG) void k_scan_reduce(const uint32_t *W, const uint64_t *n_dev,
                                                         uint64_t *partial) {
  __shared__ uint64_t sw[kScanWG / kWave];
  const uint64_t N = *n_dev;
  const uint64_t per = (N + kScanBlocks - 1) / kScanBlocks;
  const uint64_t b = (uint64_t)blockIdx.x * per, e = min(N, b + per);
  uint64_t s = 0;
  for (uint64_t k = b + threadIdx.x; k < e; k += kScanWG) s += W[k];
  uint64_t tot;
  block_excl_scan<kScanWG>(s, sw, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanWG) void k_scan_partials(uint64_t *partial, const uint64_t *n_dev,
                                                           uint64_t *S, uint64_t *total_out) {
  __shared__ uint64_t sw[kScanWG / kWave];
  constexpr int per = kScanBlocks / kScanWG;
  uint64_t v[per];
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < per; ++j) {
    v[j] = partial[threadIdx.x * per + j];
    s += v[j];
  }
  uint64_t tot;
  uint64_t run = block_excl_scan<kScanWG>(s, sw, &tot);
#pragma unroll
  for (int j = 0; j < per; ++j) {
    partial[threadIdx.x * per + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0) {
    S[*n_dev] = tot;
    if (total_out) *total_out = tot;
  }
}

__global__ __launch_bounds__(kScanWG) void k_scan_down(const uint32_t *W, const uint64_t *n_dev,
                                                       const uint64_t *partial, uint64_t *S) {
  __shared__ uint64_t sw[kScanWG / kWave];
  const uint64_t N = *n_dev;
  const uint64_t per = (N + kScanBlocks - 1) / kScanBlocks;
  const uint64_t b = (uint64_t)blockIdx.x * per, e = min(N, b + per);
  uint64_t carry = partial[blockIdx.x];
  constexpr int T = kScanWG * kScanItems;
  for (uint64_t t0 = b; t0 < e; t0 += T) {
    uint64_t v[kScanItems];
    uint64_t s = 0;
    const uint64_t k0 = t0 + (uint64_t)threadIdx.x * kScanItems;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      v[j] = (k0 + j < e) ? W[k0 + j] : 0;
      s += v[j];
    }
    uint64_t tot;
    uint64_t run = carry + block_excl_scan<kScanWG>(s, sw, &tot);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      if (k0 + j < e) S[k0 + j] = run;
      run += v[j];
    }
    carry += tot;
  }
}

// --------------------------------------------------------------- expand --
//
// One launch expands rows of level i over a range of the flat pair space.
// Pair t belongs to row r with S[r] <= t < S[r+1]; its candidate is
// gather[abase[r] + t - S[r]]: a neighbour of the row's anchor (the earlier
// matched neighbour of the new query vertex with the fewest neighbours of the
// new vertex's label, chosen when the row was written) that carries that label.
// Lanes of a wave take consecutive pairs, so neighbour reads of one row are
// coalesced.  A candidate survives the candidate-mask test, injectivity and a
// binary search for every other back-edge; when the row goes on to a further
// level it must also leave a non-empty range for the next query vertex.
//
// Per tile: the first row and the number of rows come from the launch's tile
// map (or, past its end or without one, from two 64-way searches by the
// first wave); the rows the tile touches are copied to LDS with contiguous
// loads; every item's loads are issued before any result is used, so a wave
// keeps ITEMS gathers in flight.  Survivors are compacted item by item (wave ballot, workgroup
// prefix, one atomic per tile) so consecutive lanes write consecutive rows;
// output rows are staged in LDS and copied out with contiguous stores when
// they fit.
// EXT: edge labels or induced semantics are in force (a separate
// instantiation, so the common one carries none of their registers).
// Column j of a tile's input row: from the LDS copy when the tile staged its
// rows, else from global memory (the empty asm keeps the two loads apart, so
// the LDS one is not turned into a generic-address load).
__device__ __forceinline__ int32_t row_id(bool staged, const int32_t *s_in, const int32_t *g, uint32_t li,
                                          uint64_t gi) {
  if (staged) {
    int32_t x = s_in[li];
    __asm__ volatile("" : "+v"(x));
    return x;
  }
  return g[gi];
}

template <int WG, int ITEMS, int MODE, bool EXT>
__global__ __launch_bounds__(WG) void k_expand(ExpandArgs a) {
  constexpr bool BATCHED = (MODE == kModeBatch || MODE == kModeBatchLast);
  constexpr int TILE = WG * ITEMS;
  constexpr int NW = WG / kWave;
  __shared__ uint32_t sS[TILE + 1];  // row starts relative to the tile, clamped to TILE+1
  __shared__ uint64_t sw[NW];
  __shared__ uint32_t s_cnt[ITEMS * NW];
  __shared__ uint64_t s_r0, s_base;
  __shared__ uint32_t s_total, s_R, s_lead;
  extern __shared__ int32_t dyn[];  // [TILE * i] input rows, then [TILE * width] output rows

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int i = a.L.i;
  const int width = (MODE == kModeNext || MODE == kModeBatch) ? i + 1 : a.L.q;
  // input staging holds in_cap rows; a tile touching more rows reads them
  // from global memory
  const bool stage_rows = a.stage_in != 0;
  int32_t *s_in = dyn;
  int32_t *s_out = dyn + (stage_rows ? a.in_cap * (uint32_t)i : 0u);
  // rows and pair range: from the arguments, or (device-driven launches) the
  // level's row count and scan total as the previous kernels left them in
  // device memory, the range then clamped to the capacity the host gave; a
  // total above it is flagged, and the host redoes the work in chunks
  uint64_t n_rows = a.n_rows, pair_end = a.pair_end;
  if (a.dev_pair_end) {
    n_rows = *a.dev_n_rows;
    const uint64_t total = *a.dev_pair_end;
    pair_end = min(a.pair_end, total);
    if (total > a.pair_end && blockIdx.x == 0 && threadIdx.x == 0) *a.overflow = 1;
  }
  const uint64_t npairs = pair_end > a.pair_begin ? pair_end - a.pair_begin : 0;
  const uint64_t ntiles = (npairs + TILE - 1) / TILE;
  const uint32_t G = gridDim.x, b = blockIdx.x;
  // XCD-aware order: workgroup b runs on XCD b % 8; give each XCD a
  // contiguous run of tiles so neighbouring tiles share its L2.
  const uint64_t lb = (G % 8 == 0) ? (uint64_t)(b % 8) * (G / 8) + b / 8 : b;
  const uint32_t inj_mask = ((1u << i) - 1u) & ~a.L.nbr_mask;
  uint64_t wg_count = 0;
  uint32_t probes = 0;
  uint32_t acc_k = 0xffffffffu;  // kModeBatch: this wave's pending (query, count)
  uint64_t acc_c = 0;

  for (uint64_t tile = lb; tile < ntiles; tile += G) {
    const uint64_t t0 = a.pair_begin + tile * TILE;
    const uint32_t len = (uint32_t)min((uint64_t)TILE, pair_end - t0);
    uint64_t r0;
    uint32_t R;
    if (a.use_tile_map && tile < a.tile_map_cap) {  // first row and row count, found before the launch
      const uint64_t e = a.tile_map[tile];
      r0 = e & ((uint64_t(1) << 48) - 1);
      R = (uint32_t)(e >> 48);
    } else {
    if (wid == 0) {
      // 64-way search by the first wave: S[lo] <= t0 < S[hi]; every round
      // shrinks the interval 64-fold (5 dependent loads for 10^8 rows).
      uint64_t lo = 0, hi = n_rows;
      while (hi - lo > 1) {
        const uint64_t step = (hi - lo + kWave - 1) / kWave;
        const uint64_t idx = lo + (uint64_t)lane * step;
        const bool le = idx < hi && a.S[idx] <= t0;  // true on lane 0
        const uint64_t mask = wave_ballot(le);
        const uint64_t k = 63 - __builtin_clzll(mask);
        lo += k * step;
        hi = min(hi, lo + step);
      }
      // rows touched: every row has at least one pair, so the first row
      // starting at or after the tile's end e is within len rows of r0
      // (S[r0+k] >= t0+k); the same search finds it in two rounds
      const uint64_t e = t0 + len;
      uint64_t lo2 = lo, hi2 = min(n_rows, lo + len);  // S[lo2] < e <= S[hi2]
      while (hi2 - lo2 > 1) {
        const uint64_t step = (hi2 - lo2 + kWave - 1) / kWave;
        const uint64_t idx = lo2 + (uint64_t)lane * step;
        const bool lt = idx < hi2 && a.S[idx] < e;  // true on lane 0
        const uint64_t mask = wave_ballot(lt);
        const uint64_t k = 63 - __builtin_clzll(mask);
        lo2 += k * step;
        hi2 = min(hi2, lo2 + step);
      }
      if (lane == 0) {
        s_r0 = lo;
        s_R = (uint32_t)(hi2 - lo);
      }
    }
    __syncthreads();
    r0 = s_r0;
    R = s_R;
    }
    const bool stage_in = stage_rows && R <= a.in_cap;  // uniform over the workgroup
    // row starts relative to the tile: sS[k] <= t < sS[k+1] for the pairs t
    // of row r0+k, k < R, and sS[R] >= len
    for (uint32_t k = tid; k <= R; k += WG) {
      uint32_t rel;
      if (k == 0) {
        rel = 0;  // the first row may start before the tile: its lead is s_lead
        s_lead = (uint32_t)(t0 - a.S[r0]);
      } else {
        const uint64_t v = a.S[r0 + k];
        rel = (v - t0 > (uint64_t)TILE) ? (uint32_t)TILE + 1 : (uint32_t)(v - t0);
      }
      sS[k] = rel;
    }
    // the rows are copied in the same phase (one barrier for both)
    if (stage_in && a.pack_in) {
      // packed rows: ceil(i*b/32) words each, column j in bits [j*b, j*b+b)
      const uint32_t b = (uint32_t)a.pack_bits, nw = (uint32_t)((i * b + 31) / 32);
      const uint32_t *src = reinterpret_cast<const uint32_t *>(a.rows_in) + r0 * (uint64_t)nw;
      for (uint32_t e = tid; e < R * (uint32_t)i; e += WG) s_in[e] = unpack_id(src + (e / i) * nw, e % i, b);
    } else if (stage_in) {
      const int32_t *src = a.rows_in + r0 * (uint64_t)i;
      for (uint32_t e = tid; e < R * (uint32_t)i; e += WG) s_in[e] = src[e];
    }
    __syncthreads();
    const uint32_t lead = s_lead;

    // ---- evaluation (no barriers): row, candidate, checks of every item
    uint32_t rk[ITEMS], off[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const uint32_t tl = (uint32_t)(it * WG + tid);
      uint32_t lo = 0, hi = R;  // sS[lo] <= tl < sS[hi]
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (sS[mid] <= tl)
          lo = mid;
        else
          hi = mid;
      }
      rk[it] = lo;
      off[it] = tl - sS[lo] + (lo == 0 ? lead : 0u);
    }
    int64_t ab[ITEMS];
    int ap[ITEMS];
    uint32_t qk[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      ab[it] = a.abase_in[r0 + rk[it]];
      ap[it] = a.apos_in[r0 + rk[it]];
      qk[it] = BATCHED ? a.qid_in[r0 + rk[it]] : 0u;
    }
    int32_t wv[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const bool valid = (uint32_t)(it * WG + tid) < len;
      wv[it] = a.g.gather[valid ? ab[it] + off[it] : ab[it]];
    }
    // kModeBatch: a wave whose items all belong to one query reads that
    // query's level entry once, into scalar registers
    bool wuni = true;
    uint32_t q0 = 0;
    if (BATCHED) {
      q0 = __builtin_amdgcn_readfirstlane(qk[0]);
      bool same = true;
#pragma unroll
      for (int it = 0; it < ITEMS; ++it) same = same && qk[it] == q0;
      wuni = wave_ballot(!same) == 0;
    }

    uint32_t keepbits = 0, cntbits = 0;
    uint32_t nW[ITEMS];
    int64_t nbase[ITEMS];
    uint8_t napos[ITEMS];
    auto evaluate = [&](auto uni_tag) {
      constexpr bool UNI = decltype(uni_tag)::value;
      BatchLevel ubl{};
      if (BATCHED && UNI) ubl = a.blev[q0 * kMaxQ + i];  // uniform address: scalar loads
      // level parameters of every item
      uint32_t p_nbr[ITEMS], p_next_nbr[ITEMS], p_last[ITEMS];
      int32_t p_next_label[ITEMS];
      bool cand[ITEMS];
      if (BATCHED) {
        // candidate test: every item's graph loads issued before any is used;
        // the level entries are read field by field where they are needed
        // (a wave whose items span queries reads them per item, so they do
        // not all stay in registers)
        uint2 dn[ITEMS];
        int32_t lv[ITEMS];
        const bool label_known = a.g.loff != nullptr;
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
          dn[it] = a.g.dne[wv[it]];
          lv[it] = (!label_known && a.g.lab) ? a.g.lab[wv[it]] : 0;
        }
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
          const BatchLevel *bp = a.blev + (qk[it] * kMaxQ + i);
          p_nbr[it] = UNI ? ubl.nbr_mask : bp->nbr_mask;
          p_next_nbr[it] = UNI ? ubl.next_nbr_mask : bp->next_nbr_mask;
          p_next_label[it] = UNI ? ubl.next_label : bp->next_label;
          p_last[it] = (MODE == kModeBatchLast);
          const uint32_t qdeg = UNI ? ubl.qdeg : bp->qdeg;
          const uint64_t qne = UNI ? ubl.qne : bp->qne;
          const int32_t qlab = UNI ? ubl.qlab : bp->qlab;
          const uint32_t smod = UNI ? ubl.slice_mod : bp->slice_mod;
          cand[it] = dn[it].x >= qdeg && (uint64_t)dn[it].y >= qne && (label_known || lv[it] == qlab);
          if (smod && cand[it])
            cand[it] = slice_mix(slice_id(a.g, wv[it])) % smod == (UNI ? ubl.slice_rem : bp->slice_rem);
        }
      } else {
        uint32_t cm[ITEMS];
        if (a.L.no_cmask) {
#pragma unroll
          for (int it = 0; it < ITEMS; ++it) cm[it] = 0xffffu;
        } else {
#pragma unroll
          for (int it = 0; it < ITEMS; ++it) cm[it] = a.cmask[wv[it]];
        }
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
          p_nbr[it] = a.L.nbr_mask;
          p_next_nbr[it] = a.L.next_nbr_mask;
          p_next_label[it] = a.L.next_label;
          p_last[it] = (MODE != kModeNext);
          cand[it] = (cm[it] >> a.L.qbit) & 1;
        }
      }
#pragma unroll
      for (int it = 0; it < ITEMS; ++it) {
        nW[it] = 0;
        nbase[it] = 0;
        napos[it] = 0;
        const bool valid = (uint32_t)(it * WG + tid) < len;
        const int32_t w = wv[it];
        const uint32_t k = rk[it];
        bool keep = valid && cand[it];
        const uint32_t inj = ((1u << i) - 1u) & ~p_nbr[it];
        for (uint32_t m = inj; m; m &= m - 1) {
          const int j = __builtin_ctz(m);
          keep = keep && (row_id(stage_in, s_in, a.rows_in, k * i + j, (r0 + k) * i + j) != w);
        }
        // unique-subgraph mode: id order against symmetric earlier positions
        for (uint32_t m = a.L.sym_lt | a.L.sym_gt; m; m &= m - 1) {
          const int j = __builtin_ctz(m);
          const int32_t x = row_id(stage_in, s_in, a.rows_in, k * i + j, (r0 + k) * i + j);
          keep = keep && (((a.L.sym_lt >> j) & 1) ? x < w : x > w);
        }
        // edge labels: the anchor edge, then each back-edge below
        if (EXT && a.L.use_elab && keep)
          keep = (a.g.elab_gather ? a.g.elab_gather[ab[it] + off[it]] : 0) == a.L.elab_req[ap[it]];
        for (uint32_t m = p_nbr[it]; m; m &= m - 1) {
          const int j = __builtin_ctz(m);
          if (keep && j != ap[it]) {
            const int32_t x = row_id(stage_in, s_in, a.rows_in, k * i + j, (r0 + k) * i + j);
            if (EXT && a.L.use_elab) {
              const int64_t pos = edge_pos(a.g, x, w, probes);
              keep = pos >= 0 && (a.g.elab ? a.g.elab[pos] : 0) == a.L.elab_req[j];
            } else {
              keep = has_edge(a.g, x, w, probes);
            }
          }
        }
        // induced mode: no edge to the earlier non-neighbours either
        for (uint32_t m = EXT ? a.L.non_mask : 0u; m; m &= m - 1) {
          const int j = __builtin_ctz(m);
          if (keep) {
            const int32_t x = row_id(stage_in, s_in, a.rows_in, k * i + j, (r0 + k) * i + j);
            keep = !has_edge(a.g, x, w, probes);
          }
        }
        if (MODE == kModeNext && keep && a.L.la_n)
          keep = lookahead_ok(a, w, stage_in ? s_in + k * i : a.rows_in + (r0 + k) * i);
        if ((MODE == kModeNext || MODE == kModeBatch) && keep && !p_last[it]) {
          // anchor of the next position: the earlier neighbour with the fewest
          // neighbours of the next label; an empty range ends the row here
          uint32_t best = 0xffffffffu;
          int bj = 0;
          int64_t bb = 0;
          for (uint32_t mm = p_next_nbr[it]; mm; mm &= mm - 1) {
            const int j = __builtin_ctz(mm);
            const int32_t x = (j == i) ? w : (row_id(stage_in, s_in, a.rows_in, k * i + j, (r0 + k) * i + j));
            int64_t base;
            const uint32_t d = label_range(a.g, x, p_next_label[it], base);
            if (d < best) {
              best = d;
              bj = j;
              bb = base;
            }
          }
          if (EXT && MODE == kModeNext && best > 0 && (a.L.next_sym_lt | a.L.next_sym_gt)) {
            // unique mode: keep only the ids the next position's order
            // constraints allow; the range is sorted by id, so it narrows to
            // the ids in (lo, hi) by two halving searches
            int64_t lo = -1, hi = (int64_t)1 << 31;
            for (uint32_t mm = a.L.next_sym_lt | a.L.next_sym_gt; mm; mm &= mm - 1) {
              const int j = __builtin_ctz(mm);
              const int32_t x = (j == i) ? w : (row_id(stage_in, s_in, a.rows_in, k * i + j, (r0 + k) * i + j));
              if ((a.L.next_sym_lt >> j) & 1)
                lo = max(lo, (int64_t)x);
              else
                hi = min(hi, (int64_t)x);
            }
            const int32_t *r = a.g.gather + bb;
            uint32_t f = 0, n = best;  // first entry > lo
            while (n > 0) {
              const uint32_t h = n >> 1;
              if ((int64_t)r[f + h] <= lo) {
                f += h + 1;
                n -= h + 1;
              } else {
                n = h;
              }
            }
            uint32_t e = f, m = best - f;  // first entry >= hi
            while (m > 0) {
              const uint32_t h = m >> 1;
              if ((int64_t)r[e + h] < hi) {
                e += h + 1;
                m -= h + 1;
              } else {
                m = h;
              }
            }
            bb += f;
            best = e - f;
          }
          keep = best > 0;
          nW[it] = best;
          nbase[it] = bb;
          napos[it] = (uint8_t)bj;
        }
        if (MODE == kModeBatchLast)
          cntbits |= (uint32_t)keep << it;
        else
          keepbits |= (uint32_t)keep << it;
      }
    };
    if (BATCHED && !wuni)
      evaluate(std::false_type{});
    else
      evaluate(std::true_type{});

    if (MODE == kModeCount) {
      wg_count += __builtin_popcount(keepbits);
    } else if (MODE == kModeBatchLast) {
      {
        // embeddings completed here go to their query's count; each wave keeps
        // a running (query, count) pair, flushed with one atomic when the
        // query changes (acc_k and acc_c are the same on every lane)
        if (wuni) {
          uint64_t c = 0;
#pragma unroll
          for (int it = 0; it < ITEMS; ++it) c += (uint64_t)__popcll(wave_ballot((cntbits >> it) & 1));
          if (c) {
            if (q0 != acc_k) {
              if (lane == 0 && acc_c)
                atomicAdd((unsigned long long *)(a.counts + acc_k), (unsigned long long)acc_c);
              acc_k = q0;
              acc_c = 0;
            }
            acc_c += c;
          }
        } else {
#pragma unroll
          for (int it = 0; it < ITEMS; ++it) {
            bool pend = (cntbits >> it) & 1;
            uint64_t act = wave_ballot(pend);
            while (act) {
              const int leader = __builtin_ctzll(act);
              const uint32_t lk = __shfl(qk[it], leader, kWave);
              const bool mine = pend && qk[it] == lk;
              const uint64_t same = wave_ballot(mine);
              if (lk != acc_k) {
                if (lane == 0 && acc_c)
                  atomicAdd((unsigned long long *)(a.counts + acc_k), (unsigned long long)acc_c);
                acc_k = lk;
                acc_c = 0;
              }
              acc_c += (uint64_t)__popcll(same);
              if (mine) pend = false;
              act = wave_ballot(pend);
            }
          }
        }
      }
    } else {
      // ---- compaction and writes (workgroup barriers)
      {
        // item-major compaction: survivors of item 0 of every lane, then item 1, ...
        uint32_t lofs[ITEMS];
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
          const uint64_t mask = wave_ballot((keepbits >> it) & 1);
          lofs[it] = lane_prefix(mask);
          if (lane == 0) s_cnt[it * NW + wid] = (uint32_t)__popcll(mask);
        }
        __syncthreads();
        if (wid == 0) {
          // exclusive scan of the ITEMS * NW counts (item-major), one lane each
          const uint32_t c = lane < ITEMS * NW ? s_cnt[lane] : 0;
          uint32_t inc = c;
#pragma unroll
          for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t o = __shfl_up(inc, d, kWave);
            if (lane >= d) inc += o;
          }
          if (lane < ITEMS * NW) s_cnt[lane] = inc - c;
          const uint32_t tot = __shfl(inc, kWave - 1, kWave);
          if (lane == 0) {
            s_total = tot;
            s_base = tot ? atomicAdd((unsigned long long *)a.counter, (unsigned long long)tot) : 0;
          }
        }
        __syncthreads();
        const uint32_t total = s_total;
        const uint64_t base = s_base;
        if (total > 0) {
          constexpr bool kIdOrder = (MODE == kModeNext || MODE == kModeBatch);
#pragma unroll
          for (int it = 0; it < ITEMS; ++it) {
            if (!((keepbits >> it) & 1)) continue;
            const uint32_t loc = s_cnt[it * NW + wid] + lofs[it];
            const uint64_t pos = base + loc;
            const uint32_t k = rk[it];
            const int32_t w = wv[it];
            if (kIdOrder) {
              a.W_out[pos] = nW[it];
              a.abase_out[pos] = nbase[it];
              a.apos_out[pos] = napos[it];
              if (MODE == kModeBatch) a.qid_out[pos] = (uint16_t)qk[it];
            }
            if (MODE == kModeNext && a.pack_out) {
              // packed next-level row: word d holds the bits [32d, 32d+32) of
              // the columns laid end to end at b bits each
              const uint32_t b = (uint32_t)a.pack_bits, nw = (uint32_t)((width * b + 31) / 32);
              uint32_t *o32 = reinterpret_cast<uint32_t *>(a.rows_out) + pos * (uint64_t)nw;
              for (uint32_t d = 0; d < nw; ++d) {
                uint32_t word = 0;
                for (int c = 0; c < width; ++c) {
                  const int32_t lo = c * (int32_t)b - 32 * (int32_t)d;  // column start relative to the word
                  if (lo >= 32 || lo + (int32_t)b <= 0) continue;
                  const uint32_t v =
                      (uint32_t)(c == i ? w : (row_id(stage_in, s_in, a.rows_in, k * i + c, (r0 + k) * i + c)));
                  word |= lo >= 0 ? v << lo : v >> -lo;
                }
                o32[d] = word;
              }
              continue;
            }
            // the row in output-column order (emitted rows carry the
            // caller's ids on a renumbered graph)
            auto colval = [&](int c) -> int32_t {
              const int j = kIdOrder ? c : a.L.in_pos[c];
              const int32_t x = j == i ? w : row_id(stage_in, s_in, a.rows_in, k * i + j, (r0 + k) * i + j);
              return (!kIdOrder && a.g.orig) ? a.g.orig[x] : x;
            };
            if (a.staged) {  // into the LDS copy of the tile's rows
              int32_t *o = s_out + loc * (uint32_t)width;
              for (int c = 0; c < width; ++c) o[c] = colval(c);
              continue;
            }
            int32_t *o;
            if (kIdOrder) {
              o = a.rows_out + pos * (uint64_t)width;
            } else {
              const uint64_t slot = pos - a.emit_base;
              if (slot >= a.emit_cap) continue;
              o = a.emit_rows + slot * (uint64_t)width;
            }
            // two columns per 8-byte store when the row starts 8-byte aligned
            int c = 0;
            if (((uintptr_t)o & 7) == 0) {
              for (; c + 1 < width; c += 2)
                *reinterpret_cast<int2 *>(o + c) = make_int2(colval(c), colval(c + 1));
            }
            for (; c < width; ++c) o[c] = colval(c);
          }
          if (a.staged) {
            __syncthreads();
            // contiguous copy of the tile's rows, 16-byte stores where aligned
            uint64_t nints = (uint64_t)total * width;
            int32_t *dst;
            if (kIdOrder) {
              dst = a.rows_out + base * (uint64_t)width;
            } else {
              const uint64_t slot0 = base - a.emit_base;
              const uint64_t room = slot0 < a.emit_cap ? a.emit_cap - slot0 : 0;
              if (room < total) nints = room * (uint64_t)width;
              dst = a.emit_rows + slot0 * (uint64_t)width;
            }
            const uint32_t head = (uint32_t)min<uint64_t>(nints, (4 - (((uintptr_t)dst >> 2) & 3)) & 3);
            if (tid < head) dst[tid] = s_out[tid];
            const uint32_t nvec = (uint32_t)((nints - head) >> 2);
            int4 *dv = reinterpret_cast<int4 *>(dst + head);
            for (uint32_t v = tid; v < nvec; v += WG) {
              const int32_t *sp = s_out + head + 4 * v;
              dv[v] = make_int4(sp[0], sp[1], sp[2], sp[3]);
            }
            const uint32_t tail0 = head + 4 * nvec;
            if (tail0 + tid < nints) dst[tail0 + tid] = s_out[tail0 + tid];
          }
        }
      }
    }
    __syncthreads();  // LDS buffers are rewritten by the next tile
  }
  if (MODE == kModeCount) {
    uint64_t total;
    block_excl_scan<WG>(wg_count, sw, &total);
    if (tid == 0 && total) atomicAdd((unsigned long long *)a.counter, (unsigned long long)total);
  }
  if (MODE == kModeBatchLast) {
    // merge the waves' pending (query, count) pairs, one atomic per query
    __shared__ uint32_t s_acck[NW];
    __shared__ uint64_t s_accc[NW];
    if (lane == 0) {
      s_acck[wid] = acc_k;
      s_accc[wid] = acc_c;
    }
    __syncthreads();
    if (tid == 0) {
      for (int w1 = 0; w1 < NW; ++w1) {
        if (!s_accc[w1]) continue;
        uint64_t c = s_accc[w1];
        for (int w2 = w1 + 1; w2 < NW; ++w2)
          if (s_acck[w2] == s_acck[w1]) {
            c += s_accc[w2];
            s_accc[w2] = 0;
          }
        atomicAdd((unsigned long long *)(a.counts + s_acck[w1]), (unsigned long long)c);
      }
    }
  }
  if (a.probes) {
    uint64_t total;
    block_excl_scan<WG>(probes, sw, &total);
    if (tid == 0 && total) atomicAdd((unsigned long long *)a.probes, (unsigned long long)total);
  }
}

// The expansion's tile map: for tile t of [pair_begin, pair_end), the last
// row r0 with S[r0] <= t0 and the number R of rows the tile touches (every
// row has at least one pair, so they end within len rows of r0), packed as
// r0 | R << 48; one thread per tile, two binary searches.
// Device-driven launches: the row count and pair total are read from device
// memory as the expansion reads them, and only the first `cap` tiles are
// mapped (the expansion searches for the rest).
__global__ void k_tile_rows(const uint64_t *__restrict__ S, uint64_t n_rows, uint64_t pair_begin,
                            uint64_t pair_end, uint32_t tile, const uint64_t *dev_n_rows,
                            const uint64_t *dev_pair_end, uint64_t cap, uint64_t *map) {
  if (dev_pair_end) {
    n_rows = *dev_n_rows;
    pair_end = min(pair_end, *dev_pair_end);
  }
  const uint64_t npairs = pair_end > pair_begin ? pair_end - pair_begin : 0;
  const uint64_t ntiles = min((npairs + tile - 1) / tile, cap);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += stride) {
    const uint64_t t0 = pair_begin + t * tile;
    const uint64_t e = min(t0 + tile, pair_end);
    uint64_t lo = 0, hi = n_rows;  // S[lo] <= t0 < S[hi]
    while (hi - lo > 1) {
      const uint64_t mid = lo + (hi - lo) / 2;
      if (S[mid] <= t0)
        lo = mid;
      else
        hi = mid;
    }
    uint64_t lo2 = lo, hi2 = min(n_rows, lo + (e - t0));  // S[lo2] < e <= S[hi2]
    while (hi2 - lo2 > 1) {
      const uint64_t mid = lo2 + (hi2 - lo2) / 2;
      if (S[mid] < e)
        lo2 = mid;
      else
        hi2 = mid;
    }
    map[t] = lo | ((hi2 - lo) << 48);
  }
}

__global__ void k_zero_u64(uint64_t *p, size_t count) {
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (size_t)gridDim.x * blockDim.x)
    p[k] = 0;
}

constexpr size_t kMaxStageBytes = kExpandStageBytes;

uint32_t grid_for(int64_t work, int wg, uint32_t cap);

template <int WG, int ITEMS>
void launch_expand_t(ExpandArgs a, int mode, hipStream_t s) {
  constexpr uint64_t TILE = (uint64_t)WG * ITEMS;
  const uint64_t span = a.pair_end - a.pair_begin;  // an upper bound when the range is read on the device
  const uint64_t ntiles = span / TILE + (span % TILE != 0);
  if (ntiles == 0) return;
  // persistent-style grid: a few workgroups per CU loop over the tiles, so
  // per-workgroup reductions end in few atomics
  uint64_t grid = ntiles;
  const uint64_t kMaxGrid = 8192;
  if (grid > kMaxGrid) grid = kMaxGrid;
  if (grid >= 8) grid &= ~7ull;
  const int width = (mode == kModeNext || mode == kModeBatch) ? a.L.i + 1 : a.L.q;
  // input staging: room for every row a tile can touch, or, when the level's
  // rows and pairs are known, 16 times the rows an average tile touches
  // (rounded up to a power of two, at least 64): the rare tile with more rows
  // reads them from global memory, and the LDS saved admits more workgroups
  uint64_t in_cap = TILE;
  if (a.level_pairs && !a.pack_in && !a.dev_pair_end) {
    const uint64_t est = TILE * a.n_rows / a.level_pairs + 2;
    uint64_t c = 64;
    while (c < 16 * est && c < TILE) c <<= 1;
    in_cap = std::min<uint64_t>(c, TILE);
  }
  a.in_cap = (uint32_t)in_cap;
  a.use_tile_map = 0;
  if (a.tile_map && a.tile_map_cap) {
    const uint64_t mapped = std::min<uint64_t>(ntiles, a.tile_map_cap);
    hipLaunchKernelGGL(k_tile_rows, dim3(grid_for((int64_t)mapped, 256, 4096)), dim3(256), 0, s, a.S, a.n_rows,
                       a.pair_begin, a.pair_end, (uint32_t)TILE, a.dev_n_rows, a.dev_pair_end, a.tile_map_cap,
                       a.tile_map);
    GSM_HIP(hipGetLastError());
    a.use_tile_map = 1;
  }
  const size_t in_bytes = in_cap * (size_t)a.L.i * sizeof(int32_t);
  const size_t out_bytes = TILE * (size_t)width * sizeof(int32_t);
  const size_t stage_max = a.stage_limit ? a.stage_limit : kMaxStageBytes;
  a.stage_in = (in_bytes <= stage_max) ? 1 : 0;
  if (!a.stage_in) a.in_cap = 0;
  if (a.pack_in && !a.stage_in) throw Error{GSM_E_DEVICE, "packed frontier rows need staging"};
  if ((a.pack_in || a.pack_out) && (mode == kModeBatch || mode == kModeBatchLast))
    throw Error{GSM_E_DEVICE, "packed frontier rows in a batched launch"};
  a.staged = (a.stage_out_ok && !(mode == kModeNext && a.pack_out) && mode != kModeCount &&
              mode != kModeBatchLast && (a.stage_in ? in_bytes : 0) + out_bytes <= stage_max)
                 ? 1
                 : 0;
  const size_t smem = (a.stage_in ? in_bytes : 0) + (a.staged ? out_bytes : 0);
  const dim3 gd((uint32_t)grid), bd(WG);
  const bool el = a.L.use_elab != 0 || a.L.non_mask != 0 || (a.L.next_sym_lt | a.L.next_sym_gt) != 0;
  switch (mode) {
    case kModeNext:
      if (el)
        hipLaunchKernelGGL((k_expand<WG, ITEMS, kModeNext, true>), gd, bd, smem, s, a);
      else
        hipLaunchKernelGGL((k_expand<WG, ITEMS, kModeNext, false>), gd, bd, smem, s, a);
      break;
    case kModeCount:
      if (el)
        hipLaunchKernelGGL((k_expand<WG, ITEMS, kModeCount, true>), gd, bd, smem, s, a);
      else
        hipLaunchKernelGGL((k_expand<WG, ITEMS, kModeCount, false>), gd, bd, smem, s, a);
      break;
    case kModeBatch:
      hipLaunchKernelGGL((k_expand<WG, ITEMS, kModeBatch, false>), gd, bd, smem, s, a);
      break;
    case kModeBatchLast:
      hipLaunchKernelGGL((k_expand<WG, ITEMS, kModeBatchLast, false>), gd, bd, smem, s, a);
      break;
    default:
      if (el)
        hipLaunchKernelGGL((k_expand<WG, ITEMS, kModeEmit, true>), gd, bd, smem, s, a);
      else
        hipLaunchKernelGGL((k_expand<WG, ITEMS, kModeEmit, false>), gd, bd, smem, s, a);
      break;
  }
}

template <int WG>
void launch_expand_wg(const ExpandArgs &a, int mode, int items, hipStream_t s) {
  switch (items) {
    case 1: launch_expand_t<WG, 1>(a, mode, s); break;
    case 2: launch_expand_t<WG, 2>(a, mode, s); break;
    case 8: launch_expand_t<WG, 8>(a, mode, s); break;
    default: launch_expand_t<WG, 4>(a, mode, s); break;
  }
}

uint32_t grid_for(int64_t work, int wg, uint32_t cap) {
  int64_t g = (work + wg - 1) / wg;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

}  // namespace

// --------------------------------------------------------------- launchers --

void launch_graph_stats(const gsm_graph &g, hipStream_t s) {
  if (g.n == 0) return;
  hipLaunchKernelGGL(k_graph_stats, dim3(grid_for(g.n * 16, 256, 1u << 16)), dim3(256), 0, s,
                     g.rp, g.col, g.lab, g.n, g.deg, g.ne0, g.dne);
  GSM_HIP(hipGetLastError());
}

void launch_build_hub_bitmaps(const gsm_graph &g, const int32_t *hubs, int64_t nhubs, hipStream_t s) {
  if (nhubs <= 0) return;
  hipLaunchKernelGGL(k_hub_bitmaps, dim3((uint32_t)std::min<int64_t>(nhubs, 65535)), dim3(256), 0, s, g.rp, g.col,
                     hubs, nhubs, g.hub_bits, g.hub_words);
  GSM_HIP(hipGetLastError());
}

DeviceGraph device_graph(const gsm_graph &g) {
  return DeviceGraph{g.rp,     g.col,      g.lab,         g.deg,  g.ne0,
                     g.dne,    g.col_lab ? g.col_lab : g.col,     g.loff, g.loff_stride,
                     g.n,      g.elab,     g.elab_lab ? g.elab_lab : g.elab,
                     g.vdesc, g.hub_bits, g.hub_words, g.lab_vert, g.orig};
}

void launch_filter_init(const DeviceGraph &g, const QueryArgs &qa, uint16_t *cmask, hipStream_t s) {
  if (g.n == 0) return;
  hipLaunchKernelGGL(k_filter_init, dim3(grid_for(g.n, 256, 1u << 16)), dim3(256), 0, s, g, qa, cmask);
  GSM_HIP(hipGetLastError());
}

void launch_filter_refine(const DeviceGraph &g, const int32_t *heavy, int64_t nheavy,
                          const QueryArgs &qa, const uint16_t *prev, uint16_t *next, hipStream_t s) {
  if (g.n == 0) return;
  hipLaunchKernelGGL(k_refine_light, dim3(grid_for(g.n * 16, 256, 1u << 16)), dim3(256), 0, s, g, qa,
                     prev, next);
  GSM_HIP(hipGetLastError());
  if (nheavy > 0) {
    hipLaunchKernelGGL(k_refine_heavy, dim3(grid_for(nheavy * 256, 256, 1u << 16)), dim3(256), 0, s, g,
                       qa, heavy, nheavy, prev, next);
    GSM_HIP(hipGetLastError());
  }
}

void launch_compact_first(const DeviceGraph &g, const uint16_t *cmask, uint32_t qbit,
                          int32_t next_label, int32_t *rows, uint32_t *W, int64_t *abase,
                          uint8_t *apos, uint64_t *counter, int32_t *emit_rows, uint64_t emit_cap,
                          hipStream_t s) {
  if (g.n == 0) return;
  hipLaunchKernelGGL(k_compact_first, dim3(grid_for(g.n, 256, 1u << 14)), dim3(256), 0, s, g, cmask,
                     qbit, next_label, rows, W, abase, apos, counter, emit_rows, emit_cap);
  GSM_HIP(hipGetLastError());
}

size_t scan_scratch_elems() { return kScanBlocks; }

void launch_zero_u64(uint64_t *p, size_t count, hipStream_t s) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for((int64_t)count, 256, 1024)), dim3(256), 0, s, p, count);
  GSM_HIP(hipGetLastError());
}

void launch_scan(const uint32_t *W, const uint64_t *n_dev, uint64_t *S, uint64_t *total_out,
                 uint64_t *scratch, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_reduce, dim3(kScanBlocks), dim3(kScanWG), 0, s, W, n_dev, scratch);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanWG), 0, s, scratch, n_dev, S, total_out);
  hipLaunchKernelGGL(k_scan_down, dim3(kScanBlocks), dim3(kScanWG), 0, s, W, n_dev, scratch, S);
  GSM_HIP(hipGetLastError());
}

void launch_compact_first_batch(const DeviceGraph &g, const FirstBatch *fb_dev, int nq, int64_t max_class,
                                int32_t *rows, uint16_t *qid, uint32_t *W, int64_t *abase, uint8_t *apos,
                                uint64_t *counter, uint64_t *counts, uint64_t *pairs1, hipStream_t s) {
  if (g.n == 0 || nq == 0) return;
  hipLaunchKernelGGL(k_compact_first_batch, dim3(grid_for(max_class, 256, 1024), nq), dim3(256), 0, s, g, fb_dev,
                     rows, qid, W, abase, apos, counter, counts, pairs1);
  GSM_HIP(hipGetLastError());
}

void launch_expand(const ExpandArgs &a, int mode, int wg, int items, hipStream_t s) {
  if (a.pair_end <= a.pair_begin) return;
  switch (wg) {
    case 128: launch_expand_wg<128>(a, mode, items, s); break;
    case 512: launch_expand_wg<512>(a, mode, items, s); break;
    default: launch_expand_wg<256>(a, mode, items, s); break;
  }
  GSM_HIP(hipGetLastError());
}

}  // namespace gsm
