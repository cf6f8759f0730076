// Internal types shared by the host driver and the HIP kernels of libgsm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "gsm.h"

namespace gsm {

constexpr int kMaxQ = GSM_MAX_QUERY_VERTICES;

// ------------------------------------------------------------------ errors --

void set_error(const std::string &msg);

struct Error {
  gsm_status status;
  std::string msg;
};

#define GSM_HIP(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw ::gsm::Error{GSM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// ------------------------------------------------------------ device buffer --

// Device allocation that grows on demand and is reused across calls.
// hipMalloc that throws Error{GSM_E_OOM} on failure (and when the test hook
// gsm_testing_fail_allocations has used up its allowance).
void device_alloc(void **p, size_t bytes);
// The same, stream-ordered (hipMallocAsync on s): no device-wide wait.
void device_alloc_async(void **p, size_t bytes, hipStream_t s);

// A device buffer owned by one workspace.  Growing it frees the old block
// and allocates the new one in the order of the stream that uses it
// (hipFreeAsync / hipMallocAsync), so a workspace that grows waits for its
// own stream's work only, never for other streams on the device.
// A fixed buffer is a window of memory the library does not own (the
// no-allocation scratch): it never allocates or frees, and asking it for more
// than its size is a GSM_E_BUDGET error.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  bool fixed = false;
  bool pooled = false;  // from hipMallocAsync: always returned with hipFreeAsync
  void reserve(size_t want, hipStream_t s);  // keeps no contents
  void release(hipStream_t s = nullptr);     // s: free in that stream's order
  void set_fixed(void *p, size_t b) {
    release();
    ptr = p;
    bytes = b;
    fixed = true;
  }
  template <typename T>
  T *as() const { return static_cast<T *>(ptr); }
  ~DevBuf() { release(); }
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
};

// ------------------------------------------------------------------- graph --

struct Workspace;

}  // namespace gsm

struct gsm_graph {
  int64_t n = 0;
  int64_t nnz = 0;
  bool labelled = false;
  int32_t max_label = 0;
  int64_t max_degree = 0;
  // device CSR and per-vertex data
  int64_t *rp = nullptr;     // n+1
  int32_t *col = nullptr;    // nnz
  int32_t *lab = nullptr;    // n, or null when unlabelled
  uint32_t *deg = nullptr;   // n
  uint64_t *ne0 = nullptr;   // n: sum over neighbours of (label+1); null when unlabelled
  uint2 *dne = nullptr;      // n: (degree, NE saturated to 32 bits): one load per inline test
  int32_t *heavy = nullptr;  // vertices with degree > kHeavyDegree
  int64_t nheavy = 0;
  // adjacency bitmaps of the highest-degree vertices (membership in one load):
  // bitmap s is hub_words 32-bit words at hub_bits + s * hub_words, bit w set
  // when w is a neighbour; vdesc[v] = (list start low, high, length, bitmap
  // index or -1), the one load an edge check starts with
  int4 *vdesc = nullptr;
  uint32_t *hub_bits = nullptr;
  uint64_t hub_words = 0;
  int64_t nhubs = 0;
  // vertices sorted by label (labelled graphs): the vertices of label l are
  // lab_vert[lab_start[l] .. lab_start[l+1])
  int32_t *lab_vert = nullptr;
  std::vector<int64_t> lab_start;
  // GSM_GRAPH_DEGREE_ORDER: vertices renumbered by ascending degree; every
  // array above is in the internal numbering and orig[v] is the caller's id of
  // internal vertex v (device and host copies); null / empty otherwise
  int32_t *orig = nullptr;
  std::vector<int32_t> h_orig;
  // label-grouped adjacency (labelled graphs with at most kMaxTableLabels labels):
  // row v of col_lab holds v's neighbours sorted by (label, id), and
  // loff[v * loff_stride + l] is where label l starts inside that row.
  int32_t *col_lab = nullptr;
  uint32_t *loff = nullptr;
  // edge labels per CSR entry (aligned with col), and in col_lab order; null = none
  int32_t *elab = nullptr;
  int32_t *elab_lab = nullptr;
  int32_t loff_stride = 0;  // labels + 1, or 0 when there is no table
  // host statistics for the planner
  std::vector<int64_t> label_count;  // vertices per label
  std::vector<int64_t> deg_ge;       // deg_ge[d] = #vertices with degree >= d (d <= max_degree+1)
  std::mutex mu;                     // guards ws
  gsm::Workspace *ws = nullptr;
};

struct gsm_query {
  int32_t q = 0;
  std::vector<int32_t> edges;  // 2*ne
  int32_t label[gsm::kMaxQ] = {0};
  uint32_t adj[gsm::kMaxQ] = {0};  // adjacency bitmask by query id
  // edge labels (has_elab): elab[a][b] = label of query edge {a, b}
  bool has_elab = false;
  int32_t elab[gsm::kMaxQ][gsm::kMaxQ] = {{0}};
  // symmetry: |Aut(Q)| and constraints f(sym_pairs[2k]) < f(sym_pairs[2k+1])
  uint64_t aut = 1;
  std::vector<int32_t> sym_pairs;
};

namespace gsm {

constexpr int64_t kHeavyDegree = 2048;
// Vertices of at least this degree get an adjacency bitmap, highest degree
// first, while the bitmaps fit kHubBitmapBytes and a quarter of the free
// device memory.
constexpr int64_t kHubMinDegree = 512;
constexpr uint64_t kHubBitmapBytes = uint64_t(8) << 30;
constexpr int32_t kMaxTableLabels = 64;
// Tiles a host-driven expansion launch may map before it starts (8 bytes
// each); larger launches search for their rows in the kernel.
constexpr uint64_t kTileMapWords = uint64_t(1) << 20;

// ------------------------------------------------------------------- plan --

struct Plan {
  int32_t q = 0;
  int32_t order[kMaxQ];      // query id at position i
  int32_t pos[kMaxQ];        // position of query id u
  int32_t parent[kMaxQ];     // position of the tree parent
  uint32_t backmask[kMaxQ];  // positions j < i adjacent to position i
  // per query id (filter inputs)
  int64_t qdeg[kMaxQ];
  uint64_t qne[kMaxQ];
  int32_t qlab[kMaxQ];
};

Plan make_plan(const gsm_graph &g, const gsm_query &q);

// Fills q.aut and q.sym_pairs (unique-subgraph mode).
void compute_symmetry(gsm_query &q);

// Query description handed to kernels by value.
struct QueryArgs {
  int32_t q;
  int32_t root_bit;       // query id whose candidates are sliced, -1 none
  uint32_t root_mod, root_rem;
  int32_t use_deg, use_ne;
  int32_t qlab[kMaxQ];
  uint32_t qdeg[kMaxQ];
  uint64_t qne[kMaxQ];
};

// Labels per later query vertex that the two-step look-ahead tests (those
// with the most neighbours of that label first).
constexpr int kLa2Labels = 4;

// One expansion level: rows hold positions 0..i-1; position i is matched.
struct LevelArgs {
  int32_t i;               // matched positions per input row
  int32_t q;
  uint32_t nbr_mask;       // positions j < i adjacent to position i
  uint32_t qbit;           // cmask bit (query id) of position i
  uint32_t no_cmask;       // skip the candidate mask test of position i (it can only prune)
  uint32_t next_nbr_mask;  // positions j <= i adjacent to position i+1 (0 at the last level)
  int32_t next_label;      // label of position i+1
  int32_t out_col[kMaxQ];  // emit: output column (query id) of position j
  int32_t in_pos[kMaxQ];   // emit: position of output column (query id) c
  // one-step look-ahead on a new row (0 tests = off): for each later
  // position adjacent to position i, the new vertex needs at least la_need
  // neighbours of that position's label, and one of them outside the row
  // that is a candidate of it (checked when the label group has at most
  // kLookaheadScan entries)
  // unique-subgraph mode: positions j < i whose id must be below (sym_lt)
  // or above (sym_gt) the new vertex's id
  uint32_t sym_lt, sym_gt;
  // and the same for position i+1 against positions j <= i (j = i: the new
  // vertex): the next range is cut to the ids they allow (kModeNext)
  uint32_t next_sym_lt, next_sym_gt;
  // induced mode: positions j < i not adjacent to position i, whose ids must
  // not be neighbours of the new vertex
  uint32_t non_mask;
  // edge labels: when use_elab, the edge to earlier neighbour position j must
  // carry label elab_req[j]
  int32_t use_elab;
  int32_t elab_req[kMaxQ];
  int32_t la_n;
  int32_t la_label[kMaxQ];
  uint32_t la_qbit[kMaxQ];
  uint32_t la_need[kMaxQ];
  // two-step look-ahead (la2 != 0): the witness found for look-ahead entry f
  // (a neighbour of the new vertex that could take that later query vertex)
  // must itself have at least la2_need[f][t] neighbours of label
  // la2_label[f][t], t < la2_n[f]: the later query vertex's own neighbours
  int32_t la2;
  uint8_t la2_n[kMaxQ];
  int32_t la2_label[kMaxQ][kLa2Labels];
  uint32_t la2_need[kMaxQ][kLa2Labels];
};

// Longest label group of the new vertex that the look-ahead scans.
constexpr uint32_t kLookaheadScan = 32;

// --------------------------------------------------------------- kernels --

struct DeviceGraph {
  const int64_t *rp;
  const int32_t *col;      // rows sorted by id (membership tests)
  const int32_t *lab;
  const uint32_t *deg;
  const uint64_t *ne0;
  const uint2 *dne;        // (degree, NE saturated to 32 bits)
  const int32_t *gather;   // rows the expansion reads: col_lab when the table exists, else col
  const uint32_t *loff;    // label offsets per row, or null
  int32_t loff_stride;
  int64_t n;
  const int32_t *elab;         // edge label per col entry, or null (every edge has label 0)
  const int32_t *elab_gather;  // edge label per gather entry, or null
  const int4 *vdesc;           // per vertex: list start (low, high), length, bitmap index or -1
  const uint32_t *hub_bits;
  uint64_t hub_words;
  const int32_t *lab_vert;     // vertices sorted by label, or null
  const int32_t *orig;         // caller's id of each vertex when renumbered by degree, or null
};

// Each launcher enqueues on `s` and returns immediately.
void launch_graph_stats(const gsm_graph &g, hipStream_t s);
void launch_filter_init(const DeviceGraph &g, const QueryArgs &qa, uint16_t *cmask, hipStream_t s);
void launch_filter_refine(const DeviceGraph &g, const int32_t *heavy, int64_t nheavy,
                          const QueryArgs &qa, const uint16_t *prev, uint16_t *next, hipStream_t s);
// F1: vertices with bit `qbit` set.  With rows != null, also the neighbour
// range of label next_label (W, abase), dropping vertices whose range is empty.
// With emit_rows, writes the vertices as one-column rows (capped).
void launch_compact_first(const DeviceGraph &g, const uint16_t *cmask, uint32_t qbit,
                          int32_t next_label, int32_t *rows, uint32_t *W, int64_t *abase,
                          uint8_t *apos, uint64_t *counter, int32_t *emit_rows, uint64_t emit_cap,
                          hipStream_t s);
void build_label_table(gsm_graph &g, const int64_t *h_rp, const int32_t *h_col, const int32_t *h_lab);
// Adjacency bitmaps of the listed vertices (hub_bits already
// allocated and hub_bits zeroed): bitmap s gets the neighbours of hubs[s].
void launch_build_hub_bitmaps(const gsm_graph &g, const int32_t *hubs, int64_t nhubs, hipStream_t s);
// The device view of a graph.
DeviceGraph device_graph(const gsm_graph &g);
// S[0..N] = exclusive scan of W[0..N-1]; N read from device *n_dev; scratch >= scan_scratch_bytes()
size_t scan_scratch_elems();
// p[0..count) = 0 with a kernel (no memset node, so a captured stream replays it correctly)
void launch_zero_u64(uint64_t *p, size_t count, hipStream_t s);
void launch_scan(const uint32_t *W, const uint64_t *n_dev, uint64_t *S, uint64_t *total_out,
                 uint64_t *scratch, hipStream_t s);

// kModeBatch / kModeBatchLast: rows of many queries of one size, tagged by
// query; kModeBatch writes the next level, kModeBatchLast (the queries' last
// vertex) adds to per-query counts.
enum ExpandMode { kModeNext = 0, kModeCount = 1, kModeEmit = 2, kModeBatch = 3, kModeBatchLast = 4 };

// Per (query, level) parameters of a batched expansion.
// The batched path tests candidates inline against the graph's per-vertex
// label, degree and neighbourhood encoding (round 0 of the filter), so no
// per-query candidate array is needed.
struct BatchLevel {
  uint32_t nbr_mask;       // positions j < i adjacent to position i
  uint32_t next_nbr_mask;  // positions j <= i adjacent to position i+1
  int32_t next_label;      // label of position i+1
  uint16_t qbit;           // query id of position i
  uint16_t last;           // position i is the query's last: count, do not write
  uint64_t qne;            // NE of position i's query vertex (0 = no test)
  uint32_t qdeg;           // degree of position i's query vertex (0 = no test)
  int32_t qlab;            // label of position i's query vertex
  // root slice on position i's query vertex: keep w with
  // splitmix64(w) % slice_mod == slice_rem (slice_mod 0 = no slice)
  uint32_t slice_mod, slice_rem;
};

// Root slice of one query (the gsm_match_opts convention): keep embeddings
// with splitmix64(f(qvertex)) % mod == rem; qvertex < 0 = the whole query.
struct RootSlice {
  int32_t qvertex = -1;
  uint32_t mod = 1, rem = 0;
};

struct ExpandArgs {
  DeviceGraph g;
  const uint16_t *cmask;
  const int32_t *rows_in;   // N x i
  const uint8_t *apos_in;   // N: anchor position
  const int64_t *abase_in;  // N: first gather index of the row's pair range
  const uint64_t *S;        // N+1
  uint64_t n_rows;         // N
  uint64_t pair_begin, pair_end;
  // kModeNext outputs
  int32_t *rows_out;  // x (i+1)
  uint32_t *W_out;
  uint8_t *apos_out;
  int64_t *abase_out;
  // shared counter: rows written (next) / embeddings counted (count, emit)
  uint64_t *counter;
  uint64_t *probes;  // binary-search steps of the back-edge checks
  // kModeEmit output
  int32_t *emit_rows;  // x q, query-id columns
  uint64_t emit_base;  // rows already emitted before this launch (for the cap)
  uint64_t emit_cap;
  // kModeBatch: rows of many queries; row r belongs to query qid_in[r]
  const uint16_t *qid_in;
  uint16_t *qid_out;
  const BatchLevel *blev;  // [nq * kMaxQ], entry (k, i)
  uint64_t *counts;        // per-query embedding counts
  // packed frontier rows (b = pack_bits bits per id, ceil(i*b/32) 32-bit
  // words per row of i ids): the input rows (pack_in, then they are always
  // staged in LDS) and the next level's rows (pack_out, kModeNext)
  int32_t pack_bits, pack_in, pack_out;
  // device-driven launch (dev_pair_end != null): the row count and the pair
  // total are read from *dev_n_rows and *dev_pair_end; pair_end is then the
  // capacity bound, and a total above it sets *overflow
  const uint64_t *dev_n_rows;
  const uint64_t *dev_pair_end;
  uint32_t *overflow;
  uint32_t stage_limit;  // LDS bytes for staging rows (0 = kExpandStageBytes)
  int32_t staged;        // output rows pass through LDS (dynamic shared memory)
  int32_t stage_in;      // the tile's input rows are copied to LDS
  uint32_t in_cap;       // rows the input staging holds (set by the launcher)
  uint64_t level_pairs;  // pairs of the whole level (0: unknown), sizes in_cap
  int32_t stage_out_ok;  // the caller allows output staging
  // a buffer of tile_map_cap words the launcher fills, before the expansion,
  // with the first row and row count of each of the first tile_map_cap tiles
  // (such a tile reads one word instead of searching S); null = search
  uint64_t *tile_map;
  uint64_t tile_map_cap;
  int32_t use_tile_map;  // set by the launcher
  LevelArgs L;
};

void launch_expand(const ExpandArgs &a, int mode, int wg, int items, hipStream_t s);
// Most LDS a launch uses to stage its tile's input and output rows, by
// default and at most.
constexpr size_t kExpandStageBytes = 48 * 1024;
constexpr size_t kExpandStageMax = 64 * 1024;

// Batched helpers: qpairs[q] += W[r] over the *n_dev rows r of query qid[r];
// rows whose query is marked in evicted get W = 1 and qid = retired (a query
// slot whose candidate test fails).  rows_hint bounds *n_dev (it only sizes
// the grid).
void launch_query_pairs(const uint32_t *W, const uint16_t *qid, const uint64_t *n_dev, uint64_t rows_hint,
                        uint64_t *qpairs, hipStream_t s);
void launch_retire_evicted(uint32_t *W, uint16_t *qid, const uint64_t *n_dev, uint64_t rows_hint,
                           const uint8_t *evicted, uint16_t retired, hipStream_t s);
// evicted[k] = 1 for every query k < nq with qpairs[k] > threshold (kept once set).
void launch_mark_evicted(const uint64_t *qpairs, int nq, uint64_t threshold, uint8_t *evicted, hipStream_t s);

// First frontier of every query: rows tagged with the query id; queries with a
// single vertex are counted into counts[k] directly.
struct FirstBatch {
  uint64_t qne0;      // position 0: NE (0 = no test)
  uint32_t qdeg0;     // position 0: degree (0 = no test)
  int32_t qlab0;      // position 0: label
  int32_t label1;     // label of position 1 (unused when q == 1)
  int32_t single;     // q == 1
  uint32_t slice_mod, slice_rem;  // root slice on position 0 (slice_mod 0 = none)
  int64_t vbegin, vend;           // the label class of position 0 in lab_vert (or [0, n))
};
// max_class: the largest vend - vbegin over the queries (sizes the grid).
void launch_compact_first_batch(const DeviceGraph &g, const FirstBatch *fb_dev, int nq, int64_t max_class,
                                int32_t *rows, uint16_t *qid, uint32_t *W, int64_t *abase, uint8_t *apos,
                                uint64_t *counter, uint64_t *counts, uint64_t *pairs1, hipStream_t s);
// The single-query entry: gsm_match (fixed_ws = null: the graph's workspace,
// under its lock) or gsm_match_noalloc (a fixed workspace over the
// no-allocation scratch).
gsm_status match_call(gsm_graph_t g, gsm_query_t qh, const gsm_match_opts *opts, uint64_t *count,
                      int32_t *rows, uint64_t rows_cap, uint64_t *rows_written, Workspace *fixed_ws);
// Count-only match of one query on the workspace (the single-query driver),
// restricted to the root slice rs.
uint64_t match_count_one(gsm_graph &g, const gsm_query &q, const gsm_match_opts &o, Workspace &ws,
                         const RootSlice &rs);
// A batched match (queries of one size) advanced one step at a time by its
// caller: a step is one level's scan and read-back or one chunk's expansion,
// so the serving engine can interleave the steps of several runs and start
// new arrivals between them.  Memory comes from ws within o's budget.
class StepRun {
 public:
  virtual ~StepRun() = default;
  virtual bool step() = 0;  // false once every level is done
  // Counts after the last step (waits for the stream); moved[k] != 0 when
  // query k left the shared launches (its count is then not valid here).
  virtual void finish(uint64_t *counts, std::vector<uint8_t> &moved) = 0;
};

class BatchRun : public StepRun {
 public:
  BatchRun(gsm_graph &g, const gsm_query *const *qs, int nq, const gsm_match_opts &o, Workspace &ws,
           const RootSlice *slices, uint64_t evict_pairs);
  ~BatchRun() override;
  bool step() override;
  void finish(uint64_t *counts, std::vector<uint8_t> &moved) override;

 private:
  struct Impl;
  std::unique_ptr<Impl> impl;
};

// One query, count only, on the query-uniform kernels, step by step.
std::unique_ptr<StepRun> make_single_count_run(gsm_graph &g, const gsm_query &q, const gsm_match_opts &o,
                                               Workspace &ws, const RootSlice &rs);

// Smallest budget gsm_match accepts for a query of q vertices, count only.
uint64_t min_budget_bytes_single(int64_t n, int q);
// Smallest batched budget for nq queries of q vertices (first frontiers at
// n rows each, one row per further level).
uint64_t min_budget_bytes_batch(const gsm_graph &g, int nq, int q);
// Counts of a set of queries on the workspace (the batched driver, no
// locking); slices: one root slice per query, or null for none.
void match_batch_on(gsm_graph &g, const gsm_query *const *qs, int nq, const gsm_match_opts &o,
                    Workspace &ws, uint64_t *counts, uint64_t *launches, gsm_stats *st,
                    const RootSlice *slices);

// -------------------------------------------------------------- workspace --

// Buffers of the device row sort.
struct SortBuffers {
  DevBuf keys[2], hist, offs, len, scratch;
  DevBuf rows;  // rows copied in from host memory
};

// Sorts N rows of q int32 ids in [0, n) on the device, lexicographically
// ascending, in place (radix sort of the rows packed into integer keys).
void sort_rows_device(int32_t *rows, uint64_t N, int q, int64_t n, SortBuffers &sb, hipStream_t s);

struct Workspace {
  SortBuffers sort;
  DevBuf cmask, cmask2;
  DevBuf rows[kMaxQ], W[kMaxQ], apos[kMaxQ], abase[kMaxQ], S[kMaxQ];
  DevBuf qid[kMaxQ];  // batched rows: query of each row
  DevBuf tables;      // batched per-query parameter tables
  DevBuf counts;      // batched per-query counts
  DevBuf qpairs;      // batched per-query pairs of one level
  DevBuf evicted;     // batched: queries taken out of the shared launches
  DevBuf counters;  // kMaxQ + 8 uint64
  DevBuf scan_scratch;
  DevBuf emit;      // staging for host-bound rows
  DevBuf tilemap;   // expansion tile map (kTileMapWords words)
  uint64_t *h_counters = nullptr;  // pinned host mirror (a plain host array in a fixed workspace)
  std::vector<hipEvent_t> events;  // profiling event pool
  // Fixed workspace (no device allocation): every buffer is a window of
  // [fixed_base, fixed_base + fixed_bytes); counters and scan scratch sit at
  // its start, the rest is laid out per call once the level capacities are
  // known.
  char *fixed_base = nullptr;
  size_t fixed_bytes = 0;
  uint64_t h_local[64];
  // batched groups run device-driven: the captured launch sequences of the
  // most recent groups, replayed while the same work is asked for again
  // (key: every pointer and size the launches take; most recent last), and
  // the stream they are captured on
  std::vector<std::pair<std::string, hipGraphExec_t>> graphs;
  hipStream_t capture_stream = nullptr;
  static constexpr size_t kMaxGraphs = 16;
  Workspace();
  Workspace(void *base, size_t bytes);  // fixed
  ~Workspace();
  // bytes at the start of a fixed workspace taken by counters and scan scratch
  static size_t fixed_header_bytes();
};

}  // namespace gsm
