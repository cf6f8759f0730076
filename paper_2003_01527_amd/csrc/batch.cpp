// Batched driver: many queries of one size share every launch.  Rows of all
// of them live in one frontier per level, each tagged with its query; one
// first-frontier launch, and per level one scan and one expansion launch serve
// the whole group, chunked by the memory budget exactly like a single query.
// The last level adds each completed embedding to its query's count.  Candidates are tested inline against
// the graph's label, degree and neighbourhood encoding (the filter's first
// round): per-query candidate arrays of n entries each would make every
// candidate test of a large batch miss the caches, and refinement rounds are
// a pruning choice that never changes a count.
#include <algorithm>
#include <chrono>
#include <exception>
#include <cstring>

#include <cstddef>

#include "gsm_internal.h"

namespace gsm {

namespace {

constexpr int kCntRows = 0;
constexpr int kCntPairs = 16;
constexpr int kCntProbes = 33;
constexpr int kCntOverflow = 40;  // device-driven run: a level's pairs passed its capacity

struct BatchMatcher {
  gsm_graph &g;
  std::vector<const gsm_query *> qs;
  Workspace &ws;
  hipStream_t s;
  int rounds, use_deg, use_ne, wg, items;
  uint32_t stage_bytes = 0;
  uint64_t budget;
  int nq = 0, maxq = 0;
  std::vector<Plan> plans;
  DeviceGraph dg;
  uint64_t cap[kMaxQ];
  uint64_t *dcnt;
  BatchLevel *d_bl = nullptr;
  FirstBatch *d_fb = nullptr;
  int64_t max_class = 0;  // the largest label class a first frontier scans
  uint64_t *d_counts = nullptr;
  uint64_t launches = 0;
  uint64_t level_pairs[kMaxQ] = {0};
  uint64_t level_rows[kMaxQ] = {0};
  // a query whose (row, neighbour) pairs at some level exceed evict_pairs
  // leaves the shared launches (its rows expand to nothing from then on) and
  // is matched alone afterwards: a query-uniform launch is cheaper per pair
  uint64_t evict_pairs = 0;  // 0 = never
  std::vector<uint8_t> evicted;
  std::vector<uint64_t> h_qpairs;
  bool any_evicted = false;
  std::vector<RootSlice> slices;  // per query

  BatchMatcher(gsm_graph &g_, const gsm_query *const *q_, int nq_, Workspace &ws_, hipStream_t s_,
               const RootSlice *sl)
      : g(g_), qs(q_, q_ + nq_), ws(ws_), s(s_), nq(nq_) {
    slices.assign(nq, RootSlice{});
    if (sl) slices.assign(sl, sl + nq);
    dg = device_graph(g);
    dcnt = ws.counters.as<uint64_t>();
    for (auto *q : qs) {
      plans.push_back(make_plan(g, *q));
      maxq = std::max(maxq, q->q);
    }
  }

  void sync() { GSM_HIP(hipStreamSynchronize(s)); }

  // launches of a call that fails part-way finish before the workspace is reused
  ~BatchMatcher() {
    if (std::uncaught_exceptions() > 0) (void)hipStreamSynchronize(s);
  }

  void fetch_counters() {
    GSM_HIP(hipMemcpyAsync(ws.h_counters, dcnt, 64 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    sync();
  }

  // query slot nq: rows of evicted queries are retagged to it; every
  // candidate test fails there (no vertex has 2^32 - 1 neighbours)
  void upload_tables() {
    if (!ws.fixed_base) ws.tilemap.reserve(kTileMapWords * sizeof(uint64_t), s);
    std::vector<BatchLevel> bl((size_t)(nq + 1) * kMaxQ);
    for (int i = 0; i < kMaxQ; ++i) {
      BatchLevel &e = bl[(size_t)nq * kMaxQ + i];
      std::memset(&e, 0, sizeof(e));
      e.qdeg = 0xffffffffu;
      e.qne = 0xffffffffull;
      e.qlab = -1;
    }
    std::vector<FirstBatch> fb(nq);
    std::memset(fb.data(), 0, fb.size() * sizeof(FirstBatch));
    for (int k = 0; k < nq; ++k) {
      const Plan &p = plans[k];
      for (int i = 0; i < p.q; ++i) {
        BatchLevel &e = bl[(size_t)k * kMaxQ + i];
        std::memset(&e, 0, sizeof(e));
        e.nbr_mask = p.backmask[i];
        e.next_nbr_mask = (i + 1 < p.q) ? p.backmask[i + 1] : 0;
        e.next_label = (i + 1 < p.q) ? p.qlab[p.order[i + 1]] : 0;
        e.qbit = (uint16_t)p.order[i];
        e.last = (i + 1 == p.q) ? 1 : 0;
        const int u = p.order[i];
        e.qlab = p.qlab[u];
        e.qdeg = use_deg ? (uint32_t)p.qdeg[u] : 0;
        e.qne = use_ne ? std::min<uint64_t>(p.qne[u], 0xffffffffull) : 0;
      }
      const RootSlice &rs = slices[k];
      if (rs.qvertex >= 0) {  // the slice tests the position of the sliced query vertex
        const int ps = p.pos[rs.qvertex];
        if (ps == 0) {
          fb[k].slice_mod = rs.mod;
          fb[k].slice_rem = rs.rem;
        } else {
          bl[(size_t)k * kMaxQ + ps].slice_mod = rs.mod;
          bl[(size_t)k * kMaxQ + ps].slice_rem = rs.rem;
        }
      }
      const int u0 = p.order[0];
      fb[k].qlab0 = p.qlab[u0];
      fb[k].qdeg0 = use_deg ? (uint32_t)p.qdeg[u0] : 0;
      fb[k].qne0 = use_ne ? std::min<uint64_t>(p.qne[u0], 0xffffffffull) : 0;
      fb[k].label1 = (p.q > 1) ? p.qlab[p.order[1]] : 0;
      fb[k].single = (p.q == 1) ? 1 : 0;
      // the label class the first frontier scans (empty for a label the graph lacks)
      const int32_t l0 = fb[k].qlab0;
      if (g.lab_vert) {
        const bool has = l0 >= 0 && (size_t)l0 + 1 < g.lab_start.size();
        fb[k].vbegin = has ? g.lab_start[l0] : 0;
        fb[k].vend = has ? g.lab_start[l0 + 1] : 0;
      } else {
        fb[k].vbegin = 0;
        fb[k].vend = l0 == 0 ? g.n : 0;
      }
      max_class = std::max<int64_t>(max_class, fb[k].vend - fb[k].vbegin);
    }
    const size_t b_bl = bl.size() * sizeof(BatchLevel), b_fb = nq * sizeof(FirstBatch);
    const size_t o_fb = (b_bl + 255) & ~size_t(255);
    ws.tables.reserve(o_fb + b_fb, s);
    char *base = ws.tables.as<char>();
    GSM_HIP(hipMemcpyAsync(base, bl.data(), b_bl, hipMemcpyHostToDevice, s));
    GSM_HIP(hipMemcpyAsync(base + o_fb, fb.data(), b_fb, hipMemcpyHostToDevice, s));
    d_bl = reinterpret_cast<BatchLevel *>(base);
    d_fb = reinterpret_cast<FirstBatch *>(base + o_fb);
    ws.counts.reserve((nq + 1) * sizeof(uint64_t), s);
    d_counts = ws.counts.as<uint64_t>();
    launch_zero_u64(d_counts, nq + 1, s);
  }

  void plan_capacity() {
    const uint64_t n = (uint64_t)std::max<int64_t>(g.n, 1);
    uint64_t first = 0;
    for (const Plan &p : plans) {
      const int32_t l = p.qlab[p.order[0]];
      first += (l >= 0 && (size_t)l < g.label_count.size()) ? (uint64_t)g.label_count[l] : 0;
    }
    first = std::max<uint64_t>(first, 1);
    (void)n;
    const uint64_t fixed = first * (4 + 2 + 4 + 8 + 1) + (first + 1) * 8 + 4096;
    if (budget < fixed + 64) throw Error{GSM_E_BUDGET, "memory budget below the first frontiers"};
    const uint64_t rest = budget - fixed;
    const int shares = std::max(1, maxq - 2);
    // buffers kept from earlier calls count against this budget
    uint64_t held = ws.emit.bytes + ws.tables.bytes + ws.counts.bytes + ws.qpairs.bytes + ws.evicted.bytes +
                    ws.cmask.bytes + ws.cmask2.bytes;
    for (int i = 0; i < kMaxQ; ++i)
      held += ws.rows[i].bytes + ws.S[i].bytes + ws.W[i].bytes + ws.apos[i].bytes + ws.abase[i].bytes +
              ws.qid[i].bytes;
    if (held > budget) {
      for (int i = 0; i < kMaxQ; ++i) {
        ws.rows[i].release(s);
        ws.S[i].release(s);
        ws.W[i].release(s);
        ws.apos[i].release(s);
        ws.abase[i].release(s);
        ws.qid[i].release(s);
      }
      ws.emit.release(s);
      ws.cmask.release(s);
      ws.cmask2.release(s);
    }
    for (int i = 0; i < kMaxQ; ++i) cap[i] = 0;
    cap[1] = first;
    for (int i = 2; i < maxq; ++i) {
      cap[i] = rest / shares / (uint64_t)(4 * i + 23);
      if (cap[i] < 1) throw Error{GSM_E_BUDGET, "memory budget below one row of level " + std::to_string(i)};
    }
  }

  void reserve_level(int i, uint64_t rows) {
    ws.rows[i].reserve(rows * 4 * (uint64_t)i, s);
    ws.qid[i].reserve(rows * 2, s);
    ws.W[i].reserve(rows * 4, s);
    ws.apos[i].reserve(rows, s);
    ws.abase[i].reserve(rows * 8, s);
    ws.S[i].reserve((rows + 1) * 8, s);
  }

  void evict_heavy(int i) {
    if (evict_pairs) {
      ws.qpairs.reserve((nq + 1) * sizeof(uint64_t), s);
      ws.evicted.reserve(nq + 1, s);
      h_qpairs.resize(nq + 1);
      if (evicted.size() != (size_t)nq + 1) evicted.assign(nq + 1, 0);
      launch_zero_u64(ws.qpairs.as<uint64_t>(), nq + 1, s);
      launch_query_pairs(ws.W[i].as<uint32_t>(), ws.qid[i].as<uint16_t>(), dcnt + kCntRows + i, cap[i],
                         ws.qpairs.as<uint64_t>(), s);
      GSM_HIP(hipMemcpyAsync(h_qpairs.data(), ws.qpairs.ptr, (nq + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost,
                             s));
      sync();
      bool newly = false;
      for (int k = 0; k < nq; ++k)
        if (!evicted[k] && h_qpairs[k] > evict_pairs) {
          evicted[k] = 1;
          newly = true;
        }
      if (newly) {
        GSM_HIP(hipMemcpyAsync(ws.evicted.ptr, evicted.data(), nq + 1, hipMemcpyHostToDevice, s));
        sync();
        any_evicted = true;
      }
    }
    if (any_evicted)
      launch_retire_evicted(ws.W[i].as<uint32_t>(), ws.qid[i].as<uint16_t>(), dcnt + kCntRows + i, cap[i],
                            ws.evicted.as<uint8_t>(), (uint16_t)nq, s);
  }

  // The levels still to expand, deepest last: depth-first over chunks (a
  // chunk's rows are expanded to the end before the next chunk of the same
  // level overwrites them), breadth-first inside a chunk.
  struct Frame {
    int i;                 // rows of level i (i matched vertices) are in ws.*[i]
    bool counted = false;  // N and P read back
    uint64_t N = 0, P = 0;
    uint64_t b = 0;        // next pair of the level's range to expand
  };
  std::vector<Frame> stack;

  ExpandArgs level_args(int i, uint64_t N) const {
    ExpandArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = dg;
    a.cmask = nullptr;
    a.rows_in = ws.rows[i].as<int32_t>();
    a.apos_in = ws.apos[i].as<uint8_t>();
    a.abase_in = ws.abase[i].as<int64_t>();
    a.S = ws.S[i].as<uint64_t>();
    a.n_rows = N;
    a.L.i = i;
    a.L.q = i + 1;
    a.qid_in = ws.qid[i].as<uint16_t>();
    a.blev = d_bl;
    a.counts = d_counts;
    a.probes = dcnt + kCntProbes;
    a.stage_out_ok = 1;
    a.stage_limit = stage_bytes;
    a.tile_map = ws.tilemap.as<uint64_t>();
    a.tile_map_cap = a.tile_map ? kTileMapWords : 0;
    return a;
  }

  // First frontier of every query; the level-by-level work is then done by step().
  void start() {
    upload_tables();
    launch_zero_u64(dcnt, 64, s);
    reserve_level(1, cap[1]);
    launch_compact_first_batch(dg, d_fb, nq, max_class, ws.rows[1].as<int32_t>(),
                               ws.qid[1].as<uint16_t>(), ws.W[1].as<uint32_t>(), ws.abase[1].as<int64_t>(),
                               ws.apos[1].as<uint8_t>(), dcnt + kCntRows + 1, d_counts, nullptr, s);
    stack.clear();
    if (maxq > 1) stack.push_back(Frame{1});
  }

  // One unit of work: the scan of a level and its read-back, or one chunk's
  // expansion launch.  Returns false once every level is done.
  bool step() {
    if (stack.empty()) return false;
    Frame &f = stack.back();
    const int i = f.i;
    if (!f.counted) {
      evict_heavy(i);
      launch_scan(ws.W[i].as<uint32_t>(), dcnt + kCntRows + i, ws.S[i].as<uint64_t>(), dcnt + kCntPairs + i,
                  ws.scan_scratch.as<uint64_t>(), s);
      fetch_counters();
      f.N = ws.h_counters[kCntRows + i];
      f.P = ws.h_counters[kCntPairs + i];
      f.counted = true;
      level_rows[i] += f.N;
      level_pairs[i] += f.P;
      if (f.P == 0) stack.pop_back();
      return !stack.empty();
    }
    if (f.b >= f.P) {
      stack.pop_back();
      return !stack.empty();
    }
    const bool deepest = (i + 1 >= maxq);  // every query of the batch has maxq vertices
    const uint64_t c = deepest ? f.P : cap[i + 1];
    const uint64_t b = f.b, e = std::min(f.P, b + c);
    f.b = e;
    ExpandArgs a = level_args(i, f.N);
    if (!deepest) {
      reserve_level(i + 1, e - b);
      a.rows_out = ws.rows[i + 1].as<int32_t>();
      a.W_out = ws.W[i + 1].as<uint32_t>();
      a.apos_out = ws.apos[i + 1].as<uint8_t>();
      a.abase_out = ws.abase[i + 1].as<int64_t>();
      a.qid_out = ws.qid[i + 1].as<uint16_t>();
    }
    launch_zero_u64(dcnt + kCntRows + i + 1, 1, s);
    a.counter = dcnt + kCntRows + i + 1;
    a.pair_begin = b;
    a.pair_end = e;
    launch_expand(a, deepest ? kModeBatchLast : kModeBatch, wg, items, s);
    ++launches;
    if (!deepest) stack.push_back(Frame{i + 1});  // invalidates f
    return true;
  }

  // Per-query counts once step() has returned false (waits for the stream).
  void finish(uint64_t *counts) {
    GSM_HIP(hipMemcpyAsync(counts, d_counts, nq * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    sync();
  }

  // ---- device-driven run: every level enqueued at once, its sizes read on
  // the device (no read-back between levels), each level expanded as one
  // chunk at its capacity; optionally captured once in a HIP graph and
  // replayed by later calls that launch the same work.

  // Rows per level the device-driven run provides (level 1: every first
  // frontier row; deeper: what the level's buffers already hold, at least
  // kDeviceMinRows, at most the budget's capacity).  A level whose pairs pass
  // the next one's is flagged; the chunked run that then redoes the group
  // grows the buffers, so a later run of the same work fits.
  static constexpr uint64_t kDeviceMinRows = uint64_t(1) << 20;
  uint64_t dev_cap[kMaxQ] = {0};

  uint64_t held_rows(int i) const {
    uint64_t r = ws.rows[i].bytes / (4 * (uint64_t)i);
    r = std::min<uint64_t>(r, ws.W[i].bytes / 4);
    r = std::min<uint64_t>(r, ws.apos[i].bytes);
    r = std::min<uint64_t>(r, ws.abase[i].bytes / 8);
    r = std::min<uint64_t>(r, ws.S[i].bytes / 8 ? ws.S[i].bytes / 8 - 1 : 0);
    r = std::min<uint64_t>(r, ws.qid[i].bytes / 2);
    return r;
  }

  void enqueue_device(hipStream_t st) {
    uint32_t *overflow = reinterpret_cast<uint32_t *>(dcnt + kCntOverflow);
    launch_zero_u64(dcnt, 64, st);
    if (evict_pairs) launch_zero_u64(ws.evicted.as<uint64_t>(), (nq + 1 + 7) / 8, st);
    launch_compact_first_batch(dg, d_fb, nq, max_class, ws.rows[1].as<int32_t>(), ws.qid[1].as<uint16_t>(),
                               ws.W[1].as<uint32_t>(), ws.abase[1].as<int64_t>(), ws.apos[1].as<uint8_t>(),
                               dcnt + kCntRows + 1, d_counts, nullptr, st);
    for (int i = 1; i < maxq; ++i) {
      if (evict_pairs) {
        // queries whose pairs at this level pass the threshold leave the
        // shared launches (decided on the device, kept once decided)
        launch_zero_u64(ws.qpairs.as<uint64_t>(), nq + 1, st);
        launch_query_pairs(ws.W[i].as<uint32_t>(), ws.qid[i].as<uint16_t>(), dcnt + kCntRows + i, dev_cap[i],
                           ws.qpairs.as<uint64_t>(), st);
        launch_mark_evicted(ws.qpairs.as<uint64_t>(), nq, evict_pairs, ws.evicted.as<uint8_t>(), st);
        launch_retire_evicted(ws.W[i].as<uint32_t>(), ws.qid[i].as<uint16_t>(), dcnt + kCntRows + i, dev_cap[i],
                              ws.evicted.as<uint8_t>(), (uint16_t)nq, st);
      }
      launch_scan(ws.W[i].as<uint32_t>(), dcnt + kCntRows + i, ws.S[i].as<uint64_t>(), dcnt + kCntPairs + i,
                  ws.scan_scratch.as<uint64_t>(), st);
      const bool deepest = (i + 1 >= maxq);
      ExpandArgs a = level_args(i, 0);
      a.dev_n_rows = dcnt + kCntRows + i;
      a.dev_pair_end = dcnt + kCntPairs + i;
      a.overflow = overflow;
      a.pair_begin = 0;
      a.pair_end = deepest ? UINT64_MAX : dev_cap[i + 1];
      if (!deepest) {
        launch_zero_u64(dcnt + kCntRows + i + 1, 1, st);
        a.rows_out = ws.rows[i + 1].as<int32_t>();
        a.W_out = ws.W[i + 1].as<uint32_t>();
        a.apos_out = ws.apos[i + 1].as<uint8_t>();
        a.abase_out = ws.abase[i + 1].as<int64_t>();
        a.qid_out = ws.qid[i + 1].as<uint16_t>();
      }
      a.counter = dcnt + kCntRows + i + 1;
      launch_expand(a, deepest ? kModeBatchLast : kModeBatch, wg, items, st);
      ++launches;
    }
  }

  // What a captured graph of enqueue_device depends on besides the tables
  // uploaded before each launch: every pointer and size its launches take.
  std::string device_key() const {
    std::string k;
    auto put = [&](const void *p, size_t n) { k.append(static_cast<const char *>(p), n); };
    put(&dg, sizeof(dg));
    put(&nq, sizeof(nq));
    put(&maxq, sizeof(maxq));
    put(&max_class, sizeof(max_class));
    put(dev_cap, sizeof(dev_cap));
    put(&wg, sizeof(wg));
    put(&items, sizeof(items));
    put(&evict_pairs, sizeof(evict_pairs));
    put(&stage_bytes, sizeof(stage_bytes));
    const void *ptrs[] = {d_bl, d_fb, d_counts, dcnt, ws.scan_scratch.ptr, ws.qpairs.ptr, ws.evicted.ptr,
                          ws.tilemap.ptr};
    put(ptrs, sizeof(ptrs));
    for (int i = 1; i <= maxq && i < kMaxQ; ++i) {
      const void *lv[] = {ws.rows[i].ptr, ws.W[i].ptr, ws.apos[i].ptr, ws.abase[i].ptr, ws.S[i].ptr, ws.qid[i].ptr};
      put(lv, sizeof(lv));
    }
    return k;
  }

  // Runs the group device-driven; false when some level's pairs passed its
  // capacity (the counts are then not valid: redo with start/step/finish).
  bool run_device(uint64_t *counts, bool use_graph) {
    upload_tables();
    dev_cap[1] = cap[1];
    for (int i = 2; i < maxq; ++i) dev_cap[i] = std::min(cap[i], std::max(held_rows(i), kDeviceMinRows));
    for (int i = 1; i < maxq; ++i) reserve_level(i, dev_cap[i]);
    if (evict_pairs) {
      ws.qpairs.reserve((nq + 1) * sizeof(uint64_t), s);
      ws.evicted.reserve(((nq + 1 + 7) / 8) * 8, s);
      if (evicted.size() != (size_t)nq + 1) evicted.assign(nq + 1, 0);
    }
    if (use_graph) {
      const std::string key = device_key();
      auto hit = std::find_if(ws.graphs.begin(), ws.graphs.end(),
                              [&](const std::pair<std::string, hipGraphExec_t> &e) { return e.first == key; });
      hipGraphExec_t exec = nullptr;
      if (hit != ws.graphs.end()) {
        exec = hit->second;
        std::rotate(hit, hit + 1, ws.graphs.end());  // most recent last
        launches += maxq - 1;
      } else {
        if (!ws.capture_stream) GSM_HIP(hipStreamCreateWithFlags(&ws.capture_stream, hipStreamNonBlocking));
        GSM_HIP(hipStreamBeginCapture(ws.capture_stream, hipStreamCaptureModeThreadLocal));
        hipGraph_t graph = nullptr;
        try {
          enqueue_device(ws.capture_stream);
        } catch (...) {
          (void)hipStreamEndCapture(ws.capture_stream, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          throw;
        }
        GSM_HIP(hipStreamEndCapture(ws.capture_stream, &graph));
        const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) throw Error{GSM_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
        if (ws.graphs.size() >= Workspace::kMaxGraphs) {
          (void)hipGraphExecDestroy(ws.graphs.front().second);
          ws.graphs.erase(ws.graphs.begin());
        }
        ws.graphs.emplace_back(key, exec);
      }
      GSM_HIP(hipGraphLaunch(exec, s));
    } else {
      enqueue_device(s);
    }
    GSM_HIP(hipMemcpyAsync(ws.h_counters, dcnt, 64 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    GSM_HIP(hipMemcpyAsync(counts, d_counts, nq * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    if (evict_pairs) GSM_HIP(hipMemcpyAsync(evicted.data(), ws.evicted.ptr, nq + 1, hipMemcpyDeviceToHost, s));
    sync();
    if (ws.h_counters[kCntOverflow] & 0xffffffffull) return false;
    for (int i = 1; i < maxq; ++i) {
      level_rows[i] += ws.h_counters[kCntRows + i];
      level_pairs[i] += ws.h_counters[kCntPairs + i];
    }
    return true;
  }

  // First-level (row, neighbour) pairs of every query, from the first-frontier
  // kernel in estimate mode (nothing is written but the totals).
  std::vector<uint64_t> first_level_pairs() {
    upload_tables();
    launch_zero_u64(d_counts, std::max(nq, 1), s);
    launch_compact_first_batch(dg, d_fb, nq, max_class, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                               nullptr, d_counts, s);
    std::vector<uint64_t> out(nq);
    GSM_HIP(hipMemcpyAsync(out.data(), d_counts, nq * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    sync();
    return out;
  }

  void run(uint64_t *counts) {
    start();
    while (step()) {
    }
    finish(counts);
  }
};

}  // namespace

struct BatchRun::Impl {
  BatchMatcher m;
  Impl(gsm_graph &g, const gsm_query *const *qs, int nq, Workspace &ws, hipStream_t s, const RootSlice *sl)
      : m(g, qs, nq, ws, s, sl) {}
};

BatchRun::BatchRun(gsm_graph &g, const gsm_query *const *qs, int nq, const gsm_match_opts &o, Workspace &ws,
                   const RootSlice *slices, uint64_t evict_pairs)
    : impl(new Impl(g, qs, nq, ws, (hipStream_t)o.hip_stream, slices)) {
  BatchMatcher &m = impl->m;
  m.rounds = o.filter_rounds;
  m.use_deg = o.use_degree;
  m.use_ne = o.use_ne;
  m.wg = o.wg_size ? o.wg_size : 512;
  m.items = o.tile_items ? o.tile_items : 4;
  m.budget = o.memory_budget_bytes ? o.memory_budget_bytes : (uint64_t(4) << 30);
  if (o.struct_size >= offsetof(gsm_match_opts, stage_bytes) + sizeof(uint32_t)) m.stage_bytes = o.stage_bytes;
  m.evict_pairs = evict_pairs;
  m.plan_capacity();
  m.start();
}

BatchRun::~BatchRun() = default;

bool BatchRun::step() { return impl->m.step(); }

void BatchRun::finish(uint64_t *counts, std::vector<uint8_t> &evicted) {
  impl->m.finish(counts);
  evicted.assign(impl->m.nq, 0);
  for (int k = 0; k < impl->m.nq && k < (int)impl->m.evicted.size(); ++k) evicted[k] = impl->m.evicted[k];
}

void match_batch_on(gsm_graph &g, const gsm_query *const *qs, int nq, const gsm_match_opts &o,
                    Workspace &ws, uint64_t *counts, uint64_t *launches_out, gsm_stats *st,
                    const RootSlice *slices) {
    auto slice_of = [&](int k) { return slices ? slices[k] : RootSlice{}; };
    const hipStream_t stream = (hipStream_t)o.hip_stream;
    const uint32_t flags = o.struct_size >= offsetof(gsm_match_opts, flags) + sizeof(uint32_t) ? o.flags : 0u;
    auto configure = [&](BatchMatcher &m) {
      m.rounds = o.filter_rounds;
      m.use_deg = o.use_degree;
      m.use_ne = o.use_ne;
      m.wg = o.wg_size ? o.wg_size : 512;
      m.items = o.tile_items ? o.tile_items : 4;
      m.budget = o.memory_budget_bytes ? o.memory_budget_bytes : (uint64_t(4) << 30);
      if (o.struct_size >= offsetof(gsm_match_opts, stage_bytes) + sizeof(uint32_t)) m.stage_bytes = o.stage_bytes;
    };
    const uint64_t heavy_pairs_opt = o.batch_heavy_pairs ? o.batch_heavy_pairs : (uint64_t(1) << 18);
    // split: heavy queries on launches of their own, the rest shared
    const uint64_t heavy_pairs = o.batch_heavy_pairs ? o.batch_heavy_pairs : (uint64_t(1) << 18);
    std::vector<int> light;
    std::vector<int> heavy;
    if (heavy_pairs == UINT64_MAX) {  // every query shares launches: nothing to estimate
      for (int k = 0; k < nq; ++k) light.push_back(k);
    } else {
      BatchMatcher est(g, qs, nq, ws, stream, slices);
      configure(est);
      const std::vector<uint64_t> p1 = est.first_level_pairs();
      for (int k = 0; k < nq; ++k) (qs[k]->q > 1 && p1[k] > heavy_pairs ? heavy : light).push_back(k);
    }
    uint64_t launches = 0;
    for (int k : heavy) counts[k] = match_count_one(g, *qs[k], o, ws, slice_of(k));
    // the shared launches group queries of one size, so every level of a group
    // either writes the next frontier for all its rows or counts all of them
    for (int qsize = 1; qsize <= kMaxQ; ++qsize) {
      std::vector<int> grp;
      for (int k : light)
        if (qs[k]->q == qsize) grp.push_back(k);
      if (grp.empty()) continue;
      std::vector<const gsm_query *> sub;
      std::vector<RootSlice> sub_sl;
      for (int k : grp) {
        sub.push_back(qs[k]);
        sub_sl.push_back(slice_of(k));
      }
      std::vector<uint64_t> c(grp.size());
      BatchMatcher m(g, sub.data(), (int)sub.size(), ws, stream, sub_sl.data());
      configure(m);
      m.evict_pairs = heavy_pairs_opt == UINT64_MAX ? 0 : heavy_pairs_opt;
      m.plan_capacity();
      const bool device_ok = !(flags & GSM_MATCH_HOST_LEVELS);
      if (!device_ok || !m.run_device(c.data(), !(flags & GSM_MATCH_NO_GRAPH))) {
        // a level did not fit its capacity in one chunk: level by level,
        // chunked, sizes read back
        BatchMatcher again(g, sub.data(), (int)sub.size(), ws, stream, sub_sl.data());
        configure(again);
        again.evict_pairs = m.evict_pairs;
        again.plan_capacity();
        again.run(c.data());
        again.launches += m.launches;
        std::swap(m.evicted, again.evicted);
        for (int i = 0; i < kMaxQ; ++i) {
          m.level_pairs[i] = again.level_pairs[i];
          m.level_rows[i] = again.level_rows[i];
        }
        m.launches = again.launches;
      }
      launches += m.launches;
      if (st)
        for (int i = 0; i < kMaxQ; ++i) {
          st->pairs[i] += m.level_pairs[i];
          if (i > 0) st->rows[i - 1] += m.level_rows[i];
        }
      for (size_t j = 0; j < grp.size(); ++j)
        counts[grp[j]] = (j < m.evicted.size() && m.evicted[j])
                             ? match_count_one(g, *qs[grp[j]], o, ws, slice_of(grp[j]))
                             : c[j];
    }
    if (launches_out) *launches_out = launches;
}

}  // namespace gsm

using gsm::Error;

extern "C" gsm_status gsm_match_batch(gsm_graph_t g, int32_t nq, const gsm_query_t *qs,
                                      const gsm_match_opts *opts, uint64_t *counts) {
  try {
    if (!g || nq < 0 || (nq > 0 && (!qs || !counts))) {
      gsm::set_error("gsm_match_batch: invalid arguments");
      return GSM_E_INVALID_ARG;
    }
    if (nq > 65535) {
      gsm::set_error("gsm_match_batch: at most 65535 queries per batch");
      return GSM_E_INVALID_ARG;
    }
    for (int k = 0; k < nq; ++k) {
      if (!qs[k]) {
        gsm::set_error("gsm_match_batch: NULL query");
        return GSM_E_INVALID_ARG;
      }
      if (qs[k]->has_elab) {
        gsm::set_error("gsm_match_batch: edge-labelled queries are matched one at a time (gsm_match)");
        return GSM_E_UNSUPPORTED;
      }
    }
    if (nq == 0) return GSM_OK;
    gsm_match_opts d;
    gsm_match_opts_init(&d);
    const gsm_match_opts &o = opts ? *opts : d;
    if (o.struct_size >= offsetof(gsm_match_opts, flags) + sizeof(uint32_t) &&
        (o.flags & (GSM_MATCH_UNIQUE | GSM_MATCH_LOOKAHEAD | GSM_MATCH_SORT_ROWS | GSM_MATCH_INDUCED |
                    GSM_MATCH_PACK_FRONTIER | GSM_MATCH_LOOKAHEAD2))) {
      gsm::set_error("gsm_match_batch: unique, induced, look-ahead, sorted and packed modes are single-query "
                     "options");
      return GSM_E_UNSUPPORTED;
    }
    if (o.rows_on_device || o.emit) {
      gsm::set_error("gsm_match_batch counts only: no rows or emit callback");
      return GSM_E_UNSUPPORTED;
    }
    std::vector<gsm::RootSlice> slices;
    if (o.root_qvertex >= 0) {
      if (o.root_mod == 0 || o.root_rem >= o.root_mod) {
        gsm::set_error("gsm_match_batch: root slice needs root_rem < root_mod");
        return GSM_E_INVALID_ARG;
      }
      for (int k = 0; k < nq; ++k)
        if (o.root_qvertex >= qs[k]->q) {
          gsm::set_error("gsm_match_batch: root_qvertex >= q of query " + std::to_string(k));
          return GSM_E_INVALID_ARG;
        }
      slices.assign(nq, gsm::RootSlice{o.root_qvertex, o.root_mod, o.root_rem});
    }
    if (o.filter_rounds < 0 || o.filter_rounds > 64) throw Error{GSM_E_INVALID_ARG, "filter_rounds out of [0, 64]"};
    if (o.struct_size >= offsetof(gsm_match_opts, stage_bytes) + sizeof(uint32_t) &&
        o.stage_bytes > gsm::kExpandStageMax)
      throw Error{GSM_E_INVALID_ARG, "stage_bytes above 64 KiB"};
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->ws) g->ws = new gsm::Workspace();
    uint64_t launches = 0;
    gsm_stats st;
    std::memset(&st, 0, sizeof(st));
    gsm::match_batch_on(*g, qs, nq, o, *g->ws, counts, &launches, &st, slices.empty() ? nullptr : slices.data());
    if (o.stats) {
      st.expand_launches = launches;
      const uint32_t sz = std::min<uint32_t>(o.stats->struct_size ? o.stats->struct_size : sizeof(gsm_stats),
                                             sizeof(gsm_stats));
      std::memcpy(o.stats, &st, sz);
      o.stats->struct_size = sz;
    }
    return GSM_OK;
  } catch (const Error &e) {
    gsm::set_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc &) {
    gsm::set_error("host allocation failed");
    return GSM_E_OOM;
  }
}
