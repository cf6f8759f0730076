// Single-query driver: filter, first frontier, then level-by-level expansion
// cut into memory-bounded chunks (depth-first over chunks, breadth-first
// inside a chunk), as in the verification loop of the paper's Alg. 1.
#include <algorithm>
#include <chrono>
#include <exception>
#include <cstddef>
#include <cstring>

#include "gsm_internal.h"

namespace gsm {

namespace {

// counters[] slots in the workspace
constexpr int kCntRows = 0;     // [1..15]: rows written at level i
constexpr int kCntPairs = 16;   // [16+i]: scan total of level i
constexpr int kCntResult = 32;  // embeddings counted at the last level
constexpr int kCntProbes = 33;  // binary-search steps

struct Options {
  uint64_t budget = uint64_t(4) << 30;
  int rounds = 1, use_deg = 1, use_ne = 1;
  bool rows_dev = false;
  hipStream_t stream = nullptr;
  int root_q = -1;
  uint32_t root_mod = 0, root_rem = 0;
  gsm_emit_fn emit = nullptr;
  void *emit_ctx = nullptr;
  gsm_stats *stats = nullptr;
  int items = 4, wg = 512;
  bool profile = false;
  int stage_out = 1;
  bool sort = false;
  bool lookahead = false;
  bool lookahead2 = false;
  bool unique = false;
  bool induced = false;
  bool pack = false;
  uint32_t stage_bytes = kExpandStageBytes;
};

Options read_opts(const gsm_match_opts *o, int q) {
  Options r;
  if (!o) return r;
  if (o->struct_size < sizeof(uint32_t)) throw Error{GSM_E_INVALID_ARG, "opts.struct_size not set"};
  if (o->memory_budget_bytes) r.budget = o->memory_budget_bytes;
  r.rounds = o->filter_rounds;
  r.use_deg = o->use_degree;
  r.use_ne = o->use_ne;
  r.rows_dev = o->rows_on_device != 0;
  r.stream = (hipStream_t)o->hip_stream;
  r.root_q = o->root_qvertex;
  r.root_mod = o->root_mod;
  r.root_rem = o->root_rem;
  r.emit = o->emit;
  r.emit_ctx = o->emit_ctx;
  r.stats = o->stats;
  if (o->tile_items) r.items = o->tile_items;
  if (o->wg_size) r.wg = o->wg_size;
  r.profile = o->profile != 0;
  if (o->struct_size >= offsetof(gsm_match_opts, flags) + sizeof(uint32_t)) {
    r.stage_out = (o->flags & GSM_MATCH_NO_OUTPUT_STAGING) ? 0 : 1;
    r.sort = (o->flags & GSM_MATCH_SORT_ROWS) != 0;
    r.lookahead2 = (o->flags & GSM_MATCH_LOOKAHEAD2) != 0;
    r.lookahead = r.lookahead2 || (o->flags & GSM_MATCH_LOOKAHEAD) != 0;
    r.unique = (o->flags & GSM_MATCH_UNIQUE) != 0;
    r.induced = (o->flags & GSM_MATCH_INDUCED) != 0;
    r.pack = (o->flags & GSM_MATCH_PACK_FRONTIER) != 0;
  }
  if (o->struct_size >= offsetof(gsm_match_opts, stage_bytes) + sizeof(uint32_t) && o->stage_bytes) {
    if (o->stage_bytes > kExpandStageMax) throw Error{GSM_E_INVALID_ARG, "stage_bytes above 64 KiB"};
    r.stage_bytes = o->stage_bytes;
  }
  if (r.rounds < 0 || r.rounds > 64) throw Error{GSM_E_INVALID_ARG, "filter_rounds out of [0, 64]"};
  if (r.root_q >= q) throw Error{GSM_E_INVALID_ARG, "root_qvertex >= q"};
  if (r.root_q >= 0 && r.root_mod == 0) throw Error{GSM_E_INVALID_ARG, "root_mod must be > 0"};
  if (r.root_q >= 0 && r.root_rem >= r.root_mod) throw Error{GSM_E_INVALID_ARG, "root_rem >= root_mod"};
  if (r.items != 1 && r.items != 2 && r.items != 4 && r.items != 8)
    throw Error{GSM_E_INVALID_ARG, "tile_items must be 1, 2, 4 or 8"};
  if (r.wg != 128 && r.wg != 256 && r.wg != 512)
    throw Error{GSM_E_INVALID_ARG, "wg_size must be 128, 256 or 512"};
  return r;
}

// Device bytes that do not depend on the budget: two candidate masks, the
// first frontier (at most n rows with range data) and its scan.
uint64_t fixed_bytes(int64_t nv) {
  const uint64_t n = (uint64_t)std::max<int64_t>(nv, 1);
  return 2 * n * 2 + n * (4 + 4 + 8 + 1) + (n + 1) * 8 + 4096;
}

// Smallest budget for which every level (and the staging buffer) gets a row.
uint64_t min_budget_bytes(int64_t nv, int q, bool host_rows) {
  const int shares = std::max(0, q - 2) + (host_rows ? 1 : 0);
  uint64_t per = 0;
  for (int i = 2; i < q; ++i) per = std::max<uint64_t>(per, 4 * (uint64_t)i + 21);
  if (host_rows) per = std::max<uint64_t>(per, 4 * (uint64_t)q);
  return fixed_bytes(nv) + 64 + (uint64_t)shares * per;
}

struct Matcher {
  gsm_graph &g;
  const gsm_query &qh;
  Plan p;
  Options o;
  Workspace &ws;
  hipStream_t s;
  DeviceGraph dg;
  uint64_t cap[kMaxQ];  // max rows per level buffer
  uint64_t *dcnt;       // device counters
  int pack_bits = 0;          // bits per packed id (bit width of n - 1)
  bool packed[kMaxQ] = {};    // rows of level i are packed
  // output
  int32_t *rows_user = nullptr;
  uint64_t rows_cap = 0;
  bool emit_host = false;  // rows pass through the staging buffer to the host
  uint64_t staged_cap = 0;
  uint64_t host_rows_done = 0;
  bool cancelled = false;
  std::vector<int32_t> host_stage;
  gsm_stats st;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pairs;
  size_t ev_next = 0;

  Matcher(gsm_graph &g_, const gsm_query &q_, const Options &o_, Workspace &ws_)
      : g(g_), qh(q_), o(o_), ws(ws_), s(o_.stream) {
    p = make_plan(g, qh);
    dg = device_graph(g);
    dcnt = ws.counters.as<uint64_t>();
    std::memset(&st, 0, sizeof(st));
    st.struct_size = sizeof(st);
    st.q = p.q;
    if (o.pack) {
      pack_bits = 1;
      while (pack_bits < 31 && (int64_t(1) << pack_bits) < g.n) ++pack_bits;
      // level i is packed when that saves bytes and its consumer can stage
      // its rows in LDS (the decoder runs there)
      for (int i = 2; i < p.q; ++i)
        packed[i] = (i * pack_bits + 31) / 32 < i && (uint64_t)o.wg * o.items * i * 4 <= o.stage_bytes;
    }
  }

  // bytes of one row of level i in its buffer
  uint64_t row_bytes(int i) const {
    return 4 * (uint64_t)(packed[i] ? (i * pack_bits + 31) / 32 : i);
  }

  // A call that fails part-way may have launches in flight on the stream;
  // they must finish before the next call reuses the workspace buffers.
  ~Matcher() {
    if (std::uncaught_exceptions() > 0) (void)hipStreamSynchronize(s);
  }

  QueryArgs query_args() const {
    QueryArgs qa;
    std::memset(&qa, 0, sizeof(qa));
    qa.q = p.q;
    qa.root_bit = o.root_q;
    qa.root_mod = o.root_mod ? o.root_mod : 1;
    qa.root_rem = o.root_rem;
    qa.use_deg = o.use_deg;
    qa.use_ne = o.use_ne;
    for (int u = 0; u < p.q; ++u) {
      qa.qlab[u] = p.qlab[u];
      qa.qdeg[u] = (uint32_t)p.qdeg[u];
      qa.qne[u] = p.qne[u];
    }
    return qa;
  }

  // Filter into ws.cmask (query-id bits).
  void filter() {
    ws.cmask.reserve(std::max<int64_t>(g.n, 1) * sizeof(uint16_t), s);
    const QueryArgs qa = query_args();
    launch_filter_init(dg, qa, ws.cmask.as<uint16_t>(), s);
    st.filter_bytes += (uint64_t)g.n * (4 + 4 + (g.ne0 ? 8 : 0) + 2);
    if (o.rounds > 0) ws.cmask2.reserve(std::max<int64_t>(g.n, 1) * sizeof(uint16_t), s);
    for (int r = 0; r < o.rounds; ++r) {
      launch_filter_refine(dg, g.heavy, g.nheavy, qa, ws.cmask.as<uint16_t>(),
                           ws.cmask2.as<uint16_t>(), s);
      std::swap(ws.cmask.ptr, ws.cmask2.ptr);
      std::swap(ws.cmask.bytes, ws.cmask2.bytes);
      std::swap(ws.cmask.pooled, ws.cmask2.pooled);
      st.filter_bytes += (uint64_t)(g.n + 1) * 8 + (uint64_t)g.nnz * (4 + 2 + (g.lab ? 4 : 0)) +
                         (uint64_t)g.n * 4;
    }
  }

  void sync() { GSM_HIP(hipStreamSynchronize(s)); }

  void fetch_counters() {
    GSM_HIP(hipMemcpyAsync(ws.h_counters, dcnt, 64 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    sync();
  }

  void zero_counter(int slot) { launch_zero_u64(dcnt + slot, 1, s); }

  std::pair<hipEvent_t, hipEvent_t> next_events() {
    while (ws.events.size() < 2 * (ev_next + 1)) {
      hipEvent_t e;
      GSM_HIP(hipEventCreate(&e));
      ws.events.push_back(e);
    }
    auto pr = std::make_pair(ws.events[2 * ev_next], ws.events[2 * ev_next + 1]);
    ++ev_next;
    return pr;
  }

  void expand(ExpandArgs &a, int mode) {
    a.probes = dcnt + kCntProbes;
    a.stage_out_ok = o.stage_out;
    a.stage_limit = o.stage_bytes;
    if (!ws.fixed_base) {  // (the no-allocation scratch has no room for the tile map)
      ws.tilemap.reserve(kTileMapWords * sizeof(uint64_t), s);
      a.tile_map = ws.tilemap.as<uint64_t>();
      a.tile_map_cap = kTileMapWords;
    }
    if (o.profile) {
      auto pr = next_events();
      GSM_HIP(hipEventRecord(pr.first, s));
      launch_expand(a, mode, o.wg, o.items, s);
      GSM_HIP(hipEventRecord(pr.second, s));
      ev_pairs.push_back(pr);
    } else {
      launch_expand(a, mode, o.wg, o.items, s);
    }
    st.expand_launches++;
  }

  // Level capacities from the budget.  Fixed: two cmask arrays, the first
  // frontier (<= n rows), counters.  The rest is split evenly over levels
  // 2..q-1 plus the host staging buffer when rows go to the host.
  void plan_capacity() {
    const uint64_t n = (uint64_t)std::max<int64_t>(g.n, 1);
    const uint64_t fixed = fixed_bytes(g.n);
    if (o.budget < fixed + 64) throw Error{GSM_E_BUDGET, "memory budget below the first frontier"};
    const uint64_t rest = o.budget - fixed;
    const int shares = std::max(0, p.q - 2) + (emit_host ? 1 : 0);
    for (int i = 0; i < kMaxQ; ++i) cap[i] = 0;
    cap[1] = n;
    for (int i = 2; i < p.q; ++i) {
      cap[i] = rest / shares / (row_bytes(i) + 21);
      if (cap[i] < 1) throw Error{GSM_E_BUDGET, "memory budget below one row of level " + std::to_string(i)};
    }
    if (emit_host) {
      // pairs per output chunk (a chunk's rows fit the staging buffer); a
      // device-side sink takes chunks of up to 2^30 pairs (fewer launches and
      // hand-overs), a host-side one 2^26 (its host copy stays small)
      const uint64_t chunk_max = (o.emit && o.rows_dev) ? uint64_t(1) << 30 : uint64_t(1) << 26;
      staged_cap = std::min<uint64_t>(rest / shares / (uint64_t)(4 * p.q), chunk_max);
      if (staged_cap < 1) throw Error{GSM_E_BUDGET, "memory budget below one output row"};
    }
    if (ws.fixed_base) {
      carve_fixed();
      return;
    }
    // Buffers are kept across calls (reallocation costs milliseconds); when
    // what earlier calls left behind exceeds this call's budget, start over.
    // (buffers a batched call left in the same workspace count too)
    uint64_t held = ws.cmask.bytes + ws.cmask2.bytes + ws.emit.bytes + ws.tables.bytes + ws.counts.bytes +
                    ws.qpairs.bytes + ws.evicted.bytes;
    for (int i = 0; i < kMaxQ; ++i)
      held += ws.rows[i].bytes + ws.S[i].bytes + ws.W[i].bytes + ws.apos[i].bytes + ws.abase[i].bytes +
              ws.qid[i].bytes;
    if (held > o.budget) {
      for (int i = 2; i < kMaxQ; ++i) {
        ws.rows[i].release(s);
        ws.S[i].release(s);
        ws.W[i].release(s);
        ws.apos[i].release(s);
        ws.abase[i].release(s);
      }
      for (int i = 0; i < kMaxQ; ++i) ws.qid[i].release(s);
      ws.emit.release(s);
      ws.qpairs.release(s);
      ws.evicted.release(s);
    }
  }

  // A fixed workspace: lay every buffer of this call out in the window after
  // the counters, at the capacities plan_capacity chose.
  void carve_fixed() {
    char *base = ws.fixed_base + Workspace::fixed_header_bytes();
    const char *end = ws.fixed_base + ws.fixed_bytes;
    auto take = [&](DevBuf &b, uint64_t want) {
      const uint64_t sz = (std::max<uint64_t>(want, 1) + 255) & ~uint64_t(255);
      if (sz > (uint64_t)(end - base))
        throw Error{GSM_E_BUDGET, "no-allocation scratch of " + std::to_string(ws.fixed_bytes) +
                                      " bytes too small for this graph and query"};
      b.set_fixed(base, sz);
      base += sz;
    };
    const uint64_t n = (uint64_t)std::max<int64_t>(g.n, 1);
    take(ws.cmask, n * 2);
    take(ws.cmask2, n * 2);
    for (int i = 1; i < p.q; ++i) {
      const uint64_t c = cap[i];
      take(ws.rows[i], c * row_bytes(i));
      take(ws.W[i], c * 4);
      take(ws.apos[i], c);
      take(ws.abase[i], c * 8);
      take(ws.S[i], (c + 1) * 8);
    }
    if (emit_host) take(ws.emit, p.q == 1 ? n * 4 : staged_cap * (uint64_t)p.q * 4);
  }

  void reserve_level(int i, uint64_t rows) {
    ws.rows[i].reserve(rows * row_bytes(i), s);
    ws.W[i].reserve(rows * 4, s);
    ws.apos[i].reserve(rows, s);
    ws.abase[i].reserve(rows * 8, s);
    ws.S[i].reserve((rows + 1) * 8, s);
  }

  // The last position's candidate test can only prune: its label is given
  // by the label-grouped gather (or the graph has none), every edge to it
  // and injectivity are checked explicitly, and the filter keeps every
  // vertex of an embedding.  It is kept where it carries the root slice.
  bool skips_mask(int i) const {
    const int u = p.order[i];
    return i + 1 == p.q && o.root_q != u && (g.loff || (!g.lab && p.qlab[u] == 0));
  }

  LevelArgs level_args(int i) const {
    LevelArgs L;
    std::memset(&L, 0, sizeof(L));
    L.i = i;
    L.q = p.q;
    L.nbr_mask = p.backmask[i];
    L.qbit = (uint32_t)p.order[i];
    L.next_nbr_mask = (i + 1 < p.q) ? p.backmask[i + 1] : 0;
    L.next_label = (i + 1 < p.q) ? p.qlab[p.order[i + 1]] : 0;
    for (int j = 0; j < p.q; ++j) {
      L.out_col[j] = p.order[j];
      L.in_pos[p.order[j]] = j;
    }
    L.no_cmask = skips_mask(i) ? 1 : 0;
    if (o.induced) L.non_mask = ((1u << i) - 1u) & ~p.backmask[i];
    if (qh.has_elab) {
      L.use_elab = 1;
      for (int j = 0; j < i; ++j)
        if ((p.backmask[i] >> j) & 1) L.elab_req[j] = qh.elab[p.order[i]][p.order[j]];
    }
    if (o.unique) {
      // symmetry-breaking constraints whose later vertex is placed at position i
      for (size_t k = 0; k + 1 < qh.sym_pairs.size(); k += 2) {
        const int pa = p.pos[qh.sym_pairs[k]], pb = p.pos[qh.sym_pairs[k + 1]];
        if (pb == i && pa < i) L.sym_lt |= 1u << pa;  // f(a) < f(b) = w
        if (pa == i && pb < i) L.sym_gt |= 1u << pb;  // w = f(a) < f(b)
        if (pb == i + 1 && pa <= i) L.next_sym_lt |= 1u << pa;
        if (pa == i + 1 && pb <= i) L.next_sym_gt |= 1u << pb;
      }
    }
    if (o.lookahead) {
      // later query neighbours of the vertex placed at position i
      const int u = p.order[i];
      for (int k = i + 1; k < p.q; ++k) {
        if (!((p.backmask[k] >> i) & 1)) continue;
        const int32_t lab = p.qlab[p.order[k]];
        uint32_t need = 0;  // neighbours of u with that label, matched or not
        for (int v = 0; v < qh.q; ++v)
          if (((qh.adj[u] >> v) & 1) && p.qlab[v] == lab) ++need;
        L.la_label[L.la_n] = lab;
        L.la_qbit[L.la_n] = (uint32_t)p.order[k];
        L.la_need[L.la_n] = need;
        if (o.lookahead2 && g.loff) {
          // neighbours per label of the later query vertex, largest first
          const int uk = p.order[k];
          std::vector<std::pair<uint32_t, int32_t>> by_label;
          for (int v = 0; v < qh.q; ++v) {
            if (!((qh.adj[uk] >> v) & 1)) continue;
            auto it = std::find_if(by_label.begin(), by_label.end(),
                                   [&](const std::pair<uint32_t, int32_t> &e) { return e.second == p.qlab[v]; });
            if (it == by_label.end())
              by_label.push_back({1u, p.qlab[v]});
            else
              ++it->first;
          }
          std::stable_sort(by_label.begin(), by_label.end(),
                           [](const std::pair<uint32_t, int32_t> &x, const std::pair<uint32_t, int32_t> &y) {
                             return x.first > y.first;
                           });
          const int nl = std::min<int>((int)by_label.size(), kLa2Labels);
          L.la2_n[L.la_n] = (uint8_t)nl;
          for (int t = 0; t < nl; ++t) {
            L.la2_label[L.la_n][t] = by_label[t].second;
            L.la2_need[L.la_n][t] = by_label[t].first;
          }
          L.la2 = 1;
        }
        ++L.la_n;
      }
    }
    return L;
  }

  // Hands staged rows [0, nrows) to the sink.
  void drain_stage(uint64_t nrows) {
    if (nrows == 0) return;
    if (o.emit && o.rows_dev) {  // device sink: the callback reads device memory
      sync();
      if (o.emit(o.emit_ctx, ws.emit.as<int32_t>(), nrows, p.q) != 0) cancelled = true;
    } else if (o.emit) {
      host_stage.resize(nrows * (uint64_t)p.q);
      GSM_HIP(hipMemcpyAsync(host_stage.data(), ws.emit.ptr, nrows * p.q * sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
      sync();
      if (o.emit(o.emit_ctx, host_stage.data(), nrows, p.q) != 0) cancelled = true;
    } else if (rows_user && host_rows_done < rows_cap) {
      const uint64_t take = std::min(nrows, rows_cap - host_rows_done);
      GSM_HIP(hipMemcpyAsync(rows_user + host_rows_done * p.q, ws.emit.ptr, take * p.q * sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
      sync();
    }
    host_rows_done += nrows;
  }

  // The levels still to expand, deepest last: depth-first over chunks (a
  // chunk's rows are expanded to the end before the next chunk of the same
  // level overwrites them), breadth-first inside a chunk.  Rows of level i
  // (i matched vertices) are in ws.*[i], their number in dcnt[kCntRows + i].
  struct Frame {
    int i;
    bool counted = false;  // N and P read back
    uint64_t N = 0, P = 0;
    uint64_t b = 0;        // next pair of the level's range to expand
  };
  std::vector<Frame> stack;
  uint64_t single_count = 0;  // q == 1: the candidates, counted in start()

  ExpandArgs level_expand_args(int i, uint64_t N) const {
    ExpandArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = dg;
    a.cmask = ws.cmask.as<uint16_t>();
    a.rows_in = ws.rows[i].as<int32_t>();
    a.apos_in = ws.apos[i].as<uint8_t>();
    a.abase_in = ws.abase[i].as<int64_t>();
    a.S = ws.S[i].as<uint64_t>();
    a.n_rows = N;
    a.L = level_args(i);
    a.pack_bits = pack_bits;
    a.pack_in = packed[i] ? 1 : 0;
    a.pack_out = (i + 1 < p.q && packed[i + 1]) ? 1 : 0;
    return a;
  }

  // The last level, all of it: count, rows straight to the caller's device
  // buffer, or chunks through the staging buffer to the host.
  void last_level(int i, uint64_t N, uint64_t P) {
    ExpandArgs a = level_expand_args(i, N);
    a.level_pairs = P;
    a.counter = dcnt + kCntResult;
    if (!rows_user && !o.emit) {  // count only, in launches of at most kTileMapWords tiles
      const uint64_t tile = (uint64_t)(o.wg ? o.wg : 512) * (uint64_t)(o.items ? o.items : 4);
      const uint64_t span = kTileMapWords * tile;
      for (uint64_t b = 0; b < P; b += span) {
        a.pair_begin = b;
        a.pair_end = std::min(P, b + span);
        expand(a, kModeCount);
        st.chunks[i]++;
      }
    } else if (!emit_host) {  // rows straight into the caller's device buffer
      a.pair_begin = 0;
      a.pair_end = P;
      a.emit_rows = rows_user;
      a.emit_base = 0;
      a.emit_cap = rows_cap;
      expand(a, kModeEmit);
      st.chunks[i]++;
    } else {  // through the staging buffer, one chunk at a time
      ws.emit.reserve(std::min(staged_cap, P) * p.q * sizeof(int32_t), s);
      for (uint64_t b = 0; b < P && !cancelled; b += staged_cap) {
        const uint64_t e = std::min(P, b + staged_cap);
        a.pair_begin = b;
        a.pair_end = e;
        a.emit_rows = ws.emit.as<int32_t>();
        a.emit_base = host_rows_done;
        a.emit_cap = staged_cap;
        expand(a, kModeEmit);
        st.chunks[i]++;
        fetch_counters();
        drain_stage(ws.h_counters[kCntResult] - host_rows_done);
      }
    }
  }

  // One unit of work: a level's scan and read-back, one chunk's expansion
  // to the next level, or the whole last level.  Returns false when done.
  bool step() {
    if (stack.empty() || cancelled) return false;
    Frame &f = stack.back();
    const int i = f.i;
    if (!f.counted) {
      launch_scan(ws.W[i].as<uint32_t>(), dcnt + kCntRows + i, ws.S[i].as<uint64_t>(),
                  dcnt + kCntPairs + i, ws.scan_scratch.as<uint64_t>(), s);
      fetch_counters();
      f.N = ws.h_counters[kCntRows + i];
      f.P = ws.h_counters[kCntPairs + i];
      f.counted = true;
      st.rows[i - 1] += f.N;
      st.pairs[i] += f.P;
      if (f.P == 0) stack.pop_back();
      return !stack.empty();
    }
    if (i == p.q - 1) {
      last_level(i, f.N, f.P);
      stack.pop_back();
      return !stack.empty() && !cancelled;
    }
    if (f.b >= f.P) {
      stack.pop_back();
      return !stack.empty();
    }
    const uint64_t b = f.b, e = std::min(f.P, b + cap[i + 1]);
    f.b = e;
    ExpandArgs a = level_expand_args(i, f.N);
    a.level_pairs = f.P;
    reserve_level(i + 1, e - b);
    zero_counter(kCntRows + i + 1);
    a.pair_begin = b;
    a.pair_end = e;
    a.rows_out = ws.rows[i + 1].as<int32_t>();
    a.W_out = ws.W[i + 1].as<uint32_t>();
    a.apos_out = ws.apos[i + 1].as<uint8_t>();
    a.abase_out = ws.abase[i + 1].as<int64_t>();
    a.counter = dcnt + kCntRows + i + 1;
    expand(a, kModeNext);
    st.chunks[i]++;
    stack.push_back(Frame{i + 1});  // invalidates f
    return true;
  }

  // Filter and first frontier; step() then expands level by level.
  void start() {
    launch_zero_u64(dcnt, 64, s);
    filter();
    stack.clear();
    const int q = p.q;
    const uint32_t qbit0 = (uint32_t)p.order[0];
    if (q == 1) {
      // the candidates of the single query vertex are the embeddings
      int32_t *dst = nullptr;
      uint64_t dcap = 0;
      if (rows_user || o.emit) {
        if (!emit_host) {
          dst = rows_user;
          dcap = rows_cap;
        } else {
          ws.emit.reserve(std::max<int64_t>(g.n, 1) * sizeof(int32_t), s);
          dst = ws.emit.as<int32_t>();
          dcap = (uint64_t)g.n;
        }
      }
      launch_compact_first(dg, ws.cmask.as<uint16_t>(), qbit0, 0, nullptr, nullptr, nullptr, nullptr,
                           dcnt + kCntResult, dst, dcap, s);
      fetch_counters();
      single_count = ws.h_counters[kCntResult];
      st.rows[0] = single_count;
      st.candidates_root = single_count;
      if (emit_host) drain_stage(single_count);
      return;
    }
    reserve_level(1, (uint64_t)std::max<int64_t>(g.n, 1));
    launch_compact_first(dg, ws.cmask.as<uint16_t>(), qbit0, p.qlab[p.order[1]],
                         ws.rows[1].as<int32_t>(), ws.W[1].as<uint32_t>(), ws.abase[1].as<int64_t>(),
                         ws.apos[1].as<uint8_t>(), dcnt + kCntRows + 1, nullptr, 0, s);
    stack.push_back(Frame{1});
  }

  // The count once step() has returned false (waits for the stream).
  uint64_t finish() {
    if (p.q == 1) return single_count;
    fetch_counters();
    st.candidates_root = st.rows[0];
    st.probes = ws.h_counters[kCntProbes];
    st.rows[p.q - 1] = ws.h_counters[kCntResult];
    return ws.h_counters[kCntResult];
  }

  uint64_t run() {
    start();
    while (step()) {
    }
    return finish();
  }

  // Algorithmic bytes of the expansion launches (what the method must move),
  // per row r of level i: its i ids and its anchor's two CSR offsets
  // (4i + 8); per (row, neighbour) pair the neighbour id and its candidate
  // mask entry (4 + 2; pairs are the anchor's neighbours of the new vertex's
  // label); per back-edge other than the anchor the list's two offsets (8)
  // and 4 bytes per step of a binary search of that list, for every pair that
  // reaches the check; per row written to the next level its i+1 ids; per
  // embedding handed out its q ids.  Bookkeeping this implementation adds
  // (range starts, scan entries, anchor positions) is not counted.
  void finish_stats(uint64_t count) {
    uint64_t b = 0;
    for (int i = 1; i < p.q; ++i) {
      const uint64_t others = (uint64_t)std::max(0, __builtin_popcount(p.backmask[i]) - 1);
      b += st.rows[i - 1] * (4ull * i + 8 + 8 * others) + st.pairs[i] * (skips_mask(i) ? 4 : 4 + 2);
      if (i + 1 < p.q) b += st.rows[i] * 4ull * (i + 1);
    }
    b += st.probes * 4;
    if (rows_user || o.emit) b += count * 4ull * p.q;
    st.alg_bytes = b;
    for (int i = 2; i < p.q; ++i) st.frontier_bytes += st.rows[i - 1] * row_bytes(i);
    if (o.profile) {
      double ms = 0;
      for (auto &pr : ev_pairs) {
        float t = 0;
        GSM_HIP(hipEventElapsedTime(&t, pr.first, pr.second));
        ms += t;
      }
      st.ms_expand = ms;
    }
  }
};

// Sorts rows in host or device memory on the device and waits for it.
void sort_rows(int32_t *rows, uint64_t N, int q, int64_t n, bool on_device, SortBuffers &sb, hipStream_t s) {
  if (on_device) {
    sort_rows_device(rows, N, q, n, sb, s);
  } else {
    const size_t bytes = sizeof(int32_t) * q * N;
    sb.rows.reserve(bytes, s);
    GSM_HIP(hipMemcpyAsync(sb.rows.ptr, rows, bytes, hipMemcpyHostToDevice, s));
    sort_rows_device(sb.rows.as<int32_t>(), N, q, n, sb, s);
    GSM_HIP(hipMemcpyAsync(rows, sb.rows.ptr, bytes, hipMemcpyDeviceToHost, s));
  }
  GSM_HIP(hipStreamSynchronize(s));
}

Workspace &acquire_ws(gsm_graph &g) {
  if (!g.ws) g.ws = new Workspace();
  return *g.ws;
}

}  // namespace

uint64_t min_budget_bytes_single(int64_t n, int q) { return min_budget_bytes(n, q, false); }

namespace {
// One query, count only, advanced step by step (the query-uniform kernels).
class SingleCountRun : public StepRun {
 public:
  SingleCountRun(gsm_graph &g, const gsm_query &q, const Options &o, Workspace &ws) : m(g, q, o, ws) {
    m.plan_capacity();
    m.start();
  }
  bool step() override { return m.step(); }
  void finish(uint64_t *counts, std::vector<uint8_t> &moved) override {
    counts[0] = m.finish();
    moved.assign(1, 0);
  }

 private:
  Matcher m;
};
}  // namespace

std::unique_ptr<StepRun> make_single_count_run(gsm_graph &g, const gsm_query &q, const gsm_match_opts &oo,
                                               Workspace &ws, const RootSlice &rs) {
  gsm_match_opts plain = oo;
  plain.root_qvertex = rs.qvertex;
  plain.root_mod = rs.qvertex >= 0 ? rs.mod : 0;
  plain.root_rem = rs.qvertex >= 0 ? rs.rem : 0;
  Options o = read_opts(&plain, q.q);
  o.emit = nullptr;
  o.emit_ctx = nullptr;
  o.rows_dev = false;
  o.stats = nullptr;
  return std::unique_ptr<StepRun>(new SingleCountRun(g, q, o, ws));
}

uint64_t match_count_one(gsm_graph &g, const gsm_query &q, const gsm_match_opts &oo, Workspace &ws,
                         const RootSlice &rs) {
  gsm_match_opts plain = oo;
  plain.root_qvertex = rs.qvertex;
  plain.root_mod = rs.qvertex >= 0 ? rs.mod : 0;
  plain.root_rem = rs.qvertex >= 0 ? rs.rem : 0;
  Options o = read_opts(&plain, q.q);
  o.emit = nullptr;
  o.emit_ctx = nullptr;
  o.rows_dev = false;
  o.stats = nullptr;
  Matcher m(g, q, o, ws);
  m.plan_capacity();
  const uint64_t c = m.run();
  m.sync();
  return c;
}

// The body of gsm_match.  fixed_ws != null: the no-allocation variant, on a
// fixed workspace (no graph lock, no device allocation, no sort, no events).
gsm_status match_call(gsm_graph_t g, gsm_query_t qh, const gsm_match_opts *opts, uint64_t *count,
                      int32_t *rows, uint64_t rows_cap, uint64_t *rows_written, Workspace *fixed_ws) {
  const auto t0 = std::chrono::steady_clock::now();
  try {
    if (!g || !qh || !count) {
      set_error(fixed_ws ? "gsm_match_noalloc: NULL argument" : "gsm_match: NULL argument");
      return GSM_E_INVALID_ARG;
    }
    Options o = read_opts(opts, qh->q);
    if (o.sort && o.emit) {
      set_error("GSM_MATCH_SORT_ROWS needs the rows buffer, not an emit callback");
      return GSM_E_UNSUPPORTED;
    }
    std::unique_lock<std::mutex> lk(g->mu, std::defer_lock);
    Workspace *wsp = fixed_ws;
    if (fixed_ws) {
      if (o.sort) {
        set_error("gsm_match_noalloc: GSM_MATCH_SORT_ROWS needs sort buffers; sort with gsm_sort_rows");
        return GSM_E_UNSUPPORTED;
      }
      o.profile = false;  // no event objects are created
      // the level budget is what the scratch holds after its header, minus
      // the alignment of each window
      const uint64_t room = fixed_ws->fixed_bytes - Workspace::fixed_header_bytes() - (uint64_t(24) << 10);
      if (fixed_bytes(g->n) + 64 > room) {
        set_error("gsm_match_noalloc: a graph of " + std::to_string(g->n) + " vertices needs " +
                  std::to_string(fixed_bytes(g->n) + 64) + " bytes of scratch for its candidate masks and "
                  "first frontier; the no-allocation scratch holds " + std::to_string(room));
        return GSM_E_BUDGET;
      }
      o.budget = std::min<uint64_t>(o.budget, room);
    } else {
      lk.lock();
      wsp = &acquire_ws(*g);
    }
    Workspace &ws = *wsp;
    Matcher m(*g, *qh, o, ws);
    m.rows_user = rows;
    m.rows_cap = rows ? rows_cap : 0;
    m.emit_host = (o.emit != nullptr) || (rows != nullptr && !o.rows_dev);
    m.plan_capacity();
    const uint64_t c = m.run();
    m.sync();
    m.finish_stats(c);
    *count = c;
    const uint64_t written = rows ? std::min(c, rows_cap) : 0;
    if (o.sort && written > 1) sort_rows(rows, written, qh->q, g->n, o.rows_dev, ws.sort, m.s);
    if (rows_written) *rows_written = written;
    if (o.stats) {
      m.st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      const uint32_t sz = std::min<uint32_t>(o.stats->struct_size ? o.stats->struct_size : sizeof(gsm_stats),
                                             sizeof(gsm_stats));
      std::memcpy(o.stats, &m.st, sz);
      o.stats->struct_size = sz;
    }
    if (m.cancelled) {
      set_error("emit callback stopped the match");
      return GSM_E_CANCELLED;
    }
    if (rows && c > rows_cap) {
      set_error("count exceeds rows_cap; first rows_cap rows written");
      return GSM_E_TRUNCATED;
    }
    return GSM_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return GSM_E_OOM;
  }
}

}  // namespace gsm

using gsm::Error;

extern "C" {

void gsm_match_opts_init(gsm_match_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(*o);
  o->filter_rounds = 1;
  o->use_degree = 1;
  o->use_ne = 1;
  o->root_qvertex = -1;
}

gsm_status gsm_filter(gsm_graph_t g, gsm_query_t qh, const gsm_match_opts *opts, uint16_t *cmask) {
  try {
    if (!g || !qh || !cmask) {
      gsm::set_error("gsm_filter: NULL argument");
      return GSM_E_INVALID_ARG;
    }
    const gsm::Options o = gsm::read_opts(opts, qh->q);
    std::lock_guard<std::mutex> lk(g->mu);
    gsm::Workspace &ws = gsm::acquire_ws(*g);
    gsm::Matcher m(*g, *qh, o, ws);
    m.filter();
    if (g->n)
      GSM_HIP(hipMemcpyAsync(cmask, ws.cmask.ptr, g->n * sizeof(uint16_t), hipMemcpyDeviceToHost, m.s));
    m.sync();
    if (!g->h_orig.empty()) {  // back to the caller's vertex order
      std::vector<uint16_t> t(cmask, cmask + g->n);
      for (int64_t v = 0; v < g->n; ++v) cmask[g->h_orig[v]] = t[v];
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

gsm_status gsm_match(gsm_graph_t g, gsm_query_t qh, const gsm_match_opts *opts, uint64_t *count,
                     int32_t *rows, uint64_t rows_cap, uint64_t *rows_written) {
  return gsm::match_call(g, qh, opts, count, rows, rows_cap, rows_written, nullptr);
}

gsm_status gsm_sort_rows(gsm_graph_t g, int32_t *rows, uint64_t nrows, int32_t q, int32_t rows_on_device,
                          void *hip_stream) {
  try {
    if (!g || (!rows && nrows)) {
      gsm::set_error("gsm_sort_rows: NULL argument");
      return GSM_E_INVALID_ARG;
    }
    if (q < 1 || q > gsm::kMaxQ) {
      gsm::set_error("gsm_sort_rows: q out of [1, 16]");
      return GSM_E_INVALID_ARG;
    }
    if (nrows < 2) return GSM_OK;
    std::lock_guard<std::mutex> lk(g->mu);
    gsm::Workspace &ws = gsm::acquire_ws(*g);
    gsm::sort_rows(rows, nrows, q, g->n, rows_on_device != 0, ws.sort, (hipStream_t)hip_stream);
    return GSM_OK;
  } catch (const Error &e) {
    gsm::set_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc &) {
    gsm::set_error("host allocation failed");
    return GSM_E_OOM;
  }
}

gsm_status gsm_match_min_budget(gsm_graph_t g, gsm_query_t qh, int32_t host_rows, uint64_t *bytes) {
  try {
    if (!g || !qh || !bytes) {
      gsm::set_error("gsm_match_min_budget: NULL argument");
      return GSM_E_INVALID_ARG;
    }
    *bytes = gsm::min_budget_bytes(g->n, qh->q, host_rows != 0);
    return GSM_OK;
  } catch (const Error &e) {
    gsm::set_error(e.msg);
    return e.status;
  }
}

}  // extern "C"
