// C ABI: errors, graph and query handles, the visiting-order query.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <new>
#include <thread>

#include "gsm_internal.h"

namespace gsm {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

namespace {
// failure injection for tests: number of device allocations still allowed,
// or -1 for no limit
std::atomic<int64_t> g_allocs_left{-1};
}  // namespace

namespace {
// one unit of the failure-injection allowance, or an injected failure
void take_allocation() {
  int64_t left = g_allocs_left.load();
  while (left >= 0) {
    if (left == 0) throw Error{GSM_E_OOM, "device allocation refused (failure injection)"};
    if (g_allocs_left.compare_exchange_weak(left, left - 1)) break;
  }
}
}  // namespace

void device_alloc(void **p, size_t bytes) {
  *p = nullptr;
  take_allocation();
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    throw Error{GSM_E_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
}

void device_alloc_async(void **p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  take_allocation();
  if (hipMallocAsync(p, bytes, s) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    throw Error{GSM_E_OOM, "hipMallocAsync of " + std::to_string(bytes) + " bytes failed"};
  }
}

void DevBuf::reserve(size_t want, hipStream_t s) {
  if (want <= bytes && ptr) return;
  if (fixed) {
    if (want == 0) return;
    throw Error{GSM_E_BUDGET, "no-allocation scratch: a buffer of " + std::to_string(want) +
                                  " bytes does not fit its window of " + std::to_string(bytes)};
  }
  release(s);  // stream-ordered: the old block is freed after the stream's earlier work
  if (want == 0) return;
  const size_t b = (want + 255) & ~size_t(255);
  device_alloc_async(&ptr, b, s);
  bytes = b;
  pooled = true;
}

void DevBuf::release(hipStream_t s) {
  if (ptr && !fixed) {
    if (pooled)
      (void)hipFreeAsync(ptr, s);
    else
      (void)hipFree(ptr);
  }
  ptr = nullptr;
  bytes = 0;
  fixed = false;
  pooled = false;
}

// Label-grouped copy of the adjacency: each row stably partitioned by
// neighbour label (ids stay ascending inside a label), and per-row offsets of
// every label.  Built once per graph for labelled graphs with few labels.
void build_label_table(gsm_graph &g, const int64_t *rp, const int32_t *col, const int32_t *lab) {
  const int32_t L = g.max_label + 1;
  if (!lab || L > kMaxTableLabels || g.n == 0) return;
  const int32_t stride = L + 1;
  std::vector<uint32_t> off((size_t)g.n * stride);
  std::vector<int32_t> cl((size_t)std::max<int64_t>(g.nnz, 1));
  std::vector<uint32_t> cnt(stride);
  for (int64_t v = 0; v < g.n; ++v) {
    std::fill(cnt.begin(), cnt.end(), 0u);
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k) cnt[lab[col[k]] + 1]++;
    for (int32_t l = 0; l < L; ++l) cnt[l + 1] += cnt[l];
    uint32_t *o = off.data() + (size_t)v * stride;
    for (int32_t l = 0; l <= L; ++l) o[l] = cnt[l];
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k) cl[rp[v] + cnt[lab[col[k]]]++] = col[k];
  }
  device_alloc((void **)&g.col_lab, cl.size() * sizeof(int32_t));
  GSM_HIP(hipMemcpy(g.col_lab, cl.data(), cl.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  device_alloc((void **)&g.loff, off.size() * sizeof(uint32_t));
  GSM_HIP(hipMemcpy(g.loff, off.data(), off.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  g.loff_stride = stride;
}

// Edge labels in col_lab order: the same stable per-row grouping by
// neighbour label that build_label_table applies to col.
void build_edge_label_table(gsm_graph &g, const int64_t *rp, const int32_t *col, const int32_t *lab,
                            const int32_t *elab) {
  if (!g.col_lab || !elab) return;
  const int32_t L = g.max_label + 1;
  std::vector<int32_t> el((size_t)std::max<int64_t>(g.nnz, 1));
  std::vector<uint32_t> cnt(L + 1);
  for (int64_t v = 0; v < g.n; ++v) {
    std::fill(cnt.begin(), cnt.end(), 0u);
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k) cnt[lab[col[k]] + 1]++;
    for (int32_t l = 0; l < L; ++l) cnt[l + 1] += cnt[l];
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k) el[rp[v] + cnt[lab[col[k]]]++] = elab[k];
  }
  device_alloc((void **)&g.elab_lab, el.size() * sizeof(int32_t));
  GSM_HIP(hipMemcpy(g.elab_lab, el.data(), el.size() * sizeof(int32_t), hipMemcpyHostToDevice));
}

Workspace::Workspace() {
  counters.reserve(64 * sizeof(uint64_t), nullptr);
  scan_scratch.reserve(scan_scratch_elems() * sizeof(uint64_t), nullptr);
  GSM_HIP(hipHostMalloc((void **)&h_counters, 64 * sizeof(uint64_t), hipHostMallocDefault));
  std::memset(h_counters, 0, 64 * sizeof(uint64_t));
}

size_t Workspace::fixed_header_bytes() {
  return 64 * sizeof(uint64_t) + ((scan_scratch_elems() * sizeof(uint64_t) + 255) & ~size_t(255));
}

Workspace::Workspace(void *base, size_t bytes) {
  fixed_base = static_cast<char *>(base);
  fixed_bytes = bytes;
  if (bytes < fixed_header_bytes()) throw Error{GSM_E_BUDGET, "no-allocation scratch below its header"};
  counters.set_fixed(fixed_base, 64 * sizeof(uint64_t));
  scan_scratch.set_fixed(fixed_base + 64 * sizeof(uint64_t), fixed_header_bytes() - 64 * sizeof(uint64_t));
  h_counters = h_local;
  std::memset(h_local, 0, sizeof(h_local));
}

Workspace::~Workspace() {
  for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
  if (h_counters && h_counters != h_local) (void)hipHostFree(h_counters);
  for (auto &e : events) (void)hipEventDestroy(e);
}

}  // namespace gsm

using gsm::Error;

#define GSM_API_BEGIN try {
#define GSM_API_END                                        \
  }                                                        \
  catch (const Error &e) {                                 \
    gsm::set_error(e.msg);                                 \
    return e.status;                                       \
  }                                                        \
  catch (const std::bad_alloc &) {                         \
    gsm::set_error("host allocation failed");              \
    return GSM_E_OOM;                                      \
  }                                                        \
  catch (const std::exception &e) {                        \
    gsm::set_error(e.what());                              \
    return GSM_E_DEVICE;                                   \
  }

extern "C" {

const char *gsm_status_str(gsm_status s) {
  switch (s) {
    case GSM_OK: return "ok";
    case GSM_E_INVALID_ARG: return "invalid argument";
    case GSM_E_BAD_GRAPH: return "bad graph";
    case GSM_E_BAD_QUERY: return "bad query";
    case GSM_E_OOM: return "out of memory";
    case GSM_E_BUDGET: return "memory budget too small";
    case GSM_E_DEVICE: return "device error";
    case GSM_E_TRUNCATED: return "output truncated";
    case GSM_E_CANCELLED: return "cancelled";
    case GSM_E_UNSUPPORTED: return "unsupported";
    case GSM_E_TIMEOUT: return "timeout";
  }
  return "unknown status";
}

const char *gsm_last_error(void) { return gsm::g_last_error.c_str(); }

static gsm_status validate_csr(int64_t n, const int64_t *rp, const int32_t *col) {
  if (rp[0] != 0) {
    gsm::set_error("row_ptr[0] != 0");
    return GSM_E_BAD_GRAPH;
  }
  for (int64_t v = 0; v < n; ++v) {
    if (rp[v + 1] < rp[v]) {
      gsm::set_error("row_ptr decreases at vertex " + std::to_string(v));
      return GSM_E_BAD_GRAPH;
    }
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
      const int32_t w = col[k];
      if (w < 0 || w >= n) {
        gsm::set_error("neighbour id out of range in row " + std::to_string(v));
        return GSM_E_BAD_GRAPH;
      }
      if (w == v) {
        gsm::set_error("self-loop at vertex " + std::to_string(v));
        return GSM_E_BAD_GRAPH;
      }
      if (k > rp[v] && col[k - 1] >= w) {
        gsm::set_error("row " + std::to_string(v) + " not strictly ascending");
        return GSM_E_BAD_GRAPH;
      }
    }
  }
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
      const int32_t w = col[k];
      if (!std::binary_search(col + rp[w], col + rp[w + 1], (int32_t)v)) {
        gsm::set_error("edge " + std::to_string(v) + "-" + std::to_string(w) + " not symmetric");
        return GSM_E_BAD_GRAPH;
      }
    }
  return GSM_OK;
}

// Simple undirected CSR from any adjacency: every entry v->w with v != w
// becomes the edge {v, w} stored in both rows; rows are sorted and duplicate
// entries dropped.  Offsets and ids must still be well formed.
static gsm_status strip_csr(int64_t n, const int64_t *rp, const int32_t *col, std::vector<int64_t> &out_rp,
                            std::vector<int32_t> &out_col) {
  if (rp[0] != 0) {
    gsm::set_error("row_ptr[0] != 0");
    return GSM_E_BAD_GRAPH;
  }
  std::vector<int64_t> cnt((size_t)n + 1, 0);
  for (int64_t v = 0; v < n; ++v) {
    if (rp[v + 1] < rp[v]) {
      gsm::set_error("row_ptr decreases at vertex " + std::to_string(v));
      return GSM_E_BAD_GRAPH;
    }
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
      const int32_t w = col[k];
      if (w < 0 || w >= n) {
        gsm::set_error("neighbour id out of range in row " + std::to_string(v));
        return GSM_E_BAD_GRAPH;
      }
      if (w == v) continue;
      cnt[v + 1]++;
      cnt[w + 1]++;
    }
  }
  for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  std::vector<int32_t> both((size_t)cnt[n]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t v = 0; v < n; ++v)
    for (int64_t k = rp[v]; k < rp[v + 1]; ++k) {
      const int32_t w = col[k];
      if (w == v) continue;
      both[fill[v]++] = w;
      both[fill[w]++] = (int32_t)v;
    }
  out_rp.assign((size_t)n + 1, 0);
  out_col.clear();
  out_col.reserve(both.size());
  for (int64_t v = 0; v < n; ++v) {
    auto b = both.begin() + cnt[v], e = both.begin() + cnt[v + 1];
    std::sort(b, e);
    e = std::unique(b, e);
    out_col.insert(out_col.end(), b, e);
    out_rp[v + 1] = (int64_t)out_col.size();
  }
  return GSM_OK;
}

void gsm_testing_fail_allocations(int64_t after) { gsm::g_allocs_left.store(after < 0 ? -1 : after); }

gsm_status gsm_query_set_edge_labels(gsm_query_t qh, const int32_t *edge_labels) {
  GSM_API_BEGIN
  if (!qh || (!edge_labels && !qh->edges.empty())) {
    gsm::set_error("gsm_query_set_edge_labels: NULL argument");
    return GSM_E_INVALID_ARG;
  }
  const size_t ne = qh->edges.size() / 2;
  for (size_t e = 0; e < ne; ++e)
    if (edge_labels[e] < 0) {
      gsm::set_error("negative query edge label");
      return GSM_E_BAD_QUERY;
    }
  for (size_t e = 0; e < ne; ++e) {
    const int32_t a = qh->edges[2 * e], b = qh->edges[2 * e + 1];
    qh->elab[a][b] = qh->elab[b][a] = edge_labels[e];
  }
  qh->has_elab = true;
  gsm::compute_symmetry(*qh);  // automorphisms must keep edge labels too
  return GSM_OK;
  GSM_API_END
}

gsm_status gsm_query_symmetry(gsm_query_t qh, uint64_t *aut, int32_t *pairs, int32_t pairs_cap,
                              int32_t *npairs) {
  GSM_API_BEGIN
  if (!qh || (pairs_cap > 0 && !pairs)) {
    gsm::set_error("gsm_query_symmetry: NULL argument");
    return GSM_E_INVALID_ARG;
  }
  const int32_t n = (int32_t)(qh->sym_pairs.size() / 2);
  if (aut) *aut = qh->aut;
  if (npairs) *npairs = n;
  for (int32_t k = 0; k < n && k < pairs_cap; ++k) {
    pairs[2 * k] = qh->sym_pairs[2 * k];
    pairs[2 * k + 1] = qh->sym_pairs[2 * k + 1];
  }
  return GSM_OK;
  GSM_API_END
}

// Renumbers a valid CSR by ascending degree, ties by id: orig[v'] is the
// old id of new vertex v'; rows are rebuilt in the new numbering and sorted
// (edge labels move with their entries).  Rows are split over host threads.
static void renumber_by_degree(int64_t n, const int64_t *rp, const int32_t *col, const int32_t *lab,
                               const int32_t *el, std::vector<int32_t> &orig, std::vector<int64_t> &nrp,
                               std::vector<int32_t> &ncol, std::vector<int32_t> &nlab,
                               std::vector<int32_t> &nel) {
  int64_t maxd = 0;
  for (int64_t v = 0; v < n; ++v) maxd = std::max(maxd, rp[v + 1] - rp[v]);
  std::vector<int64_t> at((size_t)maxd + 2, 0);
  for (int64_t v = 0; v < n; ++v) at[rp[v + 1] - rp[v] + 1]++;
  for (int64_t d = 0; d <= maxd; ++d) at[d + 1] += at[d];
  orig.assign((size_t)n, 0);
  for (int64_t v = 0; v < n; ++v) orig[at[rp[v + 1] - rp[v]]++] = (int32_t)v;
  std::vector<int32_t> newid((size_t)n);
  for (int64_t v = 0; v < n; ++v) newid[orig[v]] = (int32_t)v;
  nrp.assign((size_t)n + 1, 0);
  for (int64_t v = 0; v < n; ++v) nrp[v + 1] = nrp[v] + (rp[orig[v] + 1] - rp[orig[v]]);
  const int64_t nnz = nrp[n];
  ncol.assign((size_t)nnz, 0);
  if (el) nel.assign((size_t)nnz, 0);
  if (lab) {
    nlab.assign((size_t)n, 0);
    for (int64_t v = 0; v < n; ++v) nlab[v] = lab[orig[v]];
  }
  const unsigned hw = std::thread::hardware_concurrency();
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)(hw ? hw : 1), 16, nnz / 65536 + 1}));
  std::vector<std::vector<uint64_t>> keys((size_t)nt);
  if (el)
    for (auto &k : keys) k.resize((size_t)maxd);
  auto work = [&](int t) {
    for (int64_t v = n * t / nt; v < n * (t + 1) / nt; ++v) {
      const int64_t b = rp[orig[v]], d = rp[orig[v] + 1] - b, o = nrp[v];
      if (el) {
        uint64_t *kk = keys[t].data();
        for (int64_t j = 0; j < d; ++j)
          kk[j] = ((uint64_t)(uint32_t)newid[col[b + j]] << 32) | (uint32_t)el[b + j];
        std::sort(kk, kk + d);
        for (int64_t j = 0; j < d; ++j) {
          ncol[o + j] = (int32_t)(kk[j] >> 32);
          nel[o + j] = (int32_t)(uint32_t)kk[j];
        }
      } else {
        for (int64_t j = 0; j < d; ++j) ncol[o + j] = newid[col[b + j]];
        std::sort(ncol.begin() + o, ncol.begin() + o + d);
      }
    }
  };
  std::vector<std::thread> th;
  int started = 1;
  for (; started < nt; ++started) {
    try {
      th.emplace_back(work, started);
    } catch (...) {
      break;  // the ranges of threads that could not start run here
    }
  }
  for (int t = started; t < nt; ++t) work(t);
  work(0);
  for (auto &x : th) x.join();
}

gsm_status gsm_graph_create(int64_t n, const int64_t *row_ptr, const int32_t *col,
                            const int32_t *labels, uint32_t flags, gsm_graph_t *out) {
  return gsm_graph_create_ex(n, row_ptr, col, labels, nullptr, flags, out);
}

gsm_status gsm_graph_create_ex(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *labels,
                               const int32_t *edge_labels, uint32_t flags, gsm_graph_t *out) {
  GSM_API_BEGIN
  if (edge_labels && (flags & GSM_GRAPH_STRIP)) {
    gsm::set_error("gsm_graph_create_ex: edge labels cannot be combined with GSM_GRAPH_STRIP");
    return GSM_E_UNSUPPORTED;
  }
  if (!out || n < 0 || n >= (int64_t(1) << 31) || !row_ptr) {
    gsm::set_error("gsm_graph_create: invalid arguments");
    return GSM_E_INVALID_ARG;
  }
  const bool dev = flags & GSM_GRAPH_DEVICE_PTRS;
  // host views of the inputs (downloaded when the caller handed device pointers)
  std::vector<int64_t> h_rp_store;
  std::vector<int32_t> h_col_store, h_lab_store;
  const int64_t *h_rp = row_ptr;
  const int32_t *h_col = col, *h_lab = labels;
  int64_t nnz;
  if (dev) {
    h_rp_store.resize(n + 1);
    GSM_HIP(hipMemcpy(h_rp_store.data(), row_ptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    h_rp = h_rp_store.data();
    nnz = h_rp[n];
    if (nnz < 0) {
      gsm::set_error("row_ptr[n] < 0");
      return GSM_E_BAD_GRAPH;
    }
    if ((flags & (GSM_GRAPH_VALIDATE | GSM_GRAPH_STRIP | GSM_GRAPH_DEGREE_ORDER)) || labels || edge_labels) {
      h_col_store.resize(nnz);
      if (nnz)
        GSM_HIP(hipMemcpy(h_col_store.data(), col, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
      h_col = h_col_store.data();
    }
    if (labels) {
      h_lab_store.resize(n);
      if (n) GSM_HIP(hipMemcpy(h_lab_store.data(), labels, n * sizeof(int32_t), hipMemcpyDeviceToHost));
      h_lab = h_lab_store.data();
    }
  } else {
    nnz = row_ptr[n];
  }
  if (nnz > 0 && !col) {
    gsm::set_error("gsm_graph_create: col is NULL");
    return GSM_E_INVALID_ARG;
  }
  // CSR arrays to upload: the caller's, or the cleaned host copy
  const int64_t *src_rp = row_ptr;
  const int32_t *src_col = col;
  hipMemcpyKind csr_kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  std::vector<int64_t> clean_rp;
  std::vector<int32_t> clean_col;
  if (flags & GSM_GRAPH_STRIP) {
    gsm_status st = strip_csr(n, h_rp, h_col, clean_rp, clean_col);
    if (st != GSM_OK) return st;
    h_rp = src_rp = clean_rp.data();
    h_col = src_col = clean_col.data();
    nnz = clean_rp[n];
    csr_kind = hipMemcpyHostToDevice;
  }
  if (flags & GSM_GRAPH_VALIDATE) {
    gsm_status st = validate_csr(n, h_rp, h_col);
    if (st != GSM_OK) return st;
  }
  // edge labels: host view, non-negative, equal in both directions
  std::vector<int32_t> h_el_store;
  const int32_t *h_el = edge_labels;
  if (edge_labels && dev) {
    h_el_store.resize(nnz);
    if (nnz) GSM_HIP(hipMemcpy(h_el_store.data(), edge_labels, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    h_el = h_el_store.data();
  }
  if (h_el) {
    for (int64_t k = 0; k < nnz; ++k)
      if (h_el[k] < 0) {
        gsm::set_error("negative edge label at CSR entry " + std::to_string(k));
        return GSM_E_BAD_GRAPH;
      }
    if (flags & GSM_GRAPH_VALIDATE)
      for (int64_t v = 0; v < n; ++v)
        for (int64_t k = h_rp[v]; k < h_rp[v + 1]; ++k) {
          const int32_t w = h_col[k];
          const int32_t *b = h_col + h_rp[w], *e = h_col + h_rp[w + 1];
          const int32_t *it = std::lower_bound(b, e, (int32_t)v);
          if (h_el[h_rp[w] + (it - b)] != h_el[k]) {
            gsm::set_error("edge " + std::to_string(v) + "-" + std::to_string(w) + " has two labels");
            return GSM_E_BAD_GRAPH;
          }
        }
  }
  int32_t max_label = 0;
  if (h_lab)
    for (int64_t v = 0; v < n; ++v) {
      if (h_lab[v] < 0) {
        gsm::set_error("negative label at vertex " + std::to_string(v));
        return GSM_E_BAD_GRAPH;
      }
      max_label = std::max(max_label, h_lab[v]);
    }
  // GSM_GRAPH_DEGREE_ORDER: the graph is stored renumbered by ascending
  // degree (ties by id), rows re-sorted in the new numbering
  const bool reorder = (flags & GSM_GRAPH_DEGREE_ORDER) && n > 0;
  std::vector<int32_t> orig_of;
  std::vector<int64_t> re_rp;
  std::vector<int32_t> re_col, re_lab, re_el;
  if (reorder) {
    // the renumbering indexes by offsets and ids: check their ranges even
    // without GSM_GRAPH_VALIDATE
    for (int64_t v = 0; v < n; ++v)
      if (h_rp[v + 1] < h_rp[v] || h_rp[0] != 0) {
        gsm::set_error("row_ptr is not non-decreasing from 0");
        return GSM_E_BAD_GRAPH;
      }
    for (int64_t k = 0; k < nnz; ++k)
      if (h_col[k] < 0 || h_col[k] >= n) {
        gsm::set_error("neighbour id out of range at CSR entry " + std::to_string(k));
        return GSM_E_BAD_GRAPH;
      }
    renumber_by_degree(n, h_rp, h_col, h_lab, h_el, orig_of, re_rp, re_col, re_lab, re_el);
    h_rp = src_rp = re_rp.data();
    h_col = src_col = re_col.data();
    csr_kind = hipMemcpyHostToDevice;
    if (h_lab) h_lab = re_lab.data();
    if (h_el) h_el = re_el.data();
  }
  const int32_t *lab_src = reorder ? h_lab : labels;
  auto g = new gsm_graph();
  try {
    g->n = n;
    g->nnz = nnz;
    g->labelled = labels != nullptr;
    g->max_label = max_label;
    const hipMemcpyKind kind = (dev && !reorder) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    gsm::device_alloc((void **)&g->rp, (n + 1) * sizeof(int64_t));
    GSM_HIP(hipMemcpy(g->rp, src_rp, (n + 1) * sizeof(int64_t), csr_kind));
    gsm::device_alloc((void **)&g->col, std::max<int64_t>(nnz, 1) * sizeof(int32_t));
    if (nnz) GSM_HIP(hipMemcpy(g->col, src_col, nnz * sizeof(int32_t), csr_kind));
    gsm::device_alloc((void **)&g->deg, std::max<int64_t>(n, 1) * sizeof(uint32_t));
    gsm::device_alloc((void **)&g->dne, std::max<int64_t>(n, 1) * sizeof(uint2));
    if (labels) {
      gsm::device_alloc((void **)&g->lab, std::max<int64_t>(n, 1) * sizeof(int32_t));
      if (n) GSM_HIP(hipMemcpy(g->lab, lab_src, n * sizeof(int32_t), kind));
      gsm::device_alloc((void **)&g->ne0, std::max<int64_t>(n, 1) * sizeof(uint64_t));
    }
    gsm::launch_graph_stats(*g, nullptr);
    // planner statistics and the high-degree vertex list
    g->label_count.assign((size_t)max_label + 1, 0);
    int64_t maxd = 0;
    std::vector<int32_t> heavy;
    for (int64_t v = 0; v < n; ++v) {
      const int64_t d = h_rp[v + 1] - h_rp[v];
      maxd = std::max(maxd, d);
      if (d > gsm::kHeavyDegree) heavy.push_back((int32_t)v);
      g->label_count[h_lab ? h_lab[v] : 0]++;
    }
    // vertices grouped by label, ascending within a label: a batched first
    // frontier scans only the class of its first query vertex
    g->lab_start.assign((size_t)max_label + 2, 0);
    for (int32_t l = 0; l <= max_label; ++l) g->lab_start[l + 1] = g->lab_start[l] + g->label_count[l];
    if (h_lab && n > 0) {
      std::vector<int32_t> by_label((size_t)n);
      std::vector<int64_t> at(g->lab_start.begin(), g->lab_start.end() - 1);
      for (int64_t v = 0; v < n; ++v) by_label[at[h_lab[v]]++] = (int32_t)v;
      gsm::device_alloc((void **)&g->lab_vert, (size_t)n * sizeof(int32_t));
      GSM_HIP(hipMemcpy(g->lab_vert, by_label.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    g->max_degree = maxd;
    g->deg_ge.assign((size_t)maxd + 2, 0);
    for (int64_t v = 0; v < n; ++v) g->deg_ge[h_rp[v + 1] - h_rp[v]]++;
    for (int64_t d = maxd; d >= 0; --d) g->deg_ge[d] += g->deg_ge[d + 1];
    gsm::build_label_table(*g, h_rp, h_col, h_lab);
    if (h_el) {
      gsm::device_alloc((void **)&g->elab, std::max<int64_t>(nnz, 1) * sizeof(int32_t));
      if (nnz) GSM_HIP(hipMemcpy(g->elab, h_el, nnz * sizeof(int32_t), hipMemcpyHostToDevice));
      gsm::build_edge_label_table(*g, h_rp, h_col, h_lab, h_el);
    }
    g->nheavy = (int64_t)heavy.size();
    if (!heavy.empty()) {
      gsm::device_alloc((void **)&g->heavy, heavy.size() * sizeof(int32_t));
      GSM_HIP(hipMemcpy(g->heavy, heavy.data(), heavy.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    std::vector<int32_t> slot;  // bitmap index of each vertex, or -1 (empty: no bitmaps)
    if (!(flags & GSM_GRAPH_NO_HUB_BITMAPS) && n > 0) {
      // adjacency bitmaps of the highest-degree vertices, while they fit
      const uint64_t words = ((uint64_t)n + 31) / 32;
      uint64_t cap = gsm::kHubBitmapBytes;
      size_t free_b = 0, total_b = 0;
      if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) cap = std::min<uint64_t>(cap, free_b / 4);
      const uint64_t fit = cap / (words * 4);
      std::vector<int32_t> hubs;
      for (int64_t v = 0; v < n; ++v)
        if (h_rp[v + 1] - h_rp[v] >= gsm::kHubMinDegree) hubs.push_back((int32_t)v);
      std::stable_sort(hubs.begin(), hubs.end(), [&](int32_t a, int32_t b) {
        return h_rp[a + 1] - h_rp[a] > h_rp[b + 1] - h_rp[b];
      });
      if (hubs.size() > fit) hubs.resize(fit);
      if (!hubs.empty()) {
        slot.assign((size_t)n, -1);
        for (size_t k = 0; k < hubs.size(); ++k) slot[hubs[k]] = (int32_t)k;
        gsm::device_alloc((void **)&g->hub_bits, hubs.size() * words * 4);
        GSM_HIP(hipMemset(g->hub_bits, 0, hubs.size() * words * 4));
        int32_t *d_hubs = nullptr;
        gsm::device_alloc((void **)&d_hubs, hubs.size() * sizeof(int32_t));
        hipError_t e = hipMemcpy(d_hubs, hubs.data(), hubs.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        g->hub_words = words;
        g->nhubs = (int64_t)hubs.size();
        if (e == hipSuccess) {
          try {
            gsm::launch_build_hub_bitmaps(*g, d_hubs, g->nhubs, nullptr);
          } catch (...) {
            (void)hipDeviceSynchronize();
            (void)hipFree(d_hubs);
            throw;
          }
          e = hipDeviceSynchronize();
        }
        (void)hipFree(d_hubs);
        if (e != hipSuccess) throw Error{GSM_E_DEVICE, std::string("hub bitmaps: ") + hipGetErrorString(e)};
      }
    }
    if (n > 0) {
      // one 16-byte record per vertex for the edge checks: list start (two
      // halves), length, bitmap index or -1
      std::vector<int4> vd((size_t)n);
      for (int64_t v = 0; v < n; ++v) {
        const uint64_t b = (uint64_t)h_rp[v];
        vd[v] = make_int4((int32_t)(uint32_t)b, (int32_t)(uint32_t)(b >> 32), (int32_t)(h_rp[v + 1] - h_rp[v]),
                          slot.empty() ? -1 : slot[v]);
      }
      gsm::device_alloc((void **)&g->vdesc, (size_t)n * sizeof(int4));
      GSM_HIP(hipMemcpy(g->vdesc, vd.data(), (size_t)n * sizeof(int4), hipMemcpyHostToDevice));
    }
    if (reorder) {
      gsm::device_alloc((void **)&g->orig, (size_t)n * sizeof(int32_t));
      GSM_HIP(hipMemcpy(g->orig, orig_of.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice));
      g->h_orig = std::move(orig_of);
    }
    GSM_HIP(hipDeviceSynchronize());
  } catch (...) {
    gsm_graph_destroy(g);
    throw;
  }
  *out = g;
  return GSM_OK;
  GSM_API_END
}

void gsm_graph_destroy(gsm_graph_t g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  delete g->ws;
  (void)hipFree(g->rp);
  (void)hipFree(g->col);
  (void)hipFree(g->lab);
  (void)hipFree(g->deg);
  (void)hipFree(g->dne);
  (void)hipFree(g->ne0);
  (void)hipFree(g->heavy);
  (void)hipFree(g->vdesc);
  (void)hipFree(g->hub_bits);
  (void)hipFree(g->lab_vert);
  (void)hipFree(g->orig);
  (void)hipFree(g->col_lab);
  (void)hipFree(g->loff);
  (void)hipFree(g->elab);
  (void)hipFree(g->elab_lab);
  delete g;
}

gsm_status gsm_graph_info(gsm_graph_t g, int64_t *n, int64_t *nnz, int32_t *max_label,
                          int64_t *max_degree) {
  if (!g) {
    gsm::set_error("gsm_graph_info: NULL graph");
    return GSM_E_INVALID_ARG;
  }
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  if (max_label) *max_label = g->max_label;
  if (max_degree) *max_degree = g->max_degree;
  return GSM_OK;
}

gsm_status gsm_query_create(int32_t q, int32_t ne, const int32_t *edges, const int32_t *labels,
                            gsm_query_t *out) {
  GSM_API_BEGIN
  if (!out || ne < 0 || (ne > 0 && !edges)) {
    gsm::set_error("gsm_query_create: invalid arguments");
    return GSM_E_INVALID_ARG;
  }
  if (q < 1 || q > gsm::kMaxQ) {
    gsm::set_error("query size must be in [1, 16]");
    return GSM_E_BAD_QUERY;
  }
  auto qh = std::make_unique<gsm_query>();
  qh->q = q;
  for (int e = 0; e < ne; ++e) {
    const int32_t a = edges[2 * e], b = edges[2 * e + 1];
    if (a < 0 || b < 0 || a >= q || b >= q || a == b) {
      gsm::set_error("query edge " + std::to_string(e) + " out of range or a self-loop");
      return GSM_E_BAD_QUERY;
    }
    if ((qh->adj[a] >> b) & 1) {
      gsm::set_error("duplicate query edge " + std::to_string(a) + "-" + std::to_string(b));
      return GSM_E_BAD_QUERY;
    }
    qh->adj[a] |= 1u << b;
    qh->adj[b] |= 1u << a;
    qh->edges.push_back(a);
    qh->edges.push_back(b);
  }
  for (int u = 0; u < q; ++u) {
    qh->label[u] = labels ? labels[u] : 0;
    if (qh->label[u] < 0) {
      gsm::set_error("negative query label");
      return GSM_E_BAD_QUERY;
    }
  }
  uint32_t seen = 1, frontier = 1;
  while (frontier) {
    uint32_t nxt = 0;
    for (int u = 0; u < q; ++u)
      if ((frontier >> u) & 1) nxt |= qh->adj[u];
    frontier = nxt & ~seen;
    seen |= nxt;
  }
  if (seen != ((q == 32) ? 0xffffffffu : ((1u << q) - 1u))) {
    gsm::set_error("query graph is not connected");
    return GSM_E_BAD_QUERY;
  }
  gsm::compute_symmetry(*qh);
  *out = qh.release();
  return GSM_OK;
  GSM_API_END
}

void gsm_query_destroy(gsm_query_t qh) { delete qh; }

gsm_status gsm_query_plan(gsm_graph_t g, gsm_query_t qh, gsm_plan_info *out) {
  GSM_API_BEGIN
  if (!g || !qh || !out) {
    gsm::set_error("gsm_query_plan: NULL argument");
    return GSM_E_INVALID_ARG;
  }
  const gsm::Plan p = gsm::make_plan(*g, *qh);
  std::memset(out, 0, sizeof(*out));
  out->q = p.q;
  for (int i = 0; i < p.q; ++i) {
    out->order[i] = p.order[i];
    out->parent[i] = p.parent[i];
    out->backmask[i] = p.backmask[i];
  }
  return GSM_OK;
  GSM_API_END
}

}  // extern "C"
