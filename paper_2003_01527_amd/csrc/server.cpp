// Serving engine: a resident graph, an arrival queue, memory-based admission
// and worker threads that each match one batch at a time on their own stream
// and workspace, so batches of different workers overlap on the device and
// queries that arrive while others run join the next batch a worker forms.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

#include "gsm_internal.h"

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  uint64_t ticket;
  gsm_query q;       // private copy
  gsm::RootSlice slice;
  uint64_t reserve;  // admitted bytes
  gsm_result res;
  bool done = false;
};

}  // namespace

struct gsm_server {
  gsm_graph *g = nullptr;
  gsm_server_opts o;
  std::vector<uint64_t> label_deg;  // sum of degrees of the vertices of each label
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> pending;
  std::unordered_map<uint64_t, Request *> all;
  uint64_t next_ticket = 1;
  uint64_t reserved = 0;
  int active = 0;
  bool stopping = false;
  std::vector<std::thread> workers;
  std::string worker_error;

  // Frontier estimate of a query: the first level's (row, neighbour) pairs
  // are at most the degree total of its first vertex's label class; each
  // becomes at most one row of the second level.
  uint64_t estimate(const gsm_query &q) const {
    const gsm::Plan p = gsm::make_plan(*g, q);
    const int32_t l0 = p.qlab[p.order[0]];
    const uint64_t pairs = (l0 >= 0 && (size_t)l0 < label_deg.size()) ? label_deg[l0] : 0;
    const uint64_t row2 = 4 * 2 + 23;
    // the smallest budget either driver accepts for this query alone (a batch
    // of one, or the single-query path a heavy query is moved to)
    const uint64_t floor = std::max(gsm::min_budget_bytes_batch(*g, 1, p.q), gsm::min_budget_bytes_single(g->n, p.q));
    uint64_t est = pairs * row2 + floor;
    est = std::max<uint64_t>(est, floor + (uint64_t(64) << 20));
    return std::max(floor, std::min<uint64_t>(est, o.per_query_budget));
  }

  // the oldest waiting request fits now (caller holds mu)
  bool admissible() const {
    if (pending.empty() || active >= o.max_active) return false;
    const Request *r = pending.front();
    return reserved + r->reserve <= o.arena_bytes || reserved == 0;  // an oversize query runs alone
  }

  void worker_main(int wid) {
    hipStream_t stream = nullptr;
    gsm::Workspace *ws = nullptr;
    try {
      GSM_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
      ws = new gsm::Workspace();
    } catch (const gsm::Error &e) {
      std::lock_guard<std::mutex> lk(mu);
      worker_error = e.msg;
      return;
    }
    for (;;) {
      std::vector<Request *> batch;
      uint64_t budget = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        // sleep until the oldest waiting request can be admitted (it fits the
        // free arena, or nothing is running so it may run alone, and a slot
        // is free) or the server stops; a finishing batch wakes the workers
        cv_work.wait(lk, [&] { return (stopping && pending.empty()) || admissible(); });
        if (pending.empty() && stopping) break;
        // admit the oldest requests that fit the free arena
        while (!pending.empty() && (int)batch.size() < o.max_batch && admissible()) {
          Request *r = pending.front();
          pending.pop_front();
          reserved += r->reserve;
          budget += r->reserve;
          ++active;
          r->res.t_admit_ns = now_ns();
          batch.push_back(r);
        }
      }
      std::vector<const gsm_query *> qs;
      std::vector<gsm::RootSlice> slices;
      for (Request *r : batch) {
        qs.push_back(&r->q);
        slices.push_back(r->slice);
      }
      std::vector<uint64_t> counts(batch.size(), 0);
      gsm_status st = GSM_OK;
      std::string err;
      try {
        gsm_match_opts mo;
        gsm_match_opts_init(&mo);
        mo.hip_stream = stream;
        mo.memory_budget_bytes = budget;
        mo.wg_size = o.wg_size;
        mo.tile_items = o.tile_items;
        mo.batch_heavy_pairs = o.batch_heavy_pairs;
        gsm::match_batch_on(*g, qs.data(), (int)qs.size(), mo, *ws, counts.data(), nullptr, nullptr,
                            slices.data());
      } catch (const gsm::Error &e) {
        st = e.status;
        err = e.msg;
      } catch (const std::bad_alloc &) {
        st = GSM_E_OOM;
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        const uint64_t t = now_ns();
        for (size_t k = 0; k < batch.size(); ++k) {
          Request *r = batch[k];
          r->res.status = st;
          r->res.count = counts[k];
          r->res.t_done_ns = t;
          r->res.batch_size = (int32_t)batch.size();
          r->done = true;
          reserved -= r->reserve;
          --active;
        }
        if (st != GSM_OK && worker_error.empty()) worker_error = err;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    delete ws;
    (void)hipStreamDestroy(stream);
    (void)wid;
  }
};

namespace gsm {

uint64_t min_budget_bytes_batch(const gsm_graph &g, int nq, int q) {
  // first frontier of nq queries (at most n rows each) and one row per level
  const uint64_t n = (uint64_t)std::max<int64_t>(g.n, 1);
  const uint64_t first = n * (uint64_t)nq;
  uint64_t b = first * (4 + 2 + 4 + 8 + 1) + (first + 1) * 8 + 4096 + 64;
  for (int i = 2; i < q; ++i) b += 4 * (uint64_t)i + 23;
  return b;
}

}  // namespace gsm

extern "C" {

uint64_t gsm_now_ns(void) { return now_ns(); }

void gsm_server_opts_init(gsm_server_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(*o);
}

gsm_status gsm_server_create(gsm_graph_t g, const gsm_server_opts *opts, gsm_server_t *out) {
  if (!g || !out) {
    gsm::set_error("gsm_server_create: NULL argument");
    return GSM_E_INVALID_ARG;
  }
  auto srv = new gsm_server();
  srv->g = g;
  gsm_server_opts_init(&srv->o);
  if (opts) std::memcpy(&srv->o, opts, std::min<size_t>(sizeof(srv->o), opts->struct_size ? opts->struct_size : sizeof(srv->o)));
  gsm_server_opts &o = srv->o;
  if (!o.arena_bytes) o.arena_bytes = uint64_t(16) << 30;
  if (!o.per_query_budget) o.per_query_budget = uint64_t(4) << 30;
  if (o.workers <= 0) o.workers = 2;
  if (o.max_batch <= 0) o.max_batch = 64;
  if (o.max_active <= 0) o.max_active = 1024;
  if (o.workers > 16) o.workers = 16;
  // per-label degree totals for the admission estimate
  srv->label_deg.assign(g->label_count.size(), 0);
  {
    std::vector<int64_t> rp(g->n + 1);
    std::vector<int32_t> lab;
    if (hipMemcpy(rp.data(), g->rp, (g->n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess) {
      delete srv;
      gsm::set_error("gsm_server_create: reading the graph failed");
      return GSM_E_DEVICE;
    }
    if (g->lab) {
      lab.resize(g->n);
      if (g->n && hipMemcpy(lab.data(), g->lab, g->n * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) {
        delete srv;
        gsm::set_error("gsm_server_create: reading the labels failed");
        return GSM_E_DEVICE;
      }
    }
    for (int64_t v = 0; v < g->n; ++v) srv->label_deg[lab.empty() ? 0 : lab[v]] += (uint64_t)(rp[v + 1] - rp[v]);
  }
  for (int w = 0; w < o.workers; ++w) srv->workers.emplace_back([srv, w] { srv->worker_main(w); });
  *out = srv;
  return GSM_OK;
}

gsm_status gsm_server_submit_slice(gsm_server_t srv, gsm_query_t qh, int32_t root_qvertex, uint32_t root_mod,
                                   uint32_t root_rem, uint64_t *ticket) {
  if (!srv || !qh || !ticket) {
    gsm::set_error("gsm_server_submit: NULL argument");
    return GSM_E_INVALID_ARG;
  }
  if (qh->has_elab) {
    gsm::set_error("gsm_server_submit: edge-labelled queries are matched one at a time (gsm_match)");
    return GSM_E_UNSUPPORTED;
  }
  if (root_qvertex >= 0 && (root_qvertex >= qh->q || root_mod == 0 || root_rem >= root_mod)) {
    gsm::set_error("gsm_server_submit_slice: root_qvertex < q and root_rem < root_mod required");
    return GSM_E_INVALID_ARG;
  }
  auto r = new Request();
  r->q = *qh;
  if (root_qvertex >= 0) r->slice = gsm::RootSlice{root_qvertex, root_mod, root_rem};
  std::memset(&r->res, 0, sizeof(r->res));
  r->res.t_submit_ns = now_ns();
  try {
    r->reserve = srv->estimate(r->q);
  } catch (const gsm::Error &e) {
    delete r;
    gsm::set_error(e.msg);
    return e.status;
  }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) {
      delete r;
      gsm::set_error("server is stopping");
      return GSM_E_INVALID_ARG;
    }
    r->ticket = srv->next_ticket++;
    srv->all[r->ticket] = r;
    srv->pending.push_back(r);
    *ticket = r->ticket;
  }
  srv->cv_work.notify_one();
  return GSM_OK;
}

gsm_status gsm_server_submit(gsm_server_t srv, gsm_query_t qh, uint64_t *ticket) {
  return gsm_server_submit_slice(srv, qh, -1, 0, 0, ticket);
}

gsm_status gsm_server_wait(gsm_server_t srv, uint64_t ticket, int32_t timeout_ms, gsm_result *out) {
  if (!srv || !out) {
    gsm::set_error("gsm_server_wait: NULL argument");
    return GSM_E_INVALID_ARG;
  }
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->all.find(ticket);
  if (it == srv->all.end()) {
    gsm::set_error("unknown ticket");
    return GSM_E_INVALID_ARG;
  }
  Request *r = it->second;
  auto pred = [&] { return r->done; };
  if (timeout_ms < 0)
    srv->cv_done.wait(lk, pred);
  else if (!srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) {
    gsm::set_error("ticket not finished");
    return GSM_E_TIMEOUT;
  }
  *out = r->res;
  srv->all.erase(it);
  delete r;
  if (out->status != GSM_OK) gsm::set_error(srv->worker_error);
  return out->status;
}

void gsm_server_destroy(gsm_server_t srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
  }
  srv->cv_work.notify_all();
  for (auto &t : srv->workers) t.join();
  for (auto &kv : srv->all) delete kv.second;
  delete srv;
}

}  // extern "C"
