// Serving engine: a resident graph, an arrival queue, memory-based admission
// and worker threads, each with its own HIP stream.  A worker keeps several
// batched runs in flight and advances them one step at a time (a level's scan
// or one chunk's expansion), taking newly arrived queries into a new run
// between any two steps: a query that arrives while others are on the GPU
// starts at the next step instead of after the running batch.  Runs of
// different workers overlap on the device.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
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

// One batched run in a worker: queries of one size (or one query moved out
// of a shared run), its workspace and the events that time it on the device.
struct Run {
  std::vector<Request *> reqs;
  std::vector<const gsm_query *> qs;
  std::vector<gsm::RootSlice> slices;
  std::unique_ptr<gsm::Workspace> ws;
  std::unique_ptr<gsm::StepRun> br;
  uint64_t budget = 0;
  bool solo = false;
  hipEvent_t ev_start = nullptr, ev_end = nullptr;
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
  hipEvent_t ev_ref = nullptr;  // device-time origin of gsm_result's device times

  // Frontier estimate of a query: the first level's (row, neighbour) pairs
  // are at most the degree total of its first vertex's label class; each
  // becomes at most one row of the second level.
  uint64_t estimate(const gsm_query &q) const {
    const gsm::Plan p = gsm::make_plan(*g, q);
    const int32_t l0 = p.qlab[p.order[0]];
    const uint64_t pairs = (l0 >= 0 && (size_t)l0 < label_deg.size()) ? label_deg[l0] : 0;
    const uint64_t row2 = 4 * 2 + 23;
    // the smallest budget the batched driver accepts for this query alone
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

  struct Worker {
    gsm_server *srv;
    int id;
    hipStream_t stream = nullptr;
    std::vector<std::unique_ptr<Run>> runs;
    std::vector<std::unique_ptr<gsm::Workspace>> ws_pool;
    std::vector<hipEvent_t> ev_pool;

    hipEvent_t event() {
      if (!ev_pool.empty()) {
        hipEvent_t e = ev_pool.back();
        ev_pool.pop_back();
        return e;
      }
      hipEvent_t e;
      GSM_HIP(hipEventCreate(&e));
      return e;
    }

    std::unique_ptr<gsm::Workspace> workspace() {
      if (!ws_pool.empty()) {
        auto w = std::move(ws_pool.back());
        ws_pool.pop_back();
        return w;
      }
      return std::unique_ptr<gsm::Workspace>(new gsm::Workspace());
    }

    gsm_match_opts match_opts(uint64_t budget) const {
      gsm_match_opts mo;
      gsm_match_opts_init(&mo);
      mo.hip_stream = stream;
      mo.memory_budget_bytes = budget;
      mo.wg_size = srv->o.wg_size;
      mo.tile_items = srv->o.tile_items;
      return mo;
    }

    // Starts a run over reqs (first frontier launched); on an error the
    // requests are finished with it.
    void start_run(std::vector<Request *> reqs, bool solo) {
      std::unique_ptr<Run> r(new Run());
      r->reqs = std::move(reqs);
      r->solo = solo;
      for (Request *q : r->reqs) {
        r->qs.push_back(&q->q);
        r->slices.push_back(q->slice);
        r->budget += q->reserve;
      }
      try {
        r->ws = workspace();
        r->ev_start = event();
        r->ev_end = event();
        GSM_HIP(hipEventRecord(r->ev_start, stream));
        if (r->qs.size() == 1) {
          // one query: the query-uniform kernels are faster than shared launches
          r->br = gsm::make_single_count_run(*srv->g, *r->qs[0], match_opts(r->budget), *r->ws, r->slices[0]);
        } else {
          const uint64_t heavy = srv->o.batch_heavy_pairs ? srv->o.batch_heavy_pairs : (uint64_t(1) << 18);
          const uint64_t evict = heavy == UINT64_MAX ? 0 : heavy;
          r->br.reset(new gsm::BatchRun(*srv->g, r->qs.data(), (int)r->qs.size(), match_opts(r->budget), *r->ws,
                                        r->slices.data(), evict));
        }
        runs.push_back(std::move(r));
      } catch (const gsm::Error &e) {
        complete(*r, e.status, e.msg, nullptr, nullptr);
        recycle(*r);
      } catch (const std::bad_alloc &) {
        complete(*r, GSM_E_OOM, "host allocation failed", nullptr, nullptr);
        recycle(*r);
      }
    }

    void recycle(Run &r) {
      (void)hipStreamSynchronize(stream);  // no launch of this run may still use its workspace
      r.br.reset();
      if (r.ws) ws_pool.push_back(std::move(r.ws));
      if (r.ev_start) ev_pool.push_back(r.ev_start);
      if (r.ev_end) ev_pool.push_back(r.ev_end);
      r.ev_start = r.ev_end = nullptr;
    }

    // Posts the results of the requests of r that are finished (all but
    // those in moved_out, which continue in runs of their own).
    void complete(Run &r, gsm_status st, const std::string &err, const uint64_t *counts,
                  const std::vector<uint8_t> *moved_out) {
      double t0 = 0, t1 = 0;
      if (st == GSM_OK && r.ev_start && r.ev_end) {
        float a = 0, b = 0;
        if (hipEventElapsedTime(&a, srv->ev_ref, r.ev_start) == hipSuccess &&
            hipEventElapsedTime(&b, srv->ev_ref, r.ev_end) == hipSuccess) {
          t0 = a;
          t1 = b;
        }
      }
      {
        std::lock_guard<std::mutex> lk(srv->mu);
        const uint64_t t = now_ns();
        for (size_t k = 0; k < r.reqs.size(); ++k) {
          if (moved_out && k < moved_out->size() && (*moved_out)[k]) continue;
          Request *q = r.reqs[k];
          q->res.status = st;
          q->res.count = counts ? counts[k] : 0;
          q->res.t_done_ns = t;
          q->res.batch_size = (int32_t)r.reqs.size();
          q->res.worker = id;
          q->res.dev_start_ms = t0;
          q->res.dev_end_ms = t1;
          q->done = true;
          srv->reserved -= q->reserve;
          --srv->active;
        }
        if (st != GSM_OK && srv->worker_error.empty()) srv->worker_error = err;
      }
      srv->cv_done.notify_all();
      srv->cv_work.notify_all();
    }

    // Advances run k by one step; when it has finished, posts its results,
    // starts a run of its own for every query it moved out and returns true.
    bool advance(size_t k) {
      Run &r = *runs[k];
      bool more = false;
      gsm_status st = GSM_OK;
      std::string err;
      try {
        more = r.br->step();
      } catch (const gsm::Error &e) {
        st = e.status;
        err = e.msg;
      } catch (const std::bad_alloc &) {
        st = GSM_E_OOM;
        err = "host allocation failed";
      }
      if (more && st == GSM_OK) return false;
      std::vector<uint64_t> counts(r.reqs.size(), 0);
      std::vector<uint8_t> moved;
      if (st == GSM_OK) {
        try {
          GSM_HIP(hipEventRecord(r.ev_end, stream));
          r.br->finish(counts.data(), moved);
        } catch (const gsm::Error &e) {
          st = e.status;
          err = e.msg;
          moved.clear();
        }
      }
      complete(r, st, err, counts.data(), &moved);
      std::vector<Request *> alone;
      for (size_t j = 0; j < moved.size(); ++j)
        if (moved[j]) alone.push_back(r.reqs[j]);
      recycle(r);
      runs.erase(runs.begin() + k);
      for (Request *q : alone) start_run({q}, true);
      return true;
    }

    void main() {
      try {
        GSM_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
      } catch (const gsm::Error &e) {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->worker_error = e.msg;
        return;
      }
      size_t next = 0;
      for (;;) {
        std::vector<Request *> admitted;
        {
          std::unique_lock<std::mutex> lk(srv->mu);
          // idle: sleep until the oldest waiting request can be admitted (it
          // fits the free arena, or nothing runs so it may run alone, and a
          // slot is free) or the server stops; a finishing run wakes workers
          if (runs.empty())
            srv->cv_work.wait(lk, [&] { return (srv->stopping && srv->pending.empty()) || srv->admissible(); });
          if (runs.empty() && srv->pending.empty() && srv->stopping) break;
          // between two steps: admit the oldest requests that fit
          while ((int)admitted.size() < srv->o.max_batch && srv->admissible()) {
            Request *r = srv->pending.front();
            srv->pending.pop_front();
            srv->reserved += r->reserve;
            ++srv->active;
            r->res.t_admit_ns = now_ns();
            admitted.push_back(r);
          }
        }
        // the batched kernels share launches among queries of one size
        std::map<int, std::vector<Request *>> by_size;
        for (Request *r : admitted) by_size[r->q.q].push_back(r);
        for (auto &kv : by_size) start_run(std::move(kv.second), false);
        if (runs.empty()) continue;
        next %= runs.size();
        if (!advance(next)) ++next;  // a finished run was erased: the next one moved to its place
      }
      for (auto &w : ws_pool) w.reset();
      for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
      (void)hipStreamDestroy(stream);
    }
  };
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
  if (hipEventCreate(&srv->ev_ref) != hipSuccess || hipEventRecord(srv->ev_ref, nullptr) != hipSuccess ||
      hipEventSynchronize(srv->ev_ref) != hipSuccess) {
    if (srv->ev_ref) (void)hipEventDestroy(srv->ev_ref);
    delete srv;
    gsm::set_error("gsm_server_create: device timing event failed");
    return GSM_E_DEVICE;
  }
  for (int w = 0; w < o.workers; ++w)
    srv->workers.emplace_back([srv, w] {
      gsm_server::Worker wk{srv, w};
      wk.main();
    });
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
  if (srv->ev_ref) (void)hipEventDestroy(srv->ev_ref);
  delete srv;
}

}  // extern "C"
