// Serving loop: resident graphs, each with its own HIP stream and worker
// thread; update batches are submitted asynchronously and answered through
// tickets.  Requests for different graphs run at the same time on their own
// streams (their kernels overlap on the device); requests for one graph are
// applied in submission order (each result is the counts after that batch).
// Continuous batching: a worker that becomes free takes every queued batch
// of its graph, up to three, into one counting pass that keeps each
// intermediate version.  Admission by memory: a graph is admitted only if its
// estimated footprint fits the free HBM (minus a reserve); batches start only
// while the bytes of the batches in flight stay within the budget.
#include "../../include/graphlet4.h"
#include "gc_kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

using clk = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  int32_t graph = 0;
  std::vector<int32_t> iu, iv, du, dv;
  clk::time_point t_submit, t_start, t_done;
  bool done = false;
  int rc = 0;
  std::string err;
  int64_t counts[11] = {};
  gc_batch_stats stats{};
  int64_t bytes = 0;
};

struct Slot {
  gc_graph* g = nullptr;
  int64_t n = 0;
  int64_t footprint = 0;
  std::deque<std::shared_ptr<Request>> q;
  std::condition_variable cv;
  std::thread th;
  bool stop = false;
};

int fail(int code, const char* msg) {
  gc_set_error(msg);
  return code;
}

bool ids_ok(const std::vector<int32_t>& a, int64_t n) {
  for (int32_t x : a)
    if (x < 0 || x >= n) return false;
  return true;
}

constexpr int kPassMax = 3;  // batches per counting pass

}  // namespace

struct gc_server {
  gc_server_opts opts{};
  std::mutex mu;
  std::condition_variable cv_done, cv_mem;
  std::vector<std::unique_ptr<Slot>> slots;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  int64_t inflight = 0;
  int64_t graph_bytes = 0;
  bool stopping = false;

  int64_t free_hbm() {
    if (opts.hbm_budget_bytes > 0) return opts.hbm_budget_bytes - graph_bytes;
    size_t fr = 0, tot = 0;
    if (hipSetDevice(opts.device) != hipSuccess || hipMemGetInfo(&fr, &tot) != hipSuccess) return 0;
    return (int64_t)fr;
  }

  void worker(Slot* sl) {
    (void)hipSetDevice(opts.device);
    while (true) {
      std::vector<std::shared_ptr<Request>> grp;
      {
        std::unique_lock<std::mutex> lk(mu);
        sl->cv.wait(lk, [&] { return sl->stop || !sl->q.empty(); });
        if (sl->q.empty()) return;
        std::shared_ptr<Request> r = sl->q.front();
        sl->q.pop_front();
        // memory admission of the batch (the first one always runs)
        cv_mem.wait(lk, [&] { return inflight == 0 || inflight + r->bytes <= opts.batch_budget_bytes; });
        inflight += r->bytes;
        grp.push_back(r);
        // batches that queued meanwhile join the pass while the budget allows
        while ((int)grp.size() < kPassMax && !sl->q.empty() &&
               inflight + sl->q.front()->bytes <= opts.batch_budget_bytes) {
          inflight += sl->q.front()->bytes;
          grp.push_back(sl->q.front());
          sl->q.pop_front();
        }
      }
      const auto t_start = clk::now();
      std::vector<std::shared_ptr<Request>> run;
      std::vector<gc_batch_desc> descs;
      for (auto& r : grp) {
        r->t_start = t_start;
        if (!ids_ok(r->iu, sl->n) || !ids_ok(r->iv, sl->n) || !ids_ok(r->du, sl->n) || !ids_ok(r->dv, sl->n)) {
          r->rc = GC_EINVAL;
          r->err = "batch has a vertex id outside [0, n)";
          continue;
        }
        run.push_back(r);
        descs.push_back(gc_batch_desc{r->iu.data(), r->iv.data(), (int64_t)r->iu.size(), r->du.data(),
                                      r->dv.data(), (int64_t)r->du.size()});
      }
      int rc = GC_OK;
      std::string err;
      if (!run.empty()) {
        std::vector<int64_t> cnt(run.size() * 11);
        std::vector<gc_batch_stats> st(run.size());
        rc = gc_apply_batch_seq(sl->g, descs.data(), (int32_t)run.size(), (int64_t(*)[11])cnt.data(), st.data());
        if (rc) err = gc_last_error();
        for (size_t j = 0; j < run.size(); ++j) {
          std::memcpy(run[j]->counts, &cnt[j * 11], sizeof(run[j]->counts));
          run[j]->stats = st[j];
        }
      }
      const auto t_done = clk::now();
      {
        std::lock_guard<std::mutex> lk(mu);
        for (auto& r : run) {
          r->rc = rc;
          if (rc) r->err = err;
        }
        for (auto& r : grp) {
          r->t_done = t_done;
          r->done = true;
          inflight -= r->bytes;
        }
      }
      cv_mem.notify_all();
      cv_done.notify_all();
    }
  }
};

extern "C" {

int gc_server_opts_default(gc_server_opts* o) {
  if (!o) return GC_EINVAL;
  o->device = 0;
  o->max_graphs = 64;
  o->hbm_reserve_bytes = (int64_t)8 << 30;
  o->hbm_budget_bytes = 0;
  o->batch_budget_bytes = (int64_t)4 << 30;
  return GC_OK;
}

int gc_server_create(const gc_server_opts* opts, gc_server** out) {
  if (!out) return fail(GC_EINVAL, "out is NULL");
  gc_server* s = new gc_server();
  if (opts) s->opts = *opts; else gc_server_opts_default(&s->opts);
  if (s->opts.max_graphs < 1) { delete s; return fail(GC_EINVAL, "max_graphs must be >= 1"); }
  *out = s;
  return GC_OK;
}

int gc_server_add_graph(gc_server* s, int64_t n, const int32_t* src, const int32_t* dst, int64_t m,
                        const gc_options* opt, int32_t* graph_id) {
  if (!s || !graph_id) return fail(GC_EINVAL, "NULL argument");
  if (n < 1 || m < 0 || (m > 0 && (!src || !dst))) return fail(GC_EINVAL, "bad graph size or edge arrays");
  gc_options o;
  if (opt) o = *opt; else gc_options_default(&o);
  // footprint from the library's own sizing rules
  int64_t est = 0;
  if (int rc = gc_graph_footprint(n, src, dst, m, &o, &est)) return rc;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if ((int32_t)s->slots.size() >= s->opts.max_graphs) return fail(GC_EBUSY, "server holds max_graphs graphs");
    if (s->free_hbm() - s->opts.hbm_reserve_bytes < est) return fail(GC_ENOMEM, "not enough free HBM to admit the graph");
  }
  o.device = s->opts.device;
  o.stream = nullptr;  // every graph runs on its own stream
  gc_graph* g = nullptr;
  int rc = gc_graph_init(n, src, dst, m, &o, &g, nullptr);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(s->mu);
  auto sl = std::make_unique<Slot>();
  sl->g = g;
  sl->n = n;
  sl->footprint = est;
  s->graph_bytes += est;
  Slot* raw = sl.get();
  sl->th = std::thread([s, raw] { s->worker(raw); });
  *graph_id = (int32_t)s->slots.size();
  s->slots.push_back(std::move(sl));
  return GC_OK;
}

int gc_server_submit(gc_server* s, int32_t graph_id, const gc_batch_desc* b, uint64_t* ticket) {
  if (!s || !b || !ticket) return fail(GC_EINVAL, "NULL argument");
  if (b->n_ins < 0 || b->n_del < 0) return fail(GC_EINVAL, "negative batch size");
  if ((b->n_ins && (!b->ins_src || !b->ins_dst)) || (b->n_del && (!b->del_src || !b->del_dst)))
    return fail(GC_EINVAL, "null batch array");
  auto r = std::make_shared<Request>();
  r->graph = graph_id;
  r->iu.assign(b->ins_src, b->ins_src + b->n_ins);
  r->iv.assign(b->ins_dst, b->ins_dst + b->n_ins);
  r->du.assign(b->del_src, b->del_src + b->n_del);
  r->dv.assign(b->del_dst, b->del_dst + b->n_del);
  r->bytes = 64 * (b->n_ins + b->n_del) + 4096;
  r->t_submit = clk::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (graph_id < 0 || graph_id >= (int32_t)s->slots.size()) return fail(GC_EINVAL, "unknown graph id");
  r->ticket = s->next_ticket++;
  s->reqs[r->ticket] = r;
  s->slots[graph_id]->q.push_back(r);
  s->slots[graph_id]->cv.notify_one();
  *ticket = r->ticket;
  return GC_OK;
}

int gc_server_wait(gc_server* s, uint64_t ticket, int64_t counts[11], gc_batch_stats* stats, double* latency_ms) {
  if (!s) return fail(GC_EINVAL, "NULL server");
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(GC_EINVAL, "unknown ticket");
    r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    s->reqs.erase(it);
  }
  if (r->rc) return fail(r->rc, r->err.c_str());
  if (counts) std::memcpy(counts, r->counts, sizeof(r->counts));
  if (stats) *stats = r->stats;
  if (latency_ms) {
    latency_ms[0] = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    latency_ms[1] = std::chrono::duration<double, std::milli>(r->t_start - r->t_submit).count();
  }
  return GC_OK;
}

int gc_server_counts(gc_server* s, int32_t graph_id, int64_t hi[11], uint64_t lo[11]) {
  if (!s) return fail(GC_EINVAL, "NULL server");
  Slot* sl;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    if (graph_id < 0 || graph_id >= (int32_t)s->slots.size()) return fail(GC_EINVAL, "unknown graph id");
    sl = s->slots[graph_id].get();
    // wait until the graph has no queued or running request
    s->cv_done.wait(lk, [&] {
      if (!sl->q.empty()) return false;
      for (auto& kv : s->reqs)
        if (kv.second->graph == graph_id && !kv.second->done) return false;
      return true;
    });
  }
  return gc_get_counts_exact(sl->g, 0, hi, lo);
}

int gc_server_destroy(gc_server* s) {
  if (!s) return GC_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto& sl : s->slots) { sl->stop = true; sl->cv.notify_all(); }
  }
  for (auto& sl : s->slots)
    if (sl->th.joinable()) sl->th.join();
  for (auto& sl : s->slots) gc_graph_free(sl->g);
  delete s;
  return GC_OK;
}

}  // extern "C"
