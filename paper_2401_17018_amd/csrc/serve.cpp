// Served update stream with continuous batching.
//
// The paper keeps host-side preparation of the next batch off the critical
// path of the GPU search (its asynchronous pipeline, Sec. IV-A).  Here a
// server owns one worker thread per context.  Callers submit update
// requests from any thread; the worker turns the queue into device batches:
// each batch takes queued requests in submission order while they fit the
// admission limit, and closes before a request that would insert an edge
// some request of the batch deletes (or delete one it inserts), because
// such a pair must be applied in order.  Duplicates across requests
// collapse as they would in sequence, so after every batch the graph equals
// the graph that applying its requests one by one would give, and the
// batch's net result (|+| - |-| per query) equals the sum of theirs.
// Batches are applied and committed in order; a request completes when its
// batch is committed.  With TUPLES, admission also bounds a batch by its
// estimated match-buffer use (a moving estimate of tuple records per
// update), and each batch's records are copied out after its commit.  In
// every mode a work budget (max_batch_ms) can bound a batch by its
// estimated device time, from a moving estimate of device ms per update, so
// that a batch of many requests does not hold the ones queued behind it for
// longer than the budget.  On an edge-labelled graph requests name triples
// (u, v, label): a request that names a pair of the batch under another
// label, or with the other op, also closes the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/gamma.h"
#include "ctx_access.h"

namespace {

struct Request {
  uint64_t ticket;
  double t_submit;
  std::vector<uint32_t> src, dst;
  std::vector<uint8_t> op;
  std::vector<uint32_t> el;  // edge labels (empty: all 0)
};

struct BatchRecord {
  gamma_serve_batch info;
  std::vector<gamma_query_result> q;
  std::vector<uint32_t> tup, meta, ord;  // tuple records (TUPLES)
  uint32_t width = 0;
};

}  // namespace

struct gamma_server {
  gamma_ctx* ctx = nullptr;
  gamma_serve_options opt{};
  uint32_t n = 0, n_el = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> queue;
  std::deque<gamma_request_result> done;  // completed, not yet polled (ticket order)
  std::vector<BatchRecord> batches;
  uint64_t next_ticket = 0, n_committed = 0;
  bool stop = false;
  bool tuples = false;
  double budget = 0;          // tuple records a batch may be estimated to fill
  double per_update = -1.0;   // estimated tuple records per update (< 0: no batch seen yet)
  double ms_per_update = -1.0;  // estimated device ms per update (< 0: no batch seen yet)
  std::thread worker;
  std::chrono::steady_clock::time_point t0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }

  static uint32_t tag(const Request& r, size_t i) {
    return ((r.el.empty() ? 0u : r.el[i]) << 1) | (r.op[i] ? 1u : 0u);
  }

  void run() {
    std::vector<uint32_t> src, dst, el;
    std::vector<uint8_t> op;
    std::unordered_map<uint64_t, uint32_t> seen;  // pair -> label << 1 | op
    for (;;) {
      std::vector<Request> take;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || !queue.empty(); });
        if (queue.empty()) break;  // stop requested and nothing left
        // admission, in submission order
        size_t nupd = 0;
        seen.clear();
        while (!queue.empty()) {
          Request& r = queue.front();
          if (!take.empty()) {
            if (opt.coalesce == 2 || nupd + r.op.size() > opt.max_batch_updates) break;
            // admission by estimated match-buffer memory
            if (tuples && (per_update < 0 || (double)(nupd + r.op.size()) * per_update > budget)) break;
            // admission by estimated device time
            if (opt.max_batch_ms && ms_per_update >= 0 &&
                (double)(nupd + r.op.size()) * ms_per_update > (double)opt.max_batch_ms)
              break;
            bool conflict = false;
            for (size_t i = 0; i < r.op.size() && !conflict; ++i) {
              const uint64_t a = std::min(r.src[i], r.dst[i]), b = std::max(r.src[i], r.dst[i]);
              auto it = seen.find((a << 32) | b);
              conflict = it != seen.end() && it->second != tag(r, i);
            }
            if (conflict) break;
          }
          for (size_t i = 0; i < r.op.size(); ++i) {
            const uint64_t a = std::min(r.src[i], r.dst[i]), b = std::max(r.src[i], r.dst[i]);
            seen[(a << 32) | b] = tag(r, i);
          }
          nupd += r.op.size();
          take.push_back(std::move(r));
          queue.pop_front();
        }
      }
      // merge the admitted requests into one batch and apply it
      src.clear();
      dst.clear();
      op.clear();
      el.clear();
      for (auto& r : take) {
        src.insert(src.end(), r.src.begin(), r.src.end());
        dst.insert(dst.end(), r.dst.begin(), r.dst.end());
        op.insert(op.end(), r.op.begin(), r.op.end());
        if (r.el.empty())
          el.insert(el.end(), r.op.size(), 0u);
        else
          el.insert(el.end(), r.el.begin(), r.el.end());
      }
      const double t_start = now_ms();
      gamma_batch_result res;
      std::memset(&res, 0, sizeof(res));
      const gamma_status st = gamma_apply_batch_el(ctx, (uint32_t)op.size(), src.data(), dst.data(), op.data(),
                                                   n_el > 1 ? el.data() : nullptr, GAMMA_MEM_HOST, opt.flags, &res);
      const double t_done = now_ms();
      BatchRecord rec;
      std::memset(&rec.info, 0, sizeof(rec.info));
      rec.info.first_ticket = take.front().ticket;
      rec.info.n_requests = (uint32_t)take.size();
      rec.info.n_updates = (uint32_t)op.size();
      rec.info.status = st;
      rec.info.t_start_ms = t_start;
      rec.info.t_done_ms = t_done;
      if (st >= 0) {
        rec.info.n_canonical = res.n_canonical;
        rec.info.ms_device = res.stats.ms_total;
        const double mrate = (double)res.stats.ms_total / std::max<double>(op.size(), 1.0);
        ms_per_update = ms_per_update < 0 ? mrate : 0.5 * ms_per_update + 0.5 * mrate;
        rec.q.assign(res.queries, res.queries + res.n_queries);
        if (tuples) {
          const uint64_t nt = res.n_tuples;
          rec.width = res.tuple_width;
          rec.info.n_tuples = nt;
          rec.info.n_tuples_found = res.n_tuples_found;
          rec.tup.resize(std::max<uint64_t>(nt * rec.width, 1));
          rec.meta.resize(std::max<uint64_t>(nt, 1));
          if (opt.flags & GAMMA_F_SEED_ATTR) rec.ord.resize(std::max<uint64_t>(nt, 1));
          if (nt)
            gamma_copy_tuples(ctx, rec.tup.data(), rec.meta.data(), rec.ord.empty() ? nullptr : rec.ord.data(), nt,
                              GAMMA_MEM_HOST);
          const double rate = (double)res.n_tuples_found / std::max<double>(op.size(), 1.0);
          per_update = per_update < 0 ? rate : 0.5 * per_update + 0.5 * rate;
        }
      }
      std::lock_guard<std::mutex> lk(mu);
      rec.info.batch = batches.size();
      for (auto& r : take) {
        gamma_request_result d;
        std::memset(&d, 0, sizeof(d));
        d.ticket = r.ticket;
        d.batch = rec.info.batch;
        d.t_submit_ms = r.t_submit;
        d.t_done_ms = t_done;
        d.n_updates = (uint32_t)r.op.size();
        d.status = st;
        done.push_back(d);
      }
      batches.push_back(std::move(rec));
      n_committed += take.size();
      cv_done.notify_all();
    }
  }
};

extern "C" {

gamma_status gamma_serve_create(gamma_ctx* ctx, const gamma_serve_options* opt, gamma_server** out) {
  if (!ctx || !out) return GAMMA_EINVAL;
  *out = nullptr;
  gamma_serve_options o{};
  if (opt) o = *opt;
  if (o.max_batch_updates == 0) o.max_batch_updates = 1u << 17;
  if (o.coalesce == 0) o.coalesce = 1;
  if (o.tuple_fill_pct == 0) o.tuple_fill_pct = 50;
  if (o.max_batch_updates > (1u << 20) || (o.coalesce != 1 && o.coalesce != 2) || o.tuple_fill_pct > 100 ||
      (o.flags & (GAMMA_F_DRY_RUN | GAMMA_F_CANONICAL)))
    return GAMMA_EINVAL;
  const uint64_t tcap = gm::ctx_tuple_capacity(ctx);
  if ((o.flags & GAMMA_F_TUPLES) && tcap == 0) return GAMMA_EINVAL;
  uint32_t n = 0, n_el = 1;
  if (!gm::ctx_has_graph(ctx, &n, &n_el)) return GAMMA_ESTATE;
  gamma_server* s = new (std::nothrow) gamma_server();
  if (!s) return GAMMA_ENOMEM;
  s->ctx = ctx;
  s->opt = o;
  s->n = n;
  s->n_el = n_el;
  s->tuples = (o.flags & GAMMA_F_TUPLES) != 0;
  s->budget = (double)tcap * o.tuple_fill_pct / 100.0;
  s->t0 = std::chrono::steady_clock::now();
  try {
    s->worker = std::thread([s] { s->run(); });
  } catch (...) {
    delete s;
    return GAMMA_ENOMEM;
  }
  *out = s;
  return GAMMA_OK;
}

gamma_status gamma_serve_submit_el(gamma_server* s, uint32_t n_upd, const uint32_t* src, const uint32_t* dst,
                                   const uint8_t* op, const uint32_t* elab, uint64_t* ticket) {
  if (!s) return GAMMA_EINVAL;
  if (n_upd == 0 || n_upd > s->opt.max_batch_updates) return GAMMA_EINVAL;
  const gamma_status v = gamma_validate_batch(s->n, n_upd, src, dst, op);
  if (v != GAMMA_OK) return v;
  Request r;
  r.src.assign(src, src + n_upd);
  r.dst.assign(dst, dst + n_upd);
  r.op.assign(op, op + n_upd);
  if (elab) {
    r.el.assign(elab, elab + n_upd);
    // labels in range; one pair twice must be the same triple (with the same op)
    std::unordered_map<uint64_t, uint32_t> pairs;
    for (uint32_t i = 0; i < n_upd; ++i) {
      if (r.el[i] >= s->n_el) return GAMMA_EINVAL;
      const uint64_t a = std::min(src[i], dst[i]), b = std::max(src[i], dst[i]);
      auto ins = pairs.emplace((a << 32) | b, gamma_server::tag(r, i));
      if (!ins.second && ins.first->second != gamma_server::tag(r, i)) return GAMMA_ECONFLICT;
    }
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return GAMMA_ESTATE;
  r.ticket = s->next_ticket++;
  r.t_submit = s->now_ms();
  if (ticket) *ticket = r.ticket;
  s->queue.push_back(std::move(r));
  s->cv_work.notify_one();
  return GAMMA_OK;
}

gamma_status gamma_serve_submit(gamma_server* s, uint32_t n_upd, const uint32_t* src, const uint32_t* dst,
                                const uint8_t* op, uint64_t* ticket) {
  return gamma_serve_submit_el(s, n_upd, src, dst, op, nullptr, ticket);
}

gamma_status gamma_serve_poll(gamma_server* s, gamma_request_result* out, uint32_t max, uint32_t* n_out) {
  if (!s || !n_out || (max && !out)) return GAMMA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  uint32_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n_out = k;
  return GAMMA_OK;
}

gamma_status gamma_serve_drain(gamma_server* s) {
  if (!s) return GAMMA_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->n_committed == s->next_ticket; });
  return GAMMA_OK;
}

gamma_status gamma_serve_counts(gamma_server* s, uint64_t* submitted, uint64_t* committed, uint64_t* batches) {
  if (!s) return GAMMA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (submitted) *submitted = s->next_ticket;
  if (committed) *committed = s->n_committed;
  if (batches) *batches = s->batches.size();
  return GAMMA_OK;
}

gamma_status gamma_serve_get_batch(gamma_server* s, uint64_t batch, gamma_serve_batch* info,
                                   gamma_query_result* queries, uint32_t max_queries) {
  if (!s || !info) return GAMMA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (batch >= s->batches.size()) return GAMMA_EINVAL;
  const BatchRecord& r = s->batches[batch];
  *info = r.info;
  info->n_queries = (uint32_t)r.q.size();
  if (queries)
    for (uint32_t i = 0; i < std::min<uint32_t>(max_queries, (uint32_t)r.q.size()); ++i) queries[i] = r.q[i];
  return GAMMA_OK;
}

gamma_status gamma_serve_get_tuples(gamma_server* s, uint64_t batch, uint32_t* tuples, uint32_t* meta, uint32_t* ord,
                                    uint64_t max_records, uint64_t* n_records, uint32_t* width) {
  if (!s) return GAMMA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (batch >= s->batches.size()) return GAMMA_EINVAL;
  if (!s->tuples) return GAMMA_ESTATE;
  const BatchRecord& r = s->batches[batch];
  const uint64_t nt = r.info.n_tuples, k = std::min(nt, max_records);
  if (n_records) *n_records = nt;
  if (width) *width = r.width;
  if (tuples && k) std::memcpy(tuples, r.tup.data(), k * r.width * 4);
  if (meta && k) std::memcpy(meta, r.meta.data(), k * 4);
  if (ord && k && !r.ord.empty()) std::memcpy(ord, r.ord.data(), k * 4);
  return GAMMA_OK;
}

gamma_status gamma_serve_destroy(gamma_server* s) {
  if (!s) return GAMMA_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  delete s;
  return GAMMA_OK;
}

}  // extern "C"
