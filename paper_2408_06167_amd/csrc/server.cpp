// server.cpp -- continuous-batching identification server.
//
// Galleries and evaluation keys stay resident in HBM.  A worker thread owns
// several lanes (each a context sharing the tables, with its own stream and
// memory pool).  Whenever a lane is free it admits queued requests: the
// request at the head of the queue and every other queued request whose
// gallery has the same shape (d, k, stored limbs) -- whatever gallery it
// targets -- up to a batch limit, as long as the device memory the batch may
// need fits the HBM budget next to the memory the lanes already hold.  The
// admitted requests run as one batch: their queries are expanded together
// (Alg. 1) and Alg. 2 runs over every (request, gallery group) element in
// passes whose launches mix galleries.  Lanes run concurrently on the device,
// so requests arriving while others execute start as soon as a lane and
// memory free up.  Every result is the same exact function of its query and
// gallery whether it ran alone or in a batch.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>

#include "blindmatch_impl.hpp"

using namespace bm;

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct bm_server {
  bm_ctx* ctx = nullptr;
  const bm_evk* evk = nullptr;
  uint64_t budget = 0;
  uint32_t schedule = BM_S2;
  int max_batch = 32;

  struct Gal {
    std::unique_ptr<bm_gallery> g;
    bm_masks* masks = nullptr;       // owned, k > 1 only
    const u64* cmask = nullptr;      // compression mask (context cache), BM_COMPRESS only
  };
  std::vector<Gal> galleries;

  struct Req {
    uint64_t ticket;
    uint32_t gid;
    std::unique_ptr<bm_ct> q;
    double t_submit;
  };
  struct Lane {
    std::unique_ptr<Ctx> c;
    bool busy = false;
    std::vector<Req> reqs;
    std::vector<std::unique_ptr<bm_result>> results;
    uint64_t bytes = 0;
    hipEvent_t done = nullptr;
  };
  std::vector<Lane> lanes;
  std::deque<Req> queue;
  struct Done {
    int status;
    bm_result* r;
  };
  std::map<uint64_t, Done> done;
  std::map<uint64_t, bool> pending;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::thread worker;
  bool stop = false;
  uint64_t next_ticket = 1;
  uint64_t inflight = 0;
  std::vector<double> latencies;
  uint64_t batches = 0, batched = 0;

  bmx::Plan shape(const bm_gallery& g) const { return bmx::plan(ctx->c, schedule, g.k, (int)g.limbs, 0); }
  static bool same_shape(const bm_gallery& a, const bm_gallery& b) {
    return a.d == b.d && a.k == b.k && a.limbs == b.limbs;
  }

  // Device memory a batch of the requests `gids` (galleries of one shape) may
  // allocate: the queries and their expansion, one pass of Alg. 2, the
  // results (and, with compression, the group outputs before it).
  uint64_t estimate(const std::vector<uint32_t>& gids) const {
    const Ctx& c = ctx->c;
    const bm_gallery& g0 = *galleries[gids[0]].g;
    const bmx::Plan p = shape(g0);
    const u64 N = c.N, nq = gids.size(), k = g0.k;
    const u64 l = (u64)p.t, ql = (u64)p.ql;
    const u64 beta = (l + c.alpha - 1) / c.alpha, ext = l + c.K;
    const u64 qbeta = (ql + c.alpha - 1) / c.alpha, qext = ql + c.K;
    u64 elems = 0, outs = 0, pre = 0;
    for (uint32_t gid : gids) {
      const bm_gallery& g = *galleries[gid].g;
      elems += g.groups;
      outs += bmx::out_cts(p, g.groups, g.d, g.k) * 2 * (u64)p.ol * N;
      if (p.comp) pre += g.groups * 2 * (u64)p.rot * N;
    }
    const u64 pass = std::min<u64>((u64)bmx::pass_elems(c), elems);
    const u64 pair_words = (3 + 2 + 2 + 2 + 1 + 2 + 2) * l * N + (beta + 2) * ext * N;
    const u64 q_words = nq * 2 * ql * N;
    const u64 exp_words = k > 1 ? nq * k * (2 * l + 2 * ql + 2 * l) * N + nq * k * (qbeta + 2) * qext * N : 0;
    return 8 * (pass * pair_words + outs + pre + q_words + exp_words);
  }

  uint64_t held() const {
    uint64_t h = 0;
    for (const Lane& lane : lanes) h += lane.c->pool->bytes_held();
    return h;
  }

  void launch(Lane& lane) {
    Ctx& c = *lane.c;
    const int nq = (int)lane.reqs.size();
    const Gal& G0 = galleries[lane.reqs[0].gid];
    const bm_gallery& g0 = *G0.g;
    const size_t N = c.N;
    bmx::BatchPlan bp;
    bp.cls.emplace_back();
    bmx::BatchClass& K = bp.cls.back();
    K.shape = &g0;
    K.s = shape(g0);
    K.masks = G0.masks;
    K.cmask = G0.cmask;
    std::vector<const bm_gallery*> gs(nq);
    bp.out_off.resize(nq);
    bp.scale.resize(nq);
    for (int j = 0; j < nq; ++j) {
      const Req& r = lane.reqs[j];
      const bm_gallery& g = *galleries[r.gid].g;
      gs[j] = &g;
      K.queries.push_back(r.q.get());
      K.pairs.push_back((size_t)j);
      K.qidx.push_back(j);
      const double cu_scale = g.k > 1 ? r.q->scale * K.masks->scale / (double)c.primes[K.s.ql - 1].q : r.q->scale;
      bp.out_off[j] = bp.out_words;
      bp.scale[j] = bmx::result_scale(c, K.s, cu_scale, g.scale);
      bp.out_words += (size_t)bmx::out_cts(K.s, g.groups, g.d, g.k) * 2 * K.s.ol * N;
    }
    DBuf qb(&c, (size_t)nq * 2 * K.s.ql * N);
    bmx::load_queries(c, K, qb.p());
    auto store = std::make_shared<DBuf>(&c, bp.out_words);
    bmx::class_body(c, evk, bp, K, gs.data(), qb.p(), store->p());
    lane.results.clear();
    for (int j = 0; j < nq; ++j) {
      const bm_gallery& g = *gs[j];
      std::unique_ptr<bm_result> r(new bm_result);
      r->ctx = ctx;
      r->d = g.d;
      r->k = g.k;
      r->limbs = (uint32_t)K.s.ol;
      r->groups = bmx::out_cts(K.s, g.groups, g.d, g.k);
      r->packed = K.s.comp ? g.d / g.k : 0;
      r->n_templates = g.n_templates;
      r->scale = bp.scale[j];
      r->store = store;
      r->off = bp.out_off[j];
      lane.results.push_back(std::move(r));
    }
    HIP_OK(dev::event_record(lane.done, c.stream));
  }

  void finish(Lane& lane, int status) {
    const double t = now_ms();
    std::lock_guard<std::mutex> lk(mu);
    for (size_t j = 0; j < lane.reqs.size(); ++j) {
      bm_result* r = status == BM_OK ? lane.results[j].release() : nullptr;
      done[lane.reqs[j].ticket] = Done{status, r};
      pending.erase(lane.reqs[j].ticket);
      if (status == BM_OK) latencies.push_back(t - lane.reqs[j].t_submit);
    }
    batches += 1;
    batched += lane.reqs.size();
    lane.reqs.clear();
    lane.results.clear();
    inflight -= lane.bytes;
    lane.bytes = 0;
    lane.busy = false;
    cv_done.notify_all();
  }

  void fail_now(Req& r, int status) {
    done[r.ticket] = Done{status, nullptr};
    pending.erase(r.ticket);
    cv_done.notify_all();
  }

  void run() {
    for (;;) {
      bool progress = false;
      // completions
      for (Lane& lane : lanes) {
        if (!lane.busy) continue;
        hipError_t e = dev::event_query(lane.done);
        if (e == hipErrorNotReady) continue;
        finish(lane, e == hipSuccess ? BM_OK : BM_EDEVICE);
        progress = true;
      }
      // admissions
      for (Lane& lane : lanes) {
        if (lane.busy) continue;
        std::unique_lock<std::mutex> lk(mu);
        if (queue.empty()) break;
        const bm_gallery& head = *galleries[queue.front().gid].g;
        std::vector<size_t> pick;
        std::vector<uint32_t> gids;
        for (size_t i = 0; i < queue.size() && (int)pick.size() < max_batch; ++i)
          if (same_shape(*galleries[queue[i].gid].g, head)) {
            pick.push_back(i);
            gids.push_back(queue[i].gid);
          }
        // shrink the batch until what it may allocate fits next to the work
        // in flight and next to the memory the lanes hold (results still with
        // their callers included), this lane's cache counted as reusable
        uint64_t need = estimate(gids);
        auto fits = [&] {
          return inflight + need <= budget && held() - lane.c->pool->bytes_cached() + need <= budget;
        };
        while (pick.size() > 1 && !fits()) {
          pick.pop_back();
          gids.pop_back();
          need = estimate(gids);
        }
        // (a request that cannot fit an empty server was refused at submission;
        // otherwise it waits for work in flight to finish and for results to
        // be freed by their callers)
        if (!fits()) break;
        if (held() + need > budget) lane.c->pool->trim();   // give back this idle lane's cache
        lane.reqs.clear();
        for (size_t k = pick.size(); k-- > 0;) {
          lane.reqs.push_back(std::move(queue[pick[k]]));
          queue.erase(queue.begin() + (long)pick[k]);
        }
        std::reverse(lane.reqs.begin(), lane.reqs.end());
        inflight += need;
        lane.bytes = need;
        lane.busy = true;
        lk.unlock();
        try {
          launch(lane);
        } catch (const Error& e) {
          ctx->c.last_error = e.msg;
          finish(lane, e.code);
        }
        progress = true;
      }
      std::unique_lock<std::mutex> lk(mu);
      bool any_busy = false;
      for (Lane& lane : lanes) any_busy |= lane.busy;
      if (stop && queue.empty() && !any_busy) return;
      if (!progress) cv.wait_for(lk, std::chrono::microseconds(any_busy ? 50 : 2000));
    }
  }
};

extern "C" {

int bm_server_create(bm_ctx* ctx, const bm_evk* evk, uint64_t hbm_budget_bytes, uint32_t schedule,
                     bm_server** out) {
  if (!ctx || !evk || !out || hbm_budget_bytes == 0 || evk->ctx != ctx) return BM_EINVAL;
  const uint32_t base = schedule & 0xff;
  if ((base != BM_S1 && base != BM_S2) ||
      (schedule & ~(uint32_t)(0xff | BM_LEVEL_MIN | BM_COMPRESS | BM_HOIST)))
    return BM_EINVAL;
  try {
    std::unique_ptr<bm_server> s(new bm_server);
    s->ctx = ctx;
    s->evk = evk;
    s->budget = hbm_budget_bytes;
    s->schedule = schedule;
    s->lanes.resize(3);
    for (auto& lane : s->lanes) {
      lane.c = ctx->c.make_lane();
      HIP_OK(dev::event_create(&lane.done, false));
    }
    bm_server* raw = s.get();
    s->worker = std::thread([raw] { raw->run(); });
    *out = s.release();
    return BM_OK;
  } catch (const Error& e) {
    ctx->c.last_error = e.msg;
    return e.code;
  }
}

int bm_server_add_gallery(bm_server* s, bm_gallery* g, uint32_t* gallery_id) {
  if (!s || !g || !gallery_id || g->ctx != s->ctx) return BM_EINVAL;
  bm_server::Gal entry;
  try {
    const bmx::Plan p = s->shape(*g);
    if (g->k > 1) entry.masks = bmx_create_masks(s->ctx, g->d, g->k, (uint32_t)p.ql);
    if (p.comp) entry.cmask = bmx_compress_mask(s->ctx, g->d, g->k, (uint32_t)p.rot)->pt.p();
  } catch (const Error& e) {
    s->ctx->c.last_error = e.msg;
    return e.code;
  }
  entry.g.reset(g);
  std::lock_guard<std::mutex> lk(s->mu);
  *gallery_id = (uint32_t)s->galleries.size();
  s->galleries.push_back(std::move(entry));
  return BM_OK;
}

int bm_server_submit(bm_server* s, uint32_t gallery_id, bm_ct* q, uint64_t* ticket) {
  if (!s || !q || !ticket || q->ctx != s->ctx) return BM_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (gallery_id >= s->galleries.size()) return BM_EINVAL;
  const bm_gallery& g = *s->galleries[gallery_id].g;
  if (s->estimate({gallery_id}) > s->budget) return BM_EBUDGET;
  if (q->query_d && q->query_d != g.d) return BM_EDIM;
  const bmx::Plan p = s->shape(g);
  if ((int)q->limbs < p.ql || q->comps != 2) return BM_ELEVEL;
  const bm_masks* m = s->galleries[gallery_id].masks;
  const double cu_scale = g.k > 1 ? q->scale * m->scale / (double)s->ctx->c.primes[p.ql - 1].q : q->scale;
  if (cu_scale != g.scale) return BM_ESCALE;
  bm_server::Req r;
  r.ticket = s->next_ticket++;
  r.gid = gallery_id;
  r.q.reset(q);
  r.t_submit = now_ms();
  *ticket = r.ticket;
  s->pending[r.ticket] = true;
  s->queue.push_back(std::move(r));
  s->cv.notify_all();
  return BM_OK;
}

int bm_server_poll(bm_server* s, uint64_t ticket, bm_result** out) {
  if (!s || !out) return BM_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = nullptr;
  auto it = s->done.find(ticket);
  if (it == s->done.end()) return s->pending.count(ticket) ? BM_OK : BM_EINVAL;
  const int st = it->second.status;
  *out = it->second.r;
  s->done.erase(it);
  return st;
}

int bm_server_drain(bm_server* s) {
  if (!s) return BM_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [s] { return s->pending.empty(); });
  return BM_OK;
}

int bm_server_stats(bm_server* s, uint64_t* completed, double* p50_ms, double* p99_ms, double* mean_batch) {
  if (!s) return BM_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  std::vector<double> v = s->latencies;
  std::sort(v.begin(), v.end());
  auto pct = [&](double p) {
    if (v.empty()) return 0.0;
    size_t i = (size_t)std::ceil(p * v.size()) - 1;
    return v[std::min(i, v.size() - 1)];
  };
  if (completed) *completed = v.size();
  if (p50_ms) *p50_ms = pct(0.50);
  if (p99_ms) *p99_ms = pct(0.99);
  if (mean_batch) *mean_batch = s->batches ? (double)s->batched / (double)s->batches : 0.0;
  return BM_OK;
}

int bm_server_reset_stats(bm_server* s) {
  if (!s) return BM_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  s->latencies.clear();
  s->batches = s->batched = 0;
  return BM_OK;
}

void bm_server_free(bm_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->done)
    if (kv.second.r) bm_result_free(kv.second.r);
  for (auto& lane : s->lanes)
    if (lane.done) (void)dev::event_destroy(lane.done);
  for (auto& g : s->galleries)
    if (g.masks) bm_masks_free(g.masks);
  delete s;
}

}  // extern "C"
