// server.cpp -- continuous-batching identification server.
//
// Galleries and evaluation keys stay resident in HBM.  A worker thread owns
// several lanes (each a context sharing the tables, with its own stream and
// memory pool).  Whenever a lane is free it admits queued requests: all queued
// queries against the same gallery (up to a batch limit) whose estimated
// scratch and result memory fit the HBM budget next to the work already in
// flight.  The admitted queries are expanded (Alg. 1) one by one and then
// matched together in one batched Alg. 2 pass (query x group pairs share every
// launch).  Lanes run concurrently on the device, so requests arriving while
// others execute start as soon as a lane and memory free up.  Every result is
// the same exact function of its query and gallery whether it ran alone or in
// a batch.
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
  int max_batch = 8;

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
    int status = BM_OK;
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

  uint64_t estimate(const bm_gallery& g, int nq) const {
    const Ctx& c = ctx->c;
    const bmx::Plan p = shape(g);
    const int t = p.t, ql = p.ql, ol = p.ol;
    const u64 N = c.N;
    const u64 l = (u64)t;
    const u64 beta = (l + c.alpha - 1) / c.alpha, ext = l + c.K;
    u64 chunk = c.group_chunk > 0 ? (u64)c.group_chunk : (u64)(c.N >= 65536 ? 16 : 64);
    const u64 per_q = std::max<u64>(1, chunk / (u64)nq);
    const u64 pairs = std::min<u64>(per_q, g.groups) * nq;
    const u64 pair_words = (3 + 2 + 2 + 2 + 1 + 2 + 2) * l * N + (beta + 2) * ext * N;
    const u64 out_words = (u64)nq * bmx::out_cts(p, g.groups, g.d, g.k) * 2 * ol * N;
    const u64 cu_words = (u64)nq * g.k * 2 * l * N + (g.k > 1 ? g.k * 4 * (u64)ql * N : 0);
    // compression: the uncompressed outputs, the masked and rescaled copies and one rotation's scratch
    const u64 comp_words = p.comp ? (u64)nq * g.groups * 2 * (2 * p.rot + p.rot - 1) * N +
                                        pair_words
                                  : 0;
    return 8 * (pairs * pair_words + out_words + cu_words + comp_words);
  }

  void launch(Lane& lane) {
    Ctx& c = *lane.c;
    const Gal& G = galleries[lane.reqs[0].gid];
    const bm_gallery& g = *G.g;
    const int nq = (int)lane.reqs.size();
    const size_t N = c.N;
    const bmx::Plan p = shape(g);
    const int t = p.t, ql = p.ql, ol = p.ol;
    const size_t cu_stride = (size_t)g.k * 2 * t * N;
    DBuf cu(&c, (size_t)nq * cu_stride);
    DBuf cut(g.k > 1 ? DBuf(&c, (size_t)2 * ql * N) : DBuf());
    double cu_scale = 0;
    for (int j = 0; j < nq; ++j) {
      const bm_ct& q = *lane.reqs[j].q;
      if ((int)q.limbs < ql) BM_THROW(BM_ELEVEL, "query level does not fit the gallery");
      if (g.k == 1) {                     // exact drop straight into the batch buffer
        ev::drop(c, q.buf.p(), 1, 2, (int)q.limbs, t, cu.p() + j * cu_stride);
        cu_scale = q.scale;
      } else {
        const u64* qq = q.buf.p();
        if ((int)q.limbs > ql) {
          ev::drop(c, q.buf.p(), 1, 2, (int)q.limbs, ql, cut.p());
          qq = cut.p();
        }
        (p.hoist ? bmx::expand_hoisted : bmx::expand)(c, evk, qq, ql, G.masks->pt.p(), g.d, g.k,
                                                      cu.p() + j * cu_stride);
        cu_scale = q.scale * G.masks->scale / (double)c.primes[ql - 1].q;
      }
      if (cu_scale != g.scale) BM_THROW(BM_ESCALE, "query and gallery scales differ");
    }
    const u64 n_out = bmx::out_cts(p, g.groups, g.d, g.k);
    const size_t per = (size_t)n_out * 2 * ol * N;
    auto store = std::make_shared<DBuf>(&c, (size_t)nq * per);
    bmx::match_groups(c, evk, p, cu.p(), nq, cu_stride, g, G.cmask, store->p(), per);
    lane.results.clear();
    for (int j = 0; j < nq; ++j) {
      std::unique_ptr<bm_result> r(new bm_result);
      r->ctx = ctx;
      r->d = g.d;
      r->k = g.k;
      r->limbs = (uint32_t)ol;
      r->groups = n_out;
      r->packed = p.comp ? g.d / g.k : 0;
      r->n_templates = g.n_templates;
      r->scale = bmx::result_scale(c, p, cu_scale, g.scale);
      r->store = store;
      r->off = (size_t)j * per;
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
        const uint32_t gid = queue.front().gid;
        const bm_gallery& g = *galleries[gid].g;
        std::vector<size_t> pick;
        for (size_t i = 0; i < queue.size() && (int)pick.size() < max_batch; ++i)
          if (queue[i].gid == gid) pick.push_back(i);
        // shrink the batch until it fits next to the work in flight
        uint64_t need = estimate(g, (int)pick.size());
        while (pick.size() > 1 && inflight + need > budget) {
          pick.pop_back();
          need = estimate(g, (int)pick.size());
        }
        if (inflight + need > budget) {
          if (inflight == 0) {            // can never fit: reject
            Req r = std::move(queue.front());
            queue.pop_front();
            fail_now(r, BM_EBUDGET);
            progress = true;
          }
          break;
        }
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
      if (!progress) cv.wait_for(lk, std::chrono::microseconds(any_busy ? 100 : 2000));
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
  if (s->estimate(g, 1) > s->budget) return BM_EBUDGET;
  if (q->query_d && q->query_d != g.d) return BM_EDIM;
  if ((int)q->limbs < s->shape(g).ql || q->comps != 2) return BM_ELEVEL;
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
