// capi.cpp -- the extern "C" boundary: argument checks, handle lifetimes,
// exception-to-status translation.  Every entry point is declared and
// documented in include/blindmatch.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <set>
#include <thread>

#include "blindmatch_impl.hpp"

using namespace bm;

namespace {

thread_local std::string g_err;   // errors raised before a context exists

template <class F>
int guarded(bm_ctx* ctx, F&& f) {
  try {
    f();
    return BM_OK;
  } catch (const Error& e) {
    if (ctx) ctx->c.last_error = e.msg;
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->c.last_error = "host allocation failed";
    return BM_ENOMEM;
  } catch (const std::exception& e) {
    if (ctx) ctx->c.last_error = e.what();
    return BM_EINVAL;
  }
}

#define REQUIRE(cond, code, msg) \
  do {                           \
    if (!(cond)) BM_THROW((code), (msg)); \
  } while (0)

// Every handle a call takes must come from the call's context (its buffers
// are sized for that context's ring and limbs); NULL handles pass here.
template <class... H>
void same_ctx(const bm_ctx* ctx, const H*... h) {
  const bool ok = ((h == nullptr || h->ctx == ctx) && ...);
  REQUIRE(ok, BM_EINVAL, "handle made by another context");
}

// the `count` largest primes below 2^bits that are 1 mod `step` (2N, or 4N),
// in descending order
std::vector<u64> primes_below(int bits, u64 step, int count, const std::vector<u64>& avoid) {
  std::vector<u64> out;
  u64 cand = (((1ULL << bits) - 1) / step) * step + 1;
  while ((int)out.size() < count && cand > step) {
    if (h_is_prime(cand) && std::find(avoid.begin(), avoid.end(), cand) == avoid.end())
      out.push_back(cand);
    cand -= step;
  }
  return out;
}

void sync(Ctx& c) { HIP_OK(dev::stream_sync(c.stream)); }

}  // namespace

extern "C" {

const char* bm_strerror(int status) {
  switch (status) {
    case BM_OK: return "ok";
    case BM_EINVAL: return "invalid argument";
    case BM_EDIM: return "invalid dimension";
    case BM_ELEVEL: return "level mismatch or too few levels";
    case BM_ESCALE: return "scale mismatch";
    case BM_ENOKEY: return "missing Galois key";
    case BM_ENOMEM: return "out of memory";
    case BM_EBUDGET: return "HBM budget exceeded";
    case BM_EDEVICE: return "device error";
    case BM_EBUSY: return "busy";
    default: return "unknown status";
  }
}

const char* bm_last_error(const bm_ctx* ctx) {
  return ctx ? ctx->c.last_error.c_str() : g_err.c_str();
}

int bm_params_preset(int preset, bm_params* out) {
  return guarded(nullptr, [&] {
    REQUIRE(out, BM_EINVAL, "out is NULL");
    std::memset(out, 0, sizeof(*out));
    out->sigma = 3.2;
    if (preset == 1 || preset == 3) {
      const size_t N = 1u << 12;
      const u64 M = preset == 3 ? 4 * N : 2 * N;
      out->log_n = 12;
      out->ring = preset == 3 ? BM_RING_CI : BM_RING_STD;
      auto q0 = primes_below(50, M, 1, {});
      auto q12 = primes_below(40, M, 2, {});
      auto p = primes_below(51, M, 1, {});
      out->n_q = 3;
      out->q[0] = q0[0];
      out->q[1] = q12[0];
      out->q[2] = q12[1];
      out->n_p = 1;
      out->p[0] = p[0];
      out->alpha = 1;
      out->scale = std::ldexp(1.0, 40);
      out->out_limbs = 0;
    } else if (preset == 2 || preset == 4) {
      const size_t N = 1u << 16;
      const u64 M = preset == 4 ? 4 * N : 2 * N;
      out->log_n = 16;
      out->ring = preset == 4 ? BM_RING_CI : BM_RING_STD;
      auto q = primes_below(50, M, 8, {});
      auto p = primes_below(51, M, 2, {});
      out->n_q = 8;
      for (int i = 0; i < 8; ++i) out->q[i] = q[i];
      out->n_p = 2;
      out->p[0] = p[0];
      out->p[1] = p[1];
      out->alpha = 2;
      out->scale = std::ldexp(1.0, 50);
      out->out_limbs = 2;
    } else {
      BM_THROW(BM_EINVAL, "unknown preset");
    }
  });
}

int bm_ctx_create(const bm_params* p, int device, bm_ctx** out) {
  return guarded(nullptr, [&] {
    REQUIRE(p && out, BM_EINVAL, "NULL argument");
    *out = nullptr;
    REQUIRE(p->log_n >= 3 && p->log_n <= 16, BM_EINVAL, "log_n must be in [3, 16]");
    REQUIRE(p->n_q >= 1 && p->n_q <= 16 && p->n_p >= 1 && p->n_p <= 4, BM_EINVAL, "prime counts");
    REQUIRE(p->alpha >= 1 && p->alpha <= (uint32_t)MAX_ALPHA, BM_EINVAL, "alpha in [1, 4]");
    REQUIRE(p->n_q + p->n_p <= (uint32_t)MAX_PRIMES, BM_EINVAL, "too many primes");
    std::unique_ptr<bm_ctx> h(new bm_ctx);
    h->params = *p;
    Ctx& c = h->c;
    c.device = device;
    c.log_n = (int)p->log_n;
    c.N = (size_t)1 << p->log_n;
    REQUIRE(p->ring == BM_RING_STD || p->ring == BM_RING_CI, BM_EINVAL, "unknown ring");
    c.ci = p->ring == BM_RING_CI;
    c.n = c.ci ? c.N : c.N / 2;
    c.M = c.ci ? 4 * (u64)c.N : 2 * (u64)c.N;
    c.L = (int)p->n_q - 1;
    c.K = (int)p->n_p;
    c.alpha = (int)p->alpha;
    c.dnum = (int)((p->n_q + p->alpha - 1) / p->alpha);
    c.scale = p->scale;
    c.sigma = p->sigma > 0 ? p->sigma : 3.2;
    c.out_limbs = p->out_limbs;
    REQUIRE(c.scale > 1.0, BM_EINVAL, "scale must exceed 1");
    REQUIRE(c.out_limbs <= p->n_q, BM_EINVAL, "out_limbs above the chain length");
    std::vector<u64> all;
    for (uint32_t i = 0; i < p->n_q; ++i) all.push_back(p->q[i]);
    for (uint32_t i = 0; i < p->n_p; ++i) all.push_back(p->p[i]);
    for (size_t i = 0; i < all.size(); ++i) {
      const u64 q = all[i];
      REQUIRE(q > 2 && q < (1ULL << 51), BM_EINVAL, "primes must lie below 2^51");
      REQUIRE(q % c.M == 1, BM_EINVAL, c.ci ? "primes must be 1 mod 4N" : "primes must be 1 mod 2N");
      REQUIRE(h_is_prime(q), BM_EINVAL, "modulus is not prime");
      for (size_t j = 0; j < i; ++j) REQUIRE(all[j] != q, BM_EINVAL, "repeated prime");
      HostPrime hp;
      hp.q = q;
      hp.bits = 64 - __builtin_clzll(q);
      hp.psi = h_primitive_2n_root(q, c.M / 2);   // primitive M-th root
      c.primes.push_back(hp);
    }
    c.cdt = gaussian_cdt(c.sigma, 19);
    HIP_OK(dev::set_device(device));
    HIP_OK(dev::stream_create(&c.own_stream));
    c.stream = c.own_stream;
    c.pool.reset(new DevicePool(device));
    build_context_tables(c);
    (void)kern::noalloc_scratch(device);   // the no-allocation match's scratch, looked up once per device
    *out = h.release();
  });
}

void bm_ctx_free(bm_ctx* ctx) { delete ctx; }

int bm_ctx_set_group_chunk(bm_ctx* ctx, uint32_t groups) {
  return guarded(ctx, [&] {
    REQUIRE(ctx, BM_EINVAL, "NULL context");
    ctx->c.group_chunk = (int)groups;
  });
}

int bm_ctx_set_graphs(bm_ctx* ctx, int on) {
  return guarded(ctx, [&] {
    REQUIRE(ctx, BM_EINVAL, "NULL context");
    if (!on && !ctx->c.graphs.empty()) {
      HIP_OK(dev::stream_sync(ctx->c.stream));
      ctx->c.graphs.clear();
    }
    ctx->c.use_graphs = on != 0;
  });
}

int bm_ctx_set_allocator(bm_ctx* ctx, void* (*alloc_fn)(size_t, void*), void (*free_fn)(void*, void*),
                         void* user) {
  return guarded(ctx, [&] {
    REQUIRE(ctx, BM_EINVAL, "NULL context");
    REQUIRE((alloc_fn == nullptr) == (free_fn == nullptr), BM_EINVAL,
            "give both allocator callbacks, or neither");
    Ctx& c = ctx->c;
    std::shared_ptr<const AllocHook> h;
    if (alloc_fn) {
      AllocHook a;
      a.alloc = alloc_fn;
      a.free = free_fn;
      a.user = user;
      h = std::make_shared<const AllocHook>(a);
    }
    HIP_OK(dev::stream_sync(c.stream));
    c.hook = h;
    c.pool->set_hook(h);
  });
}

int bm_ctx_pool_bytes(const bm_ctx* ctx, uint64_t* bytes) {
  if (!ctx || !bytes) return BM_EINVAL;
  *bytes = ctx->c.pool->bytes_held();
  return BM_OK;
}

int bm_profile_enable(bm_ctx* ctx, int on) {
  return guarded(ctx, [&] {
    REQUIRE(ctx, BM_EINVAL, "NULL context");
    Profiler& p = *ctx->c.prof;
    if (on) p.reset();
    p.on = on != 0;
  });
}

int bm_profile_dump(bm_ctx* ctx, char* buf, size_t cap, size_t* needed) {
  return guarded(ctx, [&] {
    REQUIRE(ctx, BM_EINVAL, "NULL context");
    Profiler& p = *ctx->c.prof;
    p.collect();
    std::string out;
    char line[256];
    for (auto& kv : p.entries) {
      std::snprintf(line, sizeof(line), "%s %llu %.6f %.0f %.0f\n", kv.first.c_str(),
                    (unsigned long long)kv.second.launches, kv.second.ms, kv.second.bytes, kv.second.ops);
      out += line;
    }
    if (needed) *needed = out.size();
    if (buf && cap) {
      const size_t n = std::min(cap - 1, out.size());
      std::memcpy(buf, out.data(), n);
      buf[n] = 0;
    }
  });
}

int bm_bench_modmul(bm_ctx* ctx, uint32_t prime, uint32_t blocks, uint32_t iters, const uint64_t* seed,
                    uint64_t* words, size_t n_words, double* ms) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && seed && ms, BM_EINVAL, "NULL argument");
    Ctx& c = ctx->c;
    REQUIRE((int)prime < c.nprimes(), BM_EINVAL, "prime index out of range");
    REQUIRE(blocks >= 1 && blocks <= 65536, BM_EINVAL, "blocks must lie in 1..65536");
    REQUIRE(iters >= 2 && iters % 2 == 0 && iters <= (1u << 24), BM_EINVAL, "iters must be even, 2..2^24");
    const size_t nw = (size_t)blocks * 256 * 16;
    REQUIRE(n_words <= nw && (words || !n_words), BM_EINVAL, "n_words above the probe's output");
    for (int j = 0; j < 24; ++j) REQUIRE(seed[j] < c.primes[prime].q, BM_EINVAL, "seed words must be residues");
    c.use_stream(nullptr);
    DBuf sd(&c, 24), out(&c, nw);
    HIP_OK(dev::memcpy(sd.p(), seed, 24 * sizeof(u64), hipMemcpyHostToDevice));
    struct Ev {
      hipEvent_t e = nullptr;
      ~Ev() {
        if (e) (void)dev::event_destroy(e);
      }
    } e0, e1;
    HIP_OK(dev::event_create(&e0.e, true));
    HIP_OK(dev::event_create(&e1.e, true));
    HIP_OK(dev::event_record(e0.e, c.stream));
    kern::modmul_rate(c, (int)prime, (int)blocks, (int)iters, sd.p(), out.p());
    HIP_OK(dev::event_record(e1.e, c.stream));
    HIP_OK(dev::event_sync(e1.e));
    float t = 0.f;
    HIP_OK(dev::event_elapsed(&t, e0.e, e1.e));
    *ms = t;
    if (n_words) HIP_OK(dev::memcpy(words, out.p(), n_words * sizeof(u64), hipMemcpyDeviceToHost));
  });
}

// ------------------------------------------------------------------ keys

int bm_rotations_for(uint32_t d, uint32_t k, int32_t* out, size_t cap, size_t* n) {
  return guarded(nullptr, [&] {
    REQUIRE(n, BM_EINVAL, "n is NULL");
    REQUIRE(bmx::is_pow2(d) && bmx::is_pow2(k) && k <= d, BM_EDIM, "power-of-two k | d");
    std::vector<int32_t> r;
    const uint32_t c = d / k;
    for (uint32_t t = 0; (1u << t) < c; ++t) r.push_back((int32_t)(1u << t));
    for (uint32_t t = 0; (1u << t) < k; ++t) {
      r.push_back((int32_t)(c << t));
      r.push_back(-(int32_t)(c << t));
    }
    *n = r.size();
    if (out)
      for (size_t i = 0; i < std::min(cap, r.size()); ++i) out[i] = r[i];
  });
}

int bm_rotations_compress(uint32_t d, uint32_t k, int32_t* out, size_t cap, size_t* n) {
  return guarded(nullptr, [&] {
    REQUIRE(n, BM_EINVAL, "n is NULL");
    REQUIRE(bmx::is_pow2(d) && bmx::is_pow2(k) && k <= d, BM_EDIM, "power-of-two k | d");
    std::vector<int32_t> r;
    for (uint32_t t = 0; (1u << t) < d / k; ++t) r.push_back(-(int32_t)(1u << t));
    *n = r.size();
    if (out)
      for (size_t i = 0; i < std::min(cap, r.size()); ++i) out[i] = r[i];
  });
}

int bm_rotations_hoisted(uint32_t d, uint32_t k, int32_t* out, size_t cap, size_t* n) {
  return guarded(nullptr, [&] {
    REQUIRE(n, BM_EINVAL, "n is NULL");
    REQUIRE(bmx::is_pow2(d) && bmx::is_pow2(k) && k <= d, BM_EDIM, "power-of-two k | d");
    const int32_t c = (int32_t)(d / k);
    std::set<int32_t> r;
    for (int32_t j = 1; j < c; ++j) r.insert(j);
    for (uint32_t i = 0; i < k; ++i)
      for (uint32_t S = 1; S < k; ++S) {
        int32_t a = 0;
        for (int t = 0; (1u << t) < k; ++t)
          if ((S >> t) & 1) a += ((i >> t) & 1) ? (c << t) : -(c << t);
        r.insert(a);
      }
    std::vector<int32_t> v(r.begin(), r.end());
    *n = v.size();
    if (out)
      for (size_t i = 0; i < std::min(cap, v.size()); ++i) out[i] = v[i];
  });
}

int bm_rotations_enroll(const bm_ctx* ctx, uint32_t d, uint32_t k, int32_t* out, size_t cap, size_t* n) {
  return guarded(nullptr, [&] {
    REQUIRE(ctx && n, BM_EINVAL, "NULL argument");
    bmx::check_shape(ctx->c, d, k);
    std::vector<int32_t> r;
    const uint64_t cc = d / k, T = ctx->c.n / cc;
    for (uint32_t t = 0; (1ULL << t) < T; ++t) r.push_back((int32_t)(cc << t));
    *n = r.size();
    if (out)
      for (size_t i = 0; i < std::min(cap, r.size()); ++i) out[i] = r[i];
  });
}

// device table of an evaluation key's Galois keys by g / 2 (0 where absent),
// read by the hoisted rotation sums
static void build_gtab(Ctx& c, bm_evk* e) {
  std::vector<u64> tab(c.M / 2, 0);
  for (auto& kv : e->gk) tab[kv.first >> 1] = (u64)(uintptr_t)kv.second->k.p();
  e->gtab = DBuf(&c, c.M / 2);
  HIP_OK(dev::memcpy_async(e->gtab.p(), tab.data(), tab.size() * sizeof(u64), hipMemcpyHostToDevice, c.stream));
  sync(c);
}

// words[polys][limbs][N] (coefficient domain) must hold residues of their limbs' primes
static void check_residues(const Ctx& c, const uint64_t* words, size_t polys, int limbs) {
  for (size_t pz = 0; pz < polys; ++pz)
    for (int l = 0; l < limbs; ++l) {
      const u64 q = c.primes[l].q;
      const uint64_t* w = words + (pz * limbs + l) * c.N;
      for (size_t i = 0; i < c.N; ++i)
        if (w[i] >= q) BM_THROW(BM_EINVAL, "a word is not a residue of its limb's prime");
    }
}

// switching key from coefficient-domain words[dnum][2][L+1+K][N] into the
// device form (evaluation domain, FP64 values)
static void load_switch_key(Ctx& c, const uint64_t* words, DBuf& key) {
  const int np = c.nprimes();
  const size_t polys = (size_t)c.dnum * 2;
  check_residues(c, words, polys, np);
  key = DBuf(&c, polys * np * c.N);
  ev::import_coeffs(c, words, (int)polys, np, key.p());
  kern::words_f64(c, key.p(), polys * np * c.N, true);
  sync(c);
}

int bm_keygen(bm_ctx* ctx, uint64_t seed, const int32_t* rotations, size_t n_rot, bm_sk** sk,
              bm_pk** pk, bm_evk** evk) {
  return guarded(ctx, [&] {
    REQUIRE(ctx, BM_EINVAL, "NULL context");
    REQUIRE(n_rot == 0 || rotations, BM_EINVAL, "rotations is NULL");
    Ctx& c = ctx->c;
    c.use_stream(nullptr);
    std::unique_ptr<bm_sk> s(new bm_sk);
    s->ctx = ctx;
    ev::keygen_secret(c, seed, s.get());
    std::unique_ptr<bm_pk> p;
    if (pk) {
      p.reset(new bm_pk);
      p->ctx = ctx;
      ev::keygen_public(c, seed, s.get(), p.get());
    }
    std::unique_ptr<bm_evk> e;
    if (evk) {
      e.reset(new bm_evk);
      e->ctx = ctx;
      const int np = c.nprimes();
      const LimbMap all = kern::ext_map(c, c.L + 1);
      DBuf s2(&c, (size_t)np * c.N);
      kern::mul(c, s->s_ntt.p(), 0, s->s_ntt.p(), 0, s2.p(), 0, 1, all);
      ev::keygen_switch(c, seed, ev::DOM_RLK_A, ev::DOM_RLK_E, 0, s.get(), s2.p(), e->rlk.k);
      for (size_t i = 0; i < n_rot; ++i) {
        const u64 g = ev::galois_for_rotation(c, rotations[i]);
        if (e->gk.count(g)) continue;
        DBuf sg(&c, (size_t)np * c.N);
        kern::automorphism(c, s->s_ntt.p(), 0, sg.p(), 0, 1, np, g, g, 31);
        std::unique_ptr<bm_switch_key> key(new bm_switch_key);
        ev::keygen_switch(c, seed, ev::DOM_GK_A, ev::DOM_GK_E, g * (u64)c.dnum, s.get(), sg.p(), key->k);
        e->gk.emplace(g, std::move(key));
      }
      build_gtab(c, e.get());
    }
    sync(c);
    if (sk) *sk = s.release();
    if (pk) *pk = p.release();
    if (evk) *evk = e.release();
  });
}

int bm_sk_export(const bm_sk* sk, int64_t* s, size_t n) {
  if (!sk || !s || n != sk->s.size()) return BM_EINVAL;
  std::memcpy(s, sk->s.data(), n * sizeof(int64_t));
  return BM_OK;
}

int bm_pk_export(const bm_pk* pk, uint32_t comp, uint64_t* words, size_t n_words) {
  if (!pk) return BM_EINVAL;
  bm_ctx* ctx = pk->ctx;
  return guarded(ctx, [&] {
    Ctx& c = ctx->c;
    const size_t ln = (size_t)(c.L + 1) * c.N;
    REQUIRE(words && comp < 2 && n_words == ln, BM_EINVAL, "pk export size");
    c.use_stream(nullptr);
    ev::export_coeffs(c, pk->pk.p() + comp * ln, 1, c.L + 1, words);
  });
}

int bm_evk_export(const bm_evk* evk, uint64_t galois, uint32_t digit, uint32_t comp, uint64_t* words,
                  size_t n_words) {
  if (!evk) return BM_EINVAL;
  bm_ctx* ctx = evk->ctx;
  return guarded(ctx, [&] {
    Ctx& c = ctx->c;
    const int np = c.nprimes();
    const size_t ln = (size_t)np * c.N;
    REQUIRE(words && comp < 2 && (int)digit < c.dnum && n_words == ln, BM_EINVAL, "evk export size");
    const u64* key = galois == 0 ? evk->rlk.k.p() : bmx::galois_key(evk, galois);
    c.use_stream(nullptr);
    DBuf tmp(&c, ln);
    HIP_OK(dev::memcpy_async(tmp.p(), key + (size_t)(2 * digit + comp) * ln, ln * sizeof(u64),
                          hipMemcpyDeviceToDevice, c.stream));
    kern::words_f64(c, tmp.p(), ln, false);   // keys are held as FP64 values
    const LimbMap all = kern::ext_map(c, c.L + 1);
    kern::ntt(c, tmp.p(), 0, tmp.p(), 0, 1, all, true);
    HIP_OK(dev::memcpy_async(words, tmp.p(), ln * sizeof(u64), hipMemcpyDeviceToHost, c.stream));
    sync(c);
  });
}

int bm_pk_import(bm_ctx* ctx, const uint64_t* words, size_t n_words, bm_pk** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && words && out, BM_EINVAL, "NULL argument");
    Ctx& c = ctx->c;
    const size_t ln = (size_t)(c.L + 1) * c.N;
    REQUIRE(n_words == 2 * ln, BM_EINVAL, "public key import needs 2 (L+1) N words");
    check_residues(c, words, 2, c.L + 1);
    c.use_stream(nullptr);
    std::unique_ptr<bm_pk> p(new bm_pk);
    p->ctx = ctx;
    p->pk = DBuf(&c, 2 * ln);
    ev::import_coeffs(c, words, 2, c.L + 1, p->pk.p());
    *out = p.release();
  });
}

int bm_evk_import(bm_ctx* ctx, const uint64_t* galois, size_t n_galois, const uint64_t* words, size_t n_words,
                  bm_evk** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && words && out && (n_galois == 0 || galois), BM_EINVAL, "NULL argument");
    Ctx& c = ctx->c;
    const size_t per = (size_t)c.dnum * 2 * c.nprimes() * c.N;
    REQUIRE(n_words == (1 + n_galois) * per, BM_EINVAL, "evaluation key import needs (1 + n_galois) keys");
    std::set<u64> seen;
    for (size_t i = 0; i < n_galois; ++i) {
      const u64 g = galois[i];
      REQUIRE((g & 1) && g > 1 && g < c.M && !seen.count(g), BM_EINVAL,
              "Galois elements must be distinct odd values in (1, 2N)");
      seen.insert(g);
    }
    c.use_stream(nullptr);
    std::unique_ptr<bm_evk> e(new bm_evk);
    e->ctx = ctx;
    load_switch_key(c, words, e->rlk.k);
    for (size_t i = 0; i < n_galois; ++i) {
      std::unique_ptr<bm_switch_key> key(new bm_switch_key);
      load_switch_key(c, words + (1 + i) * per, key->k);
      e->gk.emplace(galois[i], std::move(key));
    }
    build_gtab(c, e.get());
    *out = e.release();
  });
}

int bm_evk_galois(const bm_evk* evk, uint64_t* galois, size_t cap, size_t* n) {
  if (!evk || !n || (cap && !galois)) return BM_EINVAL;
  *n = evk->gk.size();
  size_t i = 0;
  for (auto& kv : evk->gk) {
    if (i >= cap) break;
    galois[i++] = kv.first;
  }
  return BM_OK;
}

void bm_sk_free(bm_sk* sk) { delete sk; }
void bm_pk_free(bm_pk* pk) { delete pk; }
static void drop_graphs(bm_ctx* ctx) {
  if (!ctx || ctx->c.graphs.empty()) return;
  (void)dev::stream_sync(ctx->c.stream);
  ctx->c.graphs.clear();
}

void bm_evk_free(bm_evk* evk) {
  if (evk) drop_graphs(evk->ctx);
  delete evk;
}

// ------------------------------------------------------------------ encode / encrypt

int bm_ctx_params(const bm_ctx* ctx, bm_params* out) {
  return guarded(nullptr, [&] {
    REQUIRE(ctx && out, BM_EINVAL, "NULL argument");
    *out = ctx->params;
  });
}

int bm_encode(bm_ctx* ctx, const double* slots, size_t n_slots, double scale, int64_t* coeffs) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && slots && coeffs, BM_EINVAL, "NULL argument");
    REQUIRE(n_slots == ctx->c.n, BM_EINVAL, "n_slots must equal the slot count");
    ring_encode(ctx->c, slots, scale, coeffs);
  });
}

static bm_ct* new_ct(bm_ctx* ctx, uint32_t comps, uint32_t limbs, double scale) {
  std::unique_ptr<bm_ct> ct(new bm_ct);
  ct->ctx = ctx;
  ct->comps = comps;
  ct->limbs = limbs;
  ct->scale = scale;
  ct->buf = DBuf(&ctx->c, (size_t)comps * limbs * ctx->c.N);
  return ct.release();
}

int bm_encrypt_coeffs(bm_ctx* ctx, const bm_pk* pk, const int64_t* coeffs, uint32_t limbs,
                      double scale, uint64_t seed, uint64_t ct_id, bm_ct** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && pk && coeffs && out, BM_EINVAL, "NULL argument");
    same_ctx(ctx, pk);
    Ctx& c = ctx->c;
    REQUIRE(limbs >= 1 && (int)limbs <= c.L + 1, BM_ELEVEL, "limbs out of range");
    c.use_stream(nullptr);
    std::unique_ptr<bm_ct> ct(new_ct(ctx, 2, limbs, scale));
    ev::encrypt_batch(c, pk, coeffs, 1, (int)limbs, seed, &ct_id, ct->buf.p());
    sync(c);
    *out = ct.release();
  });
}

int bm_encrypt_query(bm_ctx* ctx, const bm_pk* pk, const float* q, uint32_t d, uint64_t seed,
                     uint64_t ct_id, bm_ct** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && pk && q && out, BM_EINVAL, "NULL argument");
    same_ctx(ctx, pk);
    Ctx& c = ctx->c;
    REQUIRE(bmx::is_pow2(d) && d <= c.n, BM_EDIM, "d must be a power of two <= slot count");
    std::vector<double> slots(c.n);
    for (size_t s = 0; s < c.n; ++s) slots[s] = (double)q[s % d];
    std::vector<int64_t> m(c.N);
    ring_encode(c, slots.data(), c.scale, m.data());
    c.use_stream(nullptr);
    std::unique_ptr<bm_ct> ct(new_ct(ctx, 2, c.L + 1, c.scale));
    ev::encrypt_batch(c, pk, m.data(), 1, c.L + 1, seed, &ct_id, ct->buf.p());
    sync(c);
    ct->query_d = d;
    *out = ct.release();
  });
}

int bm_encrypt_template(bm_ctx* ctx, const bm_pk* pk, const float* x, uint32_t d, uint64_t seed,
                        uint64_t ct_id, bm_ct** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && pk && x && out, BM_EINVAL, "NULL argument");
    same_ctx(ctx, pk);
    Ctx& c = ctx->c;
    REQUIRE(bmx::is_pow2(d) && d <= c.n, BM_EDIM, "d must be a power of two <= slot count");
    std::vector<double> slots(c.n, 0.0);
    for (size_t s = 0; s < d; ++s) slots[s] = (double)x[s];
    std::vector<int64_t> m(c.N);
    ring_encode(c, slots.data(), c.scale, m.data());
    c.use_stream(nullptr);
    std::unique_ptr<bm_ct> ct(new_ct(ctx, 2, c.L + 1, c.scale));
    ev::encrypt_batch(c, pk, m.data(), 1, c.L + 1, seed, &ct_id, ct->buf.p());
    sync(c);
    *out = ct.release();
  });
}

static bm_gallery* new_gallery(bm_ctx* ctx, uint32_t d, uint32_t k, uint32_t limbs, uint64_t groups,
                               uint64_t n, double scale) {
  std::unique_ptr<bm_gallery> g(new bm_gallery);
  g->ctx = ctx;
  g->d = d;
  g->k = k;
  g->limbs = limbs;
  g->groups = groups;
  g->n_templates = n;
  g->scale = scale;
  g->buf = DBuf(&ctx->c, (size_t)groups * k * 2 * limbs * ctx->c.N);
  return g.release();
}

int bm_encrypt_gallery(bm_ctx* ctx, const bm_pk* pk, const float* x, uint64_t n, uint32_t d,
                       uint32_t k, uint64_t seed, uint64_t ct_id_base, bm_gallery** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && pk && x && out && n > 0, BM_EINVAL, "NULL argument or empty gallery");
    same_ctx(ctx, pk);
    Ctx& c = ctx->c;
    bmx::check_shape(c, d, k);
    const uint32_t cc = d / k;
    const uint64_t T = c.n / cc;
    const uint64_t G = (n + T - 1) / T;
    const int lg = bmx::gallery_limbs(c, k);
    REQUIRE(lg >= 2, BM_ELEVEL, "chain too short for this k");
    c.use_stream(nullptr);
    std::unique_ptr<bm_gallery> gal(new_gallery(ctx, d, k, (uint32_t)lg, G, n, c.scale));
    const size_t N = c.N;
    const uint64_t total = G * k;
    const uint64_t batch = std::max<uint64_t>(1, std::min<uint64_t>(total, N >= 65536 ? 32 : 256));
    std::vector<int64_t> m(batch * N);
    std::vector<u64> ids(batch);
    for (uint64_t b0 = 0; b0 < total; b0 += batch) {
      const uint64_t nb = std::min(batch, total - b0);
      // pack + encode every ciphertext of this batch in parallel
      std::vector<std::thread> th;
      const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
      for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
          std::vector<double> slots(c.n);
          for (uint64_t b = t; b < nb; b += nt) {
            const uint64_t idx = b0 + b, g = idx / k, i = idx % k;
            for (size_t s = 0; s < c.n; ++s) {
              const uint64_t tid = g * T + s / cc;
              slots[s] = tid < n ? (double)x[tid * d + i * cc + s % cc] : 0.0;
            }
            ring_encode(c, slots.data(), c.scale, m.data() + b * N);
          }
        });
      for (auto& th1 : th) th1.join();
      for (uint64_t b = 0; b < nb; ++b) ids[b] = ct_id_base + b0 + b;
      ev::encrypt_batch(c, pk, m.data(), (int)nb, lg, seed, ids.data(),
                        gal->buf.p() + b0 * 2 * (size_t)lg * N);
      sync(c);
    }
    *out = gal.release();
  });
}

int bm_gallery_import(bm_ctx* ctx, const uint64_t* words, uint64_t groups, uint32_t d, uint32_t k,
                      uint32_t limbs, double scale, uint64_t n_templates, bm_gallery** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && words && out && groups > 0, BM_EINVAL, "NULL argument");
    Ctx& c = ctx->c;
    bmx::check_shape(c, d, k);
    REQUIRE(limbs >= 2 && (int)limbs <= c.L + 1, BM_ELEVEL, "limbs out of range");
    const uint64_t T = c.n / (d / k);
    REQUIRE(n_templates <= groups * T && n_templates > (groups - 1) * T, BM_EINVAL,
            "n_templates does not match the group count");
    c.use_stream(nullptr);
    std::unique_ptr<bm_gallery> gal(new_gallery(ctx, d, k, limbs, groups, n_templates, scale));
    ev::import_coeffs(c, words, (int)(groups * k * 2), (int)limbs, gal->buf.p());
    *out = gal.release();
  });
}

int bm_gallery_export(const bm_gallery* g, uint64_t* words, size_t n_words) {
  if (!g) return BM_EINVAL;
  bm_ctx* ctx = g->ctx;
  return guarded(ctx, [&] {
    Ctx& c = ctx->c;
    REQUIRE(words && n_words == g->groups * g->k * 2 * g->limbs * c.N, BM_EINVAL, "size");
    c.use_stream(nullptr);
    ev::export_coeffs(c, g->buf.p(), (int)(g->groups * g->k * 2), (int)g->limbs, words);
  });
}

int bm_gallery_info(const bm_gallery* g, uint64_t* groups, uint32_t* limbs, double* scale) {
  if (!g) return BM_EINVAL;
  if (groups) *groups = g->groups;
  if (limbs) *limbs = g->limbs;
  if (scale) *scale = g->scale;
  return BM_OK;
}

void bm_gallery_free(bm_gallery* g) {
  if (g) drop_graphs(g->ctx);
  delete g;
}

// ------------------------------------------------------------------ ciphertexts

int bm_ct_import(bm_ctx* ctx, const uint64_t* words, uint32_t comps, uint32_t limbs, double scale,
                 bm_ct** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && words && out, BM_EINVAL, "NULL argument");
    Ctx& c = ctx->c;
    REQUIRE(comps >= 2 && comps <= 3, BM_EINVAL, "comps must be 2 or 3");
    REQUIRE(limbs >= 1 && (int)limbs <= c.L + 1, BM_ELEVEL, "limbs out of range");
    c.use_stream(nullptr);
    std::unique_ptr<bm_ct> ct(new_ct(ctx, comps, limbs, scale));
    ev::import_coeffs(c, words, (int)comps, (int)limbs, ct->buf.p());
    *out = ct.release();
  });
}

int bm_ct_export(const bm_ct* ct, uint64_t* words, size_t n_words) {
  if (!ct) return BM_EINVAL;
  bm_ctx* ctx = ct->ctx;
  return guarded(ctx, [&] {
    Ctx& c = ctx->c;
    REQUIRE(words && n_words == (size_t)ct->comps * ct->limbs * c.N, BM_EINVAL, "size");
    c.use_stream(nullptr);
    ev::export_coeffs(c, ct->buf.p(), (int)ct->comps, (int)ct->limbs, words);
  });
}

int bm_ct_info(const bm_ct* ct, uint32_t* comps, uint32_t* limbs, double* scale) {
  if (!ct) return BM_EINVAL;
  if (comps) *comps = ct->comps;
  if (limbs) *limbs = ct->limbs;
  if (scale) *scale = ct->scale;
  return BM_OK;
}

void bm_ct_free(bm_ct* ct) { delete ct; }

int bm_decrypt_slots(bm_ctx* ctx, const bm_sk* sk, const bm_ct* ct, double* slots, size_t n) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && sk && ct && slots, BM_EINVAL, "NULL argument");
    same_ctx(ctx, sk, ct);
    Ctx& c = ctx->c;
    REQUIRE(n == c.n, BM_EINVAL, "n must equal the slot count");
    c.use_stream(nullptr);
    std::vector<double> m(c.N);
    ev::decrypt_coeffs(c, sk, ct->buf.p(), (int)ct->comps, (int)ct->limbs, m.data());
    ring_decode(c, m.data(), ct->scale, slots);
  });
}

// ------------------------------------------------------------------ primitive operations

int bm_ntt(bm_ctx* ctx, uint64_t* dev_words, uint32_t n_polys, uint32_t limbs,
           const uint32_t* prime_ids, int inverse, void* stream) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && dev_words && prime_ids, BM_EINVAL, "NULL argument");
    Ctx& c = ctx->c;
    REQUIRE(limbs >= 1 && limbs <= (uint32_t)MAX_LIMBS, BM_EINVAL, "limbs out of range");
    LimbMap m{};
    m.n = (int)limbs;
    for (uint32_t l = 0; l < limbs; ++l) {
      REQUIRE(prime_ids[l] < (uint32_t)c.nprimes(), BM_EINVAL, "prime id out of range");
      m.prime[l] = (int)prime_ids[l];
      m.off[l] = m.ooff[l] = (int)l;
    }
    c.use_stream(stream);
    // the caller vouches for n_polys * limbs * N words at dev_words
    audit::Scoped reg(dev_words, (size_t)n_polys * limbs * c.N * sizeof(u64));
    kern::ntt(c, dev_words, (size_t)limbs * c.N, dev_words, (size_t)limbs * c.N, (int)n_polys, m,
              inverse != 0);
  });
}

int bm_op_add(bm_ctx* ctx, const bm_ct* a, const bm_ct* b, bm_ct** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && a && b && out, BM_EINVAL, "NULL argument");
    same_ctx(ctx, a, b);
    REQUIRE(a->limbs == b->limbs, BM_ELEVEL, "level mismatch");
    REQUIRE(a->scale == b->scale, BM_ESCALE, "scale mismatch");
    Ctx& c = ctx->c;
    c.use_stream(nullptr);
    const uint32_t comps = std::max(a->comps, b->comps);
    std::unique_ptr<bm_ct> o(new_ct(ctx, comps, a->limbs, a->scale));
    const size_t ln = (size_t)a->limbs * c.N;
    const uint32_t common = std::min(a->comps, b->comps);
    kern::add(c, a->buf.p(), ln, b->buf.p(), ln, o->buf.p(), ln, (int)common, kern::chain_map(a->limbs));
    if (comps > common) {
      const bm_ct* big = a->comps > b->comps ? a : b;
      HIP_OK(dev::memcpy_async(o->buf.p() + common * ln, big->buf.p() + common * ln,
                            (comps - common) * ln * sizeof(u64), hipMemcpyDeviceToDevice, c.stream));
    }
    sync(c);
    *out = o.release();
  });
}

int bm_op_pmul(bm_ctx* ctx, const bm_ct* a, const int64_t* pt, double pt_scale, bm_ct** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && a && pt && out, BM_EINVAL, "NULL argument");
    same_ctx(ctx, a);
    Ctx& c = ctx->c;
    c.use_stream(nullptr);
    const size_t ln = (size_t)a->limbs * c.N;
    DBuf p(&c, ln);
    ev::upload_plain(c, pt, 1, (int)a->limbs, p.p());
    std::unique_ptr<bm_ct> o(new_ct(ctx, a->comps, a->limbs, a->scale * pt_scale));
    kern::mul(c, a->buf.p(), ln, p.p(), 0, o->buf.p(), ln, (int)a->comps, kern::chain_map(a->limbs));
    sync(c);
    *out = o.release();
  });
}

int bm_op_tensor(bm_ctx* ctx, const bm_ct* a, const bm_ct* b, bm_ct** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && a && b && out, BM_EINVAL, "NULL argument");
    same_ctx(ctx, a, b);
    REQUIRE(a->comps == 2 && b->comps == 2, BM_EINVAL, "tensor needs 2-component inputs");
    REQUIRE(a->limbs == b->limbs, BM_ELEVEL, "level mismatch");
    Ctx& c = ctx->c;
    c.use_stream(nullptr);
    std::unique_ptr<bm_ct> o(new_ct(ctx, 3, a->limbs, a->scale * b->scale));
    kern::tensor(c, a->buf.p(), 0, 1, (size_t)a->limbs * c.N, b->buf.p(), 0, 1, (size_t)b->limbs * c.N,
                 o->buf.p(), 0, 1, (int)a->limbs, false);
    sync(c);
    *out = o.release();
  });
}

int bm_op_relin(bm_ctx* ctx, const bm_evk* evk, const bm_ct* a, bm_ct** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && evk && a && out, BM_EINVAL, "NULL argument");
    same_ctx(ctx, evk, a);
    REQUIRE(a->comps == 3, BM_EINVAL, "relinearisation needs 3 components");
    Ctx& c = ctx->c;
    c.use_stream(nullptr);
    std::unique_ptr<bm_ct> o(new_ct(ctx, 2, a->limbs, a->scale));
    ev::relin(c, a->buf.p(), 1, (int)a->limbs, evk->rlk.k.p(), o->buf.p());
    sync(c);
    *out = o.release();
  });
}

int bm_op_rescale(bm_ctx* ctx, const bm_ct* a, bm_ct** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && a && out, BM_EINVAL, "NULL argument");
    same_ctx(ctx, a);
    REQUIRE(a->limbs >= 2, BM_ELEVEL, "no level left");
    Ctx& c = ctx->c;
    c.use_stream(nullptr);
    std::unique_ptr<bm_ct> o(new_ct(ctx, a->comps, a->limbs - 1,
                                    a->scale / (double)c.primes[a->limbs - 1].q));
    ev::rescale(c, a->buf.p(), 1, (int)a->comps, (int)a->limbs, o->buf.p());
    sync(c);
    *out = o.release();
  });
}

int bm_op_rotate(bm_ctx* ctx, const bm_evk* evk, const bm_ct* a, int32_t r, bm_ct** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && evk && a && out, BM_EINVAL, "NULL argument");
    same_ctx(ctx, evk, a);
    REQUIRE(a->comps == 2, BM_EINVAL, "rotation needs 2 components");
    Ctx& c = ctx->c;
    c.use_stream(nullptr);
    const u64 g = ev::galois_for_rotation(c, r);
    const u64* key = bmx::galois_key(evk, g);
    std::unique_ptr<bm_ct> o(new_ct(ctx, 2, a->limbs, a->scale));
    ev::rotate(c, a->buf.p(), 1, (int)a->limbs, g, key, o->buf.p(), false);
    sync(c);
    *out = o.release();
  });
}

int bm_op_drop(bm_ctx* ctx, const bm_ct* a, uint32_t limbs, bm_ct** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && a && out, BM_EINVAL, "NULL argument");
    same_ctx(ctx, a);
    REQUIRE(limbs >= 1 && limbs <= a->limbs, BM_ELEVEL, "cannot raise the level");
    Ctx& c = ctx->c;
    c.use_stream(nullptr);
    std::unique_ptr<bm_ct> o(new_ct(ctx, a->comps, limbs, a->scale));
    ev::drop(c, a->buf.p(), 1, (int)a->comps, (int)a->limbs, (int)limbs, o->buf.p());
    sync(c);
    *out = o.release();
  });
}

// ------------------------------------------------------------------ Blind-Match

static bm_masks* make_masks(bm_ctx* ctx, uint32_t d, uint32_t k, const int64_t* coeffs, double scale) {
  Ctx& c = ctx->c;
  std::unique_ptr<bm_masks> m(new bm_masks);
  m->ctx = ctx;
  m->d = d;
  m->k = k;
  m->scale = scale;
  m->pt = DBuf(&c, (size_t)k * c.mask_limbs() * c.N);
  ev::upload_plain(c, coeffs, (int)k, c.mask_limbs(), m->pt.p());
  return m.release();
}

// Library masks of Alg. 1 on the context's current stream, encoded at the
// scale of the last limb of a query with `ql` limbs.
bm_masks* bmx_create_masks(bm_ctx* ctx, uint32_t d, uint32_t k, uint32_t ql) {
  Ctx& c = ctx->c;
  bmx::check_shape(c, d, k);
  if (ql < 2 || (int)ql > c.L + 1) BM_THROW(BM_ELEVEL, "mask level out of range");
  const uint32_t cc = d / k;
  const double scale = (double)c.primes[ql - 1].q;
  std::vector<int64_t> coeffs((size_t)k * c.N);
  std::vector<double> slots(c.n);
  for (uint32_t i = 0; i < k; ++i) {
    for (size_t s = 0; s < c.n; ++s) slots[s] = ((s % d) / cc == i) ? 1.0 : 0.0;
    ring_encode(c, slots.data(), scale, coeffs.data() + (size_t)i * c.N);
  }
  return make_masks(ctx, d, k, coeffs.data(), scale);
}

// The enrollment masks of Sec. 3.2: mask_i has ones at slots [i c, (i+1) c),
// encoded at scale q_{limbs-1}; k plaintexts, cached in the context.
const bm_masks* bmx_enroll_masks(bm_ctx* ctx, uint32_t d, uint32_t k, uint32_t limbs) {
  Ctx& c = ctx->c;
  bmx::check_shape(c, d, k);
  if (limbs < 2 || (int)limbs > c.L + 1) BM_THROW(BM_ELEVEL, "mask level out of range");
  const uint64_t key = (2ULL << 62) | ((uint64_t)d << 40) | ((uint64_t)k << 20) | (uint64_t)limbs;
  auto it = ctx->mask_cache.find(key);
  if (it != ctx->mask_cache.end()) return it->second.get();
  const uint32_t cc = d / k;
  const double scale = (double)c.primes[limbs - 1].q;
  std::vector<int64_t> coeffs((size_t)k * c.N);
  std::vector<double> slots(c.n);
  for (uint32_t i = 0; i < k; ++i) {
    for (size_t s = 0; s < c.n; ++s) slots[s] = (s >= (size_t)i * cc && s < (size_t)(i + 1) * cc) ? 1.0 : 0.0;
    ring_encode(c, slots.data(), scale, coeffs.data() + (size_t)i * c.N);
  }
  bm_masks* m = make_masks(ctx, d, k, coeffs.data(), scale);
  return ctx->mask_cache.emplace(key, std::unique_ptr<bm_masks>(m)).first->second.get();
}

int bm_gallery_create(bm_ctx* ctx, uint32_t d, uint32_t k, uint64_t n_templates, uint32_t limbs,
                      bm_gallery** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && out, BM_EINVAL, "NULL argument");
    Ctx& c = ctx->c;
    bmx::check_shape(c, d, k);
    REQUIRE(n_templates > 0, BM_EINVAL, "empty gallery");
    REQUIRE(limbs >= 1 && (int)limbs <= c.L + 1, BM_ELEVEL, "limbs out of range");
    const uint64_t T = c.n / (d / k);
    c.use_stream(nullptr);
    std::unique_ptr<bm_gallery> g(new_gallery(ctx, d, k, limbs, (n_templates + T - 1) / T, n_templates,
                                              c.scale));
    kern::zero(c, g->buf.p(), g->buf.words());
    sync(c);
    *out = g.release();
  });
}

int bm_enroll(bm_ctx* ctx, const bm_evk* evk, bm_gallery* g, const bm_ct* const* users,
              const uint64_t* indices, size_t n, const bm_masks* masks, void* stream) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && evk && g && (n == 0 || (users && indices)), BM_EINVAL, "NULL argument");
    same_ctx(ctx, evk, g, masks);
    Ctx& c = ctx->c;
    c.use_stream(stream);
    if (n == 0) return;
    for (size_t i = 0; i < n; ++i) {
      REQUIRE(users[i], BM_EINVAL, "NULL user");
      same_ctx(ctx, users[i]);
    }
    const uint32_t ul = users[0]->limbs;
    REQUIRE(ul == g->limbs + 1, BM_ELEVEL, "users must sit one level above the gallery");
    const bm_masks* m = masks ? masks : bmx_enroll_masks(ctx, g->d, g->k, ul);
    REQUIRE(m->d == g->d && m->k == g->k, BM_EDIM, "masks do not match the gallery shape");
    std::vector<const u64*> ptrs(n);
    for (size_t u = 0; u < n; ++u) {
      REQUIRE(users[u] && users[u]->comps == 2 && users[u]->limbs == ul, BM_ELEVEL,
              "users must be fresh two-component ciphertexts of one level");
      REQUIRE(users[u]->scale * m->scale / (double)c.primes[ul - 1].q == g->scale, BM_ESCALE,
              "user and gallery scales differ");
      REQUIRE(indices[u] < g->n_templates, BM_EINVAL, "identifier beyond the gallery size");
      ptrs[u] = users[u]->buf.p();
    }
    bmx::enroll(c, evk, *g, ptrs.data(), (int)ul, indices, (int)n, m->pt.p());
  });
}

// The compression method's score mask: ones at slots b c (c = d/k), encoded
// at scale q_{limbs-1}; one plaintext, cached in the context.
const bm_masks* bmx_compress_mask(bm_ctx* ctx, uint32_t d, uint32_t k, uint32_t limbs) {
  Ctx& c = ctx->c;
  bmx::check_shape(c, d, k);
  if (limbs < 2 || (int)limbs > c.L + 1) BM_THROW(BM_ELEVEL, "mask level out of range");
  const uint64_t key = (1ULL << 62) | ((uint64_t)d << 40) | ((uint64_t)k << 20) | (uint64_t)limbs;
  auto it = ctx->mask_cache.find(key);
  if (it != ctx->mask_cache.end()) return it->second.get();
  const uint32_t cc = d / k;
  const double scale = (double)c.primes[limbs - 1].q;
  std::vector<int64_t> coeffs(c.N);
  std::vector<double> slots(c.n);
  for (size_t s = 0; s < c.n; ++s) slots[s] = s % cc == 0 ? 1.0 : 0.0;
  ring_encode(c, slots.data(), scale, coeffs.data());
  bm_masks* m = make_masks(ctx, d, 1, coeffs.data(), scale);
  m->k = k;
  return ctx->mask_cache.emplace(key, std::unique_ptr<bm_masks>(m)).first->second.get();
}

int bm_masks_create(bm_ctx* ctx, uint32_t d, uint32_t k, bm_masks** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && out, BM_EINVAL, "NULL argument");
    ctx->c.use_stream(nullptr);
    *out = bmx_create_masks(ctx, d, k, (uint32_t)ctx->c.L + 1);
  });
}

int bm_masks_import(bm_ctx* ctx, uint32_t d, uint32_t k, const int64_t* coeffs, double scale,
                    bm_masks** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && coeffs && out, BM_EINVAL, "NULL argument");
    bmx::check_shape(ctx->c, d, k);
    ctx->c.use_stream(nullptr);
    *out = make_masks(ctx, d, k, coeffs, scale);
  });
}

void bm_masks_free(bm_masks* m) {
  if (m) drop_graphs(m->ctx);
  delete m;
}

int bm_expand(bm_ctx* ctx, const bm_evk* evk, const bm_ct* q, const bm_masks* masks, bm_ct** outs) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && evk && q && masks && outs, BM_EINVAL, "NULL argument");
    same_ctx(ctx, evk, q, masks);
    REQUIRE(q->comps == 2, BM_EINVAL, "query must have 2 components");
    Ctx& c = ctx->c;
    REQUIRE(q->limbs >= 2, BM_ELEVEL, "query needs two limbs");
    REQUIRE(!q->query_d || q->query_d == masks->d, BM_EDIM, "query packed for another dimension than the masks");
    c.use_stream(nullptr);
    const uint32_t k = masks->k;
    const size_t nln = (size_t)(q->limbs - 1) * c.N;
    DBuf all(&c, (size_t)k * 2 * nln);
    bmx::expand(c, evk, q->buf.p(), (int)q->limbs, masks->pt.p(), masks->d, k, all.p());
    const double scale = q->scale * masks->scale / (double)c.primes[q->limbs - 1].q;
    std::vector<std::unique_ptr<bm_ct>> res;
    for (uint32_t i = 0; i < k; ++i) {
      res.emplace_back(new_ct(ctx, 2, q->limbs - 1, scale));
      HIP_OK(dev::memcpy_async(res.back()->buf.p(), all.p() + (size_t)i * 2 * nln, 2 * nln * sizeof(u64),
                            hipMemcpyDeviceToDevice, c.stream));
    }
    sync(c);
    for (uint32_t i = 0; i < k; ++i) outs[i] = res[i].release();
  });
}

using bmx::Plan;

// The plan of one match, checked against the query's level.
static Plan match_shape(const Ctx& c, const bm_ct* q, const bm_gallery* g, uint32_t schedule,
                        uint32_t out_limbs) {
  REQUIRE(q->comps == 2, BM_EINVAL, "query must have 2 components");
  REQUIRE(!q->query_d || q->query_d == g->d, BM_EDIM, "query packed for another dimension than the gallery");
  const Plan s = bmx::plan(c, schedule, g->k, (int)g->limbs, out_limbs);
  // the query is cut exactly to ql limbs: the gallery's level (k = 1) or one
  // above it (k > 1), lower under the minimum-level schedule
  REQUIRE((int)q->limbs >= s.ql, BM_ELEVEL,
          g->k == 1 ? "query below the gallery level" : "query must sit at least one level above the gallery");
  return s;
}

// Expansion (k > 1) and Alg. 2 for one query: q [2][q_limbs][N] -> out [G][2][ol][N]
static void match_body(Ctx& c, const bm_evk* evk, const u64* q, uint32_t q_limbs, const bm_gallery* g,
                       const bm_masks* m, const u64* cmask, const Plan& s, u64* out) {
  const uint32_t k = g->k;
  const u64* qq = q;
  DBuf cut;
  if ((int)q_limbs > s.ql) {             // exact level drop of the query to ql limbs
    cut = DBuf(&c, (size_t)2 * s.ql * c.N);
    ev::drop(c, q, 1, 2, (int)q_limbs, s.ql, cut.p());
    qq = cut.p();
  }
  const u64* cu = qq;
  DBuf expanded;
  if (k > 1) {
    expanded = DBuf(&c, (size_t)k * 2 * s.t * c.N);
    (s.hoist ? bmx::expand_hoisted : bmx::expand)(c, evk, qq, s.ql, m->pt.p(), g->d, k, expanded.p());
    cu = expanded.p();
  }
  bmx::match_groups(c, evk, s, cu, 1, 0, *g, cmask, out, 0);
}

// Replay (capturing on first use) the match of this shape as a HIP graph.
static void match_graph(Ctx& c, const bm_evk* evk, const bm_ct* q, const bm_gallery* g,
                        const bm_masks* m, const u64* cmask, const Plan& s, uint32_t schedule, u64* out) {
  const std::vector<uint64_t> key = {(uint64_t)evk, (uint64_t)evk->rlk.k.p(), (uint64_t)g->buf.p(),
                                     g->groups, g->k, g->d, g->limbs, (uint64_t)(m ? m->pt.p() : nullptr),
                                     (uint64_t)cmask, schedule, (uint64_t)s.ol, q->limbs, (uint64_t)c.stream,
                                     (uint64_t)c.group_chunk, (uint64_t)c.kip_variant, (uint64_t)c.ntt_views,
                                     (uint64_t)c.kip_order, (uint64_t)c.fused_occ, (uint64_t)c.col_src};
  const u64 n_out = bmx::out_cts(s, g->groups, g->d, g->k);
  GraphEntry* e = nullptr;
  for (auto& ge : c.graphs)
    if (ge->key == key) e = ge.get();
  // the graph's query slot holds the query already cut to the ql limbs the
  // match reads (the copy into it is the level drop)
  const size_t qw = (size_t)2 * s.ql * c.N, ow = (size_t)n_out * 2 * s.ol * c.N;
  if (!e) {
    std::unique_ptr<GraphEntry> ne(new GraphEntry);
    ne->key = key;
    ne->pool.reset(new DevicePool(c.device, c.hook));
    std::swap(c.pool, ne->pool);          // scratch of the capture comes from the graph's pool
    hipGraph_t graph = nullptr;
    bool capturing = false;
    // the hoisted rotation sum's fused ModDown writes every output word when
    // it lands on the output level directly: those epilogues then take their
    // output base from a device word, set to the caller's result by the
    // query copy in front of each replay (no copy out of out_slot)
    const bool by_ref = s.hoist && !s.comp && kern::fused_ok(c) && g->d / g->k > 1 && s.rot == s.ol;
    size_t covered = 0;
    try {
      ne->q_slot = DBuf(&c, qw);
      ne->out_slot = DBuf(&c, ow);
      if (by_ref) {
        ne->out_ref = DBuf(&c, 1);
        const u64* base = ne->out_slot.p();   // until a replay sets it: out_slot
        HIP_OK(dev::memcpy(ne->out_ref.p(), &base, sizeof(base), hipMemcpyHostToDevice));
        c.ref_dev = (u64* const*)ne->out_ref.p();
        c.ref_base = ne->out_slot.p();
        c.ref_words = ow;
        c.ref_hits = 0;
        c.ref_covered = 0;
      }
      HIP_OK(dev::begin_capture(c.stream));
      capturing = true;
      match_body(c, evk, ne->q_slot.p(), (uint32_t)s.ql, g, m, cmask, s, ne->out_slot.p());
      capturing = false;
      covered = c.ref_covered;
      c.ref_dev = nullptr;
      HIP_OK(dev::end_capture(c.stream, &graph));
      HIP_OK(dev::graph_instantiate(&ne->exec, graph));
      HIP_OK(dev::graph_destroy(graph));
    } catch (...) {
      c.ref_dev = nullptr;
      if (capturing) {
        hipGraph_t dead = nullptr;
        (void)dev::end_capture(c.stream, &dead);
        if (dead) (void)dev::graph_destroy(dead);
      }
      std::swap(c.pool, ne->pool);
      throw;
    }
    // every output word through the reference, or the copy as before (the
    // word then keeps pointing at out_slot)
    ne->by_ref = by_ref && covered == ow;
    std::swap(c.pool, ne->pool);
    if (c.graphs.size() >= 16) {
      HIP_OK(dev::stream_sync(c.stream));
      c.graphs.erase(c.graphs.begin());
    }
    c.graphs.push_back(std::move(ne));
    e = c.graphs.back().get();
  }
  if (e->by_ref) audit::check(out, ow * sizeof(u64), "match output");
  kern::copy_limbs(c, q->buf.p(), 0, (size_t)q->limbs * c.N, e->q_slot.p(), 1, qw, 0, qw / 2, 1, 2, s.ql,
                   e->by_ref ? (u64**)e->out_ref.p() : nullptr, out);
  HIP_OK(dev::graph_launch(e->exec, c.stream));
  if (!e->by_ref)
    kern::copy_limbs(c, e->out_slot.p(), 2 * (size_t)s.ol * c.N, (size_t)s.ol * c.N, out, 1,
                     2 * (size_t)s.ol * c.N, 0, (size_t)s.ol * c.N, (int)n_out, 2, s.ol);
}

// masks for this shape: the caller's, or the context's cached library masks
static const bm_masks* masks_for(bm_ctx* ctx, const bm_gallery* g, const bm_masks* masks, int ql) {
  if (masks) return masks;
  const uint64_t key = ((uint64_t)g->d << 40) | ((uint64_t)g->k << 20) | (uint64_t)ql;
  auto it = ctx->mask_cache.find(key);
  if (it == ctx->mask_cache.end())
    it = ctx->mask_cache.emplace(key, std::unique_ptr<bm_masks>(bmx_create_masks(ctx, g->d, g->k, ql))).first;
  return it->second.get();
}

// the compression mask of this shape (cached in the context), or NULL
static const u64* cmask_for(bm_ctx* ctx, const bm_gallery* g, const Plan& s) {
  if (!s.comp) return nullptr;
  return bmx_compress_mask(ctx, g->d, g->k, (uint32_t)s.rot)->pt.p();
}

static bm_result* new_result(bm_ctx* ctx, const bm_gallery* g, const Plan& s, double scale) {
  std::unique_ptr<bm_result> r(new bm_result);
  r->ctx = ctx;
  r->d = g->d;
  r->k = g->k;
  r->limbs = (uint32_t)s.ol;
  r->groups = bmx::out_cts(s, g->groups, g->d, g->k);
  r->packed = s.comp ? g->d / g->k : 0;
  r->n_templates = g->n_templates;
  r->scale = scale;
  return r.release();
}

static void match_one(bm_ctx* ctx, const bm_evk* evk, const bm_ct* q, const bm_gallery* g,
                      const bm_masks* masks, uint32_t schedule, uint32_t out_limbs, bm_result** out) {
  Ctx& c = ctx->c;
  const Plan s = match_shape(c, q, g, schedule, out_limbs);
  const uint32_t k = g->k;
  double cu_scale = q->scale;
  const bm_masks* m = nullptr;
  if (k > 1) {
    m = masks_for(ctx, g, masks, s.ql);
    REQUIRE(m->d == g->d && m->k == k, BM_EDIM, "masks do not match the gallery shape");
    cu_scale = q->scale * m->scale / (double)c.primes[s.ql - 1].q;
  }
  REQUIRE(cu_scale == g->scale, BM_ESCALE, "query and gallery scales differ");
  const u64* cm = cmask_for(ctx, g, s);
  std::unique_ptr<bm_result> r(new_result(ctx, g, s, bmx::result_scale(c, s, cu_scale, g->scale)));
  r->store = std::make_shared<DBuf>(&c, (size_t)r->groups * 2 * s.ol * c.N);
  if (c.use_graphs && !c.prof->on)
    match_graph(c, evk, q, g, m, cm, s, schedule, r->p());
  else
    match_body(c, evk, q->buf.p(), q->limbs, g, m, cm, s, r->p());
  *out = r.release();
}

int bm_match(bm_ctx* ctx, const bm_evk* evk, const bm_ct* q, const bm_gallery* g, const bm_masks* masks,
             uint32_t schedule, uint32_t out_limbs, void* stream, bm_result** out) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && evk && q && g && out, BM_EINVAL, "NULL argument");
    same_ctx(ctx, evk, q, g, masks);
    ctx->c.use_stream(stream);
    match_one(ctx, evk, q, g, masks, schedule, out_limbs, out);
  });
}

// The match of bm_match on caller buffers, its scratch carved out of the
// device's scratch array: walked once on the host (no launch, no HIP call) to
// measure the scratch it needs and to run every launch check, then enqueued.
int bm_match_noalloc(bm_ctx* ctx, const bm_evk* evk, const uint64_t* q_words, uint32_t q_limbs, double q_scale,
                     const bm_gallery* g, const bm_masks* masks, uint32_t schedule, uint32_t out_limbs,
                     uint64_t* out_words, size_t n_out_words, size_t* needed_words, double* out_scale,
                     void* stream) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && evk && q_words && g && needed_words, BM_EINVAL, "NULL argument");
    same_ctx(ctx, evk, g, masks);
    REQUIRE(!(schedule & BM_COMPRESS), BM_EINVAL, "the no-allocation match does not compress");
    Ctx& c = ctx->c;
    const Plan s = bmx::plan(c, schedule, g->k, (int)g->limbs, out_limbs);
    REQUIRE((int)q_limbs >= s.ql && (int)q_limbs <= c.L + 1, BM_ELEVEL,
            g->k == 1 ? "query below the gallery level" : "query must sit at least one level above the gallery");
    const size_t need = (size_t)g->groups * 2 * s.ol * c.N;
    *needed_words = need;
    if (!out_words) return;
    REQUIRE(n_out_words == need, BM_EINVAL, "output must hold groups * 2 * out_limbs * N words");
    const bm_masks* m = nullptr;
    double cu_scale = q_scale;
    if (g->k > 1) {
      REQUIRE(masks, BM_EINVAL, "a gallery with k > 1 needs masks made beforehand");
      REQUIRE(masks->d == g->d && masks->k == g->k, BM_EDIM, "masks do not match the gallery shape");
      m = masks;
      cu_scale = q_scale * m->scale / (double)c.primes[s.ql - 1].q;
    }
    REQUIRE(cu_scale == g->scale, BM_ESCALE, "query and gallery scales differ");
    c.use_stream(stream);
    audit::Scoped reg_q(q_words, (size_t)2 * q_limbs * c.N * sizeof(u64));
    audit::Scoped reg_o(out_words, need * sizeof(u64));
    void* base = kern::noalloc_scratch(c.device);
    auto run = [&](bool sizing) {
      std::shared_ptr<DevicePool> arena = std::make_shared<DevicePool>(c.device, base, NOALLOC_SCRATCH_BYTES);
      std::swap(c.pool, arena);
      try {
        if (sizing) {
          dev::SizingScope walk;
          match_body(c, evk, q_words, q_limbs, g, m, nullptr, s, out_words);
        } else {
          match_body(c, evk, q_words, q_limbs, g, m, nullptr, s, out_words);
        }
      } catch (...) {
        std::swap(c.pool, arena);
        throw;
      }
      std::swap(c.pool, arena);
    };
    run(true);    // BM_ENOMEM (nothing enqueued) when the scratch is too small
    run(false);
    if (out_scale) *out_scale = bmx::result_scale(c, s, cu_scale, g->scale);
  });
}

// ---------------------------------------------------------------- batched matching
//
// A batch of (query, gallery) pairs of any shapes.  Pairs whose galleries share
// a shape (d, k, stored limbs) form one class: the class's distinct queries
// are expanded together (one batch of query x part elements), and Alg. 2 runs
// over every (pair, gallery group) element of the class in passes of the
// context's group chunk, whatever gallery an element comes from.  The words
// are those of per-pair bm_match (every operation is exact and element-wise
// across a batch).

using bmx::BatchClass;
using bmx::BatchPlan;

static BatchPlan plan_batch(bm_ctx* ctx, const bm_ct* const* qs, const bm_gallery* const* gs, size_t n,
                            uint32_t schedule, uint32_t out_limbs) {
  Ctx& c = ctx->c;
  BatchPlan bp;
  bp.out_off.resize(n);
  bp.scale.resize(n);
  for (size_t i = 0; i < n; ++i) {
    const bm_ct* q = qs[i];
    const bm_gallery* g = gs[i];
    const Plan s = match_shape(c, q, g, schedule, out_limbs);
    BatchClass* K = nullptr;
    for (auto& cl : bp.cls)
      if (cl.shape->d == g->d && cl.shape->k == g->k && cl.shape->limbs == g->limbs) K = &cl;
    if (!K) {
      bp.cls.emplace_back();
      K = &bp.cls.back();
      K->shape = g;
      K->s = s;
      if (g->k > 1) K->masks = masks_for(ctx, g, nullptr, s.ql);
      K->cmask = cmask_for(ctx, g, s);
    }
    double cu_scale = q->scale;
    if (g->k > 1) cu_scale = q->scale * K->masks->scale / (double)c.primes[s.ql - 1].q;
    REQUIRE(cu_scale == g->scale, BM_ESCALE, "query and gallery scales differ");
    int j = 0;
    while (j < (int)K->queries.size() && K->queries[j] != q) ++j;
    if (j == (int)K->queries.size()) K->queries.push_back(q);
    K->pairs.push_back(i);
    K->qidx.push_back(j);
    bp.out_off[i] = bp.out_words;
    bp.scale[i] = bmx::result_scale(c, s, cu_scale, g->scale);
    bp.out_words += (size_t)bmx::out_cts(s, g->groups, g->d, g->k) * 2 * s.ol * c.N;
  }
  return bp;
}

static void batch_eager(Ctx& c, const bm_evk* evk, const BatchPlan& bp, const bm_gallery* const* gs, u64* out) {
  for (const BatchClass& K : bp.cls) {
    DBuf qb(&c, K.queries.size() * 2 * (size_t)K.s.ql * c.N);
    bmx::load_queries(c, K, qb.p());
    bmx::class_body(c, evk, bp, K, gs, qb.p(), out);
  }
}

// Replay (capturing on first use) the batch as one HIP graph: the queries are
// copied into the graph's per-class slots, the results out of its output slot.
static void batch_graph(Ctx& c, const bm_evk* evk, const BatchPlan& bp, const bm_ct* const* qs,
                        const bm_gallery* const* gs, size_t n, uint32_t schedule, uint32_t out_limbs, u64* out) {
  std::vector<uint64_t> key = {0xBA7C4ULL, (uint64_t)evk, (uint64_t)evk->rlk.k.p(), schedule, out_limbs,
                               (uint64_t)c.stream, (uint64_t)c.group_chunk, (uint64_t)c.kip_variant,
                               (uint64_t)c.ntt_views, (uint64_t)c.kip_order, (uint64_t)c.fused_occ,
                               (uint64_t)c.col_src, n};
  for (const BatchClass& K : bp.cls) {
    key.push_back((uint64_t)(K.masks ? K.masks->pt.p() : nullptr));
    key.push_back((uint64_t)K.cmask);
    key.push_back(K.queries.size());
    for (size_t pi = 0; pi < K.pairs.size(); ++pi) {
      const bm_gallery* g = gs[K.pairs[pi]];
      key.insert(key.end(), {K.pairs[pi], (uint64_t)K.qidx[pi], (uint64_t)g->buf.p(), g->groups, g->d, g->k,
                             g->limbs, qs[K.pairs[pi]]->limbs});
    }
  }
  GraphEntry* e = nullptr;
  for (auto& ge : c.graphs)
    if (ge->key == key) e = ge.get();
  if (!e) {
    std::unique_ptr<GraphEntry> ne(new GraphEntry);
    ne->key = key;
    ne->pool.reset(new DevicePool(c.device, c.hook));
    std::swap(c.pool, ne->pool);          // scratch of the capture comes from the graph's pool
    hipGraph_t graph = nullptr;
    bool capturing = false;
    try {
      for (const BatchClass& K : bp.cls) ne->slots.emplace_back(&c, K.queries.size() * 2 * (size_t)K.s.ql * c.N);
      ne->out_slot = DBuf(&c, bp.out_words);
      HIP_OK(dev::begin_capture(c.stream));
      capturing = true;
      for (size_t ci = 0; ci < bp.cls.size(); ++ci)
        bmx::class_body(c, evk, bp, bp.cls[ci], gs, ne->slots[ci].p(), ne->out_slot.p());
      capturing = false;
      HIP_OK(dev::end_capture(c.stream, &graph));
      HIP_OK(dev::graph_instantiate(&ne->exec, graph));
      HIP_OK(dev::graph_destroy(graph));
    } catch (...) {
      if (capturing) {
        hipGraph_t dead = nullptr;
        (void)dev::end_capture(c.stream, &dead);
        if (dead) (void)dev::graph_destroy(dead);
      }
      std::swap(c.pool, ne->pool);
      throw;
    }
    std::swap(c.pool, ne->pool);
    if (c.graphs.size() >= 16) {
      HIP_OK(dev::stream_sync(c.stream));
      c.graphs.erase(c.graphs.begin());
    }
    c.graphs.push_back(std::move(ne));
    e = c.graphs.back().get();
  }
  for (size_t ci = 0; ci < bp.cls.size(); ++ci) bmx::load_queries(c, bp.cls[ci], e->slots[ci].p());
  HIP_OK(dev::graph_launch(e->exec, c.stream));
  // the results: rows of N words, up to 65,535 rows per launch
  const size_t rows = bp.out_words / c.N;
  for (size_t r0 = 0; r0 < rows; r0 += 65535) {
    const int nr = (int)std::min<size_t>(65535, rows - r0);
    kern::copy_limbs(c, e->out_slot.p() + r0 * c.N, c.N, 0, out + r0 * c.N, 1, c.N, 0, 0, nr, 1, 1);
  }
}

static void match_batch_impl(bm_ctx* ctx, const bm_evk* evk, const bm_ct* const* qs, const bm_gallery* const* gs,
                             size_t n_pairs, uint32_t schedule, uint32_t out_limbs,
                             std::vector<std::unique_ptr<bm_result>>& res) {
  Ctx& c = ctx->c;
  const BatchPlan bp = plan_batch(ctx, qs, gs, n_pairs, schedule, out_limbs);
  auto store = std::make_shared<DBuf>(&c, bp.out_words);
  if (c.use_graphs && !c.prof->on)
    batch_graph(c, evk, bp, qs, gs, n_pairs, schedule, out_limbs, store->p());
  else
    batch_eager(c, evk, bp, gs, store->p());
  res.clear();
  res.resize(n_pairs);
  for (const BatchClass& K : bp.cls)
    for (size_t p : K.pairs) {
      res[p].reset(new_result(ctx, gs[p], K.s, bp.scale[p]));
      res[p]->store = store;
      res[p]->off = bp.out_off[p];
    }
}

static void check_pairs(bm_ctx* ctx, const bm_evk* evk, const bm_ct* const* qs, const bm_gallery* const* gs,
                        size_t n_pairs) {
  REQUIRE(ctx && evk && qs && gs, BM_EINVAL, "NULL argument");
  REQUIRE(n_pairs > 0, BM_EINVAL, "empty batch");
  same_ctx(ctx, evk);
  for (size_t i = 0; i < n_pairs; ++i) {
    REQUIRE(qs[i] && gs[i], BM_EINVAL, "NULL pair");
    same_ctx(ctx, qs[i], gs[i]);
  }
}

int bm_match_batch(bm_ctx* ctx, const bm_evk* evk, const bm_ct* const* qs, const bm_gallery* const* gs,
                   size_t n_pairs, uint32_t schedule, uint32_t out_limbs, void* stream, bm_result** outs) {
  return guarded(ctx, [&] {
    REQUIRE(outs, BM_EINVAL, "NULL argument");
    check_pairs(ctx, evk, qs, gs, n_pairs);
    ctx->c.use_stream(stream);
    std::vector<std::unique_ptr<bm_result>> res;
    match_batch_impl(ctx, evk, qs, gs, n_pairs, schedule, out_limbs, res);
    for (size_t i = 0; i < n_pairs; ++i) outs[i] = res[i].release();
  });
}

int bm_ctx_set_tuning(bm_ctx* ctx, const bm_tuning* t) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && t, BM_EINVAL, "NULL argument");
    REQUIRE(t->group_chunk <= 4096, BM_EINVAL, "group_chunk above 4096");
    REQUIRE(t->kip_variant <= 4, BM_EINVAL, "kip_variant in 0..4");
    REQUIRE(t->ntt_row_views == 0 || t->ntt_row_views == 4 || t->ntt_row_views == 8 || t->ntt_row_views == 16,
            BM_EINVAL, "ntt_row_views: 0, 4, 8 or 16");
    REQUIRE(t->kip_order <= 3, BM_EINVAL, "kip_order: 0 to 3");
    REQUIRE(t->fused_occupancy == 0 || t->fused_occupancy == 3 || t->fused_occupancy == 4, BM_EINVAL,
            "fused_occupancy: 0, 3 or 4");
    REQUIRE(t->column_sources <= 1, BM_EINVAL, "column_sources: 0 or 1");
    Ctx& c = ctx->c;
    c.group_chunk = (int)t->group_chunk;
    c.kip_variant = (int)t->kip_variant;
    c.ntt_views = (int)t->ntt_row_views;
    c.kip_order = (int)t->kip_order;
    c.fused_occ = (int)t->fused_occupancy;
    c.col_src = (int)t->column_sources;
  });
}

int bm_ctx_get_tuning(const bm_ctx* ctx, bm_tuning* t) {
  if (!ctx || !t) return BM_EINVAL;
  t->group_chunk = (uint32_t)ctx->c.group_chunk;
  t->kip_variant = (uint32_t)ctx->c.kip_variant;
  t->ntt_row_views = (uint32_t)ctx->c.ntt_views;
  t->kip_order = (uint32_t)ctx->c.kip_order;
  t->fused_occupancy = (uint32_t)ctx->c.fused_occ;
  t->column_sources = (uint32_t)ctx->c.col_src;
  return BM_OK;
}

// Times the batch under every schedule offered (skipping those whose keys or
// levels the inputs lack), then, under the fastest, each result-invariant
// knob in turn (coordinate descent: group chunk, key inner product variant
// and block order, row-pass tiling, fused-pass occupancy, where the source
// limbs' inverse column pass runs), checking that every knob setting gives
// the words of the first and last pair that the default setting gave.
int bm_autotune_batch(bm_ctx* ctx, const bm_evk* evk, const bm_ct* const* qs, const bm_gallery* const* gs,
                      size_t n_pairs, const uint32_t* schedules, size_t n_schedules, uint32_t out_limbs,
                      uint32_t* best_schedule, bm_tuning* best, double* best_ms) {
  return guarded(ctx, [&] {
    check_pairs(ctx, evk, qs, gs, n_pairs);
    REQUIRE(schedules && n_schedules > 0, BM_EINVAL, "no schedule to tune");
    Ctx& c = ctx->c;
    c.use_stream(nullptr);
    const int s_chunk = c.group_chunk, s_var = c.kip_variant, s_views = c.ntt_views, s_order = c.kip_order,
              s_occ = c.fused_occ, s_src = c.col_src;
    hipEvent_t ea, eb;
    HIP_OK(dev::event_create(&ea, true));
    HIP_OK(dev::event_create(&eb, true));
    std::vector<std::unique_ptr<bm_result>> res;
    auto words = [&]() {                       // all groups of the first and last pair
      std::vector<u64> w;
      for (size_t p : {(size_t)0, n_pairs - 1}) {
        const bm_result& r = *res[p];
        std::vector<u64> h((size_t)r.groups * 2 * r.limbs * c.N);
        ev::export_coeffs(c, r.p(), (int)(2 * r.groups), (int)r.limbs, h.data());
        w.insert(w.end(), h.begin(), h.end());
      }
      return w;
    };
    auto drop = [&] {                          // a candidate's graph and scratch are not kept
      HIP_OK(dev::stream_sync(c.stream));
      c.graphs.clear();
    };
    // a setting's time: the best of five timed runs (three for batches of
    // 20 ms and more), each of enough batches to last about 5 ms (short
    // batches are timed over many)
    int reps = 0;
    auto timed = [&](uint32_t sched) {
      drop();
      match_batch_impl(ctx, evk, qs, gs, n_pairs, sched, out_limbs, res);   // warm-up, capture
      res.clear();
      double best_run = 1e30;
      for (int run = 0; run < (best_run < 20.0 ? 5 : 3); ++run) {
        const int n = reps > 0 ? reps : 1;
        HIP_OK(dev::event_record(ea, c.stream));
        for (int rep = 0; rep < n; ++rep) match_batch_impl(ctx, evk, qs, gs, n_pairs, sched, out_limbs, res);
        HIP_OK(dev::event_record(eb, c.stream));
        HIP_OK(dev::event_sync(eb));
        float ms = 0;
        HIP_OK(dev::event_elapsed(&ms, ea, eb));
        best_run = std::min(best_run, (double)ms / n);
        if (reps == 0) reps = (int)std::min(200.0, std::max(1.0, std::ceil(5.0 / std::max(ms, 1e-3f))));
      }
      return best_run;
    };
    double bms = 1e30;
    uint32_t bsched = 0;
    try {
      for (size_t i = 0; i < n_schedules; ++i) {
        double ms;
        try {
          ms = timed(schedules[i]);
        } catch (const Error& e) {
          if (e.code != BM_ENOKEY && e.code != BM_ELEVEL) throw;
          continue;                             // this schedule is not available for these inputs
        }
        if (ms < bms) {
          bms = ms;
          bsched = schedules[i];
        }
      }
      REQUIRE(bsched != 0, BM_ENOKEY, "no offered schedule can run on these inputs");
      (void)timed(bsched);
      const std::vector<u64> ref = words();
      // each knob's values (the current one among them) are timed one after
      // another and the fastest kept, so that a knob is judged against
      // measurements of the same moment rather than an earlier best
      int* knob[6] = {&c.group_chunk, &c.kip_variant, &c.kip_order, &c.ntt_views, &c.fused_occ, &c.col_src};
      const std::vector<int> values[6] = {{8, 16, 32, 64, 128}, {0, 1, 2, 3, 4}, {0, 1, 2, 3}, {16, 8, 4}, {0, 3, 4},
                                          {0, 1}};
      for (int kn = 0; kn < 6; ++kn) {
        int pick = *knob[kn];
        double pick_ms = 1e30;
        for (int v : values[kn]) {
          *knob[kn] = v;
          const double ms = timed(bsched);
          if (!dev::dry() && words() != ref)   // (a dry run computes nothing to compare)
            BM_THROW(BM_EDEVICE, "a result-invariant knob changed the result words");
          if (ms < pick_ms) {
            pick_ms = ms;
            pick = v;
          }
        }
        *knob[kn] = pick;
        bms = pick_ms;
      }
    } catch (...) {
      res.clear();
      (void)dev::stream_sync(c.stream);
      c.graphs.clear();
      c.group_chunk = s_chunk;
      c.kip_variant = s_var;
      c.ntt_views = s_views;
      c.kip_order = s_order;
      c.fused_occ = s_occ;
      c.col_src = s_src;
      (void)dev::event_destroy(ea);
      (void)dev::event_destroy(eb);
      throw;
    }
    res.clear();
    drop();
    (void)dev::event_destroy(ea);
    (void)dev::event_destroy(eb);
    if (best_schedule) *best_schedule = bsched;
    if (best) {
      best->group_chunk = (uint32_t)c.group_chunk;
      best->kip_variant = (uint32_t)c.kip_variant;
      best->ntt_row_views = (uint32_t)c.ntt_views;
      best->kip_order = (uint32_t)c.kip_order;
      best->fused_occupancy = (uint32_t)c.fused_occ;
      best->column_sources = (uint32_t)c.col_src;
    }
    if (best_ms) *best_ms = bms;
  });
}

int bm_autotune(bm_ctx* ctx, const bm_evk* evk, const bm_ct* q, const bm_gallery* g, uint32_t schedule,
                uint32_t* best_chunk, double* best_ms) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && evk && q && g, BM_EINVAL, "NULL argument");
    same_ctx(ctx, evk, q, g);
    Ctx& c = ctx->c;
    c.use_stream(nullptr);
    const bool graphs = c.use_graphs;
    const int saved = c.group_chunk;
    hipEvent_t a, b;
    HIP_OK(dev::event_create(&a, true));
    HIP_OK(dev::event_create(&b, true));
    double best = 1e30;
    int pick = saved;
    try {
      for (int chunk : {1, 2, 4, 8, 16, 32, 64}) {
        if (chunk > 1 && (u64)(chunk / 2) >= g->groups) break;   // larger chunks change nothing
        c.group_chunk = chunk;
        bm_result* r = nullptr;
        match_one(ctx, evk, q, g, nullptr, schedule, 0, &r);    // warm-up (and capture)
        bm_result_free(r);
        HIP_OK(dev::event_record(a, c.stream));
        for (int rep = 0; rep < 3; ++rep) {
          match_one(ctx, evk, q, g, nullptr, schedule, 0, &r);
          bm_result_free(r);
        }
        HIP_OK(dev::event_record(b, c.stream));
        HIP_OK(dev::event_sync(b));
        float ms = 0;
        HIP_OK(dev::event_elapsed(&ms, a, b));
        if (ms / 3 < best) {
          best = ms / 3;
          pick = chunk;
        }
      }
    } catch (...) {
      c.group_chunk = saved;
      (void)dev::event_destroy(a);
      (void)dev::event_destroy(b);
      throw;
    }
    (void)dev::event_destroy(a);
    (void)dev::event_destroy(b);
    c.group_chunk = pick;
    c.use_graphs = graphs;
    if (best_chunk) *best_chunk = (uint32_t)pick;
    if (best_ms) *best_ms = best;
  });
}

int bm_result_info(const bm_result* r, uint64_t* groups, uint32_t* limbs, double* scale) {
  if (!r) return BM_EINVAL;
  if (groups) *groups = r->groups;
  if (limbs) *limbs = r->limbs;
  if (scale) *scale = r->scale;
  return BM_OK;
}

int bm_result_export(const bm_result* r, uint64_t group, uint64_t* words, size_t n_words) {
  if (!r) return BM_EINVAL;
  bm_ctx* ctx = r->ctx;
  return guarded(ctx, [&] {
    Ctx& c = ctx->c;
    REQUIRE(group < r->groups, BM_EINVAL, "group out of range");
    REQUIRE(words && n_words == (size_t)2 * r->limbs * c.N, BM_EINVAL, "size");
    c.use_stream(nullptr);
    ev::export_coeffs(c, r->p() + group * 2 * (size_t)r->limbs * c.N, 2, (int)r->limbs, words);
  });
}

int bm_result_export_all(const bm_result* r, uint64_t* words, size_t n_words) {
  if (!r) return BM_EINVAL;
  bm_ctx* ctx = r->ctx;
  return guarded(ctx, [&] {
    Ctx& c = ctx->c;
    REQUIRE(words && n_words == (size_t)r->groups * 2 * r->limbs * c.N, BM_EINVAL, "size");
    c.use_stream(nullptr);
    ev::export_coeffs(c, r->p(), (int)(2 * r->groups), (int)r->limbs, words);
  });
}

void bm_result_free(bm_result* r) { delete r; }

int bm_decrypt_scores(bm_ctx* ctx, const bm_sk* sk, const bm_result* r, double* scores, uint64_t n) {
  return guarded(ctx, [&] {
    REQUIRE(ctx && sk && r && scores, BM_EINVAL, "NULL argument");
    same_ctx(ctx, sk, r);
    REQUIRE(n == r->n_templates, BM_EINVAL, "n must equal the gallery size");
    Ctx& c = ctx->c;
    c.use_stream(nullptr);
    const uint32_t cc = r->d / r->k;
    const uint64_t T = c.n / cc;
    const uint64_t per = r->packed ? r->packed : 1;   // groups per result ciphertext
    std::vector<double> m(c.N), re(c.n);
    for (uint64_t o = 0; o < r->groups; ++o) {
      ev::decrypt_coeffs(c, sk, r->p() + o * 2 * (size_t)r->limbs * c.N, 2, (int)r->limbs, m.data());
      ring_decode(c, m.data(), r->scale, re.data());
      for (uint64_t j = 0; j < per; ++j) {
        const uint64_t g = o * per + j;
        for (uint64_t b = 0; b < T; ++b) {
          const uint64_t tid = g * T + b;
          if (tid < n) scores[tid] = re[b * cc + (r->packed ? j : 0)];
        }
      }
    }
  });
}

int bm_top1(const double* scores, uint64_t n, double threshold, int64_t* idx, double* best) {
  if (!scores || !idx || n == 0) return BM_EINVAL;
  uint64_t bi = 0;
  for (uint64_t i = 1; i < n; ++i)
    if (scores[i] > scores[bi]) bi = i;
  if (best) *best = scores[bi];
  *idx = scores[bi] < threshold ? -1 : (int64_t)bi;
  return BM_OK;
}

}  // extern "C"
