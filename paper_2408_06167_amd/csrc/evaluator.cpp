// evaluator.cpp -- CKKS operations over batches of RNS ciphertexts, issued as
// sequences of kernel launches on the context's stream.
#include "evaluator.hpp"

#include <algorithm>
#include <cstring>
#include <thread>

namespace bm {

// ----------------------------------------------------------------- memory

namespace audit {
namespace {
std::mutex g_mu;
std::map<uintptr_t, size_t>& live() {
  static std::map<uintptr_t, size_t> m;
  return m;
}
}  // namespace

void add(const void* p, size_t bytes) {
  std::lock_guard<std::mutex> g(g_mu);
  live()[(uintptr_t)p] = bytes;
}

void remove(const void* p) {
  std::lock_guard<std::mutex> g(g_mu);
  live().erase((uintptr_t)p);
}

void check(const void* p, size_t bytes, const char* what) {
  if (!p) BM_THROW(BM_EINVAL, std::string("launch check: null operand of ") + what);
  std::lock_guard<std::mutex> g(g_mu);
  const uintptr_t a = (uintptr_t)p;
  auto it = live().upper_bound(a);
  if (it != live().begin()) {
    --it;
    if (a >= it->first && a + bytes <= it->first + it->second) return;
  }
  BM_THROW(BM_EINVAL, std::string("launch check: ") + what + " would access outside its buffer");
}
}  // namespace audit

DevicePool::DevicePool(int device, void* base, size_t bytes)
    : arena_((char*)base), arena_bytes_(bytes), device_(device) {
  if (bytes) arena_free_[0] = bytes;
}

DevicePool::~DevicePool() {
  std::lock_guard<std::mutex> g(mu_);
  if (!arena_) free_cached();
}

void* DevicePool::arena_alloc(size_t bytes) {
  const size_t need = (bytes + 255) & ~(size_t)255;
  for (auto it = arena_free_.begin(); it != arena_free_.end(); ++it) {
    if (it->second < need) continue;
    const size_t off = it->first, len = it->second;
    arena_free_.erase(it);
    if (len > need) arena_free_[off + need] = len - need;
    held_ += need;
    peak_ = std::max(peak_, off + need);
    return arena_ + off;
  }
  BM_THROW(BM_ENOMEM, "scratch exhausted: " + std::to_string(bytes) + " more bytes needed beyond the " +
                          std::to_string(arena_bytes_) + "-byte scratch");
}

void DevicePool::arena_release(void* p, size_t bytes) {
  const size_t need = (bytes + 255) & ~(size_t)255;
  size_t off = (size_t)((char*)p - arena_), len = need;
  held_ -= need;
  auto next = arena_free_.lower_bound(off);
  if (next != arena_free_.end() && next->first == off + len) {     // merge with the following range
    len += next->second;
    next = arena_free_.erase(next);
  }
  if (next != arena_free_.begin()) {                                // and with the preceding one
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      off = prev->first;
      len += prev->second;
      arena_free_.erase(prev);
    }
  }
  arena_free_[off] = len;
}

// Frees the cached blocks, each to the allocator it came from; a caller's
// allocator may hand a block to other work at once, so the device finishes
// what is queued first.
void DevicePool::free_cached() {
  bool synced = false;
  for (auto& kv : free_) {
    void* p = kv.second;
    audit::remove(p);
    held_ -= kv.first;
    auto h = hooked_.find(p);
    if (h == hooked_.end()) {
      (void)dev::free(p);
      continue;
    }
    if (!synced) {
      (void)dev::set_device(device_);
      (void)dev::device_sync();
      synced = true;
    }
    h->second->free(p, h->second->user);
    hooked_.erase(h);
  }
  free_.clear();
  cached_ = 0;
}

void* DevicePool::new_block(size_t bytes) {
  if (hook_) {
    void* p = hook_->alloc(bytes, hook_->user);
    if (p) hooked_[p] = hook_;
    return p;
  }
  void* p = nullptr;
  if (dev::malloc(&p, bytes) != hipSuccess) {
    (void)dev::last_error();
    return nullptr;
  }
  return p;
}

void* DevicePool::alloc(size_t bytes) {
  std::lock_guard<std::mutex> g(mu_);
  if (arena_) return arena_alloc(bytes);
  auto it = free_.find(bytes);
  if (it != free_.end()) {
    void* p = it->second;
    free_.erase(it);
    cached_ -= bytes;
    return p;
  }
  void* p = new_block(bytes);
  if (!p) {
    free_cached();   // release cached blocks and retry once
    p = new_block(bytes);
    if (!p) BM_THROW(BM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  audit::add(p, bytes);
  held_ += bytes;
  return p;
}

void DevicePool::release(void* p, size_t bytes) {
  std::lock_guard<std::mutex> g(mu_);
  if (arena_) {
    arena_release(p, bytes);
    return;
  }
  free_.emplace(bytes, p);
  cached_ += bytes;
}

void DevicePool::trim() {
  std::lock_guard<std::mutex> g(mu_);
  if (!arena_) free_cached();
}

void DevicePool::set_hook(std::shared_ptr<const AllocHook> hook) {
  std::lock_guard<std::mutex> g(mu_);
  if (arena_) BM_THROW(BM_EINVAL, "an arena pool takes no allocator");
  free_cached();
  hook_ = std::move(hook);
}

DBuf::DBuf(Ctx* c, size_t words) : pool_(c->pool), words_(words) {
  p_ = words ? (u64*)pool_->alloc(words * sizeof(u64)) : nullptr;
}

DBuf::~DBuf() {
  if (p_) pool_->release(p_, words_ * sizeof(u64));
}

DBuf& DBuf::operator=(DBuf&& o) noexcept {
  if (this != &o) {
    if (p_) pool_->release(p_, words_ * sizeof(u64));
    pool_ = std::move(o.pool_);
    p_ = o.p_;
    words_ = o.words_;
    o.p_ = nullptr;
    o.words_ = 0;
  }
  return *this;
}

GraphEntry::~GraphEntry() {
  if (exec && !dev::dry()) (void)hipGraphExecDestroy(exec);
  q_slot = DBuf();
  out_slot = DBuf();
  slots.clear();
}

void Ctx::use_stream(void* s) {
  hipStream_t want = s ? (hipStream_t)s : own_stream;
  if (want != stream) {
    if (stream) HIP_OK(dev::stream_sync(stream));
    stream = want;
  }
}

Ctx::~Ctx() {
  if (stream) (void)dev::stream_sync(stream);
  graphs.clear();
  pool.reset();
  if (owns_tables)
    for (void* p : {(void*)d_primes, (void*)d_tw, (void*)d_tws, (void*)d_itw, (void*)d_itws, (void*)d_twf,
                    (void*)d_twq, (void*)d_itwf, (void*)d_itwq, (void*)d_ci, (void*)d_modup, (void*)d_moddown,
                    (void*)d_rescale})
      if (p) {
        audit::remove(p);
        (void)dev::free(p);
      }
  if (own_stream) (void)dev::stream_destroy(own_stream);
}

std::unique_ptr<Ctx> Ctx::make_lane() const {
  std::unique_ptr<Ctx> l(new Ctx);
  l->device = device;
  l->log_n = log_n;
  l->N = N;
  l->n = n;
  l->ci = ci;
  l->M = M;
  l->L = L;
  l->K = K;
  l->alpha = alpha;
  l->dnum = dnum;
  l->scale = scale;
  l->sigma = sigma;
  l->out_limbs = out_limbs;
  l->primes = primes;
  l->cdt = cdt;
  l->d_primes = d_primes;
  l->d_tw = d_tw;
  l->d_tws = d_tws;
  l->d_itw = d_itw;
  l->d_itws = d_itws;
  l->d_twf = d_twf;
  l->d_twq = d_twq;
  l->d_itwf = d_itwf;
  l->d_itwq = d_itwq;
  l->d_ci = d_ci;
  l->d_modup = d_modup;
  l->d_moddown = d_moddown;
  l->d_rescale = d_rescale;
  l->h_modup = h_modup;
  l->h_moddown = h_moddown;
  l->group_chunk = group_chunk;
  l->kip_variant = kip_variant;
  l->ntt_views = ntt_views;
  l->kip_order = kip_order;
  l->fused_occ = fused_occ;
  l->col_src = col_src;
  l->owns_tables = false;
  l->prof = prof;
  HIP_OK(dev::set_device(device));
  HIP_OK(dev::stream_create(&l->own_stream));
  l->stream = l->own_stream;
  l->hook = hook;
  l->pool.reset(new DevicePool(device, hook));
  return l;
}

// ----------------------------------------------------------------- profiler

hipEvent_t Profiler::take() {
  if (!spare_.empty()) {
    hipEvent_t e = spare_.back();
    spare_.pop_back();
    return e;
  }
  hipEvent_t e;
  HIP_OK(dev::event_create(&e, true));
  return e;
}

std::pair<hipEvent_t, hipEvent_t> Profiler::begin(const char* name, double bytes, double ops) {
  std::lock_guard<std::mutex> g(mu_);
  Pending p{name, take(), take(), bytes, ops};
  pending_.push_back(p);
  return {p.a, p.b};
}

void Profiler::collect() {
  std::lock_guard<std::mutex> g(mu_);
  for (auto& p : pending_) {
    HIP_OK(dev::event_sync(p.b));
    float ms = 0;
    HIP_OK(dev::event_elapsed(&ms, p.a, p.b));
    Entry& e = entries[p.name];
    e.launches += 1;
    e.ms += ms;
    e.bytes += p.bytes;
    e.ops += p.ops;
    spare_.push_back(p.a);
    spare_.push_back(p.b);
  }
  pending_.clear();
}

void Profiler::reset() {
  collect();
  std::lock_guard<std::mutex> g(mu_);
  entries.clear();
}

Profiler::~Profiler() {
  for (auto& p : pending_) {
    (void)dev::event_destroy(p.a);
    (void)dev::event_destroy(p.b);
  }
  for (auto e : spare_) (void)dev::event_destroy(e);
}

namespace ev {

u64 galois_for_rotation(const Ctx& c, long r) {
  const long n = (long)c.n;
  long e = ((r % n) + n) % n;
  return h_powmod(5, (u64)e, c.M);
}

// ----------------------------------------------------------------- key switching

void key_switch(Ctx& c, const u64* x, size_t sx, int B, int limbs, const u64* key, const u64* add0,
                size_t sa0, const u64* add1, size_t sa1, u64* out, size_t so) {
  key_switch2(c, x, sx, B, limbs, key, key, 31, add0, sa0, add1, sa1, out, so);
}

// a fused column pass whose sources hold only their inverse row pass
static void set_isrc(const Ctx& c, FuseArgs& f, bool on) {
  if (!on) return;
  f.isrc = 1;
  f.itwf = c.d_itwf;
  f.itwq = c.d_itwq;
}

// ModUp of every digit of x (evaluation domain) to the extended basis, back
// in evaluation form: y [B][beta][ext][N] (the digit's own slots unused), the
// residues held as FP64 values for the key inner products.
// the key inner product on whole rows (k_kip_rows) serves the plain key
// switches where the fused transforms finish inverse column passes
static bool kip_rows_ok(const Ctx& c) { return kern::fused_ok(c) && !c.ci; }

DBuf modup_eval(Ctx& c, const u64* x, size_t sx, int B, int limbs, bool col_only) {
  const size_t N = c.N;
  const ModUpTable& tb = c.h_modup[limbs];
  const int ext = tb.ext, beta = tb.beta;
  DBuf xc(&c, (size_t)B * limbs * N);
  // the fused transform unfolds (conjugate-invariant ring) on the fly, and
  // finishes the inverse transform itself where it can (isrc)
  const bool is = kern::isrc_ok(c, 1);
  if (is)
    kern::ntt_inv_rows(c, x, sx, xc.p(), (size_t)limbs * N, B, kern::chain_map(limbs));
  else
    kern::ntt(c, x, sx, xc.p(), (size_t)limbs * N, B, kern::chain_map(limbs), true, kern::fused_ok(c));
  const size_t sy = (size_t)beta * ext * N;
  DBuf y(&c, (size_t)B * sy);
  LimbMap m{};
  for (int i = 0; i < tb.npairs; ++i) {
    const int t = tb.pair_t[i];
    m.prime[m.n] = tb.ext_prime[t];
    m.off[m.n] = m.ooff[m.n] = tb.pair_j[i] * ext + t;
    ++m.n;
  }
  if (kern::fused_ok(c)) {           // conversion computed inside the forward transform
    FuseArgs f;
    f.pro = 1;
    f.ci = c.ci ? c.d_ci : nullptr;
    f.mu = c.d_modup + limbs;
    f.src = xc.p();
    f.s_hi = (size_t)limbs * N;
    f.no_row = col_only ? 1 : 0;
    set_isrc(c, f, is);
    audit::check(xc.p(), (size_t)B * limbs * N * sizeof(u64), "fused modup source");
    kern::ntt_fused(c, f, y.p(), sy, B, m, true);
  } else {
    if (col_only) BM_THROW(BM_EINVAL, "column-pass ModUp needs the fused transforms");
    kern::modup(c, xc.p(), (size_t)limbs * N, y.p(), sy, B, limbs);
    kern::ntt(c, y.p(), sy, y.p(), sy, B, m, false);
    kern::words_f64(c, y.p(), (size_t)B * sy, true);
  }
  return y;
}

// ModDown of (u, w) [B][2][ext][N] over Q_l u P plus the addends:
// out = (add0 + ModDown(u), add1 + ModDown(w))
void moddown_add(Ctx& c, u64* uw, int B, int limbs, const u64* add0, size_t sa0, const u64* add1,
                        size_t sa1, u64* out, size_t so, bool rows_done) {
  const size_t N = c.N;
  const int ext = c.h_modup[limbs].ext;
  const size_t suw = (size_t)2 * ext * N;
  LimbMap mp{};
  for (int comp = 0; comp < 2; ++comp)
    for (int kk = 0; kk < c.K; ++kk) {
      mp.prime[mp.n] = c.pid_special(kk);
      mp.off[mp.n] = mp.ooff[mp.n] = comp * ext + limbs + kk;
      ++mp.n;
    }
  const bool is = kern::isrc_ok(c, 2);
  if (rows_done) {
    // the key inner product ran the inverse row pass of the special limbs
    if (!is) kern::ntt_inv_cols(c, uw, suw, uw, suw, B, mp);
  } else if (is) {
    kern::ntt_inv_rows(c, uw, suw, uw, suw, B, mp);
  } else {
    kern::ntt(c, uw, suw, uw, suw, B, mp, true, kern::fused_ok(c));
  }
  const size_t sc = (size_t)2 * limbs * N;
  DBuf conv(&c, (size_t)B * sc);
  if (kern::fused_ok(c)) {           // conversion and finish inside the forward transform
    FuseArgs f;
    f.pro = 2;
    f.ci = c.ci ? c.d_ci : nullptr;
    f.md = c.d_moddown;
    f.src = uw;
    set_isrc(c, f, is);
    f.s_div = f.e_div = 2;           // element 2 z + comp
    f.s_hi = f.m_hi = suw;
    f.s_lo = f.m_lo = (size_t)ext * N;
    f.s_off0 = limbs;
    f.epi = 1;
    f.mnd = uw;
    f.add0 = add0;
    f.a0_hi = sa0;
    f.add1 = add1;
    f.a1_hi = sa1;
    f.out = out;
    f.o_hi = so;
    f.o_lo = (size_t)limbs * N;
    f.wtab = &c.d_moddown->pinv[0][0];
    if (c.ref_dev && out >= c.ref_base && out < c.ref_base + c.ref_words) {   // a captured match's output
      f.out_ref = c.ref_dev;
      f.out_rel = (size_t)(out - c.ref_base);
      ++c.ref_hits;
      c.ref_covered += (size_t)B * 2 * limbs * N;
    }
    audit::check(uw, (size_t)B * suw * sizeof(u64), "fused moddown source");
    if (add0) audit::check(add0, ((size_t)(B - 1) * sa0 + (size_t)limbs * N) * sizeof(u64), "moddown addend 0");
    if (add1) audit::check(add1, ((size_t)(B - 1) * sa1 + (size_t)limbs * N) * sizeof(u64), "moddown addend 1");
    audit::check(out, ((size_t)(B - 1) * so + 2 * (size_t)limbs * N) * sizeof(u64), "moddown output");
    kern::ntt_fused(c, f, conv.p(), (size_t)limbs * N, 2 * B, kern::chain_map(limbs));
    return;
  }
  kern::moddown_conv(c, uw, suw, conv.p(), sc, B, limbs);
  kern::ntt(c, conv.p(), (size_t)limbs * N, conv.p(), (size_t)limbs * N, 2 * B, kern::chain_map(limbs), false);
  kern::moddown_finish(c, uw, suw, conv.p(), sc, add0, sa0, add1, sa1, out, so, B, limbs);
}

void key_switch2(Ctx& c, const u64* x, size_t sx, int B, int limbs, const u64* key0, const u64* key1,
                 int sel, const u64* add0, size_t sa0, const u64* add1, size_t sa1, u64* out, size_t so) {
  const ModUpTable& tb = c.h_modup[limbs];
  const size_t sy = (size_t)tb.beta * tb.ext * c.N, suw = (size_t)2 * tb.ext * c.N;
  const bool rows = kip_rows_ok(c);
  DBuf y = modup_eval(c, x, sx, B, limbs, rows);
  DBuf uw(&c, (size_t)B * suw);
  if (rows)   // digits' row pass, products and the special limbs' inverse row pass in one launch
    kern::kip_rows(c, y.p(), sy, x, sx, key0, key1, sel, uw.p(), suw, B, limbs, limbs);
  else
    kern::kip(c, y.p(), sy, x, sx, key0, key1, sel, uw.p(), suw, B, limbs);
  moddown_add(c, uw.p(), B, limbs, add0, sa0, add1, sa1, out, so, rows);
}

void rotation_sum_hoisted(Ctx& c, const bm_evk* evk, const u64* in, int B, int limbs,
                          const std::vector<HoistArgs>& hs, const std::vector<const u64*>& keys, u64* out) {
  const size_t N = c.N, ln = (size_t)limbs * N;
  const ModUpTable& tb = c.h_modup[limbs];
  const size_t sy = (size_t)tb.beta * tb.ext * N, suw = (size_t)2 * tb.ext * N;
  if (hs.empty()) BM_THROW(BM_EINVAL, "no rotation amounts");
  DBuf y = modup_eval(c, in + ln, 2 * ln, B, limbs);
  DBuf uw(&c, (size_t)B * suw), c0(&c, (size_t)B * ln);
  bool rows = false;   // the special limbs already in their inverse row pass
  for (size_t part = 0; part < hs.size(); ++part) {   // amount lists longer than one launch carries
    rows = kern::kip_hoist(c, y.p(), sy, in + ln, 2 * ln, (const u64* const*)evk->gtab.p(), hs[part], keys, uw.p(),
                           suw, in, 2 * ln, c0.p(), ln, B, limbs, part > 0, hs.size() == 1);
  }
  moddown_add(c, uw.p(), B, limbs, c0.p(), ln, in + ln, 2 * ln, out, 2 * ln, rows);
}

void relin(Ctx& c, const u64* d, int B, int limbs, const u64* rlk, u64* out) {
  const size_t ln = (size_t)limbs * c.N;
  key_switch(c, d + 2 * ln, 3 * ln, B, limbs, rlk, d, 3 * ln, d + ln, 3 * ln, out, 2 * ln);
}

// Relinearisation followed by the rescale, d [B][3][limbs][N] -> out
// [B][2][limbs-1][N], with the same words as relin then rescale: the
// relinearised component is (u - NTT(conv))P^-1 + d over Q_l, and the rescale
// needs its last limb in the coefficient domain, which is
// (y - conv_last)P^-1 for y = INTT(u + P d) at that limb.  So the key inner
// product adds P d to the last limb, one inverse transform takes the special
// limbs and that limb, and one fused forward transform computes
// NTT(conv_i P^-1 + last) and finishes ((u P^-1 + d) - that) q_last^-1.
void relin_rescale(Ctx& c, const u64* d, int B, int limbs, const u64* rlk, u64* out) {
  if (!kern::fused_ok(c) || limbs < 2) {
    const size_t ln = (size_t)limbs * c.N;
    DBuf rl(&c, (size_t)B * 2 * ln);
    relin(c, d, B, limbs, rlk, rl.p());
    rescale(c, rl.p(), B, 2, limbs, out);
    return;
  }
  const size_t N = c.N, ln = (size_t)limbs * N;
  const ModUpTable& tb = c.h_modup[limbs];
  const int ext = tb.ext;
  const size_t sy = (size_t)tb.beta * ext * N, suw = (size_t)2 * ext * N;
  const bool rows = kip_rows_ok(c);
  DBuf y = modup_eval(c, d + 2 * ln, 3 * ln, B, limbs, rows);
  DBuf uw(&c, (size_t)B * suw);
  if (rows)   // the last chain limb and the special limbs leave in their inverse row pass
    kern::kip_rows(c, y.p(), sy, d + 2 * ln, 3 * ln, rlk, rlk, 31, uw.p(), suw, B, limbs, limbs - 1, d, 3 * ln, ln);
  else
    kern::kip(c, y.p(), sy, d + 2 * ln, 3 * ln, rlk, rlk, 31, uw.p(), suw, B, limbs, d, 3 * ln, ln);
  moddown_rescale(c, uw.p(), B, limbs, d, 3 * ln, d + ln, 3 * ln, out, rows);
}

// (add0 + ModDown(u), add1 + ModDown(w)) rescaled, with the words of
// moddown_add then rescale: uw [B][2][ext][N] holds u + P add0 and w + P add1
// at the last chain limb (see relin_rescale), the addends are read at their
// first limbs - 1 limbs, out [B][2][limbs-1][N].
void moddown_rescale(Ctx& c, u64* uw, int B, int limbs, const u64* add0, size_t sa0, const u64* add1,
                     size_t sa1, u64* out, bool rows_done) {
  const size_t N = c.N;
  const int nl = limbs - 1;
  const ModUpTable& tb = c.h_modup[limbs];
  const int ext = tb.ext;
  const size_t suw = (size_t)2 * ext * N;
  LimbMap mp{};
  for (int comp = 0; comp < 2; ++comp) {
    mp.prime[mp.n] = nl;
    mp.off[mp.n] = mp.ooff[mp.n] = comp * ext + nl;
    ++mp.n;
    for (int kk = 0; kk < c.K; ++kk) {
      mp.prime[mp.n] = c.pid_special(kk);
      mp.off[mp.n] = mp.ooff[mp.n] = comp * ext + limbs + kk;
      ++mp.n;
    }
  }
  const bool is = kern::isrc_ok(c, 4);
  if (rows_done) {
    // the key inner product ran the inverse row pass of these limbs
    if (!is) kern::ntt_inv_cols(c, uw, suw, uw, suw, B, mp);
  } else if (is) {
    kern::ntt_inv_rows(c, uw, suw, uw, suw, B, mp);
  } else {
    kern::ntt(c, uw, suw, uw, suw, B, mp, true, true);   // unfolded on the fly (conjugate-invariant ring)
  }
  DBuf t(&c, (size_t)B * 2 * nl * N);
  FuseArgs f;
  f.pro = 4;
  set_isrc(c, f, is);
  f.ci = c.ci ? c.d_ci : nullptr;
  f.md = c.d_moddown;
  f.src = uw;
  f.s_div = f.e_div = 2;             // element 2 z + comp
  f.s_hi = f.m_hi = suw;
  f.s_lo = f.m_lo = (size_t)ext * N;
  f.s_off0 = limbs;
  f.last_off = nl;
  f.last_pid = nl;
  f.epi = 2;
  f.mnd = uw;
  f.wmtab = &c.d_moddown->pinv[0][0];
  f.add0 = add0;
  f.a0_hi = sa0;
  f.add1 = add1;
  f.a1_hi = sa1;
  f.out = out;
  f.o_hi = (size_t)2 * nl * N;
  f.o_lo = (size_t)nl * N;
  f.wtab = c.d_rescale + (size_t)(limbs - 1) * (c.L + 1) * 2;
  audit::check(uw, (size_t)B * suw * sizeof(u64), "moddown_rescale source");
  audit::check(add0, ((size_t)(B - 1) * sa0 + (size_t)nl * N) * sizeof(u64), "moddown_rescale addend 0");
  audit::check(add1, ((size_t)(B - 1) * sa1 + (size_t)nl * N) * sizeof(u64), "moddown_rescale addend 1");
  audit::check(out, (size_t)B * 2 * nl * N * sizeof(u64), "moddown_rescale output");
  kern::ntt_fused(c, f, t.p(), (size_t)nl * N, 2 * B, kern::chain_map(nl));
}

void rescale(Ctx& c, const u64* in, int B, int comps, int limbs, u64* out) {
  if (limbs < 2) BM_THROW(BM_ELEVEL, "rescale needs at least two limbs");
  const size_t N = c.N;
  const int nl = limbs - 1;
  DBuf last(&c, (size_t)B * comps * N);
  LimbMap m = kern::single(nl, nl);
  m.ooff[0] = 0;
  const bool is = kern::isrc_ok(c, 3);
  if (is)
    kern::ntt_inv_rows(c, in, (size_t)limbs * N, last.p(), N, B * comps, m);
  else
    kern::ntt(c, in, (size_t)limbs * N, last.p(), N, B * comps, m, true, kern::fused_ok(c));
  DBuf t(&c, (size_t)B * comps * nl * N);
  if (kern::fused_ok(c)) {           // reduction and finish inside the forward transform
    if (in == out) BM_THROW(BM_EINVAL, "rescale cannot work in place");
    FuseArgs f;
    f.pro = 3;
    set_isrc(c, f, is);
    f.ci = c.ci ? c.d_ci : nullptr;
    f.src_pid = nl;
    f.src = last.p();
    f.s_hi = N;
    f.epi = 1;
    f.mnd = in;
    f.m_hi = (size_t)limbs * N;
    f.out = out;
    f.o_hi = (size_t)nl * N;
    f.wtab = c.d_rescale + (size_t)(limbs - 1) * (c.L + 1) * 2;
    audit::check(in, (size_t)B * comps * limbs * N * sizeof(u64), "rescale input");
    audit::check(out, (size_t)B * comps * nl * N * sizeof(u64), "rescale output");
    kern::ntt_fused(c, f, t.p(), (size_t)nl * N, B * comps, kern::chain_map(nl));
    return;
  }
  kern::rescale_conv(c, last.p(), (size_t)comps * N, N, t.p(), (size_t)comps * nl * N, B, comps, limbs);
  kern::ntt(c, t.p(), (size_t)nl * N, t.p(), (size_t)nl * N, B * comps, kern::chain_map(nl), false);
  kern::rescale_finish(c, in, (size_t)comps * limbs * N, t.p(), (size_t)comps * nl * N, out,
                    (size_t)comps * nl * N, B, comps, limbs);
}

void rotate(Ctx& c, const u64* in, int B, int limbs, u64 g, const u64* key, u64* out, bool add_input) {
  rotate2(c, in, B, limbs, g, key, g, key, 31, out, add_input);
}

// out = Rot(in) (+ addend): phi(c0) (+ addend0) plus the switched phi(c1)
static void rotate_impl(Ctx& c, const u64* in, int B, int limbs, u64 g0, const u64* key0, u64 g1,
                        const u64* key1, int sel, const u64* addend, u64* out) {
  const size_t ln = (size_t)limbs * c.N;
  DBuf tmp(&c, (size_t)B * 2 * ln);
  kern::automorphism(c, in, 2 * ln, tmp.p(), 2 * ln, B, 2 * limbs, g0, g1, sel);
  if (addend) kern::add(c, tmp.p(), 2 * ln, addend, 2 * ln, tmp.p(), 2 * ln, B, kern::chain_map(limbs));
  key_switch2(c, tmp.p() + ln, 2 * ln, B, limbs, key0, key1, sel, tmp.p(), 2 * ln,
              addend ? addend + ln : nullptr, 2 * ln, out, 2 * ln);
}

void rotate2(Ctx& c, const u64* in, int B, int limbs, u64 g0, const u64* key0, u64 g1, const u64* key1,
             int sel, u64* out, bool add_input) {
  rotate_impl(c, in, B, limbs, g0, key0, g1, key1, sel, add_input ? in : nullptr, out);
}

void rotate_add(Ctx& c, const u64* in, int B, int limbs, u64 g, const u64* key, const u64* addend,
                u64* out) {
  rotate_impl(c, in, B, limbs, g, key, g, key, 31, addend, out);
}

void drop(Ctx& c, const u64* in, int B, int comps, int from, int to, u64* out) {
  const size_t N = c.N;
  kern::copy_limbs(c, in, (size_t)comps * from * N, (size_t)from * N, out, 1, (size_t)comps * to * N,
                   0, (size_t)to * N, B, comps, to);
}

// ----------------------------------------------------------------- plaintexts and encryption

void upload_plain(Ctx& c, const int64_t* host, int B, int limbs, u64* out) {
  const size_t N = c.N;
  DBuf raw(&c, (size_t)B * N);
  HIP_OK(dev::memcpy_async(raw.p(), host, (size_t)B * N * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
  kern::reduce_int(c, (const int64_t*)raw.p(), out, (size_t)limbs * N, B, N, kern::chain_map(limbs));
  kern::ntt(c, out, (size_t)limbs * N, out, (size_t)limbs * N, B, kern::chain_map(limbs), false);
  HIP_OK(dev::stream_sync(c.stream));   // `host` may be released by the caller
}

template <class F>
static void parallel_for(size_t n, F f) {
  const size_t hw = std::max<size_t>(1, std::min<size_t>(16, std::thread::hardware_concurrency()));
  const size_t nt = std::min(hw, n);
  if (nt <= 1) {
    for (size_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  for (size_t t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (size_t i = t; i < n; i += nt) f(i);
    });
  for (auto& x : th) x.join();
}

void encrypt_batch(Ctx& c, const bm_pk* pk, const int64_t* m, int B, int limbs, u64 seed,
                   const u64* ct_ids, u64* out) {
  const size_t N = c.N;
  const size_t ln = (size_t)limbs * N;
  std::vector<int64_t> host((size_t)3 * B * N);
  parallel_for((size_t)3 * B, [&](size_t idx) {
    const size_t b = idx / 3, which = idx % 3;
    int64_t* dst = host.data() + (which * B + b) * N;
    if (which == 0) sample_ternary(seed, DOM_ENC_V, ct_ids[b], N, dst);
    else sample_gauss(c, seed, which == 1 ? DOM_ENC_E0 : DOM_ENC_E1, ct_ids[b], N, dst);
  });
  DBuf v(&c, (size_t)B * ln), e0(&c, (size_t)B * ln), e1(&c, (size_t)B * ln), mm(&c, (size_t)B * ln);
  upload_plain(c, host.data(), B, limbs, v.p());
  upload_plain(c, host.data() + (size_t)B * N, B, limbs, e0.p());
  upload_plain(c, host.data() + (size_t)2 * B * N, B, limbs, e1.p());
  upload_plain(c, m, B, limbs, mm.p());
  const u64* pb = pk->pk.p();
  const u64* pa = pk->pk.p() + (size_t)(c.L + 1) * N;
  const LimbMap cm = kern::chain_map(limbs);
  kern::mul(c, v.p(), ln, pb, 0, out, 2 * ln, B, cm);
  kern::add(c, out, 2 * ln, e0.p(), ln, out, 2 * ln, B, cm);
  kern::add(c, out, 2 * ln, mm.p(), ln, out, 2 * ln, B, cm);
  kern::mul(c, v.p(), ln, pa, 0, out + ln, 2 * ln, B, cm);
  kern::add(c, out + ln, 2 * ln, e1.p(), ln, out + ln, 2 * ln, B, cm);
}

void export_coeffs(Ctx& c, const u64* dev, int polys, int limbs, u64* host) {
  const size_t ln = (size_t)limbs * c.N;
  DBuf tmp(&c, (size_t)polys * ln);
  kern::ntt(c, dev, ln, tmp.p(), ln, polys, kern::chain_map(limbs), true);
  HIP_OK(dev::memcpy_async(host, tmp.p(), (size_t)polys * ln * sizeof(u64), hipMemcpyDeviceToHost, c.stream));
  HIP_OK(dev::stream_sync(c.stream));
}

void import_coeffs(Ctx& c, const u64* host, int polys, int limbs, u64* dev) {
  const size_t ln = (size_t)limbs * c.N;
  HIP_OK(dev::memcpy_async(dev, host, (size_t)polys * ln * sizeof(u64), hipMemcpyHostToDevice, c.stream));
  kern::ntt(c, dev, ln, dev, ln, polys, kern::chain_map(limbs), false);
  HIP_OK(dev::stream_sync(c.stream));
}

void decrypt_coeffs(Ctx& c, const bm_sk* sk, const u64* ct, int comps, int limbs, double* m) {
  const size_t N = c.N;
  const int use = std::min(limbs, 2);          // two limbs determine the centred message
  const size_t ln = (size_t)limbs * N;
  const LimbMap cm = kern::chain_map(use);
  DBuf acc(&c, (size_t)use * N), sp(&c, (size_t)use * N), tmp(&c, (size_t)use * N);
  HIP_OK(dev::memcpy_async(acc.p(), ct, (size_t)use * N * sizeof(u64), hipMemcpyDeviceToDevice, c.stream));
  HIP_OK(dev::memcpy_async(sp.p(), sk->s_ntt.p(), (size_t)use * N * sizeof(u64), hipMemcpyDeviceToDevice,
                        c.stream));
  for (int comp = 1; comp < comps; ++comp) {
    kern::mul(c, ct + comp * ln, 0, sp.p(), 0, tmp.p(), 0, 1, cm);
    kern::add(c, acc.p(), 0, tmp.p(), 0, acc.p(), 0, 1, cm);
    if (comp + 1 < comps) kern::mul(c, sp.p(), 0, sk->s_ntt.p(), 0, sp.p(), 0, 1, cm);
  }
  kern::ntt(c, acc.p(), 0, acc.p(), 0, 1, cm, true);
  std::vector<u64> r((size_t)use * N);
  HIP_OK(dev::memcpy_async(r.data(), acc.p(), r.size() * sizeof(u64), hipMemcpyDeviceToHost, c.stream));
  HIP_OK(dev::stream_sync(c.stream));
  const u64 q0 = c.primes[0].q;
  if (use == 1) {
    for (size_t i = 0; i < N; ++i) m[i] = r[i] > q0 / 2 ? -(double)(q0 - r[i]) : (double)r[i];
    return;
  }
  const u64 q1 = c.primes[1].q;
  const u64 inv = h_invmod(q0 % q1, q1);
  const u128 Q = (u128)q0 * q1;
  for (size_t i = 0; i < N; ++i) {
    const u64 a0 = r[i], a1 = r[N + i];
    const u64 d = (a1 + q1 - a0 % q1) % q1;
    const u128 v = (u128)a0 + (u128)q0 * h_mulmod(d, inv, q1);
    m[i] = v > Q / 2 ? -(double)(Q - v) : (double)v;
  }
}

// ----------------------------------------------------------------- keys

void keygen_secret(Ctx& c, u64 seed, bm_sk* sk) {
  const size_t N = c.N;
  sk->s.resize(N);
  sample_ternary(seed, DOM_S, 0, N, sk->s.data());
  const int np = c.nprimes();
  sk->s_ntt = DBuf(&c, (size_t)np * N);
  DBuf raw(&c, N);
  HIP_OK(dev::memcpy_async(raw.p(), sk->s.data(), N * sizeof(int64_t), hipMemcpyHostToDevice, c.stream));
  const LimbMap all = kern::ext_map(c, c.L + 1);
  kern::reduce_int(c, (const int64_t*)raw.p(), sk->s_ntt.p(), 0, 1, 0, all);
  kern::ntt(c, sk->s_ntt.p(), 0, sk->s_ntt.p(), 0, 1, all, false);
  HIP_OK(dev::stream_sync(c.stream));
}

void keygen_public(Ctx& c, u64 seed, const bm_sk* sk, bm_pk* pk) {
  const size_t N = c.N;
  const int nq = c.L + 1;
  std::vector<u64> qs(nq);
  for (int i = 0; i < nq; ++i) qs[i] = c.primes[i].q;
  std::vector<u64> a((size_t)nq * N);
  std::vector<int64_t> e(N);
  sample_uniform(seed, DOM_PK_A, 0, qs.data(), nq, N, a.data());
  sample_gauss(c, seed, DOM_PK_E, 0, N, e.data());
  pk->pk = DBuf(&c, (size_t)2 * nq * N);
  u64* b = pk->pk.p();
  u64* ad = b + (size_t)nq * N;
  HIP_OK(dev::memcpy_async(ad, a.data(), a.size() * sizeof(u64), hipMemcpyHostToDevice, c.stream));
  const LimbMap cm = kern::chain_map(nq);
  kern::ntt(c, ad, 0, ad, 0, 1, cm, false);
  DBuf ee(&c, (size_t)nq * N);
  upload_plain(c, e.data(), 1, nq, ee.p());
  kern::mul(c, ad, 0, sk->s_ntt.p(), 0, b, 0, 1, cm);
  kern::sub(c, ee.p(), 0, b, 0, b, 0, 1, cm);
  HIP_OK(dev::stream_sync(c.stream));
}

void keygen_switch(Ctx& c, u64 seed, u32 dom_a, u32 dom_e, u64 index_base, const bm_sk* sk,
                   const u64* s_prime, DBuf& key) {
  const size_t N = c.N;
  const int np = c.nprimes();
  const int nq = c.L + 1;
  std::vector<u64> qs(np);
  for (int i = 0; i < np; ++i) qs[i] = c.primes[i].q;
  std::vector<u64> a((size_t)c.dnum * np * N);
  std::vector<int64_t> e((size_t)c.dnum * N);
  parallel_for((size_t)2 * c.dnum, [&](size_t idx) {
    const int j = (int)(idx / 2);
    if (idx % 2 == 0)
      sample_uniform(seed, dom_a, index_base + j, qs.data(), np, N, a.data() + (size_t)j * np * N);
    else
      sample_gauss(c, seed, dom_e, index_base + j, N, e.data() + (size_t)j * N);
  });
  key = DBuf(&c, (size_t)c.dnum * 2 * np * N);
  const LimbMap all = kern::ext_map(c, nq);
  DBuf raw(&c, N), tmp(&c, (size_t)np * N);
  // [P]_{q_i} as Shoup pairs, for the gadget term of each digit
  std::vector<u64> pmod(2 * MAX_LIMBS, 0);
  for (int j = 0; j < c.dnum; ++j) {
    u64* bj = key.p() + (size_t)(2 * j) * np * N;
    u64* aj = key.p() + (size_t)(2 * j + 1) * np * N;
    HIP_OK(dev::memcpy_async(aj, a.data() + (size_t)j * np * N, (size_t)np * N * sizeof(u64),
                          hipMemcpyHostToDevice, c.stream));
    kern::ntt(c, aj, 0, aj, 0, 1, all, false);
    HIP_OK(dev::memcpy_async(raw.p(), e.data() + (size_t)j * N, N * sizeof(int64_t), hipMemcpyHostToDevice,
                          c.stream));
    kern::reduce_int(c, (const int64_t*)raw.p(), bj, 0, 1, 0, all);
    kern::ntt(c, bj, 0, bj, 0, 1, all, false);
    kern::mul(c, aj, 0, sk->s_ntt.p(), 0, tmp.p(), 0, 1, all);
    kern::sub(c, bj, 0, tmp.p(), 0, bj, 0, 1, all);
    // + [P]_{q_i} s' on the limbs of digit j
    LimbMap dm{};
    const int lo = j * c.alpha, hi = std::min((j + 1) * c.alpha, nq);
    for (int i = lo; i < hi; ++i) {
      const u64 qi = c.primes[i].q;
      u64 P = 1;
      for (int kk = 0; kk < c.K; ++kk) P = h_mulmod(P, c.primes[c.pid_special(kk)].q % qi, qi);
      pmod[2 * dm.n] = P;
      pmod[2 * dm.n + 1] = h_shoup(P, qi);
      dm.prime[dm.n] = i;
      dm.off[dm.n] = dm.ooff[dm.n] = i;
      ++dm.n;
    }
    DBuf scal(&c, pmod.size());
    HIP_OK(dev::memcpy_async(scal.p(), pmod.data(), pmod.size() * sizeof(u64), hipMemcpyHostToDevice, c.stream));
    kern::axpy_scalar(c, s_prime, 0, scal.p(), bj, 0, 1, dm);
    HIP_OK(dev::stream_sync(c.stream));
  }
  // the key inner products read key words as FP64 values
  kern::words_f64(c, key.p(), (size_t)c.dnum * 2 * np * N, true);
  HIP_OK(dev::stream_sync(c.stream));
}

}  // namespace ev
}  // namespace bm
