// blindmatch.cpp -- Blind-Match server side on the device: Input Ciphertext
// Expansion (Alg. 1) and HE-C^3 (Alg. 2), batched over gallery groups.
//
// Readings of the paper used here (0-indexed slots):
//   - the query is tiled, slot s holding q[s mod d]; mask_i is periodic in d
//     with ones where floor((s mod d)/c) == i, c = d/k, encoded at scale q_L;
//   - Alg. 1 rotates by -c 2^t when bit t of i is 0 and by +c 2^t otherwise;
//   - Alg. 2 starts from the trivial zero ciphertext, so the first part's
//     term is the accumulator itself;
//   - schedule S2 (an optimisation of this library) sums the degree-2
//     tensors of the k parts before one relinearisation and one rescale.
#include "blindmatch_impl.hpp"

#include <algorithm>

namespace bm {
namespace bmx {

int ilog2(u64 v) {
  int e = 0;
  while ((1ULL << e) < v) ++e;
  return e;
}

bool is_pow2(u64 v) { return v && !(v & (v - 1)); }

void check_shape(const Ctx& c, u32 d, u32 k) {
  if (!is_pow2(d) || !is_pow2(k) || k > d || d > c.n) BM_THROW(BM_EDIM, "need power-of-two k | d <= slot count");
}

const u64* galois_key(const bm_evk* evk, u64 g) {
  auto it = evk->gk.find(g);
  if (it == evk->gk.end()) BM_THROW(BM_ENOKEY, "no Galois key for element " + std::to_string(g));
  return it->second->k.p();
}

int gallery_limbs(const Ctx& c, u32 k) { return k == 1 ? c.L + 1 : c.L; }

Plan plan(const Ctx& c, uint32_t schedule, uint32_t k, int g_limbs, uint32_t out_limbs) {
  Plan s;
  s.sched = schedule & 0xff;
  s.lmin = (schedule & BM_LEVEL_MIN) != 0;
  s.comp = (schedule & BM_COMPRESS) != 0;
  s.hoist = (schedule & BM_HOIST) != 0;
  if (schedule & ~(uint32_t)(0xff | BM_LEVEL_MIN | BM_COMPRESS | BM_HOIST))
    BM_THROW(BM_EINVAL, "unknown schedule flags");
  if (s.sched != BM_S1 && s.sched != BM_S2) BM_THROW(BM_EINVAL, "schedule must be BM_S1 or BM_S2");
  s.t = s.lmin ? std::min<int>(EVAL_LIMBS + (s.comp ? 1 : 0), g_limbs) : g_limbs;
  s.ql = k > 1 ? s.t + 1 : s.t;
  const int nat = s.t - 1;                   // HE-C^3 output level
  const int top = s.comp ? nat - 1 : nat;    // highest possible output
  s.ol = out_limbs ? (int)out_limbs : (c.out_limbs ? (int)c.out_limbs : top);
  s.ol = std::min(s.ol, top);
  if (s.ol < 1) BM_THROW(BM_ELEVEL, s.comp ? "compression needs one level more" : "output level");
  s.rot = s.lmin ? s.ol + (s.comp ? 1 : 0) : nat;
  return s;
}

u64 out_cts(const Plan& p, u64 G, u32 d, u32 k) {
  const u64 cc = d / k;
  return p.comp ? (G + cc - 1) / cc : G;
}

double result_scale(const Ctx& c, const Plan& p, double cu_scale, double g_scale) {
  double s = cu_scale * g_scale / (double)c.primes[p.t - 1].q;
  if (p.comp) {                              // Mul(P) by the mask at scale q_{rot-1}, then Res
    const double qm = (double)c.primes[p.rot - 1].q;
    s = s * qm / qm;
  }
  return s;
}

void match_groups(Ctx& c, const bm_evk* evk, const Plan& p, const u64* cu, int nq, size_t cu_stride,
                  const bm_gallery& g, const u64* cmask, u64* out, size_t out_qstride) {
  if (!p.comp) {
    hec3_groups(c, evk, cu, nq, cu_stride, g.d, g.k, g.buf.p(), g.groups, (int)g.limbs, p.t, p.sched, p.rot,
                p.ol, out, out_qstride, p.hoist);
    return;
  }
  if (!cmask) BM_THROW(BM_EINVAL, "compression mask missing");
  const size_t per = (size_t)g.groups * 2 * p.rot * c.N;
  DBuf tmp(&c, (size_t)nq * per);
  hec3_groups(c, evk, cu, nq, cu_stride, g.d, g.k, g.buf.p(), g.groups, (int)g.limbs, p.t, p.sched, p.rot,
              p.rot, tmp.p(), per, p.hoist);
  for (int j = 0; j < nq; ++j)
    compress(c, evk, tmp.p() + j * per, (size_t)2 * p.rot * c.N, g.groups, g.d, g.k, cmask, p.rot, p.ol,
             out + j * out_qstride);
}

// Galois elements of a hoisted rotation sum, split into launches of at most
// HOIST_MAX elements; amounts[z][a] (per_elem: list z serves elements z,
// z + Z, z + 2Z, ... of the batch, Z the number of lists) or amounts[0][a]
// for every element.
static std::vector<HoistArgs> hoist_args(const Ctx& c, const bm_evk* evk,
                                         const std::vector<std::vector<long>>& amounts, bool per_elem,
                                         std::vector<const u64*>& keys) {
  std::vector<HoistArgs> hs;
  const int A = (int)amounts[0].size();
  const int Z = per_elem ? (int)amounts.size() : 1;
  if (per_elem && A * Z > HOIST_MAX) BM_THROW(BM_EINVAL, "too many hoisted rotations per launch");
  const int per = per_elem ? A : HOIST_MAX;
  for (int a0 = 0; a0 < A; a0 += per) {
    HoistArgs h{};
    h.A = std::min(per, A - a0);
    h.per_elem = per_elem ? 1 : 0;
    h.mod = per_elem ? Z : 1 << 30;
    for (int z = 0; z < Z; ++z)
      for (int a = 0; a < h.A; ++a) {
        const u64 g = ev::galois_for_rotation(c, amounts[z][a0 + a]);
        keys.push_back(galois_key(evk, g));                 // BM_ENOKEY when missing
        h.g[per_elem ? z * h.A + a : a] = (uint32_t)g;
      }
    hs.push_back(h);
  }
  return hs;
}

// Rotation amounts of part i once Alg. 1's steps are unrolled: one per
// non-empty subset S of the log2 k steps, sum over t in S of -c 2^t (bit t
// of i is 0) or +c 2^t (bit t of i is 1), in increasing order of S.
static std::vector<long> expansion_amounts(u32 d, u32 k, u32 i) {
  const long cc = d / k;
  std::vector<long> out;
  for (u32 S = 1; S < k; ++S) {
    long r = 0;
    for (int t = 0; (1u << t) < k; ++t)
      if ((S >> t) & 1) r += ((i >> t) & 1) ? (cc << t) : -(cc << t);
    out.push_back(r);
  }
  return out;
}

void expand_batch(Ctx& c, const bm_evk* evk, const u64* q, size_t qs, size_t qcs, int nq, int qlimbs,
                  const u64* masks, u32 d, u32 k, u64* out, bool hoist) {
  const size_t N = c.N;
  const int l = qlimbs, nl = qlimbs - 1;
  if (nl < 1) BM_THROW(BM_ELEVEL, "expansion needs two limbs");
  if (nq < 1) return;
  const size_t ln = (size_t)l * N, nln = (size_t)nl * N;
  const int E = nq * (int)k;                  // element j k + i: part i of query j
  if (hoist && k > 1) {
    // the log2 k steps of part i unrolled into one hoisted sum of the
    // rotations of Mul(P)(q, mask_i), evaluated on q itself: one ModUp of
    // every query's c1, the key inner products of all parts' amounts with
    // each mask applied to them over Q_l u P, one ModDown and Res per part
    // (the amounts depend on the part only: list i serves every query)
    std::vector<std::vector<uint32_t>> parts(k);
    std::vector<const u64*> keys;
    for (u32 i = 0; i < k; ++i)
      for (long r : expansion_amounts(d, k, i)) {
        const u64 g = ev::galois_for_rotation(c, r);
        keys.push_back(galois_key(evk, g));                 // BM_ENOKEY when missing
        parts[i].push_back((uint32_t)g);
      }
    const ModUpTable& tb = c.h_modup[l];
    const size_t sy = (size_t)tb.beta * tb.ext * N, suw = (size_t)2 * tb.ext * N;
    DBuf y = ev::modup_eval(c, q + qcs, qs, nq, l);
    DBuf uw(&c, (size_t)E * suw), ad(&c, (size_t)E * 2 * ln);
    const bool fused = kern::fused_ok(c);
    const bool rows = kern::kip_hoist_mask(c, y.p(), sy, q, qs, qcs, (const u64* const*)evk->gtab.p(), parts, keys,
                                           masks, uw.p(), suw, ad.p(), 2 * ln, nq, l, fused, fused);
    if (fused) {
      ev::moddown_rescale(c, uw.p(), E, l, ad.p(), 2 * ln, ad.p() + ln, 2 * ln, out, rows);
    } else {
      DBuf sum(&c, (size_t)E * 2 * ln);
      ev::moddown_add(c, uw.p(), E, l, ad.p(), 2 * ln, ad.p() + ln, 2 * ln, sum.p(), 2 * ln);
      ev::rescale(c, sum.p(), E, 2, l, out);
    }
    return;
  }
  // Mul(P) of every query by every mask, then one batched rescale
  DBuf pm(&c, (size_t)E * 2 * ln);
  kern::mul_ct_pt(c, q, qs, qcs, masks, (size_t)c.mask_limbs() * N, pm.p(), 2 * ln, ln, E, l, (int)k, (int)k);
  ev::rescale(c, pm.p(), E, 2, l, out);
  // step t: part i adds Rot(., -c 2^t) when bit t of i is 0 and Rot(., +c 2^t)
  // otherwise; bit t of the element index j k + i is bit t of i (k a power of
  // two), so every element of the batch picks its sign in the same launch
  const u32 cc = d / k;
  DBuf tmp(&c, (size_t)E * 2 * nln);
  u64* a = out;
  u64* b = tmp.p();
  for (int t = 0; (1u << t) < k; ++t) {
    const long r = (long)cc << t;
    const u64 gm = ev::galois_for_rotation(c, -r), gp = ev::galois_for_rotation(c, r);
    ev::rotate2(c, a, E, nl, gm, galois_key(evk, gm), gp, galois_key(evk, gp), t, b, true);
    std::swap(a, b);
  }
  if (a != out) kern::copy_limbs(c, a, 2 * nln, nln, out, 1, 2 * nln, 0, nln, E, 2, nl);
}

void expand_hoisted(Ctx& c, const bm_evk* evk, const u64* q, int qlimbs, const u64* masks, u32 d, u32 k,
                    u64* out) {
  expand_batch(c, evk, q, 0, (size_t)qlimbs * c.N, 1, qlimbs, masks, d, k, out, true);
}

void expand(Ctx& c, const bm_evk* evk, const u64* q, int qlimbs, const u64* masks, u32 d, u32 k,
            u64* out) {
  expand_batch(c, evk, q, 0, (size_t)qlimbs * c.N, 1, qlimbs, masks, d, k, out, false);
}

int pass_elems(const Ctx& c) { return c.group_chunk > 0 ? c.group_chunk : (c.N >= 65536 ? 16 : 64); }

void hec3_elems(Ctx& c, const bm_evk* evk, const std::vector<Elem>& el, size_t cu_cs, size_t cu_ps, u32 d, u32 k,
                int lg_store, int l, u32 schedule, int rot_limbs, int out_limbs, bool hoist, int per_pass) {
  const size_t N = c.N;
  const int nl = l - 1;
  if (nl < 1 || l > lg_store) BM_THROW(BM_ELEVEL, "matching needs two limbs");
  if (rot_limbs < 1 || rot_limbs > nl) BM_THROW(BM_ELEVEL, "rotation limbs out of range");
  if (out_limbs < 1 || out_limbs > rot_limbs) BM_THROW(BM_ELEVEL, "output limbs out of range");
  if (schedule != BM_S1 && schedule != BM_S2) BM_THROW(BM_EINVAL, "unknown schedule");
  if (el.empty()) return;
  const size_t ln = (size_t)l * N, nln = (size_t)nl * N, rln = (size_t)rot_limbs * N;
  const size_t gcs = (size_t)lg_store * N;          // component stride of a stored gallery ciphertext
  const size_t gpart = 2 * gcs;                      // one stored gallery ciphertext
  const size_t oct = (size_t)2 * out_limbs * N;
  const u32 cc = d / k;
  const int rots = ilog2(cc);
  const u64* rlk = evk->rlk.k.p();
  std::vector<const u64*> gks(hoist ? 0 : rots);
  std::vector<u64> gel(hoist ? 0 : rots);
  std::vector<const u64*> hkeys;
  std::vector<HoistArgs> hs;
  if (hoist) {            // rotate-and-sum as one hoisted sum of the rotations 1 .. c-1
    if (cc > 1) {
      std::vector<std::vector<long>> amounts(1);
      for (u32 r = 1; r < cc; ++r) amounts[0].push_back((long)r);
      hs = hoist_args(c, evk, amounts, false, hkeys);
    }
  } else {
    for (int t = 0; t < rots; ++t) {
      gel[t] = ev::galois_for_rotation(c, 1L << t);
      gks[t] = galois_key(evk, gel[t]);
    }
  }
  const int Bmax = (int)std::min<size_t>(per_pass > 0 ? (size_t)per_pass : (size_t)pass_elems(c), el.size());
  DBuf d3(&c, (size_t)Bmax * 3 * ln);
  DBuf acc(&c, (size_t)Bmax * 2 * nln), acc2(&c, (size_t)Bmax * 2 * nln);
  DBuf racc(rot_limbs < nl ? DBuf(&c, (size_t)Bmax * 2 * rln) : DBuf());
  std::vector<const u64*> av(Bmax), bv(Bmax);
  std::vector<u64*> ov(Bmax);
  for (size_t e0 = 0; e0 < el.size(); e0 += (size_t)Bmax) {
    const int B = (int)std::min<size_t>((size_t)Bmax, el.size() - e0);
    bool contiguous = true;                          // outputs at ov[0] + z oct
    for (int z = 0; z < B; ++z) {
      ov[z] = el[e0 + z].out;
      contiguous &= ov[z] == ov[0] + (size_t)z * oct;
    }
    auto operands = [&](u32 part) {
      for (int z = 0; z < B; ++z) {
        av[z] = el[e0 + z].cu + (size_t)part * cu_ps;
        bv[z] = el[e0 + z].gal + (size_t)part * gpart;
      }
    };
    if (schedule == BM_S1) {
      for (u32 i = 0; i < k; ++i) {
        operands(i);
        kern::tensor_ptrs(c, av.data(), cu_cs, 0, bv.data(), gcs, 0, 1, d3.p(), 3 * ln, B, l);
        u64* dst = i == 0 ? acc.p() : acc2.p();
        ev::relin_rescale(c, d3.p(), B, l, rlk, dst);
        if (i > 0) kern::add(c, acc.p(), nln, acc2.p(), nln, acc.p(), nln, 2 * B, kern::chain_map(nl));
      }
    } else {                                        // the k tensors summed in one pass
      operands(0);
      kern::tensor_ptrs(c, av.data(), cu_cs, cu_ps, bv.data(), gcs, gpart, (int)k, d3.p(), 3 * ln, B, l);
      ev::relin_rescale(c, d3.p(), B, l, rlk, acc.p());
    }
    u64* a = acc.p();
    u64* b = acc2.p();
    if (rot_limbs < nl) {                 // exact level drop before rotate-and-sum
      ev::drop(c, acc.p(), B, 2, nl, rot_limbs, racc.p());
      a = racc.p();
      b = acc.p();                        // acc is free again and large enough
    }
    if (hoist) {
      if (!hs.empty()) {
        // outputs side by side at the output level: the sum lands there directly
        if (contiguous && rot_limbs == out_limbs) {
          ev::rotation_sum_hoisted(c, evk, a, B, rot_limbs, hs, hkeys, ov[0]);
          continue;
        }
        ev::rotation_sum_hoisted(c, evk, a, B, rot_limbs, hs, hkeys, b);
        std::swap(a, b);
      }
    } else {
      for (int t = 0; t < rots; ++t) {
        ev::rotate(c, a, B, rot_limbs, gel[t], gks[t], b, true);
        std::swap(a, b);
      }
    }
    if (contiguous)
      kern::copy_limbs(c, a, 2 * rln, rln, ov[0], 1, oct, 0, (size_t)out_limbs * N, B, 2, out_limbs);
    else
      kern::copy_ptrs(c, a, 2 * rln, rln, ov.data(), (size_t)out_limbs * N, B, 2, out_limbs);
  }
}

void hec3_groups(Ctx& c, const bm_evk* evk, const u64* cu, int nq, size_t cu_stride, u32 d, u32 k,
                 const u64* gal, u64 G, int lg_store, int l, u32 schedule, int rot_limbs, int out_limbs,
                 u64* out, size_t out_qstride, bool hoist) {
  const size_t N = c.N, ln = (size_t)l * N;
  const size_t gpart = 2 * (size_t)lg_store * N, oct = (size_t)2 * out_limbs * N;
  // passes of Bg groups x nq queries (query-major inside a pass)
  const u64 per_q = std::max<u64>(1, (u64)pass_elems(c) / (u64)nq);
  const u64 Bg_max = std::min<u64>(per_q, G);
  std::vector<Elem> el;
  el.reserve((size_t)G * nq);
  for (u64 g0 = 0; g0 < G; g0 += Bg_max) {
    const u64 Bg = std::min<u64>(Bg_max, G - g0);
    for (int j = 0; j < nq; ++j)
      for (u64 gi = 0; gi < Bg; ++gi)
        el.push_back(Elem{cu + (size_t)j * cu_stride, gal + (g0 + gi) * k * gpart,
                          out + (size_t)j * out_qstride + (g0 + gi) * oct});
  }
  // whole blocks per pass; a last, partial block of groups is a pass of its own
  const int per_pass = (int)(Bg_max * (u64)nq);
  const size_t full = (size_t)(G / Bg_max) * (size_t)per_pass;
  std::vector<Elem> head(el.begin(), el.begin() + full), tail(el.begin() + full, el.end());
  hec3_elems(c, evk, head, ln, 2 * ln, d, k, lg_store, l, schedule, rot_limbs, out_limbs, hoist, per_pass);
  hec3_elems(c, evk, tail, ln, 2 * ln, d, k, lg_store, l, schedule, rot_limbs, out_limbs, hoist, per_pass);
}

void load_queries(Ctx& c, const BatchClass& K, u64* qbuf) {
  const int ql = K.s.ql;
  for (size_t j = 0; j < K.queries.size(); ++j)
    ev::drop(c, K.queries[j]->buf.p(), 1, 2, (int)K.queries[j]->limbs, ql, qbuf + j * 2 * (size_t)ql * c.N);
}

void class_body(Ctx& c, const bm_evk* evk, const BatchPlan& bp, const BatchClass& K, const bm_gallery* const* gs,
                const u64* qbuf, u64* out) {
  const Plan& s = K.s;
  const bm_gallery& g0 = *K.shape;
  const size_t N = c.N;
  const u32 d = g0.d, k = g0.k;
  const int nq = (int)K.queries.size(), ql = s.ql, t = s.t;
  const u64* cu = qbuf;
  size_t cu_cs = (size_t)ql * N, cu_ps = 2 * (size_t)ql * N, cu_stride = 2 * (size_t)ql * N;   // k = 1: ql = t
  DBuf cub;
  if (k > 1) {
    cub = DBuf(&c, (size_t)nq * k * 2 * t * N);
    expand_batch(c, evk, qbuf, 2 * (size_t)ql * N, (size_t)ql * N, nq, ql, K.masks->pt.p(), d, k, cub.p(), s.hoist);
    cu = cub.p();
    cu_cs = (size_t)t * N;
    cu_ps = 2 * (size_t)t * N;
    cu_stride = (size_t)k * 2 * t * N;
  }
  const size_t gpart = 2 * (size_t)g0.limbs * N;
  const int hl = s.comp ? s.rot : s.ol;              // limbs of the Alg. 2 outputs
  const size_t oct = 2 * (size_t)hl * N;
  size_t tmp_words = 0;                              // compression: the group outputs first
  std::vector<size_t> tmp_off(K.pairs.size());
  for (size_t pi = 0; pi < K.pairs.size(); ++pi) {
    tmp_off[pi] = tmp_words;
    tmp_words += (size_t)gs[K.pairs[pi]]->groups * oct;
  }
  DBuf tmp(s.comp ? DBuf(&c, tmp_words) : DBuf());
  std::vector<Elem> el;
  for (size_t pi = 0; pi < K.pairs.size(); ++pi) {
    const size_t p = K.pairs[pi];
    const bm_gallery& g = *gs[p];
    u64* dst = s.comp ? tmp.p() + tmp_off[pi] : out + bp.out_off[p];
    for (u64 gi = 0; gi < g.groups; ++gi)
      el.push_back(Elem{cu + (size_t)K.qidx[pi] * cu_stride, g.buf.p() + gi * k * gpart, dst + gi * oct});
  }
  hec3_elems(c, evk, el, cu_cs, cu_ps, d, k, (int)g0.limbs, t, s.sched, s.rot, hl, s.hoist);
  if (s.comp)
    for (size_t pi = 0; pi < K.pairs.size(); ++pi) {
      const size_t p = K.pairs[pi];
      compress(c, evk, tmp.p() + tmp_off[pi], oct, gs[p]->groups, d, k, K.cmask, s.rot, s.ol, out + bp.out_off[p]);
    }
}

// Compression method (Sec. 3.4, Prop. 3).  Every group output is multiplied
// by the score mask (ones at slots b c, at scale q_{rl-1}) and rescaled; the
// groups of each block of c consecutive groups are then merged by halving,
// x_j += Rot(x_{j+h}, -h) for h = P/2, ..., 1, so group g ends at slot
// b c + (g mod c) of compressed ciphertext floor(g / c).  Every merge step is
// one batched rotate-and-add over the pairs of the block.
void compress(Ctx& c, const bm_evk* evk, const u64* in, size_t in_stride, u64 G, u32 d, u32 k,
              const u64* mask, int rl, int ol, u64* out) {
  const size_t N = c.N;
  const int nl = rl - 1;
  if (nl < 1) BM_THROW(BM_ELEVEL, "compression needs two limbs");
  if (ol < 1 || ol > nl) BM_THROW(BM_ELEVEL, "output limbs out of range");
  const u64 cc = d / k;
  const size_t rln = (size_t)rl * N, ct = (size_t)2 * nl * N, oct = (size_t)2 * ol * N;
  DBuf pm(&c, G * 2 * rln), y(&c, G * ct);
  for (int comp = 0; comp < 2; ++comp)
    kern::mul(c, in + comp * rln, in_stride, mask, 0, pm.p() + comp * rln, 2 * rln, (int)G,
              kern::chain_map(rl));
  ev::rescale(c, pm.p(), (int)G, 2, rl, y.p());
  for (u64 o = 0; o * cc < G; ++o) {
    u64* base = y.p() + o * cc * ct;
    const u64 r = std::min<u64>(cc, G - o * cc);
    u64 h = 1;
    while (2 * h < r) h *= 2;
    for (; r > 1 && h >= 1; h /= 2) {
      const u64 cnt = std::min<u64>(h, r - h);
      const u64 g = ev::galois_for_rotation(c, -(long)h);
      ev::rotate_add(c, base + h * ct, (int)cnt, nl, g, galois_key(evk, g), base, base);
    }
    kern::copy_limbs(c, base, ct, (size_t)nl * N, out + o * oct, 1, oct, 0, (size_t)ol * N, 1, 2, ol);
  }
}

// Server-side enrollment (Sec. 3.2, Fig. 3).  User u's ciphertext holds its
// feature vector in slots [0, d); its identifier Index = indices[u] is
// position b = Index mod T of group Index div T.  Part i of the user is
// Res(Mul(P)(C_u, mask_i)) (mask_i: ones at [i c, (i+1) c)), rotated right by
// (b - i) c slots as left rotations by c 2^t for the set bits t of
// (i - b) mod T, ascending, and added into part i of the group.  The parts
// of a chunk of users go through every step as one batch; the elements that
// rotate at bit t are gathered, rotated together and scattered back.
void enroll(Ctx& c, const bm_evk* evk, bm_gallery& g, const u64* const* users, int user_limbs,
            const uint64_t* indices, int nu, const u64* masks) {
  const size_t N = c.N;
  const u32 d = g.d, k = g.k, cc = d / k;
  const u64 T = c.n / cc;
  const int ul = user_limbs, lg = (int)g.limbs;
  if (lg != ul - 1) BM_THROW(BM_ELEVEL, "users must sit one level above the gallery");
  const size_t uct = (size_t)2 * ul * N, ct = (size_t)2 * lg * N;
  const int logT = ilog2(T);
  std::vector<u64> gel(logT);
  std::vector<const u64*> key(logT);
  for (int t = 0; t < logT; ++t) {
    gel[t] = ev::galois_for_rotation(c, (long)cc << t);
    key[t] = galois_key(evk, gel[t]);
  }
  const int per_chunk = std::max(1, 64 / (int)k);          // users per pass
  const int rb = 64;                                          // elements per rotation batch
  for (int u0 = 0; u0 < nu; u0 += per_chunk) {
    const int U = std::min(per_chunk, nu - u0);
    const int E = U * (int)k;
    DBuf pm(&c, (size_t)E * uct), x(&c, (size_t)E * ct);
    for (int u = 0; u < U; ++u)
      for (int comp = 0; comp < 2; ++comp)
        kern::mul(c, users[u0 + u] + comp * (size_t)ul * N, 0, masks, (size_t)c.mask_limbs() * N,
                  pm.p() + (size_t)u * k * uct + comp * (size_t)ul * N, uct, (int)k, kern::chain_map(ul));
    ev::rescale(c, pm.p(), E, 2, ul, x.p());
    std::vector<u64> amount(E);
    for (int u = 0; u < U; ++u) {
      const u64 b = indices[u0 + u] % T;
      for (u32 i = 0; i < k; ++i) amount[(size_t)u * k + i] = (i + T - b) % T;
    }
    // element lists of every bit, uploaded once per chunk
    std::vector<uint32_t> sel;
    std::vector<size_t> first(logT + 1, 0);
    for (int t = 0; t < logT; ++t) {
      first[t] = sel.size();
      for (int e = 0; e < E; ++e)
        if ((amount[e] >> t) & 1) sel.push_back((uint32_t)e);
    }
    first[logT] = sel.size();
    DBuf idx(&c, sel.size() / 2 + 2);
    if (!sel.empty()) {
      HIP_OK(dev::memcpy_async(idx.p(), sel.data(), sel.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                               c.stream));
      HIP_OK(dev::stream_sync(c.stream));   // the host list may be released
    }
    DBuf a(&c, (size_t)std::min(rb, E) * ct), r(&c, (size_t)std::min(rb, E) * ct);
    for (int t = 0; t < logT; ++t)
      for (size_t s0 = first[t]; s0 < first[t + 1]; s0 += rb) {
        const int B = (int)std::min<size_t>(rb, first[t + 1] - s0);
        const uint32_t* id = (const uint32_t*)idx.p() + s0;
        const uint32_t mx = *std::max_element(sel.begin() + s0, sel.begin() + s0 + B);
        kern::move_idx(c, x.p(), ct, a.p(), ct, id, mx, false, B, ct);
        ev::rotate(c, a.p(), B, lg, gel[t], key[t], r.p(), false);
        kern::move_idx(c, r.p(), ct, x.p(), ct, id, mx, true, B, ct);
      }
    for (int u = 0; u < U; ++u) {
      const u64 grp = indices[u0 + u] / T;
      u64* dst = g.buf.p() + (size_t)grp * k * ct;
      kern::add(c, dst, (size_t)lg * N, x.p() + (size_t)u * k * ct, (size_t)lg * N, dst, (size_t)lg * N,
                2 * (int)k, kern::chain_map(lg));
    }
  }
}

}  // namespace bmx
}  // namespace bm
