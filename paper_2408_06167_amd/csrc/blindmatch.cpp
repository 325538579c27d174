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
  if (!is_pow2(d) || !is_pow2(k) || k > d || d > c.n) BM_THROW(BM_EDIM, "need power-of-two k | d <= N/2");
}

const u64* galois_key(const bm_evk* evk, u64 g) {
  auto it = evk->gk.find(g);
  if (it == evk->gk.end()) BM_THROW(BM_ENOKEY, "no Galois key for element " + std::to_string(g));
  return it->second->k.p();
}

int gallery_limbs(const Ctx& c, u32 k) { return k == 1 ? c.L + 1 : c.L; }

void expand(Ctx& c, const bm_evk* evk, const u64* q, int qlimbs, const u64* masks, u32 d, u32 k,
            u64* out) {
  const size_t N = c.N;
  const int l = qlimbs, nl = qlimbs - 1;
  if (nl < 1) BM_THROW(BM_ELEVEL, "expansion needs two limbs");
  const size_t ln = (size_t)l * N, nln = (size_t)nl * N;
  const u32 cc = d / k;
  // Mul(P) of the query by every mask, batched over the k masks
  DBuf pm(&c, (size_t)k * 2 * ln);
  for (int comp = 0; comp < 2; ++comp)
    kern::mul(c, q + comp * ln, 0, masks, (size_t)(c.L + 1) * N, pm.p() + comp * ln, 2 * ln, (int)k,
           kern::chain_map(l));
  ev::rescale(c, pm.p(), (int)k, 2, l, out);
  // step t: part i adds Rot(., -c 2^t) when bit t of i is 0 and Rot(., +c 2^t)
  // otherwise; all k parts go in one batch, the sign chosen per element.
  DBuf tmp(&c, (size_t)k * 2 * nln);
  u64* a = out;
  u64* b = tmp.p();
  for (int t = 0; (1u << t) < k; ++t) {
    const long r = (long)cc << t;
    const u64 gm = ev::galois_for_rotation(c, -r), gp = ev::galois_for_rotation(c, r);
    ev::rotate2(c, a, (int)k, nl, gm, galois_key(evk, gm), gp, galois_key(evk, gp), t, b, true);
    std::swap(a, b);
  }
  if (a != out) kern::copy_limbs(c, a, 2 * nln, nln, out, 1, 2 * nln, 0, nln, (int)k, 2, nl);
}

void hec3_groups(Ctx& c, const bm_evk* evk, const u64* cu, int nq, size_t cu_stride, u32 d, u32 k,
                 const u64* gal, u64 G, int lg_store, int l, u32 schedule, int rot_limbs, int out_limbs,
                 u64* out, size_t out_qstride) {
  const size_t N = c.N;
  const int nl = l - 1;
  if (nl < 1 || l > lg_store) BM_THROW(BM_ELEVEL, "matching needs two limbs");
  if (rot_limbs < 1 || rot_limbs > nl) BM_THROW(BM_ELEVEL, "rotation limbs out of range");
  if (out_limbs < 1 || out_limbs > rot_limbs) BM_THROW(BM_ELEVEL, "output limbs out of range");
  const size_t ln = (size_t)l * N, nln = (size_t)nl * N, rln = (size_t)rot_limbs * N;
  const size_t gpart = 2 * (size_t)lg_store * N;   // one stored gallery ciphertext
  const size_t upart = 2 * ln;                      // one expanded query part
  const size_t oct = (size_t)2 * out_limbs * N;
  const u32 cc = d / k;
  const int rots = ilog2(cc);
  const u64* rlk = evk->rlk.k.p();
  std::vector<const u64*> gks(rots);
  std::vector<u64> gel(rots);
  for (int t = 0; t < rots; ++t) {
    gel[t] = ev::galois_for_rotation(c, 1L << t);
    gks[t] = galois_key(evk, gel[t]);
  }
  // batch = (query, group) pairs; `chunk` bounds the pairs per pass
  u64 chunk = c.group_chunk > 0 ? (u64)c.group_chunk : (u64)(c.N >= 65536 ? 16 : 64);
  const u64 per_q = std::max<u64>(1, chunk / (u64)nq);
  const u64 Bg_max = std::min<u64>(per_q, G);
  const u64 Bmax = Bg_max * nq;
  DBuf d3(&c, Bmax * 3 * ln), rl(&c, Bmax * 2 * ln);
  DBuf acc(&c, Bmax * 2 * nln), acc2(&c, Bmax * 2 * nln);
  DBuf racc(rot_limbs < nl ? DBuf(&c, Bmax * 2 * rln) : DBuf());
  for (u64 g0 = 0; g0 < G; g0 += Bg_max) {
    const int Bg = (int)std::min<u64>(Bg_max, G - g0);
    const int B = Bg * nq;
    const u64* gbase = gal + g0 * k * gpart;
    if (schedule == BM_S1) {
      for (u32 i = 0; i < k; ++i) {
        kern::tensor(c, cu + (size_t)i * upart, cu_stride, Bg, ln, gbase + (size_t)i * gpart,
                     (size_t)k * gpart, Bg, (size_t)lg_store * N, d3.p(), 3 * ln, B, l, false);
        ev::relin(c, d3.p(), B, l, rlk, rl.p());
        u64* dst = i == 0 ? acc.p() : acc2.p();
        ev::rescale(c, rl.p(), B, 2, l, dst);
        if (i > 0) kern::add(c, acc.p(), nln, acc2.p(), nln, acc.p(), nln, 2 * B, kern::chain_map(nl));
      }
    } else if (schedule == BM_S2) {
      for (u32 i = 0; i < k; ++i)
        kern::tensor(c, cu + (size_t)i * upart, cu_stride, Bg, ln, gbase + (size_t)i * gpart,
                     (size_t)k * gpart, Bg, (size_t)lg_store * N, d3.p(), 3 * ln, B, l, i > 0);
      ev::relin(c, d3.p(), B, l, rlk, rl.p());
      ev::rescale(c, rl.p(), B, 2, l, acc.p());
    } else {
      BM_THROW(BM_EINVAL, "unknown schedule");
    }
    u64* a = acc.p();
    u64* b = acc2.p();
    if (rot_limbs < nl) {                 // exact level drop before rotate-and-sum
      ev::drop(c, acc.p(), B, 2, nl, rot_limbs, racc.p());
      a = racc.p();
      b = acc.p();                        // acc is free again and large enough
    }
    for (int t = 0; t < rots; ++t) {
      ev::rotate(c, a, B, rot_limbs, gel[t], gks[t], b, true);
      std::swap(a, b);
    }
    kern::copy_limbs(c, a, 2 * rln, rln, out + g0 * oct, Bg, out_qstride, oct, (size_t)out_limbs * N,
                     B, 2, out_limbs);
  }
}

}  // namespace bmx
}  // namespace bm
