// blindmatch_impl.hpp -- internal entry points of the Blind-Match layer.
#pragma once
#include "evaluator.hpp"

namespace bm {
namespace bmx {

// Limbs of one match: products (t), query as used (ql), accumulator during
// rotate-and-sum (rot) and output (ol).  With compression, rot is the level
// the compression mask multiplies and ol sits at least one limb below it.
struct Plan {
  uint32_t sched = 0;   // BM_S1 or BM_S2
  bool lmin = false;    // BM_LEVEL_MIN
  bool comp = false;    // BM_COMPRESS
  bool hoist = false;   // BM_HOIST
  int t = 0, ql = 0, rot = 0, ol = 0;
};
// products of the minimum-level schedule (one limb more with compression)
constexpr int EVAL_LIMBS = 3;
Plan plan(const Ctx& c, uint32_t schedule, uint32_t k, int g_limbs, uint32_t out_limbs);
// result ciphertexts per query: G, or ceil(G / c) when compressed
u64 out_cts(const Plan& p, u64 G, u32 d, u32 k);
// scale of the results from the scales of the expanded query and the gallery
double result_scale(const Ctx& c, const Plan& p, double cu_scale, double g_scale);
// Alg. 2 for nq queries over every group of g and, with compression, the
// compression of each query's group outputs: query j's out_cts results go to
// out + j*out_qstride as [2][ol][N] each.  cmask is the compression mask
// (BM_COMPRESS only).
void match_groups(Ctx& c, const bm_evk* evk, const Plan& p, const u64* cu, int nq, size_t cu_stride,
                  const bm_gallery& g, const u64* cmask, u64* out, size_t out_qstride);

int ilog2(u64 v);
bool is_pow2(u64 v);
void check_shape(const Ctx& c, u32 d, u32 k);
const u64* galois_key(const bm_evk* evk, u64 g);
int gallery_limbs(const Ctx& c, u32 k);
// Alg. 1: q [2][qlimbs][N], masks [k][L+1][N] -> out [k][2][qlimbs-1][N]
void expand(Ctx& c, const bm_evk* evk, const u64* q, int qlimbs, const u64* masks, u32 d, u32 k,
            u64* out);
// Alg. 2 for nq queries x G groups.  Query j's k expanded parts start at
// cu + j*cu_stride ([k][2][l][N]); gal is [G][k][2][lg_store][N] and is read
// at its first l limbs; the accumulator is cut to rot_limbs before the
// rotate-and-sum; the result of (j, g) goes to
// out + j*out_qstride + g*2*out_limbs*N.
// With hoist the rotate-and-sum is one hoisted sum of the rotations 1 .. c-1.
void hec3_groups(Ctx& c, const bm_evk* evk, const u64* cu, int nq, size_t cu_stride, u32 d, u32 k,
                 const u64* gal, u64 G, int lg_store, int l, u32 schedule, int rot_limbs, int out_limbs,
                 u64* out, size_t out_qstride, bool hoist);
// Alg. 1 with its log2 k steps unrolled into one hoisted rotation sum per part
void expand_hoisted(Ctx& c, const bm_evk* evk, const u64* q, int qlimbs, const u64* masks, u32 d, u32 k,
                    u64* out);
// Alg. 1 for nq queries in one batch of nq k elements: query j at q + j qs,
// [2][.][N] with component stride qcs, read at its first qlimbs limbs;
// out [nq][k][2][qlimbs-1][N].  Plain or hoisted (the part's amounts shared by
// every query).
void expand_batch(Ctx& c, const bm_evk* evk, const u64* q, size_t qs, size_t qcs, int nq, int qlimbs,
                  const u64* masks, u32 d, u32 k, u64* out, bool hoist);

// One (query, gallery group) element of Alg. 2: the query's k expanded parts
// at cu (part p at cu + p cu_ps, component stride cu_cs), the group's k parts
// at gal (part p at gal + p gpart, component stride lg_store N), the result
// [2][out_limbs][N] to out.
struct Elem {
  const u64* cu;
  const u64* gal;
  u64* out;
};
// Alg. 2 for any list of elements of one shape (d, k, stored gallery limbs),
// in passes of per_pass elements (0: pass_elems) in list order: every launch
// covers the elements of a pass whatever query and gallery they come from.
void hec3_elems(Ctx& c, const bm_evk* evk, const std::vector<Elem>& el, size_t cu_cs, size_t cu_ps, u32 d, u32 k,
                int lg_store, int l, u32 schedule, int rot_limbs, int out_limbs, bool hoist, int per_pass = 0);
// elements (query x group pairs) per pass: the context's group chunk, else
// 16 at N = 2^16 and 64 below
int pass_elems(const Ctx& c);

// A batch of (query, gallery) pairs split into shape classes: the pairs
// whose galleries share (d, k, stored limbs) share every launch of their
// class (one expansion batch over the class's distinct queries, Alg. 2 over
// all of its (pair, gallery group) elements).
struct BatchClass {
  const bm_gallery* shape = nullptr;     // a gallery of the class (d, k, stored limbs)
  Plan s;
  const bm_masks* masks = nullptr;       // Alg. 1 masks at scale q_{ql-1} (k > 1)
  const u64* cmask = nullptr;            // compression mask (BM_COMPRESS)
  std::vector<const bm_ct*> queries;     // distinct queries of the class
  std::vector<size_t> pairs;             // batch indices
  std::vector<int> qidx;                 // query of each pair (index into queries)
};
struct BatchPlan {
  std::vector<BatchClass> cls;
  std::vector<size_t> out_off;           // words: result of pair p at out + out_off[p]
  std::vector<double> scale;             // result scale of pair p
  size_t out_words = 0;
};
// class K's queries cut to ql limbs, side by side: qbuf [nq][2][ql][N]
void load_queries(Ctx& c, const BatchClass& K, u64* qbuf);
// the device work of class K: its queries at qbuf ([nq][2][ql][N]), the
// result of pair p to out + out_off[p]; gs[p] is pair p's gallery
void class_body(Ctx& c, const bm_evk* evk, const BatchPlan& bp, const BatchClass& K, const bm_gallery* const* gs,
                const u64* qbuf, u64* out);

// Compression method: in holds G HE-C^3 outputs [2][rl][N] at stride
// in_stride; mask [rl..][N] is the score mask at scale q_{rl-1};
// out [ceil(G/c)][2][ol][N].
void compress(Ctx& c, const bm_evk* evk, const u64* in, size_t in_stride, u64 G, u32 d, u32 k,
              const u64* mask, int rl, int ol, u64* out);

// Server-side enrollment of nu users (ciphertexts [2][user_limbs][N]) with
// identifiers indices[u] into gallery g (at user_limbs - 1 limbs); masks are
// the k enrollment masks [k][L+1][N] at scale q_{user_limbs-1}.
void enroll(Ctx& c, const bm_evk* evk, bm_gallery& g, const u64* const* users, int user_limbs,
            const uint64_t* indices, int nu, const u64* masks);

}  // namespace bmx
}  // namespace bm

// library masks of Alg. 1 for a query of `ql` limbs (scale q_{ql-1}), made on
// the context's current stream (capi.cpp; internal, not exported)
extern "C" __attribute__((visibility("hidden"))) bm_masks* bmx_create_masks(bm_ctx* ctx, uint32_t d,
                                                                             uint32_t k, uint32_t ql);
// the enrollment masks of Sec. 3.2 (mask_i: ones at slots [i c, (i+1) c))
// at scale q_{limbs-1}, k plaintexts [k][L+1][N]; cached in the context
extern "C" __attribute__((visibility("hidden"))) const bm_masks* bmx_enroll_masks(bm_ctx* ctx, uint32_t d,
                                                                                   uint32_t k, uint32_t limbs);
// the compression method's score mask (ones at slots b c, c = d/k) at scale
// q_{limbs-1}, one plaintext [L+1][N]; cached in the context
extern "C" __attribute__((visibility("hidden"))) const bm_masks* bmx_compress_mask(bm_ctx* ctx, uint32_t d,
                                                                                    uint32_t k, uint32_t limbs);
