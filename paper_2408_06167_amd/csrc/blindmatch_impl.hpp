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
