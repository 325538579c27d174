// blindmatch_impl.hpp -- internal entry points of the Blind-Match layer.
#pragma once
#include "evaluator.hpp"

namespace bm {
namespace bmx {

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
void hec3_groups(Ctx& c, const bm_evk* evk, const u64* cu, int nq, size_t cu_stride, u32 d, u32 k,
                 const u64* gal, u64 G, int lg_store, int l, u32 schedule, int rot_limbs, int out_limbs,
                 u64* out, size_t out_qstride);

}  // namespace bmx
}  // namespace bm

// library masks of Alg. 1 for a query of `ql` limbs (scale q_{ql-1}), made on
// the context's current stream (capi.cpp; internal, not exported)
extern "C" __attribute__((visibility("hidden"))) bm_masks* bmx_create_masks(bm_ctx* ctx, uint32_t d,
                                                                             uint32_t k, uint32_t ql);
