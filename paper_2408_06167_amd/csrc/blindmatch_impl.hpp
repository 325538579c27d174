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
// cu + j*cu_stride ([k][2][lg][N]); gal is [G][k][2][lg][N]; the result of
// (j, g) goes to out + j*out_qstride + g*2*out_limbs*N.
void hec3_groups(Ctx& c, const bm_evk* evk, const u64* cu, int nq, size_t cu_stride, u32 d, u32 k,
                 const u64* gal, u64 G, int lg, u32 schedule, int out_limbs, u64* out,
                 size_t out_qstride);

}  // namespace bmx
}  // namespace bm
