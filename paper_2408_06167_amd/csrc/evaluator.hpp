// evaluator.hpp -- batched CKKS operations on device buffers (host side).
#pragma once
#include "bm_internal.hpp"

namespace bm {
namespace ev {

// Domains of the seeded SHAKE-256 streams.
enum : u32 {
  DOM_S = 1, DOM_PK_A = 2, DOM_PK_E = 3, DOM_RLK_A = 4, DOM_RLK_E = 5, DOM_GK_A = 6, DOM_GK_E = 7,
  DOM_ENC_V = 8, DOM_ENC_E0 = 9, DOM_ENC_E1 = 10
};

u64 galois_for_rotation(const Ctx& c, long r);

// Hybrid key switch of x ([B][limbs][N], stride sx, evaluation domain) with
// `key`; out[b] = (KS_0(x_b) + add0_b, KS_1(x_b) + add1_b) as [2][limbs][N].
void key_switch(Ctx& c, const u64* x, size_t sx, int B, int limbs, const u64* key, const u64* add0,
                size_t sa0, const u64* add1, size_t sa1, u64* out, size_t so);
// as above; batch element z switches with key1 when bit `sel` of z is set
void key_switch2(Ctx& c, const u64* x, size_t sx, int B, int limbs, const u64* key0, const u64* key1,
                 int sel, const u64* add0, size_t sa0, const u64* add1, size_t sa1, u64* out, size_t so);
// d: [B][3][limbs][N] -> out [B][2][limbs][N]
void relin(Ctx& c, const u64* d, int B, int limbs, const u64* rlk, u64* out);
// relin followed by rescale (same words), in fewer launches at N = 2^16
void relin_rescale(Ctx& c, const u64* d, int B, int limbs, const u64* rlk, u64* out);
// in: [B][comps][limbs][N] -> out [B][comps][limbs-1][N]
void rescale(Ctx& c, const u64* in, int B, int comps, int limbs, u64* out);
// ModUp of every digit of x ([B][limbs][N], stride sx, evaluation domain) to
// Q_l u P, back in the evaluation domain as FP64 values: [B][beta][l+K][N]
// (a digit's own slots unused)
// (col_only: the fused transform's column pass only, its u64 words left at
// the pair slots for kern::kip_rows)
DBuf modup_eval(Ctx& c, const u64* x, size_t sx, int B, int limbs, bool col_only = false);
// ModDown of (u, w) [B][2][l+K][N] over Q_l u P plus the addends:
// out = (add0 + ModDown(u), add1 + ModDown(w)), [B][2][limbs][N] at stride so
// (rows_done: the special limbs already hold the row pass of their inverse
// transform, left there by kern::kip_rows)
void moddown_add(Ctx& c, u64* uw, int B, int limbs, const u64* add0, size_t sa0, const u64* add1, size_t sa1,
                 u64* out, size_t so, bool rows_done = false);
// the same then rescaled, at N = 2^16 in one inverse row pass and one fused
// transform: uw must hold u + P add0 and w + P add1 at the last chain limb;
// out [B][2][limbs-1][N]
void moddown_rescale(Ctx& c, u64* uw, int B, int limbs, const u64* add0, size_t sa0, const u64* add1,
                     size_t sa1, u64* out, bool rows_done = false);
// in: [B][2][limbs][N] -> out = Rot_g(in) (+ in when add_input)
void rotate(Ctx& c, const u64* in, int B, int limbs, u64 g, const u64* key, u64* out, bool add_input);
// batch element z rotates with (g1, key1) when bit `sel` of z is set, else (g0, key0)
// out[z] = in[z] + sum_a Rot(in[z], r(z, a)) with the rotations hoisted twice:
// one ModUp of c1, the automorphisms applied to the extended digits inside
// fused key inner products that accumulate over Q_l u P, one ModDown.  The
// amounts come in one or more HoistArgs (each at most HOIST_MAX Galois
// elements); `keys` lists the keys used (for the launch check).
void rotation_sum_hoisted(Ctx& c, const bm_evk* evk, const u64* in, int B, int limbs,
                          const std::vector<HoistArgs>& hs, const std::vector<const u64*>& keys, u64* out);
// out = addend + Rot(in) (out may alias addend, not in)
void rotate_add(Ctx& c, const u64* in, int B, int limbs, u64 g, const u64* key, const u64* addend,
                u64* out);
void rotate2(Ctx& c, const u64* in, int B, int limbs, u64 g0, const u64* key0, u64 g1, const u64* key1,
             int sel, u64* out, bool add_input);
// out = first `to` limbs of each of `comps` components of in ([B][comps][from][N])
void drop(Ctx& c, const u64* in, int B, int comps, int from, int to, u64* out);

// coefficient-domain int64 plaintexts [B][N] -> evaluation-domain residues [B][limbs][N]
void upload_plain(Ctx& c, const int64_t* host, int B, int limbs, u64* out);
// public-key encryption of B plaintexts (host int64 [B][N]) at `limbs` limbs
void encrypt_batch(Ctx& c, const bm_pk* pk, const int64_t* m, int B, int limbs, u64 seed,
                   const u64* ct_ids, u64* out);
// evaluation-domain ciphertext [comps][limbs][N] -> coefficient words on host
void export_coeffs(Ctx& c, const u64* dev, int polys, int limbs, u64* host);
void import_coeffs(Ctx& c, const u64* host, int polys, int limbs, u64* dev);
// decrypt: centred plaintext coefficients (as doubles) of ct [comps][limbs][N]
void decrypt_coeffs(Ctx& c, const bm_sk* sk, const u64* ct, int comps, int limbs, double* m);

void keygen_secret(Ctx& c, u64 seed, bm_sk* sk);
void keygen_public(Ctx& c, u64 seed, const bm_sk* sk, bm_pk* pk);
// switching key from s' (evaluation domain over all primes) to s
void keygen_switch(Ctx& c, u64 seed, u32 dom_a, u32 dom_e, u64 index_base, const bm_sk* sk,
                   const u64* s_prime, DBuf& key);

}  // namespace ev
}  // namespace bm
