/*
 * blindmatch.h -- C ABI of the MI355X Blind-Match library.
 *
 * Blind-Match (CIKM '24) identifies a biometric query against an enrolled
 * gallery without decrypting either: the server evaluates a chunked cosine
 * similarity in CKKS (Sec. 3.3: Input Ciphertext Expansion, Alg. 1, and
 * HE-C^3, Alg. 2) and the client decrypts the scores, takes the arg-max and
 * applies a threshold (Sec. 3.4 "Decryption").  This library runs the server
 * side on one AMD Instinct MI355X (gfx950) with hand-written HIP kernels over
 * RNS polynomials; keys, encryption and decryption are provided so that a
 * single process can play client and server.
 *
 * Conventions shared by every entry point
 *   - Every function returns an int status: BM_OK (0) or a negative BM_E*
 *     code.  No C++ exception crosses this boundary.  A context keeps the
 *     text of its last error (bm_last_error).
 *   - Handles (bm_ctx, bm_sk, ...) are created by the library and released by
 *     the matching bm_*_free.  Freeing NULL is a no-op.  Every handle created
 *     from a context must be freed before that context, and is used only
 *     with that context (a handle of another context is BM_EINVAL).
 *   - Host buffers passed in are read (or written) only during the call.
 *   - Ciphertexts, keys, galleries and results live in device memory (HBM)
 *     owned by their handle.  Interchange with the host is in the COEFFICIENT
 *     domain: words[comps][limbs][N], uint64, residue of limb l in [0, q_l).
 *   - `stream` arguments are a hipStream_t (passed as void*) or NULL for the
 *     context's own stream.  Calls that take a stream are asynchronous on it;
 *     all other calls return with their device work finished.  One context is
 *     single-threaded (bm_server_submit and bm_server_poll excepted);
 *     changing the stream of a context first waits for the previous stream.
 *   - Ring degree N = 2^log_n, n = N/2 complex slots carrying real data (N
 *     real slots in the conjugate-invariant ring, bm_params.ring); limb
 *     l < L+1 is chain prime q_l, the K special primes follow.  A fresh
 *     ciphertext has L+1 limbs; each rescale drops the last limb.
 */
#ifndef BLINDMATCH_H
#define BLINDMATCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  BM_OK = 0,
  BM_EINVAL = -1,   /* NULL handle or pointer, size mismatch, bad argument */
  BM_EDIM = -2,     /* d or k not a power of two, k does not divide d, d > n, query d != gallery d */
  BM_ELEVEL = -3,   /* too few limbs for the operation, or a level mismatch */
  BM_ESCALE = -4,   /* Add of ciphertexts whose scales differ */
  BM_ENOKEY = -5,   /* a needed Galois key is missing from the evaluation key */
  BM_ENOMEM = -6,   /* device or host allocation failed */
  BM_EBUDGET = -7,  /* serving: request exceeds the HBM budget */
  BM_EDEVICE = -8,  /* HIP runtime error */
  BM_EBUSY = -9     /* reserved (no call returns it: a pending ticket polls as BM_OK with NULL) */
};

enum { BM_S1 = 1, BM_S2 = 2 };   /* Alg. 2 schedules, see bm_match */
/* OR-ed into a schedule: evaluate at the minimum level, and compress the
 * group outputs into few ciphertexts (see bm_match). */
enum { BM_LEVEL_MIN = 0x100, BM_COMPRESS = 0x200, BM_HOIST = 0x400 };

typedef struct bm_ctx bm_ctx;
typedef struct bm_sk bm_sk;
typedef struct bm_pk bm_pk;
typedef struct bm_evk bm_evk;
typedef struct bm_ct bm_ct;
typedef struct bm_masks bm_masks;
typedef struct bm_gallery bm_gallery;
typedef struct bm_result bm_result;
typedef struct bm_server bm_server;

/* Rings (Sec. 2): the power-of-two cyclotomic ring Z[X]/(X^N + 1) with N/2
 * complex slots, or the conjugate-invariant ring Z[X + X^-1] of rank N with N
 * real slots.  A conjugate-invariant element is stored as its first N
 * coefficients in Z[X]/(X^2N + 1) (coefficient N is 0 and coefficient 2N - k
 * is minus coefficient k); its slots are the values at zeta^(5^j), zeta a
 * primitive 4N-th root of unity, and rotation by r is X -> X^(5^r mod 4N). */
enum { BM_RING_STD = 0, BM_RING_CI = 1 };

/* Scheme parameters.  q[0..n_q-1] are the chain primes q_0..q_L (n_q = L+1),
 * p[0..n_p-1] the special primes of hybrid key switching, `alpha` chain limbs
 * per key-switching digit (dnum = ceil(n_q / alpha)).  Every prime must be
 * below 2^51 and congruent to 1 mod 2N (mod 4N in the conjugate-invariant
 * ring).  `scale` is the encoding scale Delta, `sigma` the error standard
 * deviation.  `out_limbs` is the default number of limbs a match result is
 * dropped to (0 keeps the natural level).  `ring` is BM_RING_STD or
 * BM_RING_CI.  Below, "slots" means n = N/2 (standard) or N (conjugate-
 * invariant) and "2N" in a Galois element means the ring's root order M = 2N
 * or 4N. */
typedef struct {
  uint32_t log_n;
  uint32_t n_q, n_p, alpha;
  uint32_t out_limbs;
  uint64_t q[16];
  uint64_t p[4];
  double scale;
  double sigma;
  uint32_t ring;
} bm_params;

/* Preset 1: N = 2^12, q = {50, 40, 40}-bit, one 51-bit special prime,
 * alpha = 1, scale 2^40 (a small parity/test ring, below 128-bit security).
 * Preset 2: N = 2^16, eight 50-bit chain primes, two 51-bit special primes,
 * alpha = 2 (dnum = 4), scale 2^50, out_limbs = 2.  Each prime is the largest
 * below its bit bound that is 1 mod 2N.  Presets 3 and 4 are presets 1 and 2
 * over the conjugate-invariant ring of the same rank N (primes 1 mod 4N).
 * Returns BM_EINVAL for other values. */
int bm_params_preset(int preset, bm_params *out);

/* Create a context on HIP device `device`: validates the primes, builds the
 * NTT twiddle and base-conversion tables in device memory. */
int bm_ctx_create(const bm_params *params, int device, bm_ctx **out);
void bm_ctx_free(bm_ctx *ctx);
const char *bm_strerror(int status);
const char *bm_last_error(const bm_ctx *ctx);
/* Result-invariant tuning knob: gallery groups evaluated per batched pass
 * (0 = choose automatically).  Changes speed and scratch size, never bits. */
int bm_ctx_set_group_chunk(bm_ctx *ctx, uint32_t groups);
/* Result-invariant knob: with on != 0, bm_match captures the launches of a
 * match as a HIP graph the first time a (keys, gallery, masks, schedule,
 * output level, stream) combination is seen and replays it afterwards (the
 * query is copied into the graph's input slot, the result out of its output
 * slot).  Each graph keeps its own scratch memory; freeing an evaluation key,
 * gallery or masks handle drops the context's graphs.  Off by default.
 * Kernel profiling (bm_profile_enable) runs matches eagerly. */
int bm_ctx_set_graphs(bm_ctx *ctx, int on);
/* The parameters the context was created with. */
int bm_ctx_params(const bm_ctx *ctx, bm_params *out);
/* Device memory currently held by the context's caching pool, in bytes. */
int bm_ctx_pool_bytes(const bm_ctx *ctx, uint64_t *bytes);
/* Route the context's device memory through a caller's allocator (for
 * instance a framework's caching allocator), so that one allocator owns the
 * card.  Every later block of the context's pool -- keys, ciphertexts,
 * galleries, masks, results and match scratch -- comes from
 * alloc_fn(bytes, user), which returns a device pointer on the context's
 * device, aligned to at least 256 bytes, or NULL when it cannot (the pool then
 * returns its cached blocks and asks once more; a second NULL makes the call
 * that needed the memory fail with BM_ENOMEM).  A block goes back through
 * free_fn(ptr, user) when the pool releases it: at bm_ctx_free, on a retry
 * after a failed allocation, or when the allocator is changed; the device has
 * finished all queued work by then, so the allocator may hand the block to
 * other work at once.  The pool caches blocks by size between calls, so
 * free_fn is not called when a handle is freed.
 *
 * The call waits for the context's stream, returns the pool's cached blocks
 * to their allocators and applies to every block allocated afterwards; blocks
 * in use keep the allocator they came from.  HIP graphs captured later and
 * servers created later (whose lanes call the callbacks from their worker
 * threads, which must then be safe to call from any thread) use it too.
 * Both NULL restores hipMalloc; exactly one NULL is BM_EINVAL.  The context's
 * constant tables (twiddles, base-conversion constants) are allocated by
 * bm_ctx_create with hipMalloc and are not affected.  The callbacks and
 * `user` must stay valid until the context and every handle made from it
 * are freed.  Allocation can happen inside a HIP graph capture (relaxed
 * mode) on the context's stream, so alloc_fn must not synchronise the device. */
int bm_ctx_set_allocator(bm_ctx *ctx, void *(*alloc_fn)(size_t bytes, void *user),
                         void (*free_fn)(void *ptr, void *user), void *user);

/* Kernel timing for measurement.  bm_profile_enable(ctx, 1) clears the
 * counters and brackets every subsequent kernel launch of the context (and of
 * its server lanes) with HIP events on the launch stream; 0 stops.
 * bm_profile_dump waits for the recorded events and writes one text line per
 * kernel, "name launches total_ms algorithmic_bytes algorithmic_ops" (the
 * name is the kernel's symbol with its template arguments and may contain
 * spaces; the four numbers are the last fields),
 * into buf (NUL-terminated, truncated to cap); *needed receives the full
 * length.  Algorithmic bytes count each distinct input and output word once
 * per launch; ops are modular multiplications (butterflies for the NTT). */
int bm_profile_enable(bm_ctx *ctx, int on);
int bm_profile_dump(bm_ctx *ctx, char *buf, size_t cap, size_t *needed);

/* Issue-rate probe of the arithmetic every transform and key product is made
 * of, for the ALU side of the roofline.  Launches `blocks` x 256 threads on
 * the context's own stream; each thread runs 8 independent chains of `iters`
 * forward butterflies mod prime `prime` (chain primes first, then special
 * primes), (u, v) <- (u + v w, u - v w), in the FP64 form the NTT uses (the
 * product a w - rint(a w/q) q with its exact low half, values folded back
 * after every second round), all in registers.  Thread x starts chain j from
 * u = (seed[j] + x) mod q and v = (seed[8 + j] + 3 x) mod q, with twiddle
 * w = seed[16 + j]; seed holds 24 residues of that prime.  *ms receives the
 * kernel time from HIP events around the launch (the call waits for it), so
 * the rate is blocks * 256 * 8 * iters modular products per *ms.  The first
 * n_words of the output (thread x's 8 (u, v) pairs as residues in [0, q) at
 * words[16 x ...]) are copied to `words` for checking the arithmetic; n_words
 * may be 0.  BM_EINVAL: prime out of range, blocks outside 1..65536, iters odd
 * or outside 2..2^24, a seed word >= q, n_words above blocks * 256 * 16. */
int bm_bench_modmul(bm_ctx *ctx, uint32_t prime, uint32_t blocks, uint32_t iters, const uint64_t *seed,
                    uint64_t *words, size_t n_words, double *ms);

/* ------------------------------------------------------------------ keys */

/* Key set of Sec. 3.1 (public key for clients, evaluation key for the
 * server, decryption key for the client) from one seed.  Randomness comes
 * from SHAKE-256 over le64(seed) || le32(domain) || le64(index): domain 1
 * secret (ternary), 2/3 public-key mask/error, 4/5 relinearisation key
 * digit j, 6/7 Galois key digit j of element g at index g*dnum + j.  The
 * evaluation key holds the relinearisation key (for s^2) and one Galois key
 * (for s(X^g), g = 5^r mod 2N) per rotation r in rotations[0..n_rot-1].
 * The key set is given by rotation amounts rather than by (d, k) shapes: the
 * amounts a shape needs come from bm_rotations_for (Alg. 1 and 2),
 * bm_rotations_hoisted (BM_HOIST), bm_rotations_compress (BM_COMPRESS) and
 * bm_rotations_enroll (bm_enroll); the union over the shapes served is the
 * list to pass.  Any handle pointer may be NULL if that key is not wanted. */
int bm_keygen(bm_ctx *ctx, uint64_t seed, const int32_t *rotations, size_t n_rot,
              bm_sk **sk, bm_pk **pk, bm_evk **evk);
/* Rotation amounts Alg. 1 and Alg. 2 use for feature length d split into k
 * parts: 2^t for t < log2(d/k), and -+(d/k) 2^t for t < log2 k.  Writes at
 * most `cap` values and the count to *n. */
int bm_rotations_for(uint32_t d, uint32_t k, int32_t *out, size_t cap, size_t *n);
/* Rotation amounts the hoisted schedule (BM_HOIST) uses: 1 .. c-1 for the
 * rotate-and-sum and, when k > 1, every sum of Alg. 1's shifts over a
 * non-empty subset of its steps (at most +-(k-1) c), c = d/k. */
int bm_rotations_hoisted(uint32_t d, uint32_t k, int32_t *out, size_t cap, size_t *n);
/* Rotation amounts the compression method (BM_COMPRESS) adds: -2^t for
 * t < log2(d/k). */
int bm_rotations_compress(uint32_t d, uint32_t k, int32_t *out, size_t cap, size_t *n);
/* Rotation amounts server-side enrollment (bm_enroll) uses: c 2^t for
 * t < log2(T), c = d/k, T = (N/2)/c templates per group. */
int bm_rotations_enroll(const bm_ctx *ctx, uint32_t d, uint32_t k, int32_t *out, size_t cap, size_t *n);
/* Coefficient-domain export for checking: secret key (N signed values);
 * public key component comp (0 = b, 1 = a) as [L+1][N]; switching key digit
 * j component comp as [L+1+K][N] for the relinearisation key (galois = 0) or
 * the Galois key of element `galois`. */
int bm_sk_export(const bm_sk *sk, int64_t *s, size_t n);
int bm_pk_export(const bm_pk *pk, uint32_t comp, uint64_t *words, size_t n_words);
int bm_evk_export(const bm_evk *evk, uint64_t galois, uint32_t digit, uint32_t comp,
                  uint64_t *words, size_t n_words);
/* Key checkpoint and hand-over (Sec. 3.1: the client sends the public and
 * evaluation keys to the server).  bm_pk_import takes the coefficient-domain
 * words[2][L+1][N] of a public key (b then a, as bm_pk_export writes them).
 * bm_evk_import takes words[1 + n_galois][dnum][2][L+1+K][N]: the
 * relinearisation key, then the Galois key of element galois[i] for each i,
 * each digit j as component 0 then 1 (as bm_evk_export writes them).  Keys
 * made by bm_keygen and the same words imported give bit-identical results.
 * BM_EINVAL: a size other than stated, a word not below its limb's prime, a
 * Galois element that is even, not in (1, 2N) or repeated.  bm_evk_galois
 * lists the Galois elements of an evaluation key in increasing order (at most
 * cap of them; *n receives the count). */
int bm_pk_import(bm_ctx *ctx, const uint64_t *words, size_t n_words, bm_pk **out);
int bm_evk_import(bm_ctx *ctx, const uint64_t *galois, size_t n_galois, const uint64_t *words,
                  size_t n_words, bm_evk **out);
int bm_evk_galois(const bm_evk *evk, uint64_t *galois, size_t cap, size_t *n);
void bm_sk_free(bm_sk *sk);
void bm_pk_free(bm_pk *pk);
void bm_evk_free(bm_evk *evk);

/* ------------------------------------------------------------------ encode / encrypt */

/* Canonical-embedding encoding of n real slots at `scale`:
 * coeffs[k] = round_half_away((2/N) Re sum_j scale*slots[j] zeta^(-k 5^j)),
 * zeta = exp(i pi / N).  `n_slots` must equal N/2.  In the conjugate-invariant
 * ring the same formula at dimension 2N (zeta = exp(i pi / 2N), n_slots = N)
 * gives the coefficients 0..N-1.  Double-precision FFT: results may differ by
 * 1 from another implementation on rare coefficients. */
int bm_encode(bm_ctx *ctx, const double *slots, size_t n_slots, double scale, int64_t *coeffs);
/* Public-key encryption of the integer plaintext coeffs[N] at `limbs` chain
 * limbs: (v b + e0 + m, v a + e1), v ternary, e0/e1 Gaussian, drawn from
 * domains 8/9/10 at index ct_id. */
int bm_encrypt_coeffs(bm_ctx *ctx, const bm_pk *pk, const int64_t *coeffs, uint32_t limbs,
                      double scale, uint64_t seed, uint64_t ct_id, bm_ct **out);
/* Query ciphertext of Sec. 3.3: q[0..d-1] tiled over every slot (slot s
 * holds q[s mod d]), encoded at the context scale, encrypted at L+1 limbs. */
int bm_encrypt_query(bm_ctx *ctx, const bm_pk *pk, const float *q, uint32_t d, uint64_t seed,
                     uint64_t ct_id, bm_ct **out);
/* Encrypted, packed gallery (Sec. 3.2 layout after enrolment, Fig. 4):
 * x is n x d row-major.  With c = d/k and T = (N/2)/c templates per group,
 * group g part i slot s holds x[g T + s / c][i c + s mod c] (zero past the
 * last template).  Parts are encrypted at L+1 limbs for k = 1 and at L limbs
 * for k > 1 (the expanded query loses one level), ct_id = ct_id_base + g k + i. */
int bm_encrypt_gallery(bm_ctx *ctx, const bm_pk *pk, const float *x, uint64_t n, uint32_t d,
                       uint32_t k, uint64_t seed, uint64_t ct_id_base, bm_gallery **out);
/* Gallery assembled from coefficient-domain words[G][k][2][limbs][N]. */
int bm_gallery_import(bm_ctx *ctx, const uint64_t *words, uint64_t groups, uint32_t d,
                      uint32_t k, uint32_t limbs, double scale, uint64_t n_templates,
                      bm_gallery **out);
/* ---- server-side enrollment (Sec. 3.2, Fig. 3) */
/* Client side of enrollment: x[0..d-1] in slots [0, d), zeros elsewhere,
 * encoded at the context scale, encrypted at L+1 limbs. */
int bm_encrypt_template(bm_ctx *ctx, const bm_pk *pk, const float *x, uint32_t d, uint64_t seed,
                        uint64_t ct_id, bm_ct **out);
/* Empty gallery (every part the trivial zero ciphertext) for n_templates
 * identifiers of dimension d split into k parts, stored at `limbs` limbs
 * (L for galleries filled by bm_enroll from L+1-limb users). */
int bm_gallery_create(bm_ctx *ctx, uint32_t d, uint32_t k, uint64_t n_templates, uint32_t limbs,
                      bm_gallery **out);
/* Server-side enrollment of n users: users[u] is a bm_encrypt_template
 * ciphertext one level above the gallery, indices[u] < n_templates its
 * identifier Index (0-indexed), stored at position b = Index mod T of group
 * Index / T.  For every part i the server multiplies C_u by mask_i (ones at
 * slots [i c, (i+1) c), at scale q_top of C_u), rescales, rotates right by
 * (b - i) c slots -- left rotations by c 2^t for the set bits t of
 * (i - b) mod T, ascending (keys of bm_rotations_enroll) -- and adds the
 * result into part i of the group.  The stored layout is that of
 * bm_encrypt_gallery, one level lower.  Enrolling an identifier twice adds
 * the two vectors.  `masks` may be NULL (the library's own enrollment
 * masks), else k plaintexts made elsewhere (bm_masks_import) at scale
 * q_top of the users.  Asynchronous on `stream`; errors: BM_ELEVEL (user
 * level), BM_ESCALE, BM_EINVAL (identifier out of range), BM_ENOKEY. */
int bm_enroll(bm_ctx *ctx, const bm_evk *evk, bm_gallery *g, const bm_ct *const *users,
              const uint64_t *indices, size_t n, const bm_masks *masks, void *stream);
int bm_gallery_export(const bm_gallery *g, uint64_t *words, size_t n_words);
int bm_gallery_info(const bm_gallery *g, uint64_t *groups, uint32_t *limbs, double *scale);
void bm_gallery_free(bm_gallery *g);

/* ------------------------------------------------------------------ ciphertexts */

int bm_ct_import(bm_ctx *ctx, const uint64_t *words, uint32_t comps, uint32_t limbs,
                 double scale, bm_ct **out);
int bm_ct_export(const bm_ct *ct, uint64_t *words, size_t n_words);
int bm_ct_info(const bm_ct *ct, uint32_t *comps, uint32_t *limbs, double *scale);
void bm_ct_free(bm_ct *ct);
/* Decrypt (c0 + c1 s [+ c2 s^2]) and decode: real parts of the n slots. */
int bm_decrypt_slots(bm_ctx *ctx, const bm_sk *sk, const bm_ct *ct, double *slots, size_t n);

/* ------------------------------------------------------------------ primitive operations
 * The CKKS operations of Sec. 2 that the hot path is made of.  Each output is
 * a new handle.  All ciphertext words are exact functions of the inputs. */

/* Batched negacyclic NTT (inverse = 0) or inverse NTT (inverse = 1), in place
 * on device words[n_polys][limbs][N]; limb l of every polynomial is reduced
 * modulo the prime with id prime_ids[l] (0..L chain, L+1.. special).  The
 * forward transform leaves evaluations in bit-reversed order. */
int bm_ntt(bm_ctx *ctx, uint64_t *dev_words, uint32_t n_polys, uint32_t limbs,
           const uint32_t *prime_ids, int inverse, void *stream);
/* Add(C): equal limbs and equal scale. */
int bm_op_add(bm_ctx *ctx, const bm_ct *a, const bm_ct *b, bm_ct **out);
/* Mul(P) by the integer plaintext pt[N] with scale pt_scale. */
int bm_op_pmul(bm_ctx *ctx, const bm_ct *a, const int64_t *pt, double pt_scale, bm_ct **out);
/* First half of Mul(C): (a0 b0, a0 b1 + a1 b0, a1 b1), scale a.scale*b.scale. */
int bm_op_tensor(bm_ctx *ctx, const bm_ct *a, const bm_ct *b, bm_ct **out);
/* Second half of Mul(C): relinearise a 3-component ciphertext with the key
 * for s^2 (hybrid key switch: ModUp, key inner product, ModDown). */
int bm_op_relin(bm_ctx *ctx, const bm_evk *evk, const bm_ct *a, bm_ct **out);
/* Res: c_i <- (c_i - [c_last]_{q_i}) q_last^{-1}, last limb dropped, scale / q_last. */
int bm_op_rescale(bm_ctx *ctx, const bm_ct *a, bm_ct **out);
/* Rot: slot j of the result holds slot (j + r) mod n of a.  BM_ENOKEY if the
 * evaluation key has no Galois key for 5^r. */
int bm_op_rotate(bm_ctx *ctx, const bm_evk *evk, const bm_ct *a, int32_t r, bm_ct **out);
/* Exact level drop to the first `limbs` limbs. */
int bm_op_drop(bm_ctx *ctx, const bm_ct *a, uint32_t limbs, bm_ct **out);

/* ------------------------------------------------------------------ Blind-Match */

/* Plaintext masks of Alg. 1: mask_i has ones at slots s with
 * floor((s mod d) / c) == i, encoded at scale q_L so the rescale after Mul(P)
 * restores the query scale exactly.  bm_masks_import takes integer
 * plaintexts coeffs[k][N] made elsewhere (same definition). */
int bm_masks_create(bm_ctx *ctx, uint32_t d, uint32_t k, bm_masks **out);
int bm_masks_import(bm_ctx *ctx, uint32_t d, uint32_t k, const int64_t *coeffs, double scale,
                    bm_masks **out);
void bm_masks_free(bm_masks *m);

/* Alg. 1, Input Ciphertext Expansion: outs[i] = Res(Mul(P)(q, mask_i)),
 * then for t < log2 k add Rot(., -c 2^t) when bit t of i is 0, else
 * Rot(., +c 2^t).  outs must hold k handle slots.  BM_EDIM for a query from
 * bm_encrypt_query with another d than the masks'. */
int bm_expand(bm_ctx *ctx, const bm_evk *evk, const bm_ct *q, const bm_masks *masks,
              bm_ct **outs);

/* Server side of recognition (Sec. 3.3): Alg. 1 when k > 1, then Alg. 2 on
 * every gallery group, batched over groups on the device.
 *   schedule BM_S1: Alg. 2 as printed, acc += Res(Relin(Tensor(C_u,i, C_s,i)));
 *   schedule BM_S2: acc = Res(Relin(sum_i Tensor(C_u,i, C_s,i))) -- one key
 *                   switch and one rescale per group; same message, other bits.
 * then log2(d/k) steps acc += Rot(acc, 2^t).  The score of template g T + b is
 * at slot b c of group g.  The query needs at least the gallery's limbs
 * (k = 1) or one more (k > 1); a higher query is cut exactly.  `masks` may
 * be NULL (the library's own masks are used).  out_limbs: 0 = context
 * default, otherwise an exact level drop of each result to that many limbs (a
 * value at or above the result's natural level keeps the natural level).
 * Asynchronous on `stream`.
 * schedule | BM_LEVEL_MIN: every input is first cut by exact limb drops to
 * the level the rest needs -- the products at 3 chain limbs (gallery read in
 * place, query cut to 3 limbs, or 4 before Alg. 1 with masks at scale q_3),
 * and the accumulator at the output limbs before rotate-and-sum.  Same
 * message and accuracy, other bits, about a third of the NTTs; the query
 * and gallery keep the levels they were encrypted at.
 * schedule | BM_COMPRESS: the compression method of Sec. 3.4 (cost in
 * Prop. 3).  Each group output is multiplied by the score mask (ones at
 * slots b c, encoded at scale q_top of the output) and rescaled; then the
 * groups of every block of c = d/k consecutive groups are merged by halving,
 * x_j += Rot(x_{j+h}, -h) for h = P/2, ..., 1 (P the power of two >= the
 * block size).  The result holds ceil(G / c) ciphertexts; template g T + b
 * is at slot b c + (g mod c) of ciphertext floor(g / c).  Needs the keys of
 * bm_rotations_compress and one level more than the plain match (with
 * BM_LEVEL_MIN the products are taken at 4 limbs); BM_ELEVEL if the
 * gallery has no level to spare.
 * schedule | BM_HOIST: the rotations hoisted twice (one ModUp of c1, the
 * automorphisms applied to the extended digits inside fused key inner
 * products accumulated over Q_l u P, one ModDown).  Alg. 2's log2 c
 * rotate-and-add steps become the sum of the c - 1 rotations 1 .. c-1 of
 * the accumulator, and Alg. 1's log2 k steps of part i the sum over the
 * non-empty subsets S of its steps of Rot(C_i, sum_{t in S} -+c 2^t).
 * Same message, other bits; keys of bm_rotations_hoisted.
 * BM_EDIM: the query came from bm_encrypt_query with another d than the
 * gallery's (an imported query carries no d and is not checked). */
int bm_match(bm_ctx *ctx, const bm_evk *evk, const bm_ct *q, const bm_gallery *g,
             const bm_masks *masks, uint32_t schedule, uint32_t out_limbs, void *stream,
             bm_result **out);
/* Many (query, gallery) pairs of possibly different d, k and size in one
 * call (the batched form of the paper's cluster serving, Sec. 3.5, on one
 * GPU).  Pairs whose galleries share a shape (d, k, stored limbs) form a
 * class: the class's distinct queries are expanded in one batch (Alg. 1), and
 * Alg. 2 runs over every (pair, gallery group) element of the class in passes
 * of group_chunk elements whose launches mix galleries.  With graphs on
 * (bm_ctx_set_graphs) the whole batch is captured once as one HIP graph per
 * combination of pairs and replayed (queries copied into its slots, results
 * out of its output slot).  outs[i] receives the result of pair i; the
 * results of one call share one device allocation.  Results are bit-identical
 * to per-pair bm_match. */
int bm_match_batch(bm_ctx *ctx, const bm_evk *evk, const bm_ct *const *qs,
                   const bm_gallery *const *gs, size_t n_pairs, uint32_t schedule,
                   uint32_t out_limbs, void *stream, bm_result **outs);
/* Result-invariant kernel knobs: they change speed and scratch size, never
 * bits.  group_chunk: (query, gallery group) elements per batched Alg. 2 pass
 * (0: 16 at N = 2^16, 64 below; at most 4096).  kip_variant: shape of the
 * hoisted key inner product of the rotate-and-sum, 0..4 (0: two elements per
 * thread and four amounts' key words requested ahead at one digit; the others
 * trade elements per thread, which share each key word from registers,
 * against amounts in flight).  ntt_row_views: polynomials x rows per block of
 * the row passes of the N = 2^16 transforms, 0 (= 16), 4, 8 or 16.
 * kip_order: block order of that key inner product, 0 (the element groups of
 * a position block side by side: they share its key words through the
 * memory-side cache), 1 (the position blocks of an element group side by
 * side: its gathered digit words stay in cache), or 2 and 3 (the element
 * groups in chunks of 2 or 4, each chunk's groups side by side and its
 * position blocks one after another: the chunk's digits stay in cache while
 * each key word serves the chunk).  fused_occupancy: 0, or 3 or 4
 * to build the fused base-conversion column passes of the N = 2^16
 * transforms for that many resident blocks per compute unit.
 * column_sources: 0, the fused base-conversion column passes (N = 2^16,
 * standard ring) run the inverse column pass of their source limbs in their
 * own blocks; 1, a separate inverse column pass transforms each source limb
 * once before them (fewer launches against less repeated work).  Matches
 * captured as graphs keep the knobs they were captured with. */
typedef struct {
  uint32_t group_chunk;
  uint32_t kip_variant;
  uint32_t ntt_row_views;
  uint32_t kip_order;
  uint32_t fused_occupancy;
  uint32_t column_sources;
} bm_tuning;
int bm_ctx_set_tuning(bm_ctx *ctx, const bm_tuning *t);
int bm_ctx_get_tuning(const bm_ctx *ctx, bm_tuning *t);
/* Autotuner of a batch (the pairs of bm_match_batch, out_limbs as there):
 * times the batch under each of the n_schedules schedules offered (those
 * whose keys or levels the inputs lack are skipped), then, under the fastest,
 * each knob of bm_tuning in turn over its values (coordinate descent),
 * checking that every setting gives the same words (BM_EDEVICE otherwise).
 * The winning knobs are left set in the context and returned with the
 * schedule and the time of one batch in ms.  Timed with HIP events on the
 * context's own stream, in the launch mode the context is set to (graphs or
 * eager); graphs captured while tuning are dropped. */
int bm_autotune_batch(bm_ctx *ctx, const bm_evk *evk, const bm_ct *const *qs, const bm_gallery *const *gs,
                      size_t n_pairs, const uint32_t *schedules, size_t n_schedules, uint32_t out_limbs,
                      uint32_t *best_schedule, bm_tuning *best, double *best_ms);
/* Autotuner of the result-invariant knob `group_chunk` (query x group pairs
 * per batched pass): times bm_match of (q, g) for chunk sizes 1..64 with HIP
 * events on the context's stream, keeps the fastest in the context and
 * returns it with its time per match.  Bits never depend on the choice. */
int bm_autotune(bm_ctx *ctx, const bm_evk *evk, const bm_ct *q, const bm_gallery *g, uint32_t schedule,
                uint32_t *best_chunk, double *best_ms);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the match
 * of bm_match on caller-owned device buffers, its intermediate buffers carved
 * out of a scratch array of BM_NOALLOC_SCRATCH_BYTES that the library holds
 * once per device for the life of the process.  Nothing is allocated: no
 * hipMalloc, no hipFree, no pool or allocator call, no memset node.
 *   q_words: device words[2][q_limbs][N] of the query ciphertext in the
 *     evaluation domain (what bm_ntt's forward transform gives from the
 *     coefficient words), scale q_scale, packed for feature length g's d;
 *   masks: required when the gallery has k > 1 (bm_masks_create or
 *     bm_masks_import, made beforehand), ignored for k = 1;
 *   schedule: as bm_match without BM_COMPRESS (BM_EINVAL);
 *   out_words: device words[G][2][ol][N] in the evaluation domain, G the
 *     gallery groups and ol = min(out_limbs, or the context default when 0,
 *     the natural output level): result ciphertext g at g * 2 * ol * N.
 *     *needed_words receives G * 2 * ol * N; with out_words NULL the call
 *     only reports that size.  n_out_words must equal it (BM_EINVAL).
 *   *out_scale receives the results' scale.
 * Before anything is enqueued the whole sequence of the match is walked on
 * the host and its scratch need measured; a match that needs more than
 * BM_NOALLOC_SCRATCH_BYTES fails with BM_ENOMEM and enqueues nothing (a
 * smaller group chunk, bm_ctx_set_group_chunk, lowers the need).  The words
 * equal those of bm_match with the same arguments.  Asynchronous on `stream`.
 * Every call on a device uses that device's one scratch array, whose
 * contents are left from the previous call (no kernel here reads scratch it
 * has not written in the same call): calls that overlap on one device -- on
 * two streams, two threads or two contexts -- race on it and must be
 * serialised by the caller. */
#define BM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int bm_match_noalloc(bm_ctx *ctx, const bm_evk *evk, const uint64_t *q_words, uint32_t q_limbs,
                     double q_scale, const bm_gallery *g, const bm_masks *masks, uint32_t schedule,
                     uint32_t out_limbs, uint64_t *out_words, size_t n_out_words, size_t *needed_words,
                     double *out_scale, void *stream);
/* *groups = result ciphertexts (gallery groups, or ceil(groups / c) when
 * compressed). */
int bm_result_info(const bm_result *r, uint64_t *groups, uint32_t *limbs, double *scale);
/* Coefficient-domain words[2][limbs][N] of result ciphertext `group`. */
int bm_result_export(const bm_result *r, uint64_t group, uint64_t *words, size_t n_words);
/* Coefficient-domain words[groups][2][limbs][N] of every result ciphertext,
 * in one inverse-transform launch and one device-to-host copy (what a server
 * sends back to the client); n_words must be groups * 2 * limbs * N. */
int bm_result_export_all(const bm_result *r, uint64_t *words, size_t n_words);
void bm_result_free(bm_result *r);

/* Client side (Sec. 3.4): decrypt every result ciphertext, decode, read
 * template g T + b at slot b c of group g (compressed: at slot
 * b c + (g mod c) of ciphertext floor(g / c)).  scores must hold
 * n = n_templates values. */
int bm_decrypt_scores(bm_ctx *ctx, const bm_sk *sk, const bm_result *r, double *scores,
                      uint64_t n);
/* Arg-max of scores[0..n-1] (lowest index on ties); *idx = -1 when the best
 * score is below `threshold` (not enrolled). */
int bm_top1(const double *scores, uint64_t n, double threshold, int64_t *idx, double *best);

/* ------------------------------------------------------------------ serving */

/* Continuous-batching server over device-resident galleries.  Requests are
 * admitted while the scratch they need fits in `hbm_budget_bytes`; admitted
 * requests of equal shape are evaluated together.  A worker thread owns the
 * device; submit and poll are thread-safe. */
int bm_server_create(bm_ctx *ctx, const bm_evk *evk, uint64_t hbm_budget_bytes,
                     uint32_t schedule, bm_server **out);
/* Ownership of the gallery moves to the server. */
int bm_server_add_gallery(bm_server *s, bm_gallery *g, uint32_t *gallery_id);
/* Ownership of the query moves to the server when the call returns BM_OK
 * (on an error the caller keeps it).  BM_EBUDGET if the request can never fit
 * the budget, BM_EDIM for a query encrypted for another d than the gallery,
 * BM_ELEVEL for a query below the level the match needs. */
int bm_server_submit(bm_server *s, uint32_t gallery_id, bm_ct *q, uint64_t *ticket);
/* *out = NULL while the request is pending; then the result (caller frees).
 * Status of a failed request is returned once. */
int bm_server_poll(bm_server *s, uint64_t ticket, bm_result **out);
/* Block until every submitted request finished. */
int bm_server_drain(bm_server *s);
/* Per-request latency statistics in ms (completion minus submission). */
int bm_server_stats(bm_server *s, uint64_t *completed, double *p50_ms, double *p99_ms,
                    double *mean_batch);
/* Clear the latency and batch statistics. */
int bm_server_reset_stats(bm_server *s);
void bm_server_free(bm_server *s);

#ifdef __cplusplus
}
#endif
#endif /* BLINDMATCH_H */
