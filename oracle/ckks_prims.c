/*
 * ckks_prims.c -- plain CPU arithmetic for the CKKS oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the arithmetic floor of the
 * reference oracle that the GPU library is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, table or helper with the HIP library.
 *
 * Everything here is written for obviousness, not speed:
 *   - every modular product is ((unsigned __int128)a * b) % q, no Shoup,
 *     Barrett or Montgomery reduction anywhere;
 *   - the negacyclic product is the textbook one: twist by powers of a
 *     primitive 2N-th root psi, cyclic radix-2 NTT with an explicit
 *     bit-reversal permutation, pointwise product, inverse, untwist;
 *   - SHAKE-256 follows FIPS 202 literally, and even derives its Keccak
 *     round constants and rotation offsets from the defining LFSR and the
 *     (t+1)(t+2)/2 rule instead of transcribing tables.
 *
 * Operations follow the CKKS definitions used by the paper (Sec. 2, the
 * operation list Add / Mul(P) / Mul(C) / Rot / Res); the ring arithmetic
 * they rest on is R_q = Z_q[X]/(X^N + 1).
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* scalar modular arithmetic                                           */
/* ------------------------------------------------------------------ */

static u64 mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }

static u64 powmod(u64 b, u64 e, u64 q)
{
    u64 r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mulmod(r, b, q);
        b = mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}

/* inverse by Fermat: q is prime */
static u64 invmod(u64 a, u64 q) { return powmod(a, q - 2, q); }

u64 or_mulmod(u64 a, u64 b, u64 q) { return mulmod(a, b, q); }
u64 or_powmod(u64 b, u64 e, u64 q) { return powmod(b, e, q); }
u64 or_invmod(u64 a, u64 q) { return invmod(a % q, q); }

/* smallest x >= 2 whose power x^((q-1)/2N) has order exactly 2N
 * (for 2N a power of two that is the same as psi^N == -1). */
u64 or_find_psi(u64 q, u64 N)
{
    for (u64 x = 2; x < q; ++x) {
        u64 psi = powmod(x, (q - 1) / (2 * N), q);
        if (powmod(psi, N, q) == q - 1) return psi;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* textbook NTT negacyclic product                                      */
/* ------------------------------------------------------------------ */

static size_t bitrev(size_t x, int bits)
{
    size_t r = 0;
    for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}

/* in-place cyclic NTT of length n with primitive n-th root w:
 * A[k] = sum_j a[j] w^(jk).  Bit-reverse the input, then iterative
 * Cooley-Tukey butterflies of growing span. */
static void cyclic_ntt(u64 *a, size_t n, u64 w, u64 q)
{
    int bits = 0;
    while (((size_t)1 << bits) < n) ++bits;
    for (size_t i = 0; i < n; ++i) {
        size_t j = bitrev(i, bits);
        if (j > i) { u64 t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        u64 wl = powmod(w, n / len, q);           /* primitive len-th root */
        for (size_t start = 0; start < n; start += len) {
            u64 wk = 1;
            for (size_t k = 0; k < len / 2; ++k) {
                u64 u = a[start + k];
                u64 v = mulmod(a[start + k + len / 2], wk, q);
                a[start + k] = (u + v) % q;
                a[start + k + len / 2] = (u + q - v) % q;
                wk = mulmod(wk, wl, q);
            }
        }
    }
}

/* out = a * b in Z_q[X]/(X^n + 1); a, b in [0, q).  out may alias a or b.
 * Returns 0, or -1 if q has no primitive 2n-th root or allocation fails. */
int or_polymul(u64 q, size_t n, const u64 *a, const u64 *b, u64 *out)
{
    u64 psi = or_find_psi(q, n);
    if (!psi) return -1;
    u64 psi_inv = invmod(psi, q);
    u64 w = mulmod(psi, psi, q);           /* primitive n-th root */
    u64 w_inv = invmod(w, q);
    u64 n_inv = invmod(n % q, q);
    u64 *ta = (u64 *)malloc(n * sizeof(u64));
    u64 *tb = (u64 *)malloc(n * sizeof(u64));
    if (!ta || !tb) { free(ta); free(tb); return -1; }
    /* twist: a_i psi^i turns the negacyclic convolution into a cyclic one */
    u64 pw = 1;
    for (size_t i = 0; i < n; ++i) {
        ta[i] = mulmod(a[i] % q, pw, q);
        tb[i] = mulmod(b[i] % q, pw, q);
        pw = mulmod(pw, psi, q);
    }
    cyclic_ntt(ta, n, w, q);
    cyclic_ntt(tb, n, w, q);
    for (size_t i = 0; i < n; ++i) ta[i] = mulmod(ta[i], tb[i], q);
    cyclic_ntt(ta, n, w_inv, q);           /* inverse up to the factor n */
    pw = n_inv;
    for (size_t i = 0; i < n; ++i) {       /* scale by 1/n and untwist */
        out[i] = mulmod(ta[i], pw, q);
        pw = mulmod(pw, psi_inv, q);
    }
    free(ta);
    free(tb);
    return 0;
}

/* Independent products, run in parallel across jobs. */
int or_polymul_batch(size_t jobs, size_t n, const u64 *qs, const u64 *const *a,
                     const u64 *const *b, u64 *const *out)
{
    int err = 0;
#pragma omp parallel for schedule(dynamic) reduction(| : err)
    for (long j = 0; j < (long)jobs; ++j)
        err |= (or_polymul(qs[j], n, a[j], b[j], out[j]) != 0);
    return err ? -1 : 0;
}

/* schoolbook negacyclic product, O(n^2): used only as a pin on small n */
void or_polymul_schoolbook(u64 q, size_t n, const u64 *a, const u64 *b, u64 *out)
{
    for (size_t k = 0; k < n; ++k) out[k] = 0;
    for (size_t i = 0; i < n; ++i)
        for (size_t j = 0; j < n; ++j) {
            u64 p = mulmod(a[i], b[j], q);
            size_t k = i + j;
            if (k < n) out[k] = (out[k] + p) % q;
            else out[k - n] = (out[k - n] + q - p) % q;   /* X^n = -1 */
        }
}

/* ------------------------------------------------------------------ */
/* elementwise                                                           */
/* ------------------------------------------------------------------ */

void or_mulmod_vec(u64 q, size_t n, const u64 *a, const u64 *b, u64 *out)
{
#pragma omp parallel for if (n > 65536)
    for (long i = 0; i < (long)n; ++i) out[i] = mulmod(a[i], b[i], q);
}

/* out[i] = (a[i] * c) mod q for any 64-bit a[i] */
void or_mulmod_scalar(u64 q, size_t n, const u64 *a, u64 c, u64 *out)
{
#pragma omp parallel for if (n > 65536)
    for (long i = 0; i < (long)n; ++i) out[i] = mulmod(a[i], c, q);
}

/* ------------------------------------------------------------------ */
/* Keccak-f[1600] and SHAKE-256 (FIPS 202)                              */
/* ------------------------------------------------------------------ */

static u64 rc_table[24];
static int rho_offset[5][5];
static int keccak_ready = 0;

/* rc(t): output bit of the LFSR x^8 + x^6 + x^5 + x^4 + 1 (FIPS 202 Alg. 5) */
static int lfsr_rc(int t)
{
    if (t % 255 == 0) return 1;
    unsigned R = 0x80;                      /* R = 10000000, bit 0 is leftmost */
    for (int i = 1; i <= t % 255; ++i) {
        /* R = 0 || R, then taps at positions 0,4,5,6 take R[8] */
        unsigned r8 = R & 1;                /* position 7 before the shift */
        R >>= 1;                             /* prepend a 0 on the left */
        if (r8) R ^= 0x80 | 0x08 | 0x04 | 0x02;   /* positions 0,4,5,6 */
    }
    return (R >> 7) & 1;                    /* leftmost bit R[0] */
}

static void keccak_init_tables(void)
{
    if (keccak_ready) return;
    for (int ir = 0; ir < 24; ++ir) {
        u64 rc = 0;
        for (int j = 0; j <= 6; ++j)
            if (lfsr_rc(j + 7 * ir)) rc |= (u64)1 << ((1 << j) - 1);
        rc_table[ir] = rc;
    }
    memset(rho_offset, 0, sizeof(rho_offset));
    int x = 1, y = 0;
    for (int t = 0; t < 24; ++t) {
        rho_offset[x][y] = (((t + 1) * (t + 2)) / 2) % 64;
        int nx = y, ny = (2 * x + 3 * y) % 5;
        x = nx; y = ny;
    }
    keccak_ready = 1;
}

static u64 rotl(u64 v, int r) { return r ? (v << r) | (v >> (64 - r)) : v; }

/* A[x][y] lanes, lane (x,y) is bytes 8*(x+5y) of the state */
static void keccak_f1600(u64 A[5][5])
{
    for (int ir = 0; ir < 24; ++ir) {
        u64 C[5], D[5], B[5][5];
        for (int x = 0; x < 5; ++x) C[x] = A[x][0] ^ A[x][1] ^ A[x][2] ^ A[x][3] ^ A[x][4];
        for (int x = 0; x < 5; ++x) D[x] = C[(x + 4) % 5] ^ rotl(C[(x + 1) % 5], 1);
        for (int x = 0; x < 5; ++x)
            for (int y = 0; y < 5; ++y) A[x][y] ^= D[x];                 /* theta */
        for (int x = 0; x < 5; ++x)
            for (int y = 0; y < 5; ++y)                                     /* rho, pi */
                B[y][(2 * x + 3 * y) % 5] = rotl(A[x][y], rho_offset[x][y]);
        for (int x = 0; x < 5; ++x)
            for (int y = 0; y < 5; ++y)                                     /* chi */
                A[x][y] = B[x][y] ^ ((~B[(x + 1) % 5][y]) & B[(x + 2) % 5][y]);
        A[0][0] ^= rc_table[ir];                                            /* iota */
    }
}

typedef struct {
    u64 A[5][5];
    unsigned char buf[136];
    size_t pos;          /* bytes of buf already handed out */
} shake_t;

enum { SHAKE256_RATE = 136 };

static void state_xor_bytes(u64 A[5][5], const unsigned char *p, size_t len)
{
    for (size_t i = 0; i < len; ++i) {
        size_t lane = i / 8;
        A[lane % 5][lane / 5] ^= (u64)p[i] << (8 * (i % 8));
    }
}

static void state_get_bytes(u64 A[5][5], unsigned char *p, size_t len)
{
    for (size_t i = 0; i < len; ++i) {
        size_t lane = i / 8;
        p[i] = (unsigned char)(A[lane % 5][lane / 5] >> (8 * (i % 8)));
    }
}

static void shake_absorb_all(shake_t *s, const unsigned char *in, size_t inlen)
{
    keccak_init_tables();
    memset(s->A, 0, sizeof(s->A));
    while (inlen >= SHAKE256_RATE) {
        state_xor_bytes(s->A, in, SHAKE256_RATE);
        keccak_f1600(s->A);
        in += SHAKE256_RATE; inlen -= SHAKE256_RATE;
    }
    unsigned char last[SHAKE256_RATE];
    memset(last, 0, sizeof(last));
    memcpy(last, in, inlen);
    last[inlen] ^= 0x1F;                   /* SHAKE domain bits 1111 + pad10*1 start */
    last[SHAKE256_RATE - 1] ^= 0x80;       /* pad10*1 end */
    state_xor_bytes(s->A, last, SHAKE256_RATE);
    keccak_f1600(s->A);
    state_get_bytes(s->A, s->buf, SHAKE256_RATE);
    s->pos = 0;
}

static void shake_squeeze(shake_t *s, unsigned char *out, size_t len)
{
    while (len) {
        if (s->pos == SHAKE256_RATE) {
            keccak_f1600(s->A);
            state_get_bytes(s->A, s->buf, SHAKE256_RATE);
            s->pos = 0;
        }
        size_t take = SHAKE256_RATE - s->pos;
        if (take > len) take = len;
        memcpy(out, s->buf + s->pos, take);
        s->pos += take; out += take; len -= take;
    }
}

void or_shake256(const unsigned char *in, size_t inlen, unsigned char *out, size_t outlen)
{
    shake_t s;
    shake_absorb_all(&s, in, inlen);
    shake_squeeze(&s, out, outlen);
}

/* Stream for (seed, domain, index): SHAKE-256 over le64(seed) || le32(domain)
 * || le64(index), read as little-endian 64-bit words. */
static void stream_open(shake_t *s, u64 seed, uint32_t domain, u64 index)
{
    unsigned char msg[20];
    for (int i = 0; i < 8; ++i) msg[i] = (unsigned char)(seed >> (8 * i));
    for (int i = 0; i < 4; ++i) msg[8 + i] = (unsigned char)(domain >> (8 * i));
    for (int i = 0; i < 8; ++i) msg[12 + i] = (unsigned char)(index >> (8 * i));
    shake_absorb_all(s, msg, sizeof(msg));
}

static u64 stream_word(shake_t *s)
{
    unsigned char b[8];
    shake_squeeze(s, b, 8);
    u64 w = 0;
    for (int i = 0; i < 8; ++i) w |= (u64)b[i] << (8 * i);
    return w;
}

void or_stream_words(u64 seed, uint32_t domain, u64 index, u64 *out, size_t n)
{
    shake_t s;
    stream_open(&s, seed, domain, index);
    for (size_t i = 0; i < n; ++i) out[i] = stream_word(&s);
}

/* uniform ternary {-1,0,1}: reject u >= 3*floor(2^64/3), value (u mod 3) - 1 */
void or_sample_ternary(u64 seed, uint32_t domain, u64 index, int64_t *out, size_t n)
{
    shake_t s;
    stream_open(&s, seed, domain, index);
    const u64 bound = 3 * (UINT64_MAX / 3);   /* 3*floor((2^64-1)/3) == 3*floor(2^64/3) */
    for (size_t i = 0; i < n; ++i) {
        u64 u;
        do { u = stream_word(&s); } while (u >= bound);
        out[i] = (int64_t)(u % 3) - 1;
    }
}

/* cumulative-table sampler: x = lo + #{i : u >= cdt[i]} */
void or_sample_cdt(u64 seed, uint32_t domain, u64 index, const u64 *cdt, size_t ncdt,
                   int64_t lo, int64_t *out, size_t n)
{
    shake_t s;
    stream_open(&s, seed, domain, index);
    for (size_t i = 0; i < n; ++i) {
        u64 u = stream_word(&s);
        int64_t c = 0;
        for (size_t k = 0; k < ncdt; ++k) c += (u >= cdt[k]);
        out[i] = lo + c;
    }
}

/* uniform mod each prime, limb after limb: u & (2^bitlen(q) - 1), kept if < q */
void or_sample_uniform(u64 seed, uint32_t domain, u64 index, const u64 *qs, size_t nq,
                       size_t n, u64 *out)
{
    shake_t s;
    stream_open(&s, seed, domain, index);
    for (size_t l = 0; l < nq; ++l) {
        u64 q = qs[l];
        int bits = 0;
        while (bits < 64 && (q >> bits)) ++bits;
        u64 mask = bits >= 64 ? UINT64_MAX : (((u64)1 << bits) - 1);
        for (size_t i = 0; i < n; ++i) {
            u64 u;
            do { u = stream_word(&s) & mask; } while (u >= q);
            out[l * n + i] = u;
        }
    }
}
