// kernels.hip -- gfx950 kernels of the RNS-CKKS evaluator.
//
// All arithmetic is exact modular integer arithmetic on 64-bit words with
// primes below 2^51 (no MFMA: nothing here is a dense contraction).  The NTT,
// the key inner products and the tensor carry residues as exact integers in
// FP64, which the VALU issues at full rate; the other element-wise kernels use
// 32-bit integer arithmetic: Shoup's precomputed quotient for constant
// operands, Montgomery reduction with R = 2^64 for variable products.
//
// Grids are (element chunks, limb slot, batch element): blockIdx.y picks the
// limb (and with it the prime, uniform across the block so its constants come
// from scalar loads) and blockIdx.z the polynomial of the batch.
#include <algorithm>
#include <cstdlib>

#include <hip/hip_ext.h>

#include "bm_internal.hpp"
#include "fp64_modarith.hpp"

namespace bm {
namespace {

__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q) {
  u64 s = a + b;
  return s >= q ? s - q : s;
}
__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + (q - b); }

// a * w mod q for any 64-bit a, w < q, ws = floor(w 2^64 / q)
__device__ __forceinline__ u64 mul_shoup(u64 a, u64 w, u64 ws, u64 q) {
  u64 qh = __umul64hi(a, ws);
  u64 r = a * w - qh * q;
  return r >= q ? r - q : r;
}

// a * b * 2^-64 mod q for a < 2^64, b < q (Montgomery, qn = -q^-1 mod 2^64)
__device__ __forceinline__ u64 mont_mul(u64 a, u64 b, u64 q, u64 qn) {
  u64 lo = a * b;
  u64 hi = __umul64hi(a, b);
  u64 m = lo * qn;
  u64 t = hi + __umul64hi(m, q) + (lo != 0);
  return t >= q ? t - q : t;
}

// plain a * b mod q
__device__ __forceinline__ u64 mul_mod(u64 a, u64 b, const PrimeC& p) {
  return mont_mul(mont_mul(a, b, p.q, p.qn), p.r2, p.q, p.qn);
}

// any 64-bit word mod q (Shoup with w = 1)
__device__ __forceinline__ u64 reduce64(u64 a, const PrimeC& p) { return mul_shoup(a, 1, p.pad[0], p.q); }

// kernel launch; skipped (checks only) in dry-run mode
// Every launch sits in the scope of a Prof named pf.  With profiling on, the
// kernel is launched with its own start/stop events, which the runtime stamps
// with the kernel's execution interval (dispatch latency excluded).
#define LAUNCH(F, G, BL, L, S, ...)                                                   \
  do {                                                                                \
    if (dev::dry() || dev::sizing()) break;                                           \
    if (pf.on)                                                                        \
      hipExtLaunchKernelGGL(F, G, BL, L, S, pf.ev.first, pf.ev.second, 0, __VA_ARGS__); \
    else                                                                              \
      hipLaunchKernelGGL(F, G, BL, L, S, __VA_ARGS__);                                \
  } while (0)

constexpr int TPB = 256;        // threads per block of every kernel here
constexpr int NTT_E = 4096;     // words per NTT block held in LDS

// ---------------------------------------------------------------- NTT
//
// Forward: Cooley-Tukey with the negacyclic twist merged into the twiddles
// (W[k] = psi^{brv(k)}); stage s pairs (j, j + N/2^{s+1}) inside block
// i = j / (N/2^s) with twiddle W[2^s + i].  The output is in bit-reversed
// order: position j holds a(psi^{2 brv(j) + 1}).  Inverse: Gentleman-Sande
// with psi^{-1} in reverse stage order, then the factor N^{-1}.
//
// For N > 4096 the stages split into two passes over an N1 x N2 view of the
// limb: the first log N1 stages act on N2 columns of length N1 with the same
// twiddles for every column, the remaining log N2 stages act on N1 rows of
// length N2 with row-dependent twiddles.  One block holds 4096 words: V views
// of M = 2^logm elements, padded by one word per view in LDS.

template <bool INV>
__global__ void __launch_bounds__(TPB) k_ntt_pass(const u64* __restrict__ in, size_t in_stride,
                                                  u64* __restrict__ out, size_t out_stride,
                                                  LimbMap m, const PrimeC* __restrict__ P,
                                                  const u64* __restrict__ tw,
                                                  const u64* __restrict__ tws, int log_n, int logm,
                                                  int s0, int col, int last) {
  extern __shared__ u64 sh[];
  const int N = 1 << log_n;
  const int M = 1 << logm;
  const int E = N < NTT_E ? N : NTT_E;
  const int V = E / M;
  const int slot = blockIdx.y;
  const int pid = m.prime[slot];
  const u64 q = P[pid].q;
  const u64* W = tw + (size_t)pid * N;
  const u64* WS = tws + (size_t)pid * N;
  const u64* src = in + (size_t)blockIdx.z * in_stride + (size_t)m.off[slot] * N;
  u64* dst = out + (size_t)blockIdx.z * out_stride + (size_t)m.ooff[slot] * N;
  const int v0 = blockIdx.x * V;
  const int cstride = N >> logm;   // distance between consecutive elements of a column
  const int MP = M + 1;            // padded view length in LDS

  for (int e = threadIdx.x; e < E; e += TPB) {
    int a, v;
    size_t g;
    if (col) { a = e / V; v = e % V; g = (size_t)a * cstride + (v0 + v); }
    else     { v = e / M; a = e % M; g = (size_t)(v0 + v) * M + a; }
    sh[v * MP + a] = src[g];
  }
  __syncthreads();

  const int halfM = M >> 1;
  const int nbf = V * halfM;
  if (!INV) {
    for (int sp = 0; sp < logm; ++sp) {
      const int h = M >> (sp + 1);
      for (int bf = threadIdx.x; bf < nbf; bf += TPB) {
        const int v = bf / halfM, kk = bf % halfM;
        const int i = kk / h, r = kk % h;
        const int a0 = 2 * i * h + r;
        const int vb = col ? 0 : (v0 + v);
        const int tix = (1 << (s0 + sp)) + (vb << sp) + i;
        u64* x = sh + v * MP;
        const u64 U = x[a0];
        const u64 T = mul_shoup(x[a0 + h], W[tix], WS[tix], q);
        x[a0] = add_mod(U, T, q);
        x[a0 + h] = sub_mod(U, T, q);
      }
      __syncthreads();
    }
  } else {
    for (int sp = logm - 1; sp >= 0; --sp) {
      const int h = M >> (sp + 1);
      for (int bf = threadIdx.x; bf < nbf; bf += TPB) {
        const int v = bf / halfM, kk = bf % halfM;
        const int i = kk / h, r = kk % h;
        const int a0 = 2 * i * h + r;
        const int vb = col ? 0 : (v0 + v);
        const int tix = (1 << (s0 + sp)) + (vb << sp) + i;
        u64* x = sh + v * MP;
        const u64 U = x[a0], Vv = x[a0 + h];
        x[a0] = add_mod(U, Vv, q);
        x[a0 + h] = mul_shoup(U + (q - Vv), W[tix], WS[tix], q);
      }
      __syncthreads();
    }
  }

  const u64 ninv = P[pid].ninv, ninv_s = P[pid].ninv_s;
  for (int e = threadIdx.x; e < E; e += TPB) {
    int a, v;
    size_t g;
    if (col) { a = e / V; v = e % V; g = (size_t)a * cstride + (v0 + v); }
    else     { v = e / M; a = e % M; g = (size_t)(v0 + v) * M + a; }
    u64 x = sh[v * MP + a];
    if (last) x = mul_shoup(x, ninv, ninv_s, q);
    dst[g] = x;
  }
}

// ---------------------------------------------------------------- register-radix NTT
//
// Same transform as k_ntt_pass, organised for gfx950: every thread keeps 16
// words of one view in registers and applies four butterfly stages to them
// (a radix-16 phase) before the view is exchanged through LDS; a pass of 8
// stages is two phases, the single pass of N = 4096 is three.  Indices are
// shifts and masks only.  Twiddles of the block are staged once in LDS (8-stage
// passes) or read through the cache (12-stage pass).
//
// Arithmetic is exact integer arithmetic carried in FP64, which the CDNA4
// VALU issues at the full rate where 32-bit integer multiplies run at about
// half of it.  Residues (q < 2^51) are integers held in doubles; every
// intermediate stays an integer of magnitude below 2^53, so every operation
// below is exact:
//   fmul_mod(a, w) = a w - rint(a (w/q)) q, computed as hi = fl(a w),
//     lo = a w - hi (one FMA, exact), r = (hi - qt q) + lo (one FMA whose
//     exact result is an integer below 2^53, then an exact add).  The
//     quotient estimate is within 0.5 + |a| 2^-52 of a w / q, so
//     |r| <= q (0.5 + |a| 2^-52 (1 + 2^-52)).
//   fred(a) = a - rint(a / q) q lies in [-q/2 - 1, q/2 + 1].
// Values are brought back to |x| <= q/2 + 1 before the third stage of every
// phase and before the first stage of every phase but the first, which
// starts from residues in [0, q).  Forward (CT): from 0.5q two stages give
// 1.25q and then 2.375q (the multiplied inputs stay below 1.25q, so every
// product is below 1.13q); from [0, q) they give 2q and then 3.5q.  Inverse
// (GS): from 0.5q two stages give 1q and then 2q; from [0, q), 2q and then
// 4q (the difference fed to the product stays below 4q, so it is below
// 2.5q).  With q < 2^51 all of these stay below 2^53.  Each pass ends with
// fred and a conditional +q, so passes exchange exact residues in [0, q) as
// 64-bit words.
//
// Pass kinds: COL = columns of length 256 of one polynomial (first 8 stages of
// N = 2^16, twiddles common to all columns); ROW = one row of length 256
// taken from V polynomials that share the prime (last 8 stages, row twiddles);
// ONE = a whole N = 4096 polynomial.

// The arithmetic itself (fmul_mod, fmul_mod_q, fred, the exact conversions,
// FAcc and the radix-16 phases) lives in fp64_modarith.hpp, shared with a
// host build that checks it against exact integers at the extremes of these
// bounds.
using fpm::fmul_mod;
using fpm::fmul_mod_q;
using fpm::fred;
using fpm::u64_to_f;
using fpm::f_to_u64;
using fpm::FAcc;

// Issue-rate probe of the butterfly arithmetic above, register-resident: each
// thread runs 8 independent chains of forward butterflies (u, v) <- (u + t,
// u - t), t = fmul_mod(v, w), and folds both values back with fred after
// every second round, as the NTT passes do.  Values stay below 2.2 q < 2^53.
// Thread x starts chain j from u = (seed[j] + x) mod q, v = (seed[8 + j] + 3x)
// mod q with twiddle w = seed[16 + j] < q, and stores its 8 final (u, v) pairs
// as residues in [0, q) at out[16 x ...].
__global__ void __launch_bounds__(256) k_modmul_rate(const PrimeC* __restrict__ P, int pid, int iters,
                                                     const u64* __restrict__ seed, u64* __restrict__ out) {
  const PrimeC& pr = P[pid];
  const double q = (double)pr.q, qi = __longlong_as_double((long long)pr.pad[1]);
  const u64 x = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  double u[8], v[8], w[8], wq[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    u[j] = u64_to_f((seed[j] + x) % pr.q);
    v[j] = u64_to_f((seed[8 + j] + 3 * x) % pr.q);
    w[j] = u64_to_f(seed[16 + j]);
    wq[j] = w[j] / q;
  }
  for (int it = 0; it < iters; it += 2) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double t = fmul_mod(v[j], w[j], wq[j], q);
        const double a = __dadd_rn(u[j], t);
        v[j] = __dsub_rn(u[j], t);
        u[j] = a;
      }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      u[j] = fred(u[j], qi, q);
      v[j] = fred(v[j], qi, q);
    }
  }
  u64* o = out + 16 * x;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double a = u[j] < 0.0 ? __dadd_rn(u[j], q) : u[j];
    const double b = v[j] < 0.0 ? __dadd_rn(v[j], q) : v[j];
    o[2 * j] = f_to_u64(a);
    o[2 * j + 1] = f_to_u64(b);
  }
}

enum { NTT_COL = 0, NTT_ROW = 1, NTT_ONE = 2 };

// FUSE = 1: forward column pass whose input words come from f's prologue;
// FUSE = 2: forward row pass that stores through f's epilogue;
// FUSE = 3: forward row pass that stores the residues as FP64 values;
// FUSE = 4: as 1, in the conjugate-invariant ring (sources not yet unfolded).
// PK / EK fix the prologue kind (f.pro) of a fused column pass and the
// epilogue kind (f.epi) of a fused row pass at compile time, so that each
// instantiation holds only the registers of its own prologue or epilogue
// (0: taken from f at run time).
// OCC > 0 asks the compiler for OCC resident blocks of 256 threads per CU
// (a register budget of 512 / OCC per lane, spilling if it must): a tuning
// alternative for the register-heavy fused column passes.
// IS = 1 (FUSE = 1): the sources hold only the row pass of their inverse
// transform; the block finishes it on each source tile (f.isrc).
template <int LOGM, bool INV, int KIND, int FUSE = 0, int PK = 0, int EK = 0, int OCC = 0, int IS = 0>
__global__ void __launch_bounds__(256, OCC > 0 ? OCC : 1) k_ntt_fast(const u64* __restrict__ in, size_t in_stride,
                                                  u64* __restrict__ out, size_t out_stride,
                                                  LimbMap m, const PrimeC* __restrict__ P,
                                                  const double* __restrict__ twf,
                                                  const double* __restrict__ twq, int log_n, int s0,
                                                  int last, int B, int vz, FuseArgs f) {
  static_assert(FUSE == 0 || (!INV && (((FUSE == 1 || FUSE == 4) && KIND == NTT_COL) ||
                                       ((FUSE == 2 || FUSE == 3) && KIND == NTT_ROW))),
                "fused prologues serve forward column passes, epilogues forward row passes");
  static_assert(IS == 0 || (FUSE == 1 && LOGM == 8), "inverse source passes serve the fused column pass");
  const int pro = PK ? PK : f.pro;           // compile-time constant in the fused instantiations
  const int epi = EK ? EK : f.epi;
  constexpr bool PRO = FUSE == 1 || FUSE == 4;
  constexpr int M = 1 << LOGM;
  constexpr int TPV = M / 16;                 // threads per view
  // padded view length in LDS.  Column passes put 16 views side by side in a
  // wave (odd stride: the views land on distinct banks); row passes put 4
  // views of 16 lanes each, whose padded offsets 17 u (mod 32 doubles) fill
  // half of the banks, so a stride of 16 (mod 32) gives the next view the
  // other half.
  constexpr int VS = KIND == NTT_ROW ? M + M / 16 : M + M / 16 + 1;
  constexpr int PH = LOGM / 4;                // radix-16 phases
  extern __shared__ u64 sh_raw[];
  double* sh = reinterpret_cast<double*>(sh_raw);
  const int t = threadIdx.x;
  const int V = (int)blockDim.x / TPV;        // views in this block
  // Row passes take vz polynomials x R consecutive rows per block (R = V / vz),
  // so that small batches still fill whole waves; every row stages its own
  // twiddles (w, w/q) after the views in LDS.  Other passes: R = 1.
  const int R = KIND == NTT_ROW ? V / vz : 1;
  // [R][2][256] block twiddles (8-stage passes): w, then w/q, each in the
  // order tw_slot() gives, in which the lanes of a view read consecutive words
  double* tl = sh + V * VS;
  const int nthr = (int)blockDim.x;
  const int pid = m.prime[blockIdx.y];
  const PrimeC& pr = P[pid];
  const double q = (double)pr.q;
  const double qi = __longlong_as_double((long long)pr.pad[1]);   // 1/q
  const int N = 1 << log_n;
  const double* W = twf + (size_t)pid * N;
  const double* WQ = twq + (size_t)pid * N;
  auto pad = [](int a) { return a + (a >> 4); };

  // Lane layout: in a column pass consecutive lanes take consecutive columns
  // (views); otherwise consecutive lanes take consecutive words of one view.
  const int v = KIND == NTT_COL ? (t & 15) : t / TPV;
  const int u = KIND == NTT_COL ? (t >> 4) : t % TPV;
  // Global address of view word a: base + a * astride.
  size_t base_in, base_out, astride;
  bool valid = true;
  // FUSE = 4: block b takes columns 8b .. 8b+7 and their mirrors 256 - c, so
  // that word k and word N - k of the polynomial sit in one block (columns 0
  // and 128 are their own mirrors; block 0 takes 128 in place of 256 - 0)
  auto ci_col = [&](int vv) {
    const int b = blockIdx.x;
    return vv < 8 ? 8 * b + vv : (vv == 8 && b == 0 ? 128 : 256 - (8 * b + vv - 8));
  };
  if (KIND == NTT_COL) {
    astride = (size_t)(N >> LOGM);
    const size_t col = FUSE == 4 ? (size_t)ci_col(v) : (size_t)blockIdx.x * 16 + v;
    base_in = (size_t)blockIdx.z * in_stride + (size_t)m.off[blockIdx.y] * N + col;
    base_out = (size_t)blockIdx.z * out_stride + (size_t)m.ooff[blockIdx.y] * N + col;
  } else if (KIND == NTT_ROW) {
    astride = 1;
    const int z = blockIdx.z * vz + v % vz;
    const size_t row = (size_t)blockIdx.x * R + v / vz;
    valid = z < B;
    const size_t zz = valid ? (size_t)z : 0;
    base_in = zz * in_stride + (size_t)m.off[blockIdx.y] * N + row * M;
    base_out = zz * out_stride + (size_t)m.ooff[blockIdx.y] * N + row * M;
  } else {
    astride = 1;
    base_in = (size_t)blockIdx.z * in_stride + (size_t)m.off[blockIdx.y] * N;
    base_out = (size_t)blockIdx.z * out_stride + (size_t)m.ooff[blockIdx.y] * N;
  }
  const u64* src = in + base_in;
  u64* dst = out + base_out;

  double x[16];
  // phase p holds a = hi * 2^(LOGM-4p) + j * 2^(LOGM-4p-4) + lo,  u = hi * 2^(LOGM-4p-4) + lo
  auto addr = [&](int p, int j) {
    const int sh_lo = LOGM - 4 * p - 4;
    const int hi = u >> sh_lo, lo = u & ((1 << sh_lo) - 1);
    return (hi << (LOGM - 4 * p)) + (j << sh_lo) + lo;
  };
  // A phase mapping is "direct" when lanes that differ in the fastest lane
  // index touch consecutive global words: always for columns (lanes run over
  // columns), and for the phase with lo = u (p = 0) otherwise.
  constexpr int P_FIRST = INV ? PH - 1 : 0;
  constexpr int P_LAST = INV ? 0 : PH - 1;
  constexpr bool DIRECT_IN = KIND == NTT_COL || P_FIRST == 0;
  constexpr bool DIRECT_OUT = KIND == NTT_COL || P_LAST == 0;

  // data loads first, so that their latency overlaps the twiddle staging
  u64 raw[16] = {};
  if (!PRO && valid) {
#pragma unroll
    for (int j = 0; j < 16; ++j) raw[j] = src[(size_t)(DIRECT_IN ? addr(P_FIRST, j) : addr(0, j)) * astride];
  }
  // FUSE = 1: the words of the first source are requested here, before the
  // twiddles are staged, and combined after (see below)
  const u64* S = nullptr;
  int ns = 0, jd = 0, tt = 0;
  u64 r0[FUSE == 1 ? 16 : 1];
  (void)r0;
  // source a of slot blockIdx.y: limb offset, prime, and the two constants
  auto src_info = [&](int a, int& soff, int& spid, u64& c1, u64& c2) {
    if (pro == 1) {
      const ModUpDigit& dg = f.mu->d[jd];
      soff = spid = dg.src[a];
      c1 = dg.qhatinv[a][0];
      c2 = dg.qhat[a][tt][0];
    } else {
      soff = f.s_off0 + a;
      spid = f.md->pprime[a];
      c1 = f.md->phatinv[a][0];
      c2 = f.md->phat[a][blockIdx.y][0];
    }
  };
  if constexpr (PRO) {
    const size_t zz = blockIdx.z;
    S = f.src + (zz / f.s_div) * f.s_hi + (zz % f.s_div) * f.s_lo +
        (FUSE == 4 ? (size_t)ci_col(v) : (size_t)blockIdx.x * 16 + v);
    if (pro == 3) {
      ns = 1;
    } else {
      jd = pro == 1 ? f.mu->pair_j[blockIdx.y] : 0;
      tt = pro == 1 ? f.mu->pair_t[blockIdx.y] : 0;
      ns = pro == 1 ? f.mu->d[jd].nsrc : f.md->K;
    }
    int soff = 0, spid;
    u64 c1, c2;
    if (pro != 3) src_info(0, soff, spid, c1, c2);
    if constexpr (FUSE == 1 && !IS) {
#pragma unroll
      for (int j = 0; j < 16; ++j) r0[j] = S[((size_t)soff * N) + (size_t)addr(0, j) * astride];
    }
  }
  // IS: source a's prime (source 0 .. is_n - 1 of this block)
  auto is_pid = [&](int a) {
    if (pro == 1) return f.mu->d[jd].src[a];
    if (pro == 2) return f.md->pprime[a];
    if (pro == 3) return f.src_pid;
    return a < f.md->K ? f.md->pprime[a] : f.last_pid;
  };
  const int is_n = IS ? (pro == 4 ? f.md->K + 1 : ns) : 0;
  (void)is_pid;
  (void)is_n;
  // FUSE = 2: the epilogue's operands are requested here as well
  u64 mr[FUSE == 2 ? 16 : 1], ar[FUSE == 2 ? 16 : 1];
  const u64* Ad = nullptr;
  u64* Oe = nullptr;
  if constexpr (FUSE == 2) {
    if (valid) {
      const int slot = blockIdx.y;
      const size_t zz = blockIdx.z * vz + v % vz;
      const size_t hi = zz / f.e_div, lo = zz % f.e_div;
      const size_t pos = ((size_t)blockIdx.x * R + v / vz) * M + (size_t)slot * N;
      const u64* Mn = f.mnd + hi * f.m_hi + lo * f.m_lo + pos;
      Ad = lo == 0 ? (f.add0 ? f.add0 + hi * f.a0_hi + pos : nullptr)
                   : (f.add1 ? f.add1 + hi * f.a1_hi + pos : nullptr);
      Oe = (f.out_ref ? *f.out_ref + f.out_rel : f.out) + hi * f.o_hi + lo * f.o_lo + pos;
#pragma unroll
      for (int j = 0; j < 16; ++j) mr[j] = Mn[addr(0, j)];
      if (Ad) {
#pragma unroll
        for (int j = 0; j < 16; ++j) ar[j] = Ad[addr(0, j)];
      }
    }
  }
  // ---- stage the block's twiddles (8-stage passes).  Stage st (0..7) of the
  // pass uses 2^st twiddles b; in stages 4..7 lane hi of a view reads
  // b = (hi << k) + jj (k = st - 4, jj < 2^k), so they are kept at
  // 2^st + jj * 16 + hi: consecutive lanes, consecutive words.
  if (LOGM == 8) {
    // consecutive threads fill consecutive slots (conflict-free LDS writes);
    // four slots a thread at a time, all eight words requested before the
    // first is stored (a row pass of few polynomials stages up to 16 rows'
    // twiddles per thread, and one round trip per slot would dominate it)
    for (int k0 = t; k0 < 256 * R; k0 += 4 * nthr) {
      double sw_w[4], sw_q[4];   // staged words (names apart from the kernel's twf / twq)
      int at[4];
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4) {
        const int k = k0 + c4 * nthr;
        const int slot = k & 255, rr = k >> 8;
        at[c4] = k < 256 * R && slot != 0 ? rr * 512 + slot : -1;
        const int vb = KIND == NTT_ROW ? (int)blockIdx.x * R + rr : 0;
        const int st = 31 - __clz(slot | 1);
        const int o = slot - (1 << st);
        const int b = st < 4 ? o : ((o & 15) << (st - 4)) + (o >> 4);
        const int g = (1 << (s0 + st)) + (vb << st) + b;
        sw_w[c4] = at[c4] >= 0 ? W[g] : 0.0;
        sw_q[c4] = at[c4] >= 0 ? WQ[g] : 0.0;
      }
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4) {
        if (at[c4] >= 0) {
          tl[at[c4]] = sw_w[c4];
          tl[at[c4] + 256] = sw_q[c4];
        }
      }
    }
    if constexpr (IS) {
      // the inverse twiddles of every source prime, [a][2][256] after the
      // block's own, in the same order
      for (int k = t; k < 256 * is_n; k += nthr) {
        const int slot = k & 255, a = k >> 8;
        if (slot == 0) continue;
        const int st = 31 - __clz(slot);
        const int o = slot - (1 << st);
        const int b = st < 4 ? o : ((o & 15) << (st - 4)) + (o >> 4);
        const size_t g = (size_t)is_pid(a) * N + (1 << st) + b;
        tl[512 * (a + 1) + slot] = f.itwf[g];
        tl[512 * (a + 1) + 256 + slot] = f.itwq[g];
      }
    }
  }
  if constexpr (PRO) {
    // input word j (coefficient (addr(0, j) * astride + column)) from the sources:
    // ModUp / ModDown: sum_a [X_a q1_a]_{m_a} q2_a mod q (fast base conversion,
    // the bracket the exact residue in [0, m_a)); one limb: X mod q.
    if constexpr (IS) {
      // Each source tile first gets the column pass of its inverse transform
      // (the 8 Gentleman-Sande stages of the first-pass words, times N^-1,
      // with the word mapping of the inverse column kernel): its words are
      // then the exact coefficient-domain residues at addr(0, j), the words
      // the conversion below needs.  Same operations, same words as the
      // separate inverse column pass.
      __syncthreads();                          // twiddles staged
      // exact: finish with N^-1 and the exact residues in [0, q_a); otherwise
      // the words stay the stages' output (|w| <= 2 q_a), for a caller that
      // folds N^-1 into its own constant
      auto inv_col = [&](double (&w)[16], int a, int spid, bool exact) {
        const PrimeC& ps = P[spid];
        const double qs = (double)ps.q, qsi = __longlong_as_double((long long)ps.pad[1]);
        const double* ta = tl + 512 * (a + 1);
        // (a stage's twiddles are read at the stage: the scheduler keeps them
        // out of the registers of the earlier stages)
        auto tw1 = [&](int k, int j, double& ww, double& wq) {
          if (j == 0) __builtin_amdgcn_sched_barrier(0);
          const int slot = (1 << (4 + k)) + ((j >> (4 - k)) << 4) + u;
          ww = ta[slot];
          wq = ta[256 + slot];
        };
        fpm::gs_phase16(w, false, qsi, qs, tw1);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) sh[v * VS + pad(addr(1, j))] = w[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) w[j] = sh[v * VS + pad(addr(0, j))];
        auto tw0 = [&](int k, int j, double& ww, double& wq) {
          if (j == 0) __builtin_amdgcn_sched_barrier(0);
          const int slot = (1 << k) + (j >> (4 - k));
          ww = ta[slot];
          wq = ta[256 + slot];
        };
        fpm::gs_phase16(w, true, qsi, qs, tw0);
        if (!exact) return;
        const double ni = (double)ps.ninv, niq = __longlong_as_double((long long)ps.pad[2]);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const double r = fred(fmul_mod(w[j], ni, niq, qs), qsi, qs);
          w[j] = r < 0.0 ? __dadd_rn(r, qs) : r;
        }
      };
      // c N^-1 mod m (c < m): the conversion constant that also takes the
      // transform's N^-1, and its quotient
      auto with_ninv = [&](double cd, int spid, double& cn, double& cnq) {
        const PrimeC& ps = P[spid];
        const double ms = (double)ps.q, msi = __longlong_as_double((long long)ps.pad[1]);
        double r = fred(fmul_mod(cd, (double)ps.ninv, __longlong_as_double((long long)ps.pad[2]), ms), msi, ms);
        cn = r < 0.0 ? __dadd_rn(r, ms) : r;
        cnq = cn / ms;
      };
      // source a's first-phase words (a = 0 was requested before the staging)
      auto load = [&](double (&w)[16], int a, size_t soff) {
        (void)a;
#pragma unroll
        for (int j = 0; j < 16; ++j) w[j] = u64_to_f(S[soff * N + (size_t)addr(1, j) * astride]);
      };
      if (pro == 3) {
        double w[16];
        load(w, 0, 0);
        inv_col(w, 0, f.src_pid, true);
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = fred(w[j], qi, q);
      } else if (pro == 4) {
        // as the pro 4 branch below, from the finished source tiles
        const ModDownTable& md = *f.md;
        const int li = f.last_pid, ti = m.prime[blockIdx.y];
        const double ql = (double)P[li].q, qli = __longlong_as_double((long long)P[li].pad[1]);
        const double pl = (double)md.pinv[li][0], plq = pl / ql, pt = (double)md.pinv[ti][0], ptq = pt / q;
        // cl starts from the last limb's word y and takes away each source's
        // term (congruent to the sum the branch below subtracts at the end,
        // with the same exact residue once reduced)
        double cl[16], ci[16];
        load(cl, md.K, (size_t)f.last_off);
        inv_col(cl, md.K, li, true);
        for (int a = 0; a < md.K; ++a) {
          const int ppid = md.pprime[a];
          const double ms = (double)P[ppid].q, msi = __longlong_as_double((long long)P[ppid].pad[1]);
          double c1d, c1q;
          with_ninv((double)md.phatinv[a][0], ppid, c1d, c1q);
          const double hl = (double)md.phat[a][li][0], hlq = hl / ql, ht = (double)md.phat[a][ti][0], htq = ht / q;
          double w[16];
          load(w, a, (size_t)(f.s_off0 + a));
          inv_col(w, a, ppid, false);
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            double t1 = fred(fmul_mod(w[j], c1d, c1q, ms), msi, ms);
            t1 = t1 < 0.0 ? __dadd_rn(t1, ms) : t1;
            const double pL = fmul_mod(t1, hl, hlq, ql), pT = fmul_mod(t1, ht, htq, q);   // each within q
            cl[j] = __dsub_rn(cl[j], pL);
            ci[j] = a == 0 ? pT : __dadd_rn(ci[j], pT);
          }
          if (a & 1) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
              cl[j] = fred(cl[j], qli, ql);
              ci[j] = fred(ci[j], qi, q);
            }
          }
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          double lw = fmul_mod(fred(cl[j], qli, ql), pl, plq, ql);
          lw = fred(lw, qli, ql);
          lw = lw < 0.0 ? __dadd_rn(lw, ql) : lw;                     // exact residue mod q_last
          const double z = __dadd_rn(fmul_mod(fred(ci[j], qi, q), pt, ptq, q), fred(lw, qi, q));
          x[j] = fred(z, qi, q);
        }
      } else {
        for (int a = 0; a < ns; ++a) {
          int soff, spid;
          u64 c1, c2;
          src_info(a, soff, spid, c1, c2);
          const double ms = (double)P[spid].q, msi = __longlong_as_double((long long)P[spid].pad[1]);
          const double c2d = (double)c2, c2q = c2d / q;
          double c1d, c1q;
          with_ninv((double)c1, spid, c1d, c1q);
          double w[16];
          load(w, a, (size_t)soff);
          inv_col(w, a, spid, false);
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            double t1 = fred(fmul_mod(w[j], c1d, c1q, ms), msi, ms);
            t1 = t1 < 0.0 ? __dadd_rn(t1, ms) : t1;
            const double p2 = fmul_mod(t1, c2d, c2q, q);   // |p2| <= q
            x[j] = a == 0 ? p2 : __dadd_rn(x[j], p2);
          }
          if (a & 1) {
#pragma unroll
            for (int j = 0; j < 16; ++j) x[j] = fred(x[j], qi, q);
          }
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = fred(x[j], qi, q);
      }
    } else if constexpr (FUSE == 4) {
      // Conjugate-invariant ring: the sources hold the inverse transform before
      // its unfolding, b (coefficients modulo X^N - iota).  Every word is
      // unfolded with its mirror N - k, c_k = (b_k + iota b_{N-k}) / 2
      // (c_0 = b_0), converted, and folded for the target prime,
      // c'_k - iota' c'_{N-k}.  Mirrors sit in this block (see ci_col) and are
      // read through LDS.
      const int colv = ci_col(v);
      const int vm = (colv == 0 || colv == 128) ? v : (v < 8 ? v + 8 : v - 8);   // mirror's view
      auto mrow = [&](int a) { return colv == 0 ? (256 - a) & 255 : 255 - a; };  // mirror's row
      auto mirror = [&](double* val, double* mv) {      // mv[j] = value at the mirror of word j
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) sh[v * VS + pad(addr(0, j))] = val[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 16; ++j) mv[j] = sh[vm * VS + pad(mrow(addr(0, j)))];
      };
      const u64* ct = f.ci + 4 * (size_t)m.prime[blockIdx.y];
      const double it = (double)ct[0], itq = it / q;
      // source limb at offset soff, prime spid: c_k = (b_k + iota b_{N-k}) / 2 (c_0 = b_0),
      // exact residues in [0, m)
      auto unfold = [&](int soff, int spid, double* cc) {
        const double ms = (double)P[spid].q, msi = __longlong_as_double((long long)P[spid].pad[1]);
        const u64* cs = f.ci + 4 * (size_t)spid;
        const double is = (double)cs[0], isq = is / ms, h = (double)cs[2], hq = h / ms;
        double bm[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) cc[j] = u64_to_f(S[(size_t)soff * N + (size_t)addr(0, j) * astride]);
        mirror(cc, bm);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          if (colv == 0 && addr(0, j) == 0) continue;
          double r = fmul_mod(__dadd_rn(cc[j], fmul_mod(bm[j], is, isq, ms)), h, hq, ms);
          r = fred(r, msi, ms);
          cc[j] = r < 0.0 ? __dadd_rn(r, ms) : r;
        }
      };
      if (pro == 4) {
        // relinearisation and rescale in one (as in the standard ring, below)
        const ModDownTable& md = *f.md;
        const int li = f.last_pid, ti = m.prime[blockIdx.y];
        const double ql = (double)P[li].q, qli = __longlong_as_double((long long)P[li].pad[1]);
        const double pl = (double)md.pinv[li][0], plq = pl / ql, pt = (double)md.pinv[ti][0], ptq = pt / q;
        double cl[16], cc[16];
        for (int a = 0; a < md.K; ++a) {
          const int ppid = md.pprime[a];
          const double ms = (double)P[ppid].q, msi = __longlong_as_double((long long)P[ppid].pad[1]);
          const double c1d = (double)md.phatinv[a][0], c1q = c1d / ms;
          const double hl = (double)md.phat[a][li][0], hlq = hl / ql, ht = (double)md.phat[a][ti][0], htq = ht / q;
          unfold(f.s_off0 + a, ppid, cc);
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            double t1 = fred(fmul_mod(cc[j], c1d, c1q, ms), msi, ms);
            t1 = t1 < 0.0 ? __dadd_rn(t1, ms) : t1;
            const double pL = fmul_mod(t1, hl, hlq, ql), pT = fmul_mod(t1, ht, htq, q);
            cl[j] = a == 0 ? pL : __dadd_rn(cl[j], pL);
            x[j] = a == 0 ? pT : __dadd_rn(x[j], pT);
          }
          if (a & 1) {
#pragma unroll
            for (int j = 0; j < 16; ++j) {
              cl[j] = fred(cl[j], qli, ql);
              x[j] = fred(x[j], qi, q);
            }
          }
        }
        unfold(f.last_off, li, cc);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          double last = fmul_mod(__dsub_rn(cc[j], fred(cl[j], qli, ql)), pl, plq, ql);
          last = fred(last, qli, ql);
          last = last < 0.0 ? __dadd_rn(last, ql) : last;
          x[j] = __dadd_rn(fmul_mod(fred(x[j], qi, q), pt, ptq, q), fred(last, qi, q));
        }
      } else {
        for (int a = 0; a < ns; ++a) {
          int soff = 0, spid = f.src_pid;
          u64 c1 = 1, c2 = 1;
          if (pro != 3) src_info(a, soff, spid, c1, c2);
          const double ms = (double)P[spid].q, msi = __longlong_as_double((long long)P[spid].pad[1]);
          const double c1d = (double)c1, c1q = c1d / ms, c2d = (double)c2, c2q = c2d / q;
          double cc[16];
          unfold(soff, spid, cc);
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            double p2;
            if (pro == 3) {
              p2 = fred(cc[j], qi, q);
            } else {
              double t1 = fred(fmul_mod(cc[j], c1d, c1q, ms), msi, ms);
              t1 = t1 < 0.0 ? __dadd_rn(t1, ms) : t1;
              p2 = fmul_mod(t1, c2d, c2q, q);   // |p2| <= q
            }
            x[j] = a == 0 ? p2 : __dadd_rn(x[j], p2);
          }
          if (a & 1) {
#pragma unroll
            for (int j = 0; j < 16; ++j) x[j] = fred(x[j], qi, q);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) x[j] = fred(x[j], qi, q);
      double xm[16];
      mirror(x, xm);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const bool zero = colv == 0 && addr(0, j) == 0;
        if (!zero) x[j] = fred(__dsub_rn(x[j], fmul_mod(xm[j], it, itq, q)), qi, q);
      }
    } else if (pro == 3) {
#pragma unroll
      for (int j = 0; j < 16; ++j) x[j] = fred(u64_to_f(r0[j]), qi, q);
    } else if (pro == 4) {
      // relinearisation and rescale in one (see relin_rescale): the special
      // limbs of u and its last chain limb y = u + P d (coefficient domain)
      // give last = (y - conv_last(u_P)) P^-1 mod q_last (exact residue), and
      // the input word is conv_i(u_P) P^-1 + last mod q_i.
      const ModDownTable& md = *f.md;
      const int li = f.last_pid, ti = m.prime[blockIdx.y];
      const double ql = (double)P[li].q, qli = __longlong_as_double((long long)P[li].pad[1]);
      const double pl = (double)md.pinv[li][0], plq = pl / ql, pt = (double)md.pinv[ti][0], ptq = pt / q;
      double cl[16], ci[16];
      for (int a = 0; a < md.K; ++a) {
        const int ppid = md.pprime[a];
        const double ms = (double)P[ppid].q, msi = __longlong_as_double((long long)P[ppid].pad[1]);
        const double c1d = (double)md.phatinv[a][0], c1q = c1d / ms;
        const double hl = (double)md.phat[a][li][0], hlq = hl / ql, ht = (double)md.phat[a][ti][0], htq = ht / q;
        const u64* Sa = S + (size_t)(f.s_off0 + a) * N;
#pragma unroll
        for (int h = 0; h < 16; h += 8) {   // eight words in flight at a time
          u64 r[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) r[j] = a == 0 ? r0[h + j] : Sa[(size_t)addr(0, h + j) * astride];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            double t1 = fred(fmul_mod(u64_to_f(r[j]), c1d, c1q, ms), msi, ms);
            t1 = t1 < 0.0 ? __dadd_rn(t1, ms) : t1;
            const double pL = fmul_mod(t1, hl, hlq, ql), pT = fmul_mod(t1, ht, htq, q);   // each within q
            cl[h + j] = a == 0 ? pL : __dadd_rn(cl[h + j], pL);
            ci[h + j] = a == 0 ? pT : __dadd_rn(ci[h + j], pT);
          }
        }
        if (a & 1) {
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            cl[j] = fred(cl[j], qli, ql);
            ci[j] = fred(ci[j], qi, q);
          }
        }
      }
      const u64* Sl = S + (size_t)f.last_off * N;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double yl = u64_to_f(Sl[(size_t)addr(0, j) * astride]);
        double last = fmul_mod(__dsub_rn(yl, fred(cl[j], qli, ql)), pl, plq, ql);
        last = fred(last, qli, ql);
        last = last < 0.0 ? __dadd_rn(last, ql) : last;                 // exact residue mod q_last
        const double z = __dadd_rn(fmul_mod(fred(ci[j], qi, q), pt, ptq, q), fred(last, qi, q));
        x[j] = fred(z, qi, q);
      }
    } else {
      // source a's term of word j: [w (Q/q_a)^-1]_{q_a} (Q/q_a) mod q, |term| <= q
      auto term = [&](u64 w, double ms, double msi, double c1d, double c1q, double c2d, double c2q) {
        double t1 = fred(fmul_mod(u64_to_f(w), c1d, c1q, ms), msi, ms);
        t1 = t1 < 0.0 ? __dadd_rn(t1, ms) : t1;
        return fmul_mod(t1, c2d, c2q, q);
      };
      {   // the first source, requested before the twiddle staging (its words die here)
        int soff, spid;
        u64 c1, c2;
        src_info(0, soff, spid, c1, c2);
        const double ms = (double)P[spid].q, msi = __longlong_as_double((long long)P[spid].pad[1]);
        const double c1d = (double)c1, c2d = (double)c2;
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = term(r0[j], ms, msi, c1d, c1d / ms, c2d, c2d / q);
      }
      for (int a = 1; a < ns; ++a) {
        int soff, spid;
        u64 c1, c2;
        src_info(a, soff, spid, c1, c2);
        const double ms = (double)P[spid].q, msi = __longlong_as_double((long long)P[spid].pad[1]);
        const double c1d = (double)c1, c2d = (double)c2, c1q = c1d / ms, c2q = c2d / q;
        const u64* Sa = S + (size_t)soff * N;
#pragma unroll
        for (int h = 0; h < 16; h += 8) {   // eight words in flight at a time
          u64 r[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) r[j] = Sa[(size_t)addr(0, h + j) * astride];
#pragma unroll
          for (int j = 0; j < 8; ++j) x[h + j] = __dadd_rn(x[h + j], term(r[j], ms, msi, c1d, c1q, c2d, c2q));
        }
        if (a & 1) {
#pragma unroll
          for (int j = 0; j < 16; ++j) x[j] = fred(x[j], qi, q);
        }
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) x[j] = fred(x[j], qi, q);
    }
  } else if (DIRECT_IN) {
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = u64_to_f(raw[j]);
  } else {
    // coalesced load in the p = 0 order, transpose through LDS
    if (valid) {
#pragma unroll
      for (int j = 0; j < 16; ++j) sh[v * VS + pad(addr(0, j))] = u64_to_f(raw[j]);
    }
  }
  __syncthreads();                            // twiddles (and the transposed tile) ready
  if (!DIRECT_IN) {
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = sh[v * VS + pad(addr(P_FIRST, j))];
  }

  const double* tlv = tl + (KIND == NTT_ROW ? (v / vz) * 512 : 0);   // this view's row twiddles
  // twiddle of phase p, stage k of the phase, butterfly group hi, word j
  auto twid = [&](int p, int k, int hi, int j, double& w, double& wq) {
    if (LOGM == 8) {
      const int slot = p == 0 ? (1 << k) + (j >> (4 - k)) : (1 << (4 + k)) + ((j >> (4 - k)) << 4) + hi;
      w = tlv[slot];
      wq = tlv[256 + slot];
    } else {
      const int kk = (1 << (4 * p + k)) + (hi << k) + (j >> (4 - k));
      w = W[kk];
      wq = WQ[kk];
    }
  };

#pragma unroll
  for (int ph = 0; ph < PH; ++ph) {
    const int p = INV ? PH - 1 - ph : ph;
    const int hi = u >> (LOGM - 4 * p - 4);
    if (ph > 0) {
#pragma unroll
      for (int j = 0; j < 16; ++j) x[j] = sh[v * VS + pad(addr(p, j))];
    }
    auto tw_p = [&](int k, int j, double& w, double& wq) { twid(p, k, hi, j, w, wq); };
    if (!INV)
      fpm::ct_phase16(x, ph > 0, qi, q, tw_p);
    else
      fpm::gs_phase16(x, ph > 0, qi, q, tw_p);
    if (ph + 1 < PH) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 16; ++j) sh[v * VS + pad(addr(p, j))] = x[j];
      __syncthreads();
    }
  }

  // ---- exact residues in [0, q) (times N^-1 at the end of an inverse transform) and store
  if (last) {
    const double ni = (double)pr.ninv, niq = __longlong_as_double((long long)pr.pad[2]);
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = fmul_mod(x[j], ni, niq, q);
  }
  u64 y[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    double r = fred(x[j], qi, q);
    r = r < 0.0 ? __dadd_rn(r, q) : r;
    y[j] = FUSE == 3 ? (u64)__double_as_longlong(r) : f_to_u64(r);
  }
  if (DIRECT_OUT) {
    if (valid) {
#pragma unroll
      for (int j = 0; j < 16; ++j) dst[(size_t)addr(P_LAST, j) * astride] = y[j];
    }
  } else {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) sh_raw[v * VS + pad(addr(P_LAST, j))] = y[j];
    __syncthreads();
    if (valid) {
      if constexpr (FUSE == 2) {
        // out = (minuend - x) w (+ addend), all words exact residues
        const double wd = (double)f.wtab[2 * blockIdx.y], wq = wd / q;
        if (epi == 2) {
          // out = (minuend wm + addend - x) w
          const double wm = (double)f.wmtab[2 * blockIdx.y], wmq = wm / q;
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const int a = addr(0, j);
            double r = fmul_mod(u64_to_f(mr[j]), wm, wmq, q);                            // |r| <= q
            if (Ad) r = __dadd_rn(r, u64_to_f(ar[j]));
            r = fred(__dsub_rn(r, u64_to_f(sh_raw[v * VS + pad(a)])), qi, q);
            r = fred(fmul_mod(r, wd, wq, q), qi, q);
            r = r < 0.0 ? __dadd_rn(r, q) : r;
            Oe[a] = f_to_u64(r);
          }
        } else {
#pragma unroll
          for (int j = 0; j < 16; ++j) {
            const int a = addr(0, j);
            const double d = __dsub_rn(u64_to_f(mr[j]), u64_to_f(sh_raw[v * VS + pad(a)]));   // |d| < q
            double r = fmul_mod(d, wd, wq, q);                                                 // |r| <= q
            if (Ad) r = __dadd_rn(r, u64_to_f(ar[j]));
            r = fred(r, qi, q);
            r = r < 0.0 ? __dadd_rn(r, q) : r;
            Oe[a] = f_to_u64(r);
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int a = addr(0, j);
          dst[a] = sh_raw[v * VS + pad(a)];
        }
      }
    }
  }
}

// ---------------------------------------------------------------- elementwise

#define EW_PROLOGUE                                               \
  const int slot = blockIdx.y;                                    \
  const size_t loff = (size_t)m.off[slot] * N;                    \
  const PrimeC& pr = P[m.prime[slot]];                            \
  const u64 q = pr.q;                                             \
  (void)q;                                                        \
  const size_t bz = blockIdx.z;

#define EW_LOOP for (int i = blockIdx.x * TPB + threadIdx.x; i < N; i += gridDim.x * TPB)

__global__ void k_add(const u64* a, size_t sa, const u64* b, size_t sb, u64* o, size_t so,
                      LimbMap m, const PrimeC* P, int N) {
  EW_PROLOGUE
  const u64* A = a + bz * sa + loff;
  const u64* B = b + bz * sb + loff;
  u64* O = o + bz * so + loff;
  EW_LOOP O[i] = add_mod(A[i], B[i], q);
}

__global__ void k_sub(const u64* a, size_t sa, const u64* b, size_t sb, u64* o, size_t so,
                      LimbMap m, const PrimeC* P, int N) {
  EW_PROLOGUE
  const u64* A = a + bz * sa + loff;
  const u64* B = b + bz * sb + loff;
  u64* O = o + bz * so + loff;
  EW_LOOP O[i] = sub_mod(A[i], B[i], q);
}

__global__ void k_mul(const u64* a, size_t sa, const u64* b, size_t sb, u64* o, size_t so,
                      LimbMap m, const PrimeC* P, int N) {
  EW_PROLOGUE
  const u64* A = a + bz * sa + loff;
  const u64* B = b + bz * sb + loff;
  u64* O = o + bz * so + loff;
  EW_LOOP O[i] = mul_mod(A[i], B[i], pr);
}

// out[z][comp][l] = ct[z][comp][l] * pt[z][l] over the chain limbs l < limbs,
// both components in one launch (blockIdx.y = comp * limbs + l)
__global__ void k_mul_ct_pt(const u64* ct, size_t sct, size_t ccs, const u64* pt, size_t spt, u64* out,
                            size_t so, size_t ocs, int limbs, const PrimeC* P, int N, int ct_div, int pt_mod) {
  const int l = blockIdx.y % limbs, comp = blockIdx.y / limbs;
  const PrimeC& pr = P[l];
  const size_t bz = blockIdx.z;
  const u64* A = ct + (bz / ct_div) * sct + comp * ccs + (size_t)l * N;
  const u64* Bp = pt + (bz % pt_mod) * spt + (size_t)l * N;
  u64* O = out + bz * so + comp * ocs + (size_t)l * N;
  EW_LOOP O[i] = mul_mod(A[i], Bp[i], pr);
}

// o += s * scal[slot] (scal holds a Shoup pair per limb slot)
__global__ void k_axpy_scalar(const u64* s, size_t ss, const u64* scal, u64* o, size_t so,
                              LimbMap m, const PrimeC* P, int N) {
  EW_PROLOGUE
  const u64* S = s + bz * ss + loff;
  u64* O = o + bz * so + loff;
  const u64 w = scal[2 * slot], ws = scal[2 * slot + 1];
  EW_LOOP O[i] = add_mod(O[i], mul_shoup(S[i], w, ws, q), q);
}

__global__ void k_reduce_int(const int64_t* src, size_t ss, u64* o, size_t so, LimbMap m,
                             const PrimeC* P, int N) {
  EW_PROLOGUE
  const int64_t* S = src + bz * ss;
  u64* O = o + bz * so + loff;
  EW_LOOP {
    const int64_t x = S[i];
    if (x >= 0) {
      O[i] = reduce64((u64)x, pr);
    } else {
      const u64 r = reduce64((u64)(-x), pr);
      O[i] = r ? q - r : 0;
    }
  }
}

// (a0, a1) x (b0, b1) -> (a0 b0, a0 b1 + a1 b0, a1 b1); limb slot = chain limb.
// Batch element z multiplies the operands at A.p[z] and Bt.p[z], so one launch
// can cross any queries with any gallery groups.  a_cs and b_cs are the
// component strides of the operands (they may hold more limbs than the product
// uses: an exact level drop on the fly); with parts > 1 the tensors of the
// part pairs (a + p a_ps, b + p b_ps) are summed.
__global__ void k_tensor(PtrTab A, size_t a_cs, size_t a_ps, PtrTab Bt, size_t b_cs, size_t b_ps, int parts, u64* o,
                         size_t so, int limbs, const PrimeC* P, int N, int accumulate) {
  const int l = blockIdx.y;
  const PrimeC& pr = P[l];
  const u64 q = pr.q;
  const size_t bz = blockIdx.z;
  const size_t ln = (size_t)limbs * N;
  const u64* A0 = A.p[bz] + (size_t)l * N;
  const u64* A1 = A0 + a_cs;
  const u64* B0 = Bt.p[bz] + (size_t)l * N;
  const u64* B1 = B0 + b_cs;
  u64* O0 = o + bz * so + (size_t)l * N;
  u64* O1 = O0 + ln;
  u64* O2 = O1 + ln;
  const double qd = (double)q, qi = __longlong_as_double((long long)pr.pad[1]);
  EW_LOOP {
    FAcc f0, f1, f2;                      // exact FP64 sums of the products (see FAcc)
    // sum of the tensors of `parts` pairs of parts, four parts' words
    // requested before the first product
    constexpr int PC = 4;
    for (int p0 = 0; p0 < parts; p0 += PC) {
      u64 w[PC][4];
#pragma unroll
      for (int c = 0; c < PC; ++c) {
        const int p = p0 + c < parts ? p0 + c : parts - 1;   // a ragged chunk repeats the last part, unused
        const size_t ao = (size_t)p * a_ps + i, bo = (size_t)p * b_ps + i;
        w[c][0] = A0[ao];
        w[c][1] = A1[ao];
        w[c][2] = B0[bo];
        w[c][3] = B1[bo];
      }
      __builtin_amdgcn_sched_barrier(0);   // (the scheduler would sink each part's loads to its products)
#pragma unroll
      for (int c = 0; c < PC; ++c) {
        if (p0 + c >= parts) break;
        const double x0 = u64_to_f(w[c][0]), x1 = u64_to_f(w[c][1]);
        const double y0 = u64_to_f(w[c][2]), y1 = u64_to_f(w[c][3]);
        const double y0q = __dmul_rn(y0, qi), y1q = __dmul_rn(y1, qi);
        f0.add_f(fmul_mod(x0, y0, y0q, qd), qi, qd);
        f1.add_f(fmul_mod(x0, y1, y1q, qd), qi, qd);
        f1.add_f(fmul_mod(x1, y0, y0q, qd), qi, qd);
        f2.add_f(fmul_mod(x1, y1, y1q, qd), qi, qd);
      }
    }
    u64 d0 = f0.residue(qi, qd), d1 = f1.residue(qi, qd), d2 = f2.residue(qi, qd);
    if (accumulate) {
      d0 = add_mod(d0, O0[i], q);
      d1 = add_mod(d1, O1[i], q);
      d2 = add_mod(d2, O2[i], q);
    }
    O0[i] = d0;
    O1[i] = d1;
    O2[i] = d2;
  }
}

// Position of the source word of an automorphism X -> X^g in the bit-reversed
// evaluation domain: out[i] = in[src].  Word i holds the value at w^(1 + M/N
// brv(i)) for w a primitive M-th root of unity, M = N << ms (ms = 1: the roots
// of X^N + 1; ms = 2: the conjugate-invariant ring's evaluation points, the
// roots of X^N - w^N), and X -> X^g maps that point onto the one of
// exponent g (1 + (M/N) brv(i)) mod M, again 1 mod M/N as g is.
__device__ __forceinline__ u32 autom_src(u32 i, u32 g, int log_n, int ms) {
  const u32 rj = __brev(i) >> (32 - log_n);
  const u32 e = (u32)(((u64)((rj << ms) + 1) * g) & ((1u << (log_n + ms)) - 1));
  return __brev((e - 1) >> ms) >> (32 - log_n);
}

// evaluation-domain automorphism: out[j] = in[autom_src(j)].  blockIdx.y = row
// (comp*limbs + limb).  Batch element z uses g1 when bit `sel` of z is set,
// g0 otherwise.
__global__ void k_automorphism(const u64* in, size_t si, u64* out, size_t so, u64 g0, u64 g1, int sel,
                               int log_n, int ms) {
  const int N = 1 << log_n;
  const size_t row = (size_t)blockIdx.y * N;
  const u64* I = in + (size_t)blockIdx.z * si + row;
  u64* O = out + (size_t)blockIdx.z * so + row;
  const u64 g = ((blockIdx.z >> sel) & 1) ? g1 : g0;
  EW_LOOP O[i] = I[autom_src((u32)i, (u32)g, log_n, ms)];
}

// Conjugate-invariant ring: an element c (coefficients 0..N-1 of a polynomial
// of Z_q[X]/(X^2N+1) with c_N = 0 and c_{2N-k} = -c_k) is reduced modulo
// X^N - iota, iota = w^N for w a primitive 4N-th root, whose N roots are the
// evaluation points: b_k = c_k - iota c_{N-k} (b_0 = c_0).  The reduction is
// a ring homomorphism, invertible on such elements:
// c_k = (b_k + iota b_{N-k}) / 2 (c_0 = b_0).  One thread handles the pair
// (k, N-k), so in == out is allowed.  ci[prime] = {iota, its Shoup
// companion, 1/2, its companion}.
__global__ void k_ci_fold(const u64* in, size_t si, u64* out, size_t so, LimbMap m, const PrimeC* P,
                          const u64* ci, int N, int inverse) {
  const int slot = blockIdx.y;
  const int pid = m.prime[slot];
  const u64 q = P[pid].q;
  const u64 io = ci[4 * pid], ios = ci[4 * pid + 1], h = ci[4 * pid + 2], hs = ci[4 * pid + 3];
  const u64* I = in + (size_t)blockIdx.z * si + (size_t)m.off[slot] * N;
  u64* O = out + (size_t)blockIdx.z * so + (size_t)m.ooff[slot] * N;
  for (int k = blockIdx.x * TPB + threadIdx.x; k <= N / 2; k += gridDim.x * TPB) {
    if (k == 0) {
      O[0] = I[0];
      continue;
    }
    const u64 a = I[k], b = I[N - k];
    const u64 ib = mul_shoup(b, io, ios, q), ia = mul_shoup(a, io, ios, q);
    if (inverse) {
      O[k] = mul_shoup(add_mod(a, ib, q), h, hs, q);
      O[N - k] = mul_shoup(add_mod(b, ia, q), h, hs, q);
    } else {
      O[k] = sub_mod(a, ib, q);
      O[N - k] = sub_mod(b, ia, q);
    }
  }
}

// ModUp of every digit at `limbs` chain limbs.  blockIdx.y enumerates the
// (digit j, target slot t outside j) pairs; output y[j][t] (coefficient domain).
__global__ void k_modup(const u64* xc, size_t sx, u64* y, size_t sy, const ModUpTable* T,
                        const PrimeC* P, int N) {
  const ModUpTable& tb = *T;
  const int j = tb.pair_j[blockIdx.y], t = tb.pair_t[blockIdx.y];
  const ModUpDigit& dg = tb.d[j];
  const PrimeC& pt = P[tb.ext_prime[t]];
  const u64 qt = pt.q;
  const size_t bz = blockIdx.z;
  const u64* X = xc + bz * sx;
  u64* Y = y + bz * sy + ((size_t)j * tb.ext + t) * N;
  EW_LOOP {
    u64 acc = 0;
    for (int a = 0; a < dg.nsrc; ++a) {
      const int src = dg.src[a];
      const u64 qi = P[src].q;
      const u64 v = mul_shoup(X[(size_t)src * N + i], dg.qhatinv[a][0], dg.qhatinv[a][1], qi);
      acc = add_mod(acc, mul_shoup(v, dg.qhat[a][t][0], dg.qhat[a][t][1], qt), qt);
    }
    Y[i] = acc;
  }
}

// key inner product over every extended slot t of the level:
// u[t] = sum_j y_j[t] * b_j[key limb of t], w[t] likewise with a_j.  For the
// digit's own slots y_j[t] is the input limb itself (evaluation domain).
// With dadd, the last chain limb of each output gets P d added (P = the
// special modulus, d the component's addend: dadd + z sd + comp dcs), the
// form in which a relinearisation hands its last limb to the rescale.
__global__ void k_kip(const u64* y, size_t sy, const u64* x, size_t sx, const u64* key0,
                      const u64* key1, int sel, u64* uw, size_t suw, const ModUpTable* T,
                      int key_limbs, int L1, const PrimeC* P, int N, const u64* dadd, size_t sd, size_t dcs,
                      u64 pm, u64 pms) {
  const ModUpTable& tb = *T;
  const int t = blockIdx.y;
  const int ext = tb.ext;
  const int pid = tb.ext_prime[t];
  const PrimeC& pr = P[pid];
  const u64 q = pr.q;
  const int kl = t < tb.limbs ? t : L1 + (t - tb.limbs);
  const size_t bz = blockIdx.z;
  // per-element key choice; key words are FP64 values
  const double* key = (const double*)(((blockIdx.z >> sel) & 1) ? key1 : key0);
  u64* U = uw + bz * suw + (size_t)t * N;
  u64* Wp = U + (size_t)ext * N;
  const double qd = (double)q, qi = __longlong_as_double((long long)pr.pad[1]);
  EW_LOOP {
    FAcc su, sw;
    for (int j = 0; j < tb.beta; ++j) {
      const ModUpDigit& dg = tb.d[j];
      const bool own = t >= dg.src[0] && t < dg.src[0] + dg.nsrc;
      // ModUp digits are FP64 values, the input limbs residue words
      const double v = own ? u64_to_f(x[bz * sx + (size_t)t * N + i])
                           : __longlong_as_double((long long)y[bz * sy + ((size_t)j * ext + t) * N + i]);
      su.add(v, key[((size_t)(2 * j) * key_limbs + kl) * N + i], qi, qd);
      sw.add(v, key[((size_t)(2 * j + 1) * key_limbs + kl) * N + i], qi, qd);
    }
    u64 ru = su.residue(qi, qd), rw = sw.residue(qi, qd);
    if (dadd && t == tb.limbs - 1) {
      const u64* D = dadd + bz * sd + (size_t)t * N;
      ru = add_mod(ru, mul_shoup(D[i], pm, pms, q), q);
      rw = add_mod(rw, mul_shoup(D[dcs + i], pm, pms, q), q);
    }
    U[i] = ru;
    Wp[i] = rw;
  }
}

// The key inner product of a plain key switch at N = 2^16 on whole rows:
// block (row block, slot t, element block) takes R consecutive rows of vz
// elements (16 lanes a row, 16 words a lane) and, for every digit, either
// reads the input limb (the digit's own slots, evaluation domain) or finishes
// the digit's forward transform here: the row pass over the column-pass words
// the fused ModUp column pass left in y (u64, slot j ext + t).  Then
//   u[t] = sum_j y_j[t] b_j,  w[t] = sum_j y_j[t] a_j   (+ P d at the last chain
//   limb with dadd, as k_kip),
// and the slots from inv_from on (those the ModDown, or ModDown and rescale,
// transform back) get the row pass of their inverse transform before they are
// stored; the others are stored in the evaluation domain.  Same operations
// as the row pass, k_kip and the inverse row pass one after the other, so the
// same words.
__global__ void __launch_bounds__(256) k_kip_rows(const u64* y, size_t sy, const u64* x, size_t sx,
                                                  const u64* key0, const u64* key1, int sel, u64* uw, size_t suw,
                                                  const ModUpTable* T, int key_limbs, int L1, const PrimeC* P,
                                                  const double* twf, const double* twq, const double* itwf,
                                                  const double* itwq, int B, int vz, const u64* dadd, size_t sd,
                                                  size_t dcs, double pmd, int inv_from) {
  constexpr int LOGN = 16, M = 256, VS = M + M / 16;
  constexpr int N = 1 << LOGN;
  extern __shared__ u64 sh_raw[];
  double* sh = reinterpret_cast<double*>(sh_raw);
  const ModUpTable& tb = *T;
  const int ext = tb.ext, limbs = tb.limbs;
  const int th = threadIdx.x;
  const int V = (int)blockDim.x / 16;
  const int R = V / vz;
  const int v = th / 16, u = th % 16;
  const int ts = blockIdx.y;                                  // slot
  const int z = blockIdx.z * vz + v % vz;
  const int row = blockIdx.x * R + v / vz;
  const bool valid = z < B;
  const size_t zz = valid ? (size_t)z : 0;
  const int pid = tb.ext_prime[ts];
  const PrimeC& pr = P[pid];
  const double q = (double)pr.q, qi = __longlong_as_double((long long)pr.pad[1]);
  const int kl = ts < limbs ? ts : L1 + (ts - limbs);
  const bool inv = ts >= inv_from;
  auto pad = [](int a) { return a + (a >> 4); };
  // phase p holds word addr(p, j): p = 0, words j 16 + u; p = 1, words 16 u + j
  auto addr = [&](int p, int j) { return p == 0 ? (j << 4) + u : (u << 4) + j; };
  double* tl = sh + V * VS;                                   // [R][2][256] forward, then [R][2][256] inverse
  // four slots a thread at a time, every word requested before the first store
  const int nst = 256 * R * (inv ? 2 : 1);
  for (int k0 = th; k0 < nst; k0 += 4 * (int)blockDim.x) {
    double sw_w[4], sw_q[4];   // staged words (names apart from the kernel's twf / twq)
    int at[4];
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
      const int k = k0 + c4 * (int)blockDim.x;
      const int slot = k & 255, rr = (k >> 8) % R, iv = (k >> 8) / R;
      at[c4] = k < nst && slot != 0 ? (iv * R + rr) * 512 + slot : -1;
      const int vb = blockIdx.x * R + rr;
      const int st = 31 - __clz(slot | 1);
      const int o = slot - (1 << st);
      const int b = st < 4 ? o : ((o & 15) << (st - 4)) + (o >> 4);
      const size_t g = (size_t)pid * N + (1 << (8 + st)) + (vb << st) + b;
      sw_w[c4] = at[c4] >= 0 ? (iv ? itwf[g] : twf[g]) : 0.0;
      sw_q[c4] = at[c4] >= 0 ? (iv ? itwq[g] : twq[g]) : 0.0;
    }
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
      if (at[c4] >= 0) {
        tl[at[c4]] = sw_w[c4];
        tl[at[c4] + 256] = sw_q[c4];
      }
    }
  }
  __syncthreads();
  const double* tlf = tl + (size_t)(v / vz) * 512;
  const double* tli = tl + (size_t)(R + v / vz) * 512;
  auto twid = [&](const double* tv, int p, int k, int j, double& w, double& wq) {
    const int slot = p == 0 ? (1 << k) + (j >> (4 - k)) : (1 << (4 + k)) + ((j >> (4 - k)) << 4) + u;
    w = tv[slot];
    wq = tv[256 + slot];
  };
  // 16 words of this lane through LDS: written at phase-pf positions, read at pt
  auto exchange = [&](double (&a)[16], int pf, int pt) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) sh[v * VS + pad(addr(pf, j))] = a[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) a[j] = sh[v * VS + pad(addr(pt, j))];
  };
  const size_t rbase = (size_t)row * M;
  const double* key = (const double*)(((zz >> sel) & 1) ? key1 : key0);
  double su[16], sw[16];
  for (int d = 0; d < tb.beta; ++d) {
    const ModUpDigit& dg = tb.d[d];
    const bool own = ts >= dg.src[0] && ts < dg.src[0] + dg.nsrc;
    double val[16];
    if (own) {
      const u64* X = x + zz * sx + (size_t)ts * N + rbase;
#pragma unroll
      for (int j = 0; j < 16; ++j) val[j] = u64_to_f(X[addr(1, j)]);
    } else {
      const u64* Y = y + zz * sy + ((size_t)d * ext + ts) * N + rbase;
#pragma unroll
      for (int j = 0; j < 16; ++j) val[j] = u64_to_f(Y[addr(0, j)]);
      auto t0 = [&](int k, int j, double& w, double& wq) { twid(tlf, 0, k, j, w, wq); };
      fpm::ct_phase16(val, false, qi, q, t0);
      exchange(val, 0, 1);
      auto t1 = [&](int k, int j, double& w, double& wq) { twid(tlf, 1, k, j, w, wq); };
      fpm::ct_phase16(val, true, qi, q, t1);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double r = fred(val[j], qi, q);
        val[j] = r < 0.0 ? __dadd_rn(r, q) : r;
      }
    }
    const double* KB = key + ((size_t)(2 * d) * key_limbs + kl) * N + rbase + (size_t)u * 16;
    const double* KA = key + ((size_t)(2 * d + 1) * key_limbs + kl) * N + rbase + (size_t)u * 16;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double pu = fmul_mod_q(val[j], KB[j], qi, q), pw = fmul_mod_q(val[j], KA[j], qi, q);
      su[j] = d == 0 ? pu : __dadd_rn(su[j], pu);
      sw[j] = d == 0 ? pw : __dadd_rn(sw[j], pw);
    }
    if (d & 1) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        su[j] = fred(su[j], qi, q);
        sw[j] = fred(sw[j], qi, q);
      }
    }
  }
  if (dadd && ts == limbs - 1) {
    const u64* D = dadd + zz * sd + (size_t)ts * N + rbase;
    const double pmq = pmd / q;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      su[j] = __dadd_rn(fred(su[j], qi, q), fmul_mod(u64_to_f(D[addr(1, j)]), pmd, pmq, q));
      sw[j] = __dadd_rn(fred(sw[j], qi, q), fmul_mod(u64_to_f(D[dcs + addr(1, j)]), pmd, pmq, q));
    }
  }
  // exact residues, then (slots from inv_from on) the inverse row pass, and
  // the store of each component in the p = 0 order (coalesced)
  auto finish = [&](double (&a)[16], u64* O) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double r = fred(a[j], qi, q);
      a[j] = r < 0.0 ? __dadd_rn(r, q) : r;
    }
    if (inv) {
      auto t1 = [&](int k, int j, double& w, double& wq) { twid(tli, 1, k, j, w, wq); };
      fpm::gs_phase16(a, false, qi, q, t1);
      exchange(a, 1, 0);
      auto t0 = [&](int k, int j, double& w, double& wq) { twid(tli, 0, k, j, w, wq); };
      fpm::gs_phase16(a, true, qi, q, t0);
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double r = fred(a[j], qi, q);
        a[j] = r < 0.0 ? __dadd_rn(r, q) : r;
      }
    } else {
      exchange(a, 1, 0);
    }
    if (valid) {
#pragma unroll
      for (int j = 0; j < 16; ++j) O[addr(0, j)] = f_to_u64(a[j]);
    }
  };
  u64* U = uw + zz * suw + (size_t)ts * N + rbase;
  finish(su, U);
  finish(sw, U + (size_t)ext * N);
}

// Hoisted key inner products: for element z,
//   (u, w)[z] = sum_a sum_j phi_{g(z,a)}(y_j[z]) * key_{g(z,a), j}     over Q_l u P,
// the automorphism read as a gather (an aligned block of consecutive words
// maps onto an aligned block).  Keys come from the key table (indexed by
// g / 2).  One thread per (element, limb, position); the elements of one
// (limb, position block) are consecutive blocks, so that on one XCD they
// share the key words through L2.
constexpr int HOIST_BETA = 4;   // digits a thread handles (dnum <= 4 at every level)

// The key pointers of the hoisted kernels come from a table staged in LDS;
// read through these global-space types, their words are loaded with global
// (not flat) loads, which do not hold up the LDS and scalar-memory waits of
// the next amounts.
typedef const __attribute__((address_space(1))) double* gdp;
typedef double dv2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) dv2* gd2p;

// XCD-aware block order: the hardware deals workgroups to the 8 XCDs in
// turn, so workgroup w runs on XCD w mod 8.  Logical block
// (w mod 8) * (W / 8) + w / 8 gives every XCD one contiguous range of logical
// blocks (W a multiple of 8), whose gathered words and shared key words then
// stay in that XCD's L2.
__device__ __forceinline__ int xcd_block(int w, int W) { return (w & 7) * (W >> 3) + (w >> 3); }

// out[z] = in[z] + sum_a phi_{g(z,a)}(in[z]) on `limbs` limbs of one component
// (accumulate: out[z] += sum_a phi_{g(z,a)}(in[z]); out must not alias in).
// Runs as the first am.W blocks of a per-element hoisted key inner product
// launch (the c0 half of the hoisted rotation sum), over a 1-D XCD-aware grid
// of (element, limb, position block), position block fastest.  The grouped
// kernel (am.W = 0) forms it in its chain slots' blocks instead, where its
// gathers overlap the key sums of the other slots' blocks (79.6 against
// 81.9 us at the face configuration; the c0 sums themselves take about 15 us
// of the launch either way).
struct AutomArgs {
  const u64* in;
  size_t si;
  u64* out;
  size_t so;
  int limbs;
  int W;   // blocks of the launch that do this part
};

__device__ __forceinline__ void autom_sum_part(const AutomArgs& am, const HoistArgs& h, const PrimeC* P,
                                               int log_n, int ms, int accumulate, int w) {
  const int N = 1 << log_n;
  const int gx = (N + TPB - 1) / TPB;
  const int lb = xcd_block(w, am.W);
  const int l = (lb / gx) % am.limbs;
  const int z = lb / (gx * am.limbs);
  const int i = (lb % gx) * TPB + threadIdx.x;
  if (i >= N) return;
  const u64 q = P[l].q;
  const u64* I = am.in + (size_t)z * am.si + (size_t)l * N;
  u64* O = am.out + (size_t)z * am.so + (size_t)l * N;
  u64 acc = accumulate ? O[i] : I[i];
#pragma unroll 4
  for (int a = 0; a < h.A; ++a) {
    const u32 g = h.g[h.per_elem ? (z % h.mod) * h.A + a : a];
    acc = add_mod(acc, I[autom_src((u32)i, g, log_n, ms)], q);
  }
  O[i] = acc;
}

template <int BETA>
__global__ void k_kip_hoist(const u64* y, size_t sy, const u64* x, size_t sx, const u64* const* gtab,
                            HoistArgs h, u64* uw, size_t suw, const ModUpTable* T, int key_limbs, int L1,
                            const PrimeC* P, int log_n, int ms, int B, int accumulate, AutomArgs am) {
  if ((int)blockIdx.x < am.W) {
    autom_sum_part(am, h, P, log_n, ms, accumulate, (int)blockIdx.x);
    return;
  }
  const ModUpTable& tb = *T;
  const int N = 1 << log_n;
  const int ext = tb.ext;
  // 1-D grid of (limb, position block, element), element fastest
  const int gx = (N + TPB - 1) / TPB;
  const int lb = xcd_block((int)blockIdx.x - am.W, (int)gridDim.x - am.W);
  const int z = lb % B;
  const int pb = (lb / B) % gx;
  const int t = lb / (B * gx);
  const int i = pb * TPB + threadIdx.x;
  // key addresses of this block's amounts, staged once in LDS (they are
  // uniform across the block), so that no global load sits in front of the
  // key words inside the loop
  __shared__ const u64* kp[HOIST_MAX];
  for (int a = threadIdx.x; a < h.A; a += TPB) kp[a] = gtab[h.g[h.per_elem ? (z % h.mod) * h.A + a : a] >> 1];
  __syncthreads();
  if (i >= N || t >= ext) return;
  const PrimeC& pr = P[tb.ext_prime[t]];
  const u64 q = pr.q;
  const int kl = t < tb.limbs ? t : L1 + (t - tb.limbs);
  const double qd = (double)q, qi = __longlong_as_double((long long)pr.pad[1]);
  // row of digit j at slot t: the input limb itself for the digit's own slots
  // (ModUp digits are FP64 values, the input limbs residue words)
  const u64* src[BETA];
  bool own[BETA];
#pragma unroll
  for (int j = 0; j < BETA; ++j) {
    const ModUpDigit& dg = tb.d[j];
    own[j] = t >= dg.src[0] && t < dg.src[0] + dg.nsrc;
    src[j] = own[j] ? x + (size_t)z * sx + (size_t)t * N : y + (size_t)z * sy + ((size_t)j * ext + t) * N;
  }
  const size_t ko = (size_t)kl * N + i, kst = (size_t)key_limbs * N;
  // words of one amount: digits (gathered), key b and key a words of every digit
  struct Words {
    u64 v[BETA];
    double kb[BETA], ka[BETA];
  };
  auto load = [&](int a, Words& w) {
    const u32 g = h.g[h.per_elem ? (z % h.mod) * h.A + a : a];
    const u32 s = autom_src((u32)i, g, log_n, ms);
    const gdp key = (gdp)kp[a];
#pragma unroll
    for (int j = 0; j < BETA; ++j) {
      w.v[j] = src[j][s];
      w.kb[j] = key[ko + (size_t)(2 * j) * kst];
      w.ka[j] = key[ko + (size_t)(2 * j + 1) * kst];
    }
  };
  // exact sums in FP64: every product lies within 1.25 q of 0 (fmul_mod_q), and
  // the sums are folded back to |s| <= q/2 + 1 after every second product of
  // the two-amount window (so |s| < 3q + 1)
  double su = 0.0, sw = 0.0;
  auto mac = [&](const Words& w, int d) {
#pragma unroll
    for (int j = 0; j < BETA; ++j) {
      const double v = own[j] ? u64_to_f(w.v[j]) : __longlong_as_double((long long)w.v[j]);
      su = __dadd_rn(su, fmul_mod_q(v, w.kb[j], qi, qd));
      sw = __dadd_rn(sw, fmul_mod_q(v, w.ka[j], qi, qd));
      if ((d * BETA + j) & 1) {
        su = fred(su, qi, qd);
        sw = fred(sw, qi, qd);
      }
    }
  };
  // D buffers: the words of the next D - 1 amounts are in flight while one is
  // multiplied
  constexpr int D = 2;
  Words w[D];
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (d < h.A) load(d, w[d]);
  for (int a = 0; a < h.A; a += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (a + d < h.A) {
        mac(w[d], d);
        if (a + d + D < h.A) load(a + d + D, w[d]);
      }
    }
  }
  u64* U = uw + (size_t)z * suw + (size_t)t * N;
  auto res = [&](double s_) {
    double r = fred(s_, qi, qd);
    r = r < 0.0 ? __dadd_rn(r, qd) : r;
    return f_to_u64(r);
  };
  const u64 ru = res(su), rw = res(sw);
  U[i] = accumulate ? add_mod(U[i], ru, q) : ru;
  U[(size_t)ext * N + i] = accumulate ? add_mod(U[(size_t)ext * N + i], rw, q) : rw;
}

// Masked hoisted rotation sums (Alg. 1 with its rotations hoisted and the
// masks applied after the key inner products).  Element e = j k + i is part i
// of query j (x at x + j sx: c0, then c1 at + xcs, `limbs` limbs, evaluation
// domain); mask i is at masks + i ml N over every prime (ml limbs: the chain,
// then the specials).  h.g lists the distinct amounts of all parts, mu.parts[a]
// the parts that use amount a (bit i).
//   key sums (every slot t of Q_l u P):
//     uw[e][c] = sum over a in amounts(i) of phi_a(mask_i) * sum_d phi_a(y_d[j]) key_{a,d,c}
//   and, with dadd, P ad[e][c] added at the last chain slot (the form the
//   fused ModDown and rescale take);
//   addends (the chain slots t < `limbs`):
//     ad[e][0] = sum over r in {0} u amounts(i) of phi_r(mask_i x_0),  ad[e][1] = mask_i x_1.
// A thread serves one word of one slot for PG parts of one query: the inner
// sum of each amount is formed once and multiplied into every part of the
// group that uses it, and at a chain slot the same mask words times the
// gathered x_0 word go to the addends.  The gathers read
// phi_a(v)[pos] = v[autom_src(pos)].  (The addends once had blocks of their
// own, ahead of the key sums: they cost the launch 13 of its 51 us at the
// face configuration.)
struct MaskUse {
  uint16_t parts[HOIST_MAX];
};

template <int BETA, int PG>
__global__ void k_kip_hoist_mask(const u64* y, size_t sy, const u64* x, size_t sx, size_t xcs,
                                 const u64* const* gtab, HoistArgs h, MaskUse mu, const u64* masks, int ml,
                                 u64* uw, size_t suw, u64* ad, size_t sad, const ModUpTable* T, int key_limbs,
                                 int L1, const PrimeC* P, int log_n, int ms, int nq, int k, int dadd,
                                 double pmd, const double* itwf, const double* itwq, int inv_from) {
  const int N = 1 << log_n;
  const ModUpTable& tb = *T;
  const int limbs = tb.limbs;
  // The blocks take (position block, slot, query, part group) with the
  // position block slowest and the logical blocks dealt to the 8 XCDs in
  // contiguous ranges (xcd_block, when the block count is a multiple of 8):
  // each XCD takes an aligned eighth of the positions of every slot.  For one
  // automorphism an aligned eighth gathers from one aligned eighth of every
  // limb (the automorphisms permute the eighths; rotations keep the two
  // halves), so each amount's gathers of an XCD stay within one eighth of
  // the digits, masks and query limbs.
  const int ext = tb.ext;
  const int ngr = (k + PG - 1) / PG;                          // part groups of a query
  // (position block, slot, query and part group): the blocks of one position
  // block and slot, next to each other, share their key words through L2
  const int WB = (int)gridDim.x;
  const int lb = WB % 8 == 0 ? xcd_block((int)blockIdx.x, WB) : (int)blockIdx.x;
  const int jg = lb % (nq * ngr);
  const int t = (lb / (nq * ngr)) % ext;
  const int pb = lb / (nq * ngr * ext);
  const int j = jg / ngr, i0 = (jg % ngr) * PG;
  const int pos = pb * TPB + threadIdx.x;
  // key pointers and part sets of the amounts in LDS (a part set read from
  // the kernel arguments inside the loop would be a vector load, whose wait
  // holds up every word the chunk has requested before it)
  __shared__ const u64* kp[HOIST_MAX];
  __shared__ unsigned up[HOIST_MAX];
  for (int a = threadIdx.x; a < h.A; a += TPB) {
    kp[a] = gtab[h.g[a] >> 1];
    up[a] = mu.parts[a];
  }
  __syncthreads();
  if (pos >= N || t >= ext) return;
  const PrimeC& pr = P[tb.ext_prime[t]];
  const double q = (double)pr.q, qi = __longlong_as_double((long long)pr.pad[1]);
  const int kl = t < limbs ? t : L1 + (t - limbs);          // key limb (and mask limb) of slot t
  const u64* src[BETA];
  bool own[BETA];
#pragma unroll
  for (int d = 0; d < BETA; ++d) {
    const ModUpDigit& dg = tb.d[d];
    own[d] = t >= dg.src[0] && t < dg.src[0] + dg.nsrc;
    src[d] = own[d] ? x + (size_t)j * sx + xcs + (size_t)t * N : y + (size_t)j * sy + ((size_t)d * ext + t) * N;
  }
  const size_t ko = (size_t)kl * N + pos, kst = (size_t)key_limbs * N;
  const unsigned gmask = ((1u << PG) - 1) << i0;
  double su[PG], sw[PG];
#pragma unroll
  for (int p = 0; p < PG; ++p) su[p] = sw[p] = 0.0;
  // a chain slot's thread also forms the addends of its group's parts at its
  // position: sa[p] = sum over r in {0} u amounts(i) of mask_i[s_r] x0[s_r]
  // (the mask words the key sums read, the query's c0 gathered beside them;
  // every product within 1.25 q, the sums folded with the key sums), and
  // mask_i x1 after the loop
  const bool adh = t < limbs;
  const u64* X0 = x + (size_t)j * sx + (size_t)(adh ? t : 0) * N;
  double sa[PG];
#pragma unroll
  for (int p = 0; p < PG; ++p) {
    sa[p] = 0.0;
    if (adh && i0 + p < k)
      sa[p] = fred(fmul_mod_q(u64_to_f(masks[((size_t)(i0 + p) * ml + t) * N + pos]), u64_to_f(X0[pos]), qi, q), qi, q);
  }
  // MC amounts at a time, every word of them requested before the first
  // product (a ragged chunk repeats the last amount, unused); each amount adds
  // at most one product to a part's sums, which are folded after every
  // fold_period(q)-th amount (np counts them)
  constexpr int MC = 2;
  const int fmask = fpm::fold_period(q) - 1;
  int np = 0;
  for (int a0 = 0; a0 < h.A; a0 += MC) {
    unsigned use[MC];
    u64 v[MC][BETA], mw[MC][PG], xv[MC];
    double kb[MC][BETA], ka[MC][BETA];
#pragma unroll
    for (int c2 = 0; c2 < MC; ++c2) {
      const int a = a0 + c2 < h.A ? a0 + c2 : h.A - 1;
      use[c2] = a0 + c2 < h.A ? up[a] & gmask : 0u;
      const u32 s = autom_src((u32)pos, h.g[a], log_n, ms);
      xv[c2] = adh ? X0[s] : 0;
      const gdp key = (gdp)kp[a];
#pragma unroll
      for (int d = 0; d < BETA; ++d) {
        v[c2][d] = src[d][s];
        kb[c2][d] = key[ko + (size_t)(2 * d) * kst];
        ka[c2][d] = key[ko + (size_t)(2 * d + 1) * kst];
      }
#pragma unroll
      for (int p = 0; p < PG; ++p) mw[c2][p] = masks[((size_t)(i0 + p < k ? i0 + p : 0) * ml + kl) * N + s];
    }
#pragma unroll
    for (int c2 = 0; c2 < MC; ++c2) {
      if (a0 + c2 >= h.A) break;
      if (use[c2]) {
        double iu = 0.0, iw = 0.0;
#pragma unroll
        for (int d = 0; d < BETA; ++d) {
          const double vd = own[d] ? u64_to_f(v[c2][d]) : __longlong_as_double((long long)v[c2][d]);
          iu = __dadd_rn(iu, fmul_mod_q(vd, kb[c2][d], qi, q));
          iw = __dadd_rn(iw, fmul_mod_q(vd, ka[c2][d], qi, q));
          if (d & 1) {
            iu = fred(iu, qi, q);
            iw = fred(iw, qi, q);
          }
        }
        // the mask words multiply the reduced inner sums (|.| <= q/2 + 1)
        iu = fred(iu, qi, q);
        iw = fred(iw, qi, q);
#pragma unroll
        for (int p = 0; p < PG; ++p) {
          if ((use[c2] >> (i0 + p)) & 1) {
            const double m = u64_to_f(mw[c2][p]);
            su[p] = __dadd_rn(su[p], fmul_mod_q(iu, m, qi, q));
            sw[p] = __dadd_rn(sw[p], fmul_mod_q(iw, m, qi, q));
            if (adh) sa[p] = __dadd_rn(sa[p], fmul_mod_q(m, u64_to_f(xv[c2]), qi, q));
          }
        }
      }
      if ((++np & fmask) == 0) {
#pragma unroll
        for (int p = 0; p < PG; ++p) {
          su[p] = fred(su[p], qi, q);
          sw[p] = fred(sw[p], qi, q);
          sa[p] = fred(sa[p], qi, q);
        }
      }
    }
  }
  auto res = [&](double v) {
    const double r = fred(v, qi, q);
    return f_to_u64(r < 0.0 ? __dadd_rn(r, q) : r);
  };
  auto canon = [&](double v) {
    const double r = fred(v, qi, q);
    return r < 0.0 ? __dadd_rn(r, q) : r;
  };
  // inverse row pass of this block's row (block-uniform; N = 2^16, the
  // block's 256 positions one row of the 256 x 256 view): LDS holds the rows
  // [PG][2 components][VS], then the row's twiddles [512] (staged after the
  // sums: staged before them, their words would stay in registers)
  constexpr int VS = 256 + 16;
  const bool inv = t >= inv_from;
  extern __shared__ u64 hm_raw[];
  double* rsh = reinterpret_cast<double*>(hm_raw);
  double* ztl = rsh + PG * 2 * VS;
  if (inv) {
    const int pid = tb.ext_prime[t];
    for (int slot = (int)threadIdx.x; slot < 256; slot += TPB) {
      if (slot == 0) continue;
      const int st = 31 - __clz(slot);
      const int o = slot - (1 << st);
      const int b = st < 4 ? o : ((o & 15) << (st - 4)) + (o >> 4);
      const size_t g = (size_t)pid * N + (1 << (8 + st)) + (pb << st) + b;
      ztl[slot] = itwf[g];
      ztl[256 + slot] = itwq[g];
    }
  }
  auto pad = [](int a_) { return a_ + (a_ >> 4); };
#pragma unroll
  for (int p = 0; p < PG; ++p) {
    const int i = i0 + p;
    if (i >= k) break;
    const int e = j * k + i;
    double vu = su[p], vw = sw[p];
    if (adh) {   // the addends of part i at limb t: to ad, and P times them at the last chain limb
      const u64 a0 = res(sa[p]);
      const u64 a1 = res(fmul_mod_q(u64_to_f(masks[((size_t)i * ml + t) * N + pos]), u64_to_f(X0[xcs + pos]), qi, q));
      u64* A = ad + (size_t)e * sad + (size_t)t * N;
      A[pos] = a0;
      A[(size_t)limbs * N + pos] = a1;
      if (dadd && t == limbs - 1) {
        const double pmq = pmd / q;
        vu = __dadd_rn(fred(vu, qi, q), fmul_mod(u64_to_f(a0), pmd, pmq, q));
        vw = __dadd_rn(fred(vw, qi, q), fmul_mod(u64_to_f(a1), pmd, pmq, q));
      }
    }
    if (inv) {
      rsh[(p * 2 + 0) * VS + pad((int)threadIdx.x)] = canon(vu);
      rsh[(p * 2 + 1) * VS + pad((int)threadIdx.x)] = canon(vw);
      continue;
    }
    u64* U = uw + (size_t)e * suw + (size_t)t * N;
    U[pos] = res(vu);
    U[(size_t)ext * N + pos] = res(vw);
  }
  if (!inv) return;
  __syncthreads();
  // row v = (part p, component) of the block, lane u of 16
  const int v = (int)threadIdx.x >> 4, u = (int)threadIdx.x & 15;
  const bool act = v < 2 * min(PG, k - i0);
  double* R = rsh + (act ? v : 0) * VS;
  auto addr = [&](int p_, int jj) { return p_ == 0 ? (jj << 4) + u : (u << 4) + jj; };
  auto twid = [&](int p_, int kk, int jj, double& w, double& wq) {
    const int slot = p_ == 0 ? (1 << kk) + (jj >> (4 - kk)) : (1 << (4 + kk)) + ((jj >> (4 - kk)) << 4) + u;
    w = ztl[slot];
    wq = ztl[256 + slot];
  };
  double a[16];
  if (act) {
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) a[jj] = R[pad(addr(1, jj))];
    auto t1 = [&](int kk, int jj, double& w, double& wq) { twid(1, kk, jj, w, wq); };
    fpm::gs_phase16(a, false, qi, q, t1);
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) R[pad(addr(1, jj))] = a[jj];
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) a[jj] = R[pad(addr(0, jj))];
    auto t0 = [&](int kk, int jj, double& w, double& wq) { twid(0, kk, jj, w, wq); };
    fpm::gs_phase16(a, true, qi, q, t0);
    const int e = j * k + i0 + (v >> 1), comp = v & 1;
    u64* O = uw + (size_t)e * suw + (size_t)(comp * ext + t) * N + (size_t)pb * 256;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) O[addr(0, jj)] = f_to_u64(canon(a[jj]));
  }
}

// The same sums when every element uses the same amounts: one thread serves
// two neighbouring positions (16-byte loads: the automorphism maps an aligned
// pair of positions onto an aligned pair) of up to ZB elements of one limb, so
// each key word is loaded once and used ZB times from registers, and takes
// the amounts CH at a time, all their words requested before the first is
// used (memory latency, not arithmetic, sets the pace of this kernel).
//
// With inv_from < ext (N = 2^16: a block's 512 positions are two whole rows
// of the 256 x 256 view), the slots from inv_from on leave in the row pass
// of their inverse transform (the words an inverse row pass of the stored
// sums would give: the rows go through LDS, 16 lanes a row, as in
// k_kip_rows), so that the ModDown starts at its column pass.
template <int BETA, int ZB, int CH>
__global__ void k_kip_hoist_zb(const u64* y, size_t sy, const u64* x, size_t sx, const u64* const* gtab,
                               HoistArgs h, u64* uw, size_t suw, const ModUpTable* T, int key_limbs, int L1,
                               const PrimeC* P, int log_n, int ms, int B, int accumulate, AutomArgs am,
                               int order, const double* itwf, const double* itwq, int inv_from) {
  if ((int)blockIdx.x < am.W) {
    autom_sum_part(am, h, P, log_n, ms, accumulate, (int)blockIdx.x);
    return;
  }
  const ModUpTable& tb = *T;
  const int N = 1 << log_n;
  const int ext = tb.ext;
  // 1-D grid of (limb, position block, element group), element group fastest
  const int gx = N / (2 * TPB);
  const int ZG = (B + ZB - 1) / ZB;
  // order 0: element groups fastest (the groups of one position block share
  // its key words through L2); order 1: position blocks fastest (an XCD
  // works through one element group's positions while its gathered digit
  // words stay in L2, the key words streaming past); order 2 or 3: the
  // element groups in chunks of 2 or 4 (when they divide ZG), a chunk's
  // groups side by side and its position blocks after each other, so that
  // an XCD's L2 holds the gathered digits of the chunk's elements only while
  // each key word serves the chunk's groups (many elements: the other orders
  // re-fetch the digits for every amount, or the keys for every group).
  // The slot is slowest, so that each XCD gathers from one slot's digits
  // only (over the launch's amounts, any range of positions gathers from
  // every word of its slot); dealing every XCD all slots of an eighth of the
  // positions instead doubled the fetched bytes of this kernel.
  const int lb = xcd_block((int)blockIdx.x - am.W, (int)gridDim.x - am.W);
  const int t = lb / (ZG * gx);
  const int EG = order == 2 ? 2 : order == 3 ? 4 : 0;
  int zg, pb;
  if (EG && ZG % EG == 0) {
    const int r = lb % (ZG * gx);
    zg = (r / (EG * gx)) * EG + r % EG;
    pb = (r / EG) % gx;
  } else {
    zg = order == 1 ? (lb / gx) % ZG : lb % ZG;
    pb = order == 1 ? lb % gx : (lb / ZG) % gx;
  }
  const int i = 2 * (pb * TPB + (int)threadIdx.x);   // positions i, i + 1
  __shared__ const u64* kp[HOIST_MAX];
  for (int a = threadIdx.x; a < h.A; a += TPB) kp[a] = gtab[h.g[a] >> 1];
  __syncthreads();
  if (t >= ext) return;
  const int z0 = zg * ZB, nz = min(ZB, B - z0);
  const PrimeC& pr = P[tb.ext_prime[t]];
  const u64 q = pr.q;
  const int kl = t < tb.limbs ? t : L1 + (t - tb.limbs);
  const double qd = (double)q, qi = __longlong_as_double((long long)pr.pad[1]);
  // ModUp digits are FP64 values, the input limbs residue words
  const u64* src[BETA];
  size_t zst[BETA];
  bool own[BETA];
#pragma unroll
  for (int j = 0; j < BETA; ++j) {
    const ModUpDigit& dg = tb.d[j];
    own[j] = t >= dg.src[0] && t < dg.src[0] + dg.nsrc;
    src[j] = own[j] ? x + (size_t)z0 * sx + (size_t)t * N : y + (size_t)z0 * sy + ((size_t)j * ext + t) * N;
    zst[j] = own[j] ? sx : sy;
  }
  const size_t ko = (size_t)kl * N + i, kst = (size_t)key_limbs * N;
  double su[ZB][2], sw[ZB][2];
#pragma unroll
  for (int zz = 0; zz < ZB; ++zz) su[zz][0] = su[zz][1] = sw[zz][0] = sw[zz][1] = 0.0;
  const int fmask = fpm::fold_period(qd) - 1;   // block-uniform: the slot's prime
  int np = 0;
  for (int a0 = 0; a0 < h.A; a0 += CH) {
    dv2 kb[CH][BETA], ka[CH][BETA];
    ulonglong2 v[CH][BETA][ZB];
    bool swp[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int a = a0 + c < h.A ? a0 + c : h.A - 1;   // a ragged chunk repeats the last amount, unused
      const u32 s = autom_src((u32)i, h.g[a], log_n, ms);
      swp[c] = s & 1;                                    // position i reads the odd word of the pair
      const gdp key = (gdp)kp[a];
#pragma unroll
      for (int j = 0; j < BETA; ++j) {
        kb[c][j] = *(gd2p)(key + ko + (size_t)(2 * j) * kst);
        ka[c][j] = *(gd2p)(key + ko + (size_t)(2 * j + 1) * kst);
#pragma unroll
        for (int zz = 0; zz < ZB; ++zz)
          v[c][j][zz] = zz < nz ? *(const ulonglong2*)(src[j] + zz * zst[j] + (s & ~1u)) : make_ulonglong2(0, 0);
      }
    }
    // products; the sums are folded back to |s| <= q/2 + 1 after every
    // fold_period(q)-th product (np counts them across chunks)
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (a0 + c >= h.A) break;
#pragma unroll
      for (int j = 0; j < BETA; ++j) {
#pragma unroll
        for (int zz = 0; zz < ZB; ++zz) {
          const u64 w0 = swp[c] ? v[c][j][zz].y : v[c][j][zz].x, w1 = swp[c] ? v[c][j][zz].x : v[c][j][zz].y;
          const double v0 = own[j] ? u64_to_f(w0) : __longlong_as_double((long long)w0);
          const double v1 = own[j] ? u64_to_f(w1) : __longlong_as_double((long long)w1);
          su[zz][0] = __dadd_rn(su[zz][0], fmul_mod_q(v0, kb[c][j].x, qi, qd));
          su[zz][1] = __dadd_rn(su[zz][1], fmul_mod_q(v1, kb[c][j].y, qi, qd));
          sw[zz][0] = __dadd_rn(sw[zz][0], fmul_mod_q(v0, ka[c][j].x, qi, qd));
          sw[zz][1] = __dadd_rn(sw[zz][1], fmul_mod_q(v1, ka[c][j].y, qi, qd));
        }
        if ((++np & fmask) == 0) {
#pragma unroll
          for (int zz = 0; zz < ZB; ++zz)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
              su[zz][e] = fred(su[zz][e], qi, qd);
              sw[zz][e] = fred(sw[zz][e], qi, qd);
            }
        }
      }
    }
  }
  // the c0 half (am.W == 0: no blocks of its own): a block of a chain slot
  // also forms c0 + sum_a phi_a(c0) (or adds the sum, accumulate) at its two
  // positions of that limb for its elements, the pair read at the amount's
  // source pair as the digits are
  if (am.W == 0 && t < am.limbs) {
    const u64 ql = P[t].q;
#pragma unroll
    for (int zz = 0; zz < ZB; ++zz) {
      if (zz >= nz) break;
      const u64* I = am.in + (size_t)(z0 + zz) * am.si + (size_t)t * N;
      u64* O = am.out + (size_t)(z0 + zz) * am.so + (size_t)t * N;
      ulonglong2 acc = accumulate ? *(const ulonglong2*)(O + i) : *(const ulonglong2*)(I + i);
#pragma unroll 4
      for (int a = 0; a < h.A; ++a) {
        const u32 s = autom_src((u32)i, h.g[a], log_n, ms);
        const ulonglong2 w = *(const ulonglong2*)(I + (s & ~1u));
        acc.x = add_mod(acc.x, (s & 1) ? w.y : w.x, ql);
        acc.y = add_mod(acc.y, (s & 1) ? w.x : w.y, ql);
      }
      *(ulonglong2*)(O + i) = acc;
    }
  }
  auto canon = [&](double s_) {
    const double r = fred(s_, qi, qd);
    return r < 0.0 ? __dadd_rn(r, qd) : r;
  };
  auto res = [&](double s_) { return f_to_u64(canon(s_)); };
  // inverse row pass of this block's two rows (block-uniform): LDS holds the
  // rows [ZB][2 components][2 rows][VS] and then the rows' twiddles [2][512]
  constexpr int VS = 256 + 16;
  const bool inv = !accumulate && t >= inv_from;
  if (inv) {
    extern __shared__ u64 zb_raw[];
    double* rsh = reinterpret_cast<double*>(zb_raw);
    double* ztl = rsh + ZB * 4 * VS;
    const int pid = tb.ext_prime[t];
    for (int k = threadIdx.x; k < 512; k += TPB) {
      const int slot = k & 255, rr = k >> 8;
      if (slot == 0) continue;
      const int st = 31 - __clz(slot);
      const int o = slot - (1 << st);
      const int b = st < 4 ? o : ((o & 15) << (st - 4)) + (o >> 4);
      const size_t g = (size_t)pid * N + (1 << (8 + st)) + ((2 * pb + rr) << st) + b;
      ztl[rr * 512 + slot] = itwf[g];
      ztl[rr * 512 + 256 + slot] = itwq[g];
    }
    auto pad = [](int a_) { return a_ + (a_ >> 4); };
    const int bi = 2 * (int)threadIdx.x, br = bi >> 8, bc = bi & 255;   // row and column in the block
#pragma unroll
    for (int zz = 0; zz < ZB; ++zz) {
      if (zz >= nz) break;
      double* Ru = rsh + ((zz * 2 + 0) * 2 + br) * VS;
      double* Rw = rsh + ((zz * 2 + 1) * 2 + br) * VS;
      Ru[pad(bc)] = canon(su[zz][0]);
      Ru[pad(bc + 1)] = canon(su[zz][1]);
      Rw[pad(bc)] = canon(sw[zz][0]);
      Rw[pad(bc + 1)] = canon(sw[zz][1]);
    }
    __syncthreads();
    // row v = (element zz, component, row) of the block, lane u of 16
    const int v = (int)threadIdx.x >> 4, u = (int)threadIdx.x & 15;
    const bool act = v < 4 * nz;
    double* R = rsh + (act ? v : 0) * VS;
    const double* tv = ztl + (v & 1) * 512;
    auto addr = [&](int p_, int j) { return p_ == 0 ? (j << 4) + u : (u << 4) + j; };
    auto twid = [&](int p_, int k, int j, double& w, double& wq) {
      const int slot = p_ == 0 ? (1 << k) + (j >> (4 - k)) : (1 << (4 + k)) + ((j >> (4 - k)) << 4) + u;
      w = tv[slot];
      wq = tv[256 + slot];
    };
    double a[16];
    if (act) {
#pragma unroll
      for (int j = 0; j < 16; ++j) a[j] = R[pad(addr(1, j))];
      auto t1 = [&](int k, int j, double& w, double& wq) { twid(1, k, j, w, wq); };
      fpm::gs_phase16(a, false, qi, qd, t1);
#pragma unroll
      for (int j = 0; j < 16; ++j) R[pad(addr(1, j))] = a[j];
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int j = 0; j < 16; ++j) a[j] = R[pad(addr(0, j))];
      auto t0 = [&](int k, int j, double& w, double& wq) { twid(0, k, j, w, wq); };
      fpm::gs_phase16(a, true, qi, qd, t0);
      const int zz = v >> 2, comp = (v >> 1) & 1, rr = v & 1;
      u64* O = uw + (size_t)(z0 + zz) * suw + (size_t)(comp * ext + t) * N + (size_t)pb * 512 + rr * 256;
#pragma unroll
      for (int j = 0; j < 16; ++j) O[addr(0, j)] = f_to_u64(canon(a[j]));
    }
    return;
  }
#pragma unroll
  for (int zz = 0; zz < ZB; ++zz) {
    if (zz >= nz) break;
    u64* U = uw + (size_t)(z0 + zz) * suw + (size_t)t * N + i;
    u64* W = U + (size_t)ext * N;
    ulonglong2 ru = make_ulonglong2(res(su[zz][0]), res(su[zz][1]));
    ulonglong2 rw = make_ulonglong2(res(sw[zz][0]), res(sw[zz][1]));
    if (accumulate) {
      const ulonglong2 ou = *(ulonglong2*)U, ow = *(ulonglong2*)W;
      ru = make_ulonglong2(add_mod(ou.x, ru.x, q), add_mod(ou.y, ru.y, q));
      rw = make_ulonglong2(add_mod(ow.x, rw.x, q), add_mod(ow.y, rw.y, q));
    }
    *(ulonglong2*)U = ru;
    *(ulonglong2*)W = rw;
  }
}

// conv[c][i] = sum_k [u_c[p_k] (P/p_k)^-1]_{p_k} [P/p_k]_{q_i}   (coefficient domain)
__global__ void k_moddown_conv(const u64* uw, size_t suw, u64* conv, size_t sc,
                               const ModDownTable* D, int limbs, const PrimeC* P, int N) {
  const ModDownTable& md = *D;
  const int i = blockIdx.y % limbs, c = blockIdx.y / limbs;
  const u64 qi = P[i].q;
  const int ext = limbs + md.K;
  const size_t bz = blockIdx.z;
  const u64* Uc = uw + bz * suw + (size_t)c * ext * N;
  u64* C = conv + bz * sc + ((size_t)c * limbs + i) * N;
  for (int e = blockIdx.x * TPB + threadIdx.x; e < N; e += gridDim.x * TPB) {
    u64 acc = 0;
    for (int k = 0; k < md.K; ++k) {
      const u64 pk = P[md.pprime[k]].q;
      const u64 v = mul_shoup(Uc[(size_t)(limbs + k) * N + e], md.phatinv[k][0], md.phatinv[k][1], pk);
      acc = add_mod(acc, mul_shoup(v, md.phat[k][i][0], md.phat[k][i][1], qi), qi);
    }
    C[e] = acc;
  }
}

// out[c][i] = (u[c][i] - conv[c][i]) P^-1 mod q_i (+ add_c[i])
__global__ void k_moddown_finish(const u64* uw, size_t suw, const u64* conv, size_t sc,
                                 const u64* add0, size_t sa0, const u64* add1, size_t sa1,
                                 u64* out, size_t so, const ModDownTable* D, int limbs,
                                 const PrimeC* P, int N) {
  const ModDownTable& md = *D;
  const int i = blockIdx.y % limbs, c = blockIdx.y / limbs;
  const u64 qi = P[i].q;
  const int ext = limbs + md.K;
  const size_t bz = blockIdx.z;
  const u64* U = uw + bz * suw + ((size_t)c * ext + i) * N;
  const u64* C = conv + bz * sc + ((size_t)c * limbs + i) * N;
  const u64* A = c == 0 ? add0 : add1;
  const size_t sA = c == 0 ? sa0 : sa1;
  const u64* Ad = A ? A + bz * sA + (size_t)i * N : nullptr;
  u64* O = out + bz * so + ((size_t)c * limbs + i) * N;
  const u64 w = md.pinv[i][0], ws = md.pinv[i][1];
  for (int e = blockIdx.x * TPB + threadIdx.x; e < N; e += gridDim.x * TPB) {
    u64 r = mul_shoup(sub_mod(U[e], C[e], qi), w, ws, qi);
    if (Ad) r = add_mod(r, Ad[e], qi);
    O[e] = r;
  }
}

// t[c][i] = last_c mod q_i for i < limbs-1 (coefficient domain)
__global__ void k_rescale_conv(const u64* last, size_t sl, size_t lcs, u64* t, size_t st,
                               int comps, int limbs, const PrimeC* P, int N) {
  const int nl = limbs - 1;
  const int i = blockIdx.y % nl, c = blockIdx.y / nl;
  const PrimeC& pr = P[i];
  const size_t bz = blockIdx.z;
  const u64* Lp = last + bz * sl + (size_t)c * lcs;
  u64* T = t + bz * st + ((size_t)c * nl + i) * N;
  for (int e = blockIdx.x * TPB + threadIdx.x; e < N; e += gridDim.x * TPB) T[e] = reduce64(Lp[e], pr);
}

// out[c][i] = (in[c][i] - t[c][i]) q_last^-1 mod q_i
__global__ void k_rescale_finish(const u64* in, size_t si, const u64* t, size_t st, u64* out,
                                 size_t so, const u64* rs, int comps, int limbs, int nq,
                                 const PrimeC* P, int N) {
  const int nl = limbs - 1;
  const int i = blockIdx.y % nl, c = blockIdx.y / nl;
  const u64 qi = P[i].q;
  const size_t bz = blockIdx.z;
  const u64* I = in + bz * si + ((size_t)c * limbs + i) * N;
  const u64* T = t + bz * st + ((size_t)c * nl + i) * N;
  u64* O = out + bz * so + ((size_t)c * nl + i) * N;
  const u64* pair = rs + ((size_t)(limbs - 1) * nq + i) * 2;
  const u64 w = pair[0], ws = pair[1];
  for (int e = blockIdx.x * TPB + threadIdx.x; e < N; e += gridDim.x * TPB)
    O[e] = mul_shoup(sub_mod(I[e], T[e], qi), w, ws, qi);
}

// batch element z goes to out + (z / div) * so_hi + (z % div) * so_lo
// (with ref: one thread also stores ref_val at *ref, the output base a
// following graph replay reads)
__global__ void k_copy_limbs(const u64* in, size_t si, size_t ics, u64* out, int div, size_t so_hi,
                             size_t so_lo, size_t ocs, int limbs, int N, u64** ref, u64* ref_val) {
  if (ref && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) *ref = ref_val;
  const int l = blockIdx.y % limbs, c = blockIdx.y / limbs;
  const size_t bz = blockIdx.z;
  const u64* I = in + bz * si + c * ics + (size_t)l * N;
  u64* O = out + (bz / div) * so_hi + (bz % div) * so_lo + c * ocs + (size_t)l * N;
  for (int e = blockIdx.x * TPB + threadIdx.x; e < N; e += gridDim.x * TPB) O[e] = I[e];
}

// element z of `in` (stride si) to the address out.p[z]
__global__ void k_copy_ptrs(const u64* in, size_t si, size_t ics, OutTab out, size_t ocs, int limbs, int N) {
  const int l = blockIdx.y % limbs, c = blockIdx.y / limbs;
  const size_t bz = blockIdx.z;
  const u64* I = in + bz * si + c * ics + (size_t)l * N;
  u64* O = out.p[bz] + c * ocs + (size_t)l * N;
  for (int e = blockIdx.x * TPB + threadIdx.x; e < N; e += gridDim.x * TPB) O[e] = I[e];
}

// in place: residue word <-> bit pattern of its FP64 value (exact below 2^53)
__global__ void k_words_f64(u64* p, size_t n, int to_f64) {
  for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < n; e += (size_t)gridDim.x * TPB) {
    const u64 w = p[e];
    p[e] = to_f64 ? (u64)__double_as_longlong(u64_to_f(w)) : f_to_u64(__longlong_as_double((long long)w));
  }
}

__global__ void k_zero(u64* out, size_t words) {
  for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < words; e += (size_t)gridDim.x * TPB) out[e] = 0;
}

// element z of `words` words: gather out[z] = in[idx[z]], or scatter out[idx[z]] = in[z]
__global__ void k_move_idx(const u64* in, size_t si, u64* out, size_t so, const uint32_t* idx, int scatter,
                           size_t words) {
  const size_t z = blockIdx.z;
  const u64* I = in + (scatter ? z : (size_t)idx[z]) * si;
  u64* O = out + (scatter ? (size_t)idx[z] : z) * so;
  for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < words; e += (size_t)gridDim.x * TPB) O[e] = I[e];
}

// one element per thread (the element-wise kernels loop with a grid stride,
// so any grid is correct; small launches need every thread they can get)
inline dim3 ew_grid(size_t N, int ys, int B) {
  size_t bx = (N + TPB - 1) / TPB;
  if (bx == 0) bx = 1;
  return dim3((unsigned)bx, (unsigned)ys, (unsigned)B);
}

inline void check_launch() { HIP_OK(dev::last_error()); }

// ---- launch checks: the word range a launch touches in each operand
inline int max_off(const LimbMap& m, bool out = false) {
  int x = 0;
  for (int i = 0; i < m.n; ++i) x = std::max(x, out ? m.ooff[i] : m.off[i]);
  return x;
}
inline int min_off(const LimbMap& m, bool out = false) {
  int x = 1 << 30;
  for (int i = 0; i < m.n; ++i) x = std::min(x, out ? m.ooff[i] : m.off[i]);
  return x;
}
// operand with B batch elements of stride `st` whose last touched word is at
// `tail` words past the element start, first touched word `head`
inline void chk(const void* p, int B, size_t st, size_t head, size_t tail, const char* what) {
  if (B <= 0) return;
  const u64* base = (const u64*)p + head;
  audit::check(base, ((size_t)(B - 1) * st + tail - head) * sizeof(u64), what);
}
inline void chk_map(const Ctx& c, const void* p, int B, size_t st, const LimbMap& m, const char* what,
                    bool out = false) {
  for (int i = 0; i < m.n; ++i)
    if (m.prime[i] < 0 || m.prime[i] >= c.nprimes()) BM_THROW(BM_EINVAL, "launch check: prime id");
  chk(p, B, st, (size_t)min_off(m, out) * c.N, (size_t)(max_off(m, out) + 1) * c.N, what);
}

// Times one launch when the context's profiler is on.
struct Prof {
  bool on;
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  Prof(const Ctx& c, const char* name, double bytes, double ops) : on(c.prof && c.prof->on && !dev::sizing()) {
    if (on) ev = c.prof->begin(name, bytes, ops);
  }
  Prof(const Ctx& c, const std::string& name, double bytes, double ops) : Prof(c, name.c_str(), bytes, ops) {}
};

}  // namespace

// Scratch memory of the no-allocation match (bm_match_noalloc): its
// intermediate buffers are carved out of this array, which every context on a
// device shares.  In host code `scratch` names a host-side stand-in, never the
// device memory: kernels get the address from hipGetSymbolAddress.
static __device__ __align__(256) u64 scratch[NOALLOC_SCRATCH_BYTES / sizeof(u64)];

namespace kern {

void* noalloc_scratch(int device) {
  static std::mutex mu;
  static std::map<int, void*> ptrs;   // device -> address of that device's copy
  std::lock_guard<std::mutex> g(mu);
  auto it = ptrs.find(device);
  if (it != ptrs.end()) return it->second;
  void* p = nullptr;
  if (dev::dry()) {
    p = std::malloc(NOALLOC_SCRATCH_BYTES);   // host memory stands in for HBM
    if (!p) BM_THROW(BM_ENOMEM, "host stand-in of the scratch array");
  } else {
    HIP_OK(dev::set_device(device));
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  }
  audit::add(p, NOALLOC_SCRATCH_BYTES);
  ptrs[device] = p;
  return p;
}

LimbMap chain_map(int limbs) {
  LimbMap m{};
  m.n = limbs;
  for (int i = 0; i < limbs; ++i) { m.prime[i] = i; m.off[i] = m.ooff[i] = i; }
  return m;
}

LimbMap ext_map(const Ctx& c, int limbs) {
  LimbMap m{};
  m.n = limbs + c.K;
  for (int i = 0; i < limbs; ++i) { m.prime[i] = i; m.off[i] = m.ooff[i] = i; }
  for (int k = 0; k < c.K; ++k) {
    m.prime[limbs + k] = c.pid_special(k);
    m.off[limbs + k] = m.ooff[limbs + k] = limbs + k;
  }
  return m;
}

LimbMap single(int prime, int off) {
  LimbMap m{};
  m.n = 1;
  m.prime[0] = prime;
  m.off[0] = m.ooff[0] = off;
  return m;
}


// row-pass views per block (polynomials x rows): 16 unless tuned to 4 or 8
static int row_views(const Ctx& c) { return c.ntt_views == 4 || c.ntt_views == 8 ? c.ntt_views : 16; }

// N = 2^12: one 12-stage pass; N = 2^16: 8 column stages then 8 row stages
// (inverse: rows first).  Row passes take up to 16 polynomials per block.
// only: 0 both passes; for the inverse transform 1 the row pass only, 2 the
// column pass only (the input then holds the row pass's output)
void ntt_fast(const Ctx& c, const u64* in, size_t in_stride, u64* out, size_t out_stride, int B,
              const LimbMap& m, const LimbMap& m_out, bool inverse, int only = 0) {
  const int logn = c.log_n;
  const int N = 1 << logn;
  const double elems = (double)N * m.n * B;
  const double* tw = inverse ? c.d_itwf : c.d_twf;
  const double* tws = inverse ? c.d_itwq : c.d_twq;
  if (logn == 12) {
    chk_map(c, in, B, in_stride, m, "ntt input");
    chk_map(c, out, B, out_stride, m, "ntt output", true);
    Prof pf(c, inverse ? "k_ntt_fast<12, true, 2, 0>" : "k_ntt_fast<12, false, 2, 0>", 16.0 * elems,
            0.5 * elems * 12);
    const size_t lds = (size_t)(4096 + 256 + 1) * sizeof(u64);
    const dim3 grid(1, (unsigned)m.n, (unsigned)B);
    if (inverse)
      LAUNCH((k_ntt_fast<12, true, NTT_ONE>), grid, dim3(256), lds, c.stream, in, in_stride, out,
             out_stride, m, c.d_primes, tw, tws, logn, 0, 1, B, 1, FuseArgs{});
    else
      LAUNCH((k_ntt_fast<12, false, NTT_ONE>), grid, dim3(256), lds, c.stream, in, in_stride, out,
             out_stride, m, c.d_primes, tw, tws, logn, 0, 0, B, 1, FuseArgs{});
    check_launch();
    return;
  }
  // row passes: vz polynomials x R rows per block, R the largest power of two
  // with vz R <= V (whole waves for small batches; V = 16 or the context's
  // tuning) and at most 64 KiB of LDS
  const int V = row_views(c);
  const int vz = B < V ? B : V;
  const size_t view_words = 256 + 16 + 1;   // column views; row views are one word shorter
  auto row_lds = [&](int r) { return ((size_t)vz * r * (view_words - 1) + (size_t)512 * r) * sizeof(u64); };
  int R = 1;
  while (vz * R * 2 <= V && row_lds(2 * R) <= 65536) R *= 2;
  const int Vrow = vz * R;
  const size_t lds_col = ((size_t)16 * view_words + 512) * sizeof(u64);
  const size_t lds_row = row_lds(R);
  const dim3 gcol(N / 256 / 16, (unsigned)m.n, (unsigned)B);
  const dim3 grow((unsigned)(N / 256 / R), (unsigned)m.n, (unsigned)((B + vz - 1) / vz));
  auto col = [&](const u64* src, size_t ss, u64* dst, size_t ds, const LimbMap& mm, int last) {
    chk_map(c, src, B, ss, mm, "ntt column pass input");
    chk_map(c, dst, B, ds, mm, "ntt column pass output", true);
    Prof pf(c, inverse ? "k_ntt_fast<8, true, 0, 0>" : "k_ntt_fast<8, false, 0, 0>", 16.0 * elems, 0.5 * elems * 8);
    if (inverse)
      LAUNCH((k_ntt_fast<8, true, NTT_COL>), gcol, dim3(256), lds_col, c.stream, src, ss, dst, ds, mm,
             c.d_primes, tw, tws, logn, 0, last, B, 1, FuseArgs{});
    else
      LAUNCH((k_ntt_fast<8, false, NTT_COL>), gcol, dim3(256), lds_col, c.stream, src, ss, dst, ds, mm,
             c.d_primes, tw, tws, logn, 0, last, B, 1, FuseArgs{});
    check_launch();
  };
  auto row = [&](const u64* src, size_t ss, u64* dst, size_t ds, const LimbMap& mm) {
    chk_map(c, src, B, ss, mm, "ntt row pass input");
    chk_map(c, dst, B, ds, mm, "ntt row pass output", true);
    Prof pf(c, inverse ? "k_ntt_fast<8, true, 1, 0>" : "k_ntt_fast<8, false, 1, 0>", 16.0 * elems, 0.5 * elems * 8);
    if (inverse)
      LAUNCH((k_ntt_fast<8, true, NTT_ROW>), grow, dim3(16 * Vrow), lds_row, c.stream, src, ss, dst, ds,
             mm, c.d_primes, tw, tws, logn, 8, 0, B, vz, FuseArgs{});
    else
      LAUNCH((k_ntt_fast<8, false, NTT_ROW>), grow, dim3(16 * Vrow), lds_row, c.stream, src, ss, dst, ds,
             mm, c.d_primes, tw, tws, logn, 8, 0, B, vz, FuseArgs{});
    check_launch();
  };
  if (!inverse) {
    col(in, in_stride, out, out_stride, m, 0);
    row(out, out_stride, out, out_stride, m_out);
  } else if (only == 2) {
    col(in, in_stride, out, out_stride, m, 1);
  } else {
    row(in, in_stride, out, out_stride, m);
    if (only != 1) col(out, out_stride, out, out_stride, m_out, 1);
  }
}

void modmul_rate(const Ctx& c, int pid, int blocks, int iters, const u64* seed, u64* out) {
  if (pid < 0 || pid >= c.nprimes() || blocks < 1 || iters < 2 || (iters & 1))
    BM_THROW(BM_EINVAL, "launch check: modmul probe arguments");
  chk(seed, 1, 0, 0, 24, "modmul probe seed");
  chk(out, 1, 0, 0, (size_t)blocks * 256 * 16, "modmul probe output");
  Prof pf(c, "k_modmul_rate", 0.0, 8.0 * 256 * blocks * iters);
  LAUNCH(k_modmul_rate, dim3((unsigned)blocks), dim3(256), 0, c.stream, c.d_primes, pid, iters, seed, out);
  check_launch();
}

bool fused_ok(const Ctx& c) { return c.log_n == 16; }

void words_f64(const Ctx& c, u64* p, size_t n, bool to_f64) {
  if (n == 0) return;
  chk(p, 1, 0, 0, n, "words_f64");
  Prof pf(c, "k_words_f64", 16.0 * n, 0.0);
  const size_t bx = std::min<size_t>((n + TPB - 1) / TPB, 65536);
  LAUNCH(k_words_f64, dim3((unsigned)bx), dim3(TPB), 0, c.stream, p, n, to_f64 ? 1 : 0);
  check_launch();
}

// source primes whose inverse twiddles a fused column pass with isrc stages
// (the most any of its blocks takes)
static int isrc_count(const Ctx& c, const FuseArgs& f) {
  if (f.pro == 3) return 1;
  if (f.pro == 4) return c.K + 1;
  if (f.pro == 2) return c.K;
  int n = 0;
  const ModUpTable& tb = c.h_modup[(int)(f.mu - c.d_modup)];
  for (int j = 0; j < tb.beta; ++j) n = std::max(n, tb.d[j].nsrc);
  return n;
}

bool isrc_ok(const Ctx& c, int pro) {
  if (!fused_ok(c) || c.ci || c.col_src == 1) return false;
  const int n = pro == 3 ? 1 : pro == 4 ? c.K + 1 : pro == 2 ? c.K : c.alpha;
  return n >= 1 && n <= 5;
}

void ntt_inv_rows(const Ctx& c, const u64* in, size_t in_stride, u64* out, size_t out_stride, int B,
                  const LimbMap& m) {
  if (!fused_ok(c)) BM_THROW(BM_EINVAL, "launch check: inverse row pass needs N = 2^16");
  if (B <= 0 || m.n <= 0) return;
  LimbMap m_out = m;
  for (int i = 0; i < m.n; ++i) m_out.off[i] = m.ooff[i];
  ntt_fast(c, in, in_stride, out, out_stride, B, m, m_out, true, 1);
}

void ntt_inv_cols(const Ctx& c, const u64* in, size_t in_stride, u64* out, size_t out_stride, int B,
                  const LimbMap& m) {
  if (!fused_ok(c)) BM_THROW(BM_EINVAL, "launch check: inverse column pass needs N = 2^16");
  if (B <= 0 || m.n <= 0) return;
  ntt_fast(c, in, in_stride, out, out_stride, B, m, m, true, 2);
}

void ntt_fused(const Ctx& c, const FuseArgs& f, u64* tmp, size_t ts, int B, const LimbMap& m, bool f64_out) {
  if (!fused_ok(c)) BM_THROW(BM_EINVAL, "launch check: fused transform needs N = 2^16");
  if (B <= 0 || m.n <= 0) return;
  if (f.pro < 1 || f.pro > 4 || !f.src || f.s_div < 1 || f.e_div < 1 || (f.pro == 1 && !f.mu) ||
      ((f.pro == 2 || f.pro == 4) && !f.md) || (f.epi && (!f.mnd || !f.out || !f.wtab)) ||
      (f.epi == 2 && !f.wmtab) || (f.pro == 4 && (f.last_pid < 0 || f.last_pid >= c.nprimes() || f.last_off < 0)) ||
      (c.ci != (f.ci != nullptr)) ||
      (f.ci && f.pro == 3 && (f.src_pid < 0 || f.src_pid >= c.nprimes())) ||
      (f.isrc && (!isrc_ok(c, f.pro) || f.itwf != c.d_itwf || f.itwq != c.d_itwq ||
                  (f.pro == 3 && (f.src_pid < 0 || f.src_pid >= c.nprimes())))))
    BM_THROW(BM_EINVAL, "launch check: fused transform arguments");
  const int logn = 16, N = 1 << logn;
  LimbMap mo = m;
  for (int i = 0; i < m.n; ++i) mo.off[i] = mo.ooff[i];
  chk_map(c, tmp, B, ts, mo, "fused ntt scratch", true);
  const double elems = (double)N * m.n * B;
  // launch geometry of ntt_fast's forward passes
  const int V = row_views(c);
  const int vz = B < V ? B : V;
  const size_t view_words = 256 + 16 + 1;
  auto row_lds = [&](int r) { return ((size_t)vz * r * (view_words - 1) + (size_t)512 * r) * sizeof(u64); };
  int R = 1;
  while (vz * R * 2 <= V && row_lds(2 * R) <= 65536) R *= 2;
  const int Vrow = vz * R;
  const size_t lds_col = ((size_t)16 * view_words + 512) * sizeof(u64);
  const dim3 gcol(N / 256 / 16, (unsigned)m.n, (unsigned)B);
  const dim3 grow((unsigned)(N / 256 / R), (unsigned)m.n, (unsigned)((B + vz - 1) / vz));
  {
    // distinct words: every output word once, every source word once (a
    // digit's source limbs are read by each of its target slots, from L2)
    const double srcs = f.pro == 1 ? 2.0 : f.pro == 2 ? (double)c.K : 1.0;
    double src_words;
    if (f.pro == 1) {
      const int limbs = (int)(f.mu - c.d_modup);
      src_words = (double)N * B * limbs;
    } else if (f.pro == 2) {
      src_words = (double)N * B * c.K;
    } else if (f.pro == 4) {
      src_words = (double)N * B * (c.K + 1);
    } else {
      src_words = (double)N * B;
    }
    // the conversion prologues 1, 2 and 4 hold many registers: with the
    // fused_occupancy knob they are built for 4 resident blocks per CU
    const int occ = (c.fused_occ == 4 || c.fused_occ == 3) && f.pro != 3 ? c.fused_occ : 0;
    const int is = f.isrc ? 1 : 0;
    const std::string pname = std::string("k_ntt_fast<8, false, 0, ") + (f.ci ? "4, " : "1, ") +
                              std::to_string(f.pro) + ", 0, " + std::to_string(occ) + (is ? ", 1>" : ">");
    // the inverse column pass of the sources: 8 stages per source word
    const double is_ops = is ? 0.5 * 8 * (double)N * B * isrc_count(c, f) * m.n : 0.0;
    Prof pf(c, pname, 8.0 * (elems + src_words), 0.5 * elems * 8 + 2.0 * srcs * elems + is_ops);
    // IS: the source primes' inverse twiddles follow the block's own in LDS
    const size_t lds_is = lds_col + (size_t)(is ? isrc_count(c, f) : 0) * 512 * sizeof(double);
#define FUSED_COL(FZ, PKV, OC)                                                                                    \
  LAUNCH((k_ntt_fast<8, false, NTT_COL, FZ, PKV, 0, OC>), gcol, dim3(256), lds_col, c.stream, (const u64*)nullptr, \
         (size_t)0, tmp, ts, mo, c.d_primes, c.d_twf, c.d_twq, logn, 0, 0, B, 1, f)
#define FUSED_COL_IS(PKV, OC)                                                                                     \
  LAUNCH((k_ntt_fast<8, false, NTT_COL, 1, PKV, 0, OC, 1>), gcol, dim3(256), lds_is, c.stream, (const u64*)nullptr, \
         (size_t)0, tmp, ts, mo, c.d_primes, c.d_twf, c.d_twq, logn, 0, 0, B, 1, f)
    const int code = is * 1000 + (f.ci ? 100 : 0) + f.pro * 10 + occ;
    switch (code) {
      case 1010: FUSED_COL_IS(1, 0); break;
      case 1020: FUSED_COL_IS(2, 0); break;
      case 1030: FUSED_COL_IS(3, 0); break;
      case 1040: FUSED_COL_IS(4, 0); break;
      case 1014: FUSED_COL_IS(1, 4); break;
      case 1024: FUSED_COL_IS(2, 4); break;
      case 1044: FUSED_COL_IS(4, 4); break;
      case 1013: FUSED_COL_IS(1, 3); break;
      case 1023: FUSED_COL_IS(2, 3); break;
      case 1043: FUSED_COL_IS(4, 3); break;
      case 13: FUSED_COL(1, 1, 3); break;
      case 23: FUSED_COL(1, 2, 3); break;
      case 43: FUSED_COL(1, 4, 3); break;
      case 113: FUSED_COL(4, 1, 3); break;
      case 123: FUSED_COL(4, 2, 3); break;
      case 143: FUSED_COL(4, 4, 3); break;
      case 10: FUSED_COL(1, 1, 0); break;
      case 20: FUSED_COL(1, 2, 0); break;
      case 30: FUSED_COL(1, 3, 0); break;
      case 40: FUSED_COL(1, 4, 0); break;
      case 14: FUSED_COL(1, 1, 4); break;
      case 24: FUSED_COL(1, 2, 4); break;
      case 44: FUSED_COL(1, 4, 4); break;
      case 110: FUSED_COL(4, 1, 0); break;
      case 120: FUSED_COL(4, 2, 0); break;
      case 130: FUSED_COL(4, 3, 0); break;
      case 140: FUSED_COL(4, 4, 0); break;
      case 114: FUSED_COL(4, 1, 4); break;
      case 124: FUSED_COL(4, 2, 4); break;
      case 144: FUSED_COL(4, 4, 4); break;
      default: BM_THROW(BM_EINVAL, "launch check: fused column pass kind");
    }
#undef FUSED_COL
#undef FUSED_COL_IS
    check_launch();
  }
  if (f.no_row) {
    if (f.epi) BM_THROW(BM_EINVAL, "launch check: an epilogue needs the row pass");
    return;
  }
  if (f.epi) {
    Prof pf(c, f.epi == 2 ? "k_ntt_fast<8, false, 1, 2, 0, 2>" : "k_ntt_fast<8, false, 1, 2, 0, 1>",
            8.0 * elems * (f.add0 || f.add1 ? 4.0 : 3.0), 0.5 * elems * 8 + elems);
    if (f.epi == 2)
      LAUNCH((k_ntt_fast<8, false, NTT_ROW, 2, 0, 2>), grow, dim3(16 * Vrow), row_lds(R), c.stream, (const u64*)tmp,
             ts, (u64*)nullptr, (size_t)0, mo, c.d_primes, c.d_twf, c.d_twq, logn, 8, 0, B, vz, f);
    else
      LAUNCH((k_ntt_fast<8, false, NTT_ROW, 2, 0, 1>), grow, dim3(16 * Vrow), row_lds(R), c.stream, (const u64*)tmp,
             ts, (u64*)nullptr, (size_t)0, mo, c.d_primes, c.d_twf, c.d_twq, logn, 8, 0, B, vz, f);
  } else if (f64_out) {
    Prof pf(c, "k_ntt_fast<8, false, 1, 3>", 16.0 * elems, 0.5 * elems * 8);
    LAUNCH((k_ntt_fast<8, false, NTT_ROW, 3>), grow, dim3(16 * Vrow), row_lds(R), c.stream, (const u64*)tmp, ts,
           tmp, ts, mo, c.d_primes, c.d_twf, c.d_twq, logn, 8, 0, B, vz, FuseArgs{});
  } else {
    Prof pf(c, "k_ntt_fast<8, false, 1, 0>", 16.0 * elems, 0.5 * elems * 8);
    LAUNCH((k_ntt_fast<8, false, NTT_ROW>), grow, dim3(16 * Vrow), row_lds(R), c.stream, (const u64*)tmp, ts, tmp,
           ts, mo, c.d_primes, c.d_twf, c.d_twq, logn, 8, 0, B, vz, FuseArgs{});
  }
  check_launch();
}

// Conjugate-invariant ring: reduction modulo X^N - iota before the forward
// transform, and its inverse after the inverse transform (k_ci_fold).
void ci_fold(const Ctx& c, const u64* in, size_t si, u64* out, size_t so, int B, const LimbMap& m,
             bool inverse) {
  chk_map(c, in, B, si, m, "ci fold input");
  chk_map(c, out, B, so, m, "ci fold output", true);
  Prof pf(c, "k_ci_fold", 16.0 * c.N * m.n * B, 2.0 * c.N * m.n * B);
  size_t bx = (c.N / 2 + 1 + TPB * 2 - 1) / (TPB * 2);
  LAUNCH(k_ci_fold, dim3((unsigned)bx, (unsigned)m.n, (unsigned)B), dim3(TPB), 0, c.stream, in, si, out, so, m,
         c.d_primes, c.d_ci, (int)c.N, inverse ? 1 : 0);
  check_launch();
}

void ntt_core(const Ctx& c, const u64* in, size_t in_stride, u64* out, size_t out_stride, int B,
              const LimbMap& m, bool inverse);

void ntt(const Ctx& c, const u64* in, size_t in_stride, u64* out, size_t out_stride, int B,
         const LimbMap& m, bool inverse, bool raw) {
  if (B <= 0 || m.n <= 0) return;
  if (!c.ci || raw) {
    ntt_core(c, in, in_stride, out, out_stride, B, m, inverse);
    return;
  }
  // the second step works in place on `out`, addressed with the output offsets
  LimbMap m_out = m;
  for (int i = 0; i < m.n; ++i) m_out.off[i] = m.ooff[i];
  if (!inverse) {
    ci_fold(c, in, in_stride, out, out_stride, B, m, false);
    ntt_core(c, out, out_stride, out, out_stride, B, m_out, false);
  } else {
    ntt_core(c, in, in_stride, out, out_stride, B, m, true);
    ci_fold(c, out, out_stride, out, out_stride, B, m_out, true);
  }
}

void ntt_core(const Ctx& c, const u64* in, size_t in_stride, u64* out, size_t out_stride, int B,
              const LimbMap& m, bool inverse) {
  const int logn = c.log_n;
  const int N = 1 << logn;
  const int E = N < NTT_E ? N : NTT_E;
  const dim3 grid((unsigned)(N / E), (unsigned)m.n, (unsigned)B);
  // The second pass works in place on `out`, so it must address its input with
  // the output offsets.
  LimbMap m_out = m;
  for (int i = 0; i < m.n; ++i) m_out.off[i] = m.ooff[i];
  auto launch = [&](const u64* src, size_t ss, u64* dst, size_t ds, int logm, int s0, int col,
                    int last, const LimbMap& mm) {
    const int M = 1 << logm;
    const size_t lds = (size_t)(E / M) * (M + 1) * sizeof(u64);
    // the pass reads src at mm.off and writes dst at mm.ooff
    chk_map(c, src, B, ss, mm, "ntt pass input");
    chk_map(c, dst, B, ds, mm, "ntt pass output", true);
    const double elems = (double)N * m.n * B;
    Prof pf(c, inverse ? "k_ntt_pass<true>" : "k_ntt_pass<false>", 16.0 * elems, 0.5 * elems * logm);
    if (inverse)
      LAUNCH(k_ntt_pass<true>, grid, dim3(TPB), lds, c.stream, src, ss, dst, ds, mm,
                         c.d_primes, c.d_itw, c.d_itws, logn, logm, s0, col, last);
    else
      LAUNCH(k_ntt_pass<false>, grid, dim3(TPB), lds, c.stream, src, ss, dst, ds, mm,
                         c.d_primes, c.d_tw, c.d_tws, logn, logm, s0, col, last);
    check_launch();
  };
  if (logn == 12 || logn == 16) {
    ntt_fast(c, in, in_stride, out, out_stride, B, m, m_out, inverse);
    return;
  }
  if (logn <= 12) {
    launch(in, in_stride, out, out_stride, logn, 0, 0, inverse ? 1 : 0, m);
    return;
  }
  const int la = logn / 2, lb = logn - la;
  if (!inverse) {
    launch(in, in_stride, out, out_stride, la, 0, 1, 0, m);
    launch(out, out_stride, out, out_stride, lb, la, 0, 0, m_out);
  } else {
    launch(in, in_stride, out, out_stride, lb, la, 0, 0, m);
    launch(out, out_stride, out, out_stride, la, 0, 1, 1, m_out);
  }
}

void reduce_int(const Ctx& c, const int64_t* src, u64* out, size_t out_stride, int B,
                size_t src_stride, const LimbMap& m) {
  chk(src, B, src_stride, 0, c.N, "reduce_int input");
  chk_map(c, out, B, out_stride, m, "reduce_int output");
  Prof pf(c, "k_reduce_int", 8.0 * c.N * B * (1 + m.n), (double)c.N * B * m.n);
  LAUNCH(k_reduce_int, ew_grid(c.N, m.n, B), dim3(TPB), 0, c.stream, src, src_stride,
                     out, out_stride, m, c.d_primes, (int)c.N);
  check_launch();
}

void add(const Ctx& c, const u64* a, size_t sa, const u64* b, size_t sb, u64* o, size_t so, int B,
         const LimbMap& m) {
  chk_map(c, a, B, sa, m, "add a");
  chk_map(c, b, B, sb, m, "add b");
  chk_map(c, o, B, so, m, "add out");
  Prof pf(c, "k_add", 24.0 * c.N * B * m.n, (double)c.N * B * m.n);
  LAUNCH(k_add, ew_grid(c.N, m.n, B), dim3(TPB), 0, c.stream, a, sa, b, sb, o, so, m,
                     c.d_primes, (int)c.N);
  check_launch();
}

void sub(const Ctx& c, const u64* a, size_t sa, const u64* b, size_t sb, u64* o, size_t so, int B,
         const LimbMap& m) {
  chk_map(c, a, B, sa, m, "sub a");
  chk_map(c, b, B, sb, m, "sub b");
  chk_map(c, o, B, so, m, "sub out");
  Prof pf(c, "k_sub", 24.0 * c.N * B * m.n, (double)c.N * B * m.n);
  LAUNCH(k_sub, ew_grid(c.N, m.n, B), dim3(TPB), 0, c.stream, a, sa, b, sb, o, so, m,
                     c.d_primes, (int)c.N);
  check_launch();
}

void mul(const Ctx& c, const u64* a, size_t sa, const u64* b, size_t sb, u64* o, size_t so, int B,
         const LimbMap& m) {
  chk_map(c, a, B, sa, m, "mul a");
  chk_map(c, b, B, sb, m, "mul b");
  chk_map(c, o, B, so, m, "mul out");
  Prof pf(c, "k_mul", 24.0 * c.N * B * m.n, (double)c.N * B * m.n);
  LAUNCH(k_mul, ew_grid(c.N, m.n, B), dim3(TPB), 0, c.stream, a, sa, b, sb, o, so, m,
                     c.d_primes, (int)c.N);
  check_launch();
}

void mul_ct_pt(const Ctx& c, const u64* ct, size_t sct, size_t ccs, const u64* pt, size_t spt, u64* out, size_t so,
               size_t ocs, int B, int limbs, int ct_div, int pt_mod) {
  if (limbs < 1 || limbs > c.L + 1) BM_THROW(BM_EINVAL, "launch check: mul_ct_pt limbs");
  if (ct_div < 1 || pt_mod < 1) BM_THROW(BM_EINVAL, "launch check: mul_ct_pt divisors");
  const int n_ct = (B - 1) / ct_div + 1, n_pt = std::min(B, pt_mod);
  chk(ct, n_ct, sct, 0, ccs + (size_t)limbs * c.N, "mul_ct_pt ciphertext");
  chk(pt, n_pt, spt, 0, (size_t)limbs * c.N, "mul_ct_pt plaintext");
  chk(out, B, so, 0, ocs + (size_t)limbs * c.N, "mul_ct_pt output");
  const double cts = sct ? (double)n_ct : 1.0, pts = spt ? (double)n_pt : 1.0;
  Prof pf(c, "k_mul_ct_pt", 8.0 * c.N * limbs * (2.0 * B + 2.0 * cts + pts), 2.0 * c.N * B * limbs);
  LAUNCH(k_mul_ct_pt, ew_grid(c.N, 2 * limbs, B), dim3(TPB), 0, c.stream, ct, sct, ccs, pt, spt, out, so, ocs, limbs,
         c.d_primes, (int)c.N, ct_div, pt_mod);
  check_launch();
}

void axpy_scalar(const Ctx& c, const u64* s, size_t ss, const u64* scal, u64* o, size_t so, int B,
                 const LimbMap& m) {
  chk_map(c, s, B, ss, m, "axpy s");
  chk_map(c, o, B, so, m, "axpy out");
  audit::check(scal, 2 * sizeof(u64) * m.n, "axpy scalars");
  Prof pf(c, "k_axpy_scalar", 24.0 * c.N * B * m.n, (double)c.N * B * m.n);
  LAUNCH(k_axpy_scalar, ew_grid(c.N, m.n, B), dim3(TPB), 0, c.stream, s, ss, scal, o,
                     so, m, c.d_primes, (int)c.N);
  check_launch();
}

void tensor_ptrs(const Ctx& c, const u64* const* a, size_t a_cs, size_t a_ps, const u64* const* b, size_t b_cs,
                 size_t b_ps, int parts, u64* o, size_t so, int n, int limbs, bool accumulate) {
  if (parts < 1) BM_THROW(BM_EINVAL, "launch check: tensor parts");
  if (limbs > c.L + 1 || a_cs < (size_t)limbs * c.N || b_cs < (size_t)limbs * c.N)
    BM_THROW(BM_EINVAL, "launch check: tensor limbs");
  const size_t pa = (size_t)(parts - 1) * a_ps, pb = (size_t)(parts - 1) * b_ps;
  for (int z0 = 0; z0 < n; z0 += PTR_MAX) {
    const int B = std::min(PTR_MAX, n - z0);
    PtrTab A{}, Bt{};
    std::vector<const u64*> da, db;          // distinct operands, for the byte count
    for (int z = 0; z < B; ++z) {
      A.p[z] = a[z0 + z];
      Bt.p[z] = b[z0 + z];
      chk(A.p[z], 1, 0, 0, pa + a_cs + (size_t)limbs * c.N, "tensor a");
      chk(Bt.p[z], 1, 0, 0, pb + b_cs + (size_t)limbs * c.N, "tensor b");
      da.push_back(A.p[z]);
      db.push_back(Bt.p[z]);
    }
    u64* oz = o + (size_t)z0 * so;
    chk(oz, B, so, 0, (size_t)3 * limbs * c.N, "tensor out");
    std::sort(da.begin(), da.end());
    std::sort(db.begin(), db.end());
    const double na = (double)(std::unique(da.begin(), da.end()) - da.begin());
    const double nb = (double)(std::unique(db.begin(), db.end()) - db.begin());
    // distinct words: each query part and each gallery part once, the outputs
    Prof pf(c, "k_tensor", 8.0 * c.N * limbs * (2.0 * parts * (na + nb) + (accumulate ? 6.0 : 3.0) * B),
            4.0 * c.N * B * limbs * parts);
    LAUNCH(k_tensor, ew_grid(c.N, limbs, B), dim3(TPB), 0, c.stream, A, a_cs, a_ps, Bt, b_cs, b_ps, parts, oz, so,
           limbs, c.d_primes, (int)c.N, accumulate ? 1 : 0);
    check_launch();
  }
}

void tensor_ptrs(const Ctx& c, const u64* const* a, size_t a_cs, size_t a_ps, const u64* const* b, size_t b_cs,
                 size_t b_ps, int parts, u64* o, size_t so, int n, int limbs) {
  tensor_ptrs(c, a, a_cs, a_ps, b, b_cs, b_ps, parts, o, so, n, limbs, false);
}

void tensor(const Ctx& c, const u64* a, size_t sa, int a_div, size_t a_cs, const u64* b, size_t sb,
            int b_mod, size_t b_cs, u64* o, size_t so, int B, int limbs, bool accumulate, int parts, size_t a_ps,
            size_t b_ps) {
  if (a_div < 1 || b_mod < 1 || parts < 1) BM_THROW(BM_EINVAL, "launch check: tensor batch divisors");
  std::vector<const u64*> av(B), bv(B);
  for (int z = 0; z < B; ++z) {
    av[z] = a + (size_t)(z / a_div) * sa;
    bv[z] = b + (size_t)(z % b_mod) * sb;
  }
  tensor_ptrs(c, av.data(), a_cs, a_ps, bv.data(), b_cs, b_ps, parts, o, so, B, limbs, accumulate);
}

void automorphism(const Ctx& c, const u64* in, size_t si, u64* out, size_t so, int B, int rows,
                  u64 g0, u64 g1, int sel) {
  chk(in, B, si, 0, (size_t)rows * c.N, "automorphism in");
  chk(out, B, so, 0, (size_t)rows * c.N, "automorphism out");
  const u64 gm = c.ci ? 3 : 1;   // Galois elements are 1 mod M/N
  if ((g0 & gm) != 1 || (g1 & gm) != 1 || g0 >= c.M || g1 >= c.M)
    BM_THROW(BM_EINVAL, "launch check: Galois element");
  Prof pf(c, "k_automorphism", 16.0 * c.N * B * rows, 0.0);
  LAUNCH(k_automorphism, ew_grid(c.N, rows, B), dim3(TPB), 0, c.stream, in, si, out, so, g0, g1,
         sel, c.log_n, c.ci ? 2 : 1);
  check_launch();
}

void modup(const Ctx& c, const u64* xc, size_t sx, u64* y, size_t sy, int B, int limbs) {
  if (limbs < 1 || limbs > c.L + 1) BM_THROW(BM_EINVAL, "launch check: modup level");
  const ModUpTable& tb = c.h_modup[limbs];
  chk(xc, B, sx, 0, (size_t)limbs * c.N, "modup input");
  chk(y, B, sy, 0, (size_t)tb.beta * tb.ext * c.N, "modup output");
  double ops = 0, rd = 0;
  for (int j = 0; j < tb.beta; ++j) {
    const int ns = tb.d[j].nsrc;
    ops += (double)ns * (1 + tb.ext - ns);
    rd += ns;
  }
  Prof pf(c, "k_modup", 8.0 * c.N * B * (rd + tb.npairs), ops * c.N * B);
  LAUNCH(k_modup, ew_grid(c.N, tb.npairs, B), dim3(TPB), 0, c.stream, xc, sx, y, sy, c.d_modup + limbs,
         c.d_primes, (int)c.N);
  check_launch();
}

void kip_rows(const Ctx& c, const u64* y, size_t sy, const u64* y_own, size_t sown, const u64* key0,
              const u64* key1, int sel, u64* uw, size_t suw, int B, int limbs, int inv_from, const u64* dadd,
              size_t sd, size_t dcs) {
  const ModUpTable& tb = c.h_modup[limbs];
  if (!fused_ok(c) || c.ci) BM_THROW(BM_EINVAL, "launch check: row-pass key inner product needs N = 2^16");
  if (limbs < 1 || limbs > c.L + 1 || inv_from < 0 || inv_from > tb.ext)
    BM_THROW(BM_EINVAL, "launch check: row-pass kip level");
  if (tb.beta < 1 || tb.beta > HOIST_BETA) BM_THROW(BM_EINVAL, "launch check: digits of the row-pass kip");
  if (B <= 0) return;
  chk(y, B, sy, 0, (size_t)tb.beta * tb.ext * c.N, "row-pass kip digits");
  chk(y_own, B, sown, 0, (size_t)limbs * c.N, "row-pass kip input");
  chk(key0, 1, 0, 0, (size_t)2 * tb.beta * (c.L + 1 + c.K) * c.N, "row-pass kip key");
  chk(key1, 1, 0, 0, (size_t)2 * tb.beta * (c.L + 1 + c.K) * c.N, "row-pass kip key");
  chk(uw, B, suw, 0, (size_t)2 * tb.ext * c.N, "row-pass kip output");
  u64 pm = 0;
  if (dadd) {   // P mod q_{limbs-1}
    chk(dadd, B, sd, 0, dcs + (size_t)limbs * c.N, "row-pass kip addend");
    const u64 ql = c.primes[limbs - 1].q;
    pm = 1;
    for (int k = 0; k < c.K; ++k) pm = h_mulmod(pm, c.primes[c.pid_special(k)].q % ql, ql);
  }
  // geometry of the row passes: vz elements x R rows per block
  const int V = row_views(c);
  const int vz = B < V ? B : V;
  const size_t view_words = 256 + 16;
  auto lds = [&](int r) { return ((size_t)vz * r * view_words + (size_t)2 * 512 * r) * sizeof(double); };
  int R = 1;
  while (vz * R * 2 <= V && lds(2 * R) <= 65536) R *= 2;
  const dim3 grid((unsigned)(c.N / 256 / R), (unsigned)tb.ext, (unsigned)((B + vz - 1) / vz));
  const double elems = (double)c.N * tb.ext * B;
  // distinct words: digits (pairs) and input once, keys once, both outputs
  Prof pf(c, "k_kip_rows",
          8.0 * ((double)c.N * B * (tb.npairs + limbs) + 2.0 * tb.beta * tb.ext * c.N * (key0 == key1 ? 1 : 2) +
                 2.0 * elems),
          0.5 * c.N * 8 * ((double)tb.npairs * B + 2.0 * (tb.ext - inv_from) * B) + 2.0 * elems * tb.beta);
  LAUNCH(k_kip_rows, grid, dim3(16 * vz * R), lds(R), c.stream, y, sy, y_own, sown, key0, key1, sel, uw, suw,
         c.d_modup + limbs, c.L + 1 + c.K, c.L + 1, c.d_primes, c.d_twf, c.d_twq, c.d_itwf, c.d_itwq, B, vz, dadd,
         sd, dcs, (double)pm, inv_from);
  check_launch();
}

void kip(const Ctx& c, const u64* y, size_t sy, const u64* y_own, size_t sown, const u64* key0,
         const u64* key1, int sel, u64* uw, size_t suw, int B, int limbs, const u64* dadd, size_t sd, size_t dcs) {
  const ModUpTable& tb = c.h_modup[limbs];
  if (limbs < 1 || limbs > c.L + 1) BM_THROW(BM_EINVAL, "launch check: kip level");
  chk(y, B, sy, 0, (size_t)tb.beta * tb.ext * c.N, "kip digits");
  chk(y_own, B, sown, 0, (size_t)limbs * c.N, "kip input");
  chk(key0, 1, 0, 0, (size_t)2 * tb.beta * (c.L + 1 + c.K) * c.N, "kip key");
  chk(key1, 1, 0, 0, (size_t)2 * tb.beta * (c.L + 1 + c.K) * c.N, "kip key");
  chk(uw, B, suw, 0, (size_t)2 * tb.ext * c.N, "kip output");
  Prof pf(c, "k_kip", 8.0 * c.N * tb.ext * ((double)B * tb.beta + 2.0 * tb.beta + 2.0 * B),
          2.0 * c.N * tb.ext * tb.beta * B);
  u64 pm = 0, pms = 0;
  if (dadd) {   // P mod q_{limbs-1}
    chk(dadd, B, sd, 0, dcs + (size_t)limbs * c.N, "kip addend");
    const u64 ql = c.primes[limbs - 1].q;
    pm = 1;
    for (int k = 0; k < c.K; ++k) pm = h_mulmod(pm, c.primes[c.pid_special(k)].q % ql, ql);
    pms = h_shoup(pm, ql);
  }
  LAUNCH(k_kip, ew_grid(c.N, tb.ext, B), dim3(TPB), 0, c.stream, y, sy, y_own, sown, key0, key1, sel,
         uw, suw, c.d_modup + limbs, c.L + 1 + c.K, c.L + 1, c.d_primes, (int)c.N, dadd, sd, dcs, pm, pms);
  check_launch();
}

bool kip_hoist_mask(const Ctx& c, const u64* y, size_t sy, const u64* x, size_t sx, size_t xcs,
                    const u64* const* gtab, const std::vector<std::vector<uint32_t>>& parts,
                    const std::vector<const u64*>& keys, const u64* masks, u64* uw, size_t suw, u64* ad,
                    size_t sad, int nq, int limbs, bool dadd, bool inv_rows) {
  const ModUpTable& tb = c.h_modup[limbs];
  const int k = (int)parts.size();
  if (limbs < 2 || limbs > c.L + 1) BM_THROW(BM_EINVAL, "launch check: masked kip level");
  if (nq < 1 || k < 2 || k > 16) BM_THROW(BM_EINVAL, "launch check: masked kip parts");
  if (tb.beta < 1 || tb.beta > HOIST_BETA) BM_THROW(BM_EINVAL, "launch check: digits of the masked kip");
  // distinct Galois elements and the parts that use each
  HoistArgs h{};
  MaskUse mu{};
  const size_t k1 = parts[0].size();
  if (k1 < 1 || (size_t)k * k1 > HOIST_MAX) BM_THROW(BM_EINVAL, "launch check: masked kip amounts");
  for (int i = 0; i < k; ++i) {
    if (parts[i].size() != k1) BM_THROW(BM_EINVAL, "launch check: masked kip amount lists");
    for (size_t n = 0; n < k1; ++n) {
      const uint32_t g = parts[i][n];
      int a = 0;
      while (a < h.A && h.g[a] != g) ++a;
      if (a == h.A) h.g[h.A++] = g;
      mu.parts[a] = (uint16_t)(mu.parts[a] | (1u << i));
    }
  }
  const int E = nq * k, ml = c.L + 1 + c.K;
  chk(y, nq, sy, 0, (size_t)tb.beta * tb.ext * c.N, "masked kip digits");
  chk(x, nq, sx, 0, xcs + (size_t)limbs * c.N, "masked kip input");
  chk(gtab, 1, 0, 0, c.M / 2, "key table");
  for (const u64* key : keys) chk(key, 1, 0, 0, (size_t)2 * tb.beta * (c.L + 1 + c.K) * c.N, "masked kip key");
  chk(masks, 1, 0, 0, (size_t)k * ml * c.N, "masked kip masks");
  chk(uw, E, suw, 0, (size_t)2 * tb.ext * c.N, "masked kip output");
  chk(ad, E, sad, 0, (size_t)2 * limbs * c.N, "masked kip addends");
  u64 pm = 0;
  if (dadd) {   // P mod q_{limbs-1}
    const u64 ql = c.primes[limbs - 1].q;
    pm = 1;
    for (int kk = 0; kk < c.K; ++kk) pm = h_mulmod(pm, c.primes[c.pid_special(kk)].q % ql, ql);
  }
  // distinct words: the keys once over the extended limbs, the digits and
  // query limbs once, the masks once, both outputs and the addends
  const int PG = k == 2 ? 2 : 4, ngr = (k + PG - 1) / PG;
  Prof pf(c, "k_kip_hoist_mask<" + std::to_string(tb.beta) + ", " + std::to_string(PG) + ">",
          8.0 * ((double)h.A * 2 * tb.beta * tb.ext * c.N + (double)c.N * tb.ext * nq * tb.beta +
                 2.0 * c.N * limbs * nq + (double)k * ml * c.N + 2.0 * c.N * tb.ext * E + 2.0 * c.N * limbs * E),
          2.0 * c.N * tb.ext * nq * ((double)h.A * tb.beta + (double)k * k1) + (double)c.N * limbs * E * (k1 + 2));
  const size_t gx = (c.N + TPB - 1) / TPB;
  const size_t WB = gx * tb.ext * (size_t)nq * ngr;   // the chain slots' threads form the addends too
  if (WB > 0x7fffffff) BM_THROW(BM_EINVAL, "launch check: masked kip grid");
  // the last chain limb and the special limbs (those the fused ModDown and
  // rescale transform back) leave in their inverse row pass: a key-sum
  // block's 256 positions are one row at N = 2^16
  const bool inv = inv_rows && dadd && fused_ok(c) && !c.ci;
  const int inv_from = inv ? limbs - 1 : tb.ext;
  const size_t mlds = inv ? ((size_t)PG * 2 * (256 + 16) + 512) * sizeof(double) : 0;
#define KIP_MASK(BETA, PGV)                                                                                          \
  LAUNCH((k_kip_hoist_mask<BETA, PGV>), dim3((unsigned)WB), dim3(TPB), mlds, c.stream, y, sy, x, sx, xcs, gtab, h, \
         mu, masks, ml, uw, suw, ad, sad, c.d_modup + limbs, c.L + 1 + c.K, c.L + 1, c.d_primes, c.log_n,          \
         c.ci ? 2 : 1, nq, k, dadd ? 1 : 0, (double)pm, c.d_itwf, c.d_itwq, inv_from)
  switch (tb.beta * 10 + PG) {
    case 12: KIP_MASK(1, 2); break;
    case 14: KIP_MASK(1, 4); break;
    case 22: KIP_MASK(2, 2); break;
    case 24: KIP_MASK(2, 4); break;
    case 32: KIP_MASK(3, 2); break;
    case 34: KIP_MASK(3, 4); break;
    case 42: KIP_MASK(4, 2); break;
    default: KIP_MASK(4, 4); break;
  }
#undef KIP_MASK
  check_launch();
  return inv;
}

bool kip_hoist(const Ctx& c, const u64* y, size_t sy, const u64* y_own, size_t sown, const u64* const* gtab,
               const HoistArgs& h, const std::vector<const u64*>& keys, u64* uw, size_t suw, const u64* c0_in,
               size_t c0_si, u64* c0_out, size_t c0_so, int B, int limbs, bool accumulate, bool inv_special) {
  const ModUpTable& tb = c.h_modup[limbs];
  if (limbs < 1 || limbs > c.L + 1) BM_THROW(BM_EINVAL, "launch check: kip level");
  const int lists = h.per_elem ? std::min(B, h.mod) : 1;   // amount lists in h.g
  if (h.A < 1 || h.mod < 1 || h.A * lists > HOIST_MAX) BM_THROW(BM_EINVAL, "launch check: hoisted amounts");
  chk(y, B, sy, 0, (size_t)tb.beta * tb.ext * c.N, "hoisted kip digits");
  chk(y_own, B, sown, 0, (size_t)limbs * c.N, "hoisted kip input");
  chk(gtab, 1, 0, 0, c.M / 2, "key table");
  for (const u64* key : keys) chk(key, 1, 0, 0, (size_t)2 * tb.beta * (c.L + 1 + c.K) * c.N, "hoisted kip key");
  chk(uw, B, suw, 0, (size_t)2 * tb.ext * c.N, "hoisted kip output");
  chk(c0_in, B, c0_si, 0, (size_t)limbs * c.N, "autom_sum input");
  chk(c0_out, B, c0_so, 0, (size_t)limbs * c.N, "autom_sum output");
  if (tb.beta < 1 || tb.beta > HOIST_BETA) BM_THROW(BM_EINVAL, "launch check: digits of the hoisted kip");
  // algorithmic words: every distinct key of the launch once (over the
  // extended limbs), the digits and the input limbs once, both outputs, and
  // the c0 half (gathered sum of the rotations) that rides in the same launch
  std::vector<uint32_t> gs;
  for (int i = 0; i < h.A * lists; ++i) gs.push_back(h.g[i]);
  std::sort(gs.begin(), gs.end());
  const double distinct_keys = (double)(std::unique(gs.begin(), gs.end()) - gs.begin());
  const double keys_read = distinct_keys * 2 * tb.beta * tb.ext * c.N;
  const bool grouped = !h.per_elem && B > 1 && c.N % (2 * TPB) == 0;
  // shared amounts: ZB elements per thread (each key word loaded once, used
  // ZB times) and CH amounts' words requested per chunk; variant 0 is the
  // default of each digit count (two elements a thread measured best at the
  // face configuration), the others are the autotuner's alternatives
  static const int zb_tab[5][5] = {{0}, {2, 1, 3, 2, 4}, {2, 1, 3, 2, 2}, {2, 1, 2, 2, 2}, {2, 1, 2, 2, 2}};
  static const int ch_tab[5][5] = {{0}, {4, 4, 4, 2, 2}, {2, 2, 2, 1, 2}, {1, 1, 1, 1, 1}, {1, 1, 1, 1, 1}};
  const int var = c.kip_variant >= 0 && c.kip_variant < 5 ? c.kip_variant : 0;
  const int ZB = zb_tab[tb.beta][var], CH = ch_tab[tb.beta][var];
  const std::string pname = grouped ? "k_kip_hoist_zb<" + std::to_string(tb.beta) + ", " + std::to_string(ZB) + ", " +
                                          std::to_string(CH) + ">"
                                    : "k_kip_hoist<" + std::to_string(tb.beta) + ">";
  Prof pf(c, pname,
          8.0 * (keys_read + (double)c.N * tb.ext * B * (tb.beta + 2) + 2.0 * c.N * limbs * B),
          2.0 * c.N * tb.ext * tb.beta * B * h.A);
  const size_t gx = (c.N + TPB - 1) / TPB;
  AutomArgs am{c0_in, c0_si, c0_out, c0_so, limbs, (int)(gx * limbs * B)};
  if (am.W % 8 != 0) BM_THROW(BM_EINVAL, "launch check: autom_sum grid");
  if (grouped) {
    const size_t Wz = (c.N / (2 * TPB)) * tb.ext * (size_t)((B + ZB - 1) / ZB);
    // the chain slots' blocks form the c0 half themselves (no blocks of its own)
    am.W = 0;
    if (Wz % 8 != 0 || Wz > 0x7fffffff) BM_THROW(BM_EINVAL, "launch check: hoisted kip grid");
    // the special limbs leave in their inverse row pass (two whole rows a
    // block at N = 2^16; a single launch, not an accumulating one)
    const bool inv = inv_special && fused_ok(c) && !c.ci && !accumulate;
    const int inv_from = inv ? limbs : tb.ext;
    const size_t zlds = inv ? ((size_t)ZB * 4 * (256 + 16) + 1024) * sizeof(double) : 0;
#define KIP_HOIST_ZB(BETA, ZB_, CH_)                                                                             \
  LAUNCH((k_kip_hoist_zb<BETA, ZB_, CH_>), dim3((unsigned)(Wz + am.W)), dim3(TPB), zlds, c.stream, y, sy, y_own,    \
         sown, gtab, h, uw, suw, c.d_modup + limbs, c.L + 1 + c.K, c.L + 1, c.d_primes, c.log_n, c.ci ? 2 : 1, B, \
         accumulate ? 1 : 0, am, c.kip_order, c.d_itwf, c.d_itwq, inv_from)
    const int code = tb.beta * 100 + ZB * 10 + CH;
    switch (code) {
      case 124: KIP_HOIST_ZB(1, 2, 4); break;
      case 114: KIP_HOIST_ZB(1, 1, 4); break;
      case 134: KIP_HOIST_ZB(1, 3, 4); break;
      case 122: KIP_HOIST_ZB(1, 2, 2); break;
      case 142: KIP_HOIST_ZB(1, 4, 2); break;
      case 222: KIP_HOIST_ZB(2, 2, 2); break;
      case 212: KIP_HOIST_ZB(2, 1, 2); break;
      case 232: KIP_HOIST_ZB(2, 3, 2); break;
      case 221: KIP_HOIST_ZB(2, 2, 1); break;
      case 321: KIP_HOIST_ZB(3, 2, 1); break;
      case 311: KIP_HOIST_ZB(3, 1, 1); break;
      case 421: KIP_HOIST_ZB(4, 2, 1); break;
      case 411: KIP_HOIST_ZB(4, 1, 1); break;
      default: BM_THROW(BM_EINVAL, "launch check: hoisted kip variant");
    }
#undef KIP_HOIST_ZB
    check_launch();
    return inv;
  }
  const size_t W = gx * tb.ext * B;
  if (W % 8 != 0 || W + am.W > 0x7fffffff) BM_THROW(BM_EINVAL, "launch check: hoisted kip grid");
#define KIP_HOIST(BETA)                                                                                        \
  LAUNCH(k_kip_hoist<BETA>, dim3((unsigned)(W + am.W)), dim3(TPB), 0, c.stream, y, sy, y_own, sown, gtab, h, uw, \
         suw, c.d_modup + limbs, c.L + 1 + c.K, c.L + 1, c.d_primes, c.log_n, c.ci ? 2 : 1, B, accumulate ? 1 : 0, am)
  switch (tb.beta) {
    case 1: KIP_HOIST(1); break;
    case 2: KIP_HOIST(2); break;
    case 3: KIP_HOIST(3); break;
    default: KIP_HOIST(4); break;
  }
#undef KIP_HOIST
  check_launch();
  return false;
}

void moddown_conv(const Ctx& c, const u64* uw, size_t suw, u64* conv, size_t sc, int B, int limbs) {
  chk(uw, B, suw, 0, (size_t)2 * (limbs + c.K) * c.N, "moddown_conv input");
  chk(conv, B, sc, 0, (size_t)2 * limbs * c.N, "moddown_conv output");
  Prof pf(c, "k_moddown_conv", 8.0 * c.N * B * (2 * c.K + 2 * limbs),
          (double)c.N * B * (2 * c.K + 2 * c.K * limbs));
  LAUNCH(k_moddown_conv, ew_grid(c.N, 2 * limbs, B), dim3(TPB), 0, c.stream, uw, suw,
                     conv, sc, c.d_moddown, limbs, c.d_primes, (int)c.N);
  check_launch();
}

void moddown_finish(const Ctx& c, const u64* uw, size_t suw, const u64* conv, size_t sc,
                    const u64* add0, size_t sadd0, const u64* add1, size_t sadd1, u64* out,
                    size_t so, int B, int limbs) {
  chk(uw, B, suw, 0, (size_t)2 * (limbs + c.K) * c.N, "moddown_finish input");
  chk(conv, B, sc, 0, (size_t)2 * limbs * c.N, "moddown_finish conv");
  if (add0) chk(add0, B, sadd0, 0, (size_t)limbs * c.N, "moddown_finish add0");
  if (add1) chk(add1, B, sadd1, 0, (size_t)limbs * c.N, "moddown_finish add1");
  chk(out, B, so, 0, (size_t)2 * limbs * c.N, "moddown_finish output");
  Prof pf(c, "k_moddown_finish", 8.0 * c.N * B * 2 * limbs * (3 + (add0 ? 1 : 0)),
          2.0 * c.N * B * limbs);
  LAUNCH(k_moddown_finish, ew_grid(c.N, 2 * limbs, B), dim3(TPB), 0, c.stream, uw, suw,
                     conv, sc, add0, sadd0, add1, sadd1, out, so, c.d_moddown, limbs, c.d_primes,
                     (int)c.N);
  check_launch();
}

void rescale_conv(const Ctx& c, const u64* last, size_t sl, size_t last_comp_stride, u64* t,
                  size_t st, int B, int comps, int limbs) {
  if (limbs < 2) BM_THROW(BM_EINVAL, "launch check: rescale limbs");
  chk(last, B, sl, 0, (size_t)(comps - 1) * last_comp_stride + c.N, "rescale_conv input");
  chk(t, B, st, 0, (size_t)comps * (limbs - 1) * c.N, "rescale_conv output");
  Prof pf(c, "k_rescale_conv", 8.0 * c.N * B * comps * limbs, (double)c.N * B * comps * (limbs - 1));
  LAUNCH(k_rescale_conv, ew_grid(c.N, comps * (limbs - 1), B), dim3(TPB), 0, c.stream,
                     last, sl, last_comp_stride, t, st, comps, limbs, c.d_primes, (int)c.N);
  check_launch();
}

void rescale_finish(const Ctx& c, const u64* in, size_t si, const u64* t, size_t st, u64* out,
                    size_t so, int B, int comps, int limbs) {
  if (limbs < 2 || limbs > c.L + 1) BM_THROW(BM_EINVAL, "launch check: rescale limbs");
  chk(in, B, si, 0, (size_t)comps * limbs * c.N, "rescale_finish input");
  chk(t, B, st, 0, (size_t)comps * (limbs - 1) * c.N, "rescale_finish t");
  chk(out, B, so, 0, (size_t)comps * (limbs - 1) * c.N, "rescale_finish output");
  Prof pf(c, "k_rescale_finish", 24.0 * c.N * B * comps * (limbs - 1), (double)c.N * B * comps * (limbs - 1));
  LAUNCH(k_rescale_finish, ew_grid(c.N, comps * (limbs - 1), B), dim3(TPB), 0,
                     c.stream, in, si, t, st, out, so, c.d_rescale, comps, limbs, c.L + 1,
                     c.d_primes, (int)c.N);
  check_launch();
}

void copy_limbs(const Ctx& c, const u64* in, size_t si, size_t in_comp_stride, u64* out, int div,
                size_t so_hi, size_t so_lo, size_t out_comp_stride, int B, int comps, int limbs, u64** ref,
                u64* ref_val) {
  if (div < 1) BM_THROW(BM_EINVAL, "launch check: copy divisor");
  if (ref) chk(ref, 1, 0, 0, 1, "copy_limbs reference word");
  chk(in, B, si, 0, (size_t)(comps - 1) * in_comp_stride + (size_t)limbs * c.N, "copy_limbs input");
  {
    const size_t hi = (size_t)((B - 1) / div) * so_hi + (size_t)std::min(B - 1, div - 1) * so_lo;
    chk(out, 1, 0, 0, hi + (size_t)(comps - 1) * out_comp_stride + (size_t)limbs * c.N, "copy_limbs output");
  }
  Prof pf(c, "k_copy_limbs", 16.0 * c.N * B * comps * limbs, 0.0);
  LAUNCH(k_copy_limbs, ew_grid(c.N, comps * limbs, B), dim3(TPB), 0, c.stream, in, si,
                     in_comp_stride, out, div, so_hi, so_lo, out_comp_stride, limbs, (int)c.N, ref, ref_val);
  check_launch();
}

void copy_ptrs(const Ctx& c, const u64* in, size_t si, size_t ics, u64* const* out, size_t ocs, int n,
               int comps, int limbs) {
  chk(in, n, si, 0, (size_t)(comps - 1) * ics + (size_t)limbs * c.N, "copy_ptrs input");
  for (int z0 = 0; z0 < n; z0 += PTR_MAX) {
    const int B = std::min(PTR_MAX, n - z0);
    OutTab o{};
    for (int z = 0; z < B; ++z) {
      o.p[z] = out[z0 + z];
      chk(o.p[z], 1, 0, 0, (size_t)(comps - 1) * ocs + (size_t)limbs * c.N, "copy_ptrs output");
    }
    Prof pf(c, "k_copy_ptrs", 16.0 * c.N * B * comps * limbs, 0.0);
    LAUNCH(k_copy_ptrs, ew_grid(c.N, comps * limbs, B), dim3(TPB), 0, c.stream, in + (size_t)z0 * si, si, ics, o,
           ocs, limbs, (int)c.N);
    check_launch();
  }
}

void zero(const Ctx& c, u64* out, size_t words) {
  if (words == 0) return;
  chk(out, 1, 0, 0, words, "zero output");
  Prof pf(c, "k_zero", 8.0 * words, 0.0);
  const size_t blocks = std::min<size_t>((words + TPB * 4 - 1) / (TPB * 4), 65535);
  LAUNCH(k_zero, dim3((unsigned)blocks), dim3(TPB), 0, c.stream, out, words);
  check_launch();
}

void move_idx(const Ctx& c, const u64* in, size_t si, u64* out, size_t so, const uint32_t* idx_dev,
              uint32_t max_idx, bool scatter, int B, size_t words) {
  if (B <= 0 || words == 0) return;
  chk(in, scatter ? B : (int)max_idx + 1, si, 0, words, "move_idx input");
  chk(out, scatter ? (int)max_idx + 1 : B, so, 0, words, "move_idx output");
  chk(idx_dev, 1, 0, 0, ((size_t)B + 1) / 2, "move_idx index list");
  Prof pf(c, "k_move_idx", 16.0 * words * B, 0.0);
  const size_t blocks = std::min<size_t>((words + TPB * 4 - 1) / (TPB * 4), 65535);
  LAUNCH(k_move_idx, dim3((unsigned)blocks, 1, (unsigned)B), dim3(TPB), 0, c.stream, in, si, out, so, idx_dev,
         scatter ? 1 : 0, words);
  check_launch();
}

}  // namespace kern
}  // namespace bm
