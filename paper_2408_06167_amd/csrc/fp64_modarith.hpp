// fp64_modarith.hpp -- exact modular arithmetic on residues carried in FP64.
//
// The NTT passes, the key inner products and the tensor hold residues of
// primes q < 2^51 as exact integers in doubles (the CDNA4 VALU issues FP64
// FMA at one operation per lane per clock, 32-bit integer multiplies at about
// half of that).  Every function here is an error-free transformation: as
// long as the stated magnitude bounds hold, each result is an integer below
// 2^53 congruent to the modular definition, so the words the kernels store are
// the exact residues.  The functions are __host__ __device__ so that the same
// code can be driven on the CPU against exact integer arithmetic at the
// extremes of the bounds.  Each operation is written as one IEEE operation
// (contraction into FMAs is switched off inside each body), so the host and
// the device compute the same values.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bm {
namespace fpm {

// a w mod q for a with |a| < 2^52 / 2 and 0 <= w < q < 2^51, wq = fl(w / q):
// hi = fl(a w), lo = a w - hi (one FMA, exact), qt = rint(fl(a wq)),
// r = (hi - qt q) + lo (one FMA whose exact result is an integer below 2^53,
// then an exact add).  The quotient estimate is within 0.5 + |a| 2^-52 of
// a w / q, so |r| <= q (0.5 + |a| 2^-52 (1 + 2^-52)).
__host__ __device__ __forceinline__ double fmul_mod(double a, double w, double wq, double q) {
#pragma clang fp contract(off)
  const double hi = a * w;
  const double lo = __builtin_fma(a, w, -hi);
  const double qt = __builtin_rint(a * wq);
  return __builtin_fma(-qt, q, hi) + lo;
}

// a w mod q for |a|, w < q < 2^51, quotient from fl(fl(a w) fl(1/q)): it is
// within 0.5 + 3 (a w / q) 2^-53 < 1.25 of a w / q, so |r| <= 1.25 q, and both
// the FMA (an integer below 2^53) and the final add are exact.
__host__ __device__ __forceinline__ double fmul_mod_q(double a, double w, double qi, double q) {
#pragma clang fp contract(off)
  const double hi = a * w;
  const double lo = __builtin_fma(a, w, -hi);
  const double qt = __builtin_rint(hi * qi);
  return __builtin_fma(-qt, q, hi) + lo;
}

// Products of fmul_mod_q a running sum may take between folds: each lies
// within 1.25 q of 0, within 0.875 q when q < 2^50 (the quotient error
// 0.5 + 3 (a w / q) 2^-53 is then below 0.875), and the sum starts within
// q/2 + 1 after a fold, so 2 products (q < 2^51: at most 3 q + 1) or 8
// (q < 2^50: at most 7.5 q + 1 < 2^53) keep every partial sum exact.
__host__ __device__ __forceinline__ int fold_period(double q) { return q < 1125899906842624.0 ? 8 : 2; }

// a - rint(a fl(1/q)) q for |a| < 2^53: lies in [-q/2 - 1, q/2 + 1]
__host__ __device__ __forceinline__ double fred(double a, double qi, double q) {
#pragma clang fp contract(off)
  return __builtin_fma(-__builtin_rint(a * qi), q, a);
}

// exact conversions for 0 <= v < 2^52, through the double 2^52 + v: its
// exponent field is that of 2^52 and its 52 fraction bits are v, so one OR
// and one exact subtraction give v as a double, and one exact addition and
// one AND give it back
__host__ __device__ __forceinline__ double u64_to_f(uint64_t v) {
#pragma clang fp contract(off)
  return __builtin_bit_cast(double, v | 0x4330000000000000ull) - 4503599627370496.0;
}
__host__ __device__ __forceinline__ uint64_t f_to_u64(double x) {
#pragma clang fp contract(off)
  return __builtin_bit_cast(uint64_t, x + 4503599627370496.0) & 0x000fffffffffffffull;
}

// the exact residue in [0, q) of an integer-valued double with |a| < 2^53
__host__ __device__ __forceinline__ uint64_t residue(double a, double qi, double q) {
#pragma clang fp contract(off)
  const double r = fred(a, qi, q);
  return f_to_u64(r < 0.0 ? r + q : r);
}

// Sum of exact products v * w mod q (v, w residues in [0, q)) carried in FP64:
// each product lies within 1.25 q of 0 (fmul_mod_q), the running sum is
// folded back to |s| <= q/2 + 1 after every second term, so it stays below
// 3q + 1 < 2^53; residue() returns the exact sum in [0, q).
struct FAcc {
  double s = 0.0;
  int n = 0;
  __host__ __device__ __forceinline__ void add(double v, double w, double qi, double q) {
#pragma clang fp contract(off)
    s = s + fmul_mod_q(v, w, qi, q);
    if (++n == 2) { s = fred(s, qi, q); n = 0; }
  }
  // add one product already reduced by fmul_mod
  __host__ __device__ __forceinline__ void add_f(double p, double qi, double q) {
#pragma clang fp contract(off)
    s = s + p;
    if (++n == 2) { s = fred(s, qi, q); n = 0; }
  }
  __host__ __device__ __forceinline__ uint64_t residue(double qi, double q) const {
    return fpm::residue(s, qi, q);
  }
};

// One radix-16 phase of the negacyclic NTT on the 16 words one thread holds:
// four Cooley-Tukey stages (forward) or Gentleman-Sande stages (inverse),
// stage k pairing word j with j + (8 >> k) (forward: k = 0..3; inverse:
// k = 3..0).  twid(k, j, w, wq) gives the twiddle w of the butterfly of word j
// at stage k and fl(w / q).  Values are folded back to |x| <= q/2 + 1 before
// the third stage of the phase and, with fold_first, before its first stage.
// With the product bound of fmul_mod at q < 2^51: forward (CT), from
// |x| <= q/2 + 1 two stages give at most 1.25q and then 2.375q (the
// multiplied inputs stay below 1.25q, so every product is below 1.13q); from
// [0, q) they give 2q and then 3.5q.  Inverse (GS): from q/2 + 1 two stages
// give q and then 2q; from [0, q), 2q and then 4q.  All of these stay below
// 2^53, so every operation is exact.
template <class TW>
__host__ __device__ __forceinline__ void ct_phase16(double (&x)[16], bool fold_first, double qi, double q,
                                                     TW twid) {
#pragma clang fp contract(off)
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if ((k == 0 && fold_first) || k == 2) {
#pragma unroll
      for (int j = 0; j < 16; ++j) x[j] = fred(x[j], qi, q);
    }
    const int step = 8 >> k;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (j & step) continue;
      double w, wq;
      twid(k, j, w, wq);
      const double T = fmul_mod(x[j + step], w, wq, q);
      const double U = x[j];
      x[j] = U + T;
      x[j + step] = U - T;
    }
  }
}

template <class TW>
__host__ __device__ __forceinline__ void gs_phase16(double (&x)[16], bool fold_first, double qi, double q,
                                                     TW twid) {
#pragma clang fp contract(off)
#pragma unroll
  for (int k = 3; k >= 0; --k) {
    if ((k == 3 && fold_first) || k == 1) {
#pragma unroll
      for (int j = 0; j < 16; ++j) x[j] = fred(x[j], qi, q);
    }
    const int step = 8 >> k;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (j & step) continue;
      double w, wq;
      twid(k, j, w, wq);
      const double U = x[j], V = x[j + step];
      x[j] = U + V;
      x[j + step] = fmul_mod(U - V, w, wq, q);
    }
  }
}

}  // namespace fpm
}  // namespace bm
