// fp64_check.cpp -- host build of the library's FP64 modular arithmetic
// (paper_2408_06167_amd/csrc/fp64_modarith.hpp), driven by
// tests/test_fp64_arith.py against exact Python integers.  Test
// infrastructure: built by that test into a temporary directory, never
// linked into the library.
#include <cmath>
#include <cstddef>
#include <cstdint>

#include "../../paper_2408_06167_amd/csrc/fp64_modarith.hpp"

using namespace bm::fpm;

extern "C" {

void chk_fmul_mod(const double* a, const double* w, const double* wq, size_t n, double q, double* out) {
  for (size_t i = 0; i < n; ++i) out[i] = fmul_mod(a[i], w[i], wq[i], q);
}

void chk_fmul_mod_q(const double* a, const double* w, size_t n, double qi, double q, double* out) {
  for (size_t i = 0; i < n; ++i) out[i] = fmul_mod_q(a[i], w[i], qi, q);
}

void chk_fred(const double* a, size_t n, double qi, double q, double* out) {
  for (size_t i = 0; i < n; ++i) out[i] = fred(a[i], qi, q);
}

void chk_u64_to_f(const uint64_t* v, size_t n, double* out) {
  for (size_t i = 0; i < n; ++i) out[i] = u64_to_f(v[i]);
}

void chk_f_to_u64(const double* x, size_t n, uint64_t* out) {
  for (size_t i = 0; i < n; ++i) out[i] = f_to_u64(x[i]);
}

// FAcc over n products v[i] w[i]; *maxabs receives the largest |s| the
// accumulator held
uint64_t chk_facc(const double* v, const double* w, size_t n, double qi, double q, double* maxabs) {
  FAcc acc;
  double m = 0.0;
  for (size_t i = 0; i < n; ++i) {
    acc.add(v[i], w[i], qi, q);
    m = std::fmax(m, std::fabs(acc.s));
  }
  *maxabs = m;
  return acc.residue(qi, q);
}

// one radix-16 phase on x[16] in place; tw[(k * 16 + j) * 2 + {0, 1}] is the
// twiddle of word j at stage k and fl(w / q); *maxabs receives the largest
// |x| after any stage
void chk_phase(double* x16, const double* tw, int fold_first, int inverse, double qi, double q,
               double* maxabs) {
  double x[16];
  for (int j = 0; j < 16; ++j) x[j] = x16[j];
  double m = 0.0;
  // the twiddle callback runs before every butterfly, so it sees every value
  // the phase produces as it is produced
  auto twid = [&](int k, int j, double& w, double& wq) {
    for (int t = 0; t < 16; ++t) m = std::fmax(m, std::fabs(x[t]));
    w = tw[(k * 16 + j) * 2];
    wq = tw[(k * 16 + j) * 2 + 1];
  };
  if (inverse)
    gs_phase16(x, fold_first != 0, qi, q, twid);
  else
    ct_phase16(x, fold_first != 0, qi, q, twid);
  for (int t = 0; t < 16; ++t) m = std::fmax(m, std::fabs(x[t]));
  *maxabs = m;
  for (int j = 0; j < 16; ++j) x16[j] = x[j];
}

uint64_t chk_residue(double a, double qi, double q) { return residue(a, qi, q); }

// a sum of n products v[i] w[i] folded after every fold_period(q)-th
// product, as the key inner products of the kernels fold; *maxabs receives
// the largest |s| the sum held
uint64_t chk_fsum_period(const double* v, const double* w, size_t n, double qi, double q, double* maxabs) {
  const int per = fold_period(q);
  double s = 0.0, m = 0.0;
  for (size_t i = 0; i < n; ++i) {
    s = s + fmul_mod_q(v[i], w[i], qi, q);
    m = std::fmax(m, std::fabs(s));
    if ((int)((i + 1) % per) == 0) s = fred(s, qi, q);
  }
  *maxabs = m;
  return residue(s, qi, q);
}

int chk_fold_period(double q) { return fold_period(q); }

}  // extern "C"
