// encoder.cpp -- CKKS canonical-embedding encode/decode on the host.
//
// Slot j corresponds to the root zeta^(5^j mod 2N), zeta = exp(i pi / N);
// the conjugate root carries the conjugate value.  With all N odd-power
// roots zeta^(2t+1) indexed by t, both directions are one length-N complex
// FFT plus a twist by zeta^(+-k).
#include <cmath>
#include <complex>
#include <vector>

#include "bm_internal.hpp"

namespace bm {
namespace {

using cd = std::complex<double>;

// iterative radix-2 FFT, sign = -1: X[k] = sum x[t] e^{-2 pi i t k / n}
void fft(std::vector<cd>& a, int sign) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    const double ang = sign * 2.0 * M_PI / (double)len;
    std::vector<cd> w(len / 2);
    for (size_t k = 0; k < len / 2; ++k) w[k] = cd(std::cos(ang * k), std::sin(ang * k));
    for (size_t i = 0; i < n; i += len)
      for (size_t k = 0; k < len / 2; ++k) {
        cd u = a[i + k], v = a[i + k + len / 2] * w[k];
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
  }
}

void slot_roots(size_t N, std::vector<size_t>& ts, std::vector<size_t>& tc) {
  const size_t n = N / 2, twoN = 2 * N;
  ts.resize(n);
  tc.resize(n);
  size_t e = 1;
  for (size_t j = 0; j < n; ++j) {
    ts[j] = (e - 1) / 2;
    tc[j] = (twoN - e - 1) / 2;
    e = e * 5 % twoN;
  }
}

}  // namespace

void encode_slots(size_t N, const double* re, const double* im, double scale, int64_t* out) {
  std::vector<size_t> ts, tc;
  slot_roots(N, ts, tc);
  std::vector<cd> full(N, cd(0, 0));
  for (size_t j = 0; j < N / 2; ++j) {
    cd z(scale * re[j], im ? scale * im[j] : 0.0);
    full[ts[j]] = z;
    full[tc[j]] = std::conj(z);
  }
  fft(full, -1);
  for (size_t k = 0; k < N; ++k) {
    const double ang = -M_PI * (double)k / (double)N;
    double x = (full[k] * cd(std::cos(ang), std::sin(ang))).real() / (double)N;
    double r = std::floor(std::fabs(x) + 0.5);
    out[k] = (int64_t)(x < 0 ? -r : r);
  }
}

void decode_coeffs(size_t N, const double* m, double scale, double* re, double* im) {
  std::vector<size_t> ts, tc;
  slot_roots(N, ts, tc);
  std::vector<cd> a(N);
  for (size_t k = 0; k < N; ++k) {
    const double ang = M_PI * (double)k / (double)N;
    a[k] = m[k] * cd(std::cos(ang), std::sin(ang));
  }
  fft(a, +1);
  for (size_t j = 0; j < N / 2; ++j) {
    cd z = a[ts[j]] / scale;
    re[j] = z.real();
    if (im) im[j] = z.imag();
  }
}

// Conjugate-invariant ring R' = Z[X + X^-1] of rank N: an element is kept as
// its first N coefficients in Z[X]/(X^2N+1), the rest following from
// a(X^-1) = a(X) (c_N = 0, c_{2N-k} = -c_k).  The canonical embedding of
// Z[X]/(X^2N+1) with real slot values (slot j at zeta^(5^j), zeta of order
// 4N) produces exactly such coefficients, so encoding runs at dimension 2N
// and keeps the first N; decoding extends and takes the real parts.
void ring_encode(const Ctx& c, const double* slots, double scale, int64_t* out) {
  if (!c.ci) {
    encode_slots(c.N, slots, nullptr, scale, out);
    return;
  }
  std::vector<int64_t> full(2 * c.N);
  encode_slots(2 * c.N, slots, nullptr, scale, full.data());
  std::copy(full.begin(), full.begin() + c.N, out);
}

void ring_decode(const Ctx& c, const double* m, double scale, double* slots) {
  if (!c.ci) {
    decode_coeffs(c.N, m, scale, slots, nullptr);
    return;
  }
  const size_t N = c.N;
  std::vector<double> full(2 * N, 0.0);
  for (size_t k = 0; k < N; ++k) full[k] = m[k];
  for (size_t k = 1; k < N; ++k) full[2 * N - k] = -m[k];
  decode_coeffs(2 * N, full.data(), scale, slots, nullptr);
}

}  // namespace bm
