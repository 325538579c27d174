// host_math.cpp -- host-side number theory and table construction.
//
// The device NTT uses a primitive 2N-th root psi = g^((q-1)/2N) for a
// generator g of Z_q^*, found by factoring q-1.  Twiddles are stored in
// bit-reversed order (W[k] = psi^{brv(k)}) with Shoup companions
// floor(W[k] 2^64 / q), so a butterfly needs one 64x64-high multiply.
// Conjugate-invariant ring: the transform evaluates a polynomial reduced
// modulo X^N - zeta^N (zeta a primitive 4N-th root) at its roots
// zeta^(1 + 4 brv(i)); the same butterflies do so with twiddles
// W[2^S + B] = zeta^(2 brv(2^S + B) - N / 2^(S+1)), S = floor(log2 k).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "bm_internal.hpp"

namespace bm {

u64 h_mulmod(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }

u64 h_powmod(u64 b, u64 e, u64 q) {
  u64 r = 1 % q;
  b %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = h_mulmod(r, b, q);
    b = h_mulmod(b, b, q);
  }
  return r;
}

// extended Euclid on signed 128-bit values
u64 h_invmod(u64 a, u64 q) {
  __int128 t = 0, nt = 1, r = q, nr = a % q;
  while (nr != 0) {
    __int128 quo = r / nr, tmp;
    tmp = t - quo * nt; t = nt; nt = tmp;
    tmp = r - quo * nr; r = nr; nr = tmp;
  }
  if (r != 1) BM_THROW(BM_EINVAL, "value not invertible");
  if (t < 0) t += q;
  return (u64)t;
}

u64 h_shoup(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }

bool h_is_prime(u64 n) {
  if (n < 2) return false;
  static const u64 bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (u64 p : bases)
    if (n % p == 0) return n == p;
  u64 d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; ++s; }
  for (u64 a : bases) {
    u64 x = h_powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < s; ++i) {
      x = h_mulmod(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

// psi = g^((q-1)/2N) with g a generator: factor q-1 by trial division of its
// odd part, then test candidates g against every prime factor.
u64 h_primitive_2n_root(u64 q, size_t N) {
  u64 m = q - 1;
  std::vector<u64> fac;
  if (!(m & 1)) fac.push_back(2);
  while (!(m & 1)) m >>= 1;
  for (u64 f = 3; f * f <= m; f += 2) {
    if (m % f == 0) {
      fac.push_back(f);
      while (m % f == 0) m /= f;
    }
  }
  if (m > 1) fac.push_back(m);
  for (u64 g = 2; g < q; ++g) {
    bool gen = true;
    for (u64 f : fac)
      if (h_powmod(g, (q - 1) / f, q) == 1) { gen = false; break; }
    if (gen) return h_powmod(g, (q - 1) / (2 * N), q);
  }
  BM_THROW(BM_EINVAL, "no generator found");
}

static u32 brv(u32 x, int bits) {
  u32 r = 0;
  for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

static u64 neg_inv_2_64(u64 q) {  // -q^{-1} mod 2^64 by Newton iteration
  u64 x = q;                       // correct to 3 bits for odd q
  for (int i = 0; i < 6; ++i) x *= 2 - q * x;
  return (u64)0 - x;
}

std::vector<u64> gaussian_cdt(double sigma, int bound) {
  std::vector<long double> rho;
  long double total = 0;
  for (int x = -bound; x <= bound; ++x) {
    long double v = expl(-(long double)x * x / (2.0L * sigma * sigma));
    rho.push_back(v);
    total += v;
  }
  std::vector<u64> cdt;
  long double acc = 0;
  for (int i = 0; i < 2 * bound; ++i) {
    acc += rho[i];
    cdt.push_back((u64)floorl(ldexpl(acc / total, 64)));
  }
  return cdt;
}

static void put_pair(u64 out[2], u64 w, u64 q) {
  out[0] = w;
  out[1] = h_shoup(w, q);
}

void build_context_tables(Ctx& c) {
  const int np = c.nprimes();
  const size_t N = c.N;
  if (np > MAX_PRIMES) BM_THROW(BM_EINVAL, "too many primes");
  // ---- per-prime constants and twiddles
  std::vector<PrimeC> pc(MAX_PRIMES);
  std::vector<u64> tw(MAX_PRIMES * N), tws(MAX_PRIMES * N), itw(MAX_PRIMES * N),
      itws(MAX_PRIMES * N);
  std::vector<double> twf(MAX_PRIMES * N), twq(MAX_PRIMES * N), itwf(MAX_PRIMES * N), itwq(MAX_PRIMES * N);
  std::vector<u64> pw(N), ipw(N), ci(4 * MAX_PRIMES, 0);
  for (int i = 0; i < np; ++i) {
    const u64 q = c.primes[i].q;
    PrimeC& p = pc[i];
    std::memset(&p, 0, sizeof(p));
    p.q = q;
    p.qn = neg_inv_2_64(q);
    u64 r1 = (u64)(((u128)1 << 64) % q);
    p.r2 = h_mulmod(r1, r1, q);
    p.ninv = h_invmod(N % q, q);
    p.ninv_s = h_shoup(p.ninv, q);
    p.pad[0] = h_shoup(1, q);   // floor(2^64 / q): reduction of any 64-bit word
    if (q >= (1ULL << 51)) BM_THROW(BM_EINVAL, "primes must lie below 2^51");
    const double qd = (double)q, qinv = 1.0 / qd, niq = (double)p.ninv / qd;
    std::memcpy(&p.pad[1], &qinv, sizeof(double));
    std::memcpy(&p.pad[2], &niq, sizeof(double));
    const u64 psi = c.primes[i].psi;   // primitive M-th root
    const u64 ipsi = h_invmod(psi, q);
    const size_t E = c.ci ? 2 * N : N;  // exponents the twiddles use
    pw.resize(E);
    ipw.resize(E);
    pw[0] = ipw[0] = 1;
    for (size_t k = 1; k < E; ++k) {
      pw[k] = h_mulmod(pw[k - 1], psi, q);
      ipw[k] = h_mulmod(ipw[k - 1], ipsi, q);
    }
    if (c.ci) {
      const u64 io = h_powmod(psi, N, q), h = (q + 1) / 2;
      ci[4 * i] = io;
      ci[4 * i + 1] = h_shoup(io, q);
      ci[4 * i + 2] = h;
      ci[4 * i + 3] = h_shoup(h, q);
    }
    for (size_t k = 0; k < N; ++k) {
      u32 r = brv((u32)k, c.log_n);
      if (c.ci && k > 0) {
        int S = 31 - __builtin_clz((u32)k);
        r = 2 * r - (u32)(N >> (S + 1));
      }
      tw[i * N + k] = pw[r];
      tws[i * N + k] = h_shoup(pw[r], q);
      itw[i * N + k] = ipw[r];
      itws[i * N + k] = h_shoup(ipw[r], q);
      twf[i * N + k] = (double)pw[r];
      twq[i * N + k] = (double)pw[r] / (double)q;
      itwf[i * N + k] = (double)ipw[r];
      itwq[i * N + k] = (double)ipw[r] / (double)q;
    }
  }
  HIP_OK(dev::malloc(&c.d_primes, sizeof(PrimeC) * MAX_PRIMES));
  audit::add(c.d_primes, sizeof(PrimeC) * MAX_PRIMES);
  HIP_OK(dev::memcpy(c.d_primes, pc.data(), sizeof(PrimeC) * MAX_PRIMES, hipMemcpyHostToDevice));
  const size_t tb = sizeof(u64) * MAX_PRIMES * N;
  HIP_OK(dev::malloc(&c.d_tw, tb));
  HIP_OK(dev::malloc(&c.d_tws, tb));
  HIP_OK(dev::malloc(&c.d_itw, tb));
  HIP_OK(dev::malloc(&c.d_itws, tb));
  for (void* p : {(void*)c.d_tw, (void*)c.d_tws, (void*)c.d_itw, (void*)c.d_itws}) audit::add(p, tb);
  HIP_OK(dev::memcpy(c.d_tw, tw.data(), tb, hipMemcpyHostToDevice));
  HIP_OK(dev::memcpy(c.d_tws, tws.data(), tb, hipMemcpyHostToDevice));
  HIP_OK(dev::memcpy(c.d_itw, itw.data(), tb, hipMemcpyHostToDevice));
  HIP_OK(dev::memcpy(c.d_itws, itws.data(), tb, hipMemcpyHostToDevice));
  HIP_OK(dev::malloc(&c.d_twf, tb));
  HIP_OK(dev::malloc(&c.d_twq, tb));
  HIP_OK(dev::malloc(&c.d_itwf, tb));
  HIP_OK(dev::malloc(&c.d_itwq, tb));
  for (void* p : {(void*)c.d_twf, (void*)c.d_twq, (void*)c.d_itwf, (void*)c.d_itwq}) audit::add(p, tb);
  HIP_OK(dev::memcpy(c.d_twf, twf.data(), tb, hipMemcpyHostToDevice));
  HIP_OK(dev::memcpy(c.d_twq, twq.data(), tb, hipMemcpyHostToDevice));
  HIP_OK(dev::memcpy(c.d_itwf, itwf.data(), tb, hipMemcpyHostToDevice));
  HIP_OK(dev::memcpy(c.d_itwq, itwq.data(), tb, hipMemcpyHostToDevice));
  HIP_OK(dev::malloc(&c.d_ci, ci.size() * sizeof(u64)));
  audit::add(c.d_ci, ci.size() * sizeof(u64));
  HIP_OK(dev::memcpy(c.d_ci, ci.data(), ci.size() * sizeof(u64), hipMemcpyHostToDevice));

  // ---- ModUp tables, one per number of chain limbs l = 1..L+1
  const int nq = c.L + 1;
  c.h_modup.assign(nq + 1, ModUpTable{});
  for (int l = 1; l <= nq; ++l) {
    ModUpTable& t = c.h_modup[l];
    std::memset(&t, 0, sizeof(t));
    t.limbs = l;
    t.beta = (l + c.alpha - 1) / c.alpha;
    t.ext = l + c.K;
    if (t.ext > MAX_LIMBS || t.beta > MAX_DIGITS) BM_THROW(BM_EINVAL, "table limits exceeded");
    for (int s = 0; s < t.ext; ++s) t.ext_prime[s] = s < l ? s : c.pid_special(s - l);
    t.npairs = 0;
    for (int j = 0; j < t.beta; ++j) {
      const int lo = j * c.alpha, hi = std::min((j + 1) * c.alpha, l);
      for (int s = 0; s < t.ext; ++s) {
        if (s >= lo && s < hi) continue;
        if (t.npairs >= MAX_LIMBS) BM_THROW(BM_EINVAL, "too many ModUp targets for one launch");
        t.pair_j[t.npairs] = (int8_t)j;
        t.pair_t[t.npairs] = (int8_t)s;
        ++t.npairs;
      }
    }
    for (int j = 0; j < t.beta; ++j) {
      ModUpDigit& dg = t.d[j];
      int lo = j * c.alpha, hi = std::min((j + 1) * c.alpha, l);
      dg.nsrc = hi - lo;
      for (int a = 0; a < dg.nsrc; ++a) {
        int i = lo + a;
        dg.src[a] = i;
        const u64 qi = c.primes[i].q;
        u64 qhat_mod_qi = 1;   // (Q_j / q_i) mod q_i
        for (int b = lo; b < hi; ++b)
          if (b != i) qhat_mod_qi = h_mulmod(qhat_mod_qi, c.primes[b].q % qi, qi);
        put_pair(dg.qhatinv[a], h_invmod(qhat_mod_qi, qi), qi);
        for (int s = 0; s < t.ext; ++s) {
          const u64 mt = c.primes[t.ext_prime[s]].q;
          u64 v = 1;
          for (int b = lo; b < hi; ++b)
            if (b != i) v = h_mulmod(v, c.primes[b].q % mt, mt);
          put_pair(dg.qhat[a][s], v, mt);
        }
      }
    }
  }
  HIP_OK(dev::malloc(&c.d_modup, sizeof(ModUpTable) * (nq + 1)));
  audit::add(c.d_modup, sizeof(ModUpTable) * (nq + 1));
  HIP_OK(dev::memcpy(c.d_modup, c.h_modup.data(), sizeof(ModUpTable) * (nq + 1),
                   hipMemcpyHostToDevice));

  // ---- ModDown table
  ModDownTable& md = c.h_moddown;
  std::memset(&md, 0, sizeof(md));
  md.K = c.K;
  for (int k = 0; k < c.K; ++k) {
    md.pprime[k] = c.pid_special(k);
    const u64 pk = c.primes[c.pid_special(k)].q;
    u64 phat = 1;
    for (int k2 = 0; k2 < c.K; ++k2)
      if (k2 != k) phat = h_mulmod(phat, c.primes[c.pid_special(k2)].q % pk, pk);
    put_pair(md.phatinv[k], h_invmod(phat, pk), pk);
    for (int i = 0; i < nq; ++i) {
      const u64 qi = c.primes[i].q;
      u64 v = 1;
      for (int k2 = 0; k2 < c.K; ++k2)
        if (k2 != k) v = h_mulmod(v, c.primes[c.pid_special(k2)].q % qi, qi);
      put_pair(md.phat[k][i], v, qi);
    }
  }
  for (int i = 0; i < nq; ++i) {
    const u64 qi = c.primes[i].q;
    u64 P = 1;
    for (int k = 0; k < c.K; ++k) P = h_mulmod(P, c.primes[c.pid_special(k)].q % qi, qi);
    put_pair(md.pinv[i], h_invmod(P, qi), qi);
  }
  HIP_OK(dev::malloc(&c.d_moddown, sizeof(ModDownTable)));
  audit::add(c.d_moddown, sizeof(ModDownTable));
  HIP_OK(dev::memcpy(c.d_moddown, &md, sizeof(ModDownTable), hipMemcpyHostToDevice));

  // ---- rescale table: q_l^{-1} mod q_i
  std::vector<u64> rs((size_t)nq * nq * 2, 0);
  for (int l = 0; l < nq; ++l)
    for (int i = 0; i < nq; ++i) {
      if (i == l) continue;
      const u64 qi = c.primes[i].q;
      put_pair(&rs[((size_t)l * nq + i) * 2], h_invmod(c.primes[l].q % qi, qi), qi);
    }
  HIP_OK(dev::malloc(&c.d_rescale, rs.size() * sizeof(u64)));
  audit::add(c.d_rescale, rs.size() * sizeof(u64));
  HIP_OK(dev::memcpy(c.d_rescale, rs.data(), rs.size() * sizeof(u64), hipMemcpyHostToDevice));
}

}  // namespace bm
