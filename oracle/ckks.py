"""Plain, slow CKKS over RNS with hybrid key switching: the oracle's scheme layer.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports this module and
this module imports nothing from the library.  Only tests, the smoke check and
the benchmark's CPU-baseline leg use it.

Representation: every polynomial is kept in the COEFFICIENT domain as a numpy
uint64 array [limbs][N], each row reduced into [0, q) for its prime.  Ring
products go through `prims.polymul` (textbook NTT, u128 `%`).  No step is
fused or reordered beyond what the definitions state.

The paper (Sec. 2, "Homomorphic Encryption") uses CKKS through five
operations: Add, Mul(P), Mul(C) with relinearisation, Rot and Res.  It does
not fix the concrete scheme variant; the readings taken here are:

  * ring Z[X]/(X^N+1), N/2 complex slots carrying real data, canonical
    embedding with slot j at the root zeta^(5^j), zeta = exp(i*pi/N);
  * RNS chain q_0..q_L, special primes p_0..p_{K-1}, digits of alpha
    consecutive q-limbs, hybrid key switching (ModUp by fast base conversion,
    key inner product, ModDown);
  * rescale and ModDown subtract the non-centred residue (floor variant);
  * Rot(v, r)[j] = v[(j + r) mod n] with Galois element 5^r mod 2N, the
    automorphism applied first and the key switch done with the key for
    s(X^g);
  * randomness from SHAKE-256 streams keyed by (seed, domain, index):
    ternary secret, discrete Gaussian (sigma = 3.2, |e| <= 19, by cumulative
    table) errors, uniform masks.

Conjugate-invariant ring (the paper's setting, Sec. 2; presets 3 and 4):
R' = Z[X + X^-1] inside Z[X]/(X^2N + 1), rank N, with N real slots.  An
element is kept as its first N coefficients c_0..c_{N-1} in Z[X]/(X^2N+1);
the others follow from the invariance a(X^-1) = a(X): c_N = 0 and
c_{2N-k} = -c_k.  Products and automorphisms are taken on that extension
in Z[X]/(X^2N+1) and cut back to N coefficients; encoding is the canonical
embedding of Z[X]/(X^2N+1) with real slot values (slot j at zeta^(5^j),
zeta = exp(i pi / 2N)), whose coefficients have exactly that symmetry;
rotations use Galois elements 5^r mod 4N; all other steps are
coefficient-wise and unchanged.  Secrets, errors and masks are sampled as
the N coefficients c_0..c_{N-1}.
"""
from decimal import Decimal, getcontext
from fractions import Fraction
import math

import numpy as np

from . import prims

# --------------------------------------------------------------------------
# parameters
# --------------------------------------------------------------------------

# Stream domains of the SHAKE-256 generator.
DOM_S, DOM_PK_A, DOM_PK_E, DOM_RLK_A, DOM_RLK_E, DOM_GK_A, DOM_GK_E = 1, 2, 3, 4, 5, 6, 7
DOM_ENC_V, DOM_ENC_E0, DOM_ENC_E1 = 8, 9, 10

PRESET_PRIMES = {
    # N = 2^12: one 50-bit and two 40-bit chain primes, one 51-bit special prime
    1: dict(log_n=12,
            q=[0x3ffffffffc001, 0xfffffdc001, 0xfffffc6001],
            p=[0x7fffffffe0001], alpha=1, log_scale=40),
    # N = 2^16: eight 50-bit chain primes, two 51-bit special primes, dnum = 4
    2: dict(log_n=16,
            q=[0x3ffffffd20001, 0x3ffffffb80001, 0x3fffffed60001, 0x3fffffec80001,
               0x3fffffebe0001, 0x3fffffea60001, 0x3fffffea40001, 0x3fffffe9e0001],
            p=[0x7fffffffe0001, 0x7ffffffd20001], alpha=2, log_scale=50),
    # conjugate-invariant ring, N = 2^12 (4096 real slots): primes = 1 mod 4N
    3: dict(log_n=12,
            q=[0x3ffffffffc001, 0xfffffdc001, 0xfffff4c001],
            p=[0x7fffffffe0001], alpha=1, log_scale=40, ring="ci"),
    # conjugate-invariant ring, N = 2^16 (65536 real slots): primes = 1 mod 4N
    4: dict(log_n=16,
            q=[0x3ffffffb80001, 0x3fffffec80001, 0x3fffffea40001, 0x3fffffe940001,
               0x3fffffdd40001, 0x3fffffd900001, 0x3fffffd540001, 0x3fffffd500001],
            p=[0x7ffffff9c0001, 0x7ffffff900001], alpha=2, log_scale=50, ring="ci"),
}


class Params:
    def __init__(self, log_n, q, p, alpha, log_scale, sigma=3.2, ring="std"):
        self.log_n = int(log_n)
        self.N = 1 << self.log_n
        if ring not in ("std", "ci"):
            raise ValueError("ring")
        self.ring = ring
        self.n = self.N if ring == "ci" else self.N // 2     # slots
        self.M = 4 * self.N if ring == "ci" else 2 * self.N  # order of the Galois group's roots
        self.q = [int(x) for x in q]
        self.p = [int(x) for x in p]
        self.L = len(self.q) - 1          # top level; a fresh ciphertext has L+1 limbs
        self.K = len(self.p)
        self.alpha = int(alpha)
        self.dnum = -(-len(self.q) // self.alpha)
        self.scale = float(2.0 ** log_scale)
        self.sigma = float(sigma)
        self.P = math.prod(self.p)

    @staticmethod
    def preset(i):
        return Params(**PRESET_PRIMES[i])

    def key_primes(self):
        """All limbs a switching key lives on: q_0..q_L then p_0..p_{K-1}."""
        return self.q + self.p


# --------------------------------------------------------------------------
# sampling
# --------------------------------------------------------------------------

_CDT_CACHE = {}


def gaussian_cdt(sigma=3.2, bound=19):
    """Cumulative table C_i = floor(2^64 * F(i - bound)), i = 0 .. 2*bound-1,
    F the normalised CDF of exp(-x^2 / (2 sigma^2)) on [-bound, bound].
    Evaluated in 60-digit decimal so every floor is exact."""
    key = (sigma, bound)
    if key in _CDT_CACHE:
        return _CDT_CACHE[key]
    getcontext().prec = 60
    two_s2 = 2 * Decimal(str(sigma)) ** 2
    rho = [(-(Decimal(x * x) / two_s2)).exp() for x in range(-bound, bound + 1)]
    total = sum(rho)
    cdt = []
    acc = Decimal(0)
    for i in range(2 * bound):
        acc += rho[i]
        cdt.append(int((acc / total) * (Decimal(2) ** 64)))   # int() floors a positive Decimal
    _CDT_CACHE[key] = cdt
    return cdt


def sample_ternary(params, seed, domain, index):
    return prims.sample_ternary(seed, domain, index, params.N)


def sample_gaussian(params, seed, domain, index):
    return prims.sample_cdt(seed, domain, index, gaussian_cdt(params.sigma), -19, params.N)


def sample_uniform(params, seed, domain, index, primes):
    return prims.sample_uniform(seed, domain, index, primes, params.N)


# --------------------------------------------------------------------------
# ring arithmetic on [limbs][N] coefficient arrays
# --------------------------------------------------------------------------

def reduce_int(poly, primes):
    """Signed integer polynomial -> residues [limbs][N] in [0, q)."""
    poly = np.asarray(poly, dtype=np.int64)
    return np.stack([np.mod(poly, np.int64(q)).astype(np.uint64) for q in primes])


def add(a, b, primes):
    return np.stack([(a[i] + b[i]) % np.uint64(q) for i, q in enumerate(primes)])


def sub(a, b, primes):
    return np.stack([(a[i] + np.uint64(q) - b[i]) % np.uint64(q) for i, q in enumerate(primes)])


def neg(a, primes):
    return np.stack([(np.uint64(q) - a[i]) % np.uint64(q) for i, q in enumerate(primes)])


def ci_extend(a, q):
    """N coefficients of a conjugate-invariant element -> its 2N coefficients
    in Z_q[X]/(X^2N+1): c_N = 0, c_{2N-k} = -c_k."""
    N = a.shape[0]
    out = np.zeros(2 * N, dtype=np.uint64)
    out[:N] = a
    out[N + 1:] = ((np.uint64(q) - a[1:]) % np.uint64(q))[::-1]
    return out


def polymul_jobs(jobs, ring="std"):
    """Products of (a, b, q) jobs in the ring: negacyclic of length N, or for
    the conjugate-invariant ring on the length-2N extensions, cut to N."""
    if ring == "std":
        return prims.polymul_batch(jobs)
    N = jobs[0][0].shape[0]
    prods = prims.polymul_batch([(ci_extend(a, q), ci_extend(b, q), q) for a, b, q in jobs])
    return [p[:N].copy() for p in prods]


def mul(a, b, primes, ring="std"):
    """Ring product, limb by limb."""
    return np.stack(polymul_jobs([(a[i], b[i], q) for i, q in enumerate(primes)], ring))


def mul_scalar(a, c, primes):
    """Multiply every limb by the integer c (reduced per prime)."""
    return np.stack([prims.mulmod_scalar(a[i], int(c) % q, q) for i, q in enumerate(primes)])


def automorphism(a, g, primes, ring="std"):
    """a(X) -> a(X^g) in Z_q[X]/(X^N+1), g odd: coefficient i moves to i*g mod 2N
    and changes sign when that index is >= N (X^N = -1).  Conjugate-invariant
    ring: the same on the 2N extension, cut back to N coefficients."""
    if ring == "ci":
        ext = np.stack([ci_extend(a[i], q) for i, q in enumerate(primes)])
        return automorphism(ext, g, primes)[:, :a.shape[1]].copy()
    N = a.shape[1]
    dst = (np.arange(N, dtype=np.int64) * int(g)) % (2 * N)
    flip = dst >= N
    pos = np.where(flip, dst - N, dst)
    out = np.empty_like(a)
    for i, q in enumerate(primes):
        vals = np.where(flip, (np.uint64(q) - a[i]) % np.uint64(q), a[i])
        out[i, pos] = vals
    return out


def galois_element(params, r):
    """Galois element of a left rotation by r slots: 5^(r mod n) mod 2N
    (mod 4N in the conjugate-invariant ring, whose N slots sit at the roots
    zeta^(5^j) of order 4N)."""
    return pow(5, r % params.n, params.M)


# --------------------------------------------------------------------------
# encoding (canonical embedding)
# --------------------------------------------------------------------------

def _slot_roots(N):
    """Index t (root zeta^(2t+1)) of slot j and of its conjugate."""
    n = N // 2
    e = np.array([pow(5, j, 2 * N) for j in range(n)], dtype=np.int64)
    return (e - 1) // 2, (2 * N - e - 1) // 2


def encode(z, scale, N, ring="std"):
    """Integer coefficients m_k = round_half_away((2/N) * Re sum_j scale*z_j * zeta^(-k 5^j)).

    Conjugate-invariant ring of rank N: the encoding of the N real values in
    Z[X]/(X^2N+1), cut to its first N coefficients.

    Evaluated by one length-N FFT over all odd-power roots: the vector holding
    scale*z_j at the root of slot j and its conjugate at the conjugate root,
    transformed and untwisted by zeta^(-k)."""
    if ring == "ci":
        return encode(np.real(np.asarray(z, dtype=np.complex128)), scale, 2 * N)[:N].copy()
    z = np.asarray(z, dtype=np.complex128)
    n = N // 2
    assert z.shape == (n,)
    t_slot, t_conj = _slot_roots(N)
    full = np.zeros(N, dtype=np.complex128)
    full[t_slot] = scale * z
    full[t_conj] = np.conj(scale * z)
    k = np.arange(N)
    m = np.fft.fft(full) * np.exp(-1j * np.pi * k / N) / N
    x = m.real
    return (np.sign(x) * np.floor(np.abs(x) + 0.5)).astype(np.int64)


def encode_direct(z, scale, N):
    """Same definition evaluated term by term, O(n N): a pin for small N only."""
    n = N // 2
    z = np.asarray(z, dtype=np.complex128)
    e = np.array([pow(5, j, 2 * N) for j in range(n)], dtype=np.int64)
    out = np.empty(N, dtype=np.int64)
    for k in range(N):
        ang = -np.pi * ((k * e) % (2 * N)) / N
        x = (2.0 / N) * np.sum(scale * z * np.exp(1j * ang)).real
        out[k] = int(np.sign(x) * np.floor(abs(x) + 0.5))
    return out


def decode(m, scale, N, ring="std"):
    """Slots z_j = (1/scale) * sum_k m_k zeta^(k 5^j) for an integer (or float)
    coefficient vector m.  Evaluated with one inverse FFT.  Conjugate-invariant
    ring: the N coefficients are extended to 2N (c_N = 0, c_{2N-k} = -c_k) and
    decoded in Z[X]/(X^2N+1); the N slots are real."""
    m = np.asarray([float(v) for v in m], dtype=np.float64) if not isinstance(m, np.ndarray) \
        else m.astype(np.float64)
    if ring == "ci":
        ext = np.zeros(2 * N)
        ext[:N] = m
        ext[N + 1:] = -m[1:][::-1]
        return decode(ext, scale, 2 * N)
    k = np.arange(N)
    w = np.fft.ifft(m * np.exp(1j * np.pi * k / N)) * N
    t_slot, _ = _slot_roots(N)
    return w[t_slot] / scale


def decode_direct(m, scale, N):
    n = N // 2
    m = np.asarray([float(v) for v in m], dtype=np.float64)
    e = np.array([pow(5, j, 2 * N) for j in range(n)], dtype=np.int64)
    k = np.arange(N)
    out = np.empty(n, dtype=np.complex128)
    for j in range(n):
        out[j] = np.sum(m * np.exp(1j * np.pi * ((k * e[j]) % (2 * N)) / N)) / scale
    return out


# --------------------------------------------------------------------------
# ciphertexts and keys
# --------------------------------------------------------------------------

class Ciphertext:
    """Components c_0..c_{deg} over the first `limbs` chain primes, coefficient domain."""

    def __init__(self, comps, limbs, scale):
        self.c = [np.asarray(x, dtype=np.uint64) for x in comps]
        self.limbs = int(limbs)
        self.scale = float(scale)

    def copy(self):
        return Ciphertext([x.copy() for x in self.c], self.limbs, self.scale)


class SwitchKey:
    """dnum pairs (b_j, a_j), each [L+1+K][N]."""

    def __init__(self, b, a):
        self.b = b
        self.a = a


class KeySet:
    def __init__(self, params, s, pk, rlk, gks):
        self.params = params
        self.s = s            # int64 [N], ternary
        self.pk = pk          # (b, a), each [L+1][N]
        self.rlk = rlk        # SwitchKey for s^2
        self.gks = gks        # {galois element: SwitchKey for s(X^g)}


def _digit(params, j, limbs):
    return list(range(j * params.alpha, min((j + 1) * params.alpha, limbs)))


def switch_key(params, s, s_prime, seed, dom_a, dom_e, index_base):
    """Key switching key from s' to s (hybrid, dnum digits):
    b_j = -a_j s + e_j + [P]_{q_i} s'  on the limbs i of digit j,
    b_j = -a_j s + e_j                 on every other limb (P limbs included)."""
    primes = params.key_primes()
    s_res = reduce_int(s, primes)
    sp_res = reduce_int(s_prime, primes) if s_prime.dtype == np.int64 else s_prime
    bs, as_ = [], []
    for j in range(params.dnum):
        a = sample_uniform(params, seed, dom_a, index_base + j, primes)
        e = reduce_int(sample_gaussian(params, seed, dom_e, index_base + j), primes)
        b = sub(e, mul(a, s_res, primes, params.ring), primes)
        for i in _digit(params, j, len(params.q)):
            gadget = prims.mulmod_scalar(sp_res[i], params.P % primes[i], primes[i])
            b[i] = (b[i] + gadget) % np.uint64(primes[i])
        bs.append(b)
        as_.append(a)
    return SwitchKey(bs, as_)


def keygen(params, seed, rotations=()):
    """Secret, public, relinearisation and Galois keys from one seed."""
    N = params.N
    s = sample_ternary(params, seed, DOM_S, 0)
    q_primes = params.q
    a = sample_uniform(params, seed, DOM_PK_A, 0, q_primes)
    e = reduce_int(sample_gaussian(params, seed, DOM_PK_E, 0), q_primes)
    s_q = reduce_int(s, q_primes)
    b = sub(e, mul(a, s_q, q_primes, params.ring), q_primes)
    kp = params.key_primes()
    s_kp = reduce_int(s, kp)
    s2 = mul(s_kp, s_kp, kp, params.ring)
    rlk = switch_key(params, s, s2, seed, DOM_RLK_A, DOM_RLK_E, 0)
    gks = {}
    for r in rotations:
        g = galois_element(params, r)
        if g in gks:
            continue
        s_g = automorphism(s_kp, g, kp, params.ring)
        gks[g] = switch_key(params, s, s_g, seed, DOM_GK_A, DOM_GK_E, g * params.dnum)
    assert N == s.size
    return KeySet(params, s, (b, a), rlk, gks)


def encrypt(params, pk, m, limbs, scale, seed, ct_id):
    """Public-key encryption of the integer plaintext m at `limbs` chain primes:
    (v b + e0 + m, v a + e1) with v ternary and e0, e1 Gaussian."""
    primes = params.q[:limbs]
    v = reduce_int(sample_ternary(params, seed, DOM_ENC_V, ct_id), primes)
    e0 = reduce_int(sample_gaussian(params, seed, DOM_ENC_E0, ct_id), primes)
    e1 = reduce_int(sample_gaussian(params, seed, DOM_ENC_E1, ct_id), primes)
    mm = reduce_int(m, primes)
    b, a = pk[0][:limbs], pk[1][:limbs]
    c0 = add(add(mul(v, b, primes, params.ring), e0, primes), mm, primes)
    c1 = add(mul(v, a, primes, params.ring), e1, primes)
    return Ciphertext([c0, c1], limbs, scale)


def decrypt_residues(params, s, ct):
    """c_0 + c_1 s (+ c_2 s^2 for a degree-2 ciphertext) mod each limb prime."""
    primes = params.q[:ct.limbs]
    s_res = reduce_int(s, primes)
    acc = ct.c[0].copy()
    spow = s_res
    for comp in ct.c[1:]:
        acc = add(acc, mul(comp, spow, primes, params.ring), primes)
        spow = mul(spow, s_res, primes, params.ring)
    return acc


def crt_centered(params, res):
    """Centred integers from the residues of the first two limbs (one if only
    one is present).  Valid while |m| < q_0 q_1 / 2."""
    q0 = params.q[0]
    r0 = [int(v) for v in res[0]]
    if res.shape[0] == 1:
        return [v - q0 if v > q0 // 2 else v for v in r0]
    q1 = params.q[1]
    inv = pow(q0, -1, q1)
    Q = q0 * q1
    out = []
    for a0, a1 in zip(r0, (int(v) for v in res[1])):
        m = a0 + q0 * (((a1 - a0) * inv) % q1)
        out.append(m - Q if m > Q // 2 else m)
    return out


def decrypt_decode(params, s, ct):
    return decode(crt_centered(params, decrypt_residues(params, s, ct)), ct.scale, params.N, params.ring)


# --------------------------------------------------------------------------
# homomorphic operations
# --------------------------------------------------------------------------

def _check_same(x, y):
    if x.limbs != y.limbs:
        raise ValueError("level mismatch")
    if x.scale != y.scale:
        raise ValueError("scale mismatch")


def hadd(params, x, y):
    """Add(C): componentwise, equal level and equal scale required."""
    _check_same(x, y)
    primes = params.q[:x.limbs]
    deg = max(len(x.c), len(y.c))
    comps = []
    for i in range(deg):
        if i < len(x.c) and i < len(y.c):
            comps.append(add(x.c[i], y.c[i], primes))
        else:
            comps.append((x.c[i] if i < len(x.c) else y.c[i]).copy())
    return Ciphertext(comps, x.limbs, x.scale)


def pmul(params, x, pt, pt_scale):
    """Mul(P): multiply both components by the integer plaintext pt."""
    primes = params.q[:x.limbs]
    p = reduce_int(pt, primes)
    return Ciphertext([mul(c, p, primes, params.ring) for c in x.c], x.limbs, x.scale * pt_scale)


def tensor(params, x, y):
    """First half of Mul(C): (a0 b0, a0 b1 + a1 b0, a1 b1)."""
    _check_levels = x.limbs == y.limbs
    if not _check_levels:
        raise ValueError("level mismatch")
    primes = params.q[:x.limbs]
    a0, a1 = x.c
    b0, b1 = y.c
    d0 = mul(a0, b0, primes, params.ring)
    d1 = add(mul(a0, b1, primes, params.ring), mul(a1, b0, primes, params.ring), primes)
    d2 = mul(a1, b1, primes, params.ring)
    return Ciphertext([d0, d1, d2], x.limbs, x.scale * y.scale)


def mod_up_digit(params, x, limbs, j):
    """Fast base conversion of digit j of x (x over q_0..q_{limbs-1}) to every
    limb of Q_l u P:  y_t = sum_{i in D_j} [x_i (Q_j/q_i)^-1]_{q_i} [Q_j/q_i]_t mod t."""
    D = _digit(params, j, limbs)
    Qj = math.prod(params.q[i] for i in D)
    targets = params.q[:limbs] + params.p
    y = np.zeros((len(targets), params.N), dtype=np.uint64)
    for i in D:
        qi = params.q[i]
        qhat = Qj // qi
        v = prims.mulmod_scalar(x[i], pow(qhat % qi, -1, qi), qi)
        for t, mod in enumerate(targets):
            y[t] = (y[t] + prims.mulmod_scalar(v, qhat % mod, mod)) % np.uint64(mod)
    return y


def key_switch(params, x, limbs, key):
    """KS(x): ModUp of every digit, key inner product over Q_l u P, ModDown by P.
    x is one polynomial over q_0..q_{limbs-1}; returns (u, w) over the same primes."""
    qs = params.q[:limbs]
    ext = qs + params.p
    key_limb = list(range(limbs)) + [len(params.q) + k for k in range(params.K)]
    beta = -(-limbs // params.alpha)
    jobs = []
    for j in range(beta):
        y = mod_up_digit(params, x, limbs, j)
        for t, mod in enumerate(ext):
            jobs.append((y[t], key.b[j][key_limb[t]], mod))
            jobs.append((y[t], key.a[j][key_limb[t]], mod))
    prods = polymul_jobs(jobs, params.ring)
    u = np.zeros((len(ext), params.N), dtype=np.uint64)
    w = np.zeros((len(ext), params.N), dtype=np.uint64)
    it = iter(prods)
    for j in range(beta):
        for t, mod in enumerate(ext):
            u[t] = (u[t] + next(it)) % np.uint64(mod)
            w[t] = (w[t] + next(it)) % np.uint64(mod)
    return mod_down(params, u, limbs), mod_down(params, w, limbs)


def mod_down(params, u, limbs):
    """out_i = (u_i - sum_k [u_{p_k} (P/p_k)^-1]_{p_k} [P/p_k]_{q_i}) * P^-1 mod q_i."""
    P = params.P
    out = np.empty((limbs, params.N), dtype=np.uint64)
    vs = []
    for k, pk in enumerate(params.p):
        phat = P // pk
        vs.append(prims.mulmod_scalar(u[limbs + k], pow(phat % pk, -1, pk), pk))
    for i in range(limbs):
        qi = params.q[i]
        conv = np.zeros(params.N, dtype=np.uint64)
        for k, pk in enumerate(params.p):
            conv = (conv + prims.mulmod_scalar(vs[k], (P // pk) % qi, qi)) % np.uint64(qi)
        diff = (u[i] + np.uint64(qi) - conv) % np.uint64(qi)
        out[i] = prims.mulmod_scalar(diff, pow(P % qi, -1, qi), qi)
    return out


def relinearize(params, d, rlk):
    """Second half of Mul(C): (d0 + KS_0(d2), d1 + KS_1(d2)) with the key for s^2."""
    primes = params.q[:d.limbs]
    u, w = key_switch(params, d.c[2], d.limbs, rlk)
    return Ciphertext([add(d.c[0], u, primes), add(d.c[1], w, primes)], d.limbs, d.scale)


def rescale(params, x):
    """Res: c_i <- (c_i - [c_last]_{q_i}) * q_last^-1 mod q_i, the last limb dropped."""
    if x.limbs < 2:
        raise ValueError("no level left to rescale")
    ql = params.q[x.limbs - 1]
    comps = []
    for c in x.c:
        out = np.empty((x.limbs - 1, params.N), dtype=np.uint64)
        last = c[x.limbs - 1]
        for i in range(x.limbs - 1):
            qi = params.q[i]
            diff = (c[i] + np.uint64(qi) - last % np.uint64(qi)) % np.uint64(qi)
            out[i] = prims.mulmod_scalar(diff, pow(ql % qi, -1, qi), qi)
        comps.append(out)
    return Ciphertext(comps, x.limbs - 1, x.scale / ql)


def rotate(params, x, r, gks):
    """Rot(x, r): automorphism X -> X^g on both components, then key switch of
    the rotated c_1 with the key for s(X^g)."""
    g = galois_element(params, r)
    if g not in gks:
        raise KeyError("no Galois key for rotation %d" % r)
    primes = params.q[:x.limbs]
    c0 = automorphism(x.c[0], g, primes, params.ring)
    c1 = automorphism(x.c[1], g, primes, params.ring)
    u, w = key_switch(params, c1, x.limbs, gks[g])
    return Ciphertext([add(c0, u, primes), w], x.limbs, x.scale)


def rotation_sum_hoisted(params, x, amounts, gks):
    """x + sum_r Rot(x, r) with the rotations hoisted twice: digit ModUp of x_1
    once; for every r the automorphism applied to the extended digits and the
    key inner product with the key for s(X^g) accumulated over Q_l u P; one
    ModDown of the sums at the end; the automorphisms of x_0 added in Q_l.
    Same message as the sum of plain rotations; other rounding, so other bits
    (the automorphism of a ModUp is not the ModUp of the automorphism)."""
    l = x.limbs
    qs = params.q[:l]
    ext = qs + params.p
    key_limb = list(range(l)) + [len(params.q) + k for k in range(params.K)]
    beta = -(-l // params.alpha)
    ys = [mod_up_digit(params, x.c[1], l, j) for j in range(beta)]
    jobs = []
    for r in amounts:
        g = galois_element(params, r)
        if g not in gks:
            raise KeyError("no Galois key for rotation %d" % r)
        for j in range(beta):
            yg = automorphism(ys[j], g, ext, params.ring)
            for t, mod in enumerate(ext):
                jobs.append((yg[t], gks[g].b[j][key_limb[t]], mod))
                jobs.append((yg[t], gks[g].a[j][key_limb[t]], mod))
    prods = iter(polymul_jobs(jobs, params.ring))
    u = np.zeros((len(ext), params.N), dtype=np.uint64)
    w = np.zeros((len(ext), params.N), dtype=np.uint64)
    for _ in amounts:
        for j in range(beta):
            for t, mod in enumerate(ext):
                u[t] = (u[t] + next(prods)) % np.uint64(mod)
                w[t] = (w[t] + next(prods)) % np.uint64(mod)
    c0 = x.c[0].copy()
    for r in amounts:
        c0 = add(c0, automorphism(x.c[0], galois_element(params, r), qs, params.ring), qs)
    return Ciphertext([add(c0, mod_down(params, u, l), qs), add(x.c[1], mod_down(params, w, l), qs)],
                      l, x.scale)


def rotation_sum_masked(params, x, pt, pt_scale, amounts, gks):
    """pt x + sum_r Rot(pt x, r) for the integer plaintext pt (Mul(P) then the
    rotations), evaluated with the plaintext applied after the key inner
    products (an option of this build): digit ModUp of x_1 once; for every r
    the key inner product of the automorphism of the extended digits with
    the key for s(X^g), over Q_l u P, multiplied by phi_g(pt) read over
    Q_l u P and summed; one ModDown of each sum; the terms without a key
    switch, pt x_0 + sum_r phi_g(pt x_0) and pt x_1, added in Q_l.  Since
    phi_g is a ring automorphism, phi_g(pt x) = phi_g(pt) phi_g(x): the same
    message as Mul(P) followed by the rotations; other rounding, other bits.
    Returns the result at x's level and scale x.scale * pt_scale (no rescale)."""
    l = x.limbs
    qs = params.q[:l]
    ext = qs + params.p
    key_limb = list(range(l)) + [len(params.q) + k for k in range(params.K)]
    beta = -(-l // params.alpha)
    pt_ext = reduce_int(pt, ext)
    pt_q = pt_ext[:l]
    ys = [mod_up_digit(params, x.c[1], l, j) for j in range(beta)]
    gs = []
    jobs = []
    for r in amounts:
        g = galois_element(params, r)
        if g not in gks:
            raise KeyError("no Galois key for rotation %d" % r)
        gs.append(g)
        for j in range(beta):
            yg = automorphism(ys[j], g, ext, params.ring)
            for t, mod in enumerate(ext):
                jobs.append((yg[t], gks[g].b[j][key_limb[t]], mod))
                jobs.append((yg[t], gks[g].a[j][key_limb[t]], mod))
    prods = iter(polymul_jobs(jobs, params.ring))
    u = np.zeros((len(ext), params.N), dtype=np.uint64)
    w = np.zeros((len(ext), params.N), dtype=np.uint64)
    for g in gs:
        ur = np.zeros((len(ext), params.N), dtype=np.uint64)
        wr = np.zeros((len(ext), params.N), dtype=np.uint64)
        for j in range(beta):
            for t, mod in enumerate(ext):
                ur[t] = (ur[t] + next(prods)) % np.uint64(mod)
                wr[t] = (wr[t] + next(prods)) % np.uint64(mod)
        pg = automorphism(pt_ext, g, ext, params.ring)
        u = add(u, mul(pg, ur, ext, params.ring), ext)
        w = add(w, mul(pg, wr, ext, params.ring), ext)
    m0 = mul(pt_q, x.c[0], qs, params.ring)
    c0 = m0.copy()
    for g in gs:
        c0 = add(c0, automorphism(m0, g, qs, params.ring), qs)
    c1 = mul(pt_q, x.c[1], qs, params.ring)
    return Ciphertext([add(c0, mod_down(params, u, l), qs), add(c1, mod_down(params, w, l), qs)],
                      l, x.scale * pt_scale)


def drop_limbs(x, limbs):
    """Exact level drop: keep the first `limbs` residues."""
    if limbs > x.limbs:
        raise ValueError("cannot raise the level")
    return Ciphertext([c[:limbs].copy() for c in x.c], limbs, x.scale)
