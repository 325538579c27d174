"""Pins of the oracle's arithmetic floor against things other than itself."""
import hashlib
import random

import numpy as np
import pytest

from oracle import prims, ckks


def is_prime(n):
    """Deterministic Miller-Rabin for n < 3.3e24 (first 13 prime bases)."""
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41]
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


# ---------------------------------------------------------------- primes

@pytest.mark.parametrize("preset", [1, 2, 3, 4])
def test_preset_primes_are_ntt_friendly_primes(preset):
    P = ckks.Params.preset(preset)
    two_n = P.M          # 2N, or 4N in the conjugate-invariant ring
    for q in P.q + P.p:
        assert is_prime(q)
        assert q % two_n == 1
        assert q < (1 << 51)
    assert len(set(P.q + P.p)) == len(P.q) + len(P.p)
    # special modulus exceeds every digit product (key-switching noise bound)
    for j in range(P.dnum):
        Qj = 1
        for i in range(j * P.alpha, min((j + 1) * P.alpha, len(P.q))):
            Qj *= P.q[i]
        assert P.P > Qj


def test_preset_primes_are_largest_in_their_size_class():
    """Primes are the largest below 2^b congruent to 1 mod 2N, taken in
    descending order (checked by scanning every candidate above each)."""
    P = ckks.Params.preset(2)
    step = 2 * P.N
    expect = []
    cand = ((1 << 50) - 1) // step * step + 1
    while len(expect) < 8:
        if is_prime(cand):
            expect.append(cand)
        cand -= step
    assert expect == P.q
    c1 = ckks.Params.preset(1)
    cand = ((1 << 50) - 1) // (2 * c1.N) * (2 * c1.N) + 1
    while not is_prime(cand):
        cand -= 2 * c1.N
    assert cand == c1.q[0]


@pytest.mark.parametrize("preset", [3, 4])
def test_ci_preset_primes_are_largest_below_their_bounds(preset):
    """Conjugate-invariant presets: each size class holds the largest primes
    below 2^b congruent to 1 mod 4N, in descending order."""
    P = ckks.Params.preset(preset)
    step = P.M
    assert step == 4 * P.N

    def largest(bits, count, skip=()):
        out = []
        cand = ((1 << bits) - 1) // step * step + 1
        while len(out) < count:
            if cand not in skip and is_prime(cand):
                out.append(cand)
            cand -= step
        return out
    bits = [q.bit_length() for q in P.q]
    got = []
    for b in sorted(set(bits), reverse=True):
        got += largest(b, bits.count(b))
    assert got == P.q
    assert largest(51, len(P.p)) == P.p


# ---------------------------------------------------------------- SHAKE-256

@pytest.mark.parametrize("n_in,n_out", [(0, 32), (3, 1), (135, 200), (136, 136), (137, 500), (300, 1000)])
def test_shake256_matches_hashlib(n_in, n_out):
    rnd = random.Random(n_in * 1000 + n_out)
    data = bytes(rnd.getrandbits(8) for _ in range(n_in))
    assert prims.shake256(data, n_out) == hashlib.shake_256(data).digest(n_out)


def _hash_words(seed, domain, index, n):
    msg = seed.to_bytes(8, "little") + domain.to_bytes(4, "little") + index.to_bytes(8, "little")
    raw = hashlib.shake_256(msg).digest(8 * n)
    return [int.from_bytes(raw[8 * i:8 * i + 8], "little") for i in range(n)]


def test_stream_words_layout():
    got = prims.stream_words(0xB11D, 6, 12345, 40)
    assert [int(x) for x in got] == _hash_words(0xB11D, 6, 12345, 40)


def test_ternary_sampler_rule():
    words = _hash_words(7, 1, 0, 200)
    expect = []
    bound = 3 * ((1 << 64) // 3)
    for u in words:
        if u >= bound:
            continue
        expect.append(u % 3 - 1)
    got = prims.sample_ternary(7, 1, 0, 150)
    assert list(got) == expect[:150]


def test_uniform_sampler_rule():
    qs = [0x3ffffffffc001, 0xfffffdc001]
    n = 64
    words = _hash_words(9, 2, 3, 400)
    expect = []
    it = iter(words)
    for q in qs:
        mask = (1 << q.bit_length()) - 1
        row = []
        while len(row) < n:
            u = next(it) & mask
            if u < q:
                row.append(u)
        expect.append(row)
    got = prims.sample_uniform(9, 2, 3, qs, n)
    assert got.tolist() == expect


def test_gaussian_table_and_sampler():
    cdt = ckks.gaussian_cdt(3.2)
    assert len(cdt) == 38
    # absolute value of the first entry, floor(2^64 F(-19)), computed
    # independently of this code when the sampler was specified
    assert cdt[0] == 50861754284
    assert all(a < b for a, b in zip(cdt, cdt[1:]))
    # symmetry of the centred distribution: F(v) + F(-v-1) = 1
    for i in range(38):
        assert abs(cdt[i] + cdt[37 - i] - (1 << 64)) <= 1
    # consecutive probability masses follow exp(-x^2 / (2 sigma^2))
    mass = [cdt[0]] + [cdt[i] - cdt[i - 1] for i in range(1, 38)] + [(1 << 64) - cdt[37]]
    for x in (1, 2, 5):
        ratio = mass[19 + x] / mass[19]
        assert abs(ratio - np.exp(-x * x / (2 * 3.2 ** 2))) < 1e-9
    # the sampler applies the table: x = -19 + #{i : u >= C_i}
    words = _hash_words(11, 3, 0, 100)
    expect = [-19 + sum(u >= c for c in cdt) for u in words]
    assert list(prims.sample_cdt(11, 3, 0, cdt, -19, 100)) == expect
    big = prims.sample_cdt(12, 3, 0, cdt, -19, 400_000)
    assert abs(big.std() - 3.2) < 0.032
    assert abs(big.mean()) < 0.03
    assert big.min() >= -19 and big.max() <= 19


# ---------------------------------------------------------------- ring product

def _py_negacyclic(a, b, q):
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            if i + j < n:
                out[i + j] += a[i] * b[j]
            else:
                out[i + j - n] -= a[i] * b[j]
    return [v % q for v in out]


@pytest.mark.parametrize("n", [8, 16, 64])
def test_polymul_matches_python_schoolbook(n):
    rnd = random.Random(n)
    for q in ckks.Params.preset(2).q[:3] + ckks.Params.preset(1).q + ckks.Params.preset(2).p:
        a = [rnd.randrange(q) for _ in range(n)]
        b = [rnd.randrange(q) for _ in range(n)]
        got = prims.polymul(np.array(a, dtype=np.uint64), np.array(b, dtype=np.uint64), q)
        assert [int(x) for x in got] == _py_negacyclic(a, b, q)


def test_polymul_matches_c_schoolbook_n1024():
    rng = np.random.default_rng(0)
    for q in ckks.Params.preset(2).q + ckks.Params.preset(2).p:
        a = rng.integers(0, q, 1024, dtype=np.uint64)
        b = rng.integers(0, q, 1024, dtype=np.uint64)
        assert np.array_equal(prims.polymul(a, b, q), prims.polymul_schoolbook(a, b, q))


@pytest.mark.parametrize("preset", [1, 2])
def test_polymul_identity_and_shift_full_size(preset):
    """a * 1 = a and a * X = negacyclic shift, at the full ring size, every prime."""
    P = ckks.Params.preset(preset)
    rng = np.random.default_rng(preset)
    for q in P.q + P.p:
        a = rng.integers(0, q, P.N, dtype=np.uint64)
        one = np.zeros(P.N, dtype=np.uint64)
        one[0] = 1
        x = np.zeros(P.N, dtype=np.uint64)
        x[1] = 1
        assert np.array_equal(prims.polymul(a, one, q), a)
        sh = np.empty_like(a)
        sh[1:] = a[:-1]
        sh[0] = (q - int(a[-1])) % q
        assert np.array_equal(prims.polymul(a, x, q), sh)


def test_mulmod_vec_and_scalar():
    rnd = random.Random(5)
    q = ckks.Params.preset(2).p[1]
    a = [rnd.randrange(1 << 64) for _ in range(50)]
    b = [rnd.randrange(q) for _ in range(50)]
    got = prims.mulmod_vec(np.array(a, dtype=np.uint64), np.array(b, dtype=np.uint64), q)
    assert [int(x) for x in got] == [x * y % q for x, y in zip(a, b)]
    got = prims.mulmod_scalar(np.array(a, dtype=np.uint64), 12345678901, q)
    assert [int(x) for x in got] == [x * 12345678901 % q for x in a]
