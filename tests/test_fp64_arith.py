"""The library's FP64 modular arithmetic, built for the host, against exact
integers at the extremes of its stated bounds.

The GPU kernels carry residues of primes q < 2^51 as integers in doubles
(csrc/fp64_modarith.hpp).  Their exactness rests on magnitude bounds: a
product a w mod q within q (0.5 + |a| 2^-52 (1 + 2^-52)) of 0 for any
|a| < 2^52, fmul_mod_q within 1.25 q, a fold within q/2 + 1, accumulated sums
below 3q + 1, forward radix-16 phases below 3.5q (2.375q after a fold) and
inverse ones below 4q (2q), all below 2^53.  The same source, compiled for the
CPU, is driven here with the largest prime below 2^51 and the preset primes,
operands at +-3.5q, +-4q, 6.5q, q - 1 and 0, and checked against Python
integers: every result must be an integer congruent to the exact value and
inside the stated bound.
"""
import ctypes
import os
import random
import subprocess
from fractions import Fraction

import numpy as np
import pytest

from oracle import ckks

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "fp64_check.cpp")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _is_prime(n):
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):   # deterministic below 3.3e24
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


def _largest_prime_below(b):
    n = (1 << b) - 1
    while not _is_prime(n):
        n -= 2
    return n


Q51 = _largest_prime_below(51)
PRIMES = [Q51] + ckks.Params.preset(2).q[:2] + ckks.Params.preset(2).p + ckks.Params.preset(1).q[1:2]


@pytest.fixture(scope="module")
def chk(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("fp64") / "fp64_check.so")
    cmd = [HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-O2", "-ffp-contract=off", "-std=c++17", "-fPIC",
           "-shared", "-I", "/opt/rocm/include", SRC, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("host build of the FP64 arithmetic failed:\n" + r.stderr)
    lib = ctypes.CDLL(out)
    D = ctypes.POINTER(ctypes.c_double)
    U = ctypes.POINTER(ctypes.c_uint64)
    sz, dbl = ctypes.c_size_t, ctypes.c_double
    lib.chk_fmul_mod.argtypes = [D, D, D, sz, dbl, D]
    lib.chk_fmul_mod_q.argtypes = [D, D, sz, dbl, dbl, D]
    lib.chk_fred.argtypes = [D, sz, dbl, dbl, D]
    lib.chk_fsum_period.argtypes = [D, D, sz, ctypes.c_double, ctypes.c_double, D]
    lib.chk_fsum_period.restype = ctypes.c_uint64
    lib.chk_fold_period.argtypes = [ctypes.c_double]
    lib.chk_fold_period.restype = ctypes.c_int
    lib.chk_u64_to_f.argtypes = [U, sz, D]
    lib.chk_f_to_u64.argtypes = [D, sz, U]
    lib.chk_facc.argtypes = [D, D, sz, dbl, dbl, D]
    lib.chk_facc.restype = ctypes.c_uint64
    lib.chk_phase.argtypes = [D, D, ctypes.c_int, ctypes.c_int, dbl, dbl, D]
    lib.chk_residue.argtypes = [dbl, dbl, dbl]
    lib.chk_residue.restype = ctypes.c_uint64
    return lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _exact_int(x):
    assert float(x).is_integer(), "result %r is not an integer" % x
    return int(x)


def _operands(q):
    """Operands at the stated extremes: +-3.5q, +-4q, +-6.5q (where it is below
    2^53), +-(q - 1), q/2, 0, 1 and random."""
    rng = random.Random(q)
    fixed = [0, 1, -1, q - 1, -(q - 1), q // 2, -(q // 2), (7 * q) // 2, -((7 * q) // 2), 4 * q - 1,
             -(4 * q - 1), (13 * q) // 2, -((13 * q) // 2)]
    vals = fixed + [rng.randrange(-4 * q, 4 * q) for _ in range(200)]
    return [a for a in vals if abs(a) < 2 ** 53]        # doubles hold integers exactly below 2^53


@pytest.mark.parametrize("q", PRIMES)
def test_fmul_mod_exact_within_bound(chk, q):
    rng = random.Random(q + 1)
    ws = [0, 1, q - 1, q - 2, q // 2, (q + 1) // 2] + [rng.randrange(q) for _ in range(40)]
    A, W = [], []
    for a in _operands(q):
        for w in ws:
            A.append(a)
            W.append(w)
    a_arr, a_p = _d(A)
    w_arr, w_p = _d(W)
    wq_arr, wq_p = _d([float(w) / float(q) for w in W])     # the twiddle tables' fl(w / q)
    out, out_p = _d(np.zeros(len(A)))
    chk.chk_fmul_mod(a_p, w_p, wq_p, len(A), float(q), out_p)
    for a, w, r in zip(A, W, out):
        ri = _exact_int(r)
        assert (ri - a * w) % q == 0, "fmul_mod(%d, %d) mod %d" % (a, w, q)
        bound = q * (Fraction(1, 2) + Fraction(abs(a), 2 ** 52) * (1 + Fraction(1, 2 ** 52)))
        assert abs(ri) <= bound, "fmul_mod(%d, %d): |%d| above its bound" % (a, w, ri)
        assert abs(ri) < 2 ** 53


@pytest.mark.parametrize("q", PRIMES)
def test_fmul_mod_q_exact_within_bound(chk, q):
    rng = random.Random(q + 2)
    vals = [0, 1, q - 1, -(q - 1), q // 2, -(q // 2), q - 2] + [rng.randrange(-(q - 1), q) for _ in range(60)]
    ws = [0, 1, q - 1, q - 2, q // 2] + [rng.randrange(q) for _ in range(30)]
    A = [a for a in vals for _ in ws]
    W = [w for _ in vals for w in ws]
    a_arr, a_p = _d(A)
    w_arr, w_p = _d(W)
    out, out_p = _d(np.zeros(len(A)))
    chk.chk_fmul_mod_q(a_p, w_p, len(A), 1.0 / float(q), float(q), out_p)
    for a, w, r in zip(A, W, out):
        ri = _exact_int(r)
        assert (ri - a * w) % q == 0
        assert abs(ri) <= Fraction(5, 4) * q, "fmul_mod_q(%d, %d) = %d" % (a, w, ri)


@pytest.mark.parametrize("q", PRIMES)
def test_fred_and_residue(chk, q):
    rng = random.Random(q + 3)
    vals = [0, 1, -1, q, -q, q - 1, 3 * q + 1, -(3 * q + 1), (7 * q) // 2, -((7 * q) // 2), 4 * q, -4 * q,
            2 ** 53 - 1, -(2 ** 53 - 1)] + [rng.randrange(-(2 ** 53) + 1, 2 ** 53) for _ in range(300)]
    a_arr, a_p = _d(vals)
    assert all(float(v) == v for v in vals)
    out, out_p = _d(np.zeros(len(vals)))
    chk.chk_fred(a_p, len(vals), 1.0 / float(q), float(q), out_p)
    for a, r in zip(vals, out):
        ri = _exact_int(r)
        assert (ri - a) % q == 0
        assert abs(ri) <= q // 2 + 1
        assert chk.chk_residue(float(a), 1.0 / float(q), float(q)) == a % q


def test_exact_conversions(chk):
    rng = np.random.default_rng(4)
    v = np.concatenate([np.array([0, 1, 2 ** 32 - 1, 2 ** 32, 2 ** 52 - 1, Q51, Q51 - 1], dtype=np.uint64),
                        rng.integers(0, 2 ** 52, 1000, dtype=np.uint64)])
    f = np.zeros(len(v))
    chk.chk_u64_to_f(v.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), len(v),
                     f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert all(int(x) == int(y) for x, y in zip(f, v))
    back = np.zeros(len(v), dtype=np.uint64)
    chk.chk_f_to_u64(f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(v),
                     back.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    assert np.array_equal(back, v)


@pytest.mark.parametrize("q", PRIMES)
def test_accumulated_products(chk, q):
    """Sums of up to 64 products of residues, all operands q - 1 (the largest
    products) or mixed extremes: the exact residue, and |s| <= 3q + 1."""
    rng = random.Random(q + 5)
    cases = [([q - 1] * 64, [q - 1] * 64), ([q - 1] * 7, [q - 2] * 7), ([1] * 3, [q - 1] * 3)]
    for _ in range(20):
        n = rng.randrange(1, 65)
        pick = lambda: rng.choice([0, 1, q - 1, q - 2, q // 2, rng.randrange(q)])   # noqa: E731
        cases.append(([pick() for _ in range(n)], [pick() for _ in range(n)]))
    for v, w in cases:
        v_arr, v_p = _d(v)
        w_arr, w_p = _d(w)
        m = ctypes.c_double(0)
        r = chk.chk_facc(v_p, w_p, len(v), 1.0 / float(q), float(q), ctypes.byref(m))
        assert r == sum(a * b for a, b in zip(v, w)) % q
        assert m.value <= 3 * q + 1


@pytest.mark.parametrize("q", PRIMES)
def test_fold_period_sums(chk, q):
    """Sums folded every fold_period(q) products (8 below 2^50, else 2): the
    exact residue, and every partial sum within 7.5q + 1 (q < 2^50) or
    3q + 1, below 2^53, at the largest operands and at mixed extremes."""
    per = chk.chk_fold_period(float(q))
    assert per == (8 if q < 2 ** 50 else 2)
    bound = Fraction(15, 2) * q + 1 if per == 8 else 3 * q + 1
    assert bound < 2 ** 53
    rng = random.Random(q + 11)
    cases = [([q - 1] * 64, [q - 1] * 64), ([q - 1] * 9, [q - 2] * 9), ([q // 2] * 16, [q - 1] * 16)]
    for _ in range(20):
        n = rng.randrange(1, 65)
        pick = lambda: rng.choice([0, 1, q - 1, q - 2, q // 2, rng.randrange(q)])   # noqa: E731
        cases.append(([pick() for _ in range(n)], [pick() for _ in range(n)]))
    for v, w in cases:
        v_arr, v_p = _d(v)
        w_arr, w_p = _d(w)
        m = ctypes.c_double(0)
        r = chk.chk_fsum_period(v_p, w_p, len(v), 1.0 / float(q), float(q), ctypes.byref(m))
        assert r == sum(a * b for a, b in zip(v, w)) % q
        assert m.value <= bound


def _phase_exact(x, tw, inverse, q):
    """The same four butterfly stages in exact integers mod q."""
    x = [v % q for v in x]
    ks = (3, 2, 1, 0) if inverse else (0, 1, 2, 3)
    for k in ks:
        step = 8 >> k
        for j in range(16):
            if j & step:
                continue
            w = tw[k][j]
            U, V = x[j], x[j + step]
            if inverse:
                x[j], x[j + step] = (U + V) % q, (U - V) * w % q
            else:
                T = V * w % q
                x[j], x[j + step] = (U + T) % q, (U - T) % q
    return x


def _run_phase(chk, x, tw, fold_first, inverse, q):
    xa, xp = _d([float(v) for v in x])
    flat = []
    for k in range(4):
        for j in range(16):
            flat += [float(tw[k][j]), float(tw[k][j]) / float(q)]
    ta, tp = _d(flat)
    m = ctypes.c_double(0)
    chk.chk_phase(xp, tp, int(fold_first), int(inverse), 1.0 / float(q), float(q), ctypes.byref(m))
    return [_exact_int(v) for v in xa], m.value


@pytest.mark.parametrize("q", PRIMES)
@pytest.mark.parametrize("inverse", [False, True])
def test_radix16_phases_exact_within_bound(chk, q, inverse):
    """A pass of the NTT kernels: a phase from residues in [0, q) (its output
    within 3.5q forward, 4q inverse), then a phase that folds first (within
    2.375q forward, 2q inverse), both congruent to the exact butterflies."""
    rng = random.Random(q * 3 + inverse)
    first_bound = Fraction(7, 2) * q if not inverse else 4 * q
    second_bound = Fraction(19, 8) * q if not inverse else 2 * q
    patterns = [lambda: q - 1, lambda: 0, lambda: rng.choice([0, q - 1]), lambda: rng.randrange(q),
                lambda: rng.choice([q - 1, q // 2, 1])]
    tw_patterns = [lambda: q - 1, lambda: 1, lambda: rng.randrange(q), lambda: rng.choice([q - 1, q - 2, q // 2]),
                   lambda: q - 1 - rng.randrange(16)]
    for trial in range(120):
        xp = patterns[trial % len(patterns)]
        tp = tw_patterns[(trial // len(patterns)) % len(tw_patterns)]
        x = [xp() for _ in range(16)]
        tw1 = [[tp() for _ in range(16)] for _ in range(4)]
        tw2 = [[tp() for _ in range(16)] for _ in range(4)]
        y, m1 = _run_phase(chk, x, tw1, False, inverse, q)
        assert m1 <= first_bound, "first phase reached %.3f q" % (m1 / q)
        want = _phase_exact(x, tw1, inverse, q)
        assert [v % q for v in y] == want
        z, m2 = _run_phase(chk, y, tw2, True, inverse, q)
        assert m2 <= max(second_bound, m1), "second phase reached %.3f q" % (m2 / q)
        assert max(abs(v) for v in z) <= second_bound
        assert [v % q for v in z] == _phase_exact(want, tw2, inverse, q)
        assert m2 < 2 ** 53
