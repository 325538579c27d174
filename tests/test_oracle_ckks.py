"""Pins of the oracle's CKKS layer: closed forms, big-integer identities and
decryption to the expected messages, on tiny rings and at the full sizes."""
import math
import random

import numpy as np
import pytest

from oracle import ckks, prims


def tiny(log_n=5, preset=2):
    base = ckks.PRESET_PRIMES[preset]
    return ckks.Params(log_n=log_n, q=base["q"], p=base["p"], alpha=base["alpha"],
                       log_scale=base["log_scale"])


def crt(res, primes):
    M = math.prod(primes)
    x = 0
    for r, q in zip(res, primes):
        Mi = M // q
        x += int(r) * Mi * pow(Mi, -1, q)
    return x % M


def centred(v, M):
    v %= M
    return v - M if v > M // 2 else v


def negacyclic_int(a, b):
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            if i + j < n:
                out[i + j] += a[i] * b[j]
            else:
                out[i + j - n] -= a[i] * b[j]
    return out


def rand_slots(rng, n, scale=1.0):
    return scale * rng.uniform(-1, 1, n)


# ---------------------------------------------------------------- encoding

@pytest.mark.parametrize("log_n", [4, 6, 8, 10])
def test_encode_matches_direct_sum(log_n):
    N = 1 << log_n
    rng = np.random.default_rng(log_n)
    z = rng.uniform(-1, 1, N // 2) + 1j * rng.uniform(-1, 1, N // 2)
    a = ckks.encode(z, 2.0 ** 40, N)
    b = ckks.encode_direct(z, 2.0 ** 40, N)
    assert np.max(np.abs(a - b)) <= 1


@pytest.mark.parametrize("log_n", [4, 8])
def test_decode_matches_direct_sum(log_n):
    N = 1 << log_n
    rng = np.random.default_rng(log_n + 100)
    m = rng.integers(-2 ** 45, 2 ** 45, N)
    a = ckks.decode(m, 2.0 ** 40, N)
    b = ckks.decode_direct(m, 2.0 ** 40, N)
    assert np.max(np.abs(a - b)) < 1e-9


def test_decode_inverts_encode_full_size():
    N = 1 << 16
    rng = np.random.default_rng(3)
    z = rng.uniform(-1, 1, N // 2)
    back = ckks.decode(ckks.encode(z, 2.0 ** 50, N), 2.0 ** 50, N)
    assert np.max(np.abs(back - z)) < 2.0 ** -30


def test_encode_constant_is_constant_polynomial():
    N = 1 << 12
    m = ckks.encode(np.full(N // 2, 0.3), 2.0 ** 40, N)
    assert m[0] == round(0.3 * 2 ** 40)
    assert np.all(m[1:] == 0)


def test_encode_slot_product_is_ring_product():
    """The canonical embedding turns slot-wise products into ring products."""
    N = 32
    rng = np.random.default_rng(9)
    z1, z2 = rng.uniform(-1, 1, N // 2), rng.uniform(-1, 1, N // 2)
    m1 = ckks.encode(z1, 2.0 ** 30, N)
    m2 = ckks.encode(z2, 2.0 ** 30, N)
    prod = negacyclic_int([int(v) for v in m1], [int(v) for v in m2])
    got = ckks.decode(prod, 2.0 ** 60, N)
    assert np.max(np.abs(got - z1 * z2)) < 1e-6


# ---------------------------------------------------------------- automorphism

@pytest.mark.parametrize("r", [1, 2, 5, -3, -8])
def test_automorphism_rotates_slots_left(r):
    P = tiny(log_n=6)
    rng = np.random.default_rng(r + 50)
    z = rng.uniform(-1, 1, P.n)
    m = ckks.encode(z, P.scale, P.N)
    g = ckks.galois_element(P, r)
    res = ckks.automorphism(ckks.reduce_int(m, P.q[:2]), g, P.q[:2])
    back = ckks.decode(ckks.crt_centered(P, res), P.scale, P.N)
    assert np.max(np.abs(back - np.roll(z, -r))) < 1e-9


def test_automorphism_is_ring_homomorphism_and_invertible():
    P = tiny(log_n=7)
    rng = np.random.default_rng(1)
    primes = P.q[:2]
    a = np.stack([rng.integers(0, q, P.N, dtype=np.uint64) for q in primes])
    b = np.stack([rng.integers(0, q, P.N, dtype=np.uint64) for q in primes])
    g = ckks.galois_element(P, 3)
    lhs = ckks.automorphism(ckks.mul(a, b, primes), g, primes)
    rhs = ckks.mul(ckks.automorphism(a, g, primes), ckks.automorphism(b, g, primes), primes)
    assert np.array_equal(lhs, rhs)
    ginv = pow(g, -1, 2 * P.N)
    assert np.array_equal(ckks.automorphism(ckks.automorphism(a, g, primes), ginv, primes), a)


# ---------------------------------------------------------------- base conversion

@pytest.mark.parametrize("limbs,j", [(8, 0), (8, 3), (7, 3), (5, 1)])
def test_mod_up_is_digit_plus_small_multiple(limbs, j):
    P = tiny(log_n=4)
    rng = np.random.default_rng(limbs * 10 + j)
    x = np.stack([rng.integers(0, q, P.N, dtype=np.uint64) for q in P.q[:limbs]])
    D = list(range(j * P.alpha, min((j + 1) * P.alpha, limbs)))
    Qj = math.prod(P.q[i] for i in D)
    y = ckks.mod_up_digit(P, x, limbs, j)
    targets = P.q[:limbs] + P.p
    for c in range(P.N):
        xd = crt([x[i, c] for i in D], [P.q[i] for i in D])
        for t, mod in enumerate(targets):
            ok = any((xd + u * Qj) % mod == int(y[t, c]) for u in range(len(D)))
            assert ok


@pytest.mark.parametrize("limbs", [8, 3, 1])
def test_mod_down_exact_division(limbs):
    P = tiny(log_n=4)
    rng = np.random.default_rng(limbs)
    ext = P.q[:limbs] + P.p
    u = np.stack([rng.integers(0, q, P.N, dtype=np.uint64) for q in ext])
    out = ckks.mod_down(P, u, limbs)
    for c in range(P.N):
        v = sum(int(u[limbs + k, c]) * pow(P.P // pk % pk, -1, pk) % pk * (P.P // pk)
                for k, pk in enumerate(P.p))
        U = crt([u[t, c] for t in range(len(ext))], ext)
        assert (U - v) % P.P == 0
        want = (U - v) // P.P
        for i in range(limbs):
            assert int(out[i, c]) == want % P.q[i]


@pytest.mark.parametrize("limbs", [8, 2])
def test_rescale_exact_division(limbs):
    P = tiny(log_n=4)
    rng = np.random.default_rng(limbs + 77)
    comps = [np.stack([rng.integers(0, q, P.N, dtype=np.uint64) for q in P.q[:limbs]])
             for _ in range(2)]
    ct = ckks.Ciphertext(comps, limbs, 2.0 ** 100)
    out = ckks.rescale(P, ct)
    ql = P.q[limbs - 1]
    assert out.limbs == limbs - 1 and out.scale == 2.0 ** 100 / ql
    for comp_in, comp_out in zip(ct.c, out.c):
        for c in range(P.N):
            X = crt(comp_in[:, c], P.q[:limbs])
            assert (X - X % ql) % ql == 0
            want = (X - X % ql) // ql
            for i in range(limbs - 1):
                assert int(comp_out[i, c]) == want % P.q[i]


# ---------------------------------------------------------------- keys

@pytest.fixture(scope="module")
def tiny_keys():
    P = tiny(log_n=5)
    keys = ckks.keygen(P, 0xB11D, rotations=[1, 2, 4, -2, 3])
    return P, keys


def _small(arr, primes, bound):
    for i, q in enumerate(primes):
        v = arr[i].astype(object)
        v = np.where(v > q // 2, v - q, v)
        if np.max(np.abs(v.astype(np.float64))) > bound:
            return False
    return True


def test_public_key_is_rlwe_sample(tiny_keys):
    P, keys = tiny_keys
    b, a = keys.pk
    s = ckks.reduce_int(keys.s, P.q)
    e = ckks.add(b, ckks.mul(a, s, P.q), P.q)
    assert _small(e, P.q, 19)
    assert set(np.unique(keys.s)) <= {-1, 0, 1}


def test_switch_keys_encode_gadget(tiny_keys):
    P, keys = tiny_keys
    kp = P.key_primes()
    s = ckks.reduce_int(keys.s, kp)
    s2 = ckks.mul(s, s, kp)
    targets = [(keys.rlk, s2)]
    for g, gk in keys.gks.items():
        targets.append((gk, ckks.automorphism(s, g, kp)))
    for key, sp in targets:
        for j in range(P.dnum):
            e = ckks.add(key.b[j], ckks.mul(key.a[j], s, kp), kp)
            for i in range(j * P.alpha, (j + 1) * P.alpha):
                gadget = prims.mulmod_scalar(sp[i], P.P % kp[i], kp[i])
                e[i] = (e[i] + np.uint64(kp[i]) - gadget) % np.uint64(kp[i])
            assert _small(e, kp, 19)


def test_encrypt_decrypt_round_trip(tiny_keys):
    P, keys = tiny_keys
    rng = np.random.default_rng(4)
    m = rng.integers(-2 ** 40, 2 ** 40, P.N)
    for limbs in (8, 3, 2):
        ct = ckks.encrypt(P, keys.pk, m, limbs, P.scale, 0xB11D, 17)
        got = ckks.crt_centered(P, ckks.decrypt_residues(P, keys.s, ct))
        err = np.array([g - int(x) for g, x in zip(got, m)], dtype=np.float64)
        # |v e + e0 + e1 s| <= N*19 + 19 + N*19
        assert np.max(np.abs(err)) <= 2 * P.N * 19 + 19


def test_tensor_decrypts_to_ring_product(tiny_keys):
    P, keys = tiny_keys
    rng = np.random.default_rng(5)
    m1 = rng.integers(-2 ** 20, 2 ** 20, P.N)
    m2 = rng.integers(-2 ** 20, 2 ** 20, P.N)
    c1 = ckks.encrypt(P, keys.pk, m1, 8, 1.0, 1, 1)
    c2 = ckks.encrypt(P, keys.pk, m2, 8, 1.0, 1, 2)
    d = ckks.tensor(P, c1, c2)
    res = ckks.decrypt_residues(P, keys.s, d)
    got = [centred(crt(res[:, c], P.q), math.prod(P.q)) for c in range(P.N)]
    want = negacyclic_int([int(v) for v in m1], [int(v) for v in m2])
    diff = max(abs(g - w) for g, w in zip(got, want))
    assert diff < 2 ** 34   # noise * message terms, far below the 2^40 product scale


def test_key_switch_decrypts_to_x_times_s_prime(tiny_keys):
    P, keys = tiny_keys
    rng = np.random.default_rng(6)
    for limbs in (8, 7, 3):
        primes = P.q[:limbs]
        x = np.stack([rng.integers(0, q, P.N, dtype=np.uint64) for q in primes])
        u, w = ckks.key_switch(P, x, limbs, keys.rlk)
        s = ckks.reduce_int(keys.s, primes)
        s2 = ckks.mul(s, s, primes)
        lhs = ckks.add(u, ckks.mul(w, s, primes), primes)
        rhs = ckks.mul(x, s2, primes)
        err = ckks.sub(lhs, rhs, primes)
        # noise: sum_j y_j e_j / P + rounding, a few thousand at most
        assert _small(err, primes, 2 ** 16)


def test_relinearize_preserves_message(tiny_keys):
    P, keys = tiny_keys
    rng = np.random.default_rng(7)
    z1, z2 = rng.uniform(-1, 1, P.n), rng.uniform(-1, 1, P.n)
    c1 = ckks.encrypt(P, keys.pk, ckks.encode(z1, P.scale, P.N), 8, P.scale, 2, 1)
    c2 = ckks.encrypt(P, keys.pk, ckks.encode(z2, P.scale, P.N), 8, P.scale, 2, 2)
    d = ckks.relinearize(P, ckks.tensor(P, c1, c2), keys.rlk)
    out = ckks.rescale(P, d)
    got = ckks.decrypt_decode(P, keys.s, out)
    assert np.max(np.abs(got - z1 * z2)) < 1e-9


@pytest.mark.parametrize("r", [1, 2, 4, -2, 3])
def test_rotate_decrypts_to_rolled_slots(tiny_keys, r):
    P, keys = tiny_keys
    rng = np.random.default_rng(8 + r)
    z = rng.uniform(-1, 1, P.n)
    for limbs in (8, 7, 2):
        ct = ckks.encrypt(P, keys.pk, ckks.encode(z, P.scale, P.N), limbs, P.scale, 3, r + 10)
        got = ckks.decrypt_decode(P, keys.s, ckks.rotate(P, ct, r, keys.gks))
        assert np.max(np.abs(got - np.roll(z, -r))) < 1e-9


def test_add_rejects_mismatched_scale_or_level(tiny_keys):
    P, keys = tiny_keys
    m = np.zeros(P.N, dtype=np.int64)
    a = ckks.encrypt(P, keys.pk, m, 3, 1.0, 1, 1)
    b = ckks.encrypt(P, keys.pk, m, 3, 2.0, 1, 2)
    c = ckks.encrypt(P, keys.pk, m, 2, 1.0, 1, 3)
    with pytest.raises(ValueError):
        ckks.hadd(P, a, b)
    with pytest.raises(ValueError):
        ckks.hadd(P, a, c)


def test_rotate_without_key_raises(tiny_keys):
    P, keys = tiny_keys
    ct = ckks.encrypt(P, keys.pk, np.zeros(P.N, dtype=np.int64), 2, 1.0, 1, 1)
    with pytest.raises(KeyError):
        ckks.rotate(P, ct, 7, keys.gks)


def test_full_size_rotation_c2_params():
    """One rotation and one multiply at N = 2^16 with the C2-C5 primes."""
    P = ckks.Params.preset(2)
    keys = ckks.keygen(P, 5, rotations=[1])
    rng = np.random.default_rng(11)
    z1, z2 = rng.uniform(-1, 1, P.n), rng.uniform(-1, 1, P.n)
    limbs = 3
    c1 = ckks.encrypt(P, keys.pk, ckks.encode(z1, P.scale, P.N), limbs, P.scale, 5, 1)
    c2 = ckks.encrypt(P, keys.pk, ckks.encode(z2, P.scale, P.N), limbs, P.scale, 5, 2)
    prod = ckks.rescale(P, ckks.relinearize(P, ckks.tensor(P, c1, c2), keys.rlk))
    rot = ckks.rotate(P, prod, 1, keys.gks)
    got = ckks.decrypt_decode(P, keys.s, rot)
    assert np.max(np.abs(got - np.roll(z1 * z2, -1))) < 1e-7
