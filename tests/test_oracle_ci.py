"""Pins of the oracle's conjugate-invariant ring (the paper's CKKS setting,
Sec. 2): closure of the representation, the real canonical embedding as a
cosine transform, rotations over N real slots, and the encrypted match
against the slot simulator."""
import numpy as np
import pytest

import slot_sim
from oracle import ckks, blindmatch as bm


def tiny_ci(log_n=6):
    base = ckks.PRESET_PRIMES[2]       # primes = 1 mod 2^17, so also 1 mod 4N here
    return ckks.Params(log_n=log_n, q=base["q"], p=base["p"], alpha=2, log_scale=50, ring="ci")


def ci_full(c):
    """Integer 2N coefficients of the conjugate-invariant element c_0..c_{N-1}."""
    N = len(c)
    out = np.zeros(2 * N, dtype=object)
    out[:N] = [int(v) for v in c]
    for k in range(1, N):
        out[2 * N - k] = -int(c[k])
    return out


def test_representation_is_closed_under_products():
    """The product in Z[X]/(X^2N+1) of two invariant elements is invariant:
    c_N = 0 and c_{2N-k} = -c_k (checked with Python integers, schoolbook)."""
    rng = np.random.default_rng(1)
    N = 16
    a = ci_full(rng.integers(-50, 50, N))
    b = ci_full(rng.integers(-50, 50, N))
    prod = [0] * (2 * N)
    for i in range(2 * N):
        for j in range(2 * N):
            k = i + j
            if k >= 2 * N:
                prod[k - 2 * N] -= a[i] * b[j]
            else:
                prod[k] += a[i] * b[j]
    assert prod[N] == 0
    assert all(prod[2 * N - k] == -prod[k] for k in range(1, N))
    # and the oracle's product of the N-coefficient forms agrees with it
    P = tiny_ci(log_n=4)
    q = P.q[0]
    got = ckks.mul(ckks.reduce_int([int(v) for v in a[:N]], [q]), ckks.reduce_int([int(v) for v in b[:N]], [q]),
                   [q], "ci")
    assert [int(v) for v in got[0]] == [v % q for v in prod[:N]]


def test_decode_is_the_cosine_transform():
    """Slot j of an invariant element: (c_0 + 2 sum_k c_k cos(pi k 5^j / 2N)) / scale."""
    rng = np.random.default_rng(2)
    N = 32
    c = rng.integers(-1000, 1000, N)
    z = ckks.decode(c.astype(np.int64), 10.0, N, "ci")
    for j in range(N):
        e = pow(5, j, 4 * N)
        want = (c[0] + 2 * sum(c[k] * np.cos(np.pi * k * e / (2 * N)) for k in range(1, N))) / 10.0
        assert abs(z[j].real - want) < 1e-9 and abs(z[j].imag) < 1e-9


def test_encode_decode_roundtrip_and_products():
    N = 1 << 10
    rng = np.random.default_rng(3)
    a, b = rng.uniform(-1, 1, N), rng.uniform(-1, 1, N)
    scale = 2.0 ** 30
    ca, cb = ckks.encode(a, scale, N, "ci"), ckks.encode(b, scale, N, "ci")
    assert np.max(np.abs(ckks.decode(ca, scale, N, "ci").real - a)) < 2.0 ** -20
    # slot-wise product of the plaintexts (exact integer product in the ring)
    q = (1 << 61) - 1              # only as a wide modulus for a centred integer result
    full = np.convolve(ci_full(ca).astype(object), ci_full(cb).astype(object))
    prod = np.array([full[k] - (full[k + 2 * N] if k + 2 * N < len(full) else 0) for k in range(N)], dtype=object)
    assert all(abs(v) < q for v in prod)
    z = ckks.decode(np.array([float(v) for v in prod]), scale * scale, N, "ci")
    assert np.max(np.abs(z.real - a * b)) < 2.0 ** -18


def test_rotation_over_n_real_slots():
    P = tiny_ci(log_n=6)
    rng = np.random.default_rng(4)
    keys = ckks.keygen(P, 0xB11D, rotations=[1, 5, -3])
    z = rng.uniform(-1, 1, P.n)
    assert P.n == P.N
    ct = ckks.encrypt(P, keys.pk, ckks.encode(z, P.scale, P.N, "ci"), len(P.q), P.scale, 9, 1)
    assert np.max(np.abs(ckks.decrypt_decode(P, keys.s, ct).real - z)) < 1e-9
    for r in (1, 5, -3):
        out = ckks.rotate(P, ct, r, keys.gks)
        assert np.max(np.abs(ckks.decrypt_decode(P, keys.s, out).real - np.roll(z, -r))) < 1e-9
    # relinearised product
    w = rng.uniform(-1, 1, P.n)
    cw = ckks.encrypt(P, keys.pk, ckks.encode(w, P.scale, P.N, "ci"), len(P.q), P.scale, 9, 2)
    prod = ckks.rescale(P, ckks.relinearize(P, ckks.tensor(P, ct, cw), keys.rlk))
    assert np.max(np.abs(ckks.decrypt_decode(P, keys.s, prod).real - z * w)) < 1e-9


@pytest.mark.parametrize("d,k,schedule,hoist", [(8, 1, bm.S1, False), (8, 2, bm.S2, False),
                                                (16, 4, bm.S2, False), (16, 4, bm.S2, True)])
def test_ci_match_equals_slot_sim(d, k, schedule, hoist):
    """Blind-Match in the conjugate-invariant ring: N real slots, T = N / c
    templates per ciphertext; every slot equals the simulator."""
    P = tiny_ci(log_n=6)
    rots = set(bm.rotations_needed(P, d, k)) | (set(bm.hoisted_rotations(P, d, k)) if hoist else set())
    keys = ckks.keygen(P, 0xB11D, rotations=sorted(rots))
    rng = np.random.default_rng(d * 7 + k)
    c, T = bm.layout(P, d, k)
    assert T == P.N // c
    R = 2 * T - 1
    X = rng.standard_normal((R, d)) / np.sqrt(d)
    q = rng.standard_normal(d) / np.sqrt(d)
    qslots = bm.pack_query(P, q, d)
    cq = ckks.encrypt(P, keys.pk, ckks.encode(qslots, P.scale, P.N, "ci"), len(P.q), P.scale, 5, 1)
    lg = bm.gallery_limbs(P, k)
    gal_slots = bm.pack_gallery(P, X, d, k)
    gallery = [[ckks.encrypt(P, keys.pk, ckks.encode(v, P.scale, P.N, "ci"), lg, P.scale, 5, 100 + 10 * g + i)
                for i, v in enumerate(parts)] for g, parts in enumerate(gal_slots)]
    masks, mscale = bm.mask_coeffs(P, d, k, len(P.q))
    outs = bm.match(P, keys, cq, gallery, d, k, schedule, masks, mscale, out_limbs=2, hoist=hoist)
    sim_u = slot_sim.expand(qslots, d, k)
    for g, o in outs.items():
        got = ckks.decrypt_decode(P, keys.s, o).real
        assert np.max(np.abs(got - slot_sim.hec3(sim_u, gal_slots[g], d, k))) < 1e-8
