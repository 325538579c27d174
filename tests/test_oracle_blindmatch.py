"""Pins of the oracle's Blind-Match layer: the slot simulator, the FP64 cosine,
the paper's packing example and cost-model values."""
import os

import numpy as np
import pytest

import slot_sim
from oracle import ckks, blindmatch as bm
from workloads import tiny_gallery

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny(log_n=6):
    base = ckks.PRESET_PRIMES[2]
    return ckks.Params(log_n=log_n, q=base["q"], p=base["p"], alpha=2, log_scale=50)


# ---------------------------------------------------------------- cost model

def _read_golden():
    table, F = {}, {}
    with open(os.path.join(GOLDEN, "table1_cost_model.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "F":
                F[int(parts[1])] = float(parts[2])
            else:
                lv = int(parts[0])
                table[lv] = dict(zip(["Add", "MulC", "MulP", "Rot", "Res"], map(float, parts[1:])))
    return table, F


def test_cost_model_reproduces_printed_F():
    table, F = _read_golden()
    for n_in, want in F.items():
        assert abs(bm.cost_F(n_in, m=128, m_prime=32, l=3, table=table) - want) < 5e-3
    assert min(F, key=lambda k: bm.cost_F(k, table=table)) == 4


def test_packing_example():
    with open(os.path.join(GOLDEN, "packing_example.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    slots, m, n_in, want = map(int, rows[0])
    # the paper's ring has `slots` real slots; templates per group = slots / (m / N_in)
    assert slots // (m // n_in) == want


# ---------------------------------------------------------------- slot simulator

@pytest.mark.parametrize("d,k", [(8, 1), (8, 2), (8, 4), (8, 8), (16, 4), (32, 16)])
def test_slot_sim_expansion_tiles_chunks(d, k):
    n = 64
    rng = np.random.default_rng(d * 100 + k)
    q = rng.standard_normal(d)
    qs = q[np.arange(n) % d]
    c = d // k
    out = slot_sim.expand(qs, d, k)
    for i in range(k):
        assert np.allclose(out[i], q[i * c + np.arange(n) % c])


@pytest.mark.parametrize("d,k", [(8, 1), (8, 2), (8, 8), (16, 4)])
def test_slot_sim_hec3_gives_inner_products(d, k):
    P = tiny(log_n=7)
    n = P.n
    rng = np.random.default_rng(d + k)
    c, T = bm.layout(P, d, k)
    X = rng.standard_normal((T, d))
    q = rng.standard_normal(d)
    gal = bm.pack_gallery(P, X, d, k)
    assert len(gal) == 1
    acc = slot_sim.hec3(slot_sim.expand(bm.pack_query(P, q, d), d, k), gal[0], d, k)
    for b in range(T):
        assert abs(acc[b * c] - X[b] @ q) < 1e-12


def test_rotations_needed_cover_both_algorithms():
    P = tiny(log_n=7)
    # c = 4: Alg. 2 rotates by 1, 2; Alg. 1 by -+4 and -+8
    assert sorted(bm.rotations_needed(P, 16, 4)) == sorted([1, 2, 4, -4, 8, -8])


# ---------------------------------------------------------------- encrypted vs simulated

@pytest.fixture(scope="module")
def tiny_setup():
    P = tiny(log_n=6)
    rots = set()
    for d, k in [(8, 1), (8, 2), (8, 4), (16, 4), (32, 1)]:
        rots.update(bm.rotations_needed(P, d, k))
    keys = ckks.keygen(P, 0xB11D, rotations=sorted(rots))
    return P, keys


@pytest.mark.parametrize("d,k,schedule", [(8, 1, bm.S1), (8, 2, bm.S1), (8, 2, bm.S2),
                                          (8, 4, bm.S1), (8, 4, bm.S2), (16, 4, bm.S2)])
def test_encrypted_match_equals_slot_sim(tiny_setup, d, k, schedule):
    P, keys = tiny_setup
    rng = np.random.default_rng(d * 7 + k + schedule)
    c, T = bm.layout(P, d, k)
    R = 2 * T - 1                                     # two groups, last one ragged
    X = rng.standard_normal((R, d)) / np.sqrt(d)
    q = rng.standard_normal(d) / np.sqrt(d)
    qslots = bm.pack_query(P, q, d)
    cq = ckks.encrypt(P, keys.pk, ckks.encode(qslots, P.scale, P.N), len(P.q), P.scale, 1, 1)
    lg = bm.gallery_limbs(P, k)
    gal_slots = bm.pack_gallery(P, X, d, k)
    gallery = [[ckks.encrypt(P, keys.pk, ckks.encode(v, P.scale, P.N), lg, P.scale, 1, 100 + 10 * g + i)
                for i, v in enumerate(parts)] for g, parts in enumerate(gal_slots)]
    masks, mscale = bm.mask_coeffs(P, d, k, len(P.q))
    outs = bm.match(P, keys, cq, gallery, d, k, schedule, masks, mscale, out_limbs=2)
    sim_u = slot_sim.expand(qslots, d, k)
    for g, o in outs.items():
        assert o.limbs == 2
        got = ckks.decrypt_decode(P, keys.s, o)
        want = slot_sim.hec3(sim_u, gal_slots[g], d, k)
        assert np.max(np.abs(got - want)) < 1e-8
    scores = bm.scores_from_slots(P, {g: ckks.decrypt_decode(P, keys.s, o) for g, o in outs.items()},
                                  d, k, R)
    assert np.max(np.abs(scores - X @ q)) < 1e-8


@pytest.mark.parametrize("d,k,schedule", [(8, 1, bm.S1), (8, 4, bm.S2), (16, 4, bm.S1)])
def test_minimum_level_match_equals_slot_sim(tiny_setup, d, k, schedule):
    """Minimum-level schedule: products at 3 limbs, query cut to 4 limbs before
    Alg. 1 (masks at scale q_3), rotate-and-sum at the 2 output limbs."""
    P, keys = tiny_setup
    rng = np.random.default_rng(d + 31 * k + schedule)
    c, T = bm.layout(P, d, k)
    R = 2 * T - 3
    X = rng.standard_normal((R, d)) / np.sqrt(d)
    q = rng.standard_normal(d) / np.sqrt(d)
    qslots = bm.pack_query(P, q, d)
    cq = ckks.encrypt(P, keys.pk, ckks.encode(qslots, P.scale, P.N), len(P.q), P.scale, 3, 1)
    lg = bm.gallery_limbs(P, k)
    gal_slots = bm.pack_gallery(P, X, d, k)
    gallery = [[ckks.encrypt(P, keys.pk, ckks.encode(v, P.scale, P.N), lg, P.scale, 3, 300 + 10 * g + i)
                for i, v in enumerate(parts)] for g, parts in enumerate(gal_slots)]
    t, ql = bm.level_min_shape(P, k, lg)
    assert t == 3 and ql == (4 if k > 1 else 3)
    masks, mscale = bm.mask_coeffs(P, d, k, ql)
    outs = bm.match(P, keys, cq, gallery, d, k, schedule, masks, mscale, out_limbs=2, level_min=True)
    sim_u = slot_sim.expand(qslots, d, k)
    for g, o in outs.items():
        assert o.limbs == 2
        got = ckks.decrypt_decode(P, keys.s, o)
        assert np.max(np.abs(got - slot_sim.hec3(sim_u, gal_slots[g], d, k))) < 1e-8


def test_full_vector_inner_product_special_case(tiny_setup):
    """k = 1 and d = n: one template fills the ciphertext and the rotate-and-sum
    is the textbook sum of all slots."""
    P, keys = tiny_setup
    d = P.n
    rng = np.random.default_rng(99)
    x = rng.standard_normal(d) / np.sqrt(d)
    q = rng.standard_normal(d) / np.sqrt(d)
    cq = ckks.encrypt(P, keys.pk, ckks.encode(q, P.scale, P.N), len(P.q), P.scale, 2, 1)
    cx = ckks.encrypt(P, keys.pk, ckks.encode(x, P.scale, P.N), len(P.q), P.scale, 2, 2)
    out = bm.hec3(P, keys, [cq], [cx], d, 1, bm.S1)
    got = ckks.decrypt_decode(P, keys.s, out)
    assert np.max(np.abs(got - np.sum(q * x))) < 1e-8


def test_top1_rules():
    assert bm.top1([0.1, 0.5, 0.5, 0.2]) == (1, 0.5)
    assert bm.top1([0.1, 0.3], threshold=0.4)[0] == -1
    assert bm.top1([0.1, 0.3], threshold=0.3)[0] == 1


# ---------------------------------------------------------------- the N = 2^12 workload

def test_c1_end_to_end_scores_and_top1():
    P = ckks.Params.preset(1)
    w = tiny_gallery(seed=1)
    d, k = 16, 1
    keys = ckks.keygen(P, 0xB11D, rotations=bm.rotations_needed(P, d, k))
    X = w["gallery"].astype(np.float64)
    for qv in (w["query"], w["query_known"]):
        qv = qv.astype(np.float64)
        cq = ckks.encrypt(P, keys.pk, ckks.encode(bm.pack_query(P, qv, d), P.scale, P.N),
                          len(P.q), P.scale, 0xB11D, 1)
        gal = bm.pack_gallery(P, X, d, k)
        assert len(gal) == 1
        gallery = [[ckks.encrypt(P, keys.pk, ckks.encode(gal[0][0], P.scale, P.N), len(P.q),
                                 P.scale, 0xB11D, 1000)]]
        outs = bm.match(P, keys, cq, gallery, d, k, bm.S1)
        assert outs[0].limbs == 2
        z = {0: ckks.decrypt_decode(P, keys.s, outs[0])}
        scores = bm.scores_from_slots(P, z, d, k, X.shape[0])
        cos = (X @ qv) / (np.linalg.norm(X, axis=1) * np.linalg.norm(qv))
        assert np.max(np.abs(scores - cos)) < 1e-4
        assert bm.top1(scores)[0] == int(np.argmax(cos))
    assert bm.top1(scores)[0] == w["known"]


# ---------------------------------------------------------------- compression method

def _compressed_want(P, X, q, d, k, n_ct):
    """Closed form of the compressed layout: slot b c + r of ciphertext o holds
    <q, x_t> for t = (o c + r) T + b when that template exists, 0 elsewhere."""
    c, T = bm.layout(P, d, k)
    R = X.shape[0]
    want = np.zeros((n_ct, P.n))
    for o in range(n_ct):
        for r in range(c):
            for b in range(T):
                t = (o * c + r) * T + b
                if t < R:
                    want[o, b * c + r] = X[t] @ q
    return want


@pytest.mark.parametrize("d,k,schedule,level_min,groups", [(8, 1, bm.S1, False, 11), (8, 2, bm.S2, False, 5),
                                                            (8, 1, bm.S2, True, 8), (4, 2, bm.S1, True, 3),
                                                            (8, 1, bm.S1, False, 1)])
def test_compressed_scores_follow_closed_form_layout(tiny_setup, d, k, schedule, level_min, groups):
    """Compression (Sec. 3.4, Prop. 3): group g's scores land at slot b c + (g mod c)
    of ciphertext floor(g / c) and every other slot is zero."""
    P, keys0 = tiny_setup
    c, T = bm.layout(P, d, k)
    rots = set(bm.rotations_needed(P, d, k)) | set(bm.compress_rotations(P, d, k))
    keys = ckks.keygen(P, 0xB11D, rotations=sorted(rots))
    rng = np.random.default_rng(17 * d + k + groups)
    R = groups * T - (T // 2 if groups > 1 else 0)        # ragged last group
    X = rng.standard_normal((R, d)) / np.sqrt(d)
    q = rng.standard_normal(d) / np.sqrt(d)
    cq = ckks.encrypt(P, keys.pk, ckks.encode(bm.pack_query(P, q, d), P.scale, P.N), len(P.q), P.scale, 5, 1)
    lg = bm.gallery_limbs(P, k)
    gallery = [[ckks.encrypt(P, keys.pk, ckks.encode(v, P.scale, P.N), lg, P.scale, 5, 50 + 10 * g + i)
                for i, v in enumerate(parts)] for g, parts in enumerate(bm.pack_gallery(P, X, d, k))]
    assert len(gallery) == groups
    ql = bm.level_min_shape(P, k, lg, True)[1] if level_min else len(P.q)
    masks, mscale = bm.mask_coeffs(P, d, k, ql)
    rl = bm.compressed_rot_limbs(P, k, lg, out_limbs=2, level_min=level_min)
    cmask = bm.compress_mask_coeffs(P, d, k, rl)
    res = bm.match(P, keys, cq, gallery, d, k, schedule, masks, mscale, out_limbs=2,
                   level_min=level_min, compress_mask=cmask)
    n_ct = -(-groups // c)
    assert len(res) == n_ct
    want = _compressed_want(P, X, q, d, k, n_ct)
    t = bm.level_min_shape(P, k, lg, True)[0] if level_min else lg
    slots = []
    for o, ct in enumerate(res):
        # the mask at scale q_top and its rescale leave the HE-C^3 output scale
        assert ct.limbs == 2 and ct.scale == P.scale * P.scale / P.q[t - 1]
        z = ckks.decrypt_decode(P, keys.s, ct)
        assert np.max(np.abs(z - want[o])) < 1e-7
        slots.append(z)
    scores = bm.scores_from_compressed(P, slots, d, k, R)
    assert np.max(np.abs(scores - X @ q)) < 1e-7


def test_compression_level_rules(tiny_setup):
    P, _ = tiny_setup
    assert bm.level_min_shape(P, 2, 7, compress=True) == (4, 5)
    assert bm.compressed_rot_limbs(P, 2, 7, out_limbs=2, level_min=True) == 3
    assert bm.compressed_rot_limbs(P, 1, 8) == 7
    assert bm.compress_rotations(P, 16, 2) == [-1, -2, -4]


# ---------------------------------------------------------------- server-side enrollment

def _enrolled_want(P, X, indices, d, k, G):
    """Closed form of the stored layout: template Index = g T + b occupies
    slots [b c, (b+1) c) of part i of group g with its chunk i."""
    c, T = bm.layout(P, d, k)
    want = np.zeros((G, k, P.n))
    for x, index in zip(X, indices):
        g, b = divmod(int(index), T)
        for i in range(k):
            want[g, i, b * c:(b + 1) * c] = x[i * c:(i + 1) * c]
    return want


@pytest.mark.parametrize("d,k", [(8, 1), (8, 2), (8, 4), (4, 4), (16, 2)])
def test_enrolled_gallery_follows_closed_form_and_matches(tiny_setup, d, k):
    """Sec. 3.2 / Fig. 3: masked parts rotated right by (Index - i) c and added
    give the packed layout of the gallery (slot by slot), one level below the
    user ciphertexts, and matching it gives the inner products."""
    P, _ = tiny_setup
    c, T = bm.layout(P, d, k)
    rots = set(bm.rotations_needed(P, d, k)) | set(bm.enroll_rotations(P, d, k))
    keys = ckks.keygen(P, 0xB11D, rotations=sorted(rots))
    rng = np.random.default_rng(d * 5 + k)
    G = 2
    indices = rng.permutation(G * T)[: G * T - 1]      # random order, one position left empty
    X = rng.standard_normal((len(indices), d)) / np.sqrt(d)
    top = len(P.q)
    users = []
    for u, x in enumerate(X):
        z = np.zeros(P.n)
        z[:d] = x
        users.append(ckks.encrypt(P, keys.pk, ckks.encode(z, P.scale, P.N), top, P.scale, 7, 500 + u))
    emasks, escale = bm.enroll_mask_coeffs(P, d, k, top)
    gal = bm.enroll(P, keys, users, indices, d, k, emasks, escale)
    assert sorted(gal) == list(range(G))
    want = _enrolled_want(P, X, indices, d, k, G)
    for g in range(G):
        for i in range(k):
            ct = gal[g][i]
            assert ct.limbs == top - 1 and ct.scale == P.scale
            assert np.max(np.abs(ckks.decrypt_decode(P, keys.s, ct) - want[g, i])) < 1e-7
    # match the enrolled gallery: template Index is scored like a packed one
    q = rng.standard_normal(d) / np.sqrt(d)
    cq = ckks.encrypt(P, keys.pk, ckks.encode(bm.pack_query(P, q, d), P.scale, P.N), top, P.scale, 7, 1)
    masks, mscale = bm.mask_coeffs(P, d, k, top) if k > 1 else (None, None)
    outs = bm.match(P, keys, cq, [gal[g] for g in range(G)], d, k, bm.S2, masks, mscale, out_limbs=2)
    scores = bm.scores_from_slots(P, {g: ckks.decrypt_decode(P, keys.s, o) for g, o in outs.items()},
                                  d, k, G * T)
    assert np.max(np.abs(scores[indices] - X @ q)) < 1e-7
    empty = sorted(set(range(G * T)) - set(int(v) for v in indices))
    assert np.max(np.abs(scores[empty])) < 1e-7


def test_enrollment_without_rotation_is_the_masked_part(tiny_setup):
    """Index = i gives no rotation: part i is exactly Res(Mul(P)(C_u, mask_i))."""
    P, keys = tiny_setup
    d, k = 8, 4
    rng = np.random.default_rng(3)
    z = np.zeros(P.n)
    z[:d] = rng.standard_normal(d)
    cu = ckks.encrypt(P, keys.pk, ckks.encode(z, P.scale, P.N), len(P.q), P.scale, 7, 9)
    emasks, escale = bm.enroll_mask_coeffs(P, d, k, len(P.q))
    keys2 = ckks.keygen(P, 0xB11D, rotations=bm.enroll_rotations(P, d, k))
    gal = bm.enroll(P, keys2, [cu], [2], d, k, emasks, escale)
    direct = ckks.rescale(P, ckks.pmul(P, cu, emasks[2], escale))
    assert all(np.array_equal(a, b) for a, b in zip(gal[0][2].c, direct.c))


# ---------------------------------------------------------------- hoisted expansion

def test_expansion_amounts_unroll_alg1():
    """The subsets of Alg. 1's steps give every block shift once: part i of
    k = 4 collects the shifts that move each other chunk position onto it."""
    P = tiny(log_n=7)
    c = 4
    assert bm.expansion_amounts(P, 16, 4, 0) == [-c, -2 * c, -3 * c]
    assert bm.expansion_amounts(P, 16, 4, 3) == [c, 2 * c, 3 * c]
    assert bm.expansion_amounts(P, 16, 4, 1) == [c, -2 * c, -c]
    for k in (2, 4, 8):
        for i in range(k):
            shifts = sorted(r // (16 // k) for r in bm.expansion_amounts(P, 16, k, i))
            assert len(set(shifts)) == k - 1 and 0 not in shifts


@pytest.mark.parametrize("d,k", [(8, 2), (8, 4), (16, 4), (8, 8)])
def test_hoisted_expansion_equals_slot_sim(tiny_setup, d, k):
    P, _ = tiny_setup
    rots = set(bm.expansion_rotations_hoisted(P, d, k))
    keys = ckks.keygen(P, 0xB11D, rotations=sorted(rots))
    rng = np.random.default_rng(d * 3 + k)
    q = rng.standard_normal(d) / np.sqrt(d)
    qslots = bm.pack_query(P, q, d)
    cq = ckks.encrypt(P, keys.pk, ckks.encode(qslots, P.scale, P.N), len(P.q), P.scale, 4, 1)
    masks, mscale = bm.mask_coeffs(P, d, k, len(P.q))
    got = bm.expand_hoisted(P, keys, cq, d, k, masks, mscale)
    want = slot_sim.expand(qslots, d, k)
    for i in range(k):
        assert got[i].limbs == len(P.q) - 1
        assert np.max(np.abs(ckks.decrypt_decode(P, keys.s, got[i]) - want[i])) < 1e-9


def test_hoisted_rotation_sum_single_amount_is_a_rotation(tiny_setup):
    """One amount: x + Rot(x, r) in the slots, and the key-switch error of a
    plain rotation (the two differ only in rounding)."""
    P, keys = tiny_setup
    rng = np.random.default_rng(8)
    z = rng.standard_normal(P.n)
    x = ckks.encrypt(P, keys.pk, ckks.encode(z, P.scale, P.N), 5, P.scale, 4, 2)
    r = max(bm.rotations_needed(P, 8, 2))
    h = ckks.rotation_sum_hoisted(P, x, [r], keys.gks)
    plain = ckks.hadd(P, x, ckks.rotate(P, x, r, keys.gks))
    zh, zp = ckks.decrypt_decode(P, keys.s, h), ckks.decrypt_decode(P, keys.s, plain)
    assert np.max(np.abs(zh - (z + np.roll(z, -r)))) < 1e-9
    assert np.max(np.abs(zh - zp)) < 1e-9


def test_masked_rotation_sum_with_unit_plaintext_is_the_hoisted_sum(tiny_setup):
    """With the plaintext 1 every mask product is the identity, so the masked
    sum must return the words of the (separately pinned) hoisted rotation sum
    exactly: a dropped term, a wrong automorphism or a mask read on the wrong
    primes breaks the equality."""
    P, keys = tiny_setup
    rng = np.random.default_rng(12)
    z = rng.standard_normal(P.n)
    x = ckks.encrypt(P, keys.pk, ckks.encode(z, P.scale, P.N), 5, P.scale, 4, 3)
    amounts = sorted(bm.rotations_needed(P, 8, 2))[:2]
    one = np.zeros(P.N, dtype=np.int64)
    one[0] = 1
    m = ckks.rotation_sum_masked(P, x, one, 1.0, amounts, keys.gks)
    h = ckks.rotation_sum_hoisted(P, x, amounts, keys.gks)
    assert m.limbs == h.limbs and m.scale == h.scale
    assert all(np.array_equal(a, b) for a, b in zip(m.c, h.c))


def test_masked_rotation_sum_is_mask_then_rotations(tiny_setup):
    """Slots: pt z + sum_r Rot(pt z, r); the same message as Mul(P) followed
    by plain rotations, within the key-switch error."""
    P, keys = tiny_setup
    rng = np.random.default_rng(13)
    z = rng.standard_normal(P.n)
    mslots = (rng.random(P.n) < 0.5).astype(np.float64)
    x = ckks.encrypt(P, keys.pk, ckks.encode(z, P.scale, P.N), 5, P.scale, 4, 4)
    qtop = float(P.q[4])
    pt = ckks.encode(mslots, qtop, P.N)
    amounts = sorted(bm.rotations_needed(P, 8, 2))[:2]
    m = ckks.rotation_sum_masked(P, x, pt, qtop, amounts, keys.gks)
    want = mslots * z
    for r in amounts:
        want = want + np.roll(mslots * z, -r)
    assert np.max(np.abs(ckks.decrypt_decode(P, keys.s, m) - want)) < 1e-9
    plain = ckks.pmul(P, x, pt, qtop)
    acc = plain
    for r in amounts:
        acc = ckks.hadd(P, acc, ckks.rotate(P, plain, r, keys.gks))
    assert np.max(np.abs(ckks.decrypt_decode(P, keys.s, m) - ckks.decrypt_decode(P, keys.s, acc))) < 1e-9


@pytest.mark.parametrize("d,k,schedule", [(8, 1, bm.S1), (8, 2, bm.S2), (16, 4, bm.S2), (32, 1, bm.S2)])
def test_hoisted_match_equals_slot_sim(tiny_setup, d, k, schedule):
    """Hoisted schedule: the rotate-and-sum as one hoisted sum of the c - 1
    rotations, the expansion hoisted; every slot equals the simulator."""
    P, _ = tiny_setup
    keys = ckks.keygen(P, 0xB11D, rotations=bm.hoisted_rotations(P, d, k))
    rng = np.random.default_rng(d * 11 + k)
    c, T = bm.layout(P, d, k)
    R = 2 * T - 1
    X = rng.standard_normal((R, d)) / np.sqrt(d)
    q = rng.standard_normal(d) / np.sqrt(d)
    qslots = bm.pack_query(P, q, d)
    cq = ckks.encrypt(P, keys.pk, ckks.encode(qslots, P.scale, P.N), len(P.q), P.scale, 6, 1)
    lg = bm.gallery_limbs(P, k)
    gal_slots = bm.pack_gallery(P, X, d, k)
    gallery = [[ckks.encrypt(P, keys.pk, ckks.encode(v, P.scale, P.N), lg, P.scale, 6, 100 + 10 * g + i)
                for i, v in enumerate(parts)] for g, parts in enumerate(gal_slots)]
    masks, mscale = bm.mask_coeffs(P, d, k, len(P.q))
    outs = bm.match(P, keys, cq, gallery, d, k, schedule, masks, mscale, out_limbs=2, hoist=True)
    sim_u = slot_sim.expand(qslots, d, k)
    for g, o in outs.items():
        got = ckks.decrypt_decode(P, keys.s, o)
        assert np.max(np.abs(got - slot_sim.hec3(sim_u, gal_slots[g], d, k))) < 1e-8
