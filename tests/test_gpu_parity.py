"""GPU parity: every ciphertext word the library produces equals the oracle's.

Inputs (plaintext coefficients, ciphertext words, masks) are produced by the
oracle or the seeded generators and imported into the library through the C
ABI; outputs are exported in the coefficient domain and compared word by word
(exact integer arithmetic: the bar is bit-exactness).  Decrypted scores are
compared with the FP64 cosine (1e-4).
"""
import numpy as np
import pytest

from gpu_common import (SEED, lib_ctx, lib_keys, oracle_keys, all_rotations, face_rotations, ct_words,
                        assert_words_equal, log, C2_SHAPES)
from oracle import ckks, blindmatch as obm
from workloads import tiny_gallery, face_gallery

pytestmark = pytest.mark.gpu

C1_SHAPES = [(16, 1), (16, 2), (16, 4), (8, 8), (4, 1)]


@pytest.fixture(scope="module")
def bm():
    import paper_2408_06167_amd as bm
    return bm


def setup(preset):
    rots = all_rotations(1, C1_SHAPES) if preset == 1 else face_rotations(preset)
    P, okeys = oracle_keys(preset, rots)
    ctx = lib_ctx(preset)
    sk, pk, evk = lib_keys(preset, rots)
    return P, okeys, ctx, sk, pk, evk


def fill_words(rng, q, n, fill="random"):
    """Residues mod q: uniform, all q - 1 (the largest operands the FP64
    arithmetic meets), or a random mix of 0 and q - 1."""
    if fill == "max":
        return np.full(n, q - 1, dtype=np.uint64)
    if fill == "mixed":
        return np.where(rng.random(n) < 0.5, 0, q - 1).astype(np.uint64)
    return rng.integers(0, q, n, dtype=np.uint64)


def random_ct(P, rng, limbs, comps=2, fill="random"):
    return np.stack([np.stack([fill_words(rng, q, P.N, fill) for q in P.q[:limbs]]) for _ in range(comps)])


# ------------------------------------------------------------------ NTT (row a1)

def library_psi(q, N):
    """The device NTT's root: psi = g^((q-1)/2N), g the least generator of Z_q^*."""
    m, fac = q - 1, []
    f = 2
    while f * f <= m:
        if m % f == 0:
            fac.append(f)
            while m % f == 0:
                m //= f
        f += 1 if f == 2 else 2
    if m > 1:
        fac.append(m)
    g = 2
    while any(pow(g, (q - 1) // p, q) == 1 for p in fac):
        g += 1
    return pow(g, (q - 1) // (2 * N), q)


def brv(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2)


@pytest.mark.parametrize("preset", [1, 2])
def test_ntt_is_negacyclic_evaluation(bm, preset):
    """Forward NTT position j holds a(psi^(2 brv(j) + 1)) (sampled positions,
    evaluated with Python integers); inverse restores every word."""
    import torch
    P = ckks.Params.preset(preset)
    ctx = lib_ctx(preset)
    primes = P.q + P.p
    rng = np.random.default_rng(preset)
    host = np.stack([rng.integers(0, q, P.N, dtype=np.uint64) for q in primes])
    dev = torch.from_numpy(host.view(np.int64).copy()).cuda()
    log("ntt preset %d: %d limbs of N=%d" % (preset, len(primes), P.N))
    bm.bm_ntt(ctx, dev.data_ptr(), 1, list(range(len(primes))), inverse=False)
    torch.cuda.synchronize()
    fwd = dev.cpu().numpy().view(np.uint64)
    logn = P.log_n
    for li, q in enumerate(primes):
        psi = library_psi(q, P.N)
        a = [int(v) for v in host[li]]
        for j in rng.integers(0, P.N, 3):
            j = int(j)
            e = 2 * brv(j, logn) + 1
            w = pow(psi, e, q)
            acc, pw = 0, 1
            for coef in a:
                acc += coef * pw
                pw = pw * w % q
            assert int(fwd[li, j]) == acc % q, "prime %d position %d" % (li, j)
    bm.bm_ntt(ctx, dev.data_ptr(), 1, list(range(len(primes))), inverse=True)
    torch.cuda.synchronize()
    assert_words_equal(dev.cpu().numpy().view(np.uint64), host, "inverse(forward(a))")


@pytest.mark.parametrize("fill", ["max", "mixed"])
def test_ntt_extreme_words(bm, fill):
    """N = 2^16, every chain and special prime: polynomials of all q - 1 (and a
    mix of 0 and q - 1) through the forward transform (sampled positions
    against Python-integer evaluation) and back (every word)."""
    import torch
    P = ckks.Params.preset(2)
    ctx = lib_ctx(2)
    primes = P.q + P.p
    rng = np.random.default_rng(17)
    host = np.stack([fill_words(rng, q, P.N, fill) for q in primes])
    dev = torch.from_numpy(host.view(np.int64).copy()).cuda()
    log("ntt extreme words (%s)" % fill)
    bm.bm_ntt(ctx, dev.data_ptr(), 1, list(range(len(primes))), inverse=False)
    torch.cuda.synchronize()
    fwd = dev.cpu().numpy().view(np.uint64)
    for li, q in enumerate(primes):
        psi = library_psi(q, P.N)
        a = [int(v) for v in host[li]]
        for j in (0, P.N - 1, int(rng.integers(P.N))):
            w = pow(psi, 2 * brv(j, P.log_n) + 1, q)
            acc, pw = 0, 1
            for coef in a:
                acc += coef * pw
                pw = pw * w % q
            assert int(fwd[li, j]) == acc % q, "prime %d position %d" % (li, j)
    bm.bm_ntt(ctx, dev.data_ptr(), 1, list(range(len(primes))), inverse=True)
    torch.cuda.synchronize()
    assert_words_equal(dev.cpu().numpy().view(np.uint64), host, "inverse(forward(a))")


# ------------------------------------------------------------------ keys and encryption

@pytest.mark.parametrize("preset", [1, 2])
def test_keys_bit_exact(bm, preset):
    P, okeys, ctx, sk, pk, evk = setup(preset)
    log("keys preset %d" % preset)
    assert np.array_equal(bm.bm_sk_export(sk, P.N), okeys.s)
    for comp in (0, 1):
        assert_words_equal(bm.bm_pk_export(ctx, pk, comp, P.L + 1, P.N), okeys.pk[comp], "pk[%d]" % comp)
    nprimes = len(P.q) + len(P.p)
    for j in range(P.dnum):
        assert_words_equal(bm.bm_evk_export(ctx, evk, 0, j, 0, nprimes, P.N), okeys.rlk.b[j], "rlk.b[%d]" % j)
        assert_words_equal(bm.bm_evk_export(ctx, evk, 0, j, 1, nprimes, P.N), okeys.rlk.a[j], "rlk.a[%d]" % j)
    g = sorted(okeys.gks)[-1]
    for j in range(P.dnum):
        assert_words_equal(bm.bm_evk_export(ctx, evk, g, j, 0, nprimes, P.N), okeys.gks[g].b[j], "gk.b")
        assert_words_equal(bm.bm_evk_export(ctx, evk, g, j, 1, nprimes, P.N), okeys.gks[g].a[j], "gk.a")


@pytest.mark.parametrize("preset,limbs", [(1, 3), (1, 2), (2, 8), (2, 7)])
def test_encrypt_bit_exact(bm, preset, limbs):
    P, okeys, ctx, sk, pk, evk = setup(preset)
    rng = np.random.default_rng(limbs)
    z = rng.uniform(-1, 1, P.n)
    m = ckks.encode(z, P.scale, P.N)
    want = ckks.encrypt(P, okeys.pk, m, limbs, P.scale, SEED, 77 + limbs)
    ct = bm.bm_encrypt_coeffs(ctx, pk, m, limbs, P.scale, SEED, 77 + limbs)
    got, scale = bm.bm_ct_export(ctx, ct, P.N)
    assert scale == want.scale
    assert_words_equal(got, ct_words(want), "encrypt")
    dec = bm.bm_decrypt_slots(ctx, sk, ct, P.n)
    assert np.max(np.abs(dec - z)) < 1e-6
    bm.bm_ct_free(ct)


@pytest.mark.parametrize("preset", [1, 2])
def test_encode_within_one(bm, preset):
    P = ckks.Params.preset(preset)
    ctx = lib_ctx(preset)
    rng = np.random.default_rng(5)
    z = rng.uniform(-1, 1, P.n)
    got = bm.bm_encode(ctx, z, P.scale)
    want = ckks.encode(z, P.scale, P.N)
    assert np.max(np.abs(got - want)) <= 1


# ------------------------------------------------------------------ primitive operations (a2-a4, a6)

@pytest.mark.parametrize("preset,limbs,fill", [(1, 3, "random"), (1, 2, "random"), (2, 8, "random"),
                                               (2, 7, "random"), (2, 3, "random"), (2, 8, "max"), (2, 3, "max"),
                                               (2, 4, "mixed"), (1, 3, "max")])
def test_ops_bit_exact(bm, preset, limbs, fill):
    """Every primitive op word for word against the oracle; `max` fills every
    word with q - 1 and `mixed` with 0 or q - 1, the extremes the FP64
    arithmetic of the transforms and key inner products is bounded for."""
    P, okeys, ctx, sk, pk, evk = setup(preset)
    rng = np.random.default_rng(100 + limbs)
    log("ops preset %d limbs %d fill %s" % (preset, limbs, fill))
    a_w, b_w = random_ct(P, rng, limbs, fill=fill), random_ct(P, rng, limbs, fill=fill)
    sa = sb = P.scale
    oa, ob = ckks.Ciphertext(list(a_w), limbs, sa), ckks.Ciphertext(list(b_w), limbs, sb)
    la, lb = bm.bm_ct_import(ctx, a_w, sa), bm.bm_ct_import(ctx, b_w, sb)
    handles = [la, lb]

    def check(h, want, what):
        got, scale = bm.bm_ct_export(ctx, h, P.N)
        assert scale == want.scale, what
        assert_words_equal(got, ct_words(want), what)
        handles.append(h)

    check(bm.bm_op_add(ctx, la, lb), ckks.hadd(P, oa, ob), "add")
    t_o = ckks.tensor(P, oa, ob)
    t_l = bm.bm_op_tensor(ctx, la, lb)
    check(t_l, t_o, "tensor")
    check(bm.bm_op_relin(ctx, evk, t_l), ckks.relinearize(P, t_o, okeys.rlk), "relin")
    check(bm.bm_op_rescale(ctx, la), ckks.rescale(P, oa), "rescale")
    for r in (1, 2, -8 if preset == 1 else -16):
        check(bm.bm_op_rotate(ctx, evk, la, r), ckks.rotate(P, oa, r, okeys.gks), "rotate %d" % r)
    pt = ckks.encode(rng.uniform(-1, 1, P.n), 2.0 ** 20, P.N)
    check(bm.bm_op_pmul(ctx, la, pt, 2.0 ** 20), ckks.pmul(P, oa, pt, 2.0 ** 20), "pmul")
    check(bm.bm_op_drop(ctx, la, 1), ckks.drop_limbs(oa, 1), "drop")
    for h in handles:
        bm.bm_ct_free(h)


def test_op_errors(bm):
    P, okeys, ctx, sk, pk, evk = setup(1)
    rng = np.random.default_rng(1)
    a = bm.bm_ct_import(ctx, random_ct(P, rng, 3), P.scale)
    b = bm.bm_ct_import(ctx, random_ct(P, rng, 2), P.scale)
    c = bm.bm_ct_import(ctx, random_ct(P, rng, 3), 2 * P.scale)
    with pytest.raises(bm.BMError) as e:
        bm.bm_op_add(ctx, a, b)
    assert e.value.code == bm.BM_ELEVEL
    with pytest.raises(bm.BMError) as e:
        bm.bm_op_add(ctx, a, c)
    assert e.value.code == bm.BM_ESCALE
    with pytest.raises(bm.BMError) as e:
        bm.bm_op_rotate(ctx, evk, a, 1001)          # no key for this amount
    assert e.value.code == bm.BM_ENOKEY
    one = bm.bm_op_drop(ctx, a, 1)
    with pytest.raises(bm.BMError) as e:
        bm.bm_op_rescale(ctx, one)
    assert e.value.code == bm.BM_ELEVEL
    for h in (a, b, c, one):
        bm.bm_ct_free(h)


# ------------------------------------------------------------------ Blind-Match (a5-a8)

def oracle_gallery_words(P, okeys, X, d, k, seed_base):
    lg = obm.gallery_limbs(P, k)
    groups = obm.pack_gallery(P, X, d, k)
    cts = [[ckks.encrypt(P, okeys.pk, ckks.encode(v, P.scale, P.N), lg, P.scale, SEED,
                         seed_base + g * k + i) for i, v in enumerate(parts)]
           for g, parts in enumerate(groups)]
    words = np.stack([np.stack([ct_words(c) for c in parts]) for parts in cts])
    return cts, words, lg


@pytest.mark.parametrize("d,k", [(d, k) for d, k in C1_SHAPES if k > 1])   # k = 1 has no expansion
def test_expand_bit_exact(bm, d, k):
    P, okeys, ctx, sk, pk, evk = setup(1)
    rng = np.random.default_rng(d * 10 + k)
    q = rng.standard_normal(d)
    m = ckks.encode(obm.pack_query(P, q, d), P.scale, P.N)
    cq_o = ckks.encrypt(P, okeys.pk, m, len(P.q), P.scale, SEED, 5)
    masks, mscale = obm.mask_coeffs(P, d, k, len(P.q))
    want = obm.expand(P, okeys, cq_o, d, k, masks, mscale)
    cq = bm.bm_ct_import(ctx, ct_words(cq_o), P.scale)
    lm = bm.bm_masks_import(ctx, d, k, np.stack(masks), mscale)
    outs = bm.bm_expand(ctx, evk, cq, lm, k)
    for i in range(k):
        got, scale = bm.bm_ct_export(ctx, outs[i], P.N)
        assert scale == want[i].scale
        assert_words_equal(got, ct_words(want[i]), "expanded part %d" % i)
        bm.bm_ct_free(outs[i])
    bm.bm_masks_free(lm)
    bm.bm_ct_free(cq)


@pytest.mark.parametrize("d,k,schedule", [(16, 1, 1), (16, 2, 1), (16, 2, 2), (16, 4, 1),
                                          (16, 4, 2), (8, 8, 2), (16, 1, 0x101), (16, 4, 0x102)])
def test_match_small_ring_bit_exact(bm, d, k, schedule):
    """N = 2^12: a two-group gallery with a ragged last group."""
    P, okeys, ctx, sk, pk, evk = setup(1)
    w = tiny_gallery(seed=1, d=d)
    c, T = obm.layout(P, d, k)
    R = T + T // 2
    rng = np.random.default_rng(3)
    X = np.concatenate([w["gallery"], rng.standard_normal((R, d)).astype(np.float32)])[:R]
    X = X / np.linalg.norm(X, axis=1, keepdims=True)
    qv = w["query_known"][:d] / np.linalg.norm(w["query_known"][:d])
    log("match N=2^12 d=%d k=%d S%d R=%d" % (d, k, schedule, R))
    m = ckks.encode(obm.pack_query(P, qv, d), P.scale, P.N)
    cq_o = ckks.encrypt(P, okeys.pk, m, len(P.q), P.scale, SEED, 9)
    gal_o, words, lg = oracle_gallery_words(P, okeys, X, d, k, 1000)
    masks, mscale = obm.mask_coeffs(P, d, k, len(P.q)) if k > 1 else (None, None)
    want = obm.match(P, okeys, cq_o, gal_o, d, k, schedule & 0xff, masks, mscale,
                     level_min=bool(schedule & 0x100))
    cq = bm.bm_ct_import(ctx, ct_words(cq_o), P.scale)
    gal = bm.bm_gallery_import(ctx, words, d, k, lg, P.scale, R)
    lm = bm.bm_masks_import(ctx, d, k, np.stack(masks), mscale) if k > 1 else None
    res = bm.bm_match(ctx, evk, cq, gal, lm, schedule=schedule, out_limbs=0)
    G, limbs, scale = bm.bm_result_info(res)
    assert G == len(gal_o)
    for g in range(G):
        got, sc = bm.bm_result_export(ctx, res, g, P.N)
        assert sc == want[g].scale
        assert_words_equal(got, ct_words(want[g]), "group %d" % g)
    allw, sc = bm.bm_result_export_all(ctx, res, P.N)      # every group in one transfer
    assert_words_equal(allw, np.stack([ct_words(want[g]) for g in range(G)]), "all groups")
    scores = bm.bm_decrypt_scores(ctx, sk, res, R)
    cos = X.astype(np.float64) @ qv.astype(np.float64)
    assert np.max(np.abs(scores - cos)) < 1e-4
    assert bm.bm_top1(scores)[0] == int(np.argmax(cos))
    for h in (cq,):
        bm.bm_ct_free(h)
    bm.bm_gallery_free(gal)
    bm.bm_result_free(res)
    if lm:
        bm.bm_masks_free(lm)


# degenerate shapes: d = n (one template fills the ciphertext, the rotate-and-sum
# spans every slot: the textbook sum of all slots), a gallery of one template,
# and k = d (c = 1: no rotate-and-sum, every slot of a part is one coordinate)
DEGENERATE = [(2048, 1, 1, 1), (2048, 1, 1, 0x101), (16, 1, 1, 2), (16, 16, 5, 2), (16, 16, 5, 0x101)]


@pytest.mark.parametrize("d,k,R,schedule", DEGENERATE)
def test_match_degenerate_shapes_bit_exact(bm, d, k, R, schedule):
    P = ckks.Params.preset(1)
    rots = set()
    for d_, k_, _, _ in DEGENERATE:
        rots.update(obm.rotations_needed(P, d_, k_))
    rots = tuple(sorted(rots))
    P, okeys = oracle_keys(1, rots)
    ctx = lib_ctx(1)
    sk, pk, evk = lib_keys(1, rots)
    rng = np.random.default_rng(d + 7 * k + R)
    X = rng.standard_normal((R, d))
    X = X / np.linalg.norm(X, axis=1, keepdims=True)
    qv = X[R // 2] + 0.05 * rng.standard_normal(d)
    qv = qv / np.linalg.norm(qv)
    log("match degenerate d=%d k=%d R=%d S%#x" % (d, k, R, schedule))
    m = ckks.encode(obm.pack_query(P, qv, d), P.scale, P.N)
    cq_o = ckks.encrypt(P, okeys.pk, m, len(P.q), P.scale, SEED, 19)
    gal_o, words, lg = oracle_gallery_words(P, okeys, X, d, k, 3000)
    masks, mscale = obm.mask_coeffs(P, d, k, len(P.q)) if k > 1 else (None, None)
    want = obm.match(P, okeys, cq_o, gal_o, d, k, schedule & 0xff, masks, mscale,
                     level_min=bool(schedule & 0x100))
    cq = bm.bm_ct_import(ctx, ct_words(cq_o), P.scale)
    gal = bm.bm_gallery_import(ctx, words, d, k, lg, P.scale, R)
    lm = bm.bm_masks_import(ctx, d, k, np.stack(masks), mscale) if k > 1 else None
    res = bm.bm_match(ctx, evk, cq, gal, lm, schedule=schedule, out_limbs=0)
    G, limbs, scale = bm.bm_result_info(res)
    assert G == len(gal_o) == 1
    got, sc = bm.bm_result_export(ctx, res, 0, P.N)
    assert sc == want[0].scale
    assert_words_equal(got, ct_words(want[0]), "group 0")
    scores = bm.bm_decrypt_scores(ctx, sk, res, R)
    cos = X @ qv
    assert np.max(np.abs(scores - cos)) < 1e-4
    assert bm.bm_top1(scores)[0] == int(np.argmax(cos))
    bm.bm_ct_free(cq)
    bm.bm_gallery_free(gal)
    bm.bm_result_free(res)
    if lm:
        bm.bm_masks_free(lm)


def test_match_library_encryption_end_to_end(bm):
    """The library's own encode/encrypt of the N = 2^12 workload: scores within
    1e-4 of the FP64 cosine and the known answer found."""
    P, okeys, ctx, sk, pk, evk = setup(1)
    w = tiny_gallery(seed=1)
    X = w["gallery"]
    for qv in (w["query"], w["query_known"]):
        cq = bm.bm_encrypt_query(ctx, pk, qv, SEED, 1)
        gal = bm.bm_encrypt_gallery(ctx, pk, X, 1, SEED, 1000)
        res = bm.bm_match(ctx, evk, cq, gal)
        scores = bm.bm_decrypt_scores(ctx, sk, res, X.shape[0])
        cos = X.astype(np.float64) @ qv.astype(np.float64) / (
            np.linalg.norm(X.astype(np.float64), axis=1) * np.linalg.norm(qv.astype(np.float64)))
        assert np.max(np.abs(scores - cos)) < 1e-4
        assert bm.bm_top1(scores)[0] == int(np.argmax(cos))
        bm.bm_ct_free(cq)
        bm.bm_gallery_free(gal)
        bm.bm_result_free(res)
    assert bm.bm_top1(scores)[0] == w["known"]


def face_groups(G, level_min):
    """Groups the oracle recomputes at N = 2^16: every group of a minimum-level
    schedule (a few seconds each), else the first, a middle and the last."""
    return None if level_min and G <= 8 else sorted({0, G // 2, G - 1})


@pytest.mark.parametrize("k,schedule", [(1, 1), (4, 1), (4, 2), (16, 2), (1, 0x101), (4, 0x102),
                                        (8, 0x102)])
def test_match_face_scale_bit_exact(bm, k, schedule):
    """N = 2^16, 6,144 x 128-dim gallery: the full match runs on the GPU; the
    oracle recomputes every group of the minimum-level schedules and three
    groups (first, middle, last) of the natural-level ones, word for word."""
    P, okeys, ctx, sk, pk, evk = setup(2)
    d = 128
    w = face_gallery(seed=2)
    X = w["gallery"]
    qv = w["query_known"]
    c, T = obm.layout(P, d, k)
    log("match N=2^16 d=128 k=%d S%#x: oracle gallery encryption" % (k, schedule))
    m = ckks.encode(obm.pack_query(P, qv, d), P.scale, P.N)
    cq_o = ckks.encrypt(P, okeys.pk, m, len(P.q), P.scale, SEED, 9)
    gal_o, words, lg = oracle_gallery_words(P, okeys, X, d, k, 5000)
    G = len(gal_o)
    level_min = bool(schedule & 0x100)
    ql = obm.level_min_shape(P, k, lg)[1] if level_min else len(P.q)
    masks, mscale = obm.mask_coeffs(P, d, k, ql) if k > 1 else (None, None)
    cq = bm.bm_ct_import(ctx, ct_words(cq_o), P.scale)
    gal = bm.bm_gallery_import(ctx, words, d, k, lg, P.scale, X.shape[0])
    lm = bm.bm_masks_import(ctx, d, k, np.stack(masks), mscale) if k > 1 else None
    log("library match")
    res = bm.bm_match(ctx, evk, cq, gal, lm, schedule=schedule, out_limbs=2)
    groups = face_groups(G, level_min)
    log("oracle match on groups %s" % ("all %d" % G if groups is None else groups))
    want = obm.match(P, okeys, cq_o, gal_o, d, k, schedule & 0xff, masks, mscale, out_limbs=2,
                     groups=groups, level_min=level_min)
    assert len(want) == (G if groups is None else len(groups))
    for g, o in want.items():
        got, sc = bm.bm_result_export(ctx, res, g, P.N)
        assert sc == o.scale
        assert_words_equal(got, ct_words(o), "group %d" % g)
    scores = bm.bm_decrypt_scores(ctx, sk, res, X.shape[0])
    cos = X.astype(np.float64) @ qv.astype(np.float64)
    assert np.max(np.abs(scores - cos)) < 1e-4
    assert bm.bm_top1(scores)[0] == w["known"]
    bm.bm_ct_free(cq)
    bm.bm_gallery_free(gal)
    bm.bm_result_free(res)
    if lm:
        bm.bm_masks_free(lm)


# Other feature lengths at N = 2^16: the fingerprint workload's 16-dim
# templates (a prefix of its gallery, 2,048 templates per ciphertext, the last
# group ragged) and the batched workload's 64- and 512-dim shapes.
DIMS = [(16, 1, 3 * 2048 + 500, 0x101), (16, 1, 3 * 2048 + 500, 0x501), (16, 1, 2048 + 100, 0x001),
        (64, 2, 2500, 0x102), (64, 2, 2500, 0x502), (512, 16, 1500, 0x102), (512, 16, 1500, 0x502)]


@pytest.mark.parametrize("d,k,R,schedule", DIMS)
def test_match_face_scale_dims_bit_exact(bm, d, k, R, schedule):
    """N = 2^16 at d = 16 (k = 1), 64 (k = 2) and 512 (k = 16): every result
    word of every group equals the oracle's; scores within 1e-4 of the cosine."""
    from workloads import fingerprint_gallery, normalize
    P, okeys, ctx, sk, pk, evk = setup(2)
    if d == 16:
        w = fingerprint_gallery(seed=3, rows=R)
        X, qv = w["gallery"], w["query"]
    else:
        rng = np.random.default_rng(d + R)
        X = normalize(rng.standard_normal((R, d)))
        qv = normalize(X[R // 3] + 0.05 * rng.standard_normal(d))
    c, T = obm.layout(P, d, k)
    log("match N=2^16 d=%d k=%d R=%d schedule %#x: oracle gallery encryption" % (d, k, R, schedule))
    m = ckks.encode(obm.pack_query(P, qv, d), P.scale, P.N)
    cq_o = ckks.encrypt(P, okeys.pk, m, len(P.q), P.scale, SEED, 13)
    gal_o, words, lg = oracle_gallery_words(P, okeys, X, d, k, 7000)
    G = len(gal_o)
    assert G == -(-R // T)
    level_min, hoist = bool(schedule & 0x100), bool(schedule & 0x400)
    ql = obm.level_min_shape(P, k, lg)[1] if level_min else len(P.q)
    masks, mscale = obm.mask_coeffs(P, d, k, ql) if k > 1 else (None, None)
    cq = bm.bm_ct_import(ctx, ct_words(cq_o), P.scale)
    gal = bm.bm_gallery_import(ctx, words, d, k, lg, P.scale, R)
    lm = bm.bm_masks_import(ctx, d, k, np.stack(masks), mscale) if k > 1 else None
    log("library match")
    res = bm.bm_match(ctx, evk, cq, gal, lm, schedule=schedule, out_limbs=2)
    log("oracle match, all %d groups" % G)
    want = obm.match(P, okeys, cq_o, gal_o, d, k, schedule & 0xff, masks, mscale, out_limbs=2,
                     level_min=level_min, hoist=hoist)
    assert sorted(want) == list(range(G))
    for g, o in want.items():
        got, sc = bm.bm_result_export(ctx, res, g, P.N)
        assert sc == o.scale
        assert_words_equal(got, ct_words(o), "group %d" % g)
    scores = bm.bm_decrypt_scores(ctx, sk, res, R)
    cos = X.astype(np.float64) @ qv.astype(np.float64)
    assert np.max(np.abs(scores - cos)) < 1e-4
    assert bm.bm_top1(scores)[0] == int(np.argmax(cos))
    bm.bm_ct_free(cq)
    bm.bm_gallery_free(gal)
    bm.bm_result_free(res)
    if lm:
        bm.bm_masks_free(lm)


# ------------------------------------------------------------------ compression method (Sec. 3.4)

@pytest.mark.parametrize("d,R,schedule", [(16, 300, 0x201), (16, 300, 0x302), (4, 2300, 0x202),
                                          (16, 100, 0x201)])
def test_match_compressed_small_ring_bit_exact(bm, d, R, schedule):
    """N = 2^12, k = 1: every compressed ciphertext word equals the oracle's,
    including a ragged last block (d = 4: c = 4, five groups -> 4 + 1) and a
    single group (mask and rescale only)."""
    P, okeys, ctx, sk, pk, evk = setup(1)
    k = 1
    rng = np.random.default_rng(R + d)
    X = rng.standard_normal((R, d))
    X = (X / np.linalg.norm(X, axis=1, keepdims=True)).astype(np.float32)
    qv = X[R // 3] + 0.05 * rng.standard_normal(d).astype(np.float32)
    qv = qv / np.linalg.norm(qv)
    log("compressed match N=2^12 d=%d R=%d schedule %#x" % (d, R, schedule))
    m = ckks.encode(obm.pack_query(P, qv, d), P.scale, P.N)
    cq_o = ckks.encrypt(P, okeys.pk, m, len(P.q), P.scale, SEED, 19)
    gal_o, words, lg = oracle_gallery_words(P, okeys, X, d, k, 3000)
    level_min = bool(schedule & 0x100)
    rl = obm.compressed_rot_limbs(P, k, lg, level_min=level_min)
    want = obm.match(P, okeys, cq_o, gal_o, d, k, schedule & 0xff, level_min=level_min,
                     compress_mask=obm.compress_mask_coeffs(P, d, k, rl))
    cq = bm.bm_ct_import(ctx, ct_words(cq_o), P.scale)
    gal = bm.bm_gallery_import(ctx, words, d, k, lg, P.scale, R)
    res = bm.bm_match(ctx, evk, cq, gal, None, schedule=schedule, out_limbs=0)
    n_ct, limbs, scale = bm.bm_result_info(res)
    assert n_ct == len(want) == -(-len(gal_o) // (d // k))
    for o in range(n_ct):
        got, sc = bm.bm_result_export(ctx, res, o, P.N)
        assert sc == want[o].scale and limbs == want[o].limbs
        assert_words_equal(got, ct_words(want[o]), "compressed ciphertext %d" % o)
    scores = bm.bm_decrypt_scores(ctx, sk, res, R)
    cos = X.astype(np.float64) @ qv.astype(np.float64)
    assert np.max(np.abs(scores - cos)) < 1e-4
    assert bm.bm_top1(scores)[0] == int(np.argmax(cos))
    bm.bm_ct_free(cq)
    bm.bm_gallery_free(gal)
    bm.bm_result_free(res)


def test_compression_without_a_spare_level_is_rejected(bm):
    P, okeys, ctx, sk, pk, evk = setup(1)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((50, 16)).astype(np.float32)
    q = bm.bm_encrypt_query(ctx, pk, X[0], SEED, 1)
    g = bm.bm_encrypt_gallery(ctx, pk, X, 2, SEED, 10)      # k = 2: gallery at 2 limbs
    with pytest.raises(bm.BMError) as e:
        bm.bm_match(ctx, evk, q, g, None, schedule=2 | bm.BM_COMPRESS)
    assert e.value.code == bm.BM_ELEVEL
    bm.bm_ct_free(q)
    bm.bm_gallery_free(g)


@pytest.mark.parametrize("k,schedule", [(4, 0x302), (8, 0x301)])
def test_match_face_scale_compressed_bit_exact(bm, k, schedule):
    """N = 2^16, 6,144 x 128-dim, compressed at the minimum level: the G
    group outputs fold into one ciphertext; the oracle recomputes all of it."""
    P, okeys, ctx, sk, pk, evk = setup(2)
    d = 128
    w = face_gallery(seed=2)
    X, qv = w["gallery"], w["query_known"]
    log("compressed match N=2^16 k=%d schedule %#x: oracle gallery encryption" % (k, schedule))
    m = ckks.encode(obm.pack_query(P, qv, d), P.scale, P.N)
    cq_o = ckks.encrypt(P, okeys.pk, m, len(P.q), P.scale, SEED, 9)
    gal_o, words, lg = oracle_gallery_words(P, okeys, X, d, k, 5000)
    ql = obm.level_min_shape(P, k, lg, True)[1]
    masks, mscale = obm.mask_coeffs(P, d, k, ql)
    rl = obm.compressed_rot_limbs(P, k, lg, out_limbs=2, level_min=True)
    cq = bm.bm_ct_import(ctx, ct_words(cq_o), P.scale)
    gal = bm.bm_gallery_import(ctx, words, d, k, lg, P.scale, X.shape[0])
    lm = bm.bm_masks_import(ctx, d, k, np.stack(masks), mscale)
    log("library match")
    res = bm.bm_match(ctx, evk, cq, gal, lm, schedule=schedule, out_limbs=2)
    log("oracle match, all %d groups" % len(gal_o))
    want = obm.match(P, okeys, cq_o, gal_o, d, k, schedule & 0xff, masks, mscale, out_limbs=2,
                     level_min=True, compress_mask=obm.compress_mask_coeffs(P, d, k, rl))
    n_ct, limbs, _ = bm.bm_result_info(res)
    assert n_ct == len(want) == 1 and limbs == 2
    got, sc = bm.bm_result_export(ctx, res, 0, P.N)
    assert sc == want[0].scale
    assert_words_equal(got, ct_words(want[0]), "compressed ciphertext")
    scores = bm.bm_decrypt_scores(ctx, sk, res, X.shape[0])
    cos = X.astype(np.float64) @ qv.astype(np.float64)
    assert np.max(np.abs(scores - cos)) < 1e-4
    assert bm.bm_top1(scores)[0] == w["known"]
    bm.bm_ct_free(cq)
    bm.bm_gallery_free(gal)
    bm.bm_result_free(res)
    bm.bm_masks_free(lm)


# ------------------------------------------------------------------ hoisted schedule

@pytest.mark.parametrize("d,k,schedule", [(16, 1, 0x401), (16, 2, 0x402), (16, 4, 0x401), (8, 8, 0x402),
                                          (16, 4, 0x502), (16, 4, 0x501), (16, 1, 0x701), (16, 1, 0x702),
                                          (16, 1, 0x601), (16, 1, 0x602)])
def test_match_hoisted_small_ring_bit_exact(bm, d, k, schedule):
    """N = 2^12, BM_HOIST (with the minimum level and compression too): every
    word equals the oracle's hoisted schedule."""
    P, okeys, ctx, sk, pk, evk = setup(1)
    rng = np.random.default_rng(d * 13 + k + schedule)
    c, T = obm.layout(P, d, k)
    R = T + T // 2
    X = normalize_rows(rng.standard_normal((R, d)))
    qv = X[R // 2] + 0.02 * rng.standard_normal(d)
    qv = qv / np.linalg.norm(qv)
    log("hoisted match N=2^12 d=%d k=%d schedule %#x" % (d, k, schedule))
    m = ckks.encode(obm.pack_query(P, qv, d), P.scale, P.N)
    cq_o = ckks.encrypt(P, okeys.pk, m, len(P.q), P.scale, SEED, 29)
    gal_o, words, lg = oracle_gallery_words(P, okeys, X, d, k, 4000)
    level_min, comp = bool(schedule & 0x100), bool(schedule & 0x200)
    ql = obm.level_min_shape(P, k, lg, comp)[1] if level_min else len(P.q)
    masks, mscale = obm.mask_coeffs(P, d, k, ql) if k > 1 else (None, None)
    cmask = obm.compress_mask_coeffs(P, d, k, obm.compressed_rot_limbs(P, k, lg, level_min=level_min)) \
        if comp else None
    want = obm.match(P, okeys, cq_o, gal_o, d, k, schedule & 0xff, masks, mscale, level_min=level_min,
                     compress_mask=cmask, hoist=True)
    want = want if comp else [want[g] for g in sorted(want)]
    cq = bm.bm_ct_import(ctx, ct_words(cq_o), P.scale)
    gal = bm.bm_gallery_import(ctx, words, d, k, lg, P.scale, R)
    lm = bm.bm_masks_import(ctx, d, k, np.stack(masks), mscale) if k > 1 else None
    res = bm.bm_match(ctx, evk, cq, gal, lm, schedule=schedule, out_limbs=0)
    n_out, limbs, _ = bm.bm_result_info(res)
    assert n_out == len(want)
    for o in range(n_out):
        got, sc = bm.bm_result_export(ctx, res, o, P.N)
        assert sc == want[o].scale
        assert_words_equal(got, ct_words(want[o]), "result %d" % o)
    scores = bm.bm_decrypt_scores(ctx, sk, res, R)
    cos = X.astype(np.float64) @ qv.astype(np.float64)
    assert np.max(np.abs(scores - cos)) < 1e-4
    bm.bm_ct_free(cq)
    bm.bm_gallery_free(gal)
    bm.bm_result_free(res)
    if lm:
        bm.bm_masks_free(lm)


def normalize_rows(X):
    return (X / np.linalg.norm(X, axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("schedule", [0x502, 0x402])
def test_match_face_scale_hoisted_bit_exact(bm, schedule):
    """N = 2^16, 6,144 x 128-dim, k = 4, hoisted (0x502 is the benchmarked
    configuration): every group word for word against the oracle (the six
    groups span all three element groups of the grouped key inner product),
    scores against the cosine."""
    P, okeys, ctx, sk, pk, evk = setup(2)
    d, k = 128, 4
    w = face_gallery(seed=2)
    X, qv = w["gallery"], w["query_known"]
    log("hoisted match N=2^16 k=4 schedule %#x: oracle gallery encryption" % schedule)
    m = ckks.encode(obm.pack_query(P, qv, d), P.scale, P.N)
    cq_o = ckks.encrypt(P, okeys.pk, m, len(P.q), P.scale, SEED, 9)
    gal_o, words, lg = oracle_gallery_words(P, okeys, X, d, k, 5000)
    G = len(gal_o)
    level_min = bool(schedule & 0x100)
    ql = obm.level_min_shape(P, k, lg)[1] if level_min else len(P.q)
    masks, mscale = obm.mask_coeffs(P, d, k, ql)
    cq = bm.bm_ct_import(ctx, ct_words(cq_o), P.scale)
    gal = bm.bm_gallery_import(ctx, words, d, k, lg, P.scale, X.shape[0])
    lm = bm.bm_masks_import(ctx, d, k, np.stack(masks), mscale)
    log("library match")
    res = bm.bm_match(ctx, evk, cq, gal, lm, schedule=schedule, out_limbs=2)
    log("oracle match, all %d groups" % G)
    want = obm.match(P, okeys, cq_o, gal_o, d, k, schedule & 0xff, masks, mscale, out_limbs=2,
                     level_min=level_min, hoist=True)
    assert sorted(want) == list(range(G)) and G == 6
    for g, o in want.items():
        got, sc = bm.bm_result_export(ctx, res, g, P.N)
        assert sc == o.scale
        assert_words_equal(got, ct_words(o), "group %d" % g)
    scores = bm.bm_decrypt_scores(ctx, sk, res, X.shape[0])
    cos = X.astype(np.float64) @ qv.astype(np.float64)
    assert np.max(np.abs(scores - cos)) < 1e-4
    assert bm.bm_top1(scores)[0] == w["known"]
    bm.bm_ct_free(cq)
    bm.bm_gallery_free(gal)
    bm.bm_result_free(res)
    bm.bm_masks_free(lm)


@pytest.mark.parametrize("fill", ["max", "mixed"])
def test_match_extreme_words_face_scale(bm, fill):
    """N = 2^16, k = 4, the benchmarked schedule (0x502): a query and a
    two-group gallery whose every word is q - 1 (or a mix of 0 and q - 1)
    through the expansion, tensor, fused relinearisation and rescale, the
    hoisted key inner products and the fused ModDown: every word equals the
    oracle's (the words decrypt to nothing meaningful; only the arithmetic is
    under test)."""
    P, okeys, ctx, sk, pk, evk = setup(2)
    d, k = 128, 4
    rng = np.random.default_rng(23)
    lg = obm.gallery_limbs(P, k)
    G = 2
    qw = random_ct(P, rng, len(P.q), fill=fill)
    gw = np.stack([np.stack([random_ct(P, rng, lg, fill=fill) for _ in range(k)]) for _ in range(G)])
    cq_o = ckks.Ciphertext(list(qw), len(P.q), P.scale)
    gal_o = [[ckks.Ciphertext(list(gw[g, i]), lg, P.scale) for i in range(k)] for g in range(G)]
    ql = obm.level_min_shape(P, k, lg)[1]
    masks, mscale = obm.mask_coeffs(P, d, k, ql)
    log("extreme-word match (%s)" % fill)
    cq = bm.bm_ct_import(ctx, qw, P.scale)
    gal = bm.bm_gallery_import(ctx, gw, d, k, lg, P.scale, G * obm.layout(P, d, k)[1])
    lm = bm.bm_masks_import(ctx, d, k, np.stack(masks), mscale)
    res = bm.bm_match(ctx, evk, cq, gal, lm, schedule=0x502, out_limbs=2)
    want = obm.match(P, okeys, cq_o, gal_o, d, k, 2, masks, mscale, out_limbs=2, level_min=True, hoist=True)
    for g, o in want.items():
        got, sc = bm.bm_result_export(ctx, res, g, P.N)
        assert sc == o.scale
        assert_words_equal(got, ct_words(o), "group %d" % g)
    bm.bm_ct_free(cq)
    bm.bm_gallery_free(gal)
    bm.bm_result_free(res)
    bm.bm_masks_free(lm)
