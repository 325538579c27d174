"""GPU parity of server-side enrollment (Sec. 3.2, Fig. 3): user ciphertexts
made by the oracle are enrolled by the library; every stored word equals the
oracle's enrollment, and matching the enrolled gallery scores the users."""
import numpy as np
import pytest

from gpu_common import (SEED, lib_ctx, lib_keys, oracle_keys, all_rotations, face_rotations, ct_words,
                        assert_words_equal, log)
from oracle import ckks, blindmatch as obm
from workloads import face_gallery, normalize

pytestmark = pytest.mark.gpu

C1_SHAPES = [(16, 1), (16, 2), (16, 4), (8, 8), (4, 1)]


@pytest.fixture(scope="module")
def bm():
    import paper_2408_06167_amd as bm
    return bm


def setup(preset):
    rots = all_rotations(preset, C1_SHAPES) if preset == 1 else face_rotations(preset)
    P, okeys = oracle_keys(preset, rots)
    return P, okeys, lib_ctx(preset), lib_keys(preset, rots)


def oracle_users(P, okeys, X, id_base):
    """Oracle encryptions of the templates in slots [0, d) at the top level."""
    out = []
    for u, x in enumerate(X):
        z = np.zeros(P.n)
        z[:x.size] = x
        out.append(ckks.encrypt(P, okeys.pk, ckks.encode(z, P.scale, P.N, P.ring), len(P.q), P.scale, SEED,
                                id_base + u))
    return out


@pytest.mark.parametrize("d,k", [(16, 1), (16, 2), (16, 4), (8, 8)])
def test_enroll_small_ring_bit_exact(bm, d, k):
    """N = 2^12: users enrolled in random order at random identifiers of two
    groups (some positions left empty); every stored word equals the oracle's,
    untouched groups stay zero, and the match scores the enrolled users."""
    P, okeys, ctx, (sk, pk, evk) = setup(1)
    c, T = obm.layout(P, d, k)
    G = 3
    rng = np.random.default_rng(d + 10 * k)
    n_users = min(T + T // 2, 96)                          # the oracle enrolls every user on the CPU
    ids = np.concatenate([[0, T - 1, T, 2 * T - 1],          # both ends of groups 0 and 1
                          rng.choice(np.arange(1, T - 1), n_users // 2 - 2, replace=False),
                          rng.choice(np.arange(T + 1, 2 * T - 1), n_users - n_users // 2 - 2, replace=False)])
    ids = rng.permutation(ids)                              # random order; group 2 stays empty
    X = normalize(rng.standard_normal((ids.size, d))).astype(np.float64)
    log("enroll N=2^12 d=%d k=%d users=%d" % (d, k, ids.size))
    users_o = oracle_users(P, okeys, X, 7000)
    emasks, escale = obm.enroll_mask_coeffs(P, d, k, len(P.q))
    want = obm.enroll(P, okeys, users_o, ids, d, k, emasks, escale)
    users = [bm.bm_ct_import(ctx, ct_words(u), P.scale) for u in users_o]
    gal = bm.bm_gallery_create(ctx, d, k, G * T, len(P.q) - 1)
    lm = bm.bm_masks_import(ctx, d, k, np.stack(emasks), escale)   # integer plaintexts shared
    half = len(users) // 2                                 # two calls: the second adds into the first
    bm.bm_enroll(ctx, evk, gal, users[:half], ids[:half], lm)
    bm.bm_enroll(ctx, evk, gal, users[half:], ids[half:], lm)
    bm.bm_masks_free(lm)
    Gl, limbs, scale = bm.bm_gallery_info(gal)
    assert (Gl, limbs) == (G, len(P.q) - 1) and scale == P.scale
    words = bm.bm_gallery_export(ctx, gal, k, P.N)
    for g in range(G):
        for i in range(k):
            if g in want:
                assert want[g][i].scale == P.scale
                assert_words_equal(words[g, i], ct_words(want[g][i]), "group %d part %d" % (g, i))
            else:
                assert not words[g, i].any(), "untouched group %d is not zero" % g
    # match the enrolled gallery
    qv = normalize(X[3] + 0.01 * rng.standard_normal(d))
    cq = bm.bm_encrypt_query(ctx, pk, qv, SEED, 1)
    res = bm.bm_match(ctx, evk, cq, gal, None, schedule=2, out_limbs=0)
    scores = bm.bm_decrypt_scores(ctx, sk, res, G * T)
    assert np.max(np.abs(scores[ids] - X @ qv.astype(np.float64))) < 1e-4
    empty = np.setdiff1d(np.arange(G * T), ids)
    assert np.max(np.abs(scores[empty])) < 1e-4
    assert bm.bm_top1(scores)[0] == ids[3]
    for h in users + [cq]:
        bm.bm_ct_free(h)
    bm.bm_result_free(res)
    bm.bm_gallery_free(gal)


def test_enroll_rejects_bad_input(bm):
    P, okeys, ctx, (sk, pk, evk) = setup(1)
    gal = bm.bm_gallery_create(ctx, 16, 2, 100, len(P.q) - 1)
    u = bm.bm_encrypt_template(ctx, pk, np.ones(16, dtype=np.float32) / 4, SEED, 1)
    with pytest.raises(bm.BMError) as e:
        bm.bm_enroll(ctx, evk, gal, [u], [100])
    assert e.value.code == bm.BM_EINVAL
    low = bm.bm_op_drop(ctx, u, len(P.q) - 1)
    with pytest.raises(bm.BMError) as e:
        bm.bm_enroll(ctx, evk, gal, [low], [0])
    assert e.value.code == bm.BM_ELEVEL
    for h in (u, low):
        bm.bm_ct_free(h)
    bm.bm_gallery_free(gal)


def test_enroll_face_scale(bm):
    """N = 2^16, k = 4: the first 2,048 face-scale templates (two full groups)
    enrolled by the library from its own user ciphertexts; three users are
    re-enrolled by the oracle from the same words and compared word for word,
    and the match finds a noisy copy of template 1234 with scores within 1e-4
    of the cosine."""
    P, okeys, ctx, (sk, pk, evk) = setup(2)
    d, k = 128, 4
    c, T = obm.layout(P, d, k)
    n = 2 * T
    X = face_gallery(seed=2)["gallery"][:n]
    qv = normalize(X[1234] + 0.05 * np.random.default_rng(4).standard_normal(d))
    log("enroll N=2^16: library encryption of %d users" % n)
    users = [bm.bm_encrypt_template(ctx, pk, X[u], SEED, 20000 + u) for u in range(n)]
    gal = bm.bm_gallery_create(ctx, d, k, n, len(P.q) - 1)
    log("library enrollment")
    bm.bm_enroll(ctx, evk, gal, users, np.arange(n))
    G, limbs, _ = bm.bm_gallery_info(gal)
    cq = bm.bm_encrypt_query(ctx, pk, qv, SEED, 1)
    res = bm.bm_match(ctx, evk, cq, gal, None, schedule=2 | bm.BM_LEVEL_MIN, out_limbs=2)
    scores = bm.bm_decrypt_scores(ctx, sk, res, n)
    cos = X.astype(np.float64) @ qv.astype(np.float64)
    assert np.max(np.abs(scores - cos)) < 1e-4
    assert bm.bm_top1(scores)[0] == 1234
    # oracle re-enrollment of three users into a fresh group from the same words
    log("oracle enrollment of three users")
    picks = [0, 1023, 1249]
    users_o = []
    for u in picks:
        words = bm.bm_ct_export(ctx, users[u], P.N)[0]
        users_o.append(ckks.Ciphertext([words[0].copy(), words[1].copy()], len(P.q), P.scale))
    emasks, escale = obm.enroll_mask_coeffs(P, d, k, len(P.q))
    want = obm.enroll(P, okeys, users_o, picks, d, k, emasks, escale)
    lone = bm.bm_gallery_create(ctx, d, k, n, len(P.q) - 1)
    lm = bm.bm_masks_import(ctx, d, k, np.stack(emasks), escale)   # integer plaintexts shared
    bm.bm_enroll(ctx, evk, lone, [users[u] for u in picks], picks, lm)
    bm.bm_masks_free(lm)
    lw = bm.bm_gallery_export(ctx, lone, k, P.N)
    for g, parts in want.items():
        for i in range(k):
            assert_words_equal(lw[g, i], ct_words(parts[i]), "group %d part %d" % (g, i))
    for h in users + [cq]:
        bm.bm_ct_free(h)
    bm.bm_result_free(res)
    bm.bm_gallery_free(gal)
    bm.bm_gallery_free(lone)
