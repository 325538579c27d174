"""GPU: keys handed over in the coefficient domain (Sec. 3.1: the client sends
the public and evaluation keys to the server) give bit-identical results.

A key set is generated, every key exported (bm_pk_export, bm_evk_export),
imported into new handles (bm_pk_import, bm_evk_import), and the imported
keys must export the same words, encrypt to the same words and produce the
same match words as the generated ones."""
import numpy as np
import pytest

from gpu_common import SEED, lib_ctx, assert_words_equal, log
from workloads import normalize

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bm():
    import paper_2408_06167_amd as bm
    return bm


def export_keys(bm, ctx, pk, evk, p):
    N, L1, npr = p.N, p.n_q, p.n_q + p.n_p
    dnum = -(-p.n_q // p.alpha)
    gal = bm.bm_evk_galois(evk)
    pkw = np.stack([bm.bm_pk_export(ctx, pk, c, L1, N) for c in (0, 1)])
    evw = np.stack([np.stack([np.stack([bm.bm_evk_export(ctx, evk, g, j, c, npr, N) for c in (0, 1)])
                              for j in range(dnum)]) for g in [0] + gal])
    return gal, pkw, evw


@pytest.mark.parametrize("preset,d,k,schedule", [(1, 16, 4, 2), (1, 16, 1, 0x401), (2, 16, 1, 0x101)])
def test_imported_keys_are_bit_identical(bm, preset, d, k, schedule):
    ctx = lib_ctx(preset)
    p = bm.bm_params_preset(preset)
    rots = set(bm.bm_rotations_for(d, k))
    if schedule & bm.BM_HOIST:
        rots.update(bm.bm_rotations_hoisted(d, k))
    sk, pk, evk = bm.bm_keygen(ctx, SEED + 1, sorted(rots))
    log("key export/import preset %d d=%d k=%d" % (preset, d, k))
    gal, pkw, evw = export_keys(bm, ctx, pk, evk, p)
    pk2 = bm.bm_pk_import(ctx, pkw)
    evk2 = bm.bm_evk_import(ctx, gal, evw)
    gal2, pkw2, evw2 = export_keys(bm, ctx, pk2, evk2, p)
    assert gal2 == gal
    assert_words_equal(pkw2, pkw, "re-exported public key")
    assert_words_equal(evw2, evw, "re-exported evaluation key")
    rng = np.random.default_rng(preset * 100 + k)
    X = normalize(rng.standard_normal((p.slots // (d // k) + 37, d)))
    qv = normalize(X[5] + 0.05 * rng.standard_normal(d))
    qa = bm.bm_encrypt_query(ctx, pk, qv, SEED, 3)
    qb = bm.bm_encrypt_query(ctx, pk2, qv, SEED, 3)
    assert_words_equal(bm.bm_ct_export(ctx, qb, p.N)[0], bm.bm_ct_export(ctx, qa, p.N)[0], "query encryption")
    gal_h = bm.bm_encrypt_gallery(ctx, pk2, X, k, SEED, 400)
    ra = bm.bm_match(ctx, evk, qa, gal_h, None, schedule=schedule)
    rb = bm.bm_match(ctx, evk2, qa, gal_h, None, schedule=schedule)
    G, _, _ = bm.bm_result_info(ra)
    for g in range(G):
        assert_words_equal(bm.bm_result_export(ctx, rb, g, p.N)[0], bm.bm_result_export(ctx, ra, g, p.N)[0],
                           "group %d" % g)
    scores = bm.bm_decrypt_scores(ctx, sk, rb, X.shape[0])
    assert np.max(np.abs(scores - X.astype(np.float64) @ qv.astype(np.float64))) < 1e-4
    for h in (ra, rb):
        bm.bm_result_free(h)
    bm.bm_gallery_free(gal_h)
    for h in (qa, qb):
        bm.bm_ct_free(h)
    for f, h in ((bm.bm_sk_free, sk), (bm.bm_pk_free, pk), (bm.bm_evk_free, evk), (bm.bm_pk_free, pk2),
                 (bm.bm_evk_free, evk2)):
        f(h)
