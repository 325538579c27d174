"""GPU parity at ring degrees other than the presets' 2^12 and 2^16.

Those two sizes run the register-radix FP64 transforms; every other size in
[2^3, 2^16] runs the generic integer transform (one LDS-staged stage at a
time, Shoup products).  N = 8192 is the paper's own ring degree; N = 1024
fits one block.  Parameters follow the presets' rule (the largest primes
below 2^50, 2^40 and 2^51 that are 1 mod 2N), found here with Python
integers; the oracle and the library get the same list.
"""
import numpy as np
import pytest

from gpu_common import SEED, ct_words, assert_words_equal, log
from oracle import ckks, blindmatch as obm
from test_gpu_parity import library_psi, brv, oracle_gallery_words

pytestmark = pytest.mark.gpu


def _is_prime(n):
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
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


def primes_below(bits, M, count):
    out, c = [], ((1 << bits) - 1) // M * M + 1
    while len(out) < count:
        if c < (1 << bits) and _is_prime(c):
            out.append(c)
        c -= M
    return out


@pytest.fixture(scope="module")
def bm():
    import paper_2408_06167_amd as bm
    return bm


_CACHE = {}


def ring(bm, log_n):
    """(oracle params, oracle keys, library context, sk, pk, evk) at N = 2^log_n."""
    if log_n in _CACHE:
        return _CACHE[log_n]
    N = 1 << log_n
    q = primes_below(50, 2 * N, 1) + primes_below(40, 2 * N, 2)
    p = primes_below(51, 2 * N, 1)
    P = ckks.Params(log_n, q, p, 1, 40)
    prm = bm.bm_params_preset(1)
    prm.log_n = log_n
    for i, v in enumerate(q):
        prm.q[i] = v
    prm.p[0] = p[0]
    ctx = bm.bm_ctx_create(prm, 0)
    rots = set()
    for d, k in ((16, 1), (16, 2)):
        rots.update(obm.rotations_needed(P, d, k))
    rots = sorted(rots)
    okeys = ckks.keygen(P, SEED, rots)
    sk, pk, evk = bm.bm_keygen(ctx, SEED, rots)
    _CACHE[log_n] = (P, okeys, ctx, sk, pk, evk)
    return _CACHE[log_n]


@pytest.mark.parametrize("log_n", [10, 13])
def test_generic_ntt_is_negacyclic_evaluation(bm, log_n):
    import torch
    P, okeys, ctx, sk, pk, evk = ring(bm, log_n)
    primes = P.q + P.p
    rng = np.random.default_rng(log_n)
    host = np.stack([rng.integers(0, q, P.N, dtype=np.uint64) for q in primes])
    host[0, :] = primes[0] - 1                       # one limb of extreme words
    dev = torch.from_numpy(host.view(np.int64).copy()).cuda()
    log("generic ntt N=2^%d" % log_n)
    bm.bm_ntt(ctx, dev.data_ptr(), 1, list(range(len(primes))), inverse=False)
    torch.cuda.synchronize()
    fwd = dev.cpu().numpy().view(np.uint64)
    for li, q in enumerate(primes):
        psi = library_psi(q, P.N)
        a = [int(v) for v in host[li]]
        for j in (0, P.N - 1, int(rng.integers(P.N)), int(rng.integers(P.N))):
            w = pow(psi, 2 * brv(j, log_n) + 1, q)
            acc, pw = 0, 1
            for coef in a:
                acc += coef * pw
                pw = pw * w % q
            assert int(fwd[li, j]) == acc % q, "prime %d position %d" % (li, j)
    bm.bm_ntt(ctx, dev.data_ptr(), 1, list(range(len(primes))), inverse=True)
    torch.cuda.synchronize()
    assert_words_equal(dev.cpu().numpy().view(np.uint64), host, "inverse(forward(a))")


@pytest.mark.parametrize("log_n,k,schedule", [(13, 1, 1), (13, 2, 2), (10, 2, 1)])
def test_generic_ring_match_bit_exact(bm, log_n, k, schedule):
    """A whole match (expansion for k = 2, tensor, relinearisation, rescale,
    rotate-and-sum) at N = 2^13 and 2^10: every group word for word against
    the oracle, scores within 1e-4 of the cosine."""
    from workloads import normalize
    P, okeys, ctx, sk, pk, evk = ring(bm, log_n)
    d = 16
    c, T = obm.layout(P, d, k)
    R = T + T // 3
    rng = np.random.default_rng(log_n * 10 + k)
    X = normalize(rng.standard_normal((R, d)))
    qv = normalize(X[R // 2] + 0.05 * rng.standard_normal(d))
    log("generic ring match N=2^%d d=%d k=%d S%d" % (log_n, d, k, schedule))
    m = ckks.encode(obm.pack_query(P, qv, d), P.scale, P.N)
    cq_o = ckks.encrypt(P, okeys.pk, m, len(P.q), P.scale, SEED, 3)
    gal_o, words, lg = oracle_gallery_words(P, okeys, X, d, k, 600)
    masks, mscale = obm.mask_coeffs(P, d, k, len(P.q)) if k > 1 else (None, None)
    want = obm.match(P, okeys, cq_o, gal_o, d, k, schedule, masks, mscale)
    cq = bm.bm_ct_import(ctx, ct_words(cq_o), P.scale)
    gal = bm.bm_gallery_import(ctx, words, d, k, lg, P.scale, R)
    lm = bm.bm_masks_import(ctx, d, k, np.stack(masks), mscale) if k > 1 else None
    res = bm.bm_match(ctx, evk, cq, gal, lm, schedule=schedule, out_limbs=0)
    G, limbs, scale = bm.bm_result_info(res)
    assert G == len(gal_o) == 2
    for g in range(G):
        got, sc = bm.bm_result_export(ctx, res, g, P.N)
        assert sc == want[g].scale
        assert_words_equal(got, ct_words(want[g]), "group %d" % g)
    scores = bm.bm_decrypt_scores(ctx, sk, res, R)
    cos = X.astype(np.float64) @ qv.astype(np.float64)
    assert np.max(np.abs(scores - cos)) < 1e-4
    assert bm.bm_top1(scores)[0] == int(np.argmax(cos))
    bm.bm_ct_free(cq)
    bm.bm_gallery_free(gal)
    bm.bm_result_free(res)
    if lm:
        bm.bm_masks_free(lm)
