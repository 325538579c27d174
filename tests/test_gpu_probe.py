"""GPU: the butterfly issue-rate probe behind the ALU figure of the roofline
computes exact residues (checked against Python integers on sampled threads)
and rejects arguments outside its stated limits."""
import numpy as np
import pytest

from gpu_common import lib_ctx, log

pytestmark = pytest.mark.gpu


def chains(q, seed, x, iters):
    """The 8 (u, v) pairs of thread x after `iters` rounds of
    (u, v) <- (u + v w, u - v w) mod q, in integers."""
    out = []
    for j in range(8):
        u, v, w = (int(seed[j]) + x) % q, (int(seed[8 + j]) + 3 * x) % q, int(seed[16 + j])
        for _ in range(iters):
            t = v * w % q
            u, v = (u + t) % q, (u - t) % q
        out += [u, v]
    return out


@pytest.mark.parametrize("preset,prime", [(1, 0), (1, 3), (2, 0), (2, 9)])
def test_probe_exact(preset, prime):
    import paper_2408_06167_amd as bm
    ctx = lib_ctx(preset)
    p = bm.bm_params_preset(preset)
    q = (p.chain() + p.special())[prime]
    seed = np.random.default_rng(prime + 10 * preset).integers(0, q, size=24, dtype=np.uint64)
    seed[16] = q - 1                      # the largest twiddle
    blocks, iters = 3, 98
    log("modmul probe preset %d prime %d" % (preset, prime))
    ms, words = bm.bm_bench_modmul(ctx, prime, blocks, iters, seed, blocks * 256 * 16)
    assert ms > 0
    words = words.reshape(-1, 16)
    assert np.all(words < np.uint64(q))
    for x in (0, 1, 63, 64, 255, 256, blocks * 256 - 1):
        assert [int(w) for w in words[x]] == chains(q, seed, x, iters), "thread %d" % x


def test_probe_rejects_bad_arguments():
    import paper_2408_06167_amd as bm
    ctx = lib_ctx(1)
    q = bm.bm_params_preset(1).chain()[0]
    seed = np.ones(24, dtype=np.uint64)
    for args in ((99, 1, 2), (0, 0, 2), (0, 1, 3), (0, 1, 0), (0, 70000, 2)):
        with pytest.raises(bm.BMError) as e:
            bm.bm_bench_modmul(ctx, *args, seed)
        assert e.value.code == bm.BM_EINVAL
    bad = seed.copy()
    bad[20] = q
    with pytest.raises(bm.BMError):
        bm.bm_bench_modmul(ctx, 0, 1, 2, bad)
    with pytest.raises(bm.BMError):
        bm.bm_bench_modmul(ctx, 0, 1, 2, seed, 256 * 16 + 1)
