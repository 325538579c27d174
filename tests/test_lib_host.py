"""Host-only checks of the C-ABI library: it loads, exports every declared
symbol, and its pure host functions agree with the oracle (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "blindmatch.h")


@pytest.fixture(scope="module")
def bm():
    import paper_2408_06167_amd as bm
    if not os.path.exists(bm.LIB_PATH):
        from paper_2408_06167_amd import build
        build.build()
    return bm


def declared_in_header():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(bm_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree(bm):
    assert declared_in_header() == bm.declared_symbols()


def test_library_exports_every_declared_symbol(bm):
    out = subprocess.run(["nm", "-D", "--defined-only", bm.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [s for s in declared_in_header() if s not in exported]
    assert not missing, missing
    lib = bm.lib()
    for name in declared_in_header():
        assert getattr(lib, name) is not None


def test_presets_follow_the_prime_rule_and_match_the_oracle(bm):
    from oracle import ckks
    for preset in (1, 2, 3, 4):
        p = bm.bm_params_preset(preset)
        o = ckks.Params.preset(preset)
        assert p.log_n == o.log_n
        assert p.chain() == o.q
        assert p.special() == o.p
        assert p.alpha == o.alpha
        assert p.scale == o.scale
        assert p.ring == (bm.BM_RING_CI if o.ring == "ci" else bm.BM_RING_STD)
        assert p.slots == o.n
    with pytest.raises(bm.BMError):
        bm.bm_params_preset(5)


@pytest.mark.parametrize("d,k", [(128, 1), (128, 4), (16, 16), (512, 8)])
def test_rotation_amounts_match_the_oracle(bm, d, k):
    from oracle import ckks, blindmatch as obm
    P = ckks.Params.preset(2)
    assert sorted(bm.bm_rotations_for(d, k)) == sorted(obm.rotations_needed(P, d, k))


def test_rotation_amounts_reject_bad_shapes(bm):
    for d, k in [(100, 1), (128, 3), (8, 16)]:
        with pytest.raises(bm.BMError) as e:
            bm.bm_rotations_for(d, k)
        assert e.value.code == bm.BM_EDIM


def test_top1_rules(bm):
    assert bm.bm_top1([0.1, 0.5, 0.5, 0.2]) == (1, 0.5)
    assert bm.bm_top1([0.1, 0.3], threshold=0.4)[0] == -1
    assert bm.bm_top1([0.1, 0.3], threshold=0.3)[0] == 1
    scores = np.random.default_rng(0).standard_normal(10000)
    assert bm.bm_top1(scores)[0] == int(np.argmax(scores))


def test_strerror(bm):
    lib = bm.lib()
    assert lib.bm_strerror(bm.BM_ENOKEY) == b"missing Galois key"
    assert lib.bm_strerror(12345) == b"unknown status"


def test_null_arguments_are_rejected(bm):
    lib = bm.lib()
    assert lib.bm_params_preset(1, None) == bm.BM_EINVAL
    assert lib.bm_ctx_create(None, 0, None) == bm.BM_EINVAL
    assert lib.bm_top1(None, 0, 0.0, None, None) == bm.BM_EINVAL
    lib.bm_ct_free(None)
    lib.bm_result_free(None)
    lib.bm_server_free(None)
