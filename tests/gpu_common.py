"""Shared set-up of the GPU parity tests: one library context per preset, and
the oracle's key set for the same seed.  Oracle inputs are made by the oracle
or by the seeded generators, never by the library."""
import functools
import sys

import numpy as np

from oracle import ckks, blindmatch as obm

SEED = 0xB11D


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def lib_ctx(preset):
    import paper_2408_06167_amd as bm
    return bm.bm_ctx_create(bm.bm_params_preset(preset), 0)


@functools.lru_cache(maxsize=None)
def lib_keys(preset, rots):
    import paper_2408_06167_amd as bm
    return bm.bm_keygen(lib_ctx(preset), SEED, list(rots))


@functools.lru_cache(maxsize=None)
def oracle_keys(preset, rots):
    P = ckks.Params.preset(preset)
    return P, ckks.keygen(P, SEED, list(rots))


# shapes whose hoisted-schedule keys are generated too (c - 1 + unrolled Alg. 1
# keys each; the k = 1, 2 shapes at N = 2^16 would need 63 to 127 more)
HOIST_SHAPES = {1: None, 2: [(128, 4)], 3: None, 4: [(128, 4)]}


# N = 2^16 shapes of the face workload's k sweep, and the other dimensions the
# fingerprint (16) and batched (64, 512) workloads run at
C2_SHAPES = [(128, 1), (128, 2), (128, 4), (128, 8), (128, 16)]
C2_EXTRA_SHAPES = [(16, 1), (64, 2), (512, 16)]


def face_rotations(preset=2):
    """One rotation set for every N = 2^16 parity test, so that one key set
    (oracle and library) serves them all: every key of the k sweep's shapes,
    and the plain and hoisted keys of the other dimensions."""
    P = ckks.Params.preset(preset)
    r = set(all_rotations(preset, C2_SHAPES))
    for d, k in C2_EXTRA_SHAPES:
        r.update(obm.rotations_needed(P, d, k))
        r.update(obm.hoisted_rotations(P, d, k))
    return tuple(sorted(r))


def all_rotations(preset, shapes):
    P = ckks.Params.preset(preset)
    r = set()
    for d, k in shapes:
        r.update(obm.rotations_needed(P, d, k))
        r.update(obm.compress_rotations(P, d, k))
        r.update(obm.enroll_rotations(P, d, k))
        if HOIST_SHAPES[preset] is None or (d, k) in HOIST_SHAPES[preset]:
            r.update(obm.hoisted_rotations(P, d, k))
    return tuple(sorted(r))


def ct_words(ct):
    """Oracle ciphertext -> [comps][limbs][N] uint64."""
    return np.stack(ct.c)


def assert_words_equal(got, want, what):
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, "%s: shape %s vs %s" % (what, got.shape, want.shape)
    bad = np.argwhere(got != want)
    assert bad.size == 0, "%s: %d of %d words differ, first at %s" % (
        what, bad.shape[0], got.size, tuple(bad[0]))
