"""Reference oracle for the Blind-Match CKKS hot path.

TEST INFRASTRUCTURE ONLY.  A plain, slow, obviously correct CPU implementation
that the GPU library is checked against.  Only `tests/`, the smoke check in
`__graft_entry__` and the CPU-baseline leg of `bench.py` may import it; the
library never does, and the oracle imports nothing from the library.

Layout:
  ckks_prims.c   modular arithmetic with u128 `%`, textbook NTT product,
                 SHAKE-256 (FIPS 202) streams and samplers
  prims.py       ctypes wrappers
  ckks.py        CKKS scheme: keys, encrypt/decrypt, encode/decode, Add,
                 Mul(P), tensor, key switch, relinearise, rescale, rotate
  blindmatch.py  packing, Alg. 1, Alg. 2 (schedules S1 and S2), scores,
                 top-1, the paper's cost model F(N_in)

Every oracle function is pinned by `-m "not gpu"` tests against the
mathematics (schoolbook products, hashlib SHAKE-256, direct-sum encoding,
big-integer CRT identities, decryption to the expected slot vectors, the
paper's printed F(N_in) values).  Parity unpinned: ciphertext words against
any external HE library (none is available); encodings exactly on a .5 tie.
"""
