"""Blind-Match on top of the oracle CKKS: packing, Alg. 1 (Input Ciphertext
Expansion), Alg. 2 (HE-C^3), scores and top-1.

TEST INFRASTRUCTURE ONLY (see ckks.py).

Notation follows the paper (Sec. 3.3-3.4): m = d is the feature length,
N_in = k the number of parts, c = m / N_in the chunk length.  Slots are
0-indexed.  Readings of passages the paper leaves open:

  * the query is tiled into every slot, slot s holding q[s mod d];
  * mask_i (Sec. 3.3.1, the redefined mask) is periodic in d with ones where
    floor((s mod d) / c) == i, encoded at scale q_top so that the rescale after
    Mul(P) returns the scale to exactly Delta;
  * Alg. 1 is read 0-indexed: for i < k and t < log2 k, rotate by -c 2^t when
    bit t of i is 0 and by +c 2^t when it is 1, adding after each rotation;
  * the accumulator of Alg. 2 starts as the trivial zero ciphertext;
  * schedule S1 is Alg. 2 as printed (relinearise and rescale every part);
    S2 sums the degree-2 tensors of all parts and relinearises and rescales
    once (same message, different rounding, so different bits).
  * gallery group g, part i, slot s holds x_{g T + floor(s/c)}[i c + s mod c],
    T = n / c templates per group, zeros past the last template; the score of
    template g T + b is read at slot b c of group g's output.
  * compression method (Sec. 3.4, Prop. 3): every group output is multiplied
    by a mask with ones at the score slots b c (encoded at scale q_top of the
    output, so the rescale returns the scale to Delta) and rescaled; then the
    groups of each block of c consecutive groups are merged by halving,
    x_j += Rot(x_{j+H}, -H) for H = P/2, ..., 1 (P the power of two >= the
    block size), so group g lands at slot b c + (g mod c) of compressed
    ciphertext floor(g / c).  One Mul(P), one Rot and one Add per group as
    Prop. 3 counts them; the merge order is this build's reading.
  * minimum-level schedule (an option of this build): every ciphertext is
    first cut, by exact limb drops, to the fewest limbs the rest of the
    computation needs -- the products at EVAL_LIMBS = 3 chain limbs, the
    query one limb more when Alg. 1 runs (its masks then encoded at scale
    q_3), and the accumulator at the output limbs before rotate-and-sum.
    The paper sizes its own modulus chain this way (starting level 3).
"""
import math

import numpy as np

from . import ckks

S1, S2 = 1, 2


def log2_exact(v):
    e = int(v).bit_length() - 1
    if v <= 0 or (1 << e) != v:
        raise ValueError("%d is not a power of two" % v)
    return e


def layout(params, d, k):
    log2_exact(d)
    log2_exact(k)
    if d % k or d > params.n:
        raise ValueError("need k | d and d <= n")
    c = d // k
    T = params.n // c
    return c, T


def rotations_needed(params, d, k):
    """Rotation amounts Alg. 1 and Alg. 2 use for one (d, k) shape."""
    c, _ = layout(params, d, k)
    rots = [1 << t for t in range(log2_exact(c))]
    for t in range(log2_exact(k)):
        rots += [c << t, -(c << t)]
    return rots


def pack_query(params, q, d):
    q = np.asarray(q, dtype=np.float64)
    s = np.arange(params.n)
    return q[s % d]


def pack_gallery(params, X, d, k):
    """List over groups of k slot vectors (real, length n)."""
    X = np.asarray(X, dtype=np.float64)
    R = X.shape[0]
    c, T = layout(params, d, k)
    G = -(-R // T)
    s = np.arange(params.n)
    b, u = s // c, s % c
    groups = []
    for g in range(G):
        parts = []
        for i in range(k):
            tid = g * T + b
            valid = tid < R
            v = np.zeros(params.n)
            v[valid] = X[tid[valid], i * c + u[valid]]
            parts.append(v)
        groups.append(parts)
    return groups


def mask_slots(params, d, k, i):
    c, _ = layout(params, d, k)
    s = np.arange(params.n)
    return ((s % d) // c == i).astype(np.float64)


def mask_coeffs(params, d, k, limbs_query):
    """Integer plaintexts of mask_0..mask_{k-1} at scale q_top of the query."""
    qtop = params.q[limbs_query - 1]
    return [ckks.encode(mask_slots(params, d, k, i), float(qtop), params.N, params.ring) for i in range(k)], \
        float(qtop)


def gallery_limbs(params, k):
    return len(params.q) if k == 1 else len(params.q) - 1


def encrypt_query_coeffs(params, keys, m, seed, ct_id):
    return ckks.encrypt(params, keys.pk, m, len(params.q), params.scale, seed, ct_id)


def expand(params, keys, cq, d, k, masks, mask_scale):
    """Alg. 1: C_i = Res(Mul(P)(C_q, mask_i)), then log2 k rotate-and-add steps."""
    c, _ = layout(params, d, k)
    out = []
    for i in range(k):
        ci = ckks.rescale(params, ckks.pmul(params, cq, masks[i], mask_scale))
        for t in range(log2_exact(k)):
            r = c << t
            step = -r if ((i >> t) & 1) == 0 else r
            ci = ckks.hadd(params, ci, ckks.rotate(params, ci, step, keys.gks))
        out.append(ci)
    return out


def expansion_amounts(params, d, k, i):
    """Rotation amounts of part i once Alg. 1's log2 k steps are unrolled: one
    per non-empty subset S of the steps, sum over t in S of -c 2^t (bit t of i
    is 0) or +c 2^t (bit t of i is 1), in increasing order of the subset mask."""
    c, _ = layout(params, d, k)
    out = []
    for S in range(1, k):
        r = 0
        for t in range(log2_exact(k)):
            if (S >> t) & 1:
                r += (c << t) if (i >> t) & 1 else -(c << t)
        out.append(r)
    return out


def expansion_rotations_hoisted(params, d, k):
    """Rotation amounts the hoisted expansion needs (all parts)."""
    return sorted({r for i in range(k) for r in expansion_amounts(params, d, k, i)})


def expand_hoisted(params, keys, cq, d, k, masks, mask_scale):
    """Alg. 1 with the rotations hoisted (an option of this build): the log2 k
    rotate-and-add steps of part i unroll to Mul(P)(C_q, mask_i) + the sum
    over the non-empty subsets S of its rotations by r_S, evaluated on C_q
    with the mask applied after the key inner products and one ModDown per
    part (ckks.rotation_sum_masked), then Res.  Same message as expand(),
    other bits."""
    if k == 1:
        return [ckks.rescale(params, ckks.pmul(params, cq, masks[0], mask_scale))]
    return [ckks.rescale(params, ckks.rotation_sum_masked(params, cq, masks[i], mask_scale,
                                                          expansion_amounts(params, d, k, i), keys.gks))
            for i in range(k)]


def hec3(params, keys, cu, cs, d, k, schedule, rot_limbs=None, hoist=False):
    """Alg. 2 on one gallery group: accumulate the products of the k parts,
    then log2(c) steps of C_out += Rot(C_out, 2^t).  With rot_limbs the
    accumulator is first cut to that many limbs (exact drop).  With hoist
    (an option of this build) the log2(c) steps are evaluated as the one
    hoisted sum C_out + sum_{r=1}^{c-1} Rot(C_out, r), the same message."""
    c, _ = layout(params, d, k)
    acc = None
    if schedule == S1:
        for i in range(k):
            term = ckks.rescale(params, ckks.relinearize(
                params, ckks.tensor(params, cu[i], cs[i]), keys.rlk))
            acc = term if acc is None else ckks.hadd(params, acc, term)
    elif schedule == S2:
        deg2 = None
        for i in range(k):
            t = ckks.tensor(params, cu[i], cs[i])
            deg2 = t if deg2 is None else ckks.hadd(params, deg2, t)
        acc = ckks.rescale(params, ckks.relinearize(params, deg2, keys.rlk))
    else:
        raise ValueError("schedule")
    if rot_limbs is not None and rot_limbs < acc.limbs:
        acc = ckks.drop_limbs(acc, rot_limbs)
    if hoist:
        return ckks.rotation_sum_hoisted(params, acc, list(range(1, c)), keys.gks) if c > 1 else acc
    for t in range(log2_exact(c)):
        acc = ckks.hadd(params, acc, ckks.rotate(params, acc, 1 << t, keys.gks))
    return acc


def hoisted_rotations(params, d, k):
    """Rotation amounts of the hoisted schedule: 1 .. c-1 and, for k > 1,
    the unrolled Alg. 1 amounts."""
    c, _ = layout(params, d, k)
    r = set(range(1, c))
    if k > 1:
        r.update(expansion_rotations_hoisted(params, d, k))
    return sorted(r)


EVAL_LIMBS = 3


def level_min_shape(params, k, gallery_limbs, compress=False):
    """Limbs of the products and of the expanded query under the minimum-level
    schedule, never above what the inputs carry; compression needs one level
    more."""
    t = min(EVAL_LIMBS + (1 if compress else 0), gallery_limbs)
    return t, (t + 1 if k > 1 else t)


def compress_mask_coeffs(params, d, k, limbs):
    """Integer plaintext of the score mask (ones at slots b c) at scale
    q_{limbs-1}, the top prime of the ciphertexts it multiplies."""
    c, _ = layout(params, d, k)
    s = np.arange(params.n)
    qtop = params.q[limbs - 1]
    return ckks.encode((s % c == 0).astype(np.float64), float(qtop), params.N, params.ring), float(qtop)


def compress(params, keys, outs, d, k, mask, mask_scale):
    """Compression method: list over groups of HE-C^3 outputs -> list over
    blocks of c groups of one ciphertext each (layout in the module notes)."""
    c, _ = layout(params, d, k)
    y = [ckks.rescale(params, ckks.pmul(params, o, mask, mask_scale)) for o in outs]
    res = []
    for o in range(0, len(y), c):
        blk = y[o:o + c]
        r = len(blk)
        half = 1
        while 2 * half < r:
            half *= 2
        while half >= 1 and r > 1:
            for j in range(half):
                if j + half < r:
                    blk[j] = ckks.hadd(params, blk[j], ckks.rotate(params, blk[j + half], -half, keys.gks))
            half //= 2
        res.append(blk[0])
    return res


def enroll_mask_coeffs(params, d, k, limbs):
    """Enrollment masks (Sec. 3.2): mask_i has ones at slots [i c, (i+1) c)
    and zeros elsewhere, as integer plaintexts at scale q_{limbs-1}."""
    c, _ = layout(params, d, k)
    s = np.arange(params.n)
    qtop = params.q[limbs - 1]
    return [ckks.encode(((s >= i * c) & (s < (i + 1) * c)).astype(np.float64), float(qtop), params.N, params.ring)
            for i in range(k)], float(qtop)


def enroll_rotations(params, d, k):
    """Rotation amounts enrollment uses: c 2^t for t < log2(T)."""
    c, T = layout(params, d, k)
    return [c << t for t in range(log2_exact(T))]


def enroll(params, keys, users, indices, d, k, masks, mask_scale, gallery=None):
    """Server-side enrollment (Sec. 3.2, Fig. 3).  users[u] encrypts template u's
    feature vector in slots [0, d) (zeros elsewhere); its identifier
    Index = indices[u] (0-indexed) is position b = Index mod T of group
    g = Index div T.  For every part i: C = Res(Mul(P)(C_u, mask_i)) is rotated
    right by (b - i) c slots -- taken as left rotations by c 2^t for the set
    bits t of (i - b) mod T, ascending -- and added into part i of group g.
    `gallery` maps group -> list of k ciphertexts; missing groups start as the
    trivial zero ciphertext.  Returns the updated mapping."""
    c, T = layout(params, d, k)
    gallery = {} if gallery is None else gallery
    for cu, index in zip(users, indices):
        g, b = divmod(int(index), T)
        for i in range(k):
            x = ckks.rescale(params, ckks.pmul(params, cu, masks[i], mask_scale))
            m = (i - b) % T
            t = 0
            while m >> t:
                if (m >> t) & 1:
                    x = ckks.rotate(params, x, c << t, keys.gks)
                t += 1
            parts = gallery.setdefault(g, [None] * k)
            parts[i] = x if parts[i] is None else ckks.hadd(params, parts[i], x)
    return gallery


def compress_rotations(params, d, k):
    """Rotation amounts the compression merges use: -2^t for t < log2(c)."""
    c, _ = layout(params, d, k)
    return [-(1 << t) for t in range(log2_exact(c))]


def match(params, keys, cq, gallery, d, k, schedule, masks=None, mask_scale=None,
          out_limbs=None, groups=None, level_min=False, compress_mask=None, hoist=False):
    """Whole server side: expansion (k > 1) then HE-C^3 per gallery group.
    `gallery` is a list over groups of k ciphertexts.  Optionally only the
    listed `groups` are evaluated (sampled parity at large sizes).  With
    level_min every input is first cut to the minimum level (see above); the
    masks must then be encoded at scale q_{limbs of the cut query - 1}.
    With compress_mask = (plaintext, scale) the group outputs are compressed
    (all groups; the mask encoded at scale q_{rot limbs - 1}) and a list of
    compressed ciphertexts is returned instead of the dict over groups.
    With hoist the expansion is expand_hoisted() and the rotate-and-sum the
    hoisted sum of hec3()."""
    comp = compress_mask is not None
    if comp and groups is not None:
        raise ValueError("compression needs every group")
    idx = range(len(gallery)) if groups is None else groups
    rot_limbs = None
    g_limbs = gallery[idx[0]][0].limbs
    if not level_min and cq.limbs > g_limbs + (1 if k > 1 else 0):
        cq = ckks.drop_limbs(cq, g_limbs + (1 if k > 1 else 0))   # products at the gallery's level
    if level_min:
        t, ql = level_min_shape(params, k, gallery[0][0].limbs, comp)
        cq = ckks.drop_limbs(cq, ql)
        gallery = {g: [ckks.drop_limbs(x, t) for x in gallery[g]] for g in idx}
        extra = 1 if comp else 0
        rot_limbs = min(out_limbs + extra, t - 1) if out_limbs else t - 1
    if k == 1:
        cu = [cq]
    elif hoist:
        cu = expand_hoisted(params, keys, cq, d, k, masks, mask_scale)
    else:
        cu = expand(params, keys, cq, d, k, masks, mask_scale)
    outs = {}
    for g in idx:
        o = hec3(params, keys, cu, gallery[g], d, k, schedule, rot_limbs, hoist)
        if not comp and out_limbs is not None and out_limbs < o.limbs:
            o = ckks.drop_limbs(o, out_limbs)
        outs[g] = o
    if not comp:
        return outs
    res = compress(params, keys, [outs[g] for g in idx], d, k, *compress_mask)
    if out_limbs is not None:
        res = [ckks.drop_limbs(x, out_limbs) if out_limbs < x.limbs else x for x in res]
    return res


def compressed_rot_limbs(params, k, gallery_limbs, out_limbs=None, level_min=False):
    """Limbs of the HE-C^3 outputs that the compression mask multiplies."""
    if level_min:
        t, _ = level_min_shape(params, k, gallery_limbs, True)
        return min(out_limbs + 1, t - 1) if out_limbs else t - 1
    return gallery_limbs - 1


def scores_from_slots(params, slots_by_group, d, k, R):
    """Template g T + b is scored at slot b c of group g."""
    c, T = layout(params, d, k)
    out = np.full(R, np.nan)
    for g, z in slots_by_group.items():
        b = np.arange(T)
        tid = g * T + b
        ok = tid < R
        out[tid[ok]] = np.real(z[b[ok] * c])
    return out


def scores_from_compressed(params, slots_by_ct, d, k, R):
    """Template g T + b is scored at slot b c + (g mod c) of compressed
    ciphertext floor(g / c)."""
    c, T = layout(params, d, k)
    out = np.full(R, np.nan)
    for o, z in enumerate(slots_by_ct):
        for r in range(c):
            g = o * c + r
            b = np.arange(T)
            tid = g * T + b
            ok = tid < R
            out[tid[ok]] = np.real(z[b[ok] * c + r])
    return out


def top1(scores, threshold=None):
    """Index of the largest score (lowest index on ties); -1 if it is below
    the threshold (the client's rejection rule in Sec. 3.5)."""
    s = np.asarray(scores, dtype=np.float64)
    best = int(np.argmax(s))          # argmax returns the first maximal index
    if threshold is not None and s[best] < threshold:
        return -1, float(s[best])
    return best, float(s[best])


# --------------------------------------------------------------------------
# the paper's cost model (Props. 1-3 and F(N_in), Sec. 4)
# --------------------------------------------------------------------------

TABLE1 = {  # Table 1: mean ms per op at N = 8192 for levels 3, 2, 1
    3: dict(Add=0.44, MulC=7.87, MulP=1.25, Rot=7.50, Res=1.30),
    2: dict(Add=0.33, MulC=5.49, MulP=0.97, Rot=5.33, Res=0.95),
    1: dict(Add=0.09, MulC=3.13, MulP=0.76, Rot=2.95, Res=0.60),
}


def cost_F(n_in, m=128, m_prime=32, l=3, table=TABLE1):
    """F(N_in): Prop. 1 (expansion) at levels l and l-1, Prop. 2 (HE-C^3) at
    l-1 and l-2, Prop. 3 (compression) at l-2, as the combined formula of
    Sec. 4 writes them."""
    T = table
    lg = math.log2
    groups = math.ceil(m_prime / n_in)
    exp_t = n_in * ((T[l]["MulP"] + T[l]["Res"]) + lg(n_in) * (T[l - 1]["Rot"] + T[l - 1]["Add"]))
    hec3_t = groups * (n_in * (T[l - 1]["MulC"] + T[l - 1]["Res"] + T[l - 2]["Add"])
                       + (lg(m) - lg(n_in)) * (T[l - 2]["Rot"] + T[l - 2]["Add"]))
    comp_t = groups * (T[l - 2]["MulP"] + T[l - 2]["Rot"] + T[l - 2]["Add"])
    return exp_t + hec3_t + comp_t
