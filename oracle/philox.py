"""Philox4x32-10 and the random-number contract (oracle side, FP64).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The paper does not say how random numbers are drawn.  Both the oracle and the
HIP path therefore implement one counter-based generator from its published
definition: Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11).  A block of four
32-bit words is a pure function of a 2-word key and a 4-word counter:

    key     = (seed_lo32, seed_hi32 XOR filter_id)
    counter = (t, a, b, purpose << 24 | block)

where ``t`` is the time step, ``a`` the outer (or new outer) particle index,
``b`` the inner index, ``purpose`` one of the tags below and ``block`` the
index of the 4-word block within one draw.

Transforms (exact in FP32 and FP64):
    U24(w)      = (2 * (w >> 9) + 1) * 2**-24          in (0, 1)
    U53(w0, w1) = ((w0 << 21) | (w1 >> 11)) * 2**-53    in [0, 1)
    R24(block)  = (2 * v + 1) * 2**-24,                  in (0, 1)
                  v = (w0 & 0x1ff) | (w1 & 0x1ff) << 9 | (w2 & 0x1f) << 18
R24 is the block's remnant uniform: 23 of the low bits that U24 leaves unused.
Normals come from Box-Muller pairs: r = sqrt(-2 ln a), (r cos 2 pi b,
r sin 2 pi b) for two uniforms (a, b).  Within a block, slots (w0, w1) and
(w2, w3) form the pairs (U24(w0), U24(w1)) and (U24(w2), U24(w3)).

Layout of a draw's normals (packed): ten per two blocks.  Normal d = 10 q + r
comes, for r < 8, from block 2q + r // 4 (normals 4 per block in slot order,
cosine first), and for r = 8, 9 from the pair (R24(block 2q), R24(block 2q+1)).
The first eight normals of a draw are therefore those of blocks 0 and 1 in
slot order.  The nested look-ahead estimator's companion draws use the
block-aligned layout instead (normal d from block d // 4, no remnant pairs),
so that one block serves several companions (``normals_blocked``).
"""
import numpy as np

# Multipliers and Weyl key increments of Philox4x32 (Salmon et al. 2011).
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85

MASK32 = np.uint64(0xFFFFFFFF)

# Purpose tags of the counter's top byte.
INIT_X, INIT_Z, LA_X, LA_Z, OUTER_U, CAND_U, INNER_U, NEW_Z = range(8)
DPF_ANC_U, DPF_X, DPF_Z, MDN_U, MDN_X = range(8, 13)
# companion ancestors of the nested look-ahead estimator (one U53 per candidate)
LA_B = 13


def philox4x32_10(ctr, key):
    """Ten Philox4x32 rounds.

    ``ctr``: uint32 array (..., 4); ``key``: uint32 array (..., 2).
    Returns uint32 array (..., 4).  Each round multiplies counter words 0 and
    2 by the two multipliers (full 64-bit products), then forms
    (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is bumped by the Weyl
    constants between rounds.
    """
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (ctr[..., i].copy() for i in range(4))
    k0 = key[..., 0].copy()
    k1 = key[..., 1].copy()
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(PHILOX_W0)) & MASK32
            k1 = (k1 + np.uint64(PHILOX_W1)) & MASK32
        p0 = np.uint64(PHILOX_M0) * c0
        p1 = np.uint64(PHILOX_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
    out = np.stack([c0, c1, c2, c3], axis=-1)
    return out.astype(np.uint32)


def key_of(seed, filter_id):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    lo = seed & 0xFFFFFFFF
    hi = (seed >> 32) ^ (int(filter_id) & 0xFFFFFFFF)
    return np.array([lo, hi], dtype=np.uint32)


def words(seed, filter_id, t, a, b, purpose, block):
    """Philox words for counters (t, a, b, purpose<<24|block), broadcast over a, b."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a, b = np.broadcast_arrays(a, b)
    ctr = np.empty(a.shape + (4,), dtype=np.uint64)
    ctr[..., 0] = np.uint64(int(t) & 0xFFFFFFFF)
    ctr[..., 1] = a
    ctr[..., 2] = b
    ctr[..., 3] = np.uint64(((int(purpose) & 0xFF) << 24) | (int(block) & 0xFFFFFF))
    key = np.broadcast_to(key_of(seed, filter_id), a.shape + (2,))
    return philox4x32_10(ctr, key)


def u24(w):
    """Open-interval uniform from one word: (2*(w>>9)+1) * 2^-24."""
    w = np.asarray(w, dtype=np.uint64)
    return ((w >> np.uint64(9)) * np.uint64(2) + np.uint64(1)).astype(np.float64) * 2.0 ** -24


def u53(w0, w1):
    """53-bit uniform in [0,1) from two words."""
    w0 = np.asarray(w0, dtype=np.uint64)
    w1 = np.asarray(w1, dtype=np.uint64)
    v = (w0 << np.uint64(21)) | (w1 >> np.uint64(11))
    return v.astype(np.float64) * 2.0 ** -53


def uniform53(seed, filter_id, t, a, purpose):
    """The single U53 offset of a resampling / selection draw at (t, a, 0)."""
    w = words(seed, filter_id, t, a, 0, purpose, 0)
    return u53(w[..., 0], w[..., 1])


def uniform53_ab(seed, filter_id, t, a, b, purpose):
    """U53 offset of a draw at counter (t, a, b) (block 0)."""
    w = words(seed, filter_id, t, a, b, purpose, 0)
    return u53(w[..., 0], w[..., 1])


def r24(w):
    """The remnant uniform of a block (words on the last axis): 23 of the
    low bits U24 leaves unused, (2 v + 1) 2^-24."""
    w = np.asarray(w, dtype=np.uint64)
    v = ((w[..., 0] & np.uint64(0x1FF)) | ((w[..., 1] & np.uint64(0x1FF)) << np.uint64(9))
         | ((w[..., 2] & np.uint64(0x1F)) << np.uint64(18)))
    return (v * np.uint64(2) + np.uint64(1)).astype(np.float64) * 2.0 ** -24


def _box_muller(ua, ub):
    r = np.sqrt(-2.0 * np.log(ua))
    ang = 2.0 * np.pi * ub
    return r * np.cos(ang), r * np.sin(ang)


def normals(seed, filter_id, t, a, b, purpose, D):
    """D standard normals per counter (t, a, b) in the packed layout (ten per
    two blocks, see the module text), shape broadcast(a, b) + (D,)."""
    a = np.asarray(a)
    b = np.asarray(b)
    shape = np.broadcast(a, b).shape
    out = np.empty(shape + (D,), dtype=np.float64)
    for q in range((D + 9) // 10):
        base = 10 * q
        blocks = [words(seed, filter_id, t, a, b, purpose, 2 * q + h) if base + 4 * h < D or base + 8 < D
                  else None for h in range(2)]
        for h in range(2):
            w = blocks[h]
            for pair in range(2):
                d0 = base + 4 * h + 2 * pair
                if d0 >= D:
                    continue
                n0, n1 = _box_muller(u24(w[..., 2 * pair]), u24(w[..., 2 * pair + 1]))
                out[..., d0] = n0
                if d0 + 1 < D:
                    out[..., d0 + 1] = n1
        if base + 8 < D:
            n0, n1 = _box_muller(r24(blocks[0]), r24(blocks[1]))
            out[..., base + 8] = n0
            if base + 9 < D:
                out[..., base + 9] = n1
    return out


def normals_blocked(seed, filter_id, t, a, b, purpose, D):
    """D standard normals per counter (t, a, b) in the block-aligned layout:
    normal d from block d // 4, slot pairs as in the packed layout."""
    a = np.asarray(a)
    b = np.asarray(b)
    shape = np.broadcast(a, b).shape
    out = np.empty(shape + (D,), dtype=np.float64)
    for blk in range((D + 3) // 4):
        w = words(seed, filter_id, t, a, b, purpose, blk)
        for pair in range(2):
            d0 = 4 * blk + 2 * pair
            if d0 >= D:
                break
            n0, n1 = _box_muller(u24(w[..., 2 * pair]), u24(w[..., 2 * pair + 1]))
            out[..., d0] = n0
            if d0 + 1 < D:
                out[..., d0 + 1] = n1
    return out
