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
Normals: Box-Muller on word pairs; normal ``d`` of a draw comes from block
``d // 4``; slots (w0, w1) give normals 4b, 4b+1 = r cos, r sin and
(w2, w3) give 4b+2, 4b+3, with r = sqrt(-2 ln U24(w_even)) and the angle
2 pi U24(w_odd).
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


def normals(seed, filter_id, t, a, b, purpose, D):
    """D standard normals per counter (t, a, b), shape broadcast(a, b) + (D,)."""
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
            r = np.sqrt(-2.0 * np.log(u24(w[..., 2 * pair])))
            ang = 2.0 * np.pi * u24(w[..., 2 * pair + 1])
            out[..., d0] = r * np.cos(ang)
            if d0 + 1 < D:
                out[..., d0 + 1] = r * np.sin(ang)
    return out
