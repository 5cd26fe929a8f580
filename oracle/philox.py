"""Philox-4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), written from its
published definition with numpy uint64 arithmetic.

The paper does not say how its randomness is drawn.  Both sides of the
comparison draw every random value of the method (secret key, public-key
mask and error, encryption masks and errors, re-randomisation, flood, model
owner's output mask) from this one keyed counter-based generator, so that
results can be compared bit for bit.

Definition used here.  State: counter (x0, x1, x2, x3) and key (k0, k1), all
64-bit.  One round computes the 128-bit products M0 * x0 = (hi0, lo0) and
M1 * x2 = (hi1, lo1) and replaces the state by
(hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0); between rounds the key is bumped
by the Weyl constants (W0, W1).  Ten rounds give four output words.
"""
import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
ROUNDS = 10

_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """(hi, lo) 64-bit halves of the 128-bit product of uint64 arrays a and b."""
    a0, a1 = a & _MASK32, a >> _S32
    b0, b1 = b & _MASK32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1  # each < 2^64: exact
    mid = (p00 >> _S32) + (p01 & _MASK32) + (p10 & _MASK32)  # < 3 * 2^32: no wrap
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b  # numpy uint64 multiply wraps modulo 2^64
    return hi, lo


def philox4x64(ctr, key):
    """Apply Philox-4x64-10.

    ctr: uint64 array of shape (..., 4); key: uint64 array broadcastable to
    (..., 2).  Returns the four output words, shape (..., 4).
    """
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.broadcast_to(np.asarray(key, dtype=np.uint64), ctr.shape[:-1] + (2,))
    x0, x1, x2, x3 = (ctr[..., i].copy() for i in range(4))
    k0, k1 = key[..., 0].copy(), key[..., 1].copy()
    m0, m1 = np.uint64(M0), np.uint64(M1)
    w0, w1 = np.uint64(W0), np.uint64(W1)
    with np.errstate(over="ignore"):
        for r in range(ROUNDS):
            if r:
                k0 = k0 + w0
                k1 = k1 + w1
            hi0, lo0 = _mulhilo(m0, x0)
            hi1, lo1 = _mulhilo(m1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return np.stack([x0, x1, x2, x3], axis=-1)


def stream_words(seed, nonce, obj, purpose, limb, start, count):
    """Words [start, start+count) of the stream named by (obj, purpose, limb)
    under key (seed, nonce).

    Word g of a stream is output word g mod 4 of Philox on counter
    (g div 4, obj, purpose, limb).
    """
    if count <= 0:
        return np.zeros(0, dtype=np.uint64)
    first, last = start // 4, (start + count - 1) // 4
    blocks = np.arange(first, last + 1, dtype=np.uint64)
    ctr = np.empty((blocks.size, 4), dtype=np.uint64)
    ctr[:, 0] = blocks
    ctr[:, 1] = np.uint64(obj)
    ctr[:, 2] = np.uint64(purpose)
    ctr[:, 3] = np.uint64(limb)
    words = philox4x64(ctr, np.array([seed, nonce], dtype=np.uint64)).reshape(-1)
    off = start - first * 4
    return words[off:off + count]
