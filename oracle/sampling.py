"""Samplers drawing the method's random values from Philox streams.

The paper names no distributions.  Readings (integer-only, so both sides agree
bit for bit):

* ternary (secret key s, encryption masks u, re-randomisation mask u'):
  coefficient i takes the 32-bit half (i mod 2) of stream word i div 2 (low
  half first) and maps h to (h mod 3) - 1;
* error (e, e1, e2): centred binomial with 21 coin pairs, from stream word i:
  popcount(w & (2^21-1)) - popcount((w >> 21) & (2^21-1)), sd ~3.24;
* uniform mod q_l (public-key component a): words 2i and 2i+1 form a 128-bit
  integer, reduced mod q_l (a separate stream per limb);
* flood: words i*W .. i*W+W-1 (W = ceil((fb+1)/64), little-endian) form an
  integer V, keep its low fb+1 bits, and the flood is V - 2^fb, uniform in
  [-2^fb, 2^fb);
* model owner's mask: words 2i and 2i+1 form a 128-bit integer, reduced mod t;
* additive share (Sec. II.C): the same construction on its own stream
  (purpose P_SHARE): s0 = that value, s1 = v - s0 mod t.

Stream names: key = (seed, nonce); counter words (block, object, purpose,
limb).  Key generation uses nonce 2^64 - 1.
"""
import numpy as np

from .philox import stream_words

KEYGEN_NONCE = (1 << 64) - 1

# purposes
P_SK = 1
P_PK_A = 2
P_PK_E = 3
P_ENC_U = 16
P_ENC_E0 = 17
P_ENC_E1 = 18
P_RR_U = 32
P_RR_E0 = 33
P_RR_E1 = 34
P_FLOOD = 35
P_MASK = 36
P_SHARE = 49


def ternary(seed, nonce, obj, purpose, n):
    w = stream_words(seed, nonce, obj, purpose, 0, 0, (n + 1) // 2)
    halves = np.empty(2 * w.size, dtype=np.uint64)
    halves[0::2] = w & np.uint64(0xFFFFFFFF)
    halves[1::2] = w >> np.uint64(32)
    return (halves[:n] % np.uint64(3)).astype(np.int64) - 1


def cbd21(seed, nonce, obj, purpose, n):
    w = stream_words(seed, nonce, obj, purpose, 0, 0, n)
    m = (1 << 21) - 1
    a = [bin(int(x) & m).count("1") for x in w]
    b = [bin((int(x) >> 21) & m).count("1") for x in w]
    return np.array(a, dtype=np.int64) - np.array(b, dtype=np.int64)


def uniform_mod(seed, nonce, obj, purpose, limb, n, q):
    w = stream_words(seed, nonce, obj, purpose, limb, 0, 2 * n)
    return np.array([(int(w[2 * i]) + (int(w[2 * i + 1]) << 64)) % q for i in range(n)], dtype=np.uint64)


def flood_words(fb):
    return (fb + 1 + 63) // 64


def flood(seed, nonce, obj, n, fb, idx=None):
    """Flood values (Python ints in [-2^fb, 2^fb)) for coefficients idx (default all)."""
    W = flood_words(fb)
    if idx is None:
        w = stream_words(seed, nonce, obj, P_FLOOD, 0, 0, n * W)
        out = []
        for i in range(n):
            v = 0
            for j in range(W):
                v |= int(w[i * W + j]) << (64 * j)
            out.append((v & ((1 << (fb + 1)) - 1)) - (1 << fb))
        return out
    out = []
    for i in idx:
        w = stream_words(seed, nonce, obj, P_FLOOD, 0, i * W, W)
        v = 0
        for j in range(W):
            v |= int(w[j]) << (64 * j)
        v &= (1 << (fb + 1)) - 1
        out.append(v - (1 << fb))
    return out


def mask_mod_t(seed, nonce, obj, n, t, idx=None):
    """Model owner's mask values in [0, t) for coefficients idx (default all)."""
    if idx is None:
        w = stream_words(seed, nonce, obj, P_MASK, 0, 0, 2 * n)
        return [(int(w[2 * i]) + (int(w[2 * i + 1]) << 64)) % t for i in range(n)]
    out = []
    for i in idx:
        w = stream_words(seed, nonce, obj, P_MASK, 0, 2 * i, 2)
        out.append((int(w[0]) + (int(w[1]) << 64)) % t)
    return out


def ternary_at(seed, nonce, obj, purpose, idx):
    out = []
    for i in idx:
        w = int(stream_words(seed, nonce, obj, purpose, 0, i // 2, 1)[0])
        out.append(((w >> (32 * (i % 2))) & 0xFFFFFFFF) % 3 - 1)
    return out


def cbd21_at(seed, nonce, obj, purpose, idx):
    m = (1 << 21) - 1
    out = []
    for i in idx:
        w = int(stream_words(seed, nonce, obj, purpose, 0, i, 1)[0])
        out.append(bin(w & m).count("1") - bin((w >> 21) & m).count("1"))
    return out


def shares_mod_t(seed, nonce, obj, v, t):
    """Additive shares (s0, s1) of the integer array v over Z_t: s0[i] is the
    128-bit integer of stream words 2i, 2i+1 (purpose P_SHARE) mod t, and
    s1 = v - s0 mod t."""
    v = np.asarray(v, dtype=np.int64).ravel()
    w = stream_words(seed, nonce, obj, P_SHARE, 0, 0, 2 * v.size)
    s0 = np.array([(int(w[2 * i]) + (int(w[2 * i + 1]) << 64)) % t for i in range(v.size)], dtype=np.int64)
    return s0, np.mod(v - s0, t).astype(np.int64)
