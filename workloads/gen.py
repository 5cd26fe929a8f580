"""Seeded tensor generation for a layer: real-valued draws, fixed-point
encoding into Z_t (Sec. II.C: Encode(x) = floor(x * 2^f)), and additive
two-party shares over Z_t.

Draw order per layer, from numpy.random.default_rng(seed): X, W, dY, then the
share randomness <X>_0 and <dY>_0.  With first_layer=True the model owner's
share of X is zero (the network-input convention of Sec. III.A).
"""
import numpy as np

# Plaintext modulus: the largest prime below 2^41.  Shares are int64 in [0, t).
T_PLAIN = 2199023255531
FRAC_BITS = 12


def fixed_point(x, frac_bits=FRAC_BITS, t=T_PLAIN):
    """floor(x * 2^f) taken modulo t, as int64 in [0, t)."""
    v = np.floor(np.asarray(x, dtype=np.float64) * float(1 << frac_bits)).astype(np.int64)
    return np.mod(v, t).astype(np.int64)


def _draw(rng, dist, shape):
    kind = dist[0]
    if kind == "normal":
        return rng.normal(0.0, dist[1], size=shape)
    if kind == "uniform":
        return rng.uniform(dist[1], dist[2], size=shape)
    raise ValueError(f"unknown distribution {dist}")


def random_shares(rng, v, t=T_PLAIN, zero_first=False):
    """Split v (int64 in [0, t)) into (s0, s1) with s0 + s1 = v mod t."""
    if zero_first:
        s0 = np.zeros_like(v)
    else:
        s0 = rng.integers(0, t, size=v.shape, dtype=np.int64)
    s1 = np.mod(v - s0, t).astype(np.int64)
    return s0, s1


def layer_tensors(layer, seed, first_layer=False, t=T_PLAIN, frac_bits=FRAC_BITS, rng=None):
    """All inputs of one layer's forward and backward products.

    Returns a dict of int64 arrays in [0, t): X, W, dY (the plain fixed-point
    values) and the shares x0, x1, dy0, dy1 (party 0 = model owner).
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    X = fixed_point(_draw(rng, layer.x_dist, layer.x_shape()), frac_bits, t)
    W = fixed_point(_draw(rng, layer.w_dist, layer.w_shape()), frac_bits, t)
    dY = fixed_point(_draw(rng, layer.dy_dist, layer.y_shape()), frac_bits, t)
    x0, x1 = random_shares(rng, X, t, zero_first=first_layer)
    dy0, dy1 = random_shares(rng, dY, t)
    return dict(X=X, W=W, dY=dY, x0=x0, x1=x1, dy0=dy0, dy1=dy1)


def config_tensors(cfg):
    """Tensors for every layer of a benchmark config, drawn from one stream."""
    rng = np.random.default_rng(cfg.seed)
    out = []
    for i, layer in enumerate(cfg.layers):
        out.append(layer_tensors(layer, cfg.seed, first_layer=(cfg.first_layer_shares and i == 0), rng=rng))
    return out


def uniform_residues(seed, shape, moduli):
    """Seeded uniform residues, one independent draw per modulus along axis -2.

    Used as ciphertext-shaped inputs ([..., L, N] with entry l in [0, q_l)) when
    a test exercises the model owner's product on its own.
    """
    rng = np.random.default_rng(seed)
    out = np.empty(shape, dtype=np.uint64)
    for l, q in enumerate(moduli):
        out[..., l, :] = rng.integers(0, q, size=out[..., l, :].shape, dtype=np.uint64)
    return out
