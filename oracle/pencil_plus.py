"""Pencil+ (Sec. IV.C, Alg. 3 and Alg. 4): shared products u o v of a linear
operator with the homomorphic work moved to a preprocessing phase.  Test
infrastructure only, like every module of the oracle.

Preprocessing, per operator o: the model owner (MO) holds m masks u'_i, the
data owner (DO) m masks v'_j; for every pair the MO evaluates u'_i o Enc(v'_j)
minus a fresh mask s_ij and the DO decrypts, so the parties hold additive
shares <u'_i o v'_j>_0 = s_ij and <u'_i o v'_j>_1 = u'_i o v'_j - s_ij.  The
homomorphic product itself is the path the rest of the oracle covers
(protocol.mo_product); here the preprocessing outcome is its plain definition.

Online (no homomorphic operation): the MO publishes k_i and u~ = u - sum k_i u'_i,
the DO publishes l_j and v~ = v - sum l_j v'_j, and

    <u o v'_j>_0 = sum_i k_i <u'_i o v'_j>_0
    <u o v'_j>_1 = u~ o v'_j + sum_i k_i <u'_i o v'_j>_1
    <u o v>_0    = u o v~ + sum_j l_j <u o v'_j>_0
    <u o v>_1    = sum_j l_j <u o v'_j>_1

The four operators of one linear layer (Alg. 4): forward (u = W, v = <X>_1),
input gradient (u = W, v = <dY>_1), and the two weight-gradient cross terms
(u = <dY>_0, v = <X>_1 and u = <X>_0, v = <dY>_1).
"""
import numpy as np

from . import linear as LIN

KINDS = ("fwd", "dx", "dw01", "dw10")


def apply(layer, kind, u, v, t):
    """u o v for the operator `kind` (u the MO's operand, v the DO's), mod t."""
    if kind == "fwd":
        return LIN.layer_op(layer, "fwd", v, u, t)   # Y = X W^T
    if kind == "dx":
        return LIN.layer_op(layer, "dx", v, u, t)    # dX = dY W
    if kind == "dw01":
        return LIN.layer_op(layer, "dw", v, u, t)    # <dY>_0 with <X>_1
    if kind == "dw10":
        return LIN.layer_op(layer, "dw", u, v, t)    # <X>_0 with <dY>_1
    raise ValueError(kind)


def operand_shapes(layer, kind):
    """(shape of u, shape of v, shape of u o v)."""
    X, W, Y = layer.x_shape(), layer.w_shape(), layer.y_shape()
    return {"fwd": (W, X, Y), "dx": (W, Y, X), "dw01": (Y, X, W), "dw10": (X, Y, W)}[kind]


def combine(terms, coeffs, t, base=None):
    """base + sum_i coeffs[i] * terms[i] mod t, exact (Python integers)."""
    acc = np.zeros_like(terms[0], dtype=object) if base is None else base.astype(object)
    for x, c in zip(terms, coeffs):
        acc = acc + x.astype(object) * int(c)
    return np.asarray(acc % t, dtype=np.int64)


def prep(layer, kind, u_masks, v_masks, s, t):
    """Shares of u'_i o v'_j by definition: (s_ij, u'_i o v'_j - s_ij)."""
    m = len(u_masks)
    share0 = [[s[i][j] for j in range(m)] for i in range(m)]
    share1 = [[np.asarray((apply(layer, kind, u_masks[i], v_masks[j], t).astype(object) - s[i][j]) % t,
                          dtype=np.int64) for j in range(m)] for i in range(m)]
    return share0, share1


def online(layer, kind, u, v, u_masks, v_masks, share0, share1, k, l, t):
    """Alg. 3's online phase.  Returns the two output shares and the messages
    (u~, v~) the parties exchange."""
    m = len(u_masks)
    u_t = combine(u_masks, [(-int(c)) % t for c in k], t, base=u)          # MO -> DO
    v_t = combine(v_masks, [(-int(c)) % t for c in l], t, base=v)          # DO -> MO
    uvj0 = [combine([share0[i][j] for i in range(m)], k, t) for j in range(m)]
    uvj1 = [combine([share1[i][j] for i in range(m)], k, t, base=apply(layer, kind, u_t, v_masks[j], t))
            for j in range(m)]
    out0 = combine(uvj0, l, t, base=apply(layer, kind, u, v_t, t))
    out1 = combine(uvj1, l, t)
    return out0, out1, u_t, v_t
