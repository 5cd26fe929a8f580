"""Plaintext linear layers over Z_t (Sec. II.D, Eq. 1) and their backward
operators (Sec. III.A), by their textbook definitions.

  FC:     Y = X W^T,  dX = dY W,  dW = dY^T X              (PyTorch layout)
  Conv2d: Y[b,o,y,x] = sum_{c,i,j} Xpad[b,c,y+i,x+j] W[o,c,i,j]   (stride 1)
          dX = the adjoint of X -> Y (scatter of dY through W, padding cropped)
          dW[o,c,i,j] = sum_{b,y,x} dY[b,o,y,x] Xpad[b,c,y+i,x+j]

All arithmetic is exact modulo t.  Integer tensor contractions are done as
float64 tensordots of 14-bit digits (every partial sum stays below 2^53, so
each float result is an exact integer) and recombined modulo t;
`tensordot_mod_t_object` is the same contraction in Python integers, used to
pin the digit version on small inputs.
"""
import numpy as np

DIGIT = 14
NDIG = 3  # centred values |v| < 2^40 < 2^(3*14)


def centred(v, t):
    v = np.asarray(v, dtype=np.int64)
    return np.where(v > (t - 1) // 2, v - t, v)


def _digits(v):
    """Signed base-2^14 digits (d0, d1 in [0, 2^14), d2 signed) as float64 arrays."""
    v = np.asarray(v, dtype=np.int64)
    out = []
    for _ in range(NDIG - 1):
        d = np.mod(v, 1 << DIGIT)
        out.append(d.astype(np.float64))
        v = (v - d) >> DIGIT
    out.append(v.astype(np.float64))
    return out


def tensordot_mod_t(a, b, axes, t):
    """Exact tensordot of Z_t tensors (entries in [0, t)), reduced into [0, t)."""
    da, db = _digits(centred(a, t)), _digits(centred(b, t))
    k = 1
    ax_a = axes[0] if isinstance(axes[0], (list, tuple)) else [axes[0]]
    for ax in ax_a:
        k *= np.asarray(a).shape[ax]
    assert k < (1 << 24), "contraction too long for exact float64 digit products"
    T = [None] * (2 * NDIG - 1)
    for i in range(NDIG):
        for j in range(NDIG):
            s = np.tensordot(da[i], db[j], axes=axes)
            s = np.mod(np.rint(s).astype(np.int64), t)
            T[i + j] = s if T[i + j] is None else np.mod(T[i + j] + s, t)
    acc = T[-1]
    for d in range(len(T) - 2, -1, -1):
        acc = np.mod(acc * (1 << DIGIT) + T[d], t)
    return acc.astype(np.int64)


def tensordot_mod_t_object(a, b, axes, t):
    """The same contraction in Python integers (small inputs only)."""
    ao = np.asarray(a).astype(object)
    bo = np.asarray(b).astype(object)
    r = np.tensordot(ao, bo, axes=axes)
    return np.vectorize(lambda v: int(v) % t, otypes=[np.int64])(r) if np.ndim(r) else np.int64(int(r) % t)


def _pad(x, p):
    return x if p == 0 else np.pad(x, ((0, 0), (0, 0), (p, p), (p, p)))


def conv2d(x, W, pad, t, tdot=tensordot_mod_t):
    B, ci, h, w = x.shape
    co, _, s, _ = W.shape
    xp = _pad(x, pad)
    ho, wo = h + 2 * pad - s + 1, w + 2 * pad - s + 1
    y = np.zeros((B, co, ho, wo), dtype=np.int64)
    for i in range(s):
        for j in range(s):
            part = tdot(xp[:, :, i:i + ho, j:j + wo], W[:, :, i, j], ([1], [1]), t)  # (B, ho, wo, co)
            y = np.mod(y + part.transpose(0, 3, 1, 2), t)
    return y


def conv2d_dx(dy, W, pad, h, w, t, tdot=tensordot_mod_t):
    B, co, ho, wo = dy.shape
    _, ci, s, _ = W.shape
    dxp = np.zeros((B, ci, h + 2 * pad, w + 2 * pad), dtype=np.int64)
    for i in range(s):
        for j in range(s):
            part = tdot(dy, W[:, :, i, j], ([1], [0]), t)  # (B, ho, wo, ci)
            dxp[:, :, i:i + ho, j:j + wo] = np.mod(dxp[:, :, i:i + ho, j:j + wo] + part.transpose(0, 3, 1, 2), t)
    return dxp[:, :, pad:pad + h, pad:pad + w]


def conv2d_dw(x, dy, pad, s, t, tdot=tensordot_mod_t):
    B, ci, h, w = x.shape
    _, co, ho, wo = dy.shape
    xp = _pad(x, pad)
    dW = np.zeros((co, ci, s, s), dtype=np.int64)
    for i in range(s):
        for j in range(s):
            dW[:, :, i, j] = tdot(dy, xp[:, :, i:i + ho, j:j + wo], ([0, 2, 3], [0, 2, 3]), t)
    return dW


def layer_op(layer, op, a, b, t, tdot=tensordot_mod_t):
    """The plaintext result of one product, mod t.

    fwd: a = X, b = W -> Y;  dx: a = dY, b = W -> dX;  dw: a = X, b = dY -> dW.
    """
    if layer.kind == "fc":
        if op == "fwd":
            return tdot(a, b, ([1], [1]), t)
        if op == "dx":
            return tdot(a, b, ([1], [0]), t)
        if op == "dw":
            return tdot(b, a, ([0], [0]), t)
        raise ValueError(op)
    if op == "fwd":
        return conv2d(a, b, layer.pad, t, tdot)
    if op == "dx":
        return conv2d_dx(a, b, layer.pad, layer.h, layer.w, t, tdot)
    if op == "dw":
        return conv2d_dw(a, b, layer.pad, layer.k, t, tdot)
    raise ValueError(op)


def layer_op_at(layer, op, a, b, t, points):
    """Selected output elements of layer_op, each summed by its definition in
    Python integers.  points: index tuples into the output tensor."""
    a = np.asarray(a)
    b = np.asarray(b)
    out = []
    if layer.kind == "fc":
        for p in points:
            if op == "fwd":      # Y[b, o] = sum_i X[b, i] W[o, i]
                v = sum(int(x) * int(w) for x, w in zip(a[p[0]], b[p[1]]))
            elif op == "dx":     # dX[b, i] = sum_o dY[b, o] W[o, i]
                v = sum(int(x) * int(w) for x, w in zip(a[p[0]], b[:, p[1]]))
            else:                # dW[o, i] = sum_b dY[b, o] X[b, i]
                v = sum(int(x) * int(g) for x, g in zip(a[:, p[1]], b[:, p[0]]))
            out.append(v % t)
        return out
    k, pad = layer.k, layer.pad
    h, w = layer.h, layer.w
    ho, wo = layer.h_out, layer.w_out

    def x_at(x, bb, c, y, xx):
        y, xx = y - pad, xx - pad
        return int(x[bb, c, y, xx]) if 0 <= y < h and 0 <= xx < w else 0

    for p in points:
        v = 0
        if op == "fwd":          # Y[b, o, y, x] = sum_{c,i,j} Xpad[b, c, y+i, x+j] W[o, c, i, j]
            bb, o, y, xx = p
            for c in range(layer.c_in):
                for i in range(k):
                    for j in range(k):
                        v += x_at(a, bb, c, y + i, xx + j) * int(b[o, c, i, j])
        elif op == "dx":         # dX[b, c, y, x] = sum_{o,i,j} dY[b, o, y+p-i, x+p-j] W[o, c, i, j]
            bb, c, y, xx = p
            for o in range(layer.c_out):
                for i in range(k):
                    for j in range(k):
                        yy, xj = y + pad - i, xx + pad - j
                        if 0 <= yy < ho and 0 <= xj < wo:
                            v += int(a[bb, o, yy, xj]) * int(b[o, c, i, j])
        else:                    # dW[o, c, i, j] = sum_{b,y,x} dY[b, o, y, x] Xpad[b, c, y+i, x+j]
            o, c, i, j = p
            for bb in range(layer.batch):
                for y in range(ho):
                    for xx in range(wo):
                        v += int(b[bb, o, y, xx]) * x_at(a, bb, c, y + i, xx + j)
        out.append(v % t)
    return out
