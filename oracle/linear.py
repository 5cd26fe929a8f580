"""Plaintext linear layers over Z_t (Sec. II.D, Eq. 1) and their backward
operators (Sec. III.A), by their textbook definitions.

  FC:     Y = X W^T,  dX = dY W,  dW = dY^T X              (PyTorch layout)
  Conv2d: Y[b,o,y,x] = sum_{c,i,j} Xpad[b,c,s*y+i,s*x+j] W[o,c,i,j]   (stride s)
          dX = the adjoint of X -> Y (scatter of dY through W, padding cropped)
          dW[o,c,i,j] = sum_{b,y,x} dY[b,o,y,x] Xpad[b,c,s*y+i,s*x+j]
  Conv1d: the Conv2d case with one row, a 1 x k kernel and padding along the
          length only (tensors (batch, channels, length))

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


def _pad(x, ph, pw):
    return x if ph == 0 and pw == 0 else np.pad(x, ((0, 0), (0, 0), (ph, ph), (pw, pw)))


def _taps(i, n, s):
    """Rows i, i + s, ..., i + (n - 1) s of a padded input."""
    return slice(i, i + s * (n - 1) + 1, s)


def conv2d(x, W, ph, pw, s, t, tdot=tensordot_mod_t):
    """Y[b,o,y,x] = sum_{c,i,j} Xpad[b, c, s y + i, s x + j] W[o, c, i, j]."""
    B, ci, h, w = x.shape
    co, _, kh, kw = W.shape
    xp = _pad(x, ph, pw)
    ho, wo = (h + 2 * ph - kh) // s + 1, (w + 2 * pw - kw) // s + 1
    y = np.zeros((B, co, ho, wo), dtype=np.int64)
    for i in range(kh):
        for j in range(kw):
            part = tdot(xp[:, :, _taps(i, ho, s), _taps(j, wo, s)], W[:, :, i, j], ([1], [1]), t)  # (B, ho, wo, co)
            y = np.mod(y + part.transpose(0, 3, 1, 2), t)
    return y


def conv2d_dx(dy, W, ph, pw, s, h, w, t, tdot=tensordot_mod_t):
    """The adjoint of X -> Y: every dY[b,o,y,x] W[o,c,i,j] lands on Xpad[b,c,s y+i,s x+j]; padding cropped."""
    B, co, ho, wo = dy.shape
    _, ci, kh, kw = W.shape
    dxp = np.zeros((B, ci, h + 2 * ph, w + 2 * pw), dtype=np.int64)
    for i in range(kh):
        for j in range(kw):
            part = tdot(dy, W[:, :, i, j], ([1], [0]), t).transpose(0, 3, 1, 2)  # (B, ci, ho, wo)
            sl = (slice(None), slice(None), _taps(i, ho, s), _taps(j, wo, s))
            dxp[sl] = np.mod(dxp[sl] + part, t)
    return dxp[:, :, ph:ph + h, pw:pw + w]


def conv2d_dw(x, dy, ph, pw, s, kh, kw, t, tdot=tensordot_mod_t):
    """dW[o,c,i,j] = sum_{b,y,x} dY[b,o,y,x] Xpad[b, c, s y + i, s x + j]."""
    _, _, ho, wo = dy.shape
    xp = _pad(x, ph, pw)
    ci, co = x.shape[1], dy.shape[1]
    dW = np.zeros((co, ci, kh, kw), dtype=np.int64)
    for i in range(kh):
        for j in range(kw):
            dW[:, :, i, j] = tdot(dy, xp[:, :, _taps(i, ho, s), _taps(j, wo, s)], ([0, 2, 3], [0, 2, 3]), t)
    return dW


def _as4d(layer, v):
    """A conv1d tensor (n0, n1, len) viewed as (n0, n1, 1, len); others unchanged."""
    v = np.asarray(v)
    return v.reshape(v.shape[0], v.shape[1], 1, v.shape[2]) if layer.kind == "conv1d" else v


def _from4d(layer, v):
    return v.reshape(v.shape[0], v.shape[1], v.shape[3]) if layer.kind == "conv1d" else v


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
    ph, pw, s = layer.pad_h, layer.pad_w, layer.stride
    if op == "fwd":
        return _from4d(layer, conv2d(_as4d(layer, a), _as4d(layer, b), ph, pw, s, t, tdot))
    if op == "dx":
        return _from4d(layer, conv2d_dx(_as4d(layer, a), _as4d(layer, b), ph, pw, s, layer.h, layer.w, t, tdot))
    if op == "dw":
        return _from4d(layer, conv2d_dw(_as4d(layer, a), _as4d(layer, b), ph, pw, s, layer.kh, layer.kw, t, tdot))
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
    kh, kw, ph, pw, st = layer.kh, layer.kw, layer.pad_h, layer.pad_w, layer.stride
    h, w = layer.h, layer.w
    ho, wo = layer.h_out, layer.w_out
    a4, b4 = _as4d(layer, a), _as4d(layer, b)

    def x_at(x, bb, c, y, xx):
        y, xx = y - ph, xx - pw
        return int(x[bb, c, y, xx]) if 0 <= y < h and 0 <= xx < w else 0

    def at4(p):
        # conv1d points (n0, n1, pos) address row 0 of the 4-d view
        return (p[0], p[1], 0, p[2]) if layer.kind == "conv1d" else tuple(p)

    for p in points:
        v = 0
        if op == "fwd":          # Y[b, o, y, x] = sum_{c,i,j} Xpad[b, c, s y + i, s x + j] W[o, c, i, j]
            bb, o, y, xx = at4(p)
            for c in range(layer.c_in):
                for i in range(kh):
                    for j in range(kw):
                        v += x_at(a4, bb, c, st * y + i, st * xx + j) * int(b4[o, c, i, j])
        elif op == "dx":         # dX[b, c, y, x] = sum over (o, i, j, y', x') with s y' + i = y + p, s x' + j = x + p
            bb, c, y, xx = at4(p)
            for o in range(layer.c_out):
                for i in range(kh):
                    for j in range(kw):
                        ny, nx = y + ph - i, xx + pw - j
                        if ny % st or nx % st:
                            continue
                        yy, xj = ny // st, nx // st
                        if 0 <= yy < ho and 0 <= xj < wo:
                            v += int(a4[bb, o, yy, xj]) * int(b4[o, c, i, j])
        else:                    # dW[o, c, i, j] = sum_{b,y,x} dY[b, o, y, x] Xpad[b, c, s y + i, s x + j]
            o, c, i, j = at4(p)
            for bb in range(layer.batch):
                for y in range(ho):
                    for xx in range(wo):
                        v += int(b4[bb, o, y, xx]) * x_at(a4, bb, c, st * y + i, st * xx + j)
        out.append(v % t)
    return out
