"""Batched polynomial encodings of App. A, generalised to the three products
of a training step.

App. A encodes a convolution's input v (batch B, channels c_i, h x w) forward,
    index_v(b, c, i, j) = b*c_o*c_i*h*w + c*h*w + i*w + j,
and its kernel W (c_o x c_i x s x s) reversed,
    index_W(c', c, i, j) = O + c'*c_i*h*w - c*h*w - i*w - j,
    O = (c_i - 1)*h*w + (s - 1)*w + s - 1,
so that the ring product holds the output at
    index_y(b, c', i, j) = b*c_o*c_i*h*w + O + c'*c_i*h*w + i*w + j.
Readings of garbled or loose passages (checked by brute force in the tests):
the kernel indices i, j range over [s], not [h]; outputs are valid only for
i < h - s + 1, j < w - s + 1 (a valid correlation over the zero-padded input);
the matrix encoding is the 1x1 case (h = w = s = 1).

One primitive covers every product, a batched packed correlation
    out[m, r, y, x] = sum_{k, dy, dx} A[m, k, y+dy, x+dx] * K[r, k, dy, dx]
with A forward-encoded and K reverse-encoded (roles m <-> b, r <-> c_o,
k <-> c_i).  The backward encodings are not given in the paper; readings:
  * forward:   A = pad_p(X),            K = W,                         out = Y
  * grad X:    A = pad_{s-1-p}(dY),     K[c_i, c_o] = flip(W)[c_o, c_i],  out = dX
  * grad W:    A[c_i, b] = pad_p(X)[b, c_i],  K[c_o, b] = dY[b, c_o],     out[c_i, c_o] = dW[c_o, c_i]
For the grad-W cross terms either operand may be the ciphertext: the ring
product is commutative, so a reverse-encoded ciphertext of dY times a
forward-encoded plaintext of X lands in the same output slots (Alg. 2).

Operands larger than N slots are partitioned (App. A says they "could be
partitioned"; the scheme is a reading of it): a tile takes m_t x r_t x k_t
channels and an output window oh_t x ow_t with a kernel window kh_t x kw_t,
so the A tile is (oh_t + kh_t - 1) x (ow_t + kw_t - 1) and the tile fits when
m_t * r_t * k_t * HA_t * WA_t <= N.  Partial products over contraction tiles
(k, kernel rows, kernel columns) add up in the same output ciphertext.
"""
from dataclasses import dataclass
from math import ceil

import numpy as np

OPS = ("fwd", "dx", "dw")


@dataclass(frozen=True)
class Geometry:
    M: int
    R: int
    K: int
    HA: int
    WA: int
    KH: int
    KW: int

    @property
    def OH(self):
        return self.HA - self.KH + 1

    @property
    def OW(self):
        return self.WA - self.KW + 1


@dataclass(frozen=True)
class Tile:
    m: int
    r: int
    k: int
    oh: int
    ow: int
    kh: int
    kw: int

    @property
    def ha(self):
        return self.oh + self.kh - 1

    @property
    def wa(self):
        return self.ow + self.kw - 1

    @property
    def slots(self):
        return self.m * self.r * self.k * self.ha * self.wa

    @property
    def offset(self):
        """O of App. A for this tile."""
        return (self.k - 1) * self.ha * self.wa + (self.kh - 1) * self.wa + self.kw - 1


def _as4(a):
    """4-d view: FC tensors (n0, n1) -> (n0, n1, 1, 1); conv1d tensors
    (n0, n1, len) -> (n0, n1, 1, len)."""
    a = np.asarray(a)
    if a.ndim == 3:
        return a.reshape(a.shape[0], a.shape[1], 1, a.shape[2])
    return a.reshape(a.shape + (1,) * (4 - a.ndim)) if a.ndim < 4 else a


def _pad(a, ph, pw):
    if ph == 0 and pw == 0:
        return a
    return np.pad(a, ((0, 0), (0, 0), (ph, ph), (pw, pw)))


def geometry(layer, op):
    """Packed-correlation dimensions of op.  Stride 1 only: a strided layer is
    encoded through its space-to-depth equivalent."""
    assert getattr(layer, "stride", 1) == 1, "strided layers have no direct packed encoding"
    B, ci, co, h, w = layer.batch, layer.c_in, layer.c_out, layer.h, layer.w
    kh, kw, ph, pw = layer.kh, layer.kw, layer.pad_h, layer.pad_w
    ho, wo = layer.h_out, layer.w_out
    if op == "fwd":
        return Geometry(B, co, ci, h + 2 * ph, w + 2 * pw, kh, kw)
    if op == "dx":
        qh, qw = kh - 1 - ph, kw - 1 - pw
        assert qh >= 0 and qw >= 0, "padding larger than kernel-1 is not covered"
        return Geometry(B, ci, co, ho + 2 * qh, wo + 2 * qw, kh, kw)
    if op == "dw":
        return Geometry(ci, co, B, h + 2 * ph, w + 2 * pw, ho, wo)
    raise ValueError(op)


def virtual_a(layer, op, t):
    """The A operand (M, K, HA, WA) of op from tensor t (x for fwd/dw, dy for dx)."""
    t4 = _as4(t)
    if op == "fwd":
        return _pad(t4, layer.pad_h, layer.pad_w)
    if op == "dx":
        return _pad(t4, layer.kh - 1 - layer.pad_h, layer.kw - 1 - layer.pad_w)
    if op == "dw":
        return _pad(t4, layer.pad_h, layer.pad_w).transpose(1, 0, 2, 3)
    raise ValueError(op)


def virtual_k(layer, op, t):
    """The K operand (R, K, KH, KW) of op from tensor t (W for fwd/dx, dy for dw)."""
    t4 = _as4(t)
    if op == "fwd":
        return t4
    if op == "dx":
        return t4[:, :, ::-1, ::-1].transpose(1, 0, 2, 3)
    if op == "dw":
        return t4.transpose(1, 0, 2, 3)
    raise ValueError(op)


def from_virtual_out(layer, op, out_v):
    """Output tensor in the layer's layout from the virtual out (M, R, OH, OW)."""
    if op == "fwd":
        return out_v.reshape(layer.y_shape())
    if op == "dx":
        return out_v.reshape(layer.x_shape())
    if op == "dw":
        return out_v.transpose(1, 0, 2, 3).reshape(layer.w_shape())
    raise ValueError(op)


def to_virtual_out(layer, op, y):
    """Inverse of from_virtual_out (for the model owner's bias add and tests)."""
    g = geometry(layer, op)
    if op == "dw":
        return _as4(y).transpose(1, 0, 2, 3)
    return _as4(y).reshape(g.M, g.R, g.OH, g.OW)


@dataclass(frozen=True)
class Counts:
    nM: int
    nR: int
    nK: int
    nOY: int
    nOX: int
    nKY: int
    nKX: int

    @property
    def n_a(self):
        return self.nM * self.nK * self.nOY * self.nOX * self.nKY * self.nKX

    @property
    def n_k(self):
        return self.nR * self.nK * self.nKY * self.nKX

    @property
    def n_out(self):
        return self.nM * self.nR * self.nOY * self.nOX

    @property
    def n_products(self):
        return self.n_out * self.nK * self.nKY * self.nKX


def counts(g: Geometry, tl: Tile) -> Counts:
    return Counts(ceil(g.M / tl.m), ceil(g.R / tl.r), ceil(g.K / tl.k), ceil(g.OH / tl.oh), ceil(g.OW / tl.ow),
                  ceil(g.KH / tl.kh), ceil(g.KW / tl.kw))


def a_index(c: Counts, mi, ki, oyi, oxi, kyi, kxi):
    return ((((mi * c.nK + ki) * c.nOY + oyi) * c.nOX + oxi) * c.nKY + kyi) * c.nKX + kxi


def k_index(c: Counts, ri, ki, kyi, kxi):
    return ((ri * c.nK + ki) * c.nKY + kyi) * c.nKX + kxi


def out_index(c: Counts, mi, ri, oyi, oxi):
    return ((mi * c.nR + ri) * c.nOY + oyi) * c.nOX + oxi


def check_tile(g: Geometry, tl: Tile, n: int):
    assert min(tl.m, tl.r, tl.k, tl.oh, tl.ow, tl.kh, tl.kw) >= 1
    assert tl.m <= g.M and tl.r <= g.R and tl.k <= g.K, (g, tl)
    assert tl.oh <= g.OH and tl.ow <= g.OW and tl.kh <= g.KH and tl.kw <= g.KW, (g, tl)
    assert tl.slots <= n, f"tile {tl} needs {tl.slots} > N={n} slots"


def encode_a(A_v, g: Geometry, tl: Tile, n, mi, ki, oyi, oxi, kyi, kxi):
    """pi_v of App. A applied to one A tile: a length-n coefficient vector over Z_t."""
    poly = np.zeros(n, dtype=np.int64)
    m0, k0 = mi * tl.m, ki * tl.k
    y0, x0 = oyi * tl.oh + kyi * tl.kh, oxi * tl.ow + kxi * tl.kw
    for mm in range(tl.m):
        for kk in range(tl.k):
            for ya in range(tl.ha):
                for xa in range(tl.wa):
                    m, k, y, x = m0 + mm, k0 + kk, y0 + ya, x0 + xa
                    if m < g.M and k < g.K and y < g.HA and x < g.WA:
                        idx = mm * tl.r * tl.k * tl.ha * tl.wa + kk * tl.ha * tl.wa + ya * tl.wa + xa
                        poly[idx] = A_v[m, k, y, x]
    return poly


def encode_k(K_v, g: Geometry, tl: Tile, n, ri, ki, kyi, kxi):
    """pi_W of App. A (reverse encoding) applied to one K tile."""
    poly = np.zeros(n, dtype=np.int64)
    r0, k0, ky0, kx0 = ri * tl.r, ki * tl.k, kyi * tl.kh, kxi * tl.kw
    O = tl.offset
    for rr in range(tl.r):
        for kk in range(tl.k):
            for dy in range(tl.kh):
                for dx in range(tl.kw):
                    r, k, a, b = r0 + rr, k0 + kk, ky0 + dy, kx0 + dx
                    if r < g.R and k < g.K and a < g.KH and b < g.KW:
                        idx = O + rr * tl.k * tl.ha * tl.wa - kk * tl.ha * tl.wa - dy * tl.wa - dx
                        poly[idx] = K_v[r, k, a, b]
    return poly


def out_slots(g: Geometry, tl: Tile, mi, ri, oyi, oxi):
    """[(slot, (m, r, y, x))] for the valid outputs of one output tile (pi_y^-1 of App. A)."""
    res = []
    m0, r0, oy0, ox0 = mi * tl.m, ri * tl.r, oyi * tl.oh, oxi * tl.ow
    O = tl.offset
    for mm in range(tl.m):
        for rr in range(tl.r):
            for y in range(tl.oh):
                for x in range(tl.ow):
                    m, r, yy, xx = m0 + mm, r0 + rr, oy0 + y, ox0 + x
                    if m < g.M and r < g.R and yy < g.OH and xx < g.OW:
                        slot = mm * tl.r * tl.k * tl.ha * tl.wa + O + rr * tl.k * tl.ha * tl.wa + y * tl.wa + x
                        res.append((slot, (m, r, yy, xx)))
    return res


def a_tiles(c: Counts):
    for mi in range(c.nM):
        for ki in range(c.nK):
            for oyi in range(c.nOY):
                for oxi in range(c.nOX):
                    for kyi in range(c.nKY):
                        for kxi in range(c.nKX):
                            yield (mi, ki, oyi, oxi, kyi, kxi)


def k_tiles(c: Counts):
    for ri in range(c.nR):
        for ki in range(c.nK):
            for kyi in range(c.nKY):
                for kxi in range(c.nKX):
                    yield (ri, ki, kyi, kxi)


def out_tiles(c: Counts):
    for mi in range(c.nM):
        for ri in range(c.nR):
            for oyi in range(c.nOY):
                for oxi in range(c.nOX):
                    yield (mi, ri, oyi, oxi)
