"""The model owner's homomorphic linear-layer products and the data owner's
ends of them: Alg. 1 (forward), its pattern for the input gradient
(Sec. III.B.2) and the cross terms of Alg. 2 (weight gradient).

Model owner's product for one output tile o (the product and share steps of
Alg. 1 and Alg. 2):
    acc = sum over contraction tiles and terms of lift(P) * C        (ring products)
    acc += Enc_pk(0) with fresh u', e0', e1'                            (re-randomise)
    c0 += flood - D(s)                                                  (flood, mask)
and the model owner's output share is s at the output slots (+ bias).
The paper does not mention re-randomisation or flooding; readings: without a
fresh Enc(0) the second component P*c1 would expose P to the decryptor, and
the flood (uniform in [-2^fb, 2^fb), fb = floor(log2 Delta) - 3) hides the
product noise, which depends on P.  The mask s is uniform over Z_t on all N
coefficients, so coefficients outside the output slots (partial sums of the
weights) are hidden too.

Randomness object ids: encryption of operand kind k (0 X for forward,
1 dY for the input gradient, 2 X for the weight gradient, 3 dY for the
weight gradient), tile i: ((k + 1) << 48) | i.  Output tile i of op
(0 fwd, 1 dx, 2 dw): ((op + 5) << 48) | i.
"""
import numpy as np

from . import bfv
from . import encoding as E
from . import sampling as S
from .ring import negacyclic_coeffs, negacyclic_mul, residues

OPERAND_X_FWD, OPERAND_DY_DX, OPERAND_X_DW, OPERAND_DY_DW = 0, 1, 2, 3
OP_CODE = {"fwd": 0, "dx": 1, "dw": 2}


def enc_object(kind, i):
    return ((kind + 1) << 48) | i


def out_object(op, i):
    return ((OP_CODE[op] + 5) << 48) | i


# ----------------------------------------------------------------- encodings

def operand_polys(layer, op, tile, n, tensor, side):
    """All tile polynomials of one operand (side "a": forward-encoded A tiles,
    side "k": reverse-encoded K tiles), in tile-index order, over Z_t."""
    g = E.geometry(layer, op)
    c = E.counts(g, tile)
    if side == "a":
        A = E.virtual_a(layer, op, tensor)
        return [E.encode_a(A, g, tile, n, *ix) for ix in E.a_tiles(c)]
    K = E.virtual_k(layer, op, tensor)
    return [E.encode_k(K, g, tile, n, *ix) for ix in E.k_tiles(c)]


OPERAND_SIDE = {OPERAND_X_FWD: ("fwd", "a"), OPERAND_DY_DX: ("dx", "a"), OPERAND_X_DW: ("dw", "a"),
                OPERAND_DY_DW: ("dw", "k")}


def encrypt_operand(P, pk, layer, plan, kind, share, seed, nonce):
    """Data owner: encrypt its share tensor in the layout of operand `kind`."""
    op, side = OPERAND_SIDE[kind]
    polys = operand_polys(layer, op, plan[op], P.n, share, side)
    return [bfv.encrypt(P, pk, m, seed, nonce, enc_object(kind, i)) for i, m in enumerate(polys)]


# ----------------------------------------------------------- model owner

def _lift_limbs(P, poly):
    return [residues([bfv.lift_centred(v, P.t) for v in poly], q) for q in P.moduli]


def mo_product(P, pk, layer, op, tile, terms, seed, nonce, add_share=None, bias=None, outs=None,
               coeff_idx=None):
    """Model owner's product for `op`.

    terms: list of (a, k) where each of a, k is ("ct", [ciphertexts by tile
    index]) or ("pt", Z_t tensor in the layer's layout).  add_share: the model
    owner's share added to the A-side ciphertexts before the product (Alg. 1,
    product step).  outs: output tile indices to compute (default all).  coeff_idx:
    compute only these coefficients of each output ciphertext.

    Returns {o: ct [2][L][len]} and the model owner's share tensor (entries of
    tiles not computed are left at -1).
    """
    g = E.geometry(layer, op)
    c = E.counts(g, tile)
    n, t, L = P.n, P.t, P.num_limbs
    idx = np.arange(n) if coeff_idx is None else np.asarray(coeff_idx, dtype=np.int64)

    # encode plaintext tiles on first use
    a_list = list(E.a_tiles(c))
    k_list = list(E.k_tiles(c))
    pt_cache = {}

    def pt_poly(tensor, side, ti):
        key = (id(tensor), side, ti)
        if key not in pt_cache:
            if side == "a":
                poly = E.encode_a(E.virtual_a(layer, op, tensor), g, tile, n, *a_list[ti])
            else:
                poly = E.encode_k(E.virtual_k(layer, op, tensor), g, tile, n, *k_list[ti])
            pt_cache[key] = _lift_limbs(P, poly)
        return pt_cache[key]

    ct_cache = {}

    def a_ct(ti, cts):
        if add_share is None:
            return cts[ti]
        if ti not in ct_cache:
            m = E.encode_a(E.virtual_a(layer, op, add_share), g, tile, n, *a_list[ti])
            ct_cache[ti] = bfv.add_plain(P, cts[ti], m)
        return ct_cache[ti]

    out_v = np.full((g.M, g.R, g.OH, g.OW), -1, dtype=np.int64)
    bias_v = None
    if bias is not None:
        bias_v = np.asarray(bias, dtype=np.int64)
    result = {}
    all_outs = list(E.out_tiles(c))
    sel = range(len(all_outs)) if outs is None else outs
    for o in sel:
        mi, ri, oyi, oxi = all_outs[o]
        acc = [[[0] * len(idx) for _ in range(L)] for _ in range(2)]
        for ki in range(c.nK):
            for kyi in range(c.nKY):
                for kxi in range(c.nKX):
                    ai = E.a_index(c, mi, ki, oyi, oxi, kyi, kxi)
                    kk = E.k_index(c, ri, ki, kyi, kxi)
                    for (akind, aval), (kkind, kval) in terms:
                        if akind == "ct":
                            ct = a_ct(ai, aval)
                            pl = pt_poly(kval, "k", kk)
                        else:
                            ct = kval[kk]
                            pl = pt_poly(aval, "a", ai)
                        for l, q in enumerate(P.moduli):
                            for cc in range(2):
                                if coeff_idx is None:
                                    pr = negacyclic_mul(pl[l], ct[cc, l], q)
                                else:
                                    pr = negacyclic_coeffs(pl[l], ct[cc, l], q, idx)
                                acc[cc][l] = [(a + int(b)) % q for a, b in zip(acc[cc][l], pr)]
        obj = out_object(op, o)
        # re-randomise: + (p0*u' + e0', p1*u' + e1')
        u = S.ternary(seed, nonce, obj, S.P_RR_U, n)
        if coeff_idx is None:
            e = (S.cbd21(seed, nonce, obj, S.P_RR_E0, n), S.cbd21(seed, nonce, obj, S.P_RR_E1, n))
            fl = S.flood(seed, nonce, obj, n, P.flood_bits)
            s = S.mask_mod_t(seed, nonce, obj, n, t)
        else:
            e = (S.cbd21_at(seed, nonce, obj, S.P_RR_E0, idx), S.cbd21_at(seed, nonce, obj, S.P_RR_E1, idx))
            fl = S.flood(seed, nonce, obj, n, P.flood_bits, idx)
            s = S.mask_mod_t(seed, nonce, obj, n, t, idx)
        ds = bfv.delta_scale(s, P)
        ct_o = np.empty((2, L, len(idx)), dtype=np.uint64)
        for l, q in enumerate(P.moduli):
            ul = residues(u, q)
            for cc in range(2):
                if coeff_idx is None:
                    pu = negacyclic_mul(pk[cc, l], ul, q)
                else:
                    pu = negacyclic_coeffs(pk[cc, l], ul, q, idx)
                vals = [a + int(b) + int(ei) for a, b, ei in zip(acc[cc][l], pu, e[cc])]
                if cc == 0:
                    vals = [v + f - d for v, f, d in zip(vals, fl, ds)]
                ct_o[cc, l] = residues(vals, q)
        result[o] = ct_o
        # model owner's share: s at the output slots (+ bias on the output channel)
        pos = {int(j): p for p, j in enumerate(idx)}
        for slot, (m, r, y, x) in E.out_slots(g, tile, mi, ri, oyi, oxi):
            if slot in pos:
                v = s[pos[slot]]
                if bias_v is not None:
                    v = (v + int(bias_v[r])) % t
                out_v[m, r, y, x] = v
    return result, E.from_virtual_out(layer, op, out_v)


def decrypt_output(P, sk, layer, op, tile, cts):
    """Data owner: decrypt every output ciphertext and gather its share (pi_y^-1)."""
    g = E.geometry(layer, op)
    c = E.counts(g, tile)
    out_v = np.zeros((g.M, g.R, g.OH, g.OW), dtype=np.int64)
    for o, (mi, ri, oyi, oxi) in enumerate(E.out_tiles(c)):
        m = bfv.decrypt(P, sk, cts[o])
        for slot, (mm, r, y, x) in E.out_slots(g, tile, mi, ri, oyi, oxi):
            out_v[mm, r, y, x] = m[slot]
    return E.from_virtual_out(layer, op, out_v)


# ------------------------------------------------------- whole protocols

def linear_fwd(P, keys, layer, plan, x0, x1, W, seed, nonce, bias=None):
    """Alg. 1.  Returns (y0, y1, cts) with y0 + y1 = W o X + b mod t."""
    cts_x = encrypt_operand(P, keys["pk"], layer, plan, OPERAND_X_FWD, x1, seed, nonce)
    out, y0 = mo_product(P, keys["pk"], layer, "fwd", plan["fwd"], [(("ct", cts_x), ("pt", W))], seed, nonce,
                         add_share=x0, bias=bias)
    cts = [out[o] for o in range(len(out))]
    y1 = decrypt_output(P, keys["sk"], layer, "fwd", plan["fwd"], cts)
    return y0, y1, cts


def linear_bwd(P, keys, layer, plan, x0, x1, dy0, dy1, W, seed, nonce, enc_nonce=None):
    """Input gradient by the Alg. 1 pattern and the weight-gradient cross terms
    of Alg. 2.  Returns dict with dx0, dx1 (dx0 + dx1 = dY o_x W) and dw_mask,
    dw_dec (dw_mask + dw_dec = dY0 o X1 + dY1 o X0, the cross terms)."""
    pk = keys["pk"]
    en = nonce if enc_nonce is None else enc_nonce
    ct_dy_dx = encrypt_operand(P, pk, layer, plan, OPERAND_DY_DX, dy1, seed, en)
    ct_x_dw = encrypt_operand(P, pk, layer, plan, OPERAND_X_DW, x1, seed, en)
    ct_dy_dw = encrypt_operand(P, pk, layer, plan, OPERAND_DY_DW, dy1, seed, en)
    out_dx, dx0 = mo_product(P, pk, layer, "dx", plan["dx"], [(("ct", ct_dy_dx), ("pt", W))], seed, nonce,
                             add_share=dy0)
    out_dw, dw_mask = mo_product(P, pk, layer, "dw", plan["dw"],
                                 [(("ct", ct_x_dw), ("pt", dy0)), (("pt", x0), ("ct", ct_dy_dw))], seed, nonce)
    cts_dx = [out_dx[o] for o in range(len(out_dx))]
    cts_dw = [out_dw[o] for o in range(len(out_dw))]
    dx1 = decrypt_output(P, keys["sk"], layer, "dx", plan["dx"], cts_dx)
    dw_dec = decrypt_output(P, keys["sk"], layer, "dw", plan["dw"], cts_dw)
    return dict(dx0=dx0, dx1=dx1, dw_mask=dw_mask, dw_dec=dw_dec, cts_dx=cts_dx, cts_dw=cts_dw,
                ct_dy_dx=ct_dy_dx, ct_x_dw=ct_x_dw, ct_dy_dw=ct_dy_dw)
