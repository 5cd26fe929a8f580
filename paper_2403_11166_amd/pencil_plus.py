"""Pencil+ (Sec. IV.C, Alg. 3 and Alg. 4): the products of a linear layer with
the homomorphic work moved to a preprocessing phase, on the library's kernels.

Preprocessing of one operator (m^2 homomorphic products): the data owner (DO)
encrypts its masks v'_j, the model owner (MO) multiplies them by its masks
u'_i with a fresh output mask s_ij (the same re-randomised, flooded and masked
product as the online protocol), and the DO decrypts.  The parties keep
<u'_i o v'_j>_0 = s_ij and <u'_i o v'_j>_1 = u'_i o v'_j - s_ij.

Online (no homomorphic operation): Z_t linear combinations
(pencil_zt_combine) and one plaintext product of the layer's operator per
party (pencil_zt_linear), the per-mask products folded by linearity.

Operators (the MO's operand u, the DO's operand v):
    fwd   u = W,      v = <X>_1   -> shaped like Y
    dx    u = W,      v = <dY>_1  -> shaped like dX
    dw01  u = <dY>_0, v = <X>_1   -> shaped like W
    dw10  u = <X>_0,  v = <dY>_1  -> shaped like W
Both parties run in this process; which party computes what is marked.
"""
import torch

KINDS = ("fwd", "dx", "dw01", "dw10")


def _zeros(shape):
    return torch.zeros(shape, dtype=torch.int64, device="cuda")


def apply(ctx, layer, kind, u, v):
    """u o v mod t on the GPU (plaintext operator, pencil_zt_linear)."""
    if kind == "fwd":
        return ctx.zt_linear(layer, "fwd", v, u)
    if kind == "dx":
        return ctx.zt_linear(layer, "dx", v, u)
    if kind == "dw01":
        return ctx.zt_linear(layer, "dw", v, u)
    if kind == "dw10":
        return ctx.zt_linear(layer, "dw", u, v)
    raise ValueError(kind)


def prep(ctx, layer, plan, kind, u_masks, v_masks, nonce):
    """Alg. 3's preprocessing: returns (share0[i][j], share1[i][j]) for the m x m
    mask pairs.  Nonces nonce, nonce + 1, ... are used for the encryptions and
    products (distinct per call)."""
    m = len(u_masks)
    X, Y, Wsh = layer.x_shape(), layer.y_shape(), layer.w_shape()
    share0 = [[None] * m for _ in range(m)]
    share1 = [[None] * m for _ in range(m)]
    zero_x, zero_y, zero_w = _zeros(X), _zeros(Y), _zeros(Wsh)
    # the ciphertext the unused term of a weight-gradient product multiplies by zero
    if kind == "dw01":
        ct_zero = ctx.encrypt(layer, plan, "dy_dw", zero_y, nonce)
    elif kind == "dw10":
        ct_zero = ctx.encrypt(layer, plan, "x_dw", zero_x, nonce)
    nc = nonce + 1
    for j in range(m):
        # DO: Enc(v'_j) in the operator's layout
        operand = {"fwd": "x_fwd", "dx": "dy_dx", "dw01": "x_dw", "dw10": "dy_dw"}[kind]
        ct_v = ctx.encrypt(layer, plan, operand, v_masks[j], nc)
        nc += 1
        for i in range(m):
            # MO: u'_i o Enc(v'_j) - s_ij (re-randomised, flooded, masked)
            if kind == "fwd":
                ct, s = ctx.linear_fwd(layer, plan, ct_v, zero_x, u_masks[i], nc)
                op = "fwd"
            elif kind == "dx":
                ct, s, _, _ = ctx.linear_bwd(layer, plan, ct_v, None, None, zero_y, zero_x, u_masks[i], nc,
                                             do_dw=False)
                op = "dx"
            elif kind == "dw01":
                _, _, ct, s = ctx.linear_bwd(layer, plan, None, ct_v, ct_zero, u_masks[i], zero_x, zero_w, nc,
                                             do_dx=False)
                op = "dw"
            else:
                _, _, ct, s = ctx.linear_bwd(layer, plan, None, ct_zero, ct_v, zero_y, u_masks[i], zero_w, nc,
                                             do_dx=False)
                op = "dw"
            nc += 1
            share0[i][j] = s
            share1[i][j] = ctx.decrypt(layer, plan, op, ct)   # DO
    return share0, share1


def online(ctx, layer, kind, u, v, u_masks, v_masks, share0, share1, k, l):
    """Alg. 3's online phase.  Returns (<u o v>_0, <u o v>_1, u~, v~).

    The per-mask terms are folded by linearity before any product:
    sum_j l_j (u~ o v'_j) = u~ o (sum_j l_j v'_j), and the two-level share sums
    are one sum with coefficients k_i l_j.  Each party then runs one Z_t
    correlation per operator instead of m + 1; the outputs are the same
    integers mod t, and the messages (u~, v~) and what each party uses are
    unchanged (both parties know k and l)."""
    neg_k, neg_l = [-int(c) for c in k], [-int(c) for c in l]
    u_t = ctx.zt_combine(u_masks, neg_k, base=u)                                 # MO -> DO
    v_t = ctx.zt_combine(v_masks, neg_l, base=v)                                 # DO -> MO
    # DO: sum_j l_j <u o v'_j>_1 = u~ o (sum_j l_j v'_j) + sum_ij k_i l_j <u'_i o v'_j>_1
    v_l = ctx.zt_combine(v_masks, l)
    out1 = ctx.zt_combine_outer(share1, k, l, base=apply(ctx, layer, kind, u_t, v_l))
    # MO: u o v~ + sum_ij k_i l_j <u'_i o v'_j>_0
    out0 = ctx.zt_combine_outer(share0, k, l, base=apply(ctx, layer, kind, u, v_t))
    return out0, out1, u_t, v_t
