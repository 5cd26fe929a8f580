"""A linear layer evaluated by the encrypted two-party protocol, as a
torch.autograd.Function.

Forward (Alg. 1): the input X is split into additive shares over Z_t, the data
owner's share is encrypted, the model owner's product adds its share and
multiplies by W, and the decrypted share plus the model owner's mask
reconstruct Y = W o X.  Backward: the gradient with respect to X by the same
pattern with the transposed operator (Sec. III.B.2), and the weight gradient
as the two encrypted cross terms of Alg. 2 plus the two parties' local terms,
the bias gradient, and optionally the data owner's DP perturbation.

Tensors carry fixed-point integers in float64 (autograd rejects integer
dtypes; t < 2^53 keeps them exact) in centred form, (-t/2, t/2).  Every step
runs in libpencil's HIP kernels -- the Z_t encoding and its centred view, the
secret sharing, the products; this module sequences the calls and reserves
the nonces.
"""
import torch

from .api import Context, _get, stride_map


class EncryptedLinearEngine:
    """Context, partition and randomness of one layer's encrypted products.

    A strided layer runs as its stride-1 space-to-depth equivalent: each party
    relayouts its own shares (the maps are linear) and the gradients map back.
    dp_sd_w / dp_sd_b: standard deviations, in fixed-point units, of the data
    owner's perturbation of its weight- and bias-gradient shares (Sec. III.B.2;
    0 = none)."""

    def __init__(self, layer, ctx: Context, plan=None, dp_sd_w=0.0, dp_sd_b=0.0):
        self.layer = layer
        self.strided = int(_get(layer, "stride", 1)) > 1
        self.eq = stride_map(layer) if self.strided else layer
        self.ctx = ctx
        self.plan = ctx.plan_auto(self.eq) if plan is None else plan
        self.nonce = None  # the last nonce drawn
        self.dp_sd_w, self.dp_sd_b = float(dp_sd_w), float(dp_sd_b)

    def next_nonce(self):
        """A nonce no other engine or reservation on the context's key seed uses."""
        self.nonce = self.ctx.reserve_nonces(1)
        return self.nonce

    def shares(self, v):
        """Additive shares of v over Z_t, from a fresh nonce of the context's seed."""
        return self.ctx.zt_share(v, self.next_nonce())

    def to_eq(self, which, v):
        return self.ctx.stride_relayout(self.layer, which, v) if self.strided else v

    def from_eq(self, which, v):
        return self.ctx.stride_relayout(self.layer, which, v) if self.strided else v


class EncryptedLinearFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x, w, b, engine):
        c, L = engine.ctx, engine.eq
        X, W = c.zt_encode(x), c.zt_encode(w)
        bz = c.zt_encode(b) if b is not None else None
        x0, x1 = engine.shares(X)
        x0, x1, W = engine.to_eq("x", x0), engine.to_eq("x", x1), engine.to_eq("w", W)
        ct_x = c.encrypt(L, engine.plan, "x_fwd", x1, engine.next_nonce())
        ct_y, y0 = c.linear_fwd(L, engine.plan, ct_x, x0, W, engine.next_nonce(), bias=bz)
        y1 = c.decrypt(L, engine.plan, "fwd", ct_y)
        fctx.engine = engine
        fctx.has_bias = b is not None
        fctx.save_for_backward(x0, x1, W)
        return c.zt_decode(c.zt_combine([y0, y1], [1, 1]))

    @staticmethod
    def backward(fctx, grad_y):
        engine = fctx.engine
        c, L = engine.ctx, engine.eq
        x0, x1, W = fctx.saved_tensors
        dY = c.zt_encode(grad_y)
        dy0, dy1 = engine.shares(dY)
        n = engine.next_nonce()
        ct_dy_dx = c.encrypt(L, engine.plan, "dy_dx", dy1, n)
        ct_x_dw = c.encrypt(L, engine.plan, "x_dw", x1, n)
        ct_dy_dw = c.encrypt(L, engine.plan, "dy_dw", dy1, n)
        ct_dx, dx0, ct_dw, dw_mask = c.linear_bwd(L, engine.plan, ct_dy_dx, ct_x_dw, ct_dy_dw, dy0, x0, W,
                                                  engine.next_nonce())
        dx1 = c.decrypt(L, engine.plan, "dx", ct_dx)
        dw_dec = c.decrypt(L, engine.plan, "dw", ct_dw)
        dp_nonce = engine.next_nonce()
        # Alg. 2: the data owner adds its local term to the decryption and its
        # perturbation; the model owner adds the mask and its own local term
        dw_do = c.zt_combine([c.zt_linear(L, "dw", x1, dy1)], [1], base=dw_dec, out=dw_dec)
        if engine.dp_sd_w > 0:
            c.dp_noise_(dw_do, engine.dp_sd_w, dp_nonce, 0)
        dW = engine.from_eq("dw", c.zt_combine([dw_mask, c.zt_linear(L, "dw", x0, dy0)], [1, 1], base=dw_do))
        dX = c.zt_combine([engine.from_eq("dx", dx0), engine.from_eq("dx", dx1)], [1, 1])
        db = None
        if fctx.has_bias:
            db_do = c.bias_grad(L, dy1)
            if engine.dp_sd_b > 0:
                c.dp_noise_(db_do, engine.dp_sd_b, dp_nonce, 1)
            db = c.zt_decode(c.zt_combine([c.bias_grad(L, dy0)], [1], base=db_do))
        return c.zt_decode(dX), c.zt_decode(dW), db, None


def encrypted_linear(x, w, engine, b=None):
    """Y = W o X (+ b) through the encrypted protocol; differentiable in x, w and b."""
    return EncryptedLinearFunction.apply(x, w, b, engine)
