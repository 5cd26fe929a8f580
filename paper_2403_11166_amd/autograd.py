"""A linear layer evaluated by the encrypted two-party protocol, as a
torch.autograd.Function.

Forward (Alg. 1): the input X is split into additive shares over Z_t, the data
owner's share is encrypted, the model owner's product adds its share and
multiplies by W, and the decrypted share plus the model owner's mask
reconstruct Y = W o X.  Backward: the gradient with respect to X by the same
pattern with the transposed operator (Sec. III.B.2), and the weight gradient
as the two encrypted cross terms of Alg. 2 plus the two parties' local terms.

Tensors carry fixed-point integers in float64 (autograd rejects integer
dtypes; t < 2^53 keeps them exact) in centred form, (-t/2, t/2).  Every Z_t
product runs in libpencil's HIP kernels; this module converts dtypes and
draws the share and nonce randomness.
"""
import torch

from .api import Context


def _to_zt(x, t):
    v = torch.round(x).to(torch.int64)
    return torch.remainder(v, t).contiguous()


def _centred(v, t):
    return torch.where(v > (t - 1) // 2, v - t, v).to(torch.float64)


class EncryptedLinearEngine:
    """Context, partition and randomness of one layer's encrypted products."""

    def __init__(self, layer, ctx: Context, plan=None, seed=0):
        self.layer = layer
        self.ctx = ctx
        self.plan = ctx.plan_auto(layer) if plan is None else plan
        self.gen = torch.Generator(device=ctx.device)
        self.gen.manual_seed(seed)
        self.nonce = 1 << 32

    def next_nonce(self):
        self.nonce += 1
        return self.nonce

    def shares(self, v):
        t = self.ctx.t
        s0 = torch.randint(0, t, v.shape, generator=self.gen, device=v.device, dtype=torch.int64)
        return s0, torch.remainder(v - s0, t)


class EncryptedLinearFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x, w, engine):
        c, L, t = engine.ctx, engine.layer, engine.ctx.t
        X, W = _to_zt(x, t), _to_zt(w, t)
        x0, x1 = engine.shares(X)
        ct_x = c.encrypt(L, engine.plan, "x_fwd", x1, engine.next_nonce())
        ct_y, y0 = c.linear_fwd(L, engine.plan, ct_x, x0, W, engine.next_nonce())
        y1 = c.decrypt(L, engine.plan, "fwd", ct_y)
        fctx.engine = engine
        fctx.save_for_backward(x0, x1, W)
        return _centred(torch.remainder(y0 + y1, t), t)

    @staticmethod
    def backward(fctx, grad_y):
        engine = fctx.engine
        c, L, t = engine.ctx, engine.layer, engine.ctx.t
        x0, x1, W = fctx.saved_tensors
        dY = _to_zt(grad_y, t)
        dy0, dy1 = engine.shares(dY)
        n = engine.next_nonce()
        ct_dy_dx = c.encrypt(L, engine.plan, "dy_dx", dy1, n)
        ct_x_dw = c.encrypt(L, engine.plan, "x_dw", x1, n)
        ct_dy_dw = c.encrypt(L, engine.plan, "dy_dw", dy1, n)
        ct_dx, dx0, ct_dw, dw_mask = c.linear_bwd(L, engine.plan, ct_dy_dx, ct_x_dw, ct_dy_dw, dy0, x0, W,
                                                  engine.next_nonce())
        dx1 = c.decrypt(L, engine.plan, "dx", ct_dx)
        dw_dec = c.decrypt(L, engine.plan, "dw", ct_dw)
        # Alg. 2: the data owner adds its local term to the decryption, the model
        # owner adds the mask and its own local term
        dw_do = torch.remainder(dw_dec + c.zt_linear(L, "dw", x1, dy1), t)
        dW = torch.remainder(dw_do + dw_mask + c.zt_linear(L, "dw", x0, dy0), t)
        dX = torch.remainder(dx0 + dx1, t)
        return _centred(dX, t), _centred(dW, t), None


def encrypted_linear(x, w, engine):
    """Y = W o X through the encrypted protocol; differentiable in x and w."""
    return EncryptedLinearFunction.apply(x, w, engine)
