"""Thin Python binding over the C ABI.  PyTorch provides device memory and the
stream; every step of the product runs in libpencil.so's HIP kernels.

Ciphertexts are held in int64 tensors whose bits are the uint64 residues
([n][2][L][N]); Z_t tensors are int64 in [0, t).
"""
import ctypes
import os
import threading

import torch

from . import _abi as A

OPERANDS = {"x_fwd": A.X_FWD, "dy_dx": A.DY_DX, "x_dw": A.X_DW, "dy_dw": A.DY_DW}
OPS = {"fwd": A.OP_FWD, "dx": A.OP_DX, "dw": A.OP_DW}


KINDS = {"fc": 0, "conv": 1, "conv1d": 2}


def layer_struct(layer):
    """A pencil_layer from a LayerSpec-like object (kind 'fc' / 'conv' / 'conv1d') or a dict."""
    if isinstance(layer, A.Layer):
        return layer
    get = (lambda k: layer[k]) if isinstance(layer, dict) else (lambda k: getattr(layer, k))
    kind = KINDS.get(get("kind"), get("kind"))
    stride = _get(layer, "stride", 1)
    return A.Layer(int(kind), get("batch"), get("c_in"), get("c_out"), get("h"), get("w"), get("k"), get("pad"),
                   int(stride))


def stride_map(layer):
    """The stride-1 layer a strided layer runs as (a dict usable wherever a layer is)."""
    e = A.Layer()
    A.check(A.load().pencil_stride_map(ctypes.byref(layer_struct(layer)), ctypes.byref(e)))
    kind = {v: k for k, v in KINDS.items()}[e.kind]
    return dict(kind=kind, batch=e.batch, c_in=e.c_in, c_out=e.c_out, h=e.h, w=e.w, k=e.k, pad=e.pad, stride=1)


def tile_struct(t):
    return A.Tile(*(int(v) for v in t))


def plan_struct(plan):
    """From {'fwd': (m,r,k,oh,ow,kh,kw), 'dx': ..., 'dw': ...}; a missing op gets
    the all-zero tile, which marks it as not planned."""
    if isinstance(plan, A.Plan):
        return plan
    zero = (0,) * 7
    p = A.Plan(tile_struct(plan.get("fwd", zero)), tile_struct(plan.get("dx", zero)),
               tile_struct(plan.get("dw", zero)))
    for i, v in enumerate(plan.get("sched", (0, 0, 0))):
        p.sched[i] = int(v)
    return p


def plan_dict(p):
    return {"fwd": p.fwd.astuple(), "dx": p.dx.astuple(), "dw": p.dw.astuple(), "sched": tuple(p.sched)}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, name, dtype=torch.int64):
    if t.device.type != "cuda" or not t.is_contiguous() or t.dtype != dtype:
        raise ValueError(f"{name} must be a contiguous {str(dtype).split('.')[-1]} CUDA tensor")


# Every random value is drawn from Philox keyed by (seed, nonce): two calls that
# share a seed must not share a nonce.  Nonces drawn automatically (by the
# autograd engines and Context.reserve_nonces) come from one counter per seed
# for the whole process, starting at 2^32 so that they stay clear of the small
# explicit nonces of tests and benchmarks.
AUTO_NONCE_BASE = 1 << 32
_auto_nonces = {}
_auto_lock = threading.Lock()


def reserve_nonces(seed, count=1):
    """Reserve `count` consecutive nonces for key seed `seed`; returns the first.
    Reservations for one seed never overlap within the process."""
    if count < 1:
        raise ValueError("reserve_nonces: count must be positive")
    with _auto_lock:
        first = _auto_nonces.get(seed, AUTO_NONCE_BASE)
        if first + count > 1 << 64:
            raise RuntimeError("reserve_nonces: nonce space of this seed exhausted")
        _auto_nonces[seed] = first + count
    return first


def fresh_seed():
    """A key seed from the operating system's random source."""
    return int.from_bytes(os.urandom(8), "little")


class Context:
    """A BFV parameter set, its key pair and NTT tables on the current GPU.

    seed keys every random value (the key pair included); None draws a fresh
    one from the operating system, so that separately created contexts never
    share keys or random streams by accident."""

    def __init__(self, log2_n, num_limbs, prime_bits=60, seed=None, t=0, flood_bits=0, primes=None):
        if seed is None:
            seed = fresh_seed()
        self.lib = A.load()
        p = A.Params()
        p.log2_n, p.num_limbs, p.prime_bits, p.flood_bits = log2_n, num_limbs, prime_bits, flood_bits
        for i, q in enumerate(primes or []):
            p.primes[i] = q
        p.t, p.seed = t, seed
        torch.cuda.init()
        h = ctypes.c_void_p()
        A.check(self.lib.pencil_ctx_create(ctypes.byref(p), ctypes.byref(h)), None)
        self.h = h
        info = A.Info()
        self._check(self.lib.pencil_ctx_info(self.h, ctypes.byref(info)))
        self.n = 1 << info.log2_n
        self.L = info.num_limbs
        self.t = info.t
        self.flood_bits = info.flood_bits
        self.primes = [info.primes[i] for i in range(self.L)]
        self.psi = [info.psi[i] for i in range(self.L)]
        self.seed = info.seed
        self.device = torch.device("cuda", torch.cuda.current_device())

    @classmethod
    def for_layer(cls, layer, seed=None):
        return cls(layer.log2_n, layer.num_limbs, layer.prime_bits, seed)

    def reserve_nonces(self, count=1):
        """`count` consecutive nonces no other reservation on this key seed holds."""
        return reserve_nonces(self.seed, count)

    def _check(self, st):
        A.check(st, self.h)

    def close(self):
        if getattr(self, "h", None):
            self.lib.pencil_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- host
    def export_keys(self):
        import numpy as np
        sk = np.empty(self.n, dtype=np.int64)
        pk = np.empty((2, self.L, self.n), dtype=np.uint64)
        self._check(self.lib.pencil_export_keys(self.h, sk.ctypes.data_as(A.c_i64p), pk.ctypes.data_as(A.c_u64p)))
        return sk, pk

    def plan_auto(self, layer):
        p = A.Plan()
        self._check(self.lib.pencil_plan_auto(self.h, ctypes.byref(layer_struct(layer)), ctypes.byref(p)))
        return p

    def autotune(self, layer, plan, cache_path=None):
        """Measure the NTT width, the planner's best partitions and the nine multiply-accumulate
        schedules on this GPU and return the tuned plan (tune before encrypting with it)."""
        p = plan_struct(plan)
        q = A.Plan()
        ctypes.pointer(q)[0] = p
        self._check(self.lib.pencil_autotune(self.h, ctypes.byref(layer_struct(layer)), ctypes.byref(q),
                                             cache_path.encode() if cache_path else None))
        return q

    def ntt_loge(self):
        """log2 of the residues each NTT thread keeps (the autotuner's choice for this context)."""
        info = A.Info()
        self._check(self.lib.pencil_ctx_info(self.h, ctypes.byref(info)))
        return info.ntt_loge

    def layout(self, layer, plan):
        s = A.Sizes()
        self._check(self.lib.pencil_layout(self.h, ctypes.byref(layer_struct(layer)),
                                           ctypes.byref(plan_struct(plan)), ctypes.byref(s)))
        return s

    # ---------------------------------------------------------------- device
    def _ws(self, nbytes):
        return torch.empty(max(int(nbytes), 8), dtype=torch.uint8, device=self.device)

    def empty_cts(self, count):
        return torch.empty((int(count), 2, self.L, self.n), dtype=torch.int64, device=self.device)

    def encrypt(self, layer, plan, operand, share, nonce, out=None, ws=None):
        op = OPERANDS.get(operand, operand)
        plan = plan_struct(plan)
        sz = self.layout(layer, plan)
        _need(share, "share")
        out = self.empty_cts(sz.n_ct[op]) if out is None else out
        ws = self._ws(sz.ws_enc_bytes) if ws is None else ws
        self._check(self.lib.pencil_encrypt(self.h, ctypes.byref(layer_struct(layer)), ctypes.byref(plan), op,
                                            _ptr(share), _ptr(out), _ptr(ws), nonce, _stream()))
        return out

    def linear_fwd(self, layer, plan, ct_x1, x0, w, nonce, bias=None, ws=None, out=None):
        plan = plan_struct(plan)
        sz = self.layout(layer, plan)
        for t, nm in ((x0, "x0"), (w, "w")):
            _need(t, nm)
        ct_y = self.empty_cts(sz.n_out[0]) if out is None else out[0]
        y0 = torch.empty(_y_shape(layer), dtype=torch.int64, device=self.device) if out is None else out[1]
        ws = self._ws(sz.ws_fwd_bytes) if ws is None else ws
        self._check(self.lib.pencil_linear_fwd(self.h, ctypes.byref(layer_struct(layer)), ctypes.byref(plan),
                                               _ptr(ct_x1), _ptr(x0), _ptr(w), _ptr(bias), _ptr(ct_y), _ptr(y0),
                                               _ptr(ws), nonce, _stream()))
        return ct_y, y0

    def linear_bwd(self, layer, plan, ct_dy_dx, ct_x_dw, ct_dy_dw, dy0, x0, w, nonce, ws=None, out=None,
                   do_dx=True, do_dw=True):
        plan = plan_struct(plan)
        sz = self.layout(layer, plan)
        ws = self._ws(sz.ws_bwd_bytes) if ws is None else ws
        if out is None:
            ct_dx = self.empty_cts(sz.n_out[1]) if do_dx else None
            dx0 = torch.empty(_x_shape(layer), dtype=torch.int64, device=self.device) if do_dx else None
            ct_dw = self.empty_cts(sz.n_out[2]) if do_dw else None
            dwm = torch.empty(_w_shape(layer), dtype=torch.int64, device=self.device) if do_dw else None
        else:
            ct_dx, dx0, ct_dw, dwm = out
        self._check(self.lib.pencil_linear_bwd(self.h, ctypes.byref(layer_struct(layer)), ctypes.byref(plan),
                                               _ptr(ct_dy_dx), _ptr(ct_x_dw), _ptr(ct_dy_dw), _ptr(dy0), _ptr(x0),
                                               _ptr(w), _ptr(ct_dx), _ptr(dx0), _ptr(ct_dw), _ptr(dwm), _ptr(ws),
                                               nonce, _stream()))
        return ct_dx, dx0, ct_dw, dwm

    def decrypt(self, layer, plan, op, ct, ws=None):
        opi = OPS.get(op, op)
        plan = plan_struct(plan)
        sz = self.layout(layer, plan)
        shape = (_y_shape, _x_shape, _w_shape)[opi](layer)
        share = torch.empty(shape, dtype=torch.int64, device=self.device)
        ws = self._ws(sz.ws_dec_bytes) if ws is None else ws
        self._check(self.lib.pencil_decrypt(self.h, ctypes.byref(layer_struct(layer)), ctypes.byref(plan), opi,
                                            _ptr(ct), _ptr(share), _ptr(ws), _stream()))
        return share

    def decrypt_checked(self, layer, plan, op, ct, ws=None):
        """decrypt() plus the noise check: returns (share, largest noise as a
        fraction of q/t); raises PencilError(ENOISE) when it reaches 1/4.
        Waits for the stream."""
        opi = OPS.get(op, op)
        plan = plan_struct(plan)
        sz = self.layout(layer, plan)
        shape = (_y_shape, _x_shape, _w_shape)[opi](layer)
        share = torch.empty(shape, dtype=torch.int64, device=self.device)
        ws = self._ws(sz.ws_dec_bytes) if ws is None else ws
        frac = ctypes.c_double()
        self._check(self.lib.pencil_decrypt_checked(self.h, ctypes.byref(layer_struct(layer)), ctypes.byref(plan),
                                                    opi, _ptr(ct), _ptr(share), _ptr(ws), ctypes.byref(frac),
                                                    _stream()))
        return share, frac.value

    def zt_linear(self, layer, op, a, b):
        """Exact Z_t product of plaintext tensors with the layer's operator."""
        opi = OPS.get(op, op)
        _need(a, "a")
        _need(b, "b")
        shape = (_y_shape, _x_shape, _w_shape)[opi](layer)
        out = torch.empty(shape, dtype=torch.int64, device=self.device)
        self._check(self.lib.pencil_zt_linear(self.h, ctypes.byref(layer_struct(layer)), opi, _ptr(a), _ptr(b),
                                              _ptr(out), _stream()))
        return out

    def zt_combine(self, terms, coeffs, base=None, out=None):
        """out = base + sum_i coeffs[i] * terms[i] mod t, element-wise (int64 tensors in [0, t));
        coefficients are signed integers (the library takes them mod t)."""
        terms = list(terms)
        like = base if base is not None else terms[0]
        for x in terms + ([base] if base is not None else []):
            _need(x, "term")
            if x.shape != like.shape:
                raise ValueError("zt_combine: shape mismatch")
        out = torch.empty_like(like) if out is None else out
        n = len(terms)
        ptrs = (ctypes.c_void_p * max(n, 1))(*[x.data_ptr() for x in terms])
        cs = (ctypes.c_int64 * max(n, 1))(*[int(c) for c in coeffs])
        self._check(self.lib.pencil_zt_combine(self.h, like.numel(), n, ptrs, cs, _ptr(base), _ptr(out), _stream()))
        return out

    def zt_combine_outer(self, terms, ci, cj, base=None, out=None):
        """out = base + sum_ij ci[i] cj[j] terms[i][j] mod t (terms: nested lists, n_i x n_j)."""
        flat = [x for row in terms for x in row]
        like = base if base is not None else flat[0]
        for x in flat + ([base] if base is not None else []):
            _need(x, "term")
            if x.shape != like.shape:
                raise ValueError("zt_combine_outer: shape mismatch")
        out = torch.empty_like(like) if out is None else out
        ni, nj = len(terms), len(terms[0]) if terms else 0
        ptrs = (ctypes.c_void_p * max(ni * nj, 1))(*[x.data_ptr() for x in flat])
        a = (ctypes.c_int64 * max(ni, 1))(*[int(c) for c in ci])
        b = (ctypes.c_int64 * max(nj, 1))(*[int(c) for c in cj])
        self._check(self.lib.pencil_zt_combine_outer(self.h, like.numel(), ni, nj, ptrs, a, b, _ptr(base), _ptr(out),
                                                     _stream()))
        return out

    def bias_grad(self, layer, dy):
        """Bias-gradient share: dy summed over every axis but the channel axis, mod t."""
        _need(dy, "dy")
        if tuple(dy.shape) != tuple(_y_shape(layer)):
            raise ValueError("bias_grad: dy has the wrong shape")
        out = torch.empty(_get(layer, "c_out"), dtype=torch.int64, device=self.device)
        self._check(self.lib.pencil_bias_grad(self.h, ctypes.byref(layer_struct(layer)), _ptr(dy), _ptr(out),
                                              _stream()))
        return out

    def zt_encode(self, x):
        """float64 fixed-point integers -> int64 in [0, t) (round to nearest, mod t)."""
        x = x.detach().contiguous()
        _need(x, "x", torch.float64)
        out = torch.empty(x.shape, dtype=torch.int64, device=x.device)
        self._check(self.lib.pencil_zt_encode(self.h, x.numel(), _ptr(x), _ptr(out), _stream()))
        return out

    def zt_decode(self, v):
        """int64 in [0, t) -> centred float64 representatives."""
        v = v.contiguous()
        _need(v, "v")
        out = torch.empty(v.shape, dtype=torch.float64, device=v.device)
        self._check(self.lib.pencil_zt_decode(self.h, v.numel(), _ptr(v), _ptr(out), _stream()))
        return out

    def zt_share(self, v, nonce, obj=0):
        """Additive shares (s0 uniform over Z_t from the stream (nonce, obj), s1 = v - s0)."""
        v = v.contiguous()
        _need(v, "v")
        s0 = torch.empty_like(v)
        s1 = torch.empty_like(v)
        self._check(self.lib.pencil_zt_share(self.h, v.numel(), _ptr(v), int(nonce) & ((1 << 64) - 1),
                                             int(obj) & ((1 << 64) - 1), _ptr(s0), _ptr(s1), _stream()))
        return s0, s1

    def dp_noise_(self, x, sd, nonce, obj):
        """In place: x + floor(sd * z) mod t with z standard normal draws of the stream (nonce, obj)."""
        _need(x, "x")
        self._check(self.lib.pencil_dp_noise(self.h, x.numel(), float(sd), int(nonce) & ((1 << 64) - 1),
                                             int(obj) & ((1 << 64) - 1), _ptr(x), _stream()))
        return x

    def stride_relayout(self, layer, which, x):
        """Space-to-depth relayout between a strided layer and its stride-1 equivalent:
        which 'x' (X -> X'), 'w' (W -> W'), 'dx' (dX' -> dX) or 'dw' (dW' -> dW)."""
        wi = {"x": 0, "w": 1, "dx": 2, "dw": 3}[which]
        _need(x, "x")
        eq = stride_map(layer)
        shape = (_x_shape(eq), _w_shape(eq), _x_shape(layer), _w_shape(layer))[wi]
        want_in = (_x_shape(layer), _w_shape(layer), _x_shape(eq), _w_shape(eq))[wi]
        if tuple(x.shape) != tuple(want_in):
            raise ValueError(f"stride_relayout: input shape {tuple(x.shape)}, expected {want_in}")
        out = torch.empty(shape, dtype=torch.int64, device=self.device)
        self._check(self.lib.pencil_stride_relayout(self.h, ctypes.byref(layer_struct(layer)), wi, _ptr(x),
                                                    _ptr(out), _stream()))
        return out

    def ntt(self, polys, inverse=False):
        """In-place negacyclic NTT of an int64 tensor [count][L][N] of residues."""
        count = polys.numel() // (self.L * self.n)
        fn = self.lib.pencil_ntt_inverse if inverse else self.lib.pencil_ntt_forward
        self._check(fn(self.h, _ptr(polys), count, _stream()))
        return polys


def _get(layer, k, default=None):
    if isinstance(layer, dict):
        return layer.get(k, default) if default is not None else layer[k]
    return getattr(layer, k, default) if default is not None else getattr(layer, k)


def _kind(layer):
    k = _get(layer, "kind")
    return {v: n for n, v in KINDS.items()}.get(k, k)


def _is_fc(layer):
    return _kind(layer) == "fc"


def _x_shape(layer):
    B, ci = _get(layer, "batch"), _get(layer, "c_in")
    if _is_fc(layer):
        return (B, ci)
    if _kind(layer) == "conv1d":
        return (B, ci, _get(layer, "w"))
    return (B, ci, _get(layer, "h"), _get(layer, "w"))


def _y_shape(layer):
    B, co = _get(layer, "batch"), _get(layer, "c_out")
    if _is_fc(layer):
        return (B, co)
    h, w, k, p = _get(layer, "h"), _get(layer, "w"), _get(layer, "k"), _get(layer, "pad")
    s = max(1, int(_get(layer, "stride", 1)))
    wo = (w + 2 * p - k) // s + 1
    if _kind(layer) == "conv1d":
        return (B, co, wo)
    return (B, co, (h + 2 * p - k) // s + 1, wo)


def _w_shape(layer):
    ci, co, k = _get(layer, "c_in"), _get(layer, "c_out"), _get(layer, "k")
    if _is_fc(layer):
        return (co, ci)
    if _kind(layer) == "conv1d":
        return (co, ci, k)
    return (co, ci, k, k)


class Step:
    """All products of several layers as one batched launch sequence.

    layers: list of (Context, layer, plan); ops: subset of ("fwd", "dx", "dw").
    Bind once with the device buffers of every layer, then run() or replay a
    captured graph.  Layer i uses nonce + 2i (forward) and nonce + 2i + 1
    (backward), matching the per-layer calls made with those nonces.
    """

    def __init__(self, layers, ops=("fwd", "dx", "dw")):
        self.lib = A.load()
        self.entries = [(c, l, plan_struct(p)) for c, l, p in layers]
        n = len(layers)
        ctxs = (ctypes.c_void_p * n)(*[c.h.value for c, _, _ in self.entries])
        lays = (A.Layer * n)(*[layer_struct(l) for _, l, _ in self.entries])
        plans = (A.Plan * n)(*[p for _, _, p in self.entries])
        mask = sum(1 << OPS[o] for o in ops)
        h = ctypes.c_void_p()
        st = self.lib.pencil_step_create(ctxs, lays, plans, n, mask, ctypes.byref(h))
        if st != A.PENCIL_OK:
            raise A.PencilError(st, self.lib.pencil_last_error(None).decode())
        self.h = h
        self.ops = ops
        self._keep = None

    def _check(self, st):
        if st != A.PENCIL_OK:
            raise A.PencilError(st, self.lib.pencil_step_last_error(self.h).decode())

    def workspace_bytes(self):
        b = ctypes.c_uint64()
        self._check(self.lib.pencil_step_workspace(self.h, ctypes.byref(b)))
        return b.value

    def bind(self, ios, ws):
        """ios: one dict per layer with the tensors named as in pencil_step_io."""
        arr = (A.StepIO * len(ios))()
        for i, d in enumerate(ios):
            for k, v in d.items():
                if v is not None:
                    setattr(arr[i], k, v.data_ptr())
        self._keep = (ios, ws)
        self._check(self.lib.pencil_step_bind(self.h, arr, ctypes.c_void_p(ws.data_ptr())))

    def run(self, nonce):
        self._check(self.lib.pencil_step_run(self.h, nonce, _stream()))

    def capture(self):
        self._check(self.lib.pencil_step_graph_capture(self.h))

    def set_nonce(self, nonce):
        self._check(self.lib.pencil_step_set_nonce(self.h, nonce, _stream()))

    def replay(self):
        self._check(self.lib.pencil_step_graph_launch(self.h, _stream()))

    def close(self):
        if getattr(self, "h", None):
            self.lib.pencil_step_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
