"""The allocation-free forward product (pencil_linear_fwd_noalloc) against the
allocating one (pencil_linear_fwd), through the C ABI: the same ciphertexts
and model-owner shares bit for bit, on two calls in a row (the second on a
smaller layer, so the scratch array still holds the first call's staging),
and a layer whose workspace exceeds the scratch array is refused."""
import ctypes

import pytest
import torch

from workloads import CONFIGS, config_tensors
from workloads.configs import fc

from gpu_common import dev

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 128 << 20


def _p(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _noalloc(ctx, layer, plan, ct_x, x0, w, nonce):
    from paper_2403_11166_amd import _abi as A
    from paper_2403_11166_amd.api import layer_struct, plan_struct
    sz = ctx.layout(layer, plan)
    ct_y = ctx.empty_cts(sz.n_out[0])
    y0 = torch.empty(layer.y_shape(), dtype=torch.int64, device="cuda")
    st = ctx.lib.pencil_linear_fwd_noalloc(ctx.h, ctypes.byref(layer_struct(layer)), ctypes.byref(plan_struct(plan)),
                                           _p(ct_x), _p(x0), _p(w), None, _p(ct_y), _p(y0), nonce,
                                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, ct_y, y0


def _case(ctx, layer, ts, nonce):
    plan = ctx.plan_auto(layer)
    assert ctx.layout(layer, plan).ws_fwd_bytes <= SCRATCH_BYTES
    ct_x = ctx.encrypt(layer, plan, "x_fwd", dev(ts["x1"]), nonce)
    x0, w = dev(ts["x0"]), dev(ts["W"])
    ref_ct, ref_y0 = ctx.linear_fwd(layer, plan, ct_x, x0, w, nonce + 1)
    st, ct_y, y0 = _noalloc(ctx, layer, plan, ct_x, x0, w, nonce + 1)
    torch.cuda.synchronize()
    assert st == 0, ctx.lib.pencil_last_error(ctx.h)
    assert torch.equal(ct_y, ref_ct), "output ciphertexts differ"
    assert torch.equal(y0, ref_y0), "model owner's shares differ"


def test_noalloc_forward_matches_the_allocating_call_twice():
    from paper_2403_11166_amd import Context
    big = CONFIGS[2].layers[0]                       # FC 784 -> 128, batch 64, N = 8192
    ctx = Context(big.log2_n, big.num_limbs, big.prime_bits, seed=21)
    _case(ctx, big, config_tensors(CONFIGS[2])[0], 100)
    small = fc(8, 64, 10, x_dist=("normal", 1.0), w_dist=("normal", 0.1), log2_n=big.log2_n,
               num_limbs=big.num_limbs, prime_bits=big.prime_bits)
    from workloads.gen import layer_tensors
    _case(ctx, small, layer_tensors(small, seed=22), 200)


def test_noalloc_refuses_a_workspace_beyond_the_scratch():
    from paper_2403_11166_amd import Context
    from paper_2403_11166_amd._abi import PENCIL_EUNSUPPORTED
    layer = CONFIGS[5].layers[0]                     # conv 64 -> 64 on 32x32, N = 16384: GBs of staging
    ctx = Context(layer.log2_n, layer.num_limbs, layer.prime_bits, seed=23)
    plan = ctx.plan_auto(layer)
    assert ctx.layout(layer, plan).ws_fwd_bytes > SCRATCH_BYTES
    # the size check runs on the host before any launch; tiny stand-in buffers suffice
    buf = torch.zeros(2 * ctx.L * ctx.n, dtype=torch.int64, device="cuda")
    from paper_2403_11166_amd.api import layer_struct, plan_struct
    st = ctx.lib.pencil_linear_fwd_noalloc(ctx.h, ctypes.byref(layer_struct(layer)), ctypes.byref(plan_struct(plan)),
                                           _p(buf), _p(buf), _p(buf), None, _p(buf), _p(buf), 1, None)
    assert st == PENCIL_EUNSUPPORTED
    assert b"workspace" in ctx.lib.pencil_last_error(ctx.h)
