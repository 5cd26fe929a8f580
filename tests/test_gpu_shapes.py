"""More layer shapes on the GPU against the oracle's plain layer definitions:
the paper's Conv1d (TextCNN) and large FC layers at full size, and strided
convolutions (the MNIST CNN's stride-2 layer) run as their space-to-depth
stride-1 equivalents.  Reconstructed results are unique, so they are compared
bit for bit with the oracle's strided / 1-d layer operators."""
import numpy as np
import pytest
import torch

from oracle import linear as LN
from workloads import T_PLAIN, conv, conv1d, fc, layer_tensors

from gpu_common import dev, host_i64

pytestmark = pytest.mark.gpu

T = T_PLAIN
_ctx = {}


def context(log2_n, limbs, bits, seed=41):
    from paper_2403_11166_amd import Context
    key = (log2_n, limbs, bits, seed)
    if key not in _ctx:
        _ctx[key] = Context(log2_n, limbs, bits, seed)
    return _ctx[key]


def run_protocol(ctx, layer, ts, x0, x1, dy0, dy1, W, nonce):
    """Alg. 1 and Alg. 2 (plus the input gradient) on one stride-1 layer; every
    product on the GPU.  Returns the reconstructed Y, dX and dW."""
    plan = ctx.plan_auto(layer)
    ct_x = ctx.encrypt(layer, plan, "x_fwd", x1, nonce)
    ct_y, y0 = ctx.linear_fwd(layer, plan, ct_x, x0, W, nonce + 1)
    y1 = ctx.decrypt(layer, plan, "fwd", ct_y)
    ct_dy_dx = ctx.encrypt(layer, plan, "dy_dx", dy1, nonce + 2)
    ct_x_dw = ctx.encrypt(layer, plan, "x_dw", x1, nonce + 2)
    ct_dy_dw = ctx.encrypt(layer, plan, "dy_dw", dy1, nonce + 2)
    ct_dx, dx0, ct_dw, dwm = ctx.linear_bwd(layer, plan, ct_dy_dx, ct_x_dw, ct_dy_dw, dy0, x0, W, nonce + 3)
    dx1 = ctx.decrypt(layer, plan, "dx", ct_dx)
    dw1 = ctx.decrypt(layer, plan, "dw", ct_dw)
    loc = [ctx.zt_linear(layer, "dw", x0, dy0), ctx.zt_linear(layer, "dw", x1, dy1)]
    dW = ctx.zt_combine([dwm, dw1] + loc, [1, 1, 1, 1])
    return (ctx.zt_combine([y0, y1], [1, 1]), (dx0, dx1), dW)


FULL = [conv1d(64, 256, 128, 64, k=5, log2_n=13, num_limbs=3, prime_bits=60),      # TextCNN conv 1
        conv1d(64, 128, 128, 30, k=5, log2_n=13, num_limbs=3, prime_bits=60),      # TextCNN conv 2
        fc(64, 2048, 1001, log2_n=13, num_limbs=3, prime_bits=60)]                 # Table V's largest FC


@pytest.mark.parametrize("layer", FULL, ids=["textcnn1", "textcnn2", "fc2048x1001"])
def test_full_size_layers_reconstruct(layer):
    ctx = context(layer.log2_n, layer.num_limbs, layer.prime_bits)
    ts = layer_tensors(layer, 12)
    d = {k: dev(v) for k, v in ts.items()}
    Y, (dx0, dx1), dW = run_protocol(ctx, layer, ts, d["x0"], d["x1"], d["dy0"], d["dy1"], d["W"], 500)
    assert np.array_equal(host_i64(Y), LN.layer_op(layer, "fwd", ts["X"], ts["W"], T))
    assert np.array_equal((host_i64(dx0) + host_i64(dx1)) % T, LN.layer_op(layer, "dx", ts["dY"], ts["W"], T))
    assert np.array_equal(host_i64(dW), LN.layer_op(layer, "dw", ts["X"], ts["dY"], T))


STRIDED = [conv(64, 1, 5, 28, k=5, pad=2, stride=2, log2_n=13, num_limbs=3, prime_bits=60),   # MNIST CNN conv
           conv(3, 2, 3, 9, k=3, pad=1, stride=2, log2_n=11, num_limbs=2, prime_bits=50),
           conv(2, 3, 2, 11, k=4, pad=1, stride=3, log2_n=11, num_limbs=2, prime_bits=50),
           conv(2, 2, 3, 8, k=3, pad=0, stride=2, log2_n=11, num_limbs=2, prime_bits=50),
           conv1d(2, 3, 4, 14, k=5, pad=2, stride=2, log2_n=11, num_limbs=2, prime_bits=50)]


@pytest.mark.parametrize("layer", STRIDED, ids=["mnist_s2", "k3s2", "k4s3", "k3s2p0", "conv1d_s2"])
def test_strided_layers_reconstruct(layer):
    """Each party relayouts its own shares, the products run on the stride-1
    equivalent, and the gradients map back."""
    from paper_2403_11166_amd.api import stride_map
    ctx = context(layer.log2_n, layer.num_limbs, layer.prime_bits)
    ts = layer_tensors(layer, 13)
    eq = stride_map(layer)
    d = {k: dev(v) for k, v in ts.items()}
    rx = lambda v: ctx.stride_relayout(layer, "x", v)  # noqa: E731
    Y, (dx0e, dx1e), dWe = run_protocol(ctx, eq, ts, rx(d["x0"]), rx(d["x1"]), d["dy0"], d["dy1"],
                                        ctx.stride_relayout(layer, "w", d["W"]), 700)
    dx0, dx1 = ctx.stride_relayout(layer, "dx", dx0e), ctx.stride_relayout(layer, "dx", dx1e)
    dW = ctx.stride_relayout(layer, "dw", dWe)
    assert np.array_equal(host_i64(Y), LN.layer_op(layer, "fwd", ts["X"], ts["W"], T))
    assert np.array_equal((host_i64(dx0) + host_i64(dx1)) % T, LN.layer_op(layer, "dx", ts["dY"], ts["W"], T))
    assert np.array_equal(host_i64(dW), LN.layer_op(layer, "dw", ts["X"], ts["dY"], T))


@pytest.mark.parametrize("layer", STRIDED[1:], ids=["k3s2", "k4s3", "k3s2p0", "conv1d_s2"])
def test_relayouts_are_adjoint_pairs(layer):
    """<R_x X, Z> = <X, R_dx Z> and <R_w W, V> = <W, R_dw V>, and R_dw R_w = id."""
    from paper_2403_11166_amd.api import _w_shape, _x_shape, stride_map
    ctx = context(layer.log2_n, layer.num_limbs, layer.prime_bits)
    eq = stride_map(layer)
    rng = np.random.default_rng(3)
    X = rng.integers(0, 1 << 20, layer.x_shape())
    W = rng.integers(0, 1 << 20, layer.w_shape())
    Z = rng.integers(0, 1 << 20, _x_shape(eq))
    V = rng.integers(0, 1 << 20, _w_shape(eq))
    ip = lambda a, b: int(np.sum(a.astype(object) * b.astype(object)))  # noqa: E731
    assert ip(host_i64(ctx.stride_relayout(layer, "x", dev(X))), Z) == ip(X, host_i64(ctx.stride_relayout(layer, "dx", dev(Z))))
    assert ip(host_i64(ctx.stride_relayout(layer, "w", dev(W))), V) == ip(W, host_i64(ctx.stride_relayout(layer, "dw", dev(V))))
    assert np.array_equal(host_i64(ctx.stride_relayout(layer, "dw", ctx.stride_relayout(layer, "w", dev(W)))), W)


def test_strided_layer_rejected_by_product_entry_points():
    layer = STRIDED[1]
    ctx = context(layer.log2_n, layer.num_limbs, layer.prime_bits)
    with pytest.raises(RuntimeError, match="stride"):
        ctx.plan_auto(layer)


DEGENERATE = [fc(1, 1, 1, log2_n=10, num_limbs=2, prime_bits=50),
              fc(1, 1, 300, log2_n=10, num_limbs=2, prime_bits=50),
              fc(300, 1, 1, log2_n=10, num_limbs=2, prime_bits=50),
              fc(2, 1500, 3, log2_n=10, num_limbs=2, prime_bits=50),     # contraction longer than N
              conv(1, 1, 1, 1, k=1, pad=0, log2_n=10, num_limbs=2, prime_bits=50),
              conv(1, 1, 1, 3, k=3, pad=0, log2_n=10, num_limbs=2, prime_bits=50),   # 1 x 1 output
              conv(2, 3, 2, 1, k=3, pad=1, log2_n=10, num_limbs=2, prime_bits=50),   # 1 x 1 input, padded
              conv(1, 2, 2, 40, k=3, pad=1, log2_n=10, num_limbs=2, prime_bits=50),  # image larger than N
              conv1d(1, 1, 1, 5, k=5, log2_n=10, num_limbs=2, prime_bits=50),
              conv(1, 2, 3, 5, k=5, pad=0, stride=2, log2_n=10, num_limbs=2, prime_bits=50)]


@pytest.mark.parametrize("layer", DEGENERATE, ids=["fc1x1x1", "fc_co300", "fc_b300", "fc_ci1500", "conv1x1",
                                                   "conv_out1", "conv_in1", "conv_40x40", "conv1d_out1",
                                                   "conv_s2_out1"])
def test_degenerate_shapes_reconstruct(layer):
    from paper_2403_11166_amd.api import stride_map
    ctx = context(layer.log2_n, layer.num_limbs, layer.prime_bits)
    ts = layer_tensors(layer, 14)
    d = {k: dev(v) for k, v in ts.items()}
    if layer.stride > 1:
        eq = stride_map(layer)
        rx = lambda v: ctx.stride_relayout(layer, "x", v)  # noqa: E731
        Y, (a, b), dWe = run_protocol(ctx, eq, ts, rx(d["x0"]), rx(d["x1"]), d["dy0"], d["dy1"],
                                      ctx.stride_relayout(layer, "w", d["W"]), 900)
        dx0, dx1 = ctx.stride_relayout(layer, "dx", a), ctx.stride_relayout(layer, "dx", b)
        dW = ctx.stride_relayout(layer, "dw", dWe)
    else:
        Y, (dx0, dx1), dW = run_protocol(ctx, layer, ts, d["x0"], d["x1"], d["dy0"], d["dy1"], d["W"], 900)
    assert np.array_equal(host_i64(Y), LN.layer_op(layer, "fwd", ts["X"], ts["W"], T))
    assert np.array_equal((host_i64(dx0) + host_i64(dx1)) % T, LN.layer_op(layer, "dx", ts["dY"], ts["W"], T))
    assert np.array_equal(host_i64(dW), LN.layer_op(layer, "dw", ts["X"], ts["dY"], T))
