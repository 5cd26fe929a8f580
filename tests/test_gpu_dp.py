"""The bias gradient and the data owner's DP perturbation on the GPU against
the oracle, bit for bit, and the end of Alg. 2 (weight update with noise) run
through the whole HIP path."""
import numpy as np
import pytest

from oracle import dp as DP
from oracle import linear as LN
from workloads import CONFIGS, T_PLAIN, conv, fc, layer_tensors

from gpu_common import dev, host_i64

pytestmark = pytest.mark.gpu

T = T_PLAIN
_ctx = {}


def context(log2_n=12, limbs=2, bits=50, seed=21):
    from paper_2403_11166_amd import Context
    key = (log2_n, limbs, bits, seed)
    if key not in _ctx:
        _ctx[key] = Context(log2_n, limbs, bits, seed)
    return _ctx[key]


@pytest.mark.parametrize("count", [0, 1, 2, 3, 5, 4097, 10007])
@pytest.mark.parametrize("sd", [0.0, 1.0, 1000.5, 2.0 ** 24 * 0.37, 2.0 ** 40])
def test_dp_noise_matches_oracle(count, sd):
    ctx = context()
    x = np.random.default_rng(count).integers(0, T, count, dtype=np.int64)
    d = dev(x)
    ctx.dp_noise_(d, sd, 99, 7)
    want = DP.add_noise(x, ctx.seed, 99, 7, sd, T)
    assert np.array_equal(host_i64(d), want)


def test_dp_noise_full_weight_shapes():
    """Every weight-gradient tensor of the benchmark workloads, in one stream each."""
    ctx = context(13, 3, 60, seed=5)
    sizes = sorted({int(np.prod(l.w_shape())) for c in CONFIGS.values() for l in c.layers})
    rng = np.random.default_rng(3)
    for i, n in enumerate(sizes):
        x = rng.integers(0, T, n, dtype=np.int64)
        sd = 2.0 ** 24 * (0.1 + 0.2 * i)
        d = dev(x)
        ctx.dp_noise_(d, sd, 1000 + i, DP.OBJ_DW)
        assert np.array_equal(host_i64(d), DP.add_noise(x, 5, 1000 + i, DP.OBJ_DW, sd, T)), n


def test_dp_noise_rejects_bad_sd():
    ctx = context()
    d = dev(np.zeros(8, dtype=np.int64))
    for sd in (-1.0, float("nan"), float("inf"), 2.0 ** 53):
        with pytest.raises(RuntimeError):
            ctx.dp_noise_(d, sd, 1, 0)


BIAS_LAYERS = [fc(1, 3, 1), fc(7, 5, 3), fc(64, 784, 128), fc(128, 2048, 10), fc(5, 9, 300),
               conv(3, 2, 4, 6, k=3, pad=1), conv(2, 3, 5, 7, k=5, pad=0), conv(64, 3, 64, 32),
               conv(64, 256, 256, 8), conv(1, 1, 1, 3, k=3, pad=0)]


@pytest.mark.parametrize("layer", BIAS_LAYERS, ids=lambda l: f"{l.kind}{l.batch}x{l.c_out}x{l.h_out}")
def test_bias_grad_matches_oracle(layer):
    ctx = context()
    dy = np.random.default_rng(layer.batch * 7 + layer.c_out).integers(0, T, layer.y_shape(), dtype=np.int64)
    got = host_i64(ctx.bias_grad(layer, dev(dy)))
    assert np.array_equal(got, DP.bias_grad(layer, dy, T))


def test_bias_grad_limit():
    """With t < 2^41, 2^23 entries of t - 1 still sum exactly in 64 bits."""
    ctx = context()
    ok = conv(8, 1, 1, 1024, k=1, pad=0)        # 8 * 1024^2 = 2^23 entries per channel
    dy = np.full(ok.y_shape(), T - 1, dtype=np.int64)
    got = host_i64(ctx.bias_grad(ok, dev(dy)))
    assert np.array_equal(got, DP.bias_grad(ok, dy, T))
    big = conv(9, 1, 1, 1024, k=1, pad=0)
    with pytest.raises(RuntimeError):
        ctx.bias_grad(big, dev(np.zeros(big.y_shape(), dtype=np.int64)))


@pytest.mark.parametrize("layer", [fc(6, 10, 7, log2_n=12, num_limbs=2, prime_bits=50),
                                   conv(2, 3, 4, 6, k=3, pad=1, log2_n=12, num_limbs=2, prime_bits=50)],
                         ids=["fc", "conv"])
def test_weight_update_end_to_end(layer):
    """Alg. 2 with the bias gradient and DP noise, every step on the GPU: the DO
    decrypts the cross terms, adds its local term and noise; the MO adds the
    mask and its local term.  The MO ends with dW + e_W and db + e_b."""
    ctx = context(layer.log2_n, layer.num_limbs, layer.prime_bits, seed=31)
    ts = layer_tensors(layer, 17)
    plan = ctx.plan_auto(layer)
    nonce = 4242
    ct_x_dw = ctx.encrypt(layer, plan, "x_dw", dev(ts["x1"]), nonce)
    ct_dy_dw = ctx.encrypt(layer, plan, "dy_dw", dev(ts["dy1"]), nonce)
    ct_dy_dx = ctx.encrypt(layer, plan, "dy_dx", dev(ts["dy1"]), nonce)
    _, _, ct_dw, dw_mask = ctx.linear_bwd(layer, plan, ct_dy_dx, ct_x_dw, ct_dy_dw, dev(ts["dy0"]), dev(ts["x0"]),
                                          dev(ts["W"]), nonce + 1)
    std_w, std_b = 2.0 ** 24 * 0.05, 2.0 ** 12 * 0.05
    # DO
    dw_t = ctx.decrypt(layer, plan, "dw", ct_dw)
    local1 = ctx.zt_linear(layer, "dw", dev(ts["x1"]), dev(ts["dy1"]))
    dw_t = ctx.zt_combine([local1], [1], base=dw_t, out=dw_t)
    ctx.dp_noise_(dw_t, std_w, nonce, DP.OBJ_DW)
    db_t = ctx.dp_noise_(ctx.bias_grad(layer, dev(ts["dy1"])), std_b, nonce, DP.OBJ_DB)
    # MO
    local0 = ctx.zt_linear(layer, "dw", dev(ts["x0"]), dev(ts["dy0"]))
    dW = host_i64(ctx.zt_combine([dw_mask, local0], [1, 1], base=dw_t))
    db = host_i64(ctx.zt_combine([ctx.bias_grad(layer, dev(ts["dy0"]))], [1], base=db_t))
    ew = DP.noise(31, nonce, DP.OBJ_DW, int(np.prod(layer.w_shape())), std_w).reshape(layer.w_shape())
    eb = DP.noise(31, nonce, DP.OBJ_DB, layer.c_out, std_b)
    want_w = np.mod(LN.layer_op(layer, "dw", ts["X"], ts["dY"], T).astype(object) + ew, T).astype(np.int64)
    want_b = np.mod(DP.bias_grad(layer, ts["dY"], T).astype(object) + eb, T).astype(np.int64)
    assert np.array_equal(dW, want_w)
    assert np.array_equal(db, want_b)
