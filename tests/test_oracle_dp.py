"""Pins for the bias gradient and the data owner's DP perturbation (Sec. III.B.2)."""
import math

import mpmath
import numpy as np
import pytest
from scipy import stats

from oracle import dp as DP
from oracle import linear as LN
from oracle import params as PR
from oracle.philox import stream_words
from workloads import conv, fc, layer_tensors

T = PR.T


# ------------------------------------------------------------- bias gradient

@pytest.mark.parametrize("layer", [fc(7, 5, 3), conv(3, 2, 4, 6, k=3, pad=1), conv(2, 3, 5, 7, k=5, pad=0)])
def test_bias_grad_is_weight_gradient_of_a_constant_input(layer):
    """db is dW of the same layer shape with one all-ones input channel and a
    1x1 kernel (the footnote's sums over batch and output positions), computed
    by the plain layer operators."""
    dy = layer_tensors(layer, 3)["dY"]
    if layer.kind == "fc":
        ones_layer = fc(layer.batch, 1, layer.c_out)
        x = np.ones((layer.batch, 1), dtype=np.int64)
        ref = LN.layer_op(ones_layer, "dw", x, dy, T)[:, 0]
    else:
        ones_layer = conv(layer.batch, 1, layer.c_out, layer.h_out, k=1, pad=0)
        x = np.ones((layer.batch, 1, layer.h_out, layer.w_out), dtype=np.int64)
        ref = LN.layer_op(ones_layer, "dw", x, dy, T)[:, 0, 0, 0]
    assert (DP.bias_grad(layer, dy, T) == ref).all()


def test_bias_grad_is_adjoint_of_bias_broadcast():
    """<db, beta> = <dY, broadcast(beta)> mod t for any beta."""
    layer = conv(4, 3, 6, 5, k=3, pad=1)
    dy = layer_tensors(layer, 5)["dY"]
    beta = np.random.default_rng(9).integers(0, T, layer.c_out)
    lhs = sum(int(a) * int(b) for a, b in zip(DP.bias_grad(layer, dy, T), beta)) % T
    bb = np.broadcast_to(beta[None, :, None, None], dy.shape)
    rhs = sum(int(a) * int(b) for a, b in zip(dy.ravel(), bb.ravel())) % T
    assert lhs == rhs


def test_bias_grad_shares_reconstruct():
    layer = fc(9, 4, 6)
    ts = layer_tensors(layer, 2)
    s = (DP.bias_grad(layer, ts["dy0"], T) + DP.bias_grad(layer, ts["dy1"], T)) % T
    assert (s == DP.bias_grad(layer, ts["dY"], T)).all()


# ------------------------------------------------------------- ln and trig

def _log_inputs():
    rng = np.random.default_rng(1)
    edge = [1, 2, 3, 5, (1 << 52) - 1, 1 << 52, (1 << 52) + 1, (1 << 53) - 1, 1 << 53,
            int(round(2 ** 53 / math.sqrt(2))), int(round(2 ** 53 / math.sqrt(2))) + 1]
    k = rng.integers(1, 1 << 53, 20000, dtype=np.uint64) >> rng.integers(0, 53, 20000).astype(np.uint64)
    return np.concatenate([np.array(edge, dtype=np.uint64), np.maximum(k, np.uint64(1))])


def test_log_matches_libm_to_two_ulp():
    k = _log_inputs()
    got = DP.log_u(k)
    ref = np.array([math.log(int(v) * 2.0 ** -53) for v in k])
    ulp = np.spacing(np.maximum(np.abs(ref), 1e-300))
    err = np.abs(got - ref)
    assert (err <= 2 * ulp + 1e-300).all(), float((err / ulp).max())
    assert DP.log_u(np.array([1 << 53], dtype=np.uint64))[0] == 0.0
    assert DP.log_u(np.array([1 << 52], dtype=np.uint64))[0] == -DP.LN2


def test_trig_matches_libm():
    rng = np.random.default_rng(2)
    edge = [0, 1, 1 << 50, (1 << 50) - 1, (1 << 50) + 1, 1 << 51, 3 << 50, 1 << 52, 5 << 50, 3 << 51,
            7 << 50, (1 << 53) - 1]
    b = np.concatenate([np.array(edge, dtype=np.uint64), rng.integers(0, 1 << 53, 3000, dtype=np.uint64)])
    c, s = DP.cos_sin_turns(b)
    mpmath.mp.prec = 120
    x = [2 * mpmath.pi * mpmath.mpf(int(v)) / mpmath.mpf(2) ** 53 for v in b]
    rc = np.array([float(mpmath.cos(v)) for v in x])
    rs = np.array([float(mpmath.sin(v)) for v in x])
    assert np.abs(c - rc).max() < 3e-16
    assert np.abs(s - rs).max() < 3e-16
    # every quadrant is reached and exact at the axis points
    c4, s4 = DP.cos_sin_turns(np.array([0, 1 << 51, 1 << 52, 3 << 51], dtype=np.uint64))
    assert list(c4) == [1.0, 0.0, -1.0, 0.0] and list(s4) == [0.0, 1.0, 0.0, -1.0]


# --------------------------------------------------------------- Box-Muller

def test_pairs_are_box_muller_of_their_stream_words():
    """z_{2i}^2 + z_{2i+1}^2 = -2 ln u1 and atan2(z_{2i+1}, z_{2i}) = 2 pi u2,
    recomputed from the raw Philox words with libm."""
    seed, nonce, obj, n = 11, 77, 3, 4000
    z = DP.gaussian(seed, nonce, obj, n)
    w = stream_words(seed, nonce, obj, DP.P_DP, 0, 0, n)
    u1 = ((w[0::2] >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = (w[1::2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r2 = z[0::2] ** 2 + z[1::2] ** 2
    np.testing.assert_allclose(r2, -2.0 * np.log(u1), rtol=1e-13, atol=1e-13)
    ang = np.mod(np.arctan2(z[1::2], z[0::2]), 2 * math.pi)
    d = np.abs(ang - 2 * math.pi * u2)
    d = np.minimum(d, 2 * math.pi - d)
    big = r2 > 1e-6
    assert d[big].max() < 1e-9


def test_gaussian_distribution():
    z = DP.gaussian(5, 123, 0, 1 << 18)
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 0.06
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 0.02
    assert np.abs(z).max() <= math.sqrt(2 * 53 * math.log(2)) + 1e-9


def test_streams_differ_by_object_and_nonce():
    a = DP.gaussian(1, 2, 0, 64)
    assert not np.array_equal(a, DP.gaussian(1, 2, 1, 64))
    assert not np.array_equal(a, DP.gaussian(1, 3, 0, 64))
    assert np.array_equal(a[:17], DP.gaussian(1, 2, 0, 17))     # prefix-stable


def test_noise_floor_and_wrap():
    e = DP.noise(4, 8, 0, 1001, 2.0 ** 20)
    z = DP.gaussian(4, 8, 0, 1001)
    assert (e == np.floor(z * 2.0 ** 20)).all()
    assert (e < 0).any() and (e > 0).any()
    assert (DP.noise(4, 8, 0, 50, 0.0) == 0).all()
    x = np.zeros(1001, dtype=np.int64)
    y = DP.add_noise(x, 4, 8, 0, 2.0 ** 20, T)
    assert ((y - e) % T == 0).all() and (y >= 0).all() and (y < T).all()
    # the empirical sd of the fixed-point noise is std
    big = DP.noise(6, 1, 0, 1 << 16, 1000.0)
    assert abs(big.std() / 1000.0 - 1.0) < 0.02


# ------------------------------------------------------- Alg. 2's weight update

def test_weight_update_reconstructs_gradient_plus_noise():
    layer = conv(2, 3, 4, 5, k=3, pad=1)
    ts = layer_tensors(layer, 8)
    rng = np.random.default_rng(4)
    cross = (LN.layer_op(layer, "dw", ts["x1"], ts["dy0"], T) + LN.layer_op(layer, "dw", ts["x0"], ts["dy1"], T)) % T
    s = rng.integers(0, T, cross.shape)
    dw_dec = (cross - s) % T          # what the DO decrypts: cross - s
    std_w, std_b = 2.0 ** 18, 2.0 ** 9
    dW, db, _, _ = DP.weight_update(layer, s, dw_dec, ts["x0"], ts["x1"], ts["dy0"], ts["dy1"], 21, 5, std_w, std_b, T)
    ew = DP.noise(21, 5, DP.OBJ_DW, cross.size, std_w).reshape(cross.shape)
    eb = DP.noise(21, 5, DP.OBJ_DB, layer.c_out, std_b)
    assert ((dW - LN.layer_op(layer, "dw", ts["X"], ts["dY"], T) - ew) % T == 0).all()
    assert ((db - DP.bias_grad(layer, ts["dY"], T) - eb) % T == 0).all()
    # without noise the MO recovers the exact gradients
    dW0, db0, _, _ = DP.weight_update(layer, s, dw_dec, ts["x0"], ts["x1"], ts["dy0"], ts["dy1"], 21, 5, 0.0, 0.0, T)
    assert (dW0 == LN.layer_op(layer, "dw", ts["X"], ts["dY"], T)).all()
    assert (db0 == DP.bias_grad(layer, ts["dY"], T)).all()
