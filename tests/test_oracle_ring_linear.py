"""Pins for the oracle's ring products, transforms and plaintext layers."""
import numpy as np
import pytest
import torch

from oracle import linear as LN
from oracle import params as PR
from oracle import ring as RG
from workloads import conv, conv1d, fc

Q60 = PR.ntt_primes(60, 1)[0]


def _fold_negacyclic(full, n, q):
    """Reduce a polynomial product of degree < 2n modulo X^n + 1."""
    out = [0] * n
    for k, v in enumerate(full):
        if k < n:
            out[k] += int(v)
        else:
            out[k - n] -= int(v)
    return [x % q for x in out]


@pytest.mark.parametrize("n", [1, 2, 8, 32])
def test_negacyclic_matches_polynomial_product(n):
    rng = np.random.default_rng(n)
    a = rng.integers(0, Q60, n, dtype=np.uint64)
    b = rng.integers(0, Q60, n, dtype=np.uint64)
    full = np.convolve(a.astype(object), b.astype(object))  # product over Z
    ref = _fold_negacyclic(full, n, Q60)
    assert [int(x) for x in RG.negacyclic_mul(a, b, Q60)] == ref
    assert RG.negacyclic_mul_py(a, b, Q60) == ref
    idx = np.array([0, n - 1, n // 2])
    assert [int(x) for x in RG.negacyclic_coeffs(a, b, Q60, idx)] == [ref[i] for i in idx]


def test_negacyclic_wrap_sign():
    # X^(n-1) * X = X^n = -1
    n = 16
    a = np.zeros(n, dtype=np.uint64)
    b = np.zeros(n, dtype=np.uint64)
    a[n - 1] = 1
    b[1] = 5
    out = RG.negacyclic_mul(a, b, Q60)
    assert int(out[0]) == Q60 - 5 and int(out[1:].max()) == 0


@pytest.mark.parametrize("n", [8, 64])
def test_ntt_definition_and_convolution_theorem(n):
    q = Q60
    psi = PR.min_primitive_2n_root(q, n)
    rng = np.random.default_rng(n + 1)
    a = rng.integers(0, q, n, dtype=np.uint64)
    b = rng.integers(0, q, n, dtype=np.uint64)
    A = RG.ntt_def(a, q, psi)
    # definition written out with Python integers
    ref = [sum(int(a[j]) * pow(psi, (2 * k + 1) * j, q) for j in range(n)) % q for k in range(n)]
    assert [int(x) for x in A] == ref
    assert [int(x) for x in RG.intt_def(A, q, psi)] == [int(x) for x in a]
    B = RG.ntt_def(b, q, psi)
    C = np.array([int(x) * int(y) % q for x, y in zip(A, B)], dtype=np.uint64)
    assert [int(x) for x in RG.intt_def(C, q, psi)] == [int(x) for x in RG.negacyclic_mul(a, b, q)]


# -------------------------------------------------------------- linear layers

T = PR.T


def _small_ints(rng, shape, lim=50):
    """Z_t tensors holding small signed integers (so float64 torch ops are exact)."""
    v = rng.integers(-lim, lim + 1, shape)
    return np.mod(v, T).astype(np.int64), v


def test_tensordot_digits_match_python_ints():
    rng = np.random.default_rng(0)
    a = rng.integers(0, T, (4, 7, 3))
    b = rng.integers(0, T, (7, 5))
    assert (LN.tensordot_mod_t(a, b, ([1], [0]), T) == LN.tensordot_mod_t_object(a, b, ([1], [0]), T)).all()
    a = rng.integers(0, T, (3, 5, 6, 2))
    b = rng.integers(0, T, (3, 4, 6, 2))
    ax = ([0, 2, 3], [0, 2, 3])
    assert (LN.tensordot_mod_t(a, b, ax, T) == LN.tensordot_mod_t_object(a, b, ax, T)).all()


@pytest.mark.parametrize("layer", [conv(2, 3, 4, 6, k=3, pad=1), conv(3, 2, 5, 7, k=2, pad=0),
                                   conv(1, 4, 2, 5, k=3, pad=2),
                                   conv(2, 1, 5, 12, k=5, pad=2, stride=2), conv(2, 3, 2, 9, k=3, pad=1, stride=2),
                                   conv(1, 2, 3, 11, k=4, pad=1, stride=3), conv(2, 2, 2, 8, k=3, pad=0, stride=2)])
def test_conv_matches_torch_autograd(layer):
    """Forward, input gradient and weight gradient vs torch float64 autograd on small integers."""
    rng = np.random.default_rng(1)
    X, Xs = _small_ints(rng, layer.x_shape())
    W, Ws = _small_ints(rng, layer.w_shape())
    dY, dYs = _small_ints(rng, layer.y_shape())
    xt = torch.tensor(Xs, dtype=torch.float64, requires_grad=True)
    wt = torch.tensor(Ws, dtype=torch.float64, requires_grad=True)
    yt = torch.nn.functional.conv2d(xt, wt, padding=layer.pad, stride=layer.stride)
    yt.backward(torch.tensor(dYs, dtype=torch.float64))
    to_t = lambda v: np.mod(np.rint(v.detach().numpy()).astype(np.int64), T)  # noqa: E731
    if layer.pad <= layer.k - 1:
        assert (LN.layer_op(layer, "dx", dY, W, T) == to_t(xt.grad)).all()
    assert (LN.layer_op(layer, "fwd", X, W, T) == to_t(yt)).all()
    assert (LN.layer_op(layer, "dw", X, dY, T) == to_t(wt.grad)).all()


def test_fc_matches_torch_autograd():
    layer = fc(5, 9, 4)
    rng = np.random.default_rng(2)
    X, Xs = _small_ints(rng, layer.x_shape())
    W, Ws = _small_ints(rng, layer.w_shape())
    dY, dYs = _small_ints(rng, layer.y_shape())
    xt = torch.tensor(Xs, dtype=torch.float64, requires_grad=True)
    wt = torch.tensor(Ws, dtype=torch.float64, requires_grad=True)
    yt = torch.nn.functional.linear(xt, wt)
    yt.backward(torch.tensor(dYs, dtype=torch.float64))
    to_t = lambda v: np.mod(np.rint(v.detach().numpy()).astype(np.int64), T)  # noqa: E731
    assert (LN.layer_op(layer, "fwd", X, W, T) == to_t(yt)).all()
    assert (LN.layer_op(layer, "dx", dY, W, T) == to_t(xt.grad)).all()
    assert (LN.layer_op(layer, "dw", X, dY, T) == to_t(wt.grad)).all()


@pytest.mark.parametrize("layer", [conv(2, 3, 2, 5, k=3, pad=1), fc(3, 6, 4)])
def test_adjoint_identities_mod_t(layer):
    """<dY, f(X)> = <f_x^T(dY), X> and <dY, f_W(X)> = <dW(X, dY), W> over Z_t with full-size values."""
    rng = np.random.default_rng(3)
    X = rng.integers(0, T, layer.x_shape())
    W = rng.integers(0, T, layer.w_shape())
    dY = rng.integers(0, T, layer.y_shape())
    ip = lambda a, b: int(np.sum(a.astype(object) * b.astype(object))) % T  # noqa: E731
    Y = LN.layer_op(layer, "fwd", X, W, T)
    assert ip(dY, Y) == ip(LN.layer_op(layer, "dx", dY, W, T), X) == ip(LN.layer_op(layer, "dw", X, dY, T), W)


def test_finite_difference_exact():
    """Linear map: f(X + d) - f(X) = f(d) exactly mod t, and the gradient pairs with d."""
    layer = conv(2, 2, 3, 5, k=3, pad=1)
    rng = np.random.default_rng(4)
    X = rng.integers(0, T, layer.x_shape())
    W = rng.integers(0, T, layer.w_shape())
    d = np.zeros_like(X)
    d[1, 0, 2, 3] = 1
    diff = np.mod(LN.layer_op(layer, "fwd", np.mod(X + d, T), W, T) - LN.layer_op(layer, "fwd", X, W, T), T)
    assert (diff == LN.layer_op(layer, "fwd", d, W, T)).all()
    dY = rng.integers(0, T, layer.y_shape())
    lhs = int(np.sum(dY.astype(object) * diff.astype(object))) % T
    assert lhs == int(LN.layer_op(layer, "dx", dY, W, T)[1, 0, 2, 3])


@pytest.mark.parametrize("layer", [conv1d(2, 6, 4, 11, k=5), conv1d(3, 4, 5, 9, k=3, pad=1),
                                   conv1d(2, 3, 2, 14, k=5, pad=2, stride=2), conv1d(1, 2, 3, 5, k=5)])
def test_conv1d_matches_torch_autograd(layer):
    """Conv1d (the one-row specialisation of Conv2d) vs torch's conv1d."""
    rng = np.random.default_rng(5)
    X, Xs = _small_ints(rng, layer.x_shape())
    W, Ws = _small_ints(rng, layer.w_shape())
    dY, dYs = _small_ints(rng, layer.y_shape())
    xt = torch.tensor(Xs, dtype=torch.float64, requires_grad=True)
    wt = torch.tensor(Ws, dtype=torch.float64, requires_grad=True)
    yt = torch.nn.functional.conv1d(xt, wt, padding=layer.pad, stride=layer.stride)
    yt.backward(torch.tensor(dYs, dtype=torch.float64))
    to_t = lambda v: np.mod(np.rint(v.detach().numpy()).astype(np.int64), T)  # noqa: E731
    assert (LN.layer_op(layer, "fwd", X, W, T) == to_t(yt)).all()
    assert (LN.layer_op(layer, "dx", dY, W, T) == to_t(xt.grad)).all()
    assert (LN.layer_op(layer, "dw", X, dY, T) == to_t(wt.grad)).all()


@pytest.mark.parametrize("layer", [conv(2, 2, 3, 9, k=5, pad=2, stride=2), conv1d(2, 3, 2, 13, k=5, pad=1, stride=2),
                                   conv1d(2, 3, 4, 8, k=3)])
def test_strided_and_1d_adjoints_and_pointwise(layer):
    """Adjoint identities with full-size values, and the pointwise sums of
    layer_op_at against the whole-tensor operators."""
    rng = np.random.default_rng(6)
    X = rng.integers(0, T, layer.x_shape())
    W = rng.integers(0, T, layer.w_shape())
    dY = rng.integers(0, T, layer.y_shape())
    ip = lambda a, b: int(np.sum(a.astype(object) * b.astype(object))) % T  # noqa: E731
    Y = LN.layer_op(layer, "fwd", X, W, T)
    assert ip(dY, Y) == ip(LN.layer_op(layer, "dx", dY, W, T), X) == ip(LN.layer_op(layer, "dw", X, dY, T), W)
    for op, a, b in (("fwd", X, W), ("dx", dY, W), ("dw", X, dY)):
        full = LN.layer_op(layer, op, a, b, T)
        pts = [tuple(int(v) for v in np.unravel_index(i, full.shape)) for i in range(0, full.size, 7)]
        assert LN.layer_op_at(layer, op, a, b, T, pts) == [int(full[p]) for p in pts]
