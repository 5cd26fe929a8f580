"""Pencil+ (Alg. 3, Alg. 4) in the oracle: the online phase reconstructs the
plain operator result from preprocessed mask products, for every operator of a
linear layer, and the four operators recombine into the layer's gradients."""
import numpy as np
import pytest

from oracle import linear as LIN
from oracle import pencil_plus as PP
from workloads import T_PLAIN, conv, fc

T = T_PLAIN
LAYERS = [fc(3, 7, 5), conv(2, 3, 2, 5, k=3, pad=1), conv(2, 2, 3, 4, k=2, pad=0)]


def rnd(rng, shape):
    return rng.integers(0, T, size=shape, dtype=np.int64)


def instance(layer, kind, m, seed):
    rng = np.random.default_rng(seed)
    su, sv, _ = PP.operand_shapes(layer, kind)
    u, v = rnd(rng, su), rnd(rng, sv)
    um = [rnd(rng, su) for _ in range(m)]
    vm = [rnd(rng, sv) for _ in range(m)]
    so = PP.operand_shapes(layer, kind)[2]
    s = [[rnd(rng, so) for _ in range(m)] for _ in range(m)]
    k = rng.integers(1, T, size=m)
    l = rng.integers(1, T, size=m)
    return u, v, um, vm, s, k, l


@pytest.mark.parametrize("li", range(len(LAYERS)))
@pytest.mark.parametrize("kind", PP.KINDS)
@pytest.mark.parametrize("m", [1, 3])
def test_online_reconstructs_the_operator(li, kind, m):
    layer = LAYERS[li]
    u, v, um, vm, s, k, l = instance(layer, kind, m, 10 * li + m)
    sh0, sh1 = PP.prep(layer, kind, um, vm, s, T)
    out0, out1, u_t, v_t = PP.online(layer, kind, u, v, um, vm, sh0, sh1, k, l, T)
    want = PP.apply(layer, kind, u, v, T)
    assert np.array_equal((out0 + out1) % T, want)
    # the exchanged messages are the masked operands
    assert np.array_equal(PP.combine(um, k, T, base=u_t), u)
    assert np.array_equal(PP.combine(vm, l, T, base=v_t), v)


def test_preprocessing_shares_reconstruct_mask_products():
    layer = LAYERS[1]
    u, v, um, vm, s, k, l = instance(layer, "fwd", 2, 5)
    sh0, sh1 = PP.prep(layer, "fwd", um, vm, s, T)
    for i in range(2):
        for j in range(2):
            assert np.array_equal((sh0[i][j] + sh1[i][j]) % T, LIN.layer_op(layer, "fwd", vm[j], um[i], T))


def test_every_preprocessed_share_enters_the_result():
    """Changing any one preprocessed share (a dropped or misindexed term) breaks
    the reconstruction."""
    layer = LAYERS[0]
    m = 2
    u, v, um, vm, s, k, l = instance(layer, "fwd", m, 7)
    want = PP.apply(layer, "fwd", u, v, T)
    for side in (0, 1):
        for i in range(m):
            for j in range(m):
                sh0, sh1 = PP.prep(layer, "fwd", um, vm, s, T)
                sh = sh0 if side == 0 else sh1
                sh[i][j] = (sh[i][j] + 1) % T
                out0, out1, _, _ = PP.online(layer, "fwd", u, v, um, vm, sh0, sh1, k, l, T)
                assert not np.array_equal((out0 + out1) % T, want), (side, i, j)


@pytest.mark.parametrize("li", range(len(LAYERS)))
def test_four_operators_give_the_layer_gradients(li):
    """Alg. 4: the forward product plus the MO's local term is Y; the weight
    gradient is the two cross terms plus both local terms (bilinearity of the
    correlation in (X, dY) split into shares)."""
    layer = LAYERS[li]
    rng = np.random.default_rng(40 + li)
    X0, X1 = rnd(rng, layer.x_shape()), rnd(rng, layer.x_shape())
    dY0, dY1 = rnd(rng, layer.y_shape()), rnd(rng, layer.y_shape())
    W = rnd(rng, layer.w_shape())
    X, dY = (X0 + X1) % T, (dY0 + dY1) % T
    y = (PP.apply(layer, "fwd", W, X1, T) + LIN.layer_op(layer, "fwd", X0, W, T)) % T
    assert np.array_equal(y, LIN.layer_op(layer, "fwd", X, W, T))
    dx = (PP.apply(layer, "dx", W, dY1, T) + LIN.layer_op(layer, "dx", dY0, W, T)) % T
    assert np.array_equal(dx, LIN.layer_op(layer, "dx", dY, W, T))
    dw = (PP.apply(layer, "dw01", dY0, X1, T) + PP.apply(layer, "dw10", X0, dY1, T)
          + LIN.layer_op(layer, "dw", X0, dY0, T) + LIN.layer_op(layer, "dw", X1, dY1, T)) % T
    assert np.array_equal(dw, LIN.layer_op(layer, "dw", X, dY, T))


def test_combine_matches_loop():
    rng = np.random.default_rng(3)
    xs = [rnd(rng, (4, 5)) for _ in range(3)]
    c = [int(v) for v in rng.integers(0, T, size=3)]
    base = rnd(rng, (4, 5))
    got = PP.combine(xs, c, T, base=base)
    for idx in np.ndindex(4, 5):
        want = (int(base[idx]) + sum(ci * int(x[idx]) for ci, x in zip(c, xs))) % T
        assert got[idx] == want
