"""Pencil+ on the GPU (preprocessed products, Alg. 3 and Alg. 4) against the
oracle: the Z_t combinations, the online phase on oracle-defined
preprocessing shares (bit for bit), and the homomorphic preprocessing (its
shares reconstruct the mask products)."""
import numpy as np
import pytest

from oracle import pencil_plus as PP
from workloads import CONFIGS, T_PLAIN, conv, conv1d, fc

from gpu_common import dev, host_i64

pytestmark = pytest.mark.gpu

T = T_PLAIN
SMALL = [fc(3, 7, 5, log2_n=12, num_limbs=2, prime_bits=50),
         conv(2, 3, 2, 5, k=3, pad=1, log2_n=12, num_limbs=2, prime_bits=50)]
_ctx = {}


def context(layer, seed=21):
    from paper_2403_11166_amd import Context
    key = (layer.log2_n, layer.num_limbs, layer.prime_bits, seed)
    if key not in _ctx:
        _ctx[key] = Context(layer.log2_n, layer.num_limbs, layer.prime_bits, seed)
    return _ctx[key]


def rnd(rng, shape):
    return rng.integers(0, T, size=shape, dtype=np.int64)


def instance(layer, kind, m, seed):
    rng = np.random.default_rng(seed)
    su, sv, so = PP.operand_shapes(layer, kind)
    u, v = rnd(rng, su), rnd(rng, sv)
    um = [rnd(rng, su) for _ in range(m)]
    vm = [rnd(rng, sv) for _ in range(m)]
    s = [[rnd(rng, so) for _ in range(m)] for _ in range(m)]
    k = rng.integers(1, T, size=m)
    l = rng.integers(1, T, size=m)
    return u, v, um, vm, s, k, l


@pytest.mark.parametrize("n_terms", [0, 1, 3, 9, 16, 21, 64, 65, 130])
def test_zt_combine_matches_oracle(n_terms):
    ctx = context(SMALL[0])
    rng = np.random.default_rng(n_terms)
    xs = [rnd(rng, (37, 11)) for _ in range(n_terms)]
    base = rnd(rng, (37, 11))
    c = [int(v) - T // 2 for v in rng.integers(0, T, size=n_terms)]   # negative coefficients too
    got = ctx.zt_combine([dev(x) for x in xs], c, base=dev(base))
    want = PP.combine(xs, [ci % T for ci in c], T, base=base)
    assert np.array_equal(host_i64(got), want)
    if n_terms:
        # out aliasing base
        b = dev(base)
        ctx.zt_combine([dev(x) for x in xs], c, base=b, out=b)
        assert np.array_equal(host_i64(b), want)
        # no base
        got = ctx.zt_combine([dev(x) for x in xs], c)
        assert np.array_equal(host_i64(got), PP.combine(xs, [ci % T for ci in c], T))


@pytest.mark.parametrize("li", range(len(SMALL)))
@pytest.mark.parametrize("kind", PP.KINDS)
def test_online_phase_bit_exact(li, kind):
    from paper_2403_11166_amd import pencil_plus as GP
    layer = SMALL[li]
    ctx = context(layer)
    m = 3
    u, v, um, vm, s, k, l = instance(layer, kind, m, 100 + li)
    sh0, sh1 = PP.prep(layer, kind, um, vm, s, T)
    want = PP.online(layer, kind, u, v, um, vm, sh0, sh1, k, l, T)
    got = GP.online(ctx, layer, kind, dev(u), dev(v), [dev(x) for x in um], [dev(x) for x in vm],
                    [[dev(x) for x in row] for row in sh0], [[dev(x) for x in row] for row in sh1], k, l)
    for g, w in zip(got, want):
        assert np.array_equal(host_i64(g), w)


def test_online_phase_bit_exact_fc784x128():
    """The default workload's layer (FC 784 -> 128, batch 64), weight-gradient
    cross term (the largest output), m = 2."""
    from paper_2403_11166_amd import pencil_plus as GP
    layer = CONFIGS[2].layers[0]
    ctx = context(layer)
    m = 2
    u, v, um, vm, s, k, l = instance(layer, "dw01", m, 7)
    sh0, sh1 = PP.prep(layer, "dw01", um, vm, s, T)
    want = PP.online(layer, "dw01", u, v, um, vm, sh0, sh1, k, l, T)
    got = GP.online(ctx, layer, "dw01", dev(u), dev(v), [dev(x) for x in um], [dev(x) for x in vm],
                    [[dev(x) for x in row] for row in sh0], [[dev(x) for x in row] for row in sh1], k, l)
    for g, w in zip(got, want):
        assert np.array_equal(host_i64(g), w)


@pytest.mark.parametrize("kind", PP.KINDS)
def test_preprocessing_and_online_end_to_end(kind):
    """Homomorphic preprocessing on the GPU: every pair's shares reconstruct
    u'_i o v'_j; the online phase on those shares reconstructs u o v."""
    from paper_2403_11166_amd import pencil_plus as GP
    layer = SMALL[1]
    ctx = context(layer)
    plan = ctx.plan_auto(layer)
    m = 2
    u, v, um, vm, _, k, l = instance(layer, kind, m, 300)
    sh0, sh1 = GP.prep(ctx, layer, plan, kind, [dev(x) for x in um], [dev(x) for x in vm], 5000)
    for i in range(m):
        for j in range(m):
            rec = (host_i64(sh0[i][j]) + host_i64(sh1[i][j])) % T
            assert np.array_equal(rec, PP.apply(layer, kind, um[i], vm[j], T)), (i, j)
    out0, out1, _, _ = GP.online(ctx, layer, kind, dev(u), dev(v), [dev(x) for x in um], [dev(x) for x in vm],
                                 sh0, sh1, k, l)
    assert np.array_equal((host_i64(out0) + host_i64(out1)) % T, PP.apply(layer, kind, u, v, T))


def test_zt_linear_with_a_47_bit_t_and_long_contraction():
    """A plaintext modulus near 2^47 leaves the tiled correlation fewer terms per
    wave before its partial sums could overflow; long contractions must still
    be exact (checked in Python integers)."""
    from oracle import linear as LN
    from paper_2403_11166_amd import Context
    t47 = 140737488355213
    ctx = Context(12, 2, 50, 5, t=t47)
    assert ctx.t == t47
    rng = np.random.default_rng(47)
    for layer in (fc(2, 20000, 3, log2_n=12, num_limbs=2, prime_bits=50),
                  fc(3, 70, 5, log2_n=12, num_limbs=2, prime_bits=50)):
        x = rng.integers(0, t47, layer.x_shape(), dtype=np.int64)
        w = rng.integers(0, t47, layer.w_shape(), dtype=np.int64)
        dy = rng.integers(0, t47, layer.y_shape(), dtype=np.int64)
        got = host_i64(ctx.zt_linear(layer, "fwd", dev(x), dev(w)))
        assert np.array_equal(got, LN.tensordot_mod_t_object(x, w, ([1], [1]), t47))
        got = host_i64(ctx.zt_linear(layer, "dx", dev(dy), dev(w)))
        assert np.array_equal(got, LN.tensordot_mod_t_object(dy, w, ([1], [0]), t47))


def test_zt_linear_matrix_core_path_with_a_47_bit_t():
    """Weight-gradient-shaped correlations with many 16 x 16 output tiles run on
    the fp64 matrix-core kernel; with a 47-bit t its top digits are large."""
    from oracle import linear as LN
    from paper_2403_11166_amd import Context
    t47 = 140737488355213
    ctx = Context(12, 2, 50, 6, t=t47)
    rng = np.random.default_rng(48)
    for layer, op in ((fc(64, 600, 500, log2_n=12, num_limbs=2, prime_bits=50), "dw"),
                      (conv(2, 64, 128, 6, k=3, pad=1, log2_n=12, num_limbs=2, prime_bits=50), "dw"),
                      (conv(8, 8, 128, 12, k=3, pad=1, log2_n=12, num_limbs=2, prime_bits=50), "fwd")):
        x = rng.integers(0, t47, layer.x_shape(), dtype=np.int64)
        w = rng.integers(0, t47, layer.w_shape(), dtype=np.int64)
        dy = rng.integers(0, t47, layer.y_shape(), dtype=np.int64)
        a, b = (x, dy) if op == "dw" else (x, w)
        got = host_i64(ctx.zt_linear(layer, op, dev(a), dev(b)))
        want = LN.layer_op(layer, op, a, b, t47, tdot=LN.tensordot_mod_t_object)
        assert np.array_equal(got, want), (layer, op)


@pytest.mark.parametrize("t_plain", [T, 140737488355213])
def test_zt_linear_lane_split_contraction(t_plain):
    """Correlations with a long contraction and few outputs run with the lanes
    of a wave (or of four waves) splitting the contraction, a 2 x 2 output block
    per wave: odd row and column counts, operands strided along the
    contraction (input and weight gradients), convolution windows with padding
    and a flipped kernel, and with a 47-bit t the longest contraction one
    partial sum may hold, on all-maximal operands (checked in Python
    integers)."""
    from oracle import linear as LN
    from paper_2403_11166_amd import Context
    ctx = Context(12, 2, 50, 7, t=t_plain)
    assert ctx.t == t_plain
    rng = np.random.default_rng(t_plain % 1000)
    kw = dict(log2_n=12, num_limbs=2, prime_bits=50)
    cases = [(fc(5, 300, 3, **kw), "fwd", False), (fc(3, 7, 257, **kw), "dx", False),
             (fc(301, 5, 3, **kw), "dw", False), (fc(2, 4096, 3, **kw), "fwd", True),
             (fc(2, 4097, 3, **kw), "fwd", True), (fc(8, 1000, 16, **kw), "fwd", False),
             # convolutions: padded windows, a flipped kernel, a one-row Conv1d, and a
             # weight gradient long enough for four waves per output block
             (conv(2, 64, 3, 4, k=3, pad=1, **kw), "fwd", False), (conv(2, 3, 64, 4, k=3, pad=1, **kw), "dx", False),
             (conv1d(8, 4, 3, 300, k=5, pad=2, **kw), "dw", False), (conv(64, 3, 8, 16, k=3, pad=1, **kw), "dw", False),
             # many output tiles but three columns: the input gradient of a three-channel layer
             (conv(16, 3, 32, 16, k=3, pad=1, **kw), "dx", False)]
    for layer, op, top in cases:
        def draw(shape):
            if top:
                return np.full(shape, t_plain - 1, dtype=np.int64)
            return rng.integers(0, t_plain, shape, dtype=np.int64)
        x, w, dy = draw(layer.x_shape()), draw(layer.w_shape()), draw(layer.y_shape())
        a, b = {"fwd": (x, w), "dx": (dy, w), "dw": (x, dy)}[op]
        got = host_i64(ctx.zt_linear(layer, op, dev(a), dev(b)))
        want = LN.layer_op(layer, op, a, b, t_plain, tdot=LN.tensordot_mod_t_object)
        assert np.array_equal(got, want), (layer, op)


@pytest.mark.parametrize("batch", [32768, 32769])
def test_zt_linear_matrix_core_at_its_digit_bound(batch):
    """With t < 2^42 the matrix-core correlation splits operands into two 21-bit
    digits while one wave sums at most 2^11 contraction indices (2^9 steps of
    four); a weight gradient over a batch of 32768 with 16 waves per tile sits
    exactly at that bound, and one index more takes the three-digit form.
    Operands of the largest centred magnitude, (t - 1) / 2, make every digit
    product and diagonal sum as large as it can be; the exact result of each
    entry is batch ((t - 1) / 2)^2 mod t."""
    from paper_2403_11166_amd import Context
    ctx = Context(12, 2, 50, 9)
    layer = fc(batch, 128, 128, log2_n=12, num_limbs=2, prime_bits=50)  # 64 output tiles of 16 x 16
    h = (T - 1) // 2
    x = dev(np.full(layer.x_shape(), h, dtype=np.int64))
    dy = dev(np.full(layer.y_shape(), h, dtype=np.int64))
    got = host_i64(ctx.zt_linear(layer, "dw", x, dy))
    assert got.size == 128 * 128
    assert (got == (batch * h * h) % T).all()


@pytest.mark.parametrize("case", range(6))
def test_zt_linear_at_the_kernel_selection_boundaries(case):
    """Shapes on either side of each point where the correlation changes
    kernel: 8191 / 8192 contraction indices (one or four waves per lane-split
    block), four / five output columns (lane-split or matrix-core kernel for a
    grid of many tiles), 63 / 64 output tiles (lane-split or matrix-core
    kernel for a long contraction)."""
    from oracle import linear as LN
    from paper_2403_11166_amd import Context
    kw = dict(log2_n=12, num_limbs=2, prime_bits=50)
    layer, op = [(fc(8191, 5, 3, **kw), "dw"), (fc(8192, 5, 3, **kw), "dw"),
                 (conv(16, 4, 32, 16, k=3, pad=1, **kw), "dx"), (conv(16, 5, 32, 16, k=3, pad=1, **kw), "dx"),
                 (fc(112, 300, 144, **kw), "fwd"), (fc(128, 300, 128, **kw), "fwd")][case]
    ctx = context(SMALL[0])
    rng = np.random.default_rng(60 + case)
    x, w, dy = (rng.integers(0, T, s, dtype=np.int64) for s in (layer.x_shape(), layer.w_shape(), layer.y_shape()))
    a, b = {"fwd": (x, w), "dx": (dy, w), "dw": (x, dy)}[op]
    got = host_i64(ctx.zt_linear(layer, op, dev(a), dev(b)))
    assert np.array_equal(got, LN.layer_op(layer, op, a, b, T)), (layer, op)
