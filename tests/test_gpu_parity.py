"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
bit for bit, on seeded inputs."""
import numpy as np
import pytest
import torch

from oracle import bfv
from oracle import encoding as E
from oracle import linear as LN
from oracle import params as PR
from oracle import protocol as PRT
from oracle import ring as RG
from workloads import CONFIGS, config_tensors, layer_tensors, small_cases, conv, conv1d, fc

from gpu_common import dev, host_i64, host_u64, oracle_ct_ntt, oracle_keys, oracle_params, cts_list

pytestmark = pytest.mark.gpu

_ctx = {}


def context(log2_n, limbs, bits, seed):
    from paper_2403_11166_amd import Context
    key = (log2_n, limbs, bits, seed)
    if key not in _ctx:
        _ctx[key] = Context(log2_n, limbs, bits, seed)
    return _ctx[key]


def brv(i, bits):
    return int(format(i, f"0{bits}b")[::-1], 2)


# ----------------------------------------------------------- params and keys

@pytest.mark.parametrize("shape", [(12, 2, 50), (13, 3, 60), (14, 4, 60)])
def test_params_and_keygen_match_oracle(shape):
    log2_n, limbs, bits = shape
    ctx = context(log2_n, limbs, bits, 11)
    P = PR.make_params(log2_n, limbs, bits)
    assert list(ctx.primes) == P.moduli
    assert ctx.t == P.t
    assert list(ctx.psi) == P.psi
    assert ctx.flood_bits == P.flood_bits
    sk, pk = ctx.export_keys()
    ok = oracle_keys(ctx)
    assert (sk == ok["sk"]).all()
    assert (pk == ok["pk"]).all()


# ----------------------------------------------------------------- NTT

def test_ntt_matches_definition_n4096():
    ctx = context(12, 2, 50, 1)
    rng = np.random.default_rng(0)
    a = np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64) for q in ctx.primes])[None]
    t = torch.from_numpy(a.view(np.int64).copy()).cuda()
    ctx.ntt(t)
    got = host_u64(t)[0]
    lg = 12
    perm = np.array([brv(i, lg) for i in range(ctx.n)])
    for l, (q, psi) in enumerate(zip(ctx.primes, ctx.psi)):
        ref = RG.ntt_def(a[0, l], q, psi)
        assert (got[l] == ref[perm]).all()
    ctx.ntt(t, inverse=True)
    assert (host_u64(t) == a).all()


@pytest.mark.parametrize("shape", [(13, 3, 60), (14, 4, 60)])
def test_ntt_convolution_theorem(shape):
    ctx = context(*shape, 1)
    rng = np.random.default_rng(1)
    a = np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64) for q in ctx.primes])
    b = np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64) for q in ctx.primes])
    ta = torch.from_numpy(a.view(np.int64)[None].copy()).cuda()
    tb = torch.from_numpy(b.view(np.int64)[None].copy()).cuda()
    ctx.ntt(ta)
    ctx.ntt(tb)
    A, B = host_u64(ta)[0], host_u64(tb)[0]
    # a few transform entries against the definition a(psi^(2 rev(i) + 1))
    lg = shape[0]
    for l, (q, psi) in enumerate(zip(ctx.primes, ctx.psi)):
        for i in (0, 1, ctx.n // 3, ctx.n - 1):
            x = pow(psi, 2 * brv(i, lg) + 1, q)
            ref = 0
            for c in reversed(a[l].tolist()):
                ref = (ref * x + c) % q
            assert int(A[l, i]) == ref
    C = np.stack([np.array([int(x) * int(y) % q for x, y in zip(A[l], B[l])], dtype=np.uint64)
                  for l, q in enumerate(ctx.primes)])
    tc = torch.from_numpy(C.view(np.int64)[None].copy()).cuda()
    ctx.ntt(tc, inverse=True)
    got = host_u64(tc)[0]
    l = len(ctx.primes) - 1
    assert (got[l] == RG.negacyclic_mul(a[l], b[l], ctx.primes[l])).all()
    ctx.ntt(ta, inverse=True)
    assert (host_u64(ta)[0] == a).all()


# --------------------------------------------------- full ciphertext parity

def _plan(d):
    return {k: E.Tile(*v) for k, v in d.items()}


def _run_fwd(ctx, layer, plan, ts, enc_nonce, nonce):
    ct_x = ctx.encrypt(layer, plan, "x_fwd", dev(ts["x1"]), enc_nonce)
    ct_y, y0 = ctx.linear_fwd(layer, plan, ct_x, dev(ts["x0"]), dev(ts["W"]), nonce)
    y1 = ctx.decrypt(layer, plan, "fwd", ct_y)
    torch.cuda.synchronize()
    return ct_x, ct_y, y0, y1


def test_config1_bit_exact():
    cfg = CONFIGS[1]
    layer = cfg.layers[0]
    ctx = context(layer.log2_n, layer.num_limbs, layer.prime_bits, cfg.seed)
    ts = config_tensors(cfg)[0]
    tiles = {"fwd": (4, 10, 64, 1, 1, 1, 1)}
    plan = _plan(tiles)
    P = oracle_params(ctx)
    keys = oracle_keys(ctx)
    ct_x, ct_y, y0, y1 = _run_fwd(ctx, layer, tiles, ts, 5, 6)
    ref_x = PRT.encrypt_operand(P, keys["pk"], layer, plan, PRT.OPERAND_X_FWD, ts["x1"], cfg.seed, 5)
    assert (host_u64(ct_x) == np.stack([oracle_ct_ntt(P, c) for c in ref_x])).all()
    out, ref_y0 = PRT.mo_product(P, keys["pk"], layer, "fwd", plan["fwd"], [(("ct", ref_x), ("pt", ts["W"]))],
                                 cfg.seed, 6, add_share=ts["x0"])
    assert (host_u64(ct_y) == np.stack([out[o] for o in range(len(out))])).all()
    assert (host_i64(y0) == ref_y0).all()
    ref_y1 = PRT.decrypt_output(P, keys["sk"], layer, "fwd", plan["fwd"], [out[o] for o in range(len(out))])
    assert (host_i64(y1) == ref_y1).all()
    assert ((host_i64(y0) + host_i64(y1)) % P.t == LN.layer_op(layer, "fwd", ts["X"], ts["W"], P.t)).all()


SMALL_PLANS = [
    (small_cases()[1], {"fwd": (2, 3, 20, 1, 1, 1, 1), "dx": (3, 8, 7, 1, 1, 1, 1), "dw": (4, 3, 5, 1, 1, 1, 1)}),
    (small_cases()[2], {"fwd": (2, 2, 2, 3, 5, 3, 3), "dx": (1, 2, 3, 2, 5, 3, 3), "dw": (2, 2, 1, 3, 3, 2, 5)}),
    (small_cases()[3], {"fwd": (1, 3, 2, 4, 7, 3, 3), "dx": (2, 2, 3, 3, 4, 3, 3), "dw": (3, 4, 1, 3, 3, 4, 7)}),
    (small_cases()[4], {"fwd": (2, 2, 2, 5, 5, 2, 2), "dx": (1, 2, 2, 6, 6, 2, 2), "dw": (2, 2, 2, 2, 2, 5, 5)}),
    # Conv1d: ragged channel, length and kernel tiles
    (conv1d(2, 3, 4, 13, k=5, pad=2, log2_n=11, num_limbs=2, prime_bits=50),
     {"fwd": (2, 3, 2, 1, 6, 1, 3), "dx": (1, 2, 3, 1, 5, 1, 4), "dw": (2, 3, 1, 1, 3, 1, 6)}),
]


@pytest.mark.parametrize("case", range(len(SMALL_PLANS)))
def test_small_layers_bit_exact(case):
    layer, tiles = SMALL_PLANS[case]
    seed = 20 + case
    ctx = context(layer.log2_n, layer.num_limbs, layer.prime_bits, seed)
    plan = _plan(tiles)
    P = oracle_params(ctx)
    keys = oracle_keys(ctx)
    ts = layer_tensors(layer, seed)
    t = P.t
    # forward
    ct_x, ct_y, y0, y1 = _run_fwd(ctx, layer, tiles, ts, 100, 101)
    ref_x = PRT.encrypt_operand(P, keys["pk"], layer, plan, PRT.OPERAND_X_FWD, ts["x1"], seed, 100)
    assert (host_u64(ct_x) == np.stack([oracle_ct_ntt(P, c) for c in ref_x])).all()
    out, ref_y0 = PRT.mo_product(P, keys["pk"], layer, "fwd", plan["fwd"], [(("ct", ref_x), ("pt", ts["W"]))],
                                 seed, 101, add_share=ts["x0"])
    assert (host_u64(ct_y) == np.stack([out[o] for o in range(len(out))])).all()
    assert (host_i64(y0) == ref_y0).all()
    assert ((host_i64(y0) + host_i64(y1)) % t == LN.layer_op(layer, "fwd", ts["X"], ts["W"], t)).all()
    # backward
    cts = {}
    for name, kind, src in (("dy_dx", PRT.OPERAND_DY_DX, "dy1"), ("x_dw", PRT.OPERAND_X_DW, "x1"),
                            ("dy_dw", PRT.OPERAND_DY_DW, "dy1")):
        g = ctx.encrypt(layer, tiles, name, dev(ts[src]), 200)
        r = PRT.encrypt_operand(P, keys["pk"], layer, plan, kind, ts[src], seed, 200)
        assert (host_u64(g) == np.stack([oracle_ct_ntt(P, c) for c in r])).all(), name
        cts[name] = (g, r)
    ct_dx, dx0, ct_dw, dwm = ctx.linear_bwd(layer, tiles, cts["dy_dx"][0], cts["x_dw"][0], cts["dy_dw"][0],
                                            dev(ts["dy0"]), dev(ts["x0"]), dev(ts["W"]), 201)
    dx1 = ctx.decrypt(layer, tiles, "dx", ct_dx)
    dw1 = ctx.decrypt(layer, tiles, "dw", ct_dw)
    torch.cuda.synchronize()
    odx, odx0 = PRT.mo_product(P, keys["pk"], layer, "dx", plan["dx"], [(("ct", cts["dy_dx"][1]), ("pt", ts["W"]))],
                               seed, 201, add_share=ts["dy0"])
    assert (host_u64(ct_dx) == np.stack([odx[o] for o in range(len(odx))])).all()
    assert (host_i64(dx0) == odx0).all()
    odw, odwm = PRT.mo_product(P, keys["pk"], layer, "dw", plan["dw"],
                               [(("ct", cts["x_dw"][1]), ("pt", ts["dy0"])), (("pt", ts["x0"]), ("ct", cts["dy_dw"][1]))],
                               seed, 201)
    assert (host_u64(ct_dw) == np.stack([odw[o] for o in range(len(odw))])).all()
    assert (host_i64(dwm) == odwm).all()
    assert ((host_i64(dx0) + host_i64(dx1)) % t == LN.layer_op(layer, "dx", ts["dY"], ts["W"], t)).all()
    cross = (LN.layer_op(layer, "dw", ts["x1"], ts["dy0"], t) + LN.layer_op(layer, "dw", ts["x0"], ts["dy1"], t)) % t
    assert ((host_i64(dwm) + host_i64(dw1)) % t == cross).all()
    ref_dw1 = PRT.decrypt_output(P, keys["sk"], layer, "dw", plan["dw"], [odw[o] for o in range(len(odw))])
    assert (host_i64(dw1) == ref_dw1).all()


def test_bias_is_added_to_model_owner_share():
    layer = small_cases()[2]
    tiles = SMALL_PLANS[1][1]
    ctx = context(layer.log2_n, layer.num_limbs, layer.prime_bits, 21)
    ts = layer_tensors(layer, 3)
    bias = np.random.default_rng(5).integers(0, ctx.t, layer.c_out)
    ct_x = ctx.encrypt(layer, tiles, "x_fwd", dev(ts["x1"]), 7)
    _, y0 = ctx.linear_fwd(layer, tiles, ct_x, dev(ts["x0"]), dev(ts["W"]), 8)
    _, y0b = ctx.linear_fwd(layer, tiles, ct_x, dev(ts["x0"]), dev(ts["W"]), 8, bias=dev(bias))
    d = (host_i64(y0b) - host_i64(y0)) % ctx.t
    assert (d == bias.reshape(1, -1, 1, 1)).all()


def test_misaligned_buffers_are_rejected_on_the_host():
    """Polynomial and ciphertext buffers move in 16-byte pairs: an 8-byte-offset
    pointer is refused before any launch."""
    ctx = context(12, 2, 50, 1)
    flat = torch.zeros(ctx.L * ctx.n + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(RuntimeError, match="aligned"):
        ctx.ntt(flat[1:])
    ctx.ntt(flat[:-1])   # the aligned view is accepted
    torch.cuda.synchronize()
