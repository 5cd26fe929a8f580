"""GPU parity at the benchmark workloads' full sizes (configs 2-5), in the
launch configuration bench.py times (the planner's own partition).

* End to end: the data owner's encryptions, the model owner's forward and
  backward products and the decryptions must reconstruct the plaintext layer
  results exactly, every element of every product (the oracle's plaintext
  layers finish the largest of these shapes in tens of seconds).
* Bit for bit: the model owner's products on synthetic uniform ciphertext
  inputs, encryption and decryption are compared with the oracle on sampled
  output tiles and coefficients.
"""
import numpy as np
import pytest
import torch

from oracle import bfv
from oracle import encoding as E
from oracle import linear as LN
from oracle import protocol as PRT
from workloads import CONFIGS, config_tensors, uniform_residues

from gpu_common import dev, host_i64, host_u64, ntt_order_roots, oracle_keys, oracle_params, split30, unsplit30

pytestmark = pytest.mark.gpu

# distinct layer shapes of each workload (config 5 repeats three shapes)
CASES = [(2, 0), (3, 0), (4, 0), (4, 1), (4, 2), (4, 3), (5, 0), (5, 3), (5, 6)]
FULL_CHECK_LIMIT = 5e9  # output elements x contraction length the oracle computes in full (every case here)

_ctx = {}
_tensors = {}


def context(layer, seed):
    from paper_2403_11166_amd import Context
    key = (layer.log2_n, layer.num_limbs, layer.prime_bits, seed)
    if key not in _ctx:
        _ctx[key] = Context(layer.log2_n, layer.num_limbs, layer.prime_bits, seed)
    return _ctx[key]


def tensors(ci):
    if ci not in _tensors:
        _tensors[ci] = config_tensors(CONFIGS[ci])
    return _tensors[ci]


def plan_tiles(p):
    return {"fwd": E.Tile(*p.fwd.astuple()), "dx": E.Tile(*p.dx.astuple()), "dw": E.Tile(*p.dw.astuple())}


def contraction(layer, op):
    if op == "fwd":
        return layer.c_in * layer.k * layer.k
    if op == "dx":
        return layer.c_out * layer.k * layer.k
    return layer.batch * layer.h_out * layer.w_out


def check_op(layer, op, got, a, b, t, rng, extra=None):
    """got == layer_op(a, b) (+ extra) mod t; in full or on 48 sampled elements."""
    size = got.size
    if size * contraction(layer, op) <= FULL_CHECK_LIMIT:
        ref = LN.layer_op(layer, op, a, b, t)
        if extra is not None:
            ref = (ref + LN.layer_op(layer, op, *extra, t)) % t
        assert (got == ref).all(), f"{op}: {(got != ref).sum()} of {size} elements differ"
        return
    flat = np.unique(np.concatenate([[0, size - 1], rng.integers(0, size, 46)]))
    pts = [tuple(int(v) for v in np.unravel_index(i, got.shape)) for i in flat]
    ref = LN.layer_op_at(layer, op, a, b, t, pts)
    if extra is not None:
        ref = [(x + y) % t for x, y in zip(ref, LN.layer_op_at(layer, op, *extra, t, pts))]
    assert [int(got[p]) for p in pts] == ref, op


@pytest.mark.parametrize("ci,li", CASES)
def test_layer_end_to_end_reconstructs(ci, li):
    cfg = CONFIGS[ci]
    layer = cfg.layers[li]
    ts = tensors(ci)[li]
    ctx = context(layer, cfg.seed)
    plan = ctx.plan_auto(layer)
    t = ctx.t
    d = {k: dev(v) for k, v in ts.items()}
    ct_x = ctx.encrypt(layer, plan, "x_fwd", d["x1"], 11)
    ct_y, y0 = ctx.linear_fwd(layer, plan, ct_x, d["x0"], d["W"], 12)
    y1 = ctx.decrypt(layer, plan, "fwd", ct_y)
    c1 = ctx.encrypt(layer, plan, "dy_dx", d["dy1"], 13)
    c2 = ctx.encrypt(layer, plan, "x_dw", d["x1"], 14)
    c3 = ctx.encrypt(layer, plan, "dy_dw", d["dy1"], 15)
    ct_dx, dx0, ct_dw, dwm = ctx.linear_bwd(layer, plan, c1, c2, c3, d["dy0"], d["x0"], d["W"], 16)
    dx1 = ctx.decrypt(layer, plan, "dx", ct_dx)
    dw1 = ctx.decrypt(layer, plan, "dw", ct_dw)
    torch.cuda.synchronize()
    rng = np.random.default_rng(ci * 10 + li)
    check_op(layer, "fwd", (host_i64(y0) + host_i64(y1)) % t, ts["X"], ts["W"], t, rng)
    check_op(layer, "dx", (host_i64(dx0) + host_i64(dx1)) % t, ts["dY"], ts["W"], t, rng)
    check_op(layer, "dw", (host_i64(dwm) + host_i64(dw1)) % t, ts["x1"], ts["dy0"], t, rng,
             extra=(ts["x0"], ts["dy1"]))


def _sample_idx(n, slots, rng, k=12):
    return sorted(set([0, n - 1] + list(slots[:2]) + list(rng.integers(0, n, k))))


@pytest.mark.parametrize("ci,li", [(2, 0), (3, 0), (4, 1), (5, 6)])
def test_products_bit_exact_on_sampled_coefficients(ci, li):
    """The model owner's products on synthetic ciphertext inputs, and encryption
    and decryption, against the oracle on sampled output tiles/coefficients."""
    cfg = CONFIGS[ci]
    layer = cfg.layers[li]
    ts = tensors(ci)[li]
    ctx = context(layer, cfg.seed)
    plan = ctx.plan_auto(layer)
    tiles = plan_tiles(plan)
    sz = ctx.layout(layer, plan)
    P = oracle_params(ctx)
    keys = oracle_keys(ctx)
    rng = np.random.default_rng(100 + ci)
    L, n = ctx.L, ctx.n
    synth = {}
    for name, cnt, seed in (("x", sz.n_ct[0], 1), ("dydx", sz.n_ct[1], 2), ("xdw", sz.n_ct[2], 3),
                            ("dydw", sz.n_ct[3], 4)):
        synth[name] = uniform_residues(1000 * ci + seed, (int(cnt), 2, L, n), ctx.primes)
    # the oracle takes these as coefficient-domain ciphertexts; the library's
    # product path takes its inputs in the NTT domain (split form), so the
    # device copies are transformed (by the library's transform, itself checked
    # against the definition in the NTT parity test) and stored split
    def g(a):
        t = ctx.ntt(torch.from_numpy(a.copy().view(np.int64)).cuda())
        return torch.from_numpy(split30(host_u64(t)).view(np.int64)).cuda()

    ct_y, y0 = ctx.linear_fwd(layer, plan, g(synth["x"]), dev(ts["x0"]), dev(ts["W"]), 21)
    ct_dx, dx0, ct_dw, dwm = ctx.linear_bwd(layer, plan, g(synth["dydx"]), g(synth["xdw"]), g(synth["dydw"]),
                                            dev(ts["dy0"]), dev(ts["x0"]), dev(ts["W"]), 22)
    y1 = ctx.decrypt(layer, plan, "fwd", ct_y)
    torch.cuda.synchronize()
    got = {"fwd": (host_u64(ct_y), host_i64(y0)), "dx": (host_u64(ct_dx), host_i64(dx0)),
           "dw": (host_u64(ct_dw), host_i64(dwm))}
    terms = {"fwd": [(("ct", synth["x"]), ("pt", ts["W"]))],
             "dx": [(("ct", synth["dydx"]), ("pt", ts["W"]))],
             "dw": [(("ct", synth["xdw"]), ("pt", ts["dy0"])), (("pt", ts["x0"]), ("ct", synth["dydw"]))]}
    adds = {"fwd": ts["x0"], "dx": ts["dy0"], "dw": None}
    nonces = {"fwd": 21, "dx": 22, "dw": 22}
    for op in ("fwd", "dx", "dw"):
        gm = E.geometry(layer, op)
        c = E.counts(gm, tiles[op])
        outs = sorted({0, c.n_out - 1})
        for o in outs:
            mi, ri, oyi, oxi = list(E.out_tiles(c))[o]
            slots = [s for s, _ in E.out_slots(gm, tiles[op], mi, ri, oyi, oxi)]
            idx = _sample_idx(n, slots, rng)
            ref, share = PRT.mo_product(P, keys["pk"], layer, op, tiles[op], terms[op], cfg.seed, nonces[op],
                                        add_share=adds[op], outs=[o], coeff_idx=idx)
            assert (got[op][0][o][:, :, idx] == ref[o]).all(), (op, o)
            # model owner's share entries computed for this tile
            mask = share >= 0
            assert (got[op][1][mask] == share[mask]).all(), (op, o)
    # decryption of a synthetic-input output ciphertext at sampled output slots
    gm = E.geometry(layer, "fwd")
    c = E.counts(gm, tiles["fwd"])
    o = c.n_out - 1
    mi, ri, oyi, oxi = list(E.out_tiles(c))[o]
    pairs = E.out_slots(gm, tiles["fwd"], mi, ri, oyi, oxi)[:8]
    dec = bfv.decrypt_at(P, keys["sk"], got["fwd"][0][o], [s for s, _ in pairs])
    y1h = host_i64(y1)
    out_v = E.to_virtual_out(layer, "fwd", y1h)
    assert [int(out_v[m, r, yy, xx]) for _, (m, r, yy, xx) in pairs] == list(dec)
    # encryption: two ciphertexts of each operand layout, sampled coefficients
    for kind, src in ((PRT.OPERAND_X_FWD, "x1"), (PRT.OPERAND_DY_DX, "dy1"), (PRT.OPERAND_X_DW, "x1"),
                      (PRT.OPERAND_DY_DW, "dy1")):
        name = ("x_fwd", "dy_dx", "x_dw", "dy_dw")[kind]
        ct = unsplit30(host_u64(ctx.encrypt(layer, plan, name, dev(ts[src]), 30 + kind)))
        op, side = PRT.OPERAND_SIDE[kind]
        for j in sorted({0, ct.shape[0] - 1}):
            gm = E.geometry(layer, op)
            cc = E.counts(gm, tiles[op])
            if side == "a":
                m = E.encode_a(E.virtual_a(layer, op, ts[src]), gm, tiles[op], n, *list(E.a_tiles(cc))[j])
            else:
                m = E.encode_k(E.virtual_k(layer, op, ts[src]), gm, tiles[op], n, *list(E.k_tiles(cc))[j])
            idx = _sample_idx(n, [], rng, 4)
            # the library's ciphertexts are in the NTT domain: entry i is the
            # evaluation at psi^(2 rev(i) + 1) (stored split, undone above)
            ref = bfv.encrypt_eval_at(P, keys["pk"], m, cfg.seed, 30 + kind, PRT.enc_object(kind, j),
                                      ntt_order_roots(P, idx))
            assert [[[int(v) for v in ct[j][c, l, idx]] for l in range(P.num_limbs)] for c in range(2)] == ref, \
                (name, j)
