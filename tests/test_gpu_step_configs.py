"""The timed path at the benchmark workloads' full sizes: the batched step
(every product of every layer in a few phase launches) and its captured HIP
graph, exactly as bench.py builds them (the planner's partition, autotuned
schedules), on the FC layer 784 -> 128 (config 2), the 3 -> 64 convolution
(config 3) and the eight-layer convolution stack at N = 16384 (config 5).

* Every output ciphertext and model-owner share of the step is bit-identical
  to the per-layer calls made with nonces base + 2i (forward) and base + 2i + 1
  (backward), which the ciphertext-level parity tests pin to the oracle.
* Graph replays equal the eager step, with eager work between replays.
* Every element of Y, dX and of the weight gradient's cross terms
  (<dY>_0 o <X>_1 + <dY>_1 o <X>_0, Alg. 2) reconstructed from the step's
  outputs equals the oracle's plaintext layer, with no sampling.
"""
import pytest
import torch

from oracle import linear as LN
from workloads import CONFIGS, config_tensors

from gpu_common import dev, host_i64

pytestmark = pytest.mark.gpu

STEP_CONFIGS = (2, 3, 5)
BASE = 7000
OUTS = ("ct_y", "y0", "ct_dx", "dx0", "ct_dw", "dw_mask")

_state = {}


def _free_others(keep):
    for k in list(_state):
        if k != keep:
            del _state[k]
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def state(ci):
    """Contexts, autotuned plans, encrypted inputs, the bound step and a
    snapshot of its eager outputs for workload ci (built once)."""
    if ci in _state:
        return _state[ci]
    _free_others(ci)
    from paper_2403_11166_amd import Context, Step
    cfg = CONFIGS[ci]
    tensors = config_tensors(cfg)
    ctxs, tuned, ents = {}, {}, []
    for li, (layer, ts) in enumerate(zip(cfg.layers, tensors)):
        key = (layer.log2_n, layer.num_limbs, layer.prime_bits)
        if key not in ctxs:
            ctxs[key] = Context(layer.log2_n, layer.num_limbs, layer.prime_bits, cfg.seed)
        ctx = ctxs[key]
        shape = (key, layer.kind, layer.c_in, layer.c_out, layer.h, layer.w, layer.k, layer.pad)
        if shape not in tuned:
            tuned[shape] = ctx.autotune(layer, ctx.plan_auto(layer))
        plan = tuned[shape]
        sz = ctx.layout(layer, plan)
        d = {k: dev(v) for k, v in ts.items()}
        io = dict(ct_x1=ctx.encrypt(layer, plan, "x_fwd", d["x1"], 100 + li),
                  ct_dy_dx=ctx.encrypt(layer, plan, "dy_dx", d["dy1"], 200 + li),
                  ct_x_dw=ctx.encrypt(layer, plan, "x_dw", d["x1"], 300 + li),
                  ct_dy_dw=ctx.encrypt(layer, plan, "dy_dw", d["dy1"], 400 + li),
                  x0=d["x0"], dy0=d["dy0"], w=d["W"], bias=None,
                  ct_y=ctx.empty_cts(sz.n_out[0]), ct_dx=ctx.empty_cts(sz.n_out[1]),
                  ct_dw=ctx.empty_cts(sz.n_out[2]),
                  y0=torch.empty(layer.y_shape(), dtype=torch.int64, device="cuda"),
                  dx0=torch.empty(layer.x_shape(), dtype=torch.int64, device="cuda"),
                  dw_mask=torch.empty(layer.w_shape(), dtype=torch.int64, device="cuda"))
        ents.append((ctx, layer, plan, io))
    step = Step([(c, l, p) for c, l, p, _ in ents], ops=cfg.ops)
    ws = torch.empty(step.workspace_bytes(), dtype=torch.uint8, device="cuda")
    step.bind([io for _, _, _, io in ents], ws)
    step.run(BASE)
    torch.cuda.synchronize()
    snap = [{k: io[k].clone() for k in OUTS} for _, _, _, io in ents]
    st = dict(cfg=cfg, tensors=tensors, ents=ents, step=step, ws=ws, snap=snap)
    _state[ci] = st
    return st


def _equal_outputs(ents, snap, what):
    torch.cuda.synchronize()
    for li, (_, _, _, io) in enumerate(ents):
        for k in OUTS:
            assert torch.equal(io[k], snap[li][k]), f"{what}: layer {li} {k} differs"


def check_per_layer_calls(st):
    ents = st["ents"]
    for _, _, _, io in ents:
        for k in OUTS:
            io[k].zero_()
    for i, (ctx, layer, plan, io) in enumerate(ents):
        ctx.linear_fwd(layer, plan, io["ct_x1"], io["x0"], io["w"], BASE + 2 * i, out=(io["ct_y"], io["y0"]))
        ctx.linear_bwd(layer, plan, io["ct_dy_dx"], io["ct_x_dw"], io["ct_dy_dw"], io["dy0"], io["x0"], io["w"],
                       BASE + 2 * i + 1, out=(io["ct_dx"], io["dx0"], io["ct_dw"], io["dw_mask"]))
    _equal_outputs(ents, st["snap"], "per-layer calls")


def check_graph_replays(st):
    ents, step = st["ents"], st["step"]
    step.capture()
    for rep in range(2):
        for _, _, _, io in ents:
            for k in OUTS:
                io[k].zero_()
        step.set_nonce(BASE)
        step.replay()
        _equal_outputs(ents, st["snap"], f"graph replay {rep}")
        # the program's own eager work between replays
        x = torch.randn(4096, device="cuda")
        torch.cuda.synchronize()
        assert torch.isfinite(x.sum())


def check_reconstruction(st, li):
    """Decrypt the step's outputs of layer li and reconstruct each product in
    full against the oracle's plaintext layer (Alg. 1, Sec. III.B.2, Alg. 2)."""
    ctx, layer, plan, _ = st["ents"][li]
    out = st["snap"][li]
    ts = st["tensors"][li]
    t = ctx.t
    y1 = ctx.decrypt(layer, plan, "fwd", out["ct_y"])
    dx1 = ctx.decrypt(layer, plan, "dx", out["ct_dx"])
    dw1 = ctx.decrypt(layer, plan, "dw", out["ct_dw"])
    torch.cuda.synchronize()
    y = (host_i64(out["y0"]) + host_i64(y1)) % t
    assert (y == LN.layer_op(layer, "fwd", ts["X"], ts["W"], t)).all(), "Y"
    dx = (host_i64(out["dx0"]) + host_i64(dx1)) % t
    assert (dx == LN.layer_op(layer, "dx", ts["dY"], ts["W"], t)).all(), "dX"
    dw = (host_i64(out["dw_mask"]) + host_i64(dw1)) % t
    cross = (LN.layer_op(layer, "dw", ts["x1"], ts["dy0"], t) + LN.layer_op(layer, "dw", ts["x0"], ts["dy1"], t)) % t
    assert (dw == cross).all(), "dW cross terms"


def _cases():
    # one workload's checks run back to back, so each is built once
    out = []
    for ci in STEP_CONFIGS:
        out += [(ci, "per_layer_calls", 0), (ci, "graph_replays", 0)]
        out += [(ci, "reconstruct", li) for li in range(len(CONFIGS[ci].layers))]
    return out


@pytest.mark.parametrize("ci,check,li", _cases())
def test_timed_step(ci, check, li):
    st = state(ci)
    if check == "per_layer_calls":
        check_per_layer_calls(st)
    elif check == "graph_replays":
        check_graph_replays(st)
    else:
        check_reconstruction(st, li)
        if li == len(st["ents"]) - 1:
            _free_others(None)
