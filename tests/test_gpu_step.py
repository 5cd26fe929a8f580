"""The batched step (all products of several layers in a few phase launches,
optionally replayed as a captured HIP graph) against the per-layer calls,
which the parity tests pin to the oracle.  Outputs must be bit-identical, and
graph replays must match eager runs with the same nonces."""
import numpy as np
import pytest
import torch

from workloads import CONFIGS, conv, config_tensors, fc, layer_tensors

from gpu_common import dev, host_i64, host_u64

pytestmark = pytest.mark.gpu

_ctx = {}


def context(layer, seed):
    from paper_2403_11166_amd import Context
    key = (layer.log2_n, layer.num_limbs, layer.prime_bits, seed)
    if key not in _ctx:
        _ctx[key] = Context(layer.log2_n, layer.num_limbs, layer.prime_bits, seed)
    return _ctx[key]


def build(layers, tensors, seed, plans=None):
    """Contexts, plans (the planner's unless given), encrypted inputs and output
    buffers for every layer."""
    ents = []
    for li, (layer, ts) in enumerate(zip(layers, tensors)):
        ctx = context(layer, seed)
        plan = ctx.plan_auto(layer) if plans is None else plans[li]
        sz = ctx.layout(layer, plan)
        d = {k: dev(v) for k, v in ts.items()}
        io = dict(ct_x1=ctx.encrypt(layer, plan, "x_fwd", d["x1"], 500 + li),
                  ct_dy_dx=ctx.encrypt(layer, plan, "dy_dx", d["dy1"], 600 + li),
                  ct_x_dw=ctx.encrypt(layer, plan, "x_dw", d["x1"], 700 + li),
                  ct_dy_dw=ctx.encrypt(layer, plan, "dy_dw", d["dy1"], 800 + li),
                  x0=d["x0"], dy0=d["dy0"], w=d["W"], bias=None,
                  ct_y=ctx.empty_cts(sz.n_out[0]), ct_dx=ctx.empty_cts(sz.n_out[1]),
                  ct_dw=ctx.empty_cts(sz.n_out[2]),
                  y0=torch.empty(layer.y_shape(), dtype=torch.int64, device="cuda"),
                  dx0=torch.empty(layer.x_shape(), dtype=torch.int64, device="cuda"),
                  dw_mask=torch.empty(layer.w_shape(), dtype=torch.int64, device="cuda"))
        ents.append((ctx, layer, plan, io))
    return ents


OUTS = ("ct_y", "y0", "ct_dx", "dx0", "ct_dw", "dw_mask")


def snapshot(ents):
    torch.cuda.synchronize()
    return [{k: io[k].detach().cpu().numpy().copy() for k in OUTS} for _, _, _, io in ents]


def per_layer(ents, nonce):
    for i, (ctx, layer, plan, io) in enumerate(ents):
        ctx.linear_fwd(layer, plan, io["ct_x1"], io["x0"], io["w"], nonce + 2 * i, out=(io["ct_y"], io["y0"]))
        ctx.linear_bwd(layer, plan, io["ct_dy_dx"], io["ct_x_dw"], io["ct_dy_dw"], io["dy0"], io["x0"], io["w"],
                       nonce + 2 * i + 1, out=(io["ct_dx"], io["dx0"], io["ct_dw"], io["dw_mask"]))
    return snapshot(ents)


def clear(ents):
    for _, _, _, io in ents:
        for k in OUTS:
            io[k].zero_()


def assert_same(a, b):
    for la, lb in zip(a, b):
        for k in OUTS:
            assert np.array_equal(la[k], lb[k]), k


def make_step(ents):
    from paper_2403_11166_amd import Step
    step = Step([(c, l, p) for c, l, p, _ in ents])
    ws = torch.empty(step.workspace_bytes(), dtype=torch.uint8, device="cuda")
    step.bind([io for _, _, _, io in ents], ws)
    return step, ws


MIXED = [conv(3, 2, 3, 6, k=3, pad=1, log2_n=11, num_limbs=2, prime_bits=50),
         conv(3, 3, 4, 5, k=3, pad=1, log2_n=12, num_limbs=3, prime_bits=60),
         fc(3, 17, 5, log2_n=11, num_limbs=2, prime_bits=50),
         fc(4, 30, 6, log2_n=12, num_limbs=3, prime_bits=60)]


def test_step_equals_per_layer_calls_mixed_degrees():
    tensors = [layer_tensors(l, 90 + i) for i, l in enumerate(MIXED)]
    ents = build(MIXED, tensors, 5)
    ref = per_layer(ents, 1000)
    clear(ents)
    step, _ws = make_step(ents)
    step.run(1000)
    assert_same(snapshot(ents), ref)


def test_graph_replays_match_eager_runs():
    tensors = [layer_tensors(l, 95 + i) for i, l in enumerate(MIXED)]
    ents = build(MIXED, tensors, 6)
    step, _ws = make_step(ents)
    n = len(MIXED)
    step.run(2000)
    r0 = snapshot(ents)
    step.run(2000 + 2 * n)
    r1 = snapshot(ents)
    assert not np.array_equal(r0[0]["ct_y"], r1[0]["ct_y"])  # fresh nonce, fresh randomness
    step.capture()
    clear(ents)
    step.set_nonce(2000)
    for rep, want in enumerate((r0, r1, r0)):
        if rep == 2:
            step.set_nonce(2000)
        step.replay()
        got = snapshot(ents)
        assert_same(got, want)
        # eager work of the program between replays
        x = torch.randn(1000, device="cuda")
        torch.cuda.synchronize()
        assert torch.isfinite(x.sum())


def test_step_equals_per_layer_calls_config4():
    cfg = CONFIGS[4]
    ents = build(cfg.layers, config_tensors(cfg), cfg.seed)
    ref = per_layer(ents, 3000)
    clear(ents)
    step, _ws = make_step(ents)
    step.run(3000)
    assert_same(snapshot(ents), ref)


def test_every_schedule_variant_is_bit_identical_and_autotune_picks_one(tmp_path):
    """The multiply-accumulate schedules are schedules only: under one plan the
    outputs are identical for every candidate, and the autotuner's choice is one
    of them.  The autotuner may also pick another partition (a different
    ciphertext layout, so the inputs are encrypted with the tuned plan): the
    decrypted products are the same as under the planner's partition."""
    from paper_2403_11166_amd.api import plan_dict
    layer = MIXED[1]
    ts = layer_tensors(layer, 77)
    ctx = context(layer, 8)
    cache = str(tmp_path / "tune.txt")
    tuned = ctx.autotune(layer, ctx.plan_auto(layer), cache)
    assert all(0 <= v < 9 for v in tuned.sched)
    ents = build([layer], [ts], 8, plans=[tuned])
    _, _, plan, io = ents[0]
    chosen = list(plan.sched)
    results = []
    for v in range(9):
        for op in range(3):
            plan.sched[op] = v
        results.append(per_layer(ents, 4000))
    for r in results[1:]:
        assert_same(r, results[0])
    for op in range(3):
        plan.sched[op] = chosen[op]
    assert_same(per_layer(ents, 4000), results[0])
    # the same products under the planner's own partition decrypt to the same shares' sums
    base = build([layer], [ts], 8)
    per_layer(base, 4000)
    t = ctx.t
    for ents_, name in ((ents, "tuned"), (base, "planner")):
        c, L_, p, o = ents_[0]
        y1 = c.decrypt(L_, p, "fwd", o["ct_y"])
        dx1 = c.decrypt(L_, p, "dx", o["ct_dx"])
        dw1 = c.decrypt(L_, p, "dw", o["ct_dw"])
        torch.cuda.synchronize()
        recon = [(host_i64(o["y0"]) + host_i64(y1)) % t, (host_i64(o["dx0"]) + host_i64(dx1)) % t,
                 (host_i64(o["dw_mask"]) + host_i64(dw1)) % t]
        if name == "tuned":
            first = recon
        else:
            for a, b in zip(first, recon):
                assert np.array_equal(a, b)
    text = open(cache).read()
    assert "ntt_loge" in text and "op=2" in text and "sched" in text
    again = ctx.autotune(layer, ctx.plan_auto(layer), cache)  # cache hits: same choices, no new lines
    assert tuple(again.sched) == tuple(tuned.sched)
    assert plan_dict(again) == plan_dict(tuned)
    assert open(cache).read() == text


def test_failed_rebind_leaves_the_step_unbound():
    """A bind that fails (here: a missing weight buffer) after a good one must
    not leave the old or a partial segment table behind: run and capture both
    refuse the step until a bind succeeds again."""
    from paper_2403_11166_amd import PencilError
    tensors = [layer_tensors(l, 97 + i) for i, l in enumerate(MIXED[:2])]
    ents = build(MIXED[:2], tensors, 9)
    step, ws = make_step(ents)
    step.run(5000)
    bad = [dict(io) for _, _, _, io in ents]
    bad[1]["w"] = None
    with pytest.raises(PencilError, match="missing buffer"):
        step.bind(bad, ws)
    with pytest.raises(PencilError, match="not bound"):
        step.run(5000)
    with pytest.raises(PencilError, match="not bound"):
        step.capture()
    with pytest.raises(PencilError, match="no captured graph"):
        step.replay()
    step.bind([io for _, _, _, io in ents], ws)
    step.run(5000)
    torch.cuda.synchronize()


def test_restart_at_step_k_reproduces_the_continuous_run():
    """The state a training run carries from step to step is the key seed and
    the nonce counter: a run restarted at step k from fresh contexts (key
    generation again from the same seed), a fresh step and a fresh graph, with
    the base nonce of step k, reproduces step k of the continuous run bit for
    bit, as a graph replay and as an eager run."""
    tensors = [layer_tensors(l, 120 + i) for i, l in enumerate(MIXED)]
    n, base, k = len(MIXED), 7000, 2
    ents = build(MIXED, tensors, 17)
    step, _ws = make_step(ents)
    step.capture()
    step.set_nonce(base)
    outs = []
    for _ in range(k + 1):
        step.replay()
        outs.append(snapshot(ents))
    assert not np.array_equal(outs[0][0]["ct_y"], outs[k][0]["ct_y"])
    step.close()
    del ents, step, _ws
    _ctx.clear()
    ents2 = build(MIXED, tensors, 17)
    step2, _ws2 = make_step(ents2)
    step2.capture()
    step2.set_nonce(base + 2 * n * k)
    step2.replay()
    assert_same(snapshot(ents2), outs[k])
    clear(ents2)
    step2.run(base + 2 * n * k)
    assert_same(snapshot(ents2), outs[k])
