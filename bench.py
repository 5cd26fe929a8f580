#!/usr/bin/env python3
"""Throughput of the model owner's encrypted linear-layer products (fwd + bwd).

One step = every product of the workload's layers: the forward product
(Alg. 1), the input-gradient product and the weight-gradient cross terms
(Alg. 2), each through the whole hot path (share add + encode, NTT,
multiply-accumulate, re-randomise, inverse NTT, flood and mask), with the data
owner's ciphertexts and both parties' shares already resident in HBM.
Encryption and decryption (the data owner's ends) are outside the timed region.

Default workload: FC 784 -> 128, batch 64, forward and backward, N = 8192 with
three 60-bit RNS primes (the first layer of the paper's MNIST MLP).  After the
timed region the outputs are decrypted and checked bit for bit against exact
modular linear algebra (float64 digit products, exact below 2^53).

Prints one JSON line.  `--gpus N` with N > 1 exits: this build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Integer VALU issue peak: 256 CUs x 64 lanes x 2.4 GHz (one int32 op per lane per clock).
INT_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, help="workload index (1..5)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU oracle sample budget")
    ap.add_argument("--no-verify", action="store_true")
    return ap.parse_args()


# ------------------------------------------------------------- exact check

def _digits(v, t):
    import torch
    v = torch.where(v > (t - 1) // 2, v - t, v)
    out = []
    for _ in range(2):
        d = torch.remainder(v, 1 << 14)
        out.append(d.double())
        v = torch.div(v - d, 1 << 14, rounding_mode="floor")
    out.append(v.double())
    return out


def _lin_f64(layer, op, a, b):
    """The layer's product over float64 tensors holding integers (no rounding below 2^53)."""
    import torch
    import torch.nn.functional as F
    if layer.kind == "fc":
        return {"fwd": lambda: a @ b.t(), "dx": lambda: a @ b, "dw": lambda: b.t() @ a}[op]()
    k, p = layer.k, layer.pad
    ho, wo = layer.h_out, layer.w_out
    if op == "fwd":
        cols = F.unfold(a, k, padding=p)                           # (B, ci*k*k, ho*wo)
        return (b.reshape(b.shape[0], -1) @ cols).reshape(a.shape[0], b.shape[0], ho, wo)
    if op == "dx":                                               # a = dY, b = W
        cols = b.reshape(b.shape[0], -1).t() @ a.reshape(a.shape[0], a.shape[1], -1)  # (B, ci*k*k, ho*wo)
        return F.fold(cols, (layer.h, layer.w), k, padding=p)
    cols = F.unfold(a, k, padding=p)                               # a = X, b = dY
    g = torch.einsum("bop,bcp->oc", b.reshape(b.shape[0], b.shape[1], -1), cols)
    return g.reshape(b.shape[1], a.shape[1], k, k)


def exact_mod_t(layer, op, a, b, t):
    """Exact Z_t result of the layer's product on int64 tensors in [0, t)."""
    import torch
    da, db = _digits(a, t), _digits(b, t)
    T = [None] * 5
    for i in range(3):
        for j in range(3):
            s = torch.remainder(torch.round(_lin_f64(layer, op, da[i], db[j])).long(), t)
            T[i + j] = s if T[i + j] is None else torch.remainder(T[i + j] + s, t)
    acc = T[4]
    for d in range(3, -1, -1):
        acc = torch.remainder(acc * (1 << 14) + T[d], t)
    return acc


# ------------------------------------------------------------- work model

def kernel_work(sizes_list):
    """Algorithmic HBM bytes and int work per kernel kind over one step.

    bytes: every polynomial the kernel must read and write once (8-byte
    residues); NTT butterflies: (N/2) log2 N per limb-polynomial; MAC: one
    64 x 64 -> 128-bit multiply-accumulate per product, component, limb, slot.
    """
    work = {}
    for ctx_, sz, ops in sizes_list:
        n, L = ctx_.n, ctx_.L
        lg = n.bit_length() - 1
        poly = L * n * 8
        bfly = L * (n // 2) * lg
        for opi, op in enumerate(("fwd", "dx", "dw")):
            if op not in ops:
                continue
            n_out = sz.n_out[opi]
            if op == "fwd":
                n_ct_in, n_pt = sz.n_ct[0], sz.n_pt[0]
            elif op == "dx":
                n_ct_in, n_pt = sz.n_ct[1], sz.n_pt[1]
            else:
                n_ct_in, n_pt = sz.n_ct[2] + sz.n_ct[3], sz.n_pt[2]
            add = lambda k, b, o: work.__setitem__(k, (work.get(k, (0, 0))[0] + b, work.get(k, (0, 0))[1] + o))  # noqa
            add("ntt_ct", 2 * n_ct_in * 2 * poly, 2 * n_ct_in * bfly)
            add("ntt_pt", n_pt * poly, n_pt * bfly)
            add("ntt_ternary", n_out * poly, n_out * bfly)
            add("mac", (2 * n_ct_in + n_pt + n_out + 2 * n_out) * poly, sz.n_products[opi] * 2 * L * n)
            add("intt_out", 2 * n_out * 2 * poly, 2 * n_out * bfly)
            add("flood_mask", 2 * n_out * 2 * poly, 0)
    return work


# ------------------------------------------------------------- cpu baseline

def cpu_baseline(layer, seconds):
    """The oracle's plaintext x ciphertext product (schoolbook, per limb and
    component) timed on host cores for about `seconds`."""
    from oracle import bfv
    from oracle import params as PR
    P = PR.params_for(layer)
    rng = np.random.default_rng(0)
    ct = np.stack([np.stack([rng.integers(0, q, P.n, dtype=np.uint64) for q in P.moduli]) for _ in range(2)])
    w = rng.integers(0, P.t, P.n)
    done = 0
    t0 = time.perf_counter()
    while True:
        acc = [[[0] * P.n for _ in range(P.num_limbs)] for _ in range(2)]
        bfv.mul_plain_acc(P, acc, ct, w, P.t)
        done += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": done / el, "unit": "products/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} plaintext x ciphertext products at N={P.n}, L={P.num_limbs} "
                      f"(schoolbook negacyclic, both components, all limbs) in {el:.1f} s, single thread"}


# ------------------------------------------------------------- main

def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is described in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2403_11166_amd import Context
    from paper_2403_11166_amd import _abi as A
    from workloads import CONFIGS
    from workloads.gen import config_tensors
    import ctypes

    cfg = CONFIGS[args.config]
    tensors = config_tensors(cfg)
    torch.cuda.init()
    dev = torch.device("cuda", 0)
    ctxs = {}
    layers = []
    for li, (layer, ts) in enumerate(zip(cfg.layers, tensors)):
        key = (layer.log2_n, layer.num_limbs, layer.prime_bits)
        if key not in ctxs:
            ctxs[key] = Context(layer.log2_n, layer.num_limbs, layer.prime_bits, seed=cfg.seed)
        ctx = ctxs[key]
        plan = ctx.plan_auto(layer)
        sz = ctx.layout(layer, plan)
        d = {k: torch.from_numpy(v).to(dev) for k, v in ts.items()}
        ent = dict(layer=layer, ctx=ctx, plan=plan, sz=sz, d=d)
        ent["ct_x"] = ctx.encrypt(layer, plan, "x_fwd", d["x1"], 1000 + li)
        if "dx" in cfg.ops:
            ent["ct_dy_dx"] = ctx.encrypt(layer, plan, "dy_dx", d["dy1"], 2000 + li)
        if "dw" in cfg.ops:
            ent["ct_x_dw"] = ctx.encrypt(layer, plan, "x_dw", d["x1"], 3000 + li)
            ent["ct_dy_dw"] = ctx.encrypt(layer, plan, "dy_dw", d["dy1"], 4000 + li)
        ent["ws_f"] = ctx._ws(sz.ws_fwd_bytes)
        ent["ws_b"] = ctx._ws(sz.ws_bwd_bytes)
        ent["out_f"] = (ctx.empty_cts(sz.n_out[0]), torch.empty(layer.y_shape(), dtype=torch.int64, device=dev))
        ent["out_b"] = (ctx.empty_cts(sz.n_out[1]), torch.empty(layer.x_shape(), dtype=torch.int64, device=dev),
                        ctx.empty_cts(sz.n_out[2]), torch.empty(layer.w_shape(), dtype=torch.int64, device=dev))
        layers.append(ent)
    torch.cuda.synchronize()

    def step(nonce):
        for li, e in enumerate(layers):
            L_, c, d = e["layer"], e["ctx"], e["d"]
            c.linear_fwd(L_, e["plan"], e["ct_x"], d["x0"], d["W"], nonce * 64 + li, ws=e["ws_f"], out=e["out_f"])
            if "dx" in cfg.ops or "dw" in cfg.ops:
                c.linear_bwd(L_, e["plan"], e.get("ct_dy_dx"), e.get("ct_x_dw"), e.get("ct_dy_dw"), d["dy0"],
                             d["x0"], d["W"], nonce * 64 + li + 32, ws=e["ws_b"], out=e["out_b"],
                             do_dx="dx" in cfg.ops, do_dw="dw" in cfg.ops)

    for i in range(args.warmup):
        step(i + 1)
    torch.cuda.synchronize()
    for c in ctxs.values():
        c._check(c.lib.pencil_profile_enable(c.h, 1))
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        step(100 + i)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    stats = {}
    for c in ctxs.values():
        arr = (A.KernelStat * 16)()
        cnt = ctypes.c_int()
        c._check(c.lib.pencil_profile_read(c.h, arr, 16, ctypes.byref(cnt)))
        for i in range(cnt.value):
            nm = arr[i].name.decode()
            l0, m0 = stats.get(nm, (0, 0.0))
            stats[nm] = (l0 + arr[i].launches, m0 + arr[i].total_ms)
        c._check(c.lib.pencil_profile_enable(c.h, 0))

    products = sum(sum(e["sz"].n_products[i] for i, op in enumerate(("fwd", "dx", "dw")) if op in cfg.ops)
                   for e in layers)
    value = products / (ms_step / 1e3)

    # ------------------------------------------------------ bit-exact check
    bit_exact = None
    if not args.no_verify:
        bit_exact = True
        for e in layers:
            L_, c, d, t = e["layer"], e["ctx"], e["d"], e["ctx"].t
            y1 = c.decrypt(L_, e["plan"], "fwd", e["out_f"][0])
            ok = torch.equal(torch.remainder(e["out_f"][1] + y1, t), exact_mod_t(L_, "fwd", d["X"], d["W"], t))
            if "dx" in cfg.ops:
                dx1 = c.decrypt(L_, e["plan"], "dx", e["out_b"][0])
                ok &= torch.equal(torch.remainder(e["out_b"][1] + dx1, t), exact_mod_t(L_, "dx", d["dY"], d["W"], t))
            if "dw" in cfg.ops:
                dw1 = c.decrypt(L_, e["plan"], "dw", e["out_b"][2])
                cross = torch.remainder(exact_mod_t(L_, "dw", d["x1"], d["dy0"], t)
                                        + exact_mod_t(L_, "dw", d["x0"], d["dy1"], t), t)
                ok &= torch.equal(torch.remainder(e["out_b"][3] + dw1, t), cross)
            bit_exact &= bool(ok)

    # ------------------------------------------------------ roofline
    work = kernel_work([(e["ctx"], e["sz"], cfg.ops) for e in layers])
    per_step = {k: (stats[k][0] / args.steps, stats[k][1] / args.steps) for k in stats if stats[k][0]}
    dom = max(per_step, key=lambda k: per_step[k][1])
    launches, ms = per_step[dom]
    bytes_step, ops_step = work.get(dom, (0, 0))
    gbs = bytes_step / (ms / 1e3) / 1e9
    roof = {"kernel": dom, "launches_per_step": launches, "avg_launch_ms": ms / launches,
            "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
            "alu_work_per_step": ops_step}
    breakdown = {k: {"launches": v[0], "ms": round(v[1], 4),
                     "algo_GBps": round(work.get(k, (0, 0))[0] / (v[1] / 1e3) / 1e9, 1) if v[1] else None}
                 for k, v in sorted(per_step.items(), key=lambda kv: -kv[1][1])}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg.layers[0], args.cpu_seconds)

    first = layers[0]
    rec = {
        "metric": "encrypted linear-layer fwd+bwd products/sec at bit-exact",
        "value": round(value, 1),
        "unit": "products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": cfg.name, "N": first["ctx"].n, "L": first["ctx"].L,
                   "layers": [f"{e['layer'].kind} {e['layer'].c_in}->{e['layer'].c_out} "
                              f"{e['layer'].h}x{e['layer'].w} b{e['layer'].batch}" for e in layers],
                   "ops": list(cfg.ops), "products_per_step": int(products),
                   "plans": [{"fwd": e["plan"].fwd.astuple(), "dx": e["plan"].dx.astuple(),
                              "dw": e["plan"].dw.astuple()} for e in layers],
                   "launch": "one launch sequence per product, per layer"},
        "bit_exact": bit_exact,
        "wall_s_timed": round(wall, 3),
        "roofline": roof,
        "kernels": breakdown,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
