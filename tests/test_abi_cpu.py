"""Host-only checks of the C-ABI library: it loads without a GPU and exports
every entry point include/pencil.h declares; host-side validation and the
planner run without touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pencil.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pencil_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_abi():
    names = declared_functions()
    for n in ("pencil_ctx_create", "pencil_encrypt", "pencil_linear_fwd", "pencil_linear_bwd", "pencil_decrypt"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2403_11166_amd import _abi
    lib = _abi.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _abi.SIGNATURES, f"{name} has no ctypes signature"


def test_null_arguments_are_rejected_on_the_host():
    from paper_2403_11166_amd import _abi
    lib = _abi.load()
    h = ctypes.c_void_p()
    assert lib.pencil_ctx_create(None, ctypes.byref(h)) == _abi.PENCIL_EINVAL
    assert b"NULL" in lib.pencil_last_error(None)
    p = _abi.Params()
    p.log2_n, p.num_limbs, p.prime_bits = 9, 2, 60
    assert lib.pencil_ctx_create(ctypes.byref(p), ctypes.byref(h)) == _abi.PENCIL_EINVAL
    assert b"log2_n" in lib.pencil_last_error(None)
    p.log2_n, p.num_limbs = 12, 5
    assert lib.pencil_ctx_create(ctypes.byref(p), ctypes.byref(h)) == _abi.PENCIL_EINVAL
    p.num_limbs, p.prime_bits = 2, 70
    assert lib.pencil_ctx_create(ctypes.byref(p), ctypes.byref(h)) == _abi.PENCIL_EINVAL
    # a prime that is not 1 mod 2N
    p.prime_bits = 60
    p.primes[0], p.primes[1] = 1152921504606846883, 1152921504606748673
    assert lib.pencil_ctx_create(ctypes.byref(p), ctypes.byref(h)) == _abi.PENCIL_EINVAL
    assert b"prime" in lib.pencil_last_error(None)
    # a composite t
    p.primes[0] = p.primes[1] = 0
    p.t = 2199023255530
    assert lib.pencil_ctx_create(ctypes.byref(p), ctypes.byref(h)) == _abi.PENCIL_EINVAL
    assert lib.pencil_encrypt(None, None, None, 0, None, None, None, 0, None) == _abi.PENCIL_EINVAL
    assert lib.pencil_linear_fwd(None, None, None, *([None] * 7), 0, None) == _abi.PENCIL_EINVAL
    assert lib.pencil_ctx_destroy(None) == _abi.PENCIL_OK


def test_planner_tiles_fit_and_cover_every_workload_layer():
    """The host-only planner returns, for every layer of every workload, tiles that
    fit N slots and a valid multiply-accumulate schedule; it is deterministic."""
    from oracle import encoding as E
    from paper_2403_11166_amd import _abi
    from paper_2403_11166_amd.api import layer_struct
    from workloads import CONFIGS, small_cases
    lib = _abi.load()
    layers = [l for c in CONFIGS.values() for l in c.layers] + small_cases()
    for layer in layers:
        plans = []
        for _ in range(2):
            p = _abi.Plan()
            assert lib.pencil_plan_auto_n(layer.log2_n, ctypes.byref(layer_struct(layer)), ctypes.byref(p)) == 0
            plans.append((p.fwd.astuple(), p.dx.astuple(), p.dw.astuple(), tuple(p.sched)))
        assert plans[0] == plans[1]
        for op, t in zip(("fwd", "dx", "dw"), plans[0][:3]):
            E.check_tile(E.geometry(layer, op), E.Tile(*t), 1 << layer.log2_n)
        assert all(0 <= v < 9 for v in plans[0][3])


def test_planner_rejects_unsupported_layers():
    from paper_2403_11166_amd import _abi
    lib = _abi.load()
    p = _abi.Plan()
    bad = _abi.Layer(1, 2, 3, 4, 8, 8, 3, 3)  # pad > k - 1
    assert lib.pencil_plan_auto_n(13, ctypes.byref(bad), ctypes.byref(p)) == _abi.PENCIL_EUNSUPPORTED
    bad = _abi.Layer(0, 2, 3, 4, 2, 1, 1, 0)  # fc with h != 1
    assert lib.pencil_plan_auto_n(13, ctypes.byref(bad), ctypes.byref(p)) == _abi.PENCIL_EINVAL
    ok = _abi.Layer(0, 2, 3, 4, 1, 1, 1, 0)
    assert lib.pencil_plan_auto_n(9, ctypes.byref(ok), ctypes.byref(p)) == _abi.PENCIL_EINVAL


def test_stride_map_and_conv1d_planning():
    """Strided layers map to their space-to-depth stride-1 equivalents (host
    only); product entry points refuse strided layers; Conv1d layers and the
    equivalents plan into tiles that fit N slots."""
    from oracle import encoding as E
    from paper_2403_11166_amd import _abi
    from paper_2403_11166_amd.api import layer_struct
    from workloads import LayerSpec, conv, conv1d
    lib = _abi.load()
    cases = [(conv(64, 1, 5, 28, k=5, pad=2, stride=2), (1, 64, 4, 5, 16, 16, 3, 0, 1)),
             (conv(2, 3, 2, 11, k=4, pad=1, stride=3), (1, 2, 27, 2, 5, 5, 2, 0, 1)),
             (conv1d(2, 3, 4, 14, k=5, pad=2, stride=2), (2, 2, 6, 4, 1, 9, 3, 0, 1))]
    for layer, want in cases:
        e = _abi.Layer()
        assert lib.pencil_stride_map(ctypes.byref(layer_struct(layer)), ctypes.byref(e)) == 0
        got = tuple(getattr(e, f) for f, _ in _abi.Layer._fields_)
        assert got == want, (layer, got)
        p = _abi.Plan()
        assert lib.pencil_plan_auto_n(13, ctypes.byref(layer_struct(layer)), ctypes.byref(p)) == _abi.PENCIL_EUNSUPPORTED
        assert b"stride" in lib.pencil_last_error(None)
        kind = {0: "fc", 1: "conv", 2: "conv1d"}[e.kind]
        eq = LayerSpec(kind, e.batch, e.c_in, e.c_out, e.h, e.w, e.k, e.pad)
        assert eq.y_shape() == layer.y_shape()
        assert lib.pencil_plan_auto_n(13, ctypes.byref(layer_struct(eq)), ctypes.byref(p)) == 0
        for op, t in zip(("fwd", "dx", "dw"), (p.fwd, p.dx, p.dw)):
            E.check_tile(E.geometry(eq, op), E.Tile(*t.astuple()), 1 << 13)
    for layer in (conv1d(64, 256, 128, 64, k=5), conv1d(64, 128, 128, 30, k=5), conv1d(3, 4, 2, 9, k=3, pad=1)):
        p = _abi.Plan()
        assert lib.pencil_plan_auto_n(13, ctypes.byref(layer_struct(layer)), ctypes.byref(p)) == 0
        for op, t in zip(("fwd", "dx", "dw"), (p.fwd, p.dx, p.dw)):
            E.check_tile(E.geometry(layer, op), E.Tile(*t.astuple()), 1 << 13)
    bad = conv1d(2, 3, 4, 14, k=5, pad=2)
    s = layer_struct(bad)
    s.h = 2
    assert lib.pencil_plan_auto_n(13, ctypes.byref(s), ctypes.byref(_abi.Plan())) == _abi.PENCIL_EINVAL
