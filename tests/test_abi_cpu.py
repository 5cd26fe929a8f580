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
