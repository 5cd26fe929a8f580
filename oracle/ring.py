"""Ring arithmetic in R_q = Z_q[X]/(X^N+1) per RNS limb (Sec. II.B, Sec. V).

`negacyclic_mul` is the schoolbook definition of the ring product; the
O(N^2) loops run in the plain-C helper cref.c (built by `build_cref`), and
`negacyclic_mul_py` is the same definition in Python for tiny N.
`ntt_def` is the definitional negacyclic transform A_k = a(psi^(2k+1)).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cref.c")
_LIB = os.path.join(_HERE, "_cref.so")
_lib = None


def build_cref(force=False):
    """Compile cref.c with gcc into oracle/_cref.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build_cref()
        lib = ctypes.CDLL(_LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_negacyclic_mul.argtypes = [u64p, u64p, u64p, ctypes.c_int64, ctypes.c_uint64]
        lib.oracle_negacyclic_coeffs.argtypes = [u64p, u64p, i64p, ctypes.c_int64, u64p, ctypes.c_int64,
                                                 ctypes.c_uint64]
        lib.oracle_ntt_def.argtypes = [u64p, u64p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64]
        _lib = lib
    return _lib


def _p(a, t=ctypes.c_uint64):
    return a.ctypes.data_as(ctypes.POINTER(t))


def residues(v, q):
    """Integers (any sign, Python or numpy) reduced into [0, q) as uint64."""
    return np.array([int(x) % q for x in np.asarray(v, dtype=object).ravel()], dtype=np.uint64).reshape(
        np.shape(v))


def negacyclic_mul(a, b, q):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    assert a.shape == b.shape and a.ndim == 1
    out = np.empty_like(a)
    _load().oracle_negacyclic_mul(_p(a), _p(b), _p(out), a.size, q)
    return out


def negacyclic_coeffs(a, b, q, idx):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(idx.size, dtype=np.uint64)
    _load().oracle_negacyclic_coeffs(_p(a), _p(b), _p(idx, ctypes.c_int64), idx.size, _p(out), a.size, q)
    return out


def negacyclic_mul_py(a, b, q):
    """Schoolbook negacyclic product in Python integers (tiny N only)."""
    n = len(a)
    out = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            if k < n:
                out[k] += int(a[i]) * int(b[j])
            else:
                out[k - n] -= int(a[i]) * int(b[j])
    return [x % q for x in out]


def ntt_def(a, q, psi):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.empty_like(a)
    _load().oracle_ntt_def(_p(a), _p(out), a.size, q, psi)
    return out


def intt_def(A, q, psi):
    """Inverse of ntt_def: a_j = N^-1 sum_k A_k psi^-(2k+1) j."""
    n = len(A)
    psi_inv = pow(psi, -1, q)
    n_inv = pow(n, -1, q)
    # a_j = n^-1 * psi^-j * sum_k A_k (psi^-2)^(jk): the definition, summed directly
    w2 = psi_inv * psi_inv % q
    out = []
    for j in range(n):
        s = 0
        wj = pow(w2, j, q)
        acc = 1
        for k in range(n):
            s += int(A[k]) * acc
            acc = acc * wj % q
        out.append(s % q * pow(psi_inv, j, q) % q * n_inv % q)
    return np.array(out, dtype=np.uint64)
