"""Helpers shared by the GPU parity tests: moving tensors between the HIP
path and numpy, and the oracle's keys for a context's parameters."""
import numpy as np
import torch

from oracle import bfv
from oracle import params as PR
from oracle import ring as RG


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.int64))).cuda()


def host_u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


def host_i64(t):
    return t.detach().cpu().numpy()


def oracle_params(ctx):
    return PR.HEParams(ctx.n, list(ctx.primes), ctx.t)


_keys = {}


def oracle_keys(ctx):
    k = (ctx.n, tuple(ctx.primes), ctx.t, ctx.seed)
    if k not in _keys:
        _keys[k] = bfv.keygen(oracle_params(ctx), ctx.seed)
    return _keys[k]


def cts_list(arr):
    """uint64 [n][2][L][N] -> list of per-ciphertext arrays."""
    return [arr[i] for i in range(arr.shape[0])]


def bitrev(i, bits):
    return int(format(i, f"0{bits}b")[::-1], 2)


def ntt_order_roots(P, idx):
    """Per limb, the points psi^(2 rev(i) + 1) that NTT-domain entries idx of the
    library's transform order hold (its documented order)."""
    bits = P.n.bit_length() - 1
    return [[pow(psi, 2 * bitrev(i, bits) + 1, q) for i in idx] for q, psi in zip(P.moduli, P.psi)]


def split30(a):
    """The library's split form of residues v < 2^60: (v mod 2^30) + 2^32 floor(v / 2^30)."""
    a = np.asarray(a, dtype=np.uint64)
    return (a & np.uint64(0x3FFFFFFF)) | ((a >> np.uint64(30)) << np.uint64(32))


def unsplit30(a):
    """Residues from the library's split form."""
    a = np.asarray(a, dtype=np.uint64)
    return (a & np.uint64(0xFFFFFFFF)) | ((a >> np.uint64(32)) << np.uint64(30))


def oracle_ct_ntt(P, ct):
    """An oracle ciphertext [2][L][N] (coefficient domain) in the form the
    library's encryption produces: the definitional transform of each component
    and limb, entry i = evaluation at psi^(2 rev(i) + 1), each residue in split
    form."""
    bits = P.n.bit_length() - 1
    perm = np.array([bitrev(i, bits) for i in range(P.n)])
    out = np.empty_like(np.asarray(ct, dtype=np.uint64))
    for c in range(2):
        for l, (q, psi) in enumerate(zip(P.moduli, P.psi)):
            out[c, l] = RG.ntt_def(ct[c][l], q, psi)[perm]
    return split30(out)
