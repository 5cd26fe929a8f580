"""Helpers shared by the GPU parity tests: moving tensors between the HIP
path and numpy, and the oracle's keys for a context's parameters."""
import numpy as np
import torch

from oracle import bfv
from oracle import params as PR


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
