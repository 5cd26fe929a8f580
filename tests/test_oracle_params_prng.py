"""Pins for the oracle's parameters, Philox generator and samplers."""
import os

import numpy as np
import pytest
import sympy

from oracle import params as PR
from oracle import philox as PH
from oracle import sampling as S
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ params

@pytest.mark.parametrize("bits,count", [(50, 2), (60, 4)])
def test_ntt_primes_are_the_largest(bits, count):
    qs = PR.ntt_primes(bits, count)
    assert qs == sorted(qs, reverse=True)
    step = 1 << 15
    for q in qs:
        assert sympy.isprime(q) and q % step == 1 and q < (1 << bits)
    # no other prime = 1 mod 2^15 between consecutive entries or above the first
    top = ((1 << bits) - 1) // step * step + 1
    cand = top
    found = []
    while len(found) < count:
        if sympy.isprime(cand):
            found.append(cand)
        cand -= step
    assert found == qs


def test_plain_modulus():
    assert PR.T == sympy.prevprime(1 << 41) == workloads.T_PLAIN
    assert PR.T % 2 == 1


@pytest.mark.parametrize("q,n", [(17, 8), (97, 16), (193, 32), (257, 64), (7681, 256)])
def test_min_root_brute_force(q, n):
    # brute force over the whole field: smallest x with x^n = -1 and x^(2n) = 1
    brute = min(x for x in range(1, q) if pow(x, n, q) == q - 1)
    assert PR.min_primitive_2n_root(q, n) == brute


@pytest.mark.parametrize("log2_n,limbs,bits", [(12, 2, 50), (13, 3, 60), (14, 4, 60)])
def test_psi_is_primitive(log2_n, limbs, bits):
    P = PR.make_params(log2_n, limbs, bits)
    for q, psi in zip(P.moduli, P.psi):
        assert pow(psi, P.n, q) == q - 1
        assert sympy.n_order(psi, q) == 2 * P.n


def test_delta_and_flood_bits():
    for log2_n, limbs, bits in [(12, 2, 50), (13, 3, 60), (14, 4, 60)]:
        P = PR.make_params(log2_n, limbs, bits)
        assert P.delta == P.q // P.t
        assert 1 << (P.flood_bits + 3) <= P.delta < 1 << (P.flood_bits + 4)


# ------------------------------------------------------------------ philox

def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    for ctr, key, out in _kat():
        got = PH.philox4x64(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
        assert [int(x) for x in got] == out


def test_philox_matches_numpy():
    rng = np.random.default_rng(3)
    for _ in range(20):
        ctr = rng.integers(0, 2**63, 4, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 4, dtype=np.uint64)
        key = rng.integers(0, 2**63, 2, dtype=np.uint64)
        # numpy's Philox increments its counter before each block
        start = ctr.copy()
        start[0] = start[0] - np.uint64(1) if ctr[0] > 0 else start[0]
        if ctr[0] == 0:
            continue
        ref = np.random.Philox(key=key, counter=start).random_raw(4)
        assert [int(x) for x in PH.philox4x64(ctr, key)] == [int(x) for x in ref]


def test_stream_word_layout():
    w = PH.stream_words(5, 9, 77, 3, 2, 0, 12)
    for g in range(12):
        blk = PH.philox4x64(np.array([g // 4, 77, 3, 2], dtype=np.uint64), np.array([5, 9], dtype=np.uint64))
        assert int(w[g]) == int(blk[g % 4])
    assert [int(x) for x in PH.stream_words(5, 9, 77, 3, 2, 5, 4)] == [int(x) for x in w[5:9]]


# ------------------------------------------------------------------ samplers

def test_ternary_distribution_and_layout():
    n = 20000
    v = S.ternary(1, 2, 3, S.P_ENC_U, n)
    assert set(np.unique(v)) <= {-1, 0, 1}
    freq = np.bincount(v + 1) / n
    assert np.all(np.abs(freq - 1 / 3) < 0.02)
    w = PH.stream_words(1, 2, 3, S.P_ENC_U, 0, 0, 4)
    assert v[0] == (int(w[0]) & 0xFFFFFFFF) % 3 - 1
    assert v[1] == (int(w[0]) >> 32) % 3 - 1
    assert v[5] == (int(w[2]) >> 32) % 3 - 1
    assert list(v[[7, 100, 999]]) == S.ternary_at(1, 2, 3, S.P_ENC_U, [7, 100, 999])


def test_cbd21():
    n = 20000
    v = S.cbd21(4, 5, 6, S.P_ENC_E0, n)
    assert v.min() >= -21 and v.max() <= 21
    assert abs(v.mean()) < 0.1 and abs(v.var() - 10.5) < 0.5
    w = int(PH.stream_words(4, 5, 6, S.P_ENC_E0, 0, 17, 1)[0])
    assert v[17] == bin(w & (2**21 - 1)).count("1") - bin((w >> 21) & (2**21 - 1)).count("1")
    assert list(v[[3, 17, 4000]]) == S.cbd21_at(4, 5, 6, S.P_ENC_E0, [3, 17, 4000])


def test_uniform_flood_mask():
    q = PR.ntt_primes(60, 1)[0]
    u = S.uniform_mod(1, 1, 0, S.P_PK_A, 2, 500, q)
    assert int(u.max()) < q
    w = PH.stream_words(1, 1, 0, S.P_PK_A, 2, 0, 2)
    assert int(u[0]) == (int(w[0]) + (int(w[1]) << 64)) % q
    for fb in (55, 136, 196):
        f = S.flood(2, 3, 4, 300, fb)
        assert all(-(1 << fb) <= x < (1 << fb) for x in f)
        assert max(f) > (1 << fb) // 2 and min(f) < -(1 << fb) // 2
        assert S.flood(2, 3, 4, 300, fb, [0, 7, 299]) == [f[0], f[7], f[299]]
    t = PR.T
    m = S.mask_mod_t(2, 3, 4, 400, t)
    assert all(0 <= x < t for x in m)
    assert S.mask_mod_t(2, 3, 4, 400, t, [1, 399]) == [m[1], m[399]]


def test_additive_shares():
    """Shares of Sec. II.C: s0 from raw stream words (purpose P_SHARE), s0 + s1 = v
    mod t, s0 spread over Z_t, and a different object gives a different draw."""
    t = PR.T
    rng = np.random.default_rng(3)
    v = rng.integers(0, t, 5000, dtype=np.int64)
    s0, s1 = S.shares_mod_t(7, 8, 9, v, t)
    assert ((s0 >= 0) & (s0 < t) & (s1 >= 0) & (s1 < t)).all()
    assert (np.mod(s0 + s1, t) == v).all()
    w = PH.stream_words(7, 8, 9, S.P_SHARE, 0, 2 * 4321, 2)
    assert int(s0[4321]) == (int(w[0]) + (int(w[1]) << 64)) % t
    assert abs(s0.astype(np.float64).mean() / t - 0.5) < 0.02
    other, _ = S.shares_mod_t(7, 8, 10, v, t)
    assert not (other == s0).any()
