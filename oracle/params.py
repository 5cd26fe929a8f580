"""HE parameters: RNS primes, plaintext modulus, negacyclic roots, scaling.

The paper fixes only the shape of the parameter set: BFV with a power-of-two
degree N, plaintext modulus t and a ciphertext modulus q split into RNS
components q_i < 2^64 (Sec. II.B, Sec. V "RNS Decomposition"); its evaluation
uses three ~60-bit components for N = 8192 (Sec. VI.B).  Readings:

* each q_l is among the largest primes below 2^bits with q_l = 1 mod 2^15, so
  every N <= 16384 has a primitive 2N-th root of unity mod q_l; listed in
  descending order;
* t is the largest prime below 2^41 (odd, so the centred lift of Z_t has no
  tie);
* psi_l is the smallest primitive 2N-th root of unity mod q_l, and the
  negacyclic NTT evaluates at psi^(2k+1), k in natural order;
* Delta = floor(q/t); the flooding width is fb = floor(log2 Delta) - 3, so
  the flood never exceeds Delta/8.
"""
import functools
from dataclasses import dataclass
from typing import List

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin (the bases above decide all n < 3.3e24)."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def ntt_primes(bits: int, count: int, two_power: int = 15) -> List[int]:
    """The `count` largest primes q < 2^bits with q = 1 mod 2^two_power."""
    step = 1 << two_power
    q = ((1 << bits) - 1) // step * step + 1
    if q >= (1 << bits):
        q -= step
    out = []
    while len(out) < count:
        if is_prime(q):
            out.append(q)
        q -= step
    return out


def prev_prime(n: int) -> int:
    """Largest prime strictly below n."""
    k = n - 1
    while not is_prime(k):
        k -= 1
    return k


@functools.lru_cache(maxsize=None)
def min_primitive_2n_root(q: int, n: int) -> int:
    """Smallest x in [1, q) with x^n = -1 mod q (a primitive 2n-th root, n a power of 2).

    A primitive 2n-th root psi is found by raising small bases to (q-1)/(2n);
    the set of all of them is {psi^(2i+1)}, and the smallest is returned.
    """
    assert (q - 1) % (2 * n) == 0
    psi = None
    for g in range(2, 1 << 20):
        cand = pow(g, (q - 1) // (2 * n), q)
        if pow(cand, n, q) == q - 1:
            psi = cand
            break
    assert psi is not None
    best, sq, cur = psi, psi * psi % q, psi
    for _ in range(n):
        if cur < best:
            best = cur
        cur = cur * sq % q
    return best


@dataclass
class HEParams:
    n: int
    moduli: List[int]
    t: int

    @property
    def num_limbs(self):
        return len(self.moduli)

    @property
    def q(self):
        out = 1
        for m in self.moduli:
            out *= m
        return out

    @property
    def delta(self):
        return self.q // self.t

    @property
    def flood_bits(self):
        return self.delta.bit_length() - 1 - 3

    @property
    def psi(self):
        return [min_primitive_2n_root(q, self.n) for q in self.moduli]


def plain_modulus() -> int:
    """t: the largest prime below 2^41."""
    return prev_prime(1 << 41)


T = plain_modulus()


def make_params(log2_n: int, num_limbs: int, prime_bits: int, t: int = T) -> HEParams:
    return HEParams(1 << log2_n, ntt_primes(prime_bits, num_limbs), t)


def params_for(layer) -> HEParams:
    return make_params(layer.log2_n, layer.num_limbs, layer.prime_bits)
