"""RNS-BFV over R_{q,N} (Sec. II.B; RNS form of Sec. V), written from the
scheme's definition.  The paper names BFV "with SEAL's details" but states no
variant; readings:

* KeyGen: s ternary; a uniform in R_q (independently per RNS limb, which is
  uniform over R_q by the CRT); e an error;  pk = (-(a*s + e), a).
* Encrypt (public key, the model owner holds pk): u ternary, e0, e1 errors,
      ct = (p0*u + e0 + D(m),  p1*u + e1),
  with the exact scaling D(m) = round(q*m/t) (not floor(q/t)*m).
* Plaintext multiplicands are lifted centred: w in [0, t) becomes w - t when
  w > (t-1)/2.
* Decrypt: x = [c0 + c1*s]_q (composed from the RNS limbs by the CRT), then
  m = round(t*x/q) mod t.  q is odd and coprime to t, so round(q*m/t) and
  round(t*x/q) never meet a tie.
"""
import numpy as np

from . import sampling as S
from .ring import negacyclic_mul, residues


def crt(limbs, moduli):
    """Integers in [0, q) from their residues (limbs: L sequences of N residues)."""
    q = 1
    for m in moduli:
        q *= m
    out = [0] * len(limbs[0])
    for l, m in enumerate(moduli):
        Ql = q // m
        c = Ql * pow(Ql, -1, m)
        for i, v in enumerate(limbs[l]):
            out[i] += int(v) * c
    return [v % q for v in out]


def delta_scale(m, P):
    """D(m) = round(q*m/t) for m in [0, t), as Python ints."""
    q, t = P.q, P.t
    return [(2 * q * int(v) + t) // (2 * t) for v in m]


def lift_centred(w, t):
    w = int(w)
    return w - t if w > (t - 1) // 2 else w


def keygen(P, seed):
    n, nonce = P.n, S.KEYGEN_NONCE
    s = S.ternary(seed, nonce, 0, S.P_SK, n)
    e = S.cbd21(seed, nonce, 0, S.P_PK_E, n)
    pk = np.empty((2, P.num_limbs, n), dtype=np.uint64)
    for l, q in enumerate(P.moduli):
        a = S.uniform_mod(seed, nonce, 0, S.P_PK_A, l, n, q)
        sa = negacyclic_mul(a, residues(s, q), q)
        pk[0, l] = residues([-(int(x) + int(y)) for x, y in zip(sa, e)], q)
        pk[1, l] = a
    return dict(sk=s, pk=pk)


def encrypt(P, pk, m, seed, nonce, obj):
    """Encrypt the Z_t coefficient vector m (length N) under pk."""
    n = P.n
    u = S.ternary(seed, nonce, obj, S.P_ENC_U, n)
    e = (S.cbd21(seed, nonce, obj, S.P_ENC_E0, n), S.cbd21(seed, nonce, obj, S.P_ENC_E1, n))
    dm = delta_scale(m, P)
    ct = np.empty((2, P.num_limbs, n), dtype=np.uint64)
    for l, q in enumerate(P.moduli):
        ul = residues(u, q)
        for c in range(2):
            pu = negacyclic_mul(pk[c, l], ul, q)
            add = [int(x) + int(y) + (dm[i] if c == 0 else 0) for i, (x, y) in enumerate(zip(pu, e[c]))]
            ct[c, l] = residues(add, q)
    return ct


def phase(P, sk, ct):
    """[c0 + c1*s]_q as Python ints."""
    limbs = []
    for l, q in enumerate(P.moduli):
        c1s = negacyclic_mul(ct[1, l], residues(sk, q), q)
        limbs.append([(int(a) + int(b)) % q for a, b in zip(ct[0, l], c1s)])
    return crt(limbs, P.moduli)


def decrypt(P, sk, ct):
    q, t = P.q, P.t
    x = phase(P, sk, ct)
    return np.array([((2 * t * v + q) // (2 * q)) % t for v in x], dtype=np.int64)


def noise(P, sk, ct, m):
    """Max |[c0 + c1*s - D(m)]_q| (centred) over the coefficients."""
    q = P.q
    x = phase(P, sk, ct)
    dm = delta_scale(m, P)
    worst = 0
    for a, b in zip(x, dm):
        v = (a - b) % q
        v = v - q if v > q // 2 else v
        worst = max(worst, abs(v))
    return worst


def add_plain(P, ct, m):
    """ct + D(m) on c0 (the plaintext-ciphertext addition of Alg. 1)."""
    dm = delta_scale(m, P)
    out = ct.copy()
    for l, q in enumerate(P.moduli):
        out[0, l] = residues([int(a) + b for a, b in zip(ct[0, l], dm)], q)
    return out


def mul_plain_acc(P, acc, ct, w, t):
    """acc += lift(w) * ct (per limb, both components); acc holds Python-int lists."""
    for l, q in enumerate(P.moduli):
        wl = residues([lift_centred(v, t) for v in w], q)
        for c in range(2):
            pr = negacyclic_mul(wl, ct[c, l], q)
            acc[c][l] = [(a + int(b)) % q for a, b in zip(acc[c][l], pr)]
    return acc


def encrypt_at(P, pk, m, seed, nonce, obj, idx):
    """Coefficients idx of encrypt(P, pk, m, ...) (each one an O(N) sum)."""
    from .ring import negacyclic_coeffs
    n = P.n
    u = S.ternary(seed, nonce, obj, S.P_ENC_U, n)
    e = (S.cbd21_at(seed, nonce, obj, S.P_ENC_E0, idx), S.cbd21_at(seed, nonce, obj, S.P_ENC_E1, idx))
    dm = delta_scale([m[i] for i in idx], P)
    out = np.empty((2, P.num_limbs, len(idx)), dtype=np.uint64)
    for l, q in enumerate(P.moduli):
        ul = residues(u, q)
        for c in range(2):
            pu = negacyclic_coeffs(pk[c, l], ul, q, idx)
            out[c, l] = residues([int(x) + int(y) + (dm[i] if c == 0 else 0) for i, (x, y) in enumerate(zip(pu, e[c]))],
                                 q)
    return out


def decrypt_at(P, sk, ct, idx):
    """Coefficients idx of decrypt(P, sk, ct)."""
    from .ring import negacyclic_coeffs
    limbs = []
    for l, q in enumerate(P.moduli):
        c1s = negacyclic_coeffs(ct[1, l], residues(sk, q), q, idx)
        limbs.append([(int(ct[0, l][i]) + int(b)) % q for i, b in zip(idx, c1s)])
    x = crt(limbs, P.moduli)
    q, t = P.q, P.t
    return np.array([((2 * t * v + q) // (2 * q)) % t for v in x], dtype=np.int64)


def _powers(x, n, q):
    out = [1] * n
    for j in range(1, n):
        out[j] = out[j - 1] * x % q
    return np.array(out, dtype=object)


def encrypt_eval_at(P, pk, m, seed, nonce, obj, roots):
    """The ciphertext encrypt(P, pk, m, seed, nonce, obj) evaluated at the given
    roots of X^N + 1 (roots[l]: a list of points mod q_l).  Evaluation at such a
    root is a ring map of Z_q[X]/(X^N + 1), so each entry is
    pk_c(x) u(x) + e_c(x) (+ round(q m / t)(x) on c = 0), mod q_l.  At
    x = psi^(2k+1) this is entry k of the negacyclic NTT.  Returns
    [2][L][len(roots[l])] Python integers."""
    n = P.n
    u = S.ternary(seed, nonce, obj, S.P_ENC_U, n)
    e = (S.cbd21(seed, nonce, obj, S.P_ENC_E0, n), S.cbd21(seed, nonce, obj, S.P_ENC_E1, n))
    dm = delta_scale(m, P)
    out = [[None] * P.num_limbs for _ in range(2)]
    for l, q in enumerate(P.moduli):
        uo = np.array([int(v) % q for v in u], dtype=object)
        e0 = np.array([int(v) % q for v in e[0]], dtype=object)
        e1 = np.array([int(v) % q for v in e[1]], dtype=object)
        dmo = np.array([int(v) % q for v in dm], dtype=object)
        pk0 = np.array([int(v) for v in pk[0, l]], dtype=object)
        pk1 = np.array([int(v) for v in pk[1, l]], dtype=object)
        r0, r1 = [], []
        for x in roots[l]:
            pw = _powers(int(x), n, q)
            ux = int(np.dot(uo, pw)) % q
            r0.append((int(np.dot(pk0, pw)) * ux + int(np.dot(e0, pw)) + int(np.dot(dmo, pw))) % q)
            r1.append((int(np.dot(pk1, pw)) * ux + int(np.dot(e1, pw))) % q)
        out[0][l], out[1][l] = r0, r1
    return out
