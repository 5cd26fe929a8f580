"""Pins for the App. A encodings, the BFV scheme and the protocol products."""
import itertools
from fractions import Fraction

import numpy as np
import pytest
import sympy
from sympy.ntheory.modular import crt as sympy_crt

from oracle import bfv
from oracle import encoding as E
from oracle import linear as LN
from oracle import params as PR
from oracle import protocol as PRT
from oracle import ring as RG
from workloads import conv, conv1d, fc, layer_tensors, CONFIGS, config_tensors

T = PR.T


def ring_mul_mod_t(a, b, n):
    """Negacyclic product over Z_t via the Z-coefficient product (np.convolve on Python ints)."""
    full = np.convolve(np.asarray(a).astype(object), np.asarray(b).astype(object))
    out = [0] * n
    for k, v in enumerate(full):
        out[k % n] += int(v) if k < n else -int(v)
    return [x % T for x in out]


# -------------------------------------------------------------- App. A formulas

def test_fc_indices_are_app_a_matmul_encoding():
    """For one whole tile the generic encodings reduce to App. A's matrix formulas:
    pi_v: v_jk -> x^(k*n_o*n_i + j), pi_W: W_ij -> x^(i*n_i + n_i - 1 - j),
    result at k*n_o*n_i + i*n_i + n_i - 1."""
    B, ni, no = 3, 5, 4
    layer = fc(B, ni, no)
    n = 64
    g = E.geometry(layer, "fwd")
    tl = E.Tile(B, no, ni, 1, 1, 1, 1)
    X = np.arange(1, B * ni + 1).reshape(B, ni)
    W = np.arange(100, 100 + no * ni).reshape(no, ni)
    pa = E.encode_a(E.virtual_a(layer, "fwd", X), g, tl, n, 0, 0, 0, 0, 0, 0)
    pk = E.encode_k(E.virtual_k(layer, "fwd", W), g, tl, n, 0, 0, 0, 0)
    for j, k in itertools.product(range(ni), range(B)):
        assert pa[k * no * ni + j] == X[k, j]
    for i, j in itertools.product(range(no), range(ni)):
        assert pk[i * ni + ni - 1 - j] == W[i, j]
    slots = dict((mrxy, s) for s, mrxy in E.out_slots(g, tl, 0, 0, 0, 0))
    for i, k in itertools.product(range(no), range(B)):
        assert slots[(k, i, 0, 0)] == k * no * ni + i * ni + ni - 1


def test_conv_indices_are_app_a_conv_encoding():
    """Whole-tile conv: index_v = b*c_o*c_i*h*w + c*h*w + i*w + j,
    index_W = O + c'*c_i*h*w - c*h*w - i*w - j with kernel indices in [s],
    index_y = b*c_o*c_i*h*w + O + c'*c_i*h*w + i*w + j for valid outputs."""
    B, ci, co, h, s = 2, 2, 3, 4, 2
    layer = conv(B, ci, co, h, k=s, pad=0)
    w = h
    n = B * co * ci * h * w
    g = E.geometry(layer, "fwd")
    tl = E.Tile(B, co, ci, h - s + 1, w - s + 1, s, s)
    O = (ci - 1) * h * w + (s - 1) * w + s - 1
    assert tl.offset == O
    X = np.arange(1, B * ci * h * w + 1).reshape(B, ci, h, w)
    W = np.arange(1, co * ci * s * s + 1).reshape(co, ci, s, s) + 1000
    pa = E.encode_a(E.virtual_a(layer, "fwd", X), g, tl, n, 0, 0, 0, 0, 0, 0)
    pk = E.encode_k(E.virtual_k(layer, "fwd", W), g, tl, n, 0, 0, 0, 0)
    for b, c, i, j in itertools.product(range(B), range(ci), range(h), range(w)):
        assert pa[b * co * ci * h * w + c * h * w + i * w + j] == X[b, c, i, j]
    for c2, c, i, j in itertools.product(range(co), range(ci), range(s), range(s)):
        assert pk[O + c2 * ci * h * w - c * h * w - i * w - j] == W[c2, c, i, j]
    slots = dict((mrxy, sl) for sl, mrxy in E.out_slots(g, tl, 0, 0, 0, 0))
    for b, c2, i, j in itertools.product(range(B), range(co), range(h - s + 1), range(w - s + 1)):
        assert slots[(b, c2, i, j)] == b * co * ci * h * w + O + c2 * ci * h * w + i * w + j


def _encoded_op(layer, op, tl, n, a_t, k_t):
    """Encode every tile, multiply in Z_t[X]/(X^n+1), sum contraction tiles, decode."""
    g = E.geometry(layer, op)
    E.check_tile(g, tl, n)
    c = E.counts(g, tl)
    A = E.virtual_a(layer, op, a_t)
    K = E.virtual_k(layer, op, k_t)
    out_v = np.full((g.M, g.R, g.OH, g.OW), -1, dtype=np.int64)
    for o, (mi, ri, oyi, oxi) in enumerate(E.out_tiles(c)):
        acc = [0] * n
        for ki, kyi, kxi in itertools.product(range(c.nK), range(c.nKY), range(c.nKX)):
            pa = E.encode_a(A, g, tl, n, mi, ki, oyi, oxi, kyi, kxi)
            pk = E.encode_k(K, g, tl, n, ri, ki, kyi, kxi)
            acc = [(x + y) % T for x, y in zip(acc, ring_mul_mod_t(pa, pk, n))]
        for slot, (m, r, y, x) in E.out_slots(g, tl, mi, ri, oyi, oxi):
            out_v[m, r, y, x] = acc[slot]
    assert (out_v >= 0).all()
    return E.from_virtual_out(layer, op, out_v)


ENC_CASES = [
    # (layer, op, tile, n) -- tight tiles (slots == n), ragged tails, spatial tiling of outputs and kernels
    (fc(3, 5, 4), "fwd", E.Tile(3, 4, 5, 1, 1, 1, 1), 60),
    (fc(3, 5, 4), "fwd", E.Tile(2, 3, 2, 1, 1, 1, 1), 16),
    (fc(3, 5, 4), "dx", E.Tile(2, 5, 3, 1, 1, 1, 1), 32),
    (fc(3, 5, 4), "dw", E.Tile(4, 3, 2, 1, 1, 1, 1), 24),
    (conv(2, 2, 3, 4, k=2, pad=0), "fwd", E.Tile(2, 3, 2, 3, 3, 2, 2), 192),
    (conv(2, 2, 3, 5, k=3, pad=1), "fwd", E.Tile(1, 2, 2, 2, 3, 3, 3), 128),
    (conv(2, 2, 3, 5, k=3, pad=1), "dx", E.Tile(2, 1, 3, 3, 2, 3, 3), 128),
    (conv(2, 2, 3, 5, k=3, pad=1), "dw", E.Tile(1, 2, 2, 3, 3, 2, 4), 128),
    (conv(1, 3, 2, 6, k=3, pad=1), "dw", E.Tile(3, 2, 1, 3, 3, 6, 6), 512),
    (conv(2, 1, 1, 5, k=3, pad=2), "fwd", E.Tile(2, 1, 1, 4, 7, 3, 3), 128),
    # Conv1d: one row, 1 x k kernel, padding along the length only
    (conv1d(2, 3, 2, 9, k=5, pad=0), "fwd", E.Tile(2, 2, 3, 1, 5, 1, 5), 128),
    (conv1d(2, 3, 2, 9, k=5, pad=2), "dx", E.Tile(1, 3, 2, 1, 4, 1, 3), 64),
    (conv1d(3, 2, 2, 8, k=3, pad=1), "dw", E.Tile(2, 2, 2, 1, 2, 1, 5), 64),
]


@pytest.mark.parametrize("case", range(len(ENC_CASES)))
def test_encoded_products_equal_plain_layers(case):
    """App. A's correctness claim: the decoded ring product is the layer's result."""
    layer, op, tl, n = ENC_CASES[case]
    rng = np.random.default_rng(case)
    X = rng.integers(0, T, layer.x_shape())
    W = rng.integers(0, T, layer.w_shape())
    dY = rng.integers(0, T, layer.y_shape())
    a_t, k_t = {"fwd": (X, W), "dx": (dY, W), "dw": (X, dY)}[op]
    ref = LN.layer_op(layer, op, a_t, k_t, T) if op != "dw" else LN.layer_op(layer, op, X, dY, T)
    assert (_encoded_op(layer, op, tl, n, a_t, k_t) == ref).all()


def test_tile_too_large_rejected():
    g = E.geometry(fc(3, 5, 4), "fwd")
    with pytest.raises(AssertionError):
        E.check_tile(g, E.Tile(3, 4, 5, 1, 1, 1, 1), 59)


# -------------------------------------------------------------- BFV

SMALL = PR.HEParams(256, PR.ntt_primes(60, 2), T)


def test_crt_and_scaling_exact():
    P = PR.make_params(12, 2, 50)
    rng = np.random.default_rng(5)
    vals = [int(x) for x in rng.integers(0, 2**62, 20)]
    limbs = [[v % q for v in vals] for q in P.moduli]
    ours = bfv.crt(limbs, P.moduli)
    for i, v in enumerate(vals):
        assert ours[i] == int(sympy_crt(P.moduli, [limbs[0][i], limbs[1][i]])[0]) == v % P.q
    ms = [0, 1, T - 1, (T - 1) // 2, 123456789]
    for m, d in zip(ms, bfv.delta_scale(ms, P)):
        exact = Fraction(P.q * m, T)
        assert abs(Fraction(d) - exact) < Fraction(1, 2)  # never a tie: q odd, t odd prime


def test_keygen_relation():
    P = SMALL
    k = bfv.keygen(P, 11)
    s = k["sk"]
    assert set(np.unique(s)) <= {-1, 0, 1}
    for l, q in enumerate(P.moduli):
        # p0 + p1*s = -e, small
        p1s = RG.negacyclic_mul(k["pk"][1, l], RG.residues(s, q), q)
        e = [(-(int(a) + int(b))) % q for a, b in zip(k["pk"][0, l], p1s)]
        e = [v - q if v > q // 2 else v for v in e]
        assert max(abs(v) for v in e) <= 21


@pytest.mark.parametrize("params", [SMALL, PR.make_params(12, 2, 50)])
def test_encrypt_decrypt_roundtrip(params):
    P = params
    k = bfv.keygen(P, 3)
    rng = np.random.default_rng(6)
    m = rng.integers(0, T, P.n)
    ct = bfv.encrypt(P, k["pk"], m, 3, 9, 1)
    assert (bfv.decrypt(P, k["sk"], ct) == m).all()
    # fresh noise bound: |e0 + p0-noise*u + e1*s| <= 21 + 21N + 21N, plus D(m) rounding
    assert bfv.noise(P, k["sk"], ct, m) <= 42 * P.n + 22


def test_plain_mult_decrypts_to_ring_product():
    """Dec(lift(w) * Enc(m)) = w * m in Z_t[X]/(X^N+1)."""
    P = SMALL
    k = bfv.keygen(P, 4)
    rng = np.random.default_rng(7)
    m = rng.integers(0, T, P.n)
    w = rng.integers(0, T, P.n)
    ct = bfv.encrypt(P, k["pk"], m, 4, 1, 1)
    acc = [[[0] * P.n for _ in range(P.num_limbs)] for _ in range(2)]
    acc = bfv.mul_plain_acc(P, acc, ct, w, T)
    prod = np.array(acc, dtype=np.uint64)
    assert list(bfv.decrypt(P, k["sk"], prod)) == ring_mul_mod_t(w, m, P.n)


def test_decrypt_rounding_exact():
    P = SMALL
    k = bfv.keygen(P, 8)
    rng = np.random.default_rng(8)
    ct = np.stack([np.stack([rng.integers(0, q, P.n, dtype=np.uint64) for q in P.moduli]) for _ in range(2)])
    x = bfv.phase(P, k["sk"], ct)
    got = bfv.decrypt(P, k["sk"], ct)
    for i in range(0, P.n, 17):
        f = Fraction(T * x[i], P.q)
        r = int(f + Fraction(1, 2)) if f >= 0 else None
        assert (r % T) == got[i]
        assert f - int(f) != Fraction(1, 2)


# -------------------------------------------------------------- protocols

def test_config1_forward_reconstructs():
    cfg = CONFIGS[1]
    layer = cfg.layers[0]
    P = PR.params_for(layer)
    ts = config_tensors(cfg)[0]
    assert (ts["x0"] == 0).all()
    keys = bfv.keygen(P, cfg.seed)
    plan = {"fwd": E.Tile(4, 10, 64, 1, 1, 1, 1)}
    y0, y1, cts = PRT.linear_fwd(P, keys, layer, plan, ts["x0"], ts["x1"], ts["W"], cfg.seed, 1)
    assert ((y0 + y1) % T == LN.layer_op(layer, "fwd", ts["X"], ts["W"], T)).all()
    # masked: the decryptor's share is not the result
    assert not (y1 == LN.layer_op(layer, "fwd", ts["X"], ts["W"], T)).all()
    for ct in cts:
        m = bfv.decrypt(P, keys["sk"], ct)
        assert bfv.noise(P, keys["sk"], ct, m) < P.delta // 2


@pytest.mark.slow
def test_small_conv_backward_reconstructs():
    layer = conv(2, 2, 3, 5, k=3, pad=1, log2_n=9, num_limbs=2, prime_bits=60)
    P = PR.params_for(layer)
    ts = layer_tensors(layer, 5)
    keys = bfv.keygen(P, 7)
    plan = {"fwd": E.Tile(2, 2, 2, 3, 5, 3, 3), "dx": E.Tile(1, 2, 3, 2, 5, 3, 3), "dw": E.Tile(2, 2, 1, 3, 3, 2, 5)}
    r = PRT.linear_bwd(P, keys, layer, plan, ts["x0"], ts["x1"], ts["dy0"], ts["dy1"], ts["W"], 7, 2)
    assert ((r["dx0"] + r["dx1"]) % T == LN.layer_op(layer, "dx", ts["dY"], ts["W"], T)).all()
    cross = (LN.layer_op(layer, "dw", ts["x1"], ts["dy0"], T) + LN.layer_op(layer, "dw", ts["x0"], ts["dy1"], T)) % T
    assert ((r["dw_mask"] + r["dw_dec"]) % T == cross).all()
    local = (LN.layer_op(layer, "dw", ts["x0"], ts["dy0"], T) + LN.layer_op(layer, "dw", ts["x1"], ts["dy1"], T)) % T
    assert ((r["dw_mask"] + r["dw_dec"] + local) % T == LN.layer_op(layer, "dw", ts["X"], ts["dY"], T)).all()


def test_sampled_coefficients_match_full_product():
    layer = fc(4, 6, 3, log2_n=8, num_limbs=2, prime_bits=60)
    P = PR.params_for(layer)
    ts = layer_tensors(layer, 9)
    keys = bfv.keygen(P, 9)
    plan = {"fwd": E.Tile(2, 3, 4, 1, 1, 1, 1)}
    cts = PRT.encrypt_operand(P, keys["pk"], layer, plan, PRT.OPERAND_X_FWD, ts["x1"], 9, 3)
    terms = [(("ct", cts), ("pt", ts["W"]))]
    full, y0 = PRT.mo_product(P, keys["pk"], layer, "fwd", plan["fwd"], terms, 9, 4, add_share=ts["x0"])
    idx = [0, 5, 17, 255]
    part, _ = PRT.mo_product(P, keys["pk"], layer, "fwd", plan["fwd"], terms, 9, 4, add_share=ts["x0"],
                             outs=[1], coeff_idx=idx)
    assert (part[1] == full[1][:, :, idx]).all()


def test_flood_beyond_budget_breaks_decryption():
    """Negative case: a flood of width Delta breaks decryption, the chosen width does not."""
    P = SMALL
    k = bfv.keygen(P, 2)
    m = np.arange(P.n) % T
    ct = bfv.encrypt(P, k["pk"], m, 2, 1, 1)
    big = ct.copy()
    for l, q in enumerate(P.moduli):
        big[0, l] = RG.residues([int(v) + P.delta // 2 + 1 for v in ct[0, l]], q)
    assert not (bfv.decrypt(P, k["sk"], big) == m).all()
    ok = ct.copy()
    for l, q in enumerate(P.moduli):
        ok[0, l] = RG.residues([int(v) + (1 << P.flood_bits) for v in ct[0, l]], q)
    assert (bfv.decrypt(P, k["sk"], ok) == m).all()


def test_output_is_rerandomised_flooded_and_masked():
    """c_out - lift(P)*ct_in must be a fresh encryption of -s: it decrypts to -s (mask),
    its second component is not small (re-randomised with pk), and its noise reaches the
    flood width (flooded)."""
    layer = fc(2, 8, 3, log2_n=8, num_limbs=2, prime_bits=60)
    P = PR.params_for(layer)
    ts = layer_tensors(layer, 12)
    keys = bfv.keygen(P, 12)
    tl = E.Tile(2, 3, 8, 1, 1, 1, 1)
    plan = {"fwd": tl}
    cts = PRT.encrypt_operand(P, keys["pk"], layer, plan, PRT.OPERAND_X_FWD, ts["x1"], 12, 3)
    out, y0 = PRT.mo_product(P, keys["pk"], layer, "fwd", tl, [(("ct", cts), ("pt", ts["W"]))], 12, 4)
    g = E.geometry(layer, "fwd")
    w_poly = E.encode_k(E.virtual_k(layer, "fwd", ts["W"]), g, tl, P.n, 0, 0, 0, 0)
    acc = [[[0] * P.n for _ in range(P.num_limbs)] for _ in range(2)]
    prod = np.array(bfv.mul_plain_acc(P, acc, cts[0], w_poly, T), dtype=np.uint64)
    d = np.empty_like(prod)
    for l, q in enumerate(P.moduli):
        for c in range(2):
            d[c, l] = RG.residues([int(a) - int(b) for a, b in zip(out[0][c, l], prod[c, l])], q)
    dec = bfv.decrypt(P, keys["sk"], d)
    # the model owner's share is the mask at the output slots
    for slot, (m, r, _, _) in E.out_slots(g, tl, 0, 0, 0, 0):
        assert (int(dec[slot]) + int(y0[m, r])) % T == 0
    assert int(d[1].max()) > P.moduli[0] // 4
    assert bfv.noise(P, keys["sk"], d, dec) > (1 << (P.flood_bits - 4))


def test_encrypt_eval_at_is_the_ntt_of_the_encryption():
    """Evaluating the ciphertext at psi^(2k+1) (the ring map to Z_q) equals
    entry k of the definitional negacyclic NTT of the full encryption."""
    P = SMALL
    k = bfv.keygen(P, 17)
    m = np.random.default_rng(18).integers(0, T, P.n)
    ct = bfv.encrypt(P, k["pk"], m, 17, 4, 9)
    ks = [0, 1, 77, P.n - 1]
    roots = [[pow(psi, 2 * kk + 1, q) for kk in ks] for q, psi in zip(P.moduli, P.psi)]
    ev = bfv.encrypt_eval_at(P, k["pk"], m, 17, 4, 9, roots)
    for l, (q, psi) in enumerate(zip(P.moduli, P.psi)):
        for c in range(2):
            full = RG.ntt_def(ct[c, l], q, psi)
            assert [int(full[kk]) for kk in ks] == ev[c][l]


def test_sampled_helpers_match_full_versions():
    P = SMALL
    k = bfv.keygen(P, 13)
    rng = np.random.default_rng(14)
    m = rng.integers(0, T, P.n)
    idx = [0, 3, 100, 255]
    ct = bfv.encrypt(P, k["pk"], m, 13, 2, 7)
    assert (bfv.encrypt_at(P, k["pk"], m, 13, 2, 7, idx) == ct[:, :, idx]).all()
    assert list(bfv.decrypt_at(P, k["sk"], ct, idx)) == list(bfv.decrypt(P, k["sk"], ct)[idx])
    for layer in (conv(2, 3, 2, 5, k=3, pad=1), fc(3, 6, 4), conv1d(2, 3, 2, 7, k=3, pad=1)):
        X = rng.integers(0, T, layer.x_shape())
        W = rng.integers(0, T, layer.w_shape())
        dY = rng.integers(0, T, layer.y_shape())
        for op, a, b in (("fwd", X, W), ("dx", dY, W), ("dw", X, dY)):
            full = LN.layer_op(layer, op, a, b, T)
            pts = [tuple(int(v) for v in np.unravel_index(i, full.shape)) for i in (0, full.size // 2, full.size - 1)]
            assert LN.layer_op_at(layer, op, a, b, T, pts) == [int(full[p]) for p in pts]
