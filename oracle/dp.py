"""What the parties add to Alg. 2 to finish a training step's weight update
(Sec. III.B.2): the bias gradient and the data owner's differential-privacy
perturbation.  Test infrastructure only, like every module of the oracle.

Bias gradient.  For an FC layer dY is B x n_o and the bias gradient sums it
over the batch; for a convolution it sums dY (B x c_o x h' x w') over the
batch and the output rows and columns.  Each party sums its own share mod t;
the DO sends its sum to the MO.

Perturbation.  The DO adds e ~ N(0, sigma^2 C^2 / B) to each entry of its
decrypted weight-gradient share and of its bias-gradient share (DPSGD with
clipping bound C).  In fixed point the added value is floor(std * z) mod t,
with std = sigma C / sqrt(B) * 2^scale given in fixed-point units (the scale is
2f for dW, a product of two f-bit operands, and f for db).

Reading (the paper names no sampler; this one makes the two sides agree bit
for bit because every step is an IEEE double operation with a single rounding,
evaluated in a fixed order):
  * stream: key (seed, nonce), counter (block, obj, P_DP, 0); entry i uses
    stream words a = 2 (i div 2) and a + 1;
  * Box-Muller: u1 = ((w_a >> 11) + 1) 2^-53 in (0, 1], the 53-bit integer
    b = w_{a+1} >> 11 gives u2 = b 2^-53 in [0, 1);
    r = sqrt(-2 ln u1); z = r cos(2 pi u2) for even i, r sin(2 pi u2) for odd i;
  * ln u for u = k 2^-53 (k in [1, 2^53]): u = m 2^e with m in [1/sqrt 2, sqrt 2)
    (m from the bit length of k, halved range folded by doubling);
    s = (m - 1) / (m + 1); ln m = 2 s sum_{j<=11} s^(2j) / (2j + 1) (the atanh
    series, Horner in s^2); ln u = e ln2 + ln m;
  * cos and sin of 2 pi b 2^-53: quadrant q = round(b / 2^51) (integer), the
    exact remainder d = b - q 2^51 gives theta = (d 2^-53) 2 pi in
    [-pi/4, pi/4]; Taylor series to theta^22 (cos) and theta^23 (sin), Horner
    in theta^2, coefficients built as c_0 = 1, c_j = c_{j-1} / -((2j-1) 2j)
    (cos) and c_0 = 1, c_j = c_{j-1} / -(2j (2j+1)) (sin); then rotated by q.
The largest |z| is sqrt(2 * 53 ln 2) ~ 8.57 (u1 = 2^-53): tails beyond 8.57
sigma are cut.
"""
import numpy as np

from . import linear as LIN
from .philox import stream_words

P_DP = 48

SQRT_HALF = 0.7071067811865476
LN2 = 0.6931471805599453
TWO_PI = 6.283185307179586
LOG_TERMS = 12      # s^0 .. s^22 inside the bracket
TRIG_TERMS = 12     # theta^0 .. theta^22 (cos), theta^1 .. theta^23 (sin)


# ------------------------------------------------------------- bias gradient

def bias_grad(layer, dy, t):
    """Sum of dY over every axis but the channel axis (axis 1), mod t, exact."""
    dy = np.asarray(dy, dtype=np.int64)
    axes = tuple(a for a in range(dy.ndim) if a != 1)
    acc = dy.astype(object).sum(axis=axes)
    return np.array([int(v) % t for v in acc], dtype=np.int64)


# ------------------------------------------------------ Gaussian from Philox

def _series_log_coeffs():
    return [1.0 / float(2 * j + 1) for j in range(LOG_TERMS)]


def _series_trig_coeffs():
    cc, cs = [1.0], [1.0]
    for j in range(1, TRIG_TERMS):
        cc.append(cc[-1] / -float((2 * j - 1) * (2 * j)))
        cs.append(cs[-1] / -float((2 * j) * (2 * j + 1)))
    return cc, cs


def log_u(k):
    """ln(k 2^-53) for integers k in [1, 2^53] (uint64 array) as float64."""
    kf = np.asarray(k, dtype=np.uint64).astype(np.float64)       # exact: k <= 2^53
    m, bl = np.frexp(kf)                                         # kf = m 2^bl, m in [0.5, 1)
    e = bl.astype(np.int64) - 53
    low = m < SQRT_HALF
    m = np.where(low, m * 2.0, m)
    e = np.where(low, e - 1, e)
    s = (m - 1.0) / (m + 1.0)
    s2 = s * s
    c = _series_log_coeffs()
    p = np.full_like(s, c[-1])
    for j in range(LOG_TERMS - 2, -1, -1):
        p = p * s2 + c[j]
    lnm = (s * p) * 2.0
    return e.astype(np.float64) * LN2 + lnm


def cos_sin_turns(b):
    """(cos, sin) of 2 pi b 2^-53 for integers b in [0, 2^53) (uint64 array)."""
    b = np.asarray(b, dtype=np.uint64).astype(np.int64)
    q = (b + (1 << 50)) >> 51                                    # 0..4
    d = b - (q << 51)                                            # |d| <= 2^50
    theta = (d.astype(np.float64) * 2.0 ** -53) * TWO_PI
    t2 = theta * theta
    cc, cs = _series_trig_coeffs()
    pc = np.full_like(theta, cc[-1])
    ps = np.full_like(theta, cs[-1])
    for j in range(TRIG_TERMS - 2, -1, -1):
        pc = pc * t2 + cc[j]
        ps = ps * t2 + cs[j]
    c, s = pc, theta * ps
    qm = q & 3
    cos = np.select([qm == 0, qm == 1, qm == 2], [c, -s, -c], s)
    sin = np.select([qm == 0, qm == 1, qm == 2], [s, c, -s], -c)
    return cos, sin


def gaussian(seed, nonce, obj, n):
    """Standard normal draws z_0 .. z_{n-1} of the stream (obj, P_DP)."""
    if n <= 0:
        return np.zeros(0, dtype=np.float64)
    npair = (n + 1) // 2
    w = stream_words(seed, nonce, obj, P_DP, 0, 0, 2 * npair)
    k = (w[0::2] >> np.uint64(11)) + np.uint64(1)
    b = w[1::2] >> np.uint64(11)
    r = np.sqrt(log_u(k) * -2.0)
    cos, sin = cos_sin_turns(b)
    z = np.empty(2 * npair, dtype=np.float64)
    z[0::2] = r * cos
    z[1::2] = r * sin
    return z[:n]


def noise(seed, nonce, obj, n, std):
    """floor(std * z_i) as int64 (the perturbation in fixed-point units)."""
    z = gaussian(seed, nonce, obj, n)
    return np.floor(z * float(std)).astype(np.int64)


def add_noise(x, seed, nonce, obj, std, t):
    """x + floor(std * z) mod t, entry by entry in x's C order."""
    x = np.asarray(x, dtype=np.int64)
    e = noise(seed, nonce, obj, x.size, std).reshape(x.shape)
    return np.mod(x.astype(object) + e.astype(object), t).astype(np.int64)


# --------------------------------------------- the weight update (Alg. 2 end)

OBJ_DW = 0
OBJ_DB = 1


def weight_update(layer, dw_mask, dw_dec, x0, x1, dy0, dy1, seed, nonce, std_w, std_b, t):
    """The end of Alg. 2 plus the bias gradient, with the DO's perturbation.

    DO: dW~ = dw_dec + <dY>_1 o <X>_1 + e_W (the decrypted cross-term share plus
        its local term, perturbed) and db~ = sum <dY>_1 + e_b;
    MO: dW = dW~ + dw_mask + <dY>_0 o <X>_0 and db = db~ + sum <dY>_0.
    Returns (dW, db, dw_tilde, db_tilde)."""
    local1 = LIN.layer_op(layer, "dw", x1, dy1, t)
    local0 = LIN.layer_op(layer, "dw", x0, dy0, t)
    dw_tilde = add_noise(np.mod(dw_dec.astype(object) + local1, t).astype(np.int64), seed, nonce, OBJ_DW, std_w, t)
    db_tilde = add_noise(bias_grad(layer, dy1, t), seed, nonce, OBJ_DB, std_b, t)
    dW = np.mod(dw_tilde.astype(object) + dw_mask + local0, t).astype(np.int64)
    db = np.mod(db_tilde.astype(object) + bias_grad(layer, dy0, t), t).astype(np.int64)
    return dW, db, dw_tilde, db_tilde
