"""Philox4x32-10 counter-based generator and Box-Muller normals (host side).

Definition (Salmon et al., SC'11, section 3.2): a 128-bit counter
(c0, c1, c2, c3) and a 64-bit key (k0, k1) go through ten rounds.  One round
computes the two 32x32->64 products hi0:lo0 = M0*c0 and hi1:lo1 = M1*c2 and
returns (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is advanced by the
Weyl constants (W0, W1) before every round but the first.

Uniforms: the four output words of one call give two 53-bit integers
m1 = (x0 >> 5) * 2^26 + (x1 >> 6) and m2 = (x2 >> 5) * 2^26 + (x3 >> 6);
u1 = (m1 + 1) * 2^-53 lies in (0, 1] and u2 = m2 * 2^-53 in [0, 1).
Normals (Box-Muller): rho = sqrt(-2 ln u1), z_even = rho * cos(2 pi u2),
z_odd = rho * sin(2 pi u2).  Entry e of a stream uses call e >> 1 and takes
z_even or z_odd by e & 1.

ln, cos and sin are this module's own (ln_unit, cos_sin_turns): series
evaluated with + - * / and exact operations (frexp, floor, negation) in a
fixed order, on constants that are the doubles nearest their exact values.
The device generator (synth/csrc/synth_gen.hip, built without contraction
of multiply-adds) evaluates the same operations in the same order, and
sqrt is correctly rounded on both sides, so host and device draw the same
doubles bit for bit.
"""
from fractions import Fraction
from math import factorial

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on arrays of 32-bit counter words.

    c0..c3 are broadcastable integer arrays holding values < 2^32; k0, k1 are
    Python ints < 2^32.  Returns four uint32 arrays.
    """
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    ka, kb = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r:
            ka = (ka + W0) & 0xFFFFFFFF
            kb = (kb + W1) & 0xFFFFFFFF
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(ka), lo1,
                          hi0 ^ c3 ^ np.uint64(kb), lo0)
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def uniforms53(x0, x1, x2, x3):
    """Two 53-bit uniforms per Philox call: u1 in (0, 1], u2 in [0, 1)."""
    x0 = np.asarray(x0, dtype=np.uint64)
    x1 = np.asarray(x1, dtype=np.uint64)
    x2 = np.asarray(x2, dtype=np.uint64)
    x3 = np.asarray(x3, dtype=np.uint64)
    m1 = ((x0 >> np.uint64(5)) << np.uint64(26)) | (x1 >> np.uint64(6))
    m2 = ((x2 >> np.uint64(5)) << np.uint64(26)) | (x3 >> np.uint64(6))
    scale = 2.0 ** -53
    u1 = (m1.astype(np.float64) + 1.0) * scale
    u2 = m2.astype(np.float64) * scale
    return u1, u2


LN2 = float.fromhex("0x1.62e42fefa39efp-1")        # nearest double to ln 2
HALF_PI = float.fromhex("0x1.921fb54442d18p+0")   # nearest double to pi / 2
SQRT_HALF = float.fromhex("0x1.6a09e667f3bcdp-1")  # nearest double to sqrt(1/2)
# 1 / (2k + 1), k = 0..11, and (-1)^k / (2k + 1)!, k = 0..9, and
# (-1)^k / (2k)!, k = 0..10, each the nearest double
LOG_COEF = tuple(float(Fraction(1, 2 * k + 1)) for k in range(12))
SIN_COEF = tuple(float(Fraction((-1) ** k, factorial(2 * k + 1))) for k in range(10))
COS_COEF = tuple(float(Fraction((-1) ** k, factorial(2 * k))) for k in range(11))


def _horner(coef, z):
    p = np.full(np.shape(z), coef[-1], dtype=np.float64)
    for c in coef[-2::-1]:
        p = p * z + c
    return p


def ln_unit(u):
    """Natural logarithm for u in (0, 1].  u = m 2^e with m in [sqrt(1/2),
    sqrt(2)) (frexp, then one doubling), and ln m = 2 artanh(s) =
    2 s sum_k s^(2k) / (2k + 1) with s = (m - 1) / (m + 1), |s| <= 0.172, the
    series cut after s^22 (the rest is below 1e-19 of the sum)."""
    u = np.asarray(u, dtype=np.float64)
    f, e = np.frexp(u)
    low = f < SQRT_HALF
    m = np.where(low, f * 2.0, f)
    e = np.where(low, e - 1, e).astype(np.float64)
    s = (m - 1.0) / (m + 1.0)
    t = s * _horner(LOG_COEF, s * s)
    return e * LN2 + (t + t)


def cos_sin_turns(u):
    """(cos 2 pi u, sin 2 pi u) for u in [0, 1).  4u = q + r with q the
    nearest integer and |r| <= 1/2 (both exact), theta = r pi / 2, so that
    |theta| <= pi / 4; Taylor series of cos and sin in theta cut after
    theta^20 and theta^19 (the rest is below 1e-21), then the quadrant
    q mod 4 rotates (cos, sin)."""
    u = np.asarray(u, dtype=np.float64)
    w = 4.0 * u
    q = np.floor(w + 0.5)
    th = (w - q) * HALF_PI
    x2 = th * th
    sn = th * _horner(SIN_COEF, x2)
    cs = _horner(COS_COEF, x2)
    qm = q.astype(np.int64) & 3
    cos = np.select([qm == 0, qm == 1, qm == 2], [cs, -sn, -cs], sn)
    sin = np.select([qm == 0, qm == 1, qm == 2], [sn, cs, -sn], -cs)
    return cos, sin


def normals(first, count, stream_id, tag, seed):
    """Standard normals for entries [first, first + count) of one stream.

    A stream is identified by (stream_id, tag) under the 64-bit ``seed``;
    entry e uses Philox counter (lo32(e >> 1), hi32(e >> 1), stream_id, tag).
    """
    e = np.arange(first, first + count, dtype=np.uint64)
    call = e >> np.uint64(1)
    x0, x1, x2, x3 = philox4x32_10(call & _MASK, call >> _S32,
                                   np.uint64(stream_id & 0xFFFFFFFF),
                                   np.uint64(tag & 0xFFFFFFFF),
                                   seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    u1, u2 = uniforms53(x0, x1, x2, x3)
    rho = np.sqrt(-2.0 * ln_unit(u1))
    cos, sin = cos_sin_turns(u2)
    odd = (e & np.uint64(1)).astype(bool)
    return np.where(odd, rho * sin, rho * cos)
