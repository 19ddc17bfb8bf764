"""Monte Carlo sample draws of Algorithm 1 (the Gamma_u sampling step).

Algorithm 1 draws M deformations around Delta U_i / sqrt(alpha-bar_i) with
covariance (1 / alpha-bar_i - 1) I.  The standard normal draws epsilon are
fixed by this counter-based specification so that every implementation draws
the same numbers:

* Generator: Philox4x32-10 of Salmon, Moraes, Dror and Shaw (SC'11, "Parallel
  random numbers: as easy as 1, 2, 3"): 10 rounds, multipliers 0xD2511F53 and
  0xCD9E8D57, Weyl key increments 0x9E3779B9 and 0xBB67AE85.
* Key (lo32(seed), hi32(seed)); counter (e >> 2, m, (kappa << 16) | i,
  instance_id) for element e = (k * T + t) * d_u + d of sample m at denoising
  step i of iteration kappa.  Output word j of a block feeds element 4(e>>2)+j.
* Uniform from a word x: u = (2 (x >> 9) + 1) * 2^-24, exact in FP32, in (0, 1).
* Box-Muller (Box and Muller, 1958) on word pairs (x0, x1) and (x2, x3):
  rho = sqrt(-2 ln u_a), z_even = rho cos(2 pi u_b), z_odd = rho sin(2 pi u_b).
* ln and the sine/cosine are evaluated in IEEE FP32, one correctly rounded
  operation at a time, in the order written below; fma(a, b, c) is a*b + c
  rounded once (IEEE fusedMultiplyAdd), everything else is a single operation:
  - ln: u = 2^e f with f in [0.75, 1.5); s = (f - 1) / (f + 1); s2 = s*s;
    q = fma(fma(fma(1/9, s2, 1/7), s2, 1/5), s2, 1/3) (the atanh series
    1/3 + s^2/5 + s^4/7 + s^6/9 in Horner form); t = fma(s*s2, q, s);
    ln u = fma(e, LN2_HI, fma(e, LN2_LO, 2 t)), LN2_HI = 355/512,
    LN2_LO = RN32(ln 2 - 355/512).
  - angle: u_b = (2 j + 1) 2^-24 with j = x_b >> 9; quadrant
    q = (2 j + 1 + 2^21) >> 22 in 0..4, r = ((2 j + 1) - q 2^22) 2^-23 in
    [-1/4, 1/4] (both exact), y = r * RN32(pi), y2 = y*y;
    sin y = fma(y*y2, P, y), P = fma(fma(1/9!, y2, -1/7!), y2, 1/5!) * ... in
    Horner form: P = fma(fma(fma(1/9!, y2, -1/7!), y2, 1/5!), y2, -1/3!);
    cos y = fma(y2, C, 1), C = fma(fma(fma(1/8!, y2, -1/6!), y2, 1/4!), y2, -1/2!);
    then rotate by q quarter turns.
  Series coefficients are the FP32 roundings of the exact rationals.  The
  series lengths are the shortest that keep ln, sin and cos within 2 ulp (or
  2^-23 absolute near zeros of sin and cos) over every reachable input.

fma32 obtains the single rounding from FP64: the product of two FP32
numbers is exact in FP64, the sum with c is rounded to odd in FP64 (round to
nearest, then the exact TwoSum error decides whether to step to the odd
neighbour), and rounding that to FP32 is the correctly rounded fused result
because FP64 carries more than 24 + 2 bits (Boldo and Melquiond, "Emulation
of FMA and correctly rounded sums: proved algorithms using rounding to odd",
IEEE Trans. Computers 57(4), 2008).

Pinned by the published Philox4x32-10 known-answer vectors
(tests/golden/philox4x32_10_kat.txt), by exhaustive error bounds of ln and
sin/cos against FP64 over every reachable input, by exact rational checks of
fma32, and by moment and Kolmogorov-Smirnov tests of the normals
(tests/test_oracle_noise.py).
"""
import numpy as np

_U32 = np.uint64(0xFFFFFFFF)
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)

F = np.float32


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 block function; arguments are uint32-valued arrays or ints.

    Returns four uint64 arrays holding the 32-bit output words.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & _U32
    c1 = np.asarray(c1, dtype=np.uint64) & _U32
    c2 = np.asarray(c2, dtype=np.uint64) & _U32
    c3 = np.asarray(c3, dtype=np.uint64) & _U32
    k0 = np.asarray(k0, dtype=np.uint64) & _U32
    k1 = np.asarray(k1, dtype=np.uint64) & _U32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & _U32
            k1 = (k1 + PHILOX_W1) & _U32
        p0 = PHILOX_M0 * c0          # < 2^64, exact in uint64
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _U32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _U32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def fma32(a, b, c):
    """a*b + c rounded once to FP32 (correctly rounded fused multiply-add)."""
    a = np.asarray(a, dtype=F).astype(np.float64)
    b = np.asarray(b, dtype=F).astype(np.float64)
    c = np.asarray(c, dtype=F).astype(np.float64)
    p = a * b                                   # exact: 24 + 24 bits fit in 53
    s = p + c                                   # nearest FP64
    bv = s - p                                  # TwoSum: s + err == p + c exactly
    err = (p - (s - bv)) + (c - bv)
    even = (s.view(np.uint64) & np.uint64(1)) == 0
    step = (err != 0) & even                    # inexact and even: take the odd neighbour
    s = np.where(step, np.nextafter(s, np.where(err > 0, np.inf, -np.inf)), s)
    return s.astype(F)


def uniform24(x):
    """(2 (x >> 9) + 1) * 2^-24 as FP32 (exact)."""
    j = (np.asarray(x, dtype=np.uint64) >> np.uint64(9)).astype(np.int64)
    return (2 * j + 1).astype(F) * F(2.0 ** -24)


# --- FP32 natural logarithm (operation order fixed, see module docstring)
_LN2_HI = F(355.0 / 512.0)
_LN2_LO = F(np.log(2.0) - 355.0 / 512.0)
_A3, _A5, _A7, _A9 = (F(1) / F(3), F(1) / F(5), F(1) / F(7), F(1) / F(9))


def ln32(u):
    """ln(u) for positive normal FP32 u, evaluated per the FP32 recipe."""
    u = np.asarray(u, dtype=F)
    bits = u.view(np.uint32).astype(np.int64)
    e = (bits >> 23) - 127
    f = ((bits & 0x7FFFFF) | 0x3F800000).astype(np.uint32).view(F)
    big = f >= F(1.5)
    f = np.where(big, f * F(0.5), f).astype(F)
    e = np.where(big, e + 1, e)
    s = ((f - F(1)) / (f + F(1))).astype(F)
    s2 = s * s
    q = fma32(fma32(fma32(_A9, s2, _A7), s2, _A5), s2, _A3)
    t = fma32(s * s2, q, s)
    lnf = F(2) * t
    ef = e.astype(F)
    return fma32(ef, _LN2_HI, fma32(ef, _LN2_LO, lnf))


# --- FP32 sine and cosine of 2 pi u_b
_PI = F(np.pi)
_S3, _S5, _S7, _S9 = (F(-1) / F(6), F(1) / F(120), F(-1) / F(5040), F(1) / F(362880))
_C2, _C4, _C6, _C8 = (F(-1) / F(2), F(1) / F(24), F(-1) / F(720), F(1) / F(40320))


def sincos2pi32(x):
    """(sin, cos) of 2 pi u_b where u_b is the uniform made from word x."""
    j = (np.asarray(x, dtype=np.uint64) >> np.uint64(9)).astype(np.int64)
    jj = 2 * j + 1
    q = (jj + (1 << 21)) >> 22
    rn = jj - (q << 22)
    r = rn.astype(F) * F(2.0 ** -23)
    y = r * _PI
    y2 = y * y
    sp = fma32(fma32(fma32(_S9, y2, _S7), y2, _S5), y2, _S3)
    sn = fma32(y * y2, sp, y)
    cp = fma32(fma32(fma32(_C8, y2, _C6), y2, _C4), y2, _C2)
    cs = fma32(y2, cp, F(1))
    q = q & 3
    sin_o = np.select([q == 0, q == 1, q == 2], [sn, cs, -sn], -cs).astype(F)
    cos_o = np.select([q == 0, q == 1, q == 2], [cs, -sn, -cs], sn).astype(F)
    return sin_o, cos_o


def box_muller(xa, xb):
    """Two standard normals (rho cos, rho sin) from words xa (radius) and xb (angle)."""
    rho = np.sqrt(F(-2) * ln32(uniform24(xa))).astype(F)
    s, c = sincos2pi32(xb)
    return (rho * c).astype(F), (rho * s).astype(F)


def normals_from_block(w0, w1, w2, w3):
    """The four FP32 normals of one Philox output block, in element order."""
    z0, z1 = box_muller(w0, w1)
    z2, z3 = box_muller(w2, w3)
    return z0, z1, z2, z3


def draw(seed, instance_id, kappa, step, n_samples, dim, samples=None):
    """epsilon[e][m] for e < dim, m < n_samples at denoising step i of iteration kappa.

    Returns an FP32 array of shape [dim][n_samples] (samples contiguous), or
    [dim][len(samples)] for the listed sample indices only.
    """
    if not (0 <= kappa < 65536 and 0 <= step < 65536):
        raise ValueError("iteration and step must fit 16 bits")
    seed = int(seed)
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    groups = (dim + 3) // 4
    g = np.arange(groups, dtype=np.uint64)[:, None]
    midx = np.arange(n_samples) if samples is None else np.asarray(samples)
    m = midx.astype(np.uint64)[None, :]
    c2 = (int(kappa) << 16) | int(step)
    w = philox4x32_10(g, m, np.uint64(c2), np.uint64(int(instance_id)), k0, k1)
    w = [np.broadcast_to(x, (groups, m.shape[1])) for x in w]
    z = normals_from_block(*w)
    out = np.stack(z, axis=1).reshape(groups * 4, m.shape[1])
    return np.ascontiguousarray(out[:dim])
