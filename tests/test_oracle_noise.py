"""Pins of the sample draws: Philox known answers, FP32 ln/sin/cos error
bounds over every reachable input, normal statistics and the counter layout."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import noise

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(t, 16) for t in line.split()])
    return rows


def test_philox_known_answers():
    rows = _kat_rows()
    assert len(rows) == 3
    for row in rows:
        ctr, key, want = row[0:4], row[4:6], row[6:10]
        got = noise.philox4x32_10(*ctr, *key)
        assert [int(v) for v in got] == want


def test_uniform_range_and_exactness():
    x = np.array([0, 511, 512, 0xFFFFFFFF, 0x80000000], dtype=np.uint64)
    u = noise.uniform24(x).astype(np.float64)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24 and u[2] == 3 * 2.0 ** -24
    assert u[3] == 1 - 2.0 ** -24 and u[4] == 0.5 + 2.0 ** -24
    assert (u > 0).all() and (u < 1).all()


def _all_words():
    return np.arange(1 << 23, dtype=np.uint64) << np.uint64(9)


def test_ln32_within_2ulp_over_all_inputs():
    u = noise.uniform24(_all_words())
    got = noise.ln32(u).astype(np.float64)
    ref = np.log(u.astype(np.float64))
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(got - ref) / ulp) <= 2.0


def test_sincos_within_2ulp_over_all_inputs():
    x = _all_words()
    s, c = noise.sincos2pi32(x)
    ang = 2.0 * np.pi * noise.uniform24(x).astype(np.float64)
    for got, ref in ((s, np.sin(ang)), (c, np.cos(ang))):
        err = np.abs(got.astype(np.float64) - ref)
        ulp = np.spacing(np.maximum(np.abs(ref), 1e-30).astype(np.float32)).astype(np.float64)
        assert np.max(np.minimum(err / ulp, err / 2.0 ** -24)) <= 2.0
        assert np.max(err) <= 1.2e-7


def test_normals_statistics():
    z = noise.draw(seed=12345, instance_id=0, kappa=0, step=7, n_samples=4096, dim=256).astype(np.float64)
    flat = z.ravel()
    n = flat.size
    assert abs(flat.mean()) < 5.0 / np.sqrt(n)
    assert abs(flat.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert abs(stats.skew(flat)) < 5.0 * np.sqrt(6.0 / n)
    assert abs(stats.kurtosis(flat)) < 5.0 * np.sqrt(24.0 / n)
    assert stats.kstest(flat, "norm").pvalue > 1e-4
    # the two outputs of one Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(z[0::4].ravel(), z[1::4].ravel())[0, 1]) < 5.0 / np.sqrt(n / 4)
    # neighbouring samples are uncorrelated
    assert abs(np.corrcoef(z[:, :-1].ravel(), z[:, 1:].ravel())[0, 1]) < 5.0 / np.sqrt(n)


def test_counter_layout_elementwise():
    seed, inst, kappa, step, M, D = 0x1234567890ABCDEF, 3, 2, 99, 5, 11
    z = noise.draw(seed, inst, kappa, step, M, D)
    assert z.shape == (D, M) and z.dtype == np.float32
    for e in range(D):
        for m in range(M):
            w = noise.philox4x32_10(e >> 2, m, (kappa << 16) | step, inst,
                                    seed & 0xFFFFFFFF, seed >> 32)
            w = [np.uint64(int(v)) for v in w]
            j = e & 3
            pair = (w[0], w[1]) if j < 2 else (w[2], w[3])
            a, b = noise.box_muller(np.array([pair[0]]), np.array([pair[1]]))
            want = (a if j % 2 == 0 else b)[0]
            assert z[e, m] == want


def test_streams_differ():
    base = noise.draw(0, 0, 0, 1, 64, 16)
    for kw in (dict(seed=1), dict(instance_id=1), dict(kappa=1), dict(step=2)):
        args = dict(seed=0, instance_id=0, kappa=0, step=1, n_samples=64, dim=16)
        args.update(kw)
        assert not np.array_equal(base, noise.draw(**args))
    # prefix property: a longer draw extends a shorter one
    assert np.array_equal(noise.draw(0, 0, 0, 1, 64, 10), base[:10])
    assert np.array_equal(noise.draw(0, 0, 0, 1, 32, 16), base[:, :32])


def test_rejects_wide_counters():
    with pytest.raises(ValueError):
        noise.draw(0, 0, 65536, 1, 4, 4)


def test_sample_subset_matches_full_draw():
    full = noise.draw(5, 1, 0, 3, 40, 13)
    sub = noise.draw(5, 1, 0, 3, 40, 13, samples=[0, 7, 39, 12])
    assert np.array_equal(sub, full[:, [0, 7, 39, 12]])


def _round_to_f32_exact(x):
    """Nearest FP32 (ties to even) of an exact rational, by bisection on neighbours."""
    from fractions import Fraction
    g = np.float32(float(x))                    # within one FP32 step of x
    best = None
    for cand in (np.nextafter(g, np.float32(-np.inf)), g, np.nextafter(g, np.float32(np.inf))):
        d = abs(Fraction(float(cand)) - x)
        if best is None or d < best[0] or (d == best[0] and (int(cand.view(np.uint32)) & 1) == 0):
            best = (d, cand)
    return best[1]


def test_fma32_is_correctly_rounded():
    """fma32 against exact rational arithmetic: random operands, near-total
    cancellation (the hard cases for a double rounding), exact midpoints and
    the operand ranges of the ln and sin/cos recipes."""
    from fractions import Fraction
    rng = np.random.default_rng(7)
    cases = []
    for _ in range(3000):
        a, b = np.float32(rng.normal() * 4), np.float32(rng.normal())
        cases.append((a, b, np.float32(rng.normal())))
        # c close to -a*b: the exact sum keeps bits far below FP32's last place
        cases.append((a, b, np.float32(-(np.float64(a) * np.float64(b)) * (1 + rng.normal() * 1e-6))))
        # c in [1, 2) and a*b half an FP32 step of c (an exact midpoint, ties
        # to even), or a hair above or below it
        m = np.float32(rng.uniform(1, 2))
        sgn = rng.choice([-1.0, 1.0])
        for b in (1.0, 1.0 + 2.0 ** -20, 1.0 - 2.0 ** -20):
            cases.append((np.float32(2.0 ** -24), np.float32(sgn * b), m))
        # a*b = 2^-24 - 2^-70: the exact sum sits just inside an FP32 midpoint
        # but rounds onto it in FP64, where a plain double rounding goes wrong
        # whenever c's last bit is odd
        for cm in (m, np.nextafter(m, np.float32(2))):
            cases.append((np.float32(2.0 ** -24 * (1 + 2.0 ** -23)), np.float32(sgn * (1 - 2.0 ** -23)), cm))
    for s2 in np.float32(rng.uniform(0, 0.05, 500)):
        cases.append((np.float32(1) / np.float32(9), s2, np.float32(1) / np.float32(7)))
    a, b, c = (np.array(v, dtype=np.float32) for v in zip(*cases))
    got = noise.fma32(a, b, c)
    for ai, bi, ci, gi in zip(a, b, c, got):
        exact = Fraction(float(ai)) * Fraction(float(bi)) + Fraction(float(ci))
        assert gi.view(np.uint32) == _round_to_f32_exact(exact).view(np.uint32), (ai, bi, ci)
