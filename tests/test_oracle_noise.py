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
