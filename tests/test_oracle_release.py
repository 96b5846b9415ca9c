"""Pins of the oracle's release step (pac_noised, NULL coin, posterior, diversity).

Each check uses a closed form or a statistical property fixed by the paper's
definitions (Sec. 2 PAC Privacy, Sec. 4.1 noise function, Sec. 3.2 NULLs):
the released noise has variance Var_P[y]/(2B), the posterior after k releases
is the normalised product of Gaussian likelihoods, a zero-variance or
infinite-budget cell releases y_{j*}, the NULL coin has probability
(m - popcount K)/m.
"""
import math

import numpy as np
import pytest

from oracle import pac_ref as R


def _ys(seed, k, m=64, scale=100.0):
    g = np.random.default_rng(seed)
    return [g.normal(1000.0, scale, size=m) for _ in range(k)]


def test_uniform_prior_noise_variance_is_var_over_2B():
    ys = _ys(0, 1)
    B, seed = 1.0 / 128, 1234
    j = R.secret_world(seed, 64)
    vals, nulls, _, _ = R.pac_noised_sequence(ys, [64], [100], 64, B, seed)
    z = R.standard_normal(seed, 0)
    delta = np.var(ys[0], ddof=0) / (2 * B)
    assert nulls[0] == 0
    assert math.isclose((vals[0] - ys[0][j]) / z, math.sqrt(delta), rel_tol=1e-12)


def test_weighted_variance_and_posterior_closed_form():
    ys = _ys(1, 4)
    B, seed, m = 0.05, 77, 64
    j = R.secret_world(seed, m)
    vals, nulls, _, P = R.pac_noised_sequence(ys, [m] * 4, [100] * 4, m, B, seed)
    assert not nulls.any()
    logp = np.full(m, -math.log(m))
    for c in range(4):
        Pc = np.exp(logp - logp.max())
        Pc /= Pc.sum()
        mu = float(np.average(ys[c], weights=Pc))
        s2 = float(np.average((ys[c] - mu) ** 2, weights=Pc))
        delta = s2 / (2 * B)
        z = R.standard_normal(seed, c)
        assert math.isclose(vals[c], ys[c][j] + math.sqrt(delta) * z, rel_tol=1e-12)
        logp = logp - (vals[c] - ys[c]) ** 2 / (2 * delta)
    want = np.exp(logp - logp.max())
    want /= want.sum()
    np.testing.assert_allclose(P, want, rtol=1e-9, atol=1e-300)


def test_infinite_budget_and_zero_variance_release_the_secret_world():
    ys = _ys(2, 3)
    seed = 5
    j = R.secret_world(seed, 64)
    vals, _, flags, P = R.pac_noised_sequence(ys, [64] * 3, [50] * 3, 64, math.inf, seed)
    assert np.array_equal(vals, np.array([y[j] for y in ys]))
    assert np.all(flags & R.CELL_ZERO_VARIANCE)
    assert np.allclose(P, 1.0 / 64)
    flat = [np.full(64, 7.0)]
    v2, _, f2, _ = R.pac_noised_sequence(flat, [64], [50], 64, 0.01, seed)
    assert v2[0] == 7.0 and f2[0] & R.CELL_ZERO_VARIANCE


def test_monte_carlo_noise_moments():
    y = _ys(3, 1, scale=10.0)[0]
    B = 0.25
    N = 20000
    d = np.empty(N)
    for s in range(N):
        j = R.secret_world(s, 64)
        v, _, _, _ = R.pac_noised_sequence([y], [64], [10], 64, B, s)
        d[s] = v[0] - y[j]
    delta = np.var(y) / (2 * B)
    assert abs(d.mean()) < 5 * math.sqrt(delta / N)
    assert abs(d.var() / delta - 1.0) < 5 * math.sqrt(2.0 / N)


def test_secret_world_is_uniform():
    N = 64 * 400
    h = np.bincount([R.secret_world(s, 64) for s in range(N)], minlength=64)
    chi2 = float(((h - 400) ** 2 / 400).sum())
    assert chi2 < 120  # 63 dof, p ~ 1e-5 threshold


def test_null_coin_frequency():
    y = np.arange(64, dtype=np.float64)
    N = 20000
    nulls = 0
    for s in range(N):
        _, n, f, _ = R.pac_noised_sequence([y], [48], [10], 64, 0.1, s)
        nulls += int(n[0])
        assert bool(f[0] & R.CELL_NULL) == bool(n[0])
    p = 16 / 64
    assert abs(nulls / N - p) < 5 * math.sqrt(p * (1 - p) / N)
    # popcount 64: never NULL; popcount 0: always NULL
    assert R.pac_noised_sequence([y], [64], [10], 64, 0.1, 1)[1][0] == 0
    assert R.pac_noised_sequence([y], [0], [10], 64, 0.1, 1)[1][0] == 1


def test_null_cell_leaves_posterior_unchanged():
    ys = _ys(4, 2)
    seed = next(s for s in range(1000) if R.null_uniform(s, 0) < 0.5 <= R.null_uniform(s, 1))
    vals, nulls, _, P = R.pac_noised_sequence(ys, [32, 64], [10, 10], 64, 0.1, seed)
    assert list(nulls) == [1, 0]
    # the second cell sees the uniform prior
    j = R.secret_world(seed, 64)
    delta = np.var(ys[1]) / 0.2
    assert math.isclose(vals[1], ys[1][j] + math.sqrt(delta) * R.standard_normal(seed, 1), rel_tol=1e-12)


def test_standard_normal_moments():
    z = np.array([R.standard_normal(9, c) for c in range(40000)])
    assert abs(z.mean()) < 0.03 and abs(z.var() - 1) < 0.03
    assert abs(np.mean(z ** 3)) < 0.06 and abs(np.mean(z ** 4) - 3) < 0.15


def test_cell_vectors_scale_avg_and_diversity():
    cnt = np.array([[4, 0, 2] + [1] * 61], dtype=np.int64)
    isum = np.array([[[40, 0, 10] + [3] * 61]], dtype=np.int64)
    counters = {"count": cnt, "isum": isum, "fsum": np.zeros((1, 0, 64)), "nrows": np.array([8])}
    yc = R.cell_vector(counters, 0, R.KIND_COUNT, 0, R.FLAG_SCALE2)
    assert np.array_equal(yc, 2.0 * cnt[0])
    ys = R.cell_vector(counters, 0, R.KIND_SUM_I, 0, R.FLAG_SCALE2)
    assert np.array_equal(ys, 2.0 * isum[0, 0])
    ya = R.cell_vector(counters, 0, R.KIND_AVG_I, 0, R.FLAG_SCALE2)
    assert ya[0] == 10.0 and ya[1] == 0.0 and ya[2] == 5.0 and ya[3] == 3.0
    yt = R.cell_vector(counters, 0, R.KIND_AVG_I, 0, R.FLAG_AVG_TOTALCOUNT)
    assert yt[0] == 2 * 40 / 8
    assert R.diversity_flag(100, 33, 64) and not R.diversity_flag(100, 50, 64)
    assert not R.diversity_flag(5, 33, 64) and R.diversity_flag(20, 70, 128)
    with pytest.raises(ValueError):
        R.pac_noised_sequence([yc], [33], [100], 64, 0.1, 1, flags=R.FLAG_STRICT_DIVERSITY)


def test_fixed_prior_keeps_uniform_posterior():
    ys = _ys(6, 3)
    _, _, _, P = R.pac_noised_sequence(ys, [64] * 3, [10] * 3, 64, 0.1, 3, flags=R.FLAG_SCALE2 | R.FLAG_FIXED_PRIOR)
    assert np.allclose(P, 1 / 64)
