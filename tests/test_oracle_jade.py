"""Pins of the oracle's JADE control-parameter adaptation and archive
(sections "Selection" and "Evolution by neighborhood similarity": JADE with
archive in every domain; the adaptation itself is JADE's published one)."""
import numpy as np
import pytest
from scipy import stats

import oracle
from tests import _tiny

GRID = 2.0 ** 24


def _words(n, seed):
    return np.random.default_rng(seed).integers(0, 2 ** 64, size=(n, 4), dtype=np.uint64)


def test_cr_draws_are_clipped_normal_on_the_grid():
    k_cr, _, _ = oracle.jade_draws(_words(20000, 1), 0.5, 0.5, 32)
    cr = k_cr / GRID
    assert np.all((k_cr >= 0) & (k_cr <= 2 ** 24))
    # N(0.5, 0.1): clipping at 0 and 1 is 5 sigma away
    assert stats.kstest(cr, stats.norm(0.5, 0.1).cdf).pvalue > 1e-3
    k_lo, _, _ = oracle.jade_draws(_words(20000, 2), 0.02, 0.5, 32)
    # mu near 0: the mass below 0 (P(Z < -0.2)) sits at exactly 0
    assert abs(np.mean(k_lo == 0) - stats.norm.cdf(-0.2)) < 0.012


def test_f_draws_are_truncated_cauchy():
    _, k_f, _ = oracle.jade_draws(_words(20000, 3), 0.5, 0.5, 32)
    f = k_f / GRID
    assert np.all((k_f >= 1) & (k_f <= 2 ** 24))
    # Cauchy(0.5, 0.1) redrawn below 0 and cut at 1: conditional on acceptance
    c = stats.cauchy(0.5, 0.1)
    p0 = c.cdf(0.0)
    p_one = (1.0 - c.cdf(1.0)) / (1.0 - p0)
    assert abs(np.mean(k_f == 2 ** 24) - p_one) < 0.006
    inner = f[k_f < 2 ** 24]
    cdf = lambda x: (c.cdf(x) - p0) / (c.cdf(1.0) - p0)  # noqa: E731
    assert stats.kstest(inner, cdf).pvalue > 1e-3


def test_f_falls_back_to_the_mean_after_three_rejections():
    # mu_F far below 0: every Cauchy draw is negative
    _, k_f, _ = oracle.jade_draws(_words(100, 4), 0.5, -50.0, 32)
    assert np.all(k_f == 1)
    _, k_f, _ = oracle.jade_draws(_words(2000, 5), 0.5, 1e-3, 32)
    # near-zero mean: about half the draws fail thrice in a row only rarely;
    # the accepted values stay in (0, 1]
    assert np.all((k_f >= 1) & (k_f <= 2 ** 24))


def test_archive_positions_are_uniform():
    _, _, a = oracle.jade_draws(_words(16000, 6), 0.5, 0.5, 16)
    counts = np.bincount(a, minlength=16)
    assert a.min() >= 0 and a.max() < 16
    assert stats.chisquare(counts).pvalue > 1e-3


def test_constant_parameters_and_empty_archive_give_the_plain_trial():
    rng = np.random.default_rng(7)
    np_, P = 12, 3
    pop = rng.uniform(-1, 1, size=(np_, P)).astype(np.float32)
    S = rng.random(np_)
    lo = np.full(P, -1.0, np.float32)
    hi = np.full(P, 1.0, np.float32)
    w = _words(np_, 8)
    F, CR = 0.5, 0.875  # CR on the 2^-24 grid
    plain = oracle.de_trial(pop, S, w, F, CR, lo, hi)
    jade = oracle.jade_trial(pop, S, np.zeros((0, P), np.float32), w,
                             np.full(np_, int(F * GRID)), np.full(np_, int(CR * GRID)), lo, hi)
    np.testing.assert_array_equal(plain, jade)


def test_second_difference_vector_draws_from_population_and_archive():
    # zero population, F = 1, CR = 1, wide box: trial = -x_r2, which names r2
    np_, P, n_arch = 10, 1, 6
    pop = np.zeros((np_, P), np.float32)
    archive = (np.arange(n_arch, dtype=np.float32) + 1.0).reshape(n_arch, P)
    lo, hi = np.full(P, -100.0, np.float32), np.full(P, 100.0, np.float32)
    hits = np.zeros(n_arch + 1)
    n_rounds = 1500
    for r in range(n_rounds):
        w = _words(np_, 100 + r)
        t = oracle.jade_trial(pop, np.zeros(np_), archive, w, np.full(np_, 2 ** 24),
                              np.full(np_, 2 ** 24), lo, hi)[:, 0]
        idx = np.rint(-t).astype(int)          # 0: a population member, k: archive entry k-1
        hits += np.bincount(idx, minlength=n_arch + 1)
    total = hits.sum()
    # r2 uniform over the NP + |A| - 2 members other than i and r1
    expect_arch = n_arch / (np_ + n_arch - 2)
    assert abs(hits[1:].sum() / total - expect_arch) < 0.01
    assert stats.chisquare(hits[1:]).pvalue > 1e-3


SPHERE = dict(np_lo=20, np_hi=20, ng_f=40, np_bf=5, ng_bf=1, n_cycle=0, n_bucket=1,
              ens_enabled=0, F=0.5, CR=0.5)


def _flat_line(n_cmp=2, nt=60):
    tr = np.zeros((n_cmp, nt))
    return _tiny.line(tr, [1] * n_cmp, [100.0] * n_cmp, window=3, op=3, ap=0)


def test_jade_search_converges_on_the_sphere_and_keeps_counts():
    L = _flat_line()
    bounds = (np.array([-1.0, -1.0, -1.0], np.float32), np.array([1.0, 1.0, 1.0], np.float32), 0)
    p, S, ev = L.search(bounds, dict(SPHERE, adapt=1), 3, objective=1)
    assert ev == 2 * 60 * 20 * 41
    # optimum at box-normalised 0.3, 0.4, 0.5: x = 2 z - 1
    target = np.array([-0.4, -0.2, 0.0])
    err = np.abs(p.reshape(-1, 3) - target).max(axis=1)
    assert np.median(err) < 1e-3 and np.mean(S > 0.999) > 0.9


def test_jade_without_generations_is_the_plain_search():
    L = _flat_line()
    bounds = (np.array([-1.0, -1.0, -1.0], np.float32), np.array([1.0, 1.0, 1.0], np.float32), 0)
    a = L.search(bounds, dict(SPHERE, ng_f=0, adapt=1), 5, objective=1)
    b = L.search(bounds, dict(SPHERE, ng_f=0, adapt=0), 5, objective=1)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


@pytest.mark.parametrize("ens_on", [0, 1])
def test_jade_reaches_the_fixed_parameter_quality_at_a_small_budget(ens_on):
    # sphere mock at 16 x 20, plain and with the ENS sweep
    L = _flat_line(n_cmp=8, nt=60)
    bounds = (np.array([-1.0, -1.0, -1.0], np.float32), np.array([1.0, 1.0, 1.0], np.float32), 0)
    de = dict(SPHERE, np_lo=16, np_hi=16, ng_f=20, ens_enabled=ens_on, n_bucket=4, n_cycle=0)
    _, S_fixed, _ = L.search(bounds, dict(de, adapt=0, CR=0.9), 11, objective=1)
    _, S_jade, _ = L.search(bounds, dict(de, adapt=1, CR=0.5), 11, objective=1)
    print(f"ens={ens_on}: mean S fixed {S_fixed.mean():.5f} jade {S_jade.mean():.5f}")
    assert S_jade.mean() >= S_fixed.mean() - 0.01
