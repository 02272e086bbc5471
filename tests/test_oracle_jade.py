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


# ---------------------------------------------------------------------------
# the written-out series against the library functions, and the draws
# against the textbook constructions (Box-Muller, inverse Cauchy CDF)

_PI_LD = np.longdouble("3.14159265358979323846264338327950288")
EPS = 2.0 ** -53


def _uniform_words(n, seed):
    return np.random.default_rng(seed).integers(0, 2 ** 64, size=n, dtype=np.uint64)


def test_series_ln_within_four_ulp_of_the_library_log():
    # the inputs the CR draws feed it: (top 53 bits + 1) 2^-53, plus a wide
    # log-uniform range
    u = ((_uniform_words(1_000_000, 21) >> np.uint64(11)).astype(np.float64) + 1.0) * EPS
    u = np.concatenate([u, np.exp(np.random.default_rng(22).uniform(-700, 700, 200_000))])
    ref = np.log(u.astype(np.longdouble))
    got = oracle.jade_series("ln", u)
    ulp = np.spacing(np.abs(ref).astype(np.float64))
    assert np.all(np.abs(got - ref) <= 4 * ulp)


def test_series_cos_turns_within_eight_eps_of_the_library_cos():
    t = (_uniform_words(1_000_000, 23) >> np.uint64(11)).astype(np.float64) * EPS
    t = np.concatenate([t, np.arange(8) / 8.0])        # quarter-turn boundaries
    ref = np.cos(2 * _PI_LD * t.astype(np.longdouble))
    got = oracle.jade_series("cos_turns", t)
    assert np.all(np.abs(got - ref) <= 8 * EPS)


def test_series_tan_half_turn_within_its_conditioning_of_the_library_tan():
    # x = (h + 1/2) 2^-32 - 1/2 for 32-bit h, as in the F draws; the rounding
    # of the argument pi |x| alone moves tan by about eps (1 + tan^2)
    h = (_uniform_words(1_000_000, 24) >> np.uint64(32)).astype(np.float64)
    x = (h + 0.5) * 2.0 ** -32 - 0.5
    x = np.concatenate([x, [-0.5 + 2.0 ** -33, 0.5 - 2.0 ** -33, 0.0, 0.25, -0.25]])
    ref = np.tan(_PI_LD * x.astype(np.longdouble))
    got = oracle.jade_series("tan_half_turn", x)
    bound = 8 * EPS * (1.0 + np.abs(ref).astype(np.float64)) ** 2
    assert np.all(np.abs(got - ref) <= bound)
    # odd symmetry is exact by construction
    np.testing.assert_array_equal(oracle.jade_series("tan_half_turn", -x), -got)


def test_draws_are_box_muller_and_inverse_cauchy_of_their_words():
    n = 200_000
    w = _words(n, 31)
    mu_cr, mu_f, np_ = 0.45, 0.6, 24
    k_cr, k_f, a_idx = oracle.jade_draws(w, mu_cr, mu_f, np_)
    # CR ~ N(mu_CR, 0.1) by Box-Muller from the top 53 bits of words 0 and 1
    u1 = ((w[:, 0] >> np.uint64(11)).astype(np.float64) + 1.0) * EPS
    u2 = (w[:, 1] >> np.uint64(11)).astype(np.float64) * EPS
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    cr = np.clip(mu_cr + 0.1 * z, 0.0, 1.0)
    want_cr = np.rint(cr * GRID).astype(np.int64)
    # F ~ Cauchy(mu_F, 0.1) by the inverse CDF, cut to 1, redrawn up to three
    # times where not positive, else mu_F
    halves = [w[:, 2] >> np.uint64(32), w[:, 2] & np.uint64(0xFFFFFFFF), w[:, 3] >> np.uint64(32)]
    want_f = np.zeros(n, np.int64)
    for hh in halves:
        f = mu_f + 0.1 * np.tan(np.pi * ((hh.astype(np.float64) + 0.5) * 2.0 ** -32 - 0.5))
        f = np.minimum(f, 1.0)
        take = (want_f == 0) & (f > 0.0)
        want_f[take] = np.rint(f[take] * GRID)
    want_f[want_f == 0] = max(1, int(np.rint(mu_f * GRID)))
    # library and series may round a value lying within an ulp of a grid
    # half-step to neighbouring grid points; nothing else may differ
    assert np.abs(k_cr - want_cr).max() <= 1 and np.mean(k_cr == want_cr) > 0.9999
    assert np.abs(k_f - want_f).max() <= 1 and np.mean(k_f == want_f) > 0.9999
    want_a = ((w[:, 3] & np.uint64(0xFFFFFFFF)).astype(np.uint64) * np.uint64(np_)) >> np.uint64(32)
    np.testing.assert_array_equal(a_idx, want_a.astype(np.int32))


# ---------------------------------------------------------------------------
# the adaptation bookkeeping by hand: two generations of NP = 5

def _k(v):
    return int(round(v * GRID))


def test_two_generations_of_adaptation_by_hand():
    np_, P = 5, 1
    pop0 = np.array([[0.1], [0.2], [0.3], [0.4], [0.5]], np.float32)
    S0 = np.full(np_, 0.5)
    lo, hi = np.array([-10.0], np.float32), np.array([10.0], np.float32)
    de_words = _words(2 * np_, 41).reshape(2, np_, 4)
    # generation 1 draws (CR, F, archive position) and trial scores: slots 0,
    # 2 (a tie counts as success) and 3 replace their parents, 1 and 4 fail
    cr1, f1, a1 = [0.5, 0.125, 0.75, 0.875, 0.25], [0.625, 0.25, 0.375, 0.875, 0.125], [3, 1, 4, 0, 2]
    st1 = [0.6, 0.4, 0.5, 0.7, 0.1]
    # generation 2: slots 0, 1 and 4 succeed; the archive holds 3 entries, so
    # slots 0 and 1 are appended and slot 4 overwrites its drawn position 0
    cr2, f2, a2 = [0.25, 0.5, 0.0625, 0.75, 1.0], [0.5, 0.75, 1.0, 0.25, 0.125], [2, 3, 1, 4, 0]
    st2 = [0.9, 0.8, 0.1, 0.2, 0.55]
    draws = np.array([[[_k(c), _k(f), a] for c, f, a in zip(cr1, f1, a1)],
                      [[_k(c), _k(f), a] for c, f, a in zip(cr2, f2, a2)]], np.int32)
    r = oracle.jade_run(pop0, S0, de_words, [st1, st2], 0.5, 0.5, lo, hi, draws=draws)
    t1, t2 = r["trials"][0][:, 0], r["trials"][1][:, 0]

    # after generation 1: mu_CR = 0.9 * 0.5 + 0.1 * (0.5 + 0.75 + 0.875) / 3
    #                     mu_F  = 0.9 * 0.5 + 0.1 * (0.625^2 + 0.375^2 + 0.875^2) / (0.625 + 0.375 + 0.875)
    mu_cr1 = 0.45 + 0.1 * (2.125 / 3.0)
    mu_f1 = 0.45 + 0.1 * (1.296875 / 1.875)
    assert r["mu"][0, 0] == pytest.approx(mu_cr1, rel=1e-15)
    assert r["mu"][0, 1] == pytest.approx(mu_f1, rel=1e-15)
    # the arithmetic mean of F, or means over every slot, give other values
    assert abs(mu_f1 - (0.45 + 0.1 * 0.625)) > 1e-3
    assert abs(mu_cr1 - (0.45 + 0.1 * 0.5)) > 1e-3
    assert r["n_arch"][0] == 3
    np.testing.assert_array_equal(r["archive"][0][:3, 0], np.float32([0.1, 0.3, 0.4]))

    # generation 2 reads the population after generation 1's selection
    pop1 = np.array([[t1[0]], [0.2], [t1[2]], [t1[3]], [0.5]], np.float32)
    S1 = np.array([0.6, 0.5, 0.5, 0.7, 0.5])
    want_t2 = oracle.jade_trial(pop1, S1, r["archive"][0][:3], de_words[1], draws[1, :, 1],
                                draws[1, :, 0], lo, hi)[:, 0]
    np.testing.assert_array_equal(t2, want_t2)
    mu_cr2 = 0.9 * mu_cr1 + 0.1 * ((0.25 + 0.5 + 1.0) / 3.0)
    mu_f2 = 0.9 * mu_f1 + 0.1 * ((0.25 + 0.5625 + 0.015625) / (0.5 + 0.75 + 0.125))
    assert r["mu"][1, 0] == pytest.approx(mu_cr2, rel=1e-15)
    assert r["mu"][1, 1] == pytest.approx(mu_f2, rel=1e-15)
    # archive: slot 0's parent (t1[0]) appended at 3, slot 1's (0.2) at 4, then
    # the full archive takes slot 4's parent (0.5) at slot 4's position 0
    assert r["n_arch"][1] == 5
    np.testing.assert_array_equal(r["archive"][1][:, 0], np.float32([0.5, 0.3, 0.4, t1[0], 0.2]))
    # final population: the successful trials of generation 2 over pop1
    want_pop = pop1[:, 0].copy()
    for i in (0, 1, 4):
        want_pop[i] = t2[i]
    np.testing.assert_array_equal(r["pop"][:, 0], want_pop)
    np.testing.assert_array_equal(r["S"], [0.9, 0.8, 0.5, 0.7, 0.55])


def test_draws_of_each_generation_use_the_updated_means():
    np_, P, ng = 8, 3, 4
    rng = np.random.default_rng(51)
    pop = rng.uniform(-1, 1, size=(np_, P)).astype(np.float32)
    S = rng.random(np_)
    lo, hi = np.full(P, -1.0, np.float32), np.full(P, 1.0, np.float32)
    de_words = _words(ng * np_, 52).reshape(ng, np_, 4)
    jade_words = _words(ng * np_, 53).reshape(ng, np_, 4)
    St = rng.random((ng, np_)) * 2.0        # about three quarters succeed
    r = oracle.jade_run(pop, S, de_words, St, 0.5, 0.6, lo, hi, jade_words=jade_words)
    cur_pop, cur_S = pop.copy(), S.copy()
    mu = (0.6, 0.5)
    arch = np.zeros((0, P), np.float32)
    for g in range(ng):
        k_cr, k_f, _ = oracle.jade_draws(jade_words[g], mu[0], mu[1], np_)
        want = oracle.jade_trial(cur_pop, cur_S, arch, de_words[g], k_f, k_cr, lo, hi)
        np.testing.assert_array_equal(r["trials"][g], want)
        ok = St[g] >= cur_S
        cur_pop[ok] = want[ok]
        cur_S[ok] = St[g][ok]
        mu = tuple(r["mu"][g])
        arch = r["archive"][g][: r["n_arch"][g]]
    assert r["n_arch"][-1] == np_
