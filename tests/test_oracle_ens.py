"""Pins of the oracle's ENS sweep (sections "Information propagation" and
"Evolution by neighborhood similarity"), with and without time-sample skipping."""
import numpy as np
import pytest

import oracle
from paper_2304_11399_amd.counts import evals_ens
from synth import make_workload, base_bounds
from tests import _tiny

ENS = dict(np_lo=8, np_hi=8, ng_f=6, np_bf=5, ng_bf=1, n_cycle=1, n_bucket=4,
           ens_enabled=1, F=0.5, CR=0.9)


@pytest.fixture(scope="module")
def small_crs():
    g, wl = make_workload("crs_ens", n_cmp=12, nt=300, snr=3.0)
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    return L, base_bounds(wl)


def test_exchange_off_equals_plain_de(small_crs):
    L, bounds = small_crs
    de_ens = dict(ENS, n_cycle=0)
    de_plain = dict(ENS, n_cycle=0, ens_enabled=0)
    pa, Sa, ea = L.search(bounds, de_ens, 7, t_begin=100, t_end=160, inject=0)
    pb, Sb, eb = L.search(bounds, de_plain, 7, t_begin=100, t_end=160)
    np.testing.assert_array_equal(pa, pb)
    np.testing.assert_array_equal(Sa, Sb)
    assert ea == eb


def test_counts_match_formula(small_crs):
    L, bounds = small_crs
    for n_cycle in (0, 1, 2):
        de = dict(ENS, n_cycle=n_cycle)
        _, _, ev = L.search(bounds, de, 3, t_begin=50, t_end=90)
        p_d = L.n_cmp * 40
        assert ev == evals_ens(p_d, 8, 6, 5, 1, n_cycle, 0)


def test_cycles_never_lower_a_sample(small_crs):
    L, bounds = small_crs
    p0, S0, _ = L.search(bounds, dict(ENS, n_cycle=0), 5, t_begin=120, t_end=200)
    p1, S1, _ = L.search(bounds, dict(ENS, n_cycle=1), 5, t_begin=120, t_end=200)
    p2, S2, _ = L.search(bounds, dict(ENS, n_cycle=2), 5, t_begin=120, t_end=200)
    assert np.all(S1 >= S0) and np.all(S2 >= S1)
    assert np.mean(S1 > S0) > 0.3
    # the reported score is the score of the reported parameters
    cmp = np.repeat(np.arange(L.n_cmp), 80)
    t = np.tile(np.arange(120, 200), L.n_cmp)
    Sr, _, _ = L.semblance(cmp, t, p2.reshape(-1, 3).astype(np.float64))
    np.testing.assert_array_equal(Sr, S2.reshape(-1))


def test_buckets_are_independent_units(small_crs):
    # a bucket processed alone reproduces its part of the whole line bitwise
    L, bounds = small_crs
    pa, Sa, _ = L.search(bounds, ENS, 11, t_begin=60, t_end=100)
    cmp_b = np.arange(4, 8, dtype=np.int32)
    pb, Sb, _ = L.search(bounds, ENS, 11, cmp_out=cmp_b, t_begin=60, t_end=100)
    np.testing.assert_array_equal(pa[4:8], pb)
    np.testing.assert_array_equal(Sa[4:8], Sb)


def _flat_mock():
    # same objective at every (t, trace): the sphere mock with t-independent bounds
    tr = np.zeros((6, 40))
    return _tiny.line(tr, [1] * 6, [100.0] * 6, window=3, op=3, ap=0)


def test_forward_injection_chain():
    # with NG_f = 0 a trace's best is the best of its random draws and of the
    # previous trace's best, which scores the same everywhere: non-decreasing
    L = _flat_mock()
    bounds = (np.array([-1.0, -1.0, -1.0], np.float32), np.array([1.0, 1.0, 1.0], np.float32), 0)
    de = dict(ENS, np_lo=6, np_hi=6, ng_f=0, n_cycle=0, n_bucket=6)
    _, S0, _ = L.search(bounds, de, 4, objective=1)
    assert np.all(np.diff(S0, axis=0) >= 0.0)
    _, Sno, _ = L.search(bounds, de, 4, objective=1, inject=0)
    assert np.any(np.diff(Sno, axis=0) < 0.0)


def test_backward_forward_seeds():
    # NG_bf = 0: after (B, F) each sample holds the max over its own best, the
    # (t-1) and (t+1) bests of the previous stage, and the previous trace's
    # best of the same sweep
    L = _flat_mock()
    bounds = (np.array([-1.0, -1.0, -1.0], np.float32), np.array([1.0, 1.0, 1.0], np.float32), 0)
    base = dict(ENS, np_lo=6, np_hi=6, ng_f=0, np_bf=5, ng_bf=0, n_bucket=6)
    _, S0, _ = L.search(bounds, dict(base, n_cycle=0), 8, objective=1)
    _, S1, _ = L.search(bounds, dict(base, n_cycle=1), 8, objective=1)
    assert np.all(S1 >= S0)
    assert np.all(S1[:, 1:] >= S0[:, :-1])     # t-1 neighbour of the previous stage
    assert np.all(S1[:, :-1] >= S0[:, 1:])     # t+1 neighbour
    assert np.all(np.diff(S1, axis=0) >= 0.0)  # last sweep runs left to right
    # the backward sweep carried the rightmost trace's best all the way left
    assert np.all(S1[0] >= S0[-1])


def test_bucket_edges_do_not_exchange():
    # the sweep restarts at each bucket: a bucket's first trace gets nothing
    # from the last trace of the bucket before it
    L = _flat_mock()
    bounds = (np.array([-1.0, -1.0, -1.0], np.float32), np.array([1.0, 1.0, 1.0], np.float32), 0)
    de = dict(ENS, np_lo=6, np_hi=6, ng_f=0, n_cycle=0, n_bucket=3)
    _, Sb, _ = L.search(bounds, de, 4, objective=1)
    _, Si, _ = L.search(bounds, de, 4, objective=1, inject=0)
    np.testing.assert_array_equal(Sb[3], Si[3])
    np.testing.assert_array_equal(Sb[0], Si[0])


# ---------------------------------------------------------------- time skipping
@pytest.mark.parametrize("n_skip", [1, 2])
def test_skip_counts_match_paper_formula(small_crs, n_skip):
    # eq. ens_semblance: ceil(P_d/(N_skip+1)) (S_f + N_cycle S_bf + (2 N_cycle + 1) N_skip),
    # exact when the grid length is a multiple of N_skip + 1
    L, bounds = small_crs
    for n_cycle in (0, 1, 2):
        de = dict(ENS, n_cycle=n_cycle, n_skip=n_skip)
        n_t = 60 if n_skip == 2 else 40
        _, _, ev = L.search(bounds, de, 3, t_begin=50, t_end=50 + n_t)
        assert ev == evals_ens(L.n_cmp * n_t, 8, 6, 5, 1, n_cycle, n_skip)


def test_skip_zero_is_the_plain_sweep(small_crs):
    L, bounds = small_crs
    a = L.search(bounds, dict(ENS, n_skip=0), 5, t_begin=100, t_end=140)
    b = L.search(bounds, ENS, 5, t_begin=100, t_end=140)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_skipped_samples_lie_between_their_neighbours():
    # stage 0 only, t-independent box: a skipped sample is the point at
    # (t - ta)/(tb - ta) along the segment joining the estimated neighbours
    L = _flat_mock()
    bounds = (np.array([-1.0, -1.0, -1.0], np.float32), np.array([1.0, 1.0, 1.0], np.float32), 0)
    de = dict(ENS, np_lo=6, np_hi=6, ng_f=1, n_cycle=0, n_bucket=6, n_skip=2)
    p, S, _ = L.search(bounds, de, 4, objective=1)
    n_t = p.shape[1]
    for o in range(p.shape[0]):
        for t in range(n_t):
            if t % 3 == 0:
                continue
            ta = t - t % 3
            tb = ta + 3
            if tb >= n_t:
                np.testing.assert_array_equal(p[o, t], p[o, ta])
                continue
            w = (t - ta) / 3.0
            ref = p[o, ta] + w * (p[o, tb] - p[o, ta])
            np.testing.assert_allclose(p[o, t], ref, rtol=0, atol=1e-6)


def test_skip_cycles_never_lower_a_sample(small_crs):
    L, bounds = small_crs
    base = dict(ENS, n_skip=2)
    _, S0, _ = L.search(bounds, dict(base, n_cycle=0), 5, t_begin=120, t_end=180)
    _, S1, _ = L.search(bounds, dict(base, n_cycle=1), 5, t_begin=120, t_end=180)
    assert np.all(S1 >= S0)
    assert np.mean(S1 > S0) > 0.3
