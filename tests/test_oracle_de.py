"""Pins of the oracle's per-domain differential evolution.

Section "JADE applied to traveltime parameter search": uniform initialisation
in the box, the best individual (P = 1), a mutant from the i-th member, the
best and two other random members, crossover, synchronous pairwise selection,
NP (1 + NG) evaluations per domain (eq. jade_semblance).
"""
import math

import numpy as np
import pytest

import oracle
from tests import _tiny

LO = np.array([0.0, -1.0, 10.0], np.float32)
HI = np.array([1.0, 1.0, 20.0], np.float32)


def _words(r1_hi, r2_lo, jr_hi, cr0, cr1, cr2):
    return [(r1_hi << 32) | r2_lo, (jr_hi << 32) | cr0, (cr1 << 32) | cr2, 0]


def test_hand_computed_step():
    pop = np.array([[0.10, 0.50, 11.0],
                    [0.20, -0.25, 15.0],
                    [0.80, 0.75, 12.0],
                    [0.40, 0.00, 19.0],
                    [0.55, -0.90, 13.5]], np.float32)
    S = np.array([0.1, 0.7, 0.3, 0.7, 0.2])   # best = 1 (lowest index of the tie)
    NO, YES = 0xFFFFFFFF, 0
    words = np.array([
        # i=0: r1 draw 1 of {1,2,3,4} -> 2; r2 draw 0 of {1,3,4} -> 1; jr 0; take d1
        _words(1 << 30, 0, 0, NO, YES, NO),
        # i=1: r1 draw 3 of {0,2,3,4} -> 4; r2 draw 2 of {0,2,3} -> 3; jr 2; take none else
        _words(3 << 30, 0xB0000000, 0xB0000000, NO, NO, NO),
        # i=2: r1 draw 0 -> 0; r2 draw 1 of {1,3,4} -> 3; jr 1; take all
        _words(0, 0x60000000, 0x60000000, YES, YES, YES),
        # i=3: r1 draw 2 of {0,1,2,4} -> 2; r2 draw 0 of {0,1,4} -> 0; jr 0
        _words(2 << 30, 0, 0, NO, NO, NO),
        # i=4: r1 draw 3 of {0,1,2,3} -> 3; r2 draw 2 of {0,1,2} -> 2; jr 2; take d0
        _words(3 << 30, 0xB0000000, 0xB0000000, YES, NO, NO),
    ], dtype=np.uint64)
    F = np.float32(0.5)
    out = oracle.de_trial(pop, S, words, F, 0.9, LO, HI)

    def mut(i, b, r1, r2, d):
        x = pop[i, d]
        v = np.float32(np.float32(x + np.float32(F * np.float32(pop[b, d] - x)))
                       + np.float32(F * np.float32(pop[r1, d] - pop[r2, d])))
        if v < LO[d]:
            v = np.float32(np.float32(LO[d] + x) * np.float32(0.5))
        elif v > HI[d]:
            v = np.float32(np.float32(HI[d] + x) * np.float32(0.5))
        return v

    exp = pop.copy()
    exp[0, 0] = mut(0, 1, 2, 1, 0)
    exp[0, 1] = mut(0, 1, 2, 1, 1)
    exp[1, 2] = mut(1, 1, 4, 3, 2)
    exp[2, :] = [mut(2, 1, 0, 3, d) for d in range(3)]
    exp[3, 0] = mut(3, 1, 2, 0, 0)
    exp[4, 0] = mut(4, 1, 3, 2, 0)
    exp[4, 2] = mut(4, 1, 3, 2, 2)
    np.testing.assert_array_equal(out, exp)
    # spot values written out by hand: i=0 d=0: 0.1 + 0.5*(0.2-0.1) + 0.5*(0.8-0.2) = 0.45
    assert abs(out[0, 0] - 0.45) < 1e-7
    # i=2 d=1: 0.75 + 0.5*(-0.25-0.75) + 0.5*(0.1... ) -> r1=0 (0.5), r2=3 (0.0): 0.5
    assert abs(out[2, 1] - 0.5) < 1e-7


def test_repair_is_midpoint_toward_parent():
    pop = np.array([[0.05, 0.0, 15.0], [0.9, 0.0, 15.0], [0.0, 0.0, 15.0], [0.95, 0.0, 15.0]],
                   np.float32)
    S = np.array([0.0, 0.0, 1.0, 0.0])  # best = 2 at the lower edge
    # i=0: r1 -> 1, r2 -> 3; v0 = .05 + .5(0 - .05) + .5(.9 - .95) = 0.0 (in box)
    # i=1: r1 draw 1 of {0,2,3} -> 2, r2 draw 1 of {0,3} -> 3:
    #      v0 = .9 + .5(0 - .9) + .5(0 - .95) = -0.025 < 0 -> (0 + .9)/2
    words = np.array([_words(0, 0, 0, 0, 0xFFFFFFFF, 0xFFFFFFFF),
                      _words(1 << 31, 0x80000000, 0, 0, 0xFFFFFFFF, 0xFFFFFFFF),
                      _words(0, 0, 0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF),
                      _words(0, 0, 0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF)], np.uint64)
    out = oracle.de_trial(pop, S, words, 0.5, 0.9, LO, HI)
    assert out[1, 0] == np.float32(0.45)
    assert LO[0] <= out[0, 0] <= HI[0]


def test_index_draws_distinct_and_uniform():
    rng = np.random.default_rng(11)
    npop, P = 7, 3
    # coordinates 50 + i/4: every DE operation below is exact in binary32
    pop = np.repeat((50.0 + 0.25 * np.arange(npop, dtype=np.float32))[:, None], P, axis=1)
    lo = np.zeros(3, np.float32)
    hi = np.full(3, 100.0, np.float32)
    S = np.zeros(npop)
    S[0] = 1.0  # best = 0: with F = 1, CR = 1 the trial is x_r1 - x_r2 + x_0
    counts = np.zeros((npop, npop, npop))
    for _ in range(3000):
        words = rng.integers(0, 2 ** 63, size=(npop, 4), dtype=np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, size=(npop, 4), dtype=np.uint64)
        out = oracle.de_trial(pop, S, words, 1.0, 1.0, lo, hi)
        diff = np.rint((out[:, 0] - pop[0, 0]) / np.float32(0.25)).astype(int)  # r1 - r2
        for i in range(npop):
            w0 = int(words[i, 0])
            r1 = ((w0 >> 32) * (npop - 1)) >> 32
            r1 += r1 >= i
            assert r1 != i
            r2 = r1 - diff[i]
            assert r2 != i and r2 != r1
            counts[i, r1, r2] += 1
    # every ordered pair of distinct indices other than i appears about equally often
    for i in range(npop):
        c = counts[i][counts[i] > 0]
        assert c.size == (npop - 1) * (npop - 2)
        chi2 = ((c - c.mean()) ** 2 / c.mean()).sum()
        assert chi2 < 80  # dof 29: p < 1e-6 above this


def test_zero_F_returns_parent_and_cr_zero_changes_one_dim():
    rng = np.random.default_rng(12)
    pop = rng.random((6, 3)).astype(np.float32)
    S = rng.random(6)
    words = rng.integers(0, 2 ** 63, size=(6, 4), dtype=np.uint64)
    out = oracle.de_trial(pop, S, words, 0.0, 0.9, np.zeros(3, np.float32), np.ones(3, np.float32))
    np.testing.assert_array_equal(out, pop)
    out = oracle.de_trial(pop, S, words, 0.5, 0.0, np.zeros(3, np.float32), np.ones(3, np.float32))
    assert np.all((out != pop).sum(axis=1) <= 1)
    jr = ((words[:, 1] >> np.uint64(32)) * np.uint64(3)) >> np.uint64(32)
    for i in range(6):
        same = [d for d in range(3) if d != jr[i]]
        np.testing.assert_array_equal(out[i, same], pop[i, same])


def _mock_line(op=1, n_cmp=3, nt=64, dt=0.004):
    tr = np.zeros((n_cmp, nt))
    return _tiny.line(tr, [1] * n_cmp, [100.0] * n_cmp, dt=dt, window=3, op=op, ap=0)


DE = dict(np_lo=16, np_hi=16, ng_f=60, np_bf=5, ng_bf=1, n_cycle=0, n_bucket=8,
          ens_enabled=0, F=0.5, CR=0.9)


def test_eval_count_and_sphere_convergence():
    L = _mock_line(op=3)
    bounds = (np.array([-1.0, -2.0, 0.0], np.float32), np.array([1.0, 2.0, 5.0], np.float32), 0)
    params, S, ev = L.search(bounds, DE, seed=3, t_begin=10, t_end=30, objective=1)
    assert ev == 3 * 20 * 16 * (1 + 60)            # P_d NP (1 + NG)
    # DE can stall on a few domains: nearly all converge, none stays far off
    assert np.mean(S > 0.999) > 0.95 and S.min() > 0.95
    z = (params - bounds[0]) / (bounds[1] - bounds[0])
    assert np.median(np.abs(z - np.array([0.3, 0.4, 0.5])).max(axis=-1)) < 0.005


def test_initial_population_spans_box():
    # NG = 0: the result is the best of NP uniform draws; over many samples
    # the normalised coordinates fill [0,1) without leaving it
    L = _mock_line(op=3, n_cmp=20, nt=400)
    de = dict(DE, np_lo=4, np_hi=4, ng_f=0)
    bounds = (np.array([-1.0, -2.0, 0.0], np.float32), np.array([1.0, 2.0, 5.0], np.float32), 0)
    params, S, ev = L.search(bounds, de, seed=5, objective=1)
    assert ev == 20 * 400 * 4
    z = (params.reshape(-1, 3) - bounds[0]) / (bounds[1] - bounds[0])
    assert z.min() >= 0.0 and z.max() <= 1.0
    assert z.min() < 0.02 and z.max() > 0.98


def test_scale_invariance_power_of_two():
    # bounds given for (A, B t0, C t0) and divided by t0 = 2^-k per sample are
    # an exact per-coordinate rescale: the same draws give bitwise scaled results
    dt = 2.0 ** -8
    L = _mock_line(op=3, nt=300, dt=dt)
    lo = np.array([-1.0, -2.0, 0.5], np.float32)
    hi = np.array([1.0, 2.0, 5.0], np.float32)
    de = dict(DE, ng_f=20)
    for n0 in (64, 128, 256):
        t0 = n0 * dt
        pa, Sa, _ = L.search((lo, hi, 0b110), de, 9, t_begin=n0, t_end=n0 + 1, objective=1)
        pb, Sb, _ = L.search((lo, hi, 0), de, 9, t_begin=n0, t_end=n0 + 1, objective=1)
        np.testing.assert_array_equal(Sa, Sb)
        np.testing.assert_array_equal(pa[..., 0], pb[..., 0])
        np.testing.assert_array_equal(pa[..., 1:] * np.float32(t0), pb[..., 1:])


def test_selection_keeps_parents_on_loss():
    # NG generations never lower any slot's score; with the needle objective
    # (zero almost everywhere) nothing better is found from a zero start and
    # the result stays a valid in-box individual
    L = _mock_line(op=1)
    bounds = (np.array([0.0, 0, 0], np.float32), np.array([1.0, 0, 0], np.float32), 0)
    de = dict(DE, np_lo=8, np_hi=8, ng_f=5)
    params, S, ev = L.search(bounds, de, seed=2, t_begin=0, t_end=64, objective=2)
    assert set(np.unique(S)).issubset({0.0, 1.0})
    assert np.all((params >= 0) & (params <= 1))
    assert ev == 3 * 64 * 8 * 6


@pytest.mark.parametrize("cr", [0.0, 0.25, 0.9, 1.0])
def test_crossover_threshold_exact(cr):
    # dimension d is taken from the mutant iff its 32-bit draw < ceil(CR 2^32)
    thr = math.ceil(float(np.float32(cr)) * 2 ** 32)
    pop = np.array([[0.1, 0.1, 11.0], [0.9, 0.9, 19.0], [0.5, 0.5, 15.0], [0.3, 0.3, 13.0]],
                   np.float32)
    S = np.array([0.0, 1.0, 0.0, 0.0])
    for draw in {0, max(thr - 1, 0), min(thr, 0xFFFFFFFF), 0xFFFFFFFF}:
        words = np.array([_words(0, 0, 0xFFFFFFFF, 0xFFFFFFFF, draw, 0xFFFFFFFF)] * 4, np.uint64)
        out = oracle.de_trial(pop, S, words, 0.5, cr, LO, HI)
        # jr = 2 for all slots, dimension 1 is the probe
        assert (out[0, 1] != pop[0, 1]) == (draw < thr)
