"""Pins of the oracle's traveltime / gather / semblance against closed forms.

The paper fixes only the range of the objective (eqs. f and S: values in
[0,1]); the rest follows from the standard semblance definition and the
exactness of linear interpolation on affine signals.
"""
import numpy as np
import pytest

import oracle
from synth import make_workload, random_candidates, base_bounds
from tests import _tiny

DT = 0.004


def _tau(t0, C, h):
    return np.sqrt(t0 * t0 + C * h * h) / np.float64(np.float32(DT))


def _event_line(offsets, nt, n0, C, profile, window=5):
    """One CMP whose trace i holds profile(m - tau_i) for |m - tau_i| <= 6."""
    dt = float(np.float32(DT))
    tr = np.zeros((len(offsets), nt))
    m = np.arange(nt)
    for i, h in enumerate(offsets):
        tau = np.sqrt((n0 * dt) ** 2 + C * h * h) / dt
        x = m - tau
        tr[i] = np.where(np.abs(x) <= 6.0, profile(x), 0.0)
    return _tiny.line(tr, [len(offsets)], offsets, dt=DT, window=window)


def test_range_random_inputs():
    g, wl = make_workload("cmp_small")
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    cmp, t, p = random_candidates(20000, g.n_cmp, g.nt, g.dt, 1, base_bounds(wl), seed=3,
                                  spread=3.0)
    S, M, _ = L.semblance(cmp, t, p)
    assert np.all(S >= 0.0) and np.all(S <= 1.0 + 1e-15)
    assert np.any(M == 0) or True
    assert S.max() > 0.5  # the events are found by some random candidates


def test_range_crs_random():
    g, wl = make_workload("crs_ens", n_cmp=24, snr=1.0)
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    cmp, t, p = random_candidates(4000, g.n_cmp, g.nt, g.dt, 3, base_bounds(wl), seed=4,
                                  spread=2.0)
    S, M, _ = L.semblance(cmp, t, p)
    assert np.all(S >= 0.0) and np.all(S <= 1.0 + 1e-15)
    assert np.all(M <= 17 * 48)


@pytest.mark.parametrize("n0", [40, 75])
def test_constant_event_scores_one(n0):
    C = 1.0 / 2000.0 ** 2
    offs = [25.0, 150.0, 310.0, 475.0, 600.0]
    L = _event_line(offs, 256, n0, C, lambda x: np.ones_like(x))
    S, M, _ = L.semblance([0], [n0], [[C]])
    assert M[0] == len(offs)
    assert abs(1.0 - S[0]) <= 1e-12


def test_linear_ramp_event_scores_one():
    # lerp reproduces an affine signal exactly for any fractional traveltime,
    # so every trace contributes the window 2 + 0.3 k; swapped weights would not
    C = 1.0 / 1800.0 ** 2
    offs = [25.0, 137.0, 260.0, 333.0, 480.0, 590.0]
    L = _event_line(offs, 256, 60, C, lambda x: 2.0 + 0.3 * x)
    S, M, _ = L.semblance([0], [60], [[C]])
    assert M[0] == len(offs)
    assert abs(1.0 - S[0]) <= 1e-12
    # off the true operator the windows differ and S drops
    S2, _, _ = L.semblance([0], [60], [[C * 1.3]])
    assert S2[0] < 1.0 - 1e-4


def test_one_live_trace_gives_one_over_M():
    rng = np.random.default_rng(5)
    tr = np.zeros((7, 128))
    tr[3] = rng.standard_normal(128)
    L = _tiny.line(tr, [7], np.linspace(25, 400, 7), window=5)
    S, M, _ = L.semblance([0], [50], [[1.0 / 2500.0 ** 2]])
    assert M[0] == 7
    assert abs(S[0] - 1.0 / 7.0) <= 1e-12


def test_opposite_sign_pair_cancels():
    rng = np.random.default_rng(6)
    a = rng.standard_normal(128)
    tr = np.stack([a, -a])
    L = _tiny.line(tr, [2], [200.0, 200.0], window=5)
    S, M, _ = L.semblance([0], [40], [[1.0 / 2000.0 ** 2]])
    assert M[0] == 2 and abs(S[0]) <= 1e-12


def test_single_trace_scores_one():
    rng = np.random.default_rng(7)
    L = _tiny.line(rng.standard_normal((1, 128)), [1], [300.0], window=7)
    S, M, _ = L.semblance([0], [50], [[1.0 / 2200.0 ** 2]])
    assert M[0] == 1 and abs(S[0] - 1.0) <= 1e-12


def test_scale_and_permutation_invariance():
    g, wl = make_workload("crs_ens", n_cmp=20, snr=2.0)
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    cmp, t, p = random_candidates(500, g.n_cmp, g.nt, g.dt, 3, base_bounds(wl), seed=8,
                                  cmp_range=(6, 14))
    S, _, _ = L.semblance(cmp, t, p)
    L2 = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"],
                                 traces=g.traces.astype(np.float64) * 3.7)
    S2, _, _ = L2.semblance(cmp, t, p)
    assert np.max(np.abs(S - S2)) <= 1e-12
    # reverse the trace order inside every CMP (offsets travel with their traces)
    perm = np.concatenate([np.arange(g.cmp_ptr[c], g.cmp_ptr[c + 1])[::-1]
                           for c in range(g.n_cmp)])
    L3 = oracle.Line(g.traces[perm], g.cmp_ptr, g.offset[perm], g.dt, g.dx, wl["window"],
                     wl["op"], wl["ap_lo"], wl["ap_hi"])
    S3, _, _ = L3.semblance(cmp, t, p)
    assert np.max(np.abs(S - S3)) <= 1e-12


@pytest.mark.parametrize("shift,expect", [(2, 1.0), (3, 0.0), (-2, 1.0), (-3, 0.0)])
def test_window_is_centred(shift, expect):
    # C = 0 puts every trace's traveltime exactly on sample n0 (f = 0); a
    # spike at n0 + shift is inside a centred 5-sample window iff |shift| <= 2
    n0 = 50
    tr = np.zeros((4, 128))
    tr[:, n0 + shift] = 1.0
    L = _tiny.line(tr, [4], [100.0, 200.0, 300.0, 400.0], window=5)
    S, M, _ = L.semblance([0], [n0], [[0.0]])
    assert M[0] == 4
    assert abs(S[0] - expect) <= 1e-12


def test_excluded_traces_do_not_count():
    # the far trace's traveltime falls past the record end: M = 2, S = 1
    C = 1.0 / 2000.0 ** 2
    L = _event_line([100.0, 200.0, 5000.0], 200, 60, C, lambda x: np.ones_like(x))
    S, M, _ = L.semblance([0], [60], [[C]])
    assert M[0] == 2
    assert abs(S[0] - 1.0) <= 1e-12
    # nothing participates at all: S = 0
    S0, M0, _ = L.semblance([0], [60], [[1.0]])
    assert M0[0] == 0 and S0[0] == 0.0


def test_samples_outside_record_read_zero():
    # t0 = 0, C = 0: tau = 0 on both traces, the window reads samples -2..3;
    # a wrap into the previous trace's last sample would break S = 1
    nt = 64
    tr = np.zeros((2, nt))
    tr[:, 0] = 1.0
    tr[0, nt - 1] = 5.0
    tr[1, nt - 1] = 0.0
    L = _tiny.line(tr, [2], [100.0, 200.0], window=5)
    S, M, _ = L.semblance([0], [0], [[0.0]])
    assert M[0] == 2 and abs(S[0] - 1.0) <= 1e-12
    # and at the last sample the window runs past the end
    tr2 = np.zeros((2, nt))
    tr2[:, nt - 1] = 1.0
    tr2[1, 0] = 7.0
    L2 = _tiny.line(tr2, [2], [100.0, 200.0], window=5)
    S2, M2, _ = L2.semblance([0], [nt - 1], [[0.0]])
    assert M2[0] == 2 and abs(S2[0] - 1.0) <= 1e-12


def test_crs_operator_uses_neighbour_cmps():
    # three CMPs, one trace each at the same offset; with A = B = C = 0 the
    # traveltime is t0 everywhere, so identical traces give 1 when the
    # aperture covers them and the outer traces are ignored when it does not
    rng = np.random.default_rng(9)
    a = rng.standard_normal(128)
    b = rng.standard_normal(128)
    tr = np.stack([b, a, a])
    L1 = _tiny.line(tr, [1, 1, 1], [100.0, 100.0, 100.0], window=5, op=3, ap=1)
    S1, M1, _ = L1.semblance([2], [60], [[0.0, 0.0, 0.0]])
    assert M1[0] == 2 and abs(S1[0] - 1.0) <= 1e-12  # CMPs 1, 2 (CMP 3 does not exist)
    L0 = _tiny.line(tr, [1, 1, 1], [100.0, 100.0, 100.0], window=5, op=3, ap=0)
    S0, M0, _ = L0.semblance([0], [60], [[0.0, 0.0, 0.0]])
    assert M0[0] == 1 and abs(S0[0] - 1.0) <= 1e-12


def test_crs_midpoint_term_sign():
    # a planar dipping event (exact Levin moveout) is fitted by A = 2 sin/v,
    # B = 0, C t0 = cos^2/v^2; the opposite sign of A scores clearly lower
    v, th = 2000.0, np.radians(10.0)
    dt = float(np.float32(DT))
    n_cmp, dx, nt, n0, jc = 9, 12.5, 200, 70, 4
    offs = np.array([50.0, 150.0, 250.0])
    tr = []
    for c in range(n_cmp):
        t0m = n0 * dt + 2.0 * (c - jc) * dx * np.sin(th) / v
        for h in offs:
            tau = np.sqrt(t0m ** 2 + (h * np.cos(th) / v) ** 2) / dt
            x = np.arange(nt) - tau
            tr.append(np.where(np.abs(x) <= 6, 1.0 + 0.2 * x, 0.0))
    L = _tiny.line(np.array(tr), [3] * n_cmp, np.tile(offs, n_cmp), window=5, op=3, ap=4)
    t0 = n0 * dt
    p = [2 * np.sin(th) / v, 0.0, np.cos(th) ** 2 / v ** 2 / t0]
    S, M, _ = L.semblance([jc], [n0], [p])
    assert M[0] == 27 and abs(S[0] - 1.0) <= 1e-12
    Sm, _, _ = L.semblance([jc], [n0], [[-p[0], p[1], p[2]]])
    assert Sm[0] < 0.9


def _ricker_line(dt, w, f=25.0, C=1.0 / 2000.0 ** 2, t0=0.4):
    dt = float(np.float32(dt))
    offs = np.linspace(25.0, 600.0, 24)
    nt = int(round(1.0 / dt))
    tr = np.zeros((offs.size, nt))
    tt = np.arange(nt) * dt
    for i, h in enumerate(offs):
        te = np.sqrt(t0 * t0 + C * h * h)
        a = (np.pi * f * (tt - te)) ** 2
        tr[i] = (1.0 - 2.0 * a) * np.exp(-a)
    L = oracle.Line(tr, np.array([0, offs.size]), offs, dt, 12.5, 2 * w + 1, 1)
    n0 = int(round(t0 / L.dt))
    return L, n0, C


def test_ricker_interpolation_error_converges():
    # lerp error is O(dt^2) per sample; semblance loss is its squared spread
    # across traces, O(dt^4): halving dt (same window duration) cuts 1 - S ~16x
    L1, n1, C = _ricker_line(0.004, 2)
    L2, n2, _ = _ricker_line(0.002, 4)
    S1, _, _ = L1.semblance([0], [n1], [[C]])
    S2, _, _ = L2.semblance([0], [n2], [[C]])
    r = (1.0 - S1[0]) / (1.0 - S2[0])
    assert 1.0 - S1[0] < 1e-2
    assert 10.0 < r < 24.0, r
