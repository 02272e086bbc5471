"""Pins of the oracle's zero-offset stack and panel RMS (the quality outputs of
sections "Qualitative analysis" and "Quantitative analysis")."""
import numpy as np

import oracle
from tests import _tiny

DT = float(np.float32(0.004))  # the line holds dt in binary32


def _affine_line(tau, level, slope, nt=200, cmp_sizes=None, offsets=None, op=1, ap=0, dx=12.5):
    """Traces that are affine in time through each trace's own traveltime:
    u_i[n] = level_i + slope_i (n - tau_i).  Linear interpolation is exact for
    affine data, so the interpolated amplitude at tau_i is level_i exactly."""
    n = np.arange(nt, dtype=np.float64)
    tr = level[:, None] + slope[:, None] * (n[None, :] - tau[:, None])
    sizes = cmp_sizes if cmp_sizes is not None else [len(tau)]
    offs = offsets if offsets is not None else np.zeros(len(tau))
    return _tiny.line(tr, sizes, offs, dt=DT, dx=dx, window=5, op=op, ap=ap)


def test_cmp_stack_is_the_fold_mean_of_the_levels():
    # CMP operator t^2 = t0^2 + C h^2 with C = 1/v^2; each trace's own level
    h = np.array([100.0, 300.0, 500.0, 700.0, 900.0])
    v, n0 = 2000.0, 80
    C = 1.0 / v ** 2
    tau = np.sqrt((n0 * DT) ** 2 + C * h ** 2) / DT
    rng = np.random.default_rng(0)
    level, slope = rng.normal(size=5), rng.normal(size=5)
    L = _affine_line(tau, level, slope, offsets=h)
    st, M = L.stack([0], [n0], [[C]])
    assert M[0] == 5
    np.testing.assert_allclose(st[0], level.mean(), rtol=0, atol=1e-12)
    # a wrong operator picks other amplitudes on the sloped traces
    st_wrong, _ = L.stack([0], [n0], [[C * 1.2]])
    assert abs(st_wrong[0] - level.mean()) > 1e-3


def test_traces_past_the_record_leave_the_fold():
    # long offsets at a late t0 fall past nt-1 and are excluded from M and the mean
    h = np.array([100.0, 400.0, 1600.0, 3200.0])
    v, n0, nt = 1500.0, 180, 200
    C = 1.0 / v ** 2
    tau = np.sqrt((n0 * DT) ** 2 + C * h ** 2) / DT
    inside = tau <= nt - 1
    assert inside.sum() == 2
    level = np.array([1.0, 2.0, 10.0, 20.0])
    L = _affine_line(np.minimum(tau, nt - 1), level, np.zeros(4), nt=nt, offsets=h)
    st, M = L.stack([0], [n0], [[C]])
    assert M[0] == 2
    np.testing.assert_allclose(st[0], 1.5, rtol=0, atol=1e-12)


def test_empty_fold_stacks_to_zero():
    # C < 0 with long offsets: t^2 < 0 for every trace
    h = np.array([1000.0, 2000.0])
    L = _affine_line(np.array([10.0, 10.0]), np.ones(2), np.zeros(2), offsets=h)
    st, M = L.stack([0], [5], [[-1e-3]])
    assert M[0] == 0 and st[0] == 0.0


def test_crs_stack_uses_the_midpoint_terms():
    # three CMPs (aperture 1) of two offsets each; CRS traveltimes with A, B, C
    dx, n0 = 25.0, 60
    A, B, C = 4e-4, 3e-7, 2.0e-7
    t0 = n0 * DT
    cmp_of = np.repeat(np.arange(3), 2)
    h = np.tile([200.0, 600.0], 3)
    dm = (cmp_of - 1) * dx
    tau = np.sqrt((t0 + A * dm) ** 2 + B * t0 * dm ** 2 + C * t0 * h ** 2) / DT
    rng = np.random.default_rng(1)
    level, slope = rng.normal(size=6), 0.5 + rng.random(6)
    L = _affine_line(tau, level, slope, cmp_sizes=[2, 2, 2], offsets=h, op=3, ap=1, dx=dx)
    st, M = L.stack([1], [n0], [[A, B, C]])
    assert M[0] == 6
    np.testing.assert_allclose(st[0], level.mean(), rtol=0, atol=1e-12)
    # the sign of the A dm term matters
    st_neg, _ = L.stack([1], [n0], [[-A, B, C]])
    assert abs(st_neg[0] - level.mean()) > 1e-3


def test_stack_is_linear_in_the_data_and_ignores_trace_order():
    rng = np.random.default_rng(2)
    tr = rng.normal(size=(6, 120))
    h = np.array([100.0, 200.0, 300.0, 400.0, 500.0, 600.0])
    L1 = _tiny.line(tr, [6], h, dt=DT, window=5, op=1)
    L2 = _tiny.line(3.5 * tr, [6], h, dt=DT, window=5, op=1)
    perm = rng.permutation(6)
    L3 = _tiny.line(tr[perm], [6], h[perm], dt=DT, window=5, op=1)
    t = np.arange(10, 110, dtype=np.int32)
    p = np.full((t.size, 1), 1 / 2200.0 ** 2)
    cmp = np.zeros(t.size, np.int32)
    a, _ = L1.stack(cmp, t, p)
    b, _ = L2.stack(cmp, t, p)
    c, _ = L3.stack(cmp, t, p)
    np.testing.assert_allclose(b, 3.5 * a, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(c, a, rtol=1e-12, atol=1e-14)


def test_rms_closed_forms():
    assert oracle.rms([3.0, 4.0]) == np.sqrt(12.5)
    assert oracle.rms(np.full(7, -2.5)) == 2.5
    assert oracle.rms(np.zeros(0)) == 0.0
