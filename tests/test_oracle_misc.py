"""Pins of the oracle's gradient, polish, quantiser, reference maximum and
parameter recovery on tiny noise-free gathers."""
import numpy as np
import pytest
import torch

import oracle
from synth import make_gather, make_workload, random_candidates, base_bounds
from tests import _tiny


# ---------------------------------------------------------------- generator
def test_philox_matches_numpy():
    # numpy's Philox bit generator is Philox-4x64-10; it advances its counter
    # by one before producing a block, so block(c) == numpy(counter=c-1)
    rng = np.random.default_rng(1)
    for _ in range(200):
        key = rng.integers(0, 2 ** 64, size=2, dtype=np.uint64)
        ctr = rng.integers(0, 2 ** 64, size=4, dtype=np.uint64)
        ctr[0] = max(int(ctr[0]), 1)
        ref = np.random.Philox(key=key, counter=np.array([ctr[0] - np.uint64(1), *ctr[1:]],
                                                         dtype=np.uint64)).random_raw(4)
        np.testing.assert_array_equal(oracle.philox4x64_10(ctr, key), ref)


# ---------------------------------------------------------------- gradient
def _fd_check(L, cmp, t, p, rel=1e-4):
    S0, g = L.semblance_grad(cmp, t, p)
    ok = rej = 0
    for c in range(len(cmp)):
        for d in range(L.op):
            # small enough that a stencil rarely straddles an integer traveltime
            # of any of the hundreds of aperture traces (a kink of the lerp)
            step = 1e-7 * abs(p[c, d]) if p[c, d] != 0 else 1e-13
            fds = []
            for hstep in (step, step / 2):
                pp, pm = p[c].copy(), p[c].copy()
                pp[d] += hstep
                pm[d] -= hstep
                Sp, Mp, _ = L.semblance([cmp[c]], [t[c]], [pp])
                Sm, Mm, _ = L.semblance([cmp[c]], [t[c]], [pm])
                if Mp[0] != Mm[0]:
                    fds = None
                    break
                fds.append((Sp[0] - Sm[0]) / (2 * hstep))
            scale = max(abs(fds[0]) if fds else 0.0, 1e-6)
            if fds is None or abs(fds[0] - fds[1]) > 1e-5 * scale:
                rej += 1  # a kink of the interpolant lies inside the stencil
                continue
            assert abs(g[c, d] - fds[1]) <= rel * scale + 1e-7, (c, d, g[c, d], fds)
            ok += 1
    return ok, rej


def test_gradient_matches_finite_differences():
    g, wl = make_workload("crs_ens", n_cmp=20, nt=400, snr=3.0)
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    cmp, t, p = random_candidates(60, g.n_cmp, g.nt, g.dt, 3, base_bounds(wl), seed=13,
                                  cmp_range=(4, 16), t_range=(100, 380))
    ok, rej = _fd_check(L, cmp, t, p.astype(np.float64))
    assert ok >= 100 and rej < ok


def test_gradient_cmp_operator_fd():
    g, wl = make_workload("cmp_small")
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    cmp, t, p = random_candidates(80, g.n_cmp, g.nt, g.dt, 1, base_bounds(wl), seed=14,
                                  t_range=(20, 240))
    ok, rej = _fd_check(L, cmp, t, p.astype(np.float64))
    assert ok >= 50


def test_gradient_vanishes_at_exact_fit():
    # linear-ramp event on the true operator: S = 1 is the maximum, and with
    # no traveltime on an integer sample the semblance is smooth there
    dt = float(np.float32(0.004))
    C = 1.0 / 1900.0 ** 2
    offs = np.array([37.0, 151.0, 263.0, 377.0, 489.0])
    n0 = 55
    tr = np.zeros((offs.size, 200))
    for i, h in enumerate(offs):
        tau = np.sqrt((n0 * dt) ** 2 + C * h * h) / dt
        assert abs(tau - round(tau)) > 0.01
        x = np.arange(200) - tau
        tr[i] = np.where(np.abs(x) <= 6, 1.0 + 0.25 * x, 0.0)
    L = _tiny.line(tr, [offs.size], offs, window=5)
    S, gr = L.semblance_grad([0], [n0], [[C]])
    assert abs(S[0] - 1.0) < 1e-12
    assert abs(gr[0, 0]) * C < 1e-9


# ---------------------------------------------------------------- polish
def test_polish_never_lowers_and_usually_raises():
    g, wl = make_workload("crs_ens", n_cmp=16, nt=500, snr=3.0)
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    bounds = base_bounds(wl)
    de = dict(wl["de"], np_lo=8, np_hi=8, ng_f=4, n_cycle=0, ens_enabled=0)
    params, S, _ = L.search(bounds, de, 5, cmp_out=np.arange(6, 10), t_begin=100, t_end=400)
    cmp = np.repeat(np.arange(6, 10), 300)
    t = np.tile(np.arange(100, 400), 4)
    p_out, S_out = L.polish(bounds, cmp, t, params.reshape(-1, 3), 0.01, 10)
    S_in = S.reshape(-1)
    assert np.all(S_out >= S_in)
    assert np.mean(S_out > S_in + 1e-6) > 0.3
    Sr, _, _ = L.semblance(cmp, t, p_out)
    np.testing.assert_array_equal(Sr, S_out)


# ---------------------------------------------------------------- quantiser
def _awkward_values(n=4096, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((8, n)).astype(np.float32) * np.exp(rng.normal(0, 3, (8, 1)))
    x[1, :64] = np.float32(1e-6) * rng.standard_normal(64)  # binary16 subnormal range
    x[2] = 0.0                                               # all-zero trace -> scale 1
    x[3, :20] = np.float32(2.0 ** -14) * (1 + np.arange(20) / 2048.0)  # ties near the edge
    return x.astype(np.float32)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_quantiser_matches_library_rounding(dtype):
    u = _awkward_values()
    q, s = oracle.quantize(u, dtype)
    peak = np.abs(u).max(axis=1).astype(np.float64)
    # the scale is a power of two with peak <= s < 2 peak (1 for the zero trace)
    mant, _ = np.frexp(s)
    assert np.all(mant == 0.5)
    nz = peak > 0
    assert np.all((peak[nz] <= s[nz]) & (s[nz] < 2 * peak[nz])) and np.all(s[~nz] == 1.0)
    s_ref = s
    x = (u / s_ref[:, None]).astype(np.float32)
    # division by a power of two is exact (no binary32 underflow here)
    np.testing.assert_array_equal(x.astype(np.float64) * s_ref[:, None], u.astype(np.float64))
    if dtype == "f16":
        ref = x.astype(np.float16).view(np.uint16)          # numpy: round to nearest even
    else:
        ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(q, ref)


@pytest.mark.parametrize("dtype,unit", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_quantiser_error_bound(dtype, unit):
    u = _awkward_values(seed=3)
    q, s = oracle.quantize(u, dtype)
    back = oracle.dequantize(q, s, dtype)
    x = u.astype(np.float64)
    bound = s[:, None].astype(np.float64) * np.maximum(np.abs(x) / s[:, None] * unit, 2.0 ** -25) \
        + np.abs(x) * 2.0 ** -24
    assert np.all(np.abs(back - x) <= bound)


# ---------------------------------------------------------------- recovery
def test_cmp_brute_force_recovers_velocity():
    v = 2000.0
    g = make_gather(1, 12.5, np.arange(25.0, 601.0, 25.0), 256, 0.004,
                    [dict(kind="flat", t0=0.5, v=v)], 25.0, None, 1, noise=False)
    L = oracle.Line.from_gather(g, 5, 1)
    n0 = 125  # t0 = 0.5 s
    grid = np.linspace(1 / 4000 ** 2, 1 / 1500 ** 2, 2001)
    S, _, _ = L.semblance(np.zeros(grid.size, np.int32), np.full(grid.size, n0, np.int32),
                          grid[:, None])
    best = grid[np.argmax(S)]
    assert abs(best - 1 / v ** 2) <= grid[1] - grid[0]
    assert S.max() > 0.999


def test_crs_brute_force_recovers_planar_dip():
    v, dip = 2000.0, 10.0
    dt = 0.004
    n0 = 60
    g = make_gather(17, 12.5, np.arange(25.0, 201.0, 25.0), 128, dt,
                    [dict(kind="planar", dip_deg=dip, t0=n0 * float(np.float32(dt)))], 30.0,
                    None, 1, v=v, noise=False)
    L = oracle.Line.from_gather(g, 5, 3, ap_lo=8, ap_hi=8)
    th = np.radians(dip)
    t0 = n0 * L.dt
    truth = np.array([2 * np.sin(th) / v, 0.0, np.cos(th) ** 2 / v ** 2 / t0])
    S_t, M_t, _ = L.semblance([8], [n0], [truth])
    assert M_t[0] == 17 * 8 and S_t[0] > 0.995
    bounds = (np.array([-1e-3, -2e-6, 1 / 4000 ** 2], np.float32),
              np.array([1e-3, 2e-6, 1 / 1500 ** 2], np.float32), 0b110)
    # fine brute-force grid over the box
    lo, hi = L.sample_bounds(bounds, n0)
    axes = [np.linspace(lo[d], hi[d], n) for d, n in enumerate((81, 21, 81))]
    P = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, 3)
    S, _, _ = L.semblance(np.full(len(P), 8, np.int32), np.full(len(P), n0, np.int32), P)
    pb = P[np.argmax(S)]
    steps = [a[1] - a[0] for a in axes]
    assert abs(pb[0] - truth[0]) <= steps[0]
    assert abs(pb[2] - truth[2]) <= 2 * steps[2]
    # traveltime-equivalent check of the whole vector at the far trace: dt/10
    def tt(p, dm, h):
        return np.sqrt((t0 + p[0] * dm) ** 2 + p[1] * t0 * dm ** 2 + p[2] * t0 * h ** 2)
    for dm in (-100.0, 0.0, 100.0):
        assert abs(tt(pb, dm, 200.0) - tt(truth, dm, 200.0)) < L.dt / 10 + 1e-12
    # the reference maximum finds at least the brute-force maximum (within 1e-4)
    S_ref, p_ref = L.sref(bounds, [8], [n0], (25, 9, 33), n_refine=8)
    assert S_ref[0] >= S.max() - 1e-4
    assert S_ref[0] >= S_t[0] - 1e-4


def test_sref_against_fine_brute_force_cmp():
    g, wl = make_workload("cmp_small")
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    bounds = base_bounds(wl)
    cmp = np.array([0, 3, 7, 11, 15, 5], np.int32)
    t = np.array([75, 137, 200, 40, 230, 100], np.int32)
    S_ref, p_ref = L.sref(bounds, cmp, t, (2049,), n_refine=3)
    fine = np.linspace(bounds[0][0], bounds[1][0], 40001)
    for c in range(len(cmp)):
        S, _, _ = L.semblance(np.full(fine.size, cmp[c], np.int32),
                              np.full(fine.size, t[c], np.int32), fine[:, None])
        assert S_ref[c] >= S.max() - 1e-4
        assert S_ref[c] <= 1.0


# ---------------------------------------------------------------- traveltime sensitivity
def test_traveltime_sensitivity_is_the_sum_of_per_trace_derivatives():
    # per-trace derivatives by finite differences of the oracle's S in each
    # trace's offset alone (CMP operator: dtau_i/dh_i = C h_i / (t_i dt))
    rng = np.random.default_rng(5)
    nt, dt = 160, float(np.float32(0.004))
    offs = np.sort(rng.uniform(50.0, 900.0, 10))
    kern = np.exp(-0.5 * (np.arange(-6, 7) / 2.0) ** 2)
    tr = np.array([np.convolve(rng.standard_normal(nt), kern, mode="same") for _ in offs])
    C, n0 = 1.0 / 2200.0 ** 2, 70
    L = _tiny.line(tr, [offs.size], offs, dt=dt, window=7)
    l1 = L.tau_sensitivity([0], [n0], [[C]])[0]
    total, checked = 0.0, 0
    for i, h in enumerate(offs):
        t_i = np.sqrt((n0 * dt) ** 2 + C * h * h)
        dtau_dh = C * h / (t_i * dt)
        fd = []
        for eps in (1e-6 * h, 0.5e-6 * h):
            op, om = offs.copy(), offs.copy()
            op[i] += eps
            om[i] -= eps
            Sp = _tiny.line(tr, [offs.size], op, dt=dt, window=7).semblance([0], [n0], [[C]])[0][0]
            Sm = _tiny.line(tr, [offs.size], om, dt=dt, window=7).semblance([0], [n0], [[C]])[0][0]
            fd.append((Sp - Sm) / (2 * eps) / dtau_dh)
        assert abs(fd[0] - fd[1]) <= 1e-4 * max(abs(fd[1]), 1e-6)   # no interpolation kink inside
        total += abs(fd[1])
        checked += 1
    assert checked == offs.size and l1 > 0
    assert abs(l1 - total) <= 1e-5 * total


def test_traveltime_sensitivity_vanishes_for_one_trace_and_bounds_the_gradient():
    # M = 1: S = 1 whatever the traveltime
    tr = np.sin(np.arange(100) * 0.3)[None, :]
    L1 = _tiny.line(tr, [1], [300.0], window=5)
    assert L1.tau_sensitivity([0], [40], [[1.0 / 2000.0 ** 2]])[0] == 0.0
    # chain rule and the triangle inequality: |dS/dC| <= max_i dtau_i/dC * sum_i |dS/dtau_i|,
    # and dtau_i/dC = h_i^2 / (2 t_i dt) <= h_max^2 / (2 t0 dt) for C > 0
    g, wl = make_workload("cmp_small")
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    cmp, t, p = random_candidates(300, g.n_cmp, g.nt, g.dt, 1, base_bounds(wl), seed=21,
                                  t_range=(20, 240))
    _, grad = L.semblance_grad(cmp, t, p.astype(np.float64))
    l1 = L.tau_sensitivity(cmp, t, p)
    dt = float(np.float32(g.dt))
    bound = np.max(g.offset) ** 2 / (2 * t * dt * dt) * l1
    assert np.all(np.abs(grad[:, 0]) <= bound * (1 + 1e-9) + 1e-15)
    assert np.mean(l1 > 0) > 0.99


def test_kink_margin_of_known_traveltimes():
    dt = float(np.float32(0.004))
    n0, h = 40, 300.0
    tr = np.sin(np.arange(120) * 0.2)[None, :]
    L = _tiny.line(tr, [1], [h], dt=dt, window=5)
    # C = 0: tau = n0 exactly, on a whole sample
    assert L.kink_margin([0], [n0], [[0.0]])[0] == 0.0
    # tau = n0 + 1.25: a quarter sample from a whole sample, relative to 1 + 1.25
    C = (((n0 + 1.25) * dt) ** 2 - (n0 * dt) ** 2) / h ** 2
    assert abs(L.kink_margin([0], [n0], [[C]])[0] - 0.25 / 2.25) < 1e-9
    # a trace past the record does not count
    C_far = (((119.5) * dt) ** 2 - (n0 * dt) ** 2) / h ** 2
    assert L.kink_margin([0], [n0], [[C_far]])[0] == np.inf
