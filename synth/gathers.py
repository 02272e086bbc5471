"""Seeded synthetic CMP-sorted gathers and candidate draws.

The gathers stand in for the field and Kirchhoff datasets the paper measures on
(section "Numerical experiments"), which are not available here.  Each trace is
a sum of unit-peak Ricker wavelets placed on exact constant-velocity
traveltimes, plus iid Gaussian noise:

* planar dipping reflectors: exact Levin moveout
  ``t^2 = t0(m)^2 + h^2 cos^2(theta) / v^2`` with ``t0(m) = t0c + 2 (m - x0) sin(theta) / v``;
* circular (anticline / syncline) reflectors: specular point found by
  minimising the source-reflector-receiver path (Fermat);
* point diffractors: exact double square root.

Offsets ``h`` are full source-receiver offsets.  Noise has standard deviation
``1 / snr`` (peak-amplitude signal-to-noise ratio for a unit Ricker peak).
Traces are sorted by (CMP, offset); ``cmp_ptr`` is the CSR row pointer of the
CMPs.  Sample ``n`` of every trace sits at time ``n * dt``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ---------------------------------------------------------------------------
# workload descriptions


def _offsets(first, last, step):
    return np.arange(first, last + 0.5 * step, step, dtype=np.float64)


_V = 2000.0  # constant medium velocity of the CRS workloads (m/s)

# CRS parameter box: A in s/m, B*t0 and C*t0 in s^2/m^2; bits 1 and 2 of the
# mask say that B and C bounds are divided per sample by max(t0, dt).
_CRS_BOUNDS = dict(lo=(-1.0e-3, -2.0e-6, 1.0 / 4000.0 ** 2),
                   hi=(1.0e-3, 2.0e-6, 1.0 / 1500.0 ** 2), inv_t0_mask=0b110)
_CMP_BOUNDS = dict(lo=(1.0 / 4000.0 ** 2, 0.0, 0.0), hi=(1.0 / 1500.0 ** 2, 0.0, 0.0),
                   inv_t0_mask=0)


def _crs_events(t_scale):
    """Six reflectors (four planar, two curved) and two diffractors."""
    ev = []
    for dip, t0 in ((0.0, 0.6), (5.0, 1.0), (-8.0, 1.5), (12.0, 2.2)):
        ev.append(dict(kind="planar", dip_deg=dip, t0=t0 * t_scale))
    ev.append(dict(kind="anticline", radius=3000.0, t0=2.8 * t_scale))
    ev.append(dict(kind="syncline", radius=6000.0, t0=3.4 * t_scale))
    ev.append(dict(kind="diffractor", frac=0.3, t0=1.8 * t_scale))
    ev.append(dict(kind="diffractor", frac=0.7, t0=2.6 * t_scale))
    return ev


WORKLOADS = {
    # CMP operator, plain DE
    "cmp_small": dict(
        n_cmp=16, dx=12.5, offsets=_offsets(25, 600, 25), nt=256, dt=0.004,
        events=[dict(kind="flat", t0=0.30, v=1800.0), dict(kind="flat", t0=0.55, v=2400.0),
                dict(kind="flat", t0=0.80, v=3000.0)],
        v=None, f_peak=25.0, snr=5.0, amp_sigma=0.0, data_seed=1001,
        op=1, window=5, ap_lo=0, ap_hi=0, bounds=_CMP_BOUNDS,
        de=dict(np_lo=16, np_hi=16, ng_f=30, np_bf=5, ng_bf=1, n_cycle=0, n_bucket=16,
                ens_enabled=0, F=0.5, CR=0.9, polish_steps=0, polish_lr=0.01),
        store="f32", search_seed=7),
    # CRS operator, DE + ENS
    "crs_ens": dict(
        n_cmp=256, dx=12.5, offsets=_offsets(25, 1200, 25), nt=1000, dt=0.004,
        events=_crs_events(1.0), v=_V, f_peak=30.0, snr=3.0, amp_sigma=0.0, data_seed=1002,
        op=3, window=7, ap_lo=8, ap_hi=8, bounds=_CRS_BOUNDS,
        de=dict(np_lo=32, np_hi=32, ng_f=80, np_bf=5, ng_bf=1, n_cycle=1, n_bucket=64,
                ens_enabled=1, F=0.5, CR=0.9, polish_steps=0, polish_lr=0.01),
        store="f32", search_seed=7),
    # CRS, uneven apertures and populations
    "crs_uneven": dict(
        n_cmp=1024, dx=12.5, offsets=_offsets(25, 1500, 25), nt=1500, dt=0.004,
        events=_crs_events(1.5), v=_V, f_peak=30.0, snr=3.0, amp_sigma=0.0, data_seed=1003,
        op=3, window=7, ap_lo=2, ap_hi=16, bounds=_CRS_BOUNDS,
        de=dict(np_lo=16, np_hi=64, ng_f=80, np_bf=5, ng_bf=1, n_cycle=1, n_bucket=64,
                ens_enabled=1, F=0.5, CR=0.9, polish_steps=0, polish_lr=0.01),
        store="f32", search_seed=7),
    # CRS, log-normal trace amplitudes, reduced-precision storage
    "crs_precision": dict(
        n_cmp=1024, dx=12.5, offsets=_offsets(25, 1500, 25), nt=1500, dt=0.004,
        events=_crs_events(1.5), v=_V, f_peak=30.0, snr=3.0, amp_sigma=1.0, data_seed=1004,
        op=3, window=7, ap_lo=2, ap_hi=16, bounds=_CRS_BOUNDS,
        de=dict(np_lo=16, np_hi=64, ng_f=80, np_bf=5, ng_bf=1, n_cycle=1, n_bucket=64,
                ens_enabled=1, F=0.5, CR=0.9, polish_steps=0, polish_lr=0.01),
        store="f16", search_seed=7),
    # CRS, differentiable polish after the evolutionary search
    "crs_diff": dict(
        n_cmp=2048, dx=12.5, offsets=_offsets(25, 2400, 25), nt=2000, dt=0.002,
        events=_crs_events(1.0), v=_V, f_peak=40.0, snr=2.0, amp_sigma=0.0, data_seed=1005,
        op=3, window=7, ap_lo=8, ap_hi=8, bounds=_CRS_BOUNDS,
        de=dict(np_lo=32, np_hi=32, ng_f=40, np_bf=5, ng_bf=1, n_cycle=1, n_bucket=64,
                ens_enabled=1, F=0.5, CR=0.9, polish_steps=10, polish_lr=0.01),
        store="f16", search_seed=7),
}


@dataclasses.dataclass
class Gather:
    """A CMP-sorted prestack line."""
    traces: np.ndarray      # [n_tr, nt] float32
    cmp_ptr: np.ndarray     # [n_cmp + 1] int64
    offset: np.ndarray      # [n_tr] float32, full offset (m)
    nt: int
    dt: float
    dx: float
    n_cmp: int
    events: list
    v: float | None

    @property
    def n_tr(self):
        return int(self.traces.shape[0])

    def cmp_of_trace(self):
        return np.repeat(np.arange(self.n_cmp, dtype=np.int32), np.diff(self.cmp_ptr))


# ---------------------------------------------------------------------------
# kinematics (exact, constant velocity)


def _golden_min(fun, lo, hi, iters=90):
    """Vectorised golden-section minimisation of fun on [lo, hi] (elementwise)."""
    g = (math.sqrt(5.0) - 1.0) / 2.0
    a, b = lo.copy(), hi.copy()
    for _ in range(iters):
        c = b - g * (b - a)
        d = a + g * (b - a)
        left = fun(c) < fun(d)
        b = np.where(left, d, b)
        a = np.where(left, a, c)
    x = 0.5 * (a + b)
    return x, fun(x)


def _event_times(ev, xs, xr, xm, h, x0, line_len, v_default):
    """Two-way traveltime (s) of one event for source xs, receiver xr.

    Returns (t, valid) arrays.
    """
    kind = ev["kind"]
    if kind == "flat":
        v = ev["v"]
        t = np.sqrt(ev["t0"] ** 2 + (h / v) ** 2)
        return t, np.ones_like(t, dtype=bool)
    v = v_default
    if kind == "planar":
        th = math.radians(ev["dip_deg"])
        t0m = ev["t0"] + 2.0 * (xm - x0) * math.sin(th) / v
        t = np.sqrt(np.maximum(t0m, 0.0) ** 2 + (h * math.cos(th) / v) ** 2)
        return t, t0m > 0.0
    if kind == "diffractor":
        xd = ev["frac"] * line_len
        zd = 0.5 * v * ev["t0"]
        t = (np.sqrt(zd ** 2 + (xs - xd) ** 2) + np.sqrt(zd ** 2 + (xr - xd) ** 2)) / v
        return t, np.ones_like(t, dtype=bool)
    if kind in ("anticline", "syncline"):
        R = ev["radius"]
        zref = 0.5 * v * ev["t0"]          # reflector depth below the line centre
        xc = x0
        if kind == "anticline":
            zc, sgn = zref + R, -1.0        # centre below, upper arc
        else:
            zc, sgn = zref - R, 1.0         # centre above, lower arc

        def point(phi):
            return xc + R * np.sin(phi), zc + sgn * R * np.cos(phi)

        def path(phi):
            px, pz = point(phi)
            return (np.hypot(xs - px, pz) + np.hypot(xr - px, pz)) / v

        if kind == "anticline":
            phi0 = np.arctan2(xm - xc, zc)
        else:
            phi0 = np.arctan2(xm - xc, -zc)
        phi, t = _golden_min(path, phi0 - 0.6, phi0 + 0.6)
        px, pz = point(phi)
        valid = (pz > 0.0) & (np.abs(phi) < 1.3)
        return t, valid
    raise ValueError(kind)


def _ricker(tau, f):
    a = (math.pi * f * tau) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def make_gather(n_cmp, dx, offsets, nt, dt, events, f_peak, snr, seed,
                amp_sigma=0.0, v=None, noise=True):
    """Synthesise a CMP-sorted line (see module docstring)."""
    rng = np.random.default_rng(seed)
    offsets = np.asarray(offsets, dtype=np.float64)
    n_off = offsets.size
    n_tr = n_cmp * n_off
    cmp_idx = np.repeat(np.arange(n_cmp), n_off)
    h = np.tile(offsets, n_cmp)
    xm = cmp_idx * dx
    xs, xr = xm - 0.5 * h, xm + 0.5 * h
    line_len = (n_cmp - 1) * dx
    x0 = 0.5 * line_len
    traces = np.zeros((n_tr, nt), dtype=np.float64)
    half = int(math.ceil(2.0 / f_peak / dt)) + 1
    k = np.arange(-half, half + 1)
    rows = np.arange(n_tr)[:, None]
    for ev in events:
        t, valid = _event_times(ev, xs, xr, xm, h, x0, line_len, v)
        t = np.where(valid, t, -1.0)
        c = np.rint(t / dt).astype(np.int64)
        cols = c[:, None] + k[None, :]
        vals = _ricker(cols * dt - t[:, None], f_peak)
        ok = valid[:, None] & (cols >= 0) & (cols < nt)
        vals = np.where(ok, vals, 0.0)
        cols = np.clip(cols, 0, nt - 1)
        traces[rows, cols] += vals
    if noise and snr is not None and snr > 0:
        traces += rng.standard_normal((n_tr, nt)) / snr
    if amp_sigma > 0:
        traces *= np.exp(amp_sigma * rng.standard_normal(n_tr))[:, None]
    cmp_ptr = np.arange(n_cmp + 1, dtype=np.int64) * n_off
    return Gather(traces=traces.astype(np.float32), cmp_ptr=cmp_ptr,
                  offset=h.astype(np.float32), nt=nt, dt=dt, dx=dx, n_cmp=n_cmp,
                  events=list(events), v=v)


def make_workload(name, **overrides):
    """Build the gather of a named workload; returns (gather, workload dict)."""
    wl = dict(WORKLOADS[name])
    wl.update(overrides)
    g = make_gather(wl["n_cmp"], wl["dx"], wl["offsets"], wl["nt"], wl["dt"], wl["events"],
                    wl["f_peak"], wl["snr"], wl["data_seed"], wl.get("amp_sigma", 0.0),
                    wl.get("v"))
    return g, wl


def base_bounds(wl):
    b = wl["bounds"]
    return (np.array(b["lo"], dtype=np.float32), np.array(b["hi"], dtype=np.float32),
            int(b["inv_t0_mask"]))


def random_candidates(n, n_cmp, nt, dt, nparam, bounds, seed, cmp_range=None, t_range=None,
                      spread=1.0):
    """Draw n (cmp, t, params) triples, params uniform in each sample's box.

    ``bounds = (lo, hi, inv_t0_mask)``; a bound whose mask bit is set is
    divided by max(t0, dt).  ``spread > 1`` widens the box around its centre
    (to reach the excluded-trace and empty cases).  Returned sorted by
    (cmp, t) so that neighbouring candidates share an aperture.
    """
    rng = np.random.default_rng(seed)
    lo, hi, mask = bounds
    c0, c1 = cmp_range if cmp_range is not None else (0, n_cmp)
    t0_, t1_ = t_range if t_range is not None else (0, nt)
    cmp = rng.integers(c0, c1, size=n).astype(np.int32)
    t = rng.integers(t0_, t1_, size=n).astype(np.int32)
    order = np.lexsort((t, cmp))
    cmp, t = cmp[order], t[order]
    z = rng.random((n, nparam))
    tt = np.maximum(t.astype(np.float64) * dt, dt)
    p = np.empty((n, nparam), dtype=np.float64)
    for d in range(nparam):
        l, hh = float(lo[d]), float(hi[d])
        mid, half = 0.5 * (l + hh), 0.5 * (hh - l) * spread
        val = mid - half + 2.0 * half * z[:, d]
        if mask >> d & 1:
            val = val / tt
        p[:, d] = val
    return cmp, t, p.astype(np.float32)
