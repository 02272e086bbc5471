"""Write the reference maxima S_ref used by the semblance-gap metric.

Calls only the oracle (binary64 grid search with Nelder-Mead refinement) on
the seeded synthetic workloads; run from the repository root:

    python tests/golden/make_sref.py [workload ...]

Evaluation sets: every sample for the small CMP workload; for the CRS
workloads 1024 seeded random samples plus 256 samples lying on the planar
reflectors, where the analytic parameters (A = 2 sin(theta)/v, B = 0,
C t0 = cos^2(theta)/v^2, exact for a planar reflector in a constant-velocity
medium) also enter the maximum.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import base_bounds, make_workload  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))

# grid points per axis (A, B t0, C t0): neighbouring points change the far
# trace's traveltime by about a quarter period of the wavelet
GRIDS = {"cmp_small": (2049,), "crs_ens": (25, 5, 33), "crs_uneven": (25, 5, 33),
         "crs_precision": (25, 5, 33), "crs_diff": (29, 5, 41)}


def planar_samples(g, wl, n, rng):
    evs = [e for e in g.events if e["kind"] == "planar"]
    v = wl["v"]
    x0 = 0.5 * (g.n_cmp - 1) * g.dx
    dt = float(np.float32(g.dt))
    out = []
    while len(out) < n:
        e = evs[rng.integers(len(evs))]
        j = int(rng.integers(wl["ap_hi"], g.n_cmp - wl["ap_hi"]))
        th = np.radians(e["dip_deg"])
        t0m = e["t0"] + 2.0 * (j * g.dx - x0) * np.sin(th) / v
        n0 = int(round(t0m / dt))
        if not (5 <= n0 < g.nt - 5):
            continue
        t0 = n0 * dt
        out.append((j, n0, 2 * np.sin(th) / v, 0.0, np.cos(th) ** 2 / v ** 2 / t0))
    return out


def make(name):
    g, wl = make_workload(name)
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    bounds = base_bounds(wl)
    rng = np.random.default_rng(20240)
    if name == "cmp_small":
        cmp = np.repeat(np.arange(g.n_cmp), g.nt).astype(np.int32)
        t = np.tile(np.arange(g.nt), g.n_cmp).astype(np.int32)
        planar = np.zeros(cmp.size, bool)
        p_true = np.full((cmp.size, 1), np.nan)
    else:
        pick = np.sort(rng.choice(g.n_cmp * g.nt, 1024, replace=False))
        cmp_r, t_r = pick // g.nt, pick % g.nt
        ps = planar_samples(g, wl, 256, rng)
        cmp = np.concatenate([cmp_r, [p[0] for p in ps]]).astype(np.int32)
        t = np.concatenate([t_r, [p[1] for p in ps]]).astype(np.int32)
        planar = np.concatenate([np.zeros(cmp_r.size, bool), np.ones(len(ps), bool)])
        p_true = np.concatenate([np.full((cmp_r.size, 3), np.nan),
                                 np.array([p[2:] for p in ps])])
    t1 = time.time()
    S_ref, p_ref = L.sref(bounds, cmp, t, GRIDS[name], n_refine=8 if wl["op"] == 3 else 3)
    if planar.any():
        lo_hi = [L.sample_bounds(bounds, tt) for tt in t[planar]]
        inside = np.array([np.all((pt >= lo) & (pt <= hi)) for pt, (lo, hi) in
                           zip(p_true[planar], lo_hi)])
        S_true, _, _ = L.semblance(cmp[planar], t[planar], p_true[planar])
        S_true = np.where(inside, S_true, -1.0)
        idx = np.where(planar)[0]
        better = S_true > S_ref[idx]
        S_ref[idx[better]] = S_true[better]
        p_ref[idx[better]] = p_true[planar][better]
    print(f"{name}: {cmp.size} samples in {time.time() - t1:.1f} s; mean S_ref {S_ref.mean():.4f}")
    np.savez_compressed(os.path.join(OUT, f"sref_{name}.npz"), cmp=cmp, t=t, S_ref=S_ref,
                        p_ref=p_ref, planar=planar,
                        fingerprint=np.float64((g.traces.astype(np.float64) ** 2).sum()))


if __name__ == "__main__":
    for name in sys.argv[1:] or ["cmp_small", "crs_ens"]:
        make(name)
