"""Full-size workloads on the GPU, checked on sampled outputs the oracle
computes one by one: the uneven batch (NP 16 to 64, aperture 2 to 16), the
binary16 / bfloat16 storage line, the binary16 + polish line, and the CRS +
ENS line with JADE and with N_skip = 2, each in the launch configuration the
benchmark times: the launch shapes come from the library's committed shape
file, as in the benchmark (a copy of it, so that a device it has no line for
measures its shapes without touching the committed file)."""
import os

import numpy as np
import pytest

import oracle
from tests._tol import s_tol
from paper_2304_11399_amd.counts import evals_ens
from synth import base_bounds, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOL_S = 1e-5


@pytest.fixture(scope="module")
def ens():
    import paper_2304_11399_amd as e
    assert torch.cuda.is_available()
    return e


def _shape(ctx):
    st = ctx.stats()
    return {k: {f: st[k].get(f) for f in ("waves", "item_order", "dense", "packed")}
            for k in ("explore", "exploit")}, st["tune_ms"]


def _expected_evals(de, g):
    if de["np_lo"] == de["np_hi"]:
        return evals_ens(g.n_cmp * g.nt, de["np_lo"], de["ng_f"], de["np_bf"], de["ng_bf"],
                         de["n_cycle"], 0)
    first = sum(oracle.pop_size(de, g.nt, t) * (1 + de["ng_f"]) for t in range(g.nt))
    return g.n_cmp * (first + de["n_cycle"] * g.nt * 2 * (de["np_bf"] * (1 + de["ng_bf"]) - 1))


def _gap(name, S64, g):
    ref = np.load(os.path.join(ROOT, "tests", "golden", f"sref_{name}.npz"))
    fp = float((g.traces.astype(np.float64) ** 2).sum())
    assert abs(fp / float(ref["fingerprint"]) - 1.0) < 1e-9, "reference maxima made for other data"
    found = S64.reshape(-1)[ref["cmp"].astype(np.int64) * g.nt + ref["t"]]
    return np.maximum(ref["S_ref"] - found, 0.0)


@pytest.mark.parametrize("name,store", [("crs_uneven", "f32"), ("crs_precision", "f16"),
                                        ("crs_precision", "bf16"), ("crs_diff", "f16")])
def test_full_size_workload(ens, bench_shapes, name, store):
    g, wl = make_workload(name)
    ctx = ens.Context()
    ctx.bind(torch.from_numpy(g.traces).cuda(), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"],
             wl["window"], wl["ap_lo"], wl["ap_hi"], store=store)
    de = wl["de"]
    out = ctx.search(base_bounds(wl), de, seed=wl["search_seed"], keep_pre_polish=True)
    print(f"{name} {store}: launch shapes {_shape(ctx)}")
    assert out["n_evals"] == _expected_evals(de, g)
    P_d = g.n_cmp * g.nt
    pick = np.sort(np.random.default_rng(3).choice(P_d, 1500, replace=False))
    cmp, t = (pick // g.nt).astype(np.int32), (pick % g.nt).astype(np.int32)
    p = out["params"].cpu().numpy().reshape(-1, 3)[pick].astype(np.float64)
    S = out["S"].cpu().numpy().reshape(-1)[pick]
    traces = None
    if store != "f32":
        q, s = oracle.quantize(g.traces, store)
        traces = oracle.dequantize(q, s, store)
    Lq = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"], traces=traces)
    S_q, _, margin = Lq.semblance(cmp, t, p)
    sel = margin >= 0.05
    err = np.abs(S - S_q)[sel]
    bound = s_tol(store, Lq, cmp[sel], t[sel], p[sel])
    del Lq
    L32 = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    S_32, _, margin32 = L32.semblance(cmp, t, p)
    S64 = out["S64"].cpu().numpy()
    err64 = np.abs(S64.reshape(-1)[pick] - S_32)[margin32 > 1e-6]
    gap = _gap(name, S64, g)
    print(f"{name} {store}: max|S - S_oracle(stored)| {err.max():.2e} ({np.max(err / bound):.3f} of the "
          f"bound); max|S64 - S_oracle| {err64.max():.2e}; mean gap {gap.mean():.2e} "
          f"({np.mean(gap <= 1e-3):.3f} <= 1e-3)")
    assert np.all(err <= bound)
    assert err64.max() < 1e-11
    assert gap.mean() <= 1e-3
    if de.get("polish_steps", 0) > 0:
        assert torch.all(out["S"] >= out["S_pre_polish"])


@pytest.mark.parametrize("variant", ["jade", "skip2"])
def test_full_size_crs_ens_variants(ens, bench_shapes, variant):
    # the benchmark's equal-accuracy variants at the full C2 size: JADE (R8)
    # and time-sample skipping with N_skip = 2 (R13)
    g, wl = make_workload("crs_ens")
    ctx = ens.Context()
    ctx.bind(torch.from_numpy(g.traces).cuda(), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"],
             wl["window"], wl["ap_lo"], wl["ap_hi"])
    de = dict(wl["de"], adapt=1, CR=0.5) if variant == "jade" else dict(wl["de"], n_skip=2)
    out = ctx.search(base_bounds(wl), de, seed=wl["search_seed"])
    print(f"crs_ens {variant}: launch shapes {_shape(ctx)}")
    P_d = g.n_cmp * g.nt
    if variant == "jade":
        assert out["n_evals"] == evals_ens(P_d, 32, 80, 5, 1, 1, 0)
    else:
        # 1000 samples per trace is not a multiple of 3, so the paper's formula
        # is not exact; the count does not depend on the data and every CMP
        # costs the same, so it is the oracle's count for one CMP times n_cmp
        g1, wl1 = make_workload("crs_ens", n_cmp=1)
        L1 = oracle.Line.from_gather(g1, wl1["window"], wl1["op"], wl1["ap_lo"], wl1["ap_hi"])
        _, _, ev1 = L1.search(base_bounds(wl1), de, wl["search_seed"])
        assert out["n_evals"] == g.n_cmp * ev1
    pick = np.sort(np.random.default_rng(4).choice(P_d, 1500, replace=False))
    cmp, t = (pick // g.nt).astype(np.int32), (pick % g.nt).astype(np.int32)
    p = out["params"].cpu().numpy().reshape(-1, 3)[pick].astype(np.float64)
    S = out["S"].cpu().numpy().reshape(-1)[pick]
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    S_or, _, margin = L.semblance(cmp, t, p)
    err = np.abs(S - S_or)[margin >= 0.05]
    gap = _gap("crs_ens", out["S64"].cpu().numpy(), g)
    print(f"crs_ens {variant}: evals {out['n_evals']}, max|S - S_oracle| {err.max():.2e}, "
          f"mean gap {gap.mean():.2e} ({np.mean(gap <= 1e-3):.3f} <= 1e-3)")
    assert err.max() <= TOL_S
    # measured: JADE 1.1e-4, N_skip = 2 1.2e-3 (skipping trades accuracy)
    assert gap.mean() <= (1e-3 if variant == "jade" else 2e-3)
