"""GPU search (plain per-sample evolution and ENS) against the oracle."""
import numpy as np
import pytest

import oracle
from tests._tol import s_tol
from paper_2304_11399_amd.counts import evals_ens, evals_jade
from synth import base_bounds, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_S = 1e-5


@pytest.fixture(scope="module")
def ens():
    import paper_2304_11399_amd as e
    assert torch.cuda.is_available()
    return e


def _setup(ens, name, store="f32", **over):
    g, wl = make_workload(name, **over)
    ctx = ens.Context()
    ctx.bind(torch.from_numpy(g.traces).cuda(), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"],
             wl["window"], wl["ap_lo"], wl["ap_hi"], store=store)
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    return ctx, g, wl, L


def _grid(n_out, t_begin, t_end, cmp_out=None):
    cmp = np.repeat(np.arange(n_out) if cmp_out is None else np.asarray(cmp_out), t_end - t_begin)
    t = np.tile(np.arange(t_begin, t_end), n_out)
    return cmp.astype(np.int32), t.astype(np.int32)


def _check_scores(out, L, cmp, t, P, label, store="f32"):
    p = out["params"].cpu().numpy().reshape(-1, P)
    S = out["S"].cpu().numpy().reshape(-1).astype(np.float64)
    S_or, M_or, margin = L.semblance(cmp, t, p.astype(np.float64))
    ok = margin >= 0.05
    err = np.abs(S - S_or)[ok]
    bound = s_tol(store, L, cmp[ok], t[ok], p[ok])
    print(f"{label}: samples={len(cmp)} max|S - S_oracle(p)|={err.max():.2e} "
          f"({np.max(err / bound):.3f} of the bound)")
    assert np.all(err <= bound)
    if out["S64"] is not None:
        S64 = out["S64"].cpu().numpy().reshape(-1)
        assert np.abs(S64 - S_or)[margin > 1e-6].max() < 1e-11
    return p, S, S_or


def test_plain_de_cmp_small_matches_oracle(ens):
    ctx, g, wl, L = _setup(ens, "cmp_small")
    de, bounds = wl["de"], base_bounds(wl)
    cmp, t = _grid(g.n_cmp, 0, g.nt)
    # a few generations: the binary32 device run and the oracle take the same
    # decisions almost everywhere (the draws and the trial arithmetic are
    # bitwise equal; only near-ties of the scores can split them)
    short = dict(de, ng_f=3)
    o3 = ctx.search(bounds, short, seed=wl["search_seed"])
    p3, _, _ = _check_scores(o3, L, cmp, t, 1, "cmp_small NG=3")
    p3_or, _, ev3 = L.search(bounds, short, wl["search_seed"])
    assert ev3 == o3["n_evals"] == evals_jade(g.n_cmp * g.nt, 16, 3)
    same3 = np.all(p3 == p3_or.reshape(-1, 1), axis=1).mean()
    print(f"identical after 3 generations: {same3:.4f}")
    assert same3 > 0.9
    # the full budget: converged populations differ by less than binary32 can
    # order, so compare the outcome (score and distance to the reference maximum)
    out = ctx.search(bounds, de, seed=wl["search_seed"])
    P_d = g.n_cmp * g.nt
    assert out["n_evals"] == evals_jade(P_d, 16, 30)
    p, S, _ = _check_scores(out, L, cmp, t, 1, "cmp_small plain DE")
    p_or, S_or_run, ev = L.search(bounds, de, wl["search_seed"])
    assert ev == out["n_evals"]
    same = np.all(p == p_or.reshape(-1, 1), axis=1)
    rel = np.abs(p[:, 0] - p_or.reshape(-1)) / np.abs(p_or.reshape(-1))
    print(f"identical after 30 generations: {same.mean():.4f}; median rel. parameter "
          f"difference {np.median(rel):.2e}")
    S_ref, _ = L.sref(bounds, cmp, t, (2049,), n_refine=3)
    gap = np.maximum(S_ref - out["S64"].cpu().numpy().reshape(-1), 0)
    gap_or = np.maximum(S_ref - S_or_run.reshape(-1), 0)
    print(f"gap mean {gap.mean():.2e} p95 {np.quantile(gap, 0.95):.2e} max {gap.max():.2e}; "
          f"oracle run gap mean {gap_or.mean():.2e}")
    # the device search is as good as the oracle's own run of the same budget;
    # at the configured NP 16 x NG 30 that is a mean gap just above 1e-3 (a few
    # populations settle on side maxima, and more generations do not move them)
    assert abs(gap.mean() - gap_or.mean()) <= 2e-4
    assert np.median(gap) <= 1e-4
    # the raised budget, NP 24 x NG 30 (a larger population, the same
    # generations), reaches the 1e-3 bar on the device and in the oracle
    raised = dict(de, np_lo=24, np_hi=24)
    out24 = ctx.search(bounds, raised, seed=wl["search_seed"])
    assert out24["n_evals"] == evals_jade(P_d, 24, 30)
    _check_scores(out24, L, cmp, t, 1, "cmp_small plain DE 24x30")
    _, S_or24, _ = L.search(bounds, raised, wl["search_seed"])
    gap24 = np.maximum(S_ref - out24["S64"].cpu().numpy().reshape(-1), 0)
    gap24_or = np.maximum(S_ref - S_or24.reshape(-1), 0)
    print(f"NP 24 x NG 30: gap mean {gap24.mean():.2e} (oracle run {gap24_or.mean():.2e}), "
          f"{np.mean(gap24 <= 1e-3):.3f} <= 1e-3")
    assert gap24.mean() <= 1e-3 and gap24_or.mean() <= 1e-3


def test_search_is_deterministic_and_sliced_variants_agree(ens):
    ctx, g, wl, L = _setup(ens, "crs_ens", n_cmp=16, nt=240)
    de = dict(wl["de"], np_lo=16, np_hi=16, ng_f=12, n_bucket=8)
    bounds = base_bounds(wl)
    a = ctx.search(bounds, de, seed=3, t_begin=10, t_end=230)
    b = ctx.search(bounds, de, seed=3, t_begin=10, t_end=230)
    assert torch.equal(a["params"], b["params"]) and torch.equal(a["S"], b["S"])
    cmp, t = _grid(16, 10, 230)
    for nsl in (1, 2, 8):
        ctx.set_tuning(waves_per_sample_group=nsl)
        o = ctx.search(bounds, de, seed=3, t_begin=10, t_end=230)
        assert o["n_evals"] == a["n_evals"]
        _check_scores(o, L, cmp, t, 3, f"nsl={nsl}")
    ctx.set_tuning(0)


def test_ens_small_matches_oracle(ens):
    ctx, g, wl, L = _setup(ens, "crs_ens", n_cmp=16, nt=300)
    de = dict(wl["de"], np_lo=16, np_hi=16, ng_f=10, n_bucket=8)
    bounds = base_bounds(wl)
    out = ctx.search(bounds, de, seed=11, t_begin=40, t_end=280)
    n_s = 16 * 240
    assert out["n_evals"] == evals_ens(n_s, 16, 10, 5, 1, 1, 0)
    cmp, t = _grid(16, 40, 280)
    p, S, _ = _check_scores(out, L, cmp, t, 3, "ens small")
    p_or, S_run, ev = L.search(bounds, de, 11, t_begin=40, t_end=280)
    assert ev == out["n_evals"]
    same = np.all(p == p_or.reshape(-1, 3), axis=1)
    print(f"ENS identical trajectories: {same.mean():.4f}; mean S gpu {S.mean():.5f} "
          f"oracle {S_run.mean():.5f}")
    # the same draws and decisions up to binary32 ties (97-98% measured), and
    # both searches reach the same quality
    assert same.mean() >= 0.95
    assert abs(S.mean() - S_run.mean()) < 2e-3


def test_ens_exchange_off_equals_plain_de(ens):
    ctx, g, wl, L = _setup(ens, "crs_ens", n_cmp=12, nt=200)
    base = dict(wl["de"], np_lo=16, np_hi=16, ng_f=6, n_bucket=4, n_cycle=0)
    bounds = base_bounds(wl)
    # the same launch shape for both, so that the partial sums meet in the same order
    ctx.set_tuning(waves_per_sample_group=4, item_order=1)
    a = ctx.search(bounds, dict(base, inject=0), seed=5)
    b = ctx.search(bounds, dict(base, ens_enabled=0), seed=5)
    assert torch.equal(a["params"], b["params"]) and torch.equal(a["S"], b["S"])
    assert a["n_evals"] == b["n_evals"]


def test_ens_cycles_never_lower_a_sample(ens):
    ctx, g, wl, L = _setup(ens, "crs_ens", n_cmp=12, nt=200)
    base = dict(wl["de"], np_lo=12, np_hi=12, ng_f=5, n_bucket=6)
    bounds = base_bounds(wl)
    s0 = ctx.search(bounds, dict(base, n_cycle=0), seed=9)["S"]
    s1 = ctx.search(bounds, dict(base, n_cycle=1), seed=9)["S"]
    s2 = ctx.search(bounds, dict(base, n_cycle=2), seed=9)["S"]
    assert torch.all(s1 >= s0) and torch.all(s2 >= s1)
    assert (s1 > s0).float().mean() > 0.2


def test_polish_monotone_and_consistent(ens):
    ctx, g, wl, L = _setup(ens, "crs_diff", store="f16", n_cmp=24, nt=400)
    de = dict(wl["de"], np_lo=12, np_hi=12, ng_f=6, n_bucket=12, polish_steps=10)
    bounds = base_bounds(wl)
    out = ctx.search(bounds, de, seed=2, t_begin=50, t_end=350, keep_pre_polish=True)
    pre, post = out["S_pre_polish"], out["S"]
    assert torch.all(post >= pre)
    frac = (post > pre + 1e-6).float().mean().item()
    print(f"polish improved {frac:.3f} of the samples; mean gain {(post - pre).mean().item():.2e}")
    assert frac > 0.2
    q, s = oracle.quantize(g.traces, "f16")
    Lq = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"],
                                 traces=oracle.dequantize(q, s, "f16"))
    cmp, t = _grid(24, 50, 350)
    _check_scores(dict(out, S64=None), Lq, cmp, t, 3, "polished f16", store="f16")


def test_full_crs_ens_workload(ens, bench_shapes):
    # the full C2 line in the launch shapes the benchmark times
    ctx, g, wl, L = _setup(ens, "crs_ens")
    de, bounds = wl["de"], base_bounds(wl)
    out = ctx.search(bounds, de, seed=wl["search_seed"])
    st = ctx.stats()
    print("crs_ens launch shapes", {k: {f: st[k].get(f) for f in ("waves", "item_order", "dense")}
                                    for k in ("explore", "exploit")}, "tune_ms", st["tune_ms"])
    P_d = g.n_cmp * g.nt
    assert out["n_evals"] == evals_ens(P_d, 32, 80, 5, 1, 1, 0)
    rng = np.random.default_rng(1)
    pick = np.sort(rng.choice(P_d, 2000, replace=False))
    cmp, t = (pick // g.nt).astype(np.int32), (pick % g.nt).astype(np.int32)
    p = out["params"].cpu().numpy().reshape(-1, 3)[pick]
    S = out["S"].cpu().numpy().reshape(-1)[pick]
    S_or, _, margin = L.semblance(cmp, t, p.astype(np.float64))
    assert np.abs(S - S_or)[margin >= 0.05].max() <= TOL_S
    S64 = out["S64"].cpu().numpy().reshape(-1)[pick]
    assert np.abs(S64 - S_or)[margin > 1e-6].max() < 1e-11
