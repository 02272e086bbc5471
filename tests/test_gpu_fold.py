"""Ragged folds: lines whose CMPs hold 0, 1, 2, 3 and other odd and even trace
counts (traces dropped at random from a regular line), on every storage type.

The trace loops take a CMP's traces in pairs and finish an odd count with one
trace, and a sliced search deals each CMP's traces over several waves; the
regular synthetic lines (24 to 96 offsets per CMP) reach the single-trace
tail only for some slice counts.  Here every loop meets empty CMPs, single
traces and odd tails: the semblance per candidate and the adjoint per element
against the oracle on the same stored samples, and the search in several
launch shapes, whose every output the oracle re-scores (binary32 rows: the
trajectories also follow the oracle's).  Silent traces (all zeros) are the
degenerate case of the definition (E = 0, S = 0)."""
import dataclasses

import numpy as np
import pytest

import oracle
from tests._tol import s_tol
from synth import base_bounds, make_workload, random_candidates

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MARGIN = 0.05    # samples: a trace this close to a participation edge may flip
EDGE, KINK, REL = 0.05, 4e-6, 1e-3


@pytest.fixture(scope="module")
def ens():
    import paper_2304_11399_amd as e
    assert torch.cuda.is_available()
    return e


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def ragged(name, seed, **over):
    """The workload's line with a random subset of each CMP's traces kept (in
    offset order); the first CMPs keep 0, 1, 2 and 3 traces, one CMP in the
    middle keeps none."""
    g, wl = make_workload(name, **over)
    rng = np.random.default_rng(seed)
    fold = np.diff(g.cmp_ptr)
    keep_n = rng.integers(0, fold + 1)
    keep_n[:4] = [0, 1, 2, 3]
    keep_n[g.n_cmp // 2] = 0
    idx = np.concatenate([np.sort(rng.choice(np.arange(g.cmp_ptr[c], g.cmp_ptr[c + 1]), keep_n[c],
                                             replace=False)) for c in range(g.n_cmp)]).astype(np.int64)
    cmp_ptr = np.concatenate([[0], np.cumsum(keep_n)]).astype(np.int64)
    g2 = dataclasses.replace(g, traces=np.ascontiguousarray(g.traces[idx]), cmp_ptr=cmp_ptr,
                             offset=np.ascontiguousarray(g.offset[idx]))
    return g2, wl, keep_n


def _bind(ens, g, wl, store):
    ctx = ens.Context()
    ctx.bind(_dev(g.traces), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"], wl["window"], wl["ap_lo"],
             wl["ap_hi"], store=store)
    traces = None
    if store != "f32":
        q, s = oracle.quantize(g.traces, store)
        traces = oracle.dequantize(q, s, store)
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"], traces=traces)
    return ctx, L


@pytest.mark.parametrize("name", ["cmp_small", "crs_ens"])
@pytest.mark.parametrize("store", ["f32", "f16", "bf16"])
def test_semblance_on_ragged_folds(ens, name, store):
    g, wl, keep_n = ragged(name, seed=31, **({"n_cmp": 40} if name == "crs_ens" else {}))
    print(f"{name}: folds {np.bincount(keep_n)[:4]} CMPs with 0..3 traces, {np.sum(keep_n % 2)} odd, "
          f"max {keep_n.max()}")
    ctx, L = _bind(ens, g, wl, store)
    P = wl["op"]
    cmp, t, p = random_candidates(8000, g.n_cmp, g.nt, g.dt, P, base_bounds(wl), seed=32)
    S, M = ctx.semblance_eval(_dev(cmp), _dev(t), _dev(p), with_M=True)
    S, M = S.cpu().numpy().astype(np.float64), M.cpu().numpy()
    S_or, M_or, margin = L.semblance(cmp, t, p.astype(np.float64))
    flip = M != M_or
    assert np.all(margin[flip] < MARGIN) and flip.mean() < 1e-3
    ok = ~flip
    err = np.abs(S - S_or)[ok]
    bound = s_tol(store, L, cmp[ok], t[ok], p[ok])
    empty = (M_or == 0) & ok
    print(f"{name} {store}: {cmp.size} candidates, {empty.sum()} with no participating trace, "
          f"max|dS| {err.max():.2e} ({np.max(err / bound):.3f} of the bound)")
    assert np.all(err <= bound)
    assert np.all(S[empty] == 0.0)
    if name == "cmp_small":
        # the CMP operator reads its own CMP only: an empty CMP scores 0 everywhere
        assert np.all(S[np.isin(cmp, np.flatnonzero(keep_n == 0))] == 0.0)


@pytest.mark.parametrize("store", ["f32", "f16"])
def test_adjoint_on_ragged_folds(ens, store):
    g, wl, _ = ragged("crs_ens", seed=33, n_cmp=40)
    ctx, L = _bind(ens, g, wl, store)
    bounds = base_bounds(wl)
    cmp, t, p = random_candidates(3000, g.n_cmp, g.nt, g.dt, 3, bounds, seed=34, t_range=(20, g.nt))
    gr = ctx.semblance_backward(_dev(cmp), _dev(t), _dev(p), _dev(np.ones(cmp.size, np.float32)))
    gr = gr.cpu().numpy().astype(np.float64)
    p64 = p.astype(np.float64)
    _, g_or = L.semblance_grad(cmp, t, p64)
    _, M_or, margin = L.semblance(cmp, t, p64)
    kink = L.kink_margin(cmp, t, p64)
    span = np.stack([np.subtract(*L.sample_bounds(bounds, tt)[::-1]) for tt in t])
    gz, gz_or = gr * span, g_or * span
    keep = (margin >= EDGE) & (kink >= KINK) & (M_or > 0)
    print(f"ragged crs_ens {store}: {cmp.size} pairs, {np.sum(M_or == 0)} empty, "
          f"{np.sum(margin < EDGE)} at an edge, {np.sum((kink < KINK) & (margin >= EDGE))} at a kink; "
          f"{keep.sum()} compared")
    assert keep.sum() >= 1000
    assert np.all(gr[(M_or == 0) & (margin >= EDGE)] == 0.0)
    for d in range(3):
        scale = np.maximum(np.abs(gz_or[keep, d]), np.median(np.abs(gz_or[keep, d])))
        rel = np.abs(gz[keep, d] - gz_or[keep, d]) / scale
        assert rel.max() <= REL, f"d={d}: rel {rel.max():.3e}"


SHAPES = {
    "one slice": dict(waves_per_sample_group=1, item_order=1, occupancy=1),
    "eight slices, 64 registers": dict(waves_per_sample_group=8, item_order=3, occupancy=2),
    "packed over 4 waves": dict(waves_per_sample_group=2, item_order=2, occupancy=2, packing=4),
}


@pytest.mark.parametrize("shape", list(SHAPES))
@pytest.mark.parametrize("store", ["f32", "f16", "bf16"])
def test_search_on_ragged_folds(ens, store, shape):
    g, wl, _ = ragged("crs_ens", seed=35, n_cmp=16, nt=240)
    ctx, L = _bind(ens, g, wl, store)
    ctx.set_tuning(**SHAPES[shape])
    de = dict(wl["de"], np_lo=16, np_hi=16, ng_f=8, n_bucket=8)
    bounds = base_bounds(wl)
    out = ctx.search(bounds, de, seed=36, t_begin=20, t_end=220)
    st = ctx.stats()
    n_out, n_t = g.n_cmp, 200
    cmp = np.repeat(np.arange(n_out), n_t).astype(np.int32)
    t = np.tile(np.arange(20, 220), n_out).astype(np.int32)
    p = out["params"].cpu().numpy().reshape(-1, 3)
    S = out["S"].cpu().numpy().reshape(-1).astype(np.float64)
    S_or, _, margin = L.semblance(cmp, t, p.astype(np.float64))
    ok = margin >= MARGIN
    err = np.abs(S - S_or)[ok]
    bound = s_tol(store, L, cmp[ok], t[ok], p[ok])
    print(f"ragged search {store}, {shape} (explore {st['explore']['waves']} waves, packed "
          f"{st['explore']['packed']}): max|S - S_oracle(p)| {err.max():.2e} "
          f"({np.max(err / bound):.3f} of the bound)")
    assert np.all(err <= bound)
    p_or, S_run, ev = L.search(bounds, de, 36, t_begin=20, t_end=220)
    assert ev == out["n_evals"]
    if store == "f32":
        # the same draws and decisions up to binary32 ties
        same = np.all(p == p_or.reshape(-1, 3), axis=1)
        print(f"  identical trajectories {same.mean():.4f}")
        assert same.mean() >= 0.95
    assert abs(S.mean() - S_run.mean()) < 2e-3


@pytest.mark.parametrize("store", ["f32", "f16", "bf16"])
def test_silent_traces_score_zero(ens, store):
    # traces of zeros: E = 0, so S = 0 by definition (eq. S), with no NaN in
    # the scores, the gradient or the search; the CMP operator reads its own
    # CMP only, so silent CMPs score 0 for every candidate
    g, wl = make_workload("cmp_small")
    silent = np.array([2, 3, 4, 5, 11])
    traces = g.traces.copy()
    for c in silent:
        traces[g.cmp_ptr[c]:g.cmp_ptr[c + 1]] = 0.0
    g = dataclasses.replace(g, traces=traces)
    ctx, L = _bind(ens, g, wl, store)
    cmp, t, p = random_candidates(4000, g.n_cmp, g.nt, g.dt, 1, base_bounds(wl), seed=37)
    S, M = ctx.semblance_eval(_dev(cmp), _dev(t), _dev(p), with_M=True)
    S, M = S.cpu().numpy(), M.cpu().numpy()
    S_or, M_or, _ = L.semblance(cmp, t, p.astype(np.float64))
    quiet = np.isin(cmp, silent)
    assert np.all(S[quiet] == 0.0) and np.all(S_or[quiet] == 0.0)
    assert np.any(M[quiet] > 0)
    gr = ctx.semblance_backward(_dev(cmp), _dev(t), _dev(p), _dev(np.ones(cmp.size, np.float32)))
    gr = gr.cpu().numpy()
    assert np.all(np.isfinite(gr)) and np.all(gr[quiet] == 0.0)
    de = dict(wl["de"], np_lo=8, np_hi=8, ng_f=4)
    out = ctx.search(base_bounds(wl), de, seed=38)
    S_out = out["S"].cpu().numpy().reshape(g.n_cmp, -1)
    assert np.all(np.isfinite(out["params"].cpu().numpy())) and np.all(S_out[silent] == 0.0)
    assert np.all(out["S64"].cpu().numpy().reshape(g.n_cmp, -1)[silent] == 0.0)
