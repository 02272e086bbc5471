"""GPU ENS with time-sample skipping (N_skip 1 and 2) against the oracle:
evaluation counts, scores of the reported parameters, interpolated samples,
search quality, graph replay."""
import numpy as np
import pytest

import oracle
from paper_2304_11399_amd.counts import evals_ens
from synth import base_bounds, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_S = 1e-5


@pytest.fixture(scope="module")
def ens():
    import paper_2304_11399_amd as e
    assert torch.cuda.is_available()
    return e


@pytest.fixture(scope="module")
def line(ens):
    g, wl = make_workload("crs_ens", n_cmp=16, nt=300)
    ctx = ens.Context()
    ctx.bind(torch.from_numpy(g.traces).cuda(), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"],
             wl["window"], wl["ap_lo"], wl["ap_hi"])
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    return ctx, g, wl, L


def _grid(n_out, t_begin, t_end):
    cmp = np.repeat(np.arange(n_out), t_end - t_begin)
    t = np.tile(np.arange(t_begin, t_end), n_out)
    return cmp.astype(np.int32), t.astype(np.int32)


def _scores_match(out, L, cmp, t, label):
    p = out["params"].cpu().numpy().reshape(-1, 3)
    S = out["S"].cpu().numpy().reshape(-1).astype(np.float64)
    S_or, _, margin = L.semblance(cmp, t, p.astype(np.float64))
    err = np.abs(S - S_or)[margin >= 0.05]
    print(f"{label}: max|S - S_oracle(p)| = {err.max():.2e}")
    assert err.max() <= TOL_S
    return p, S


@pytest.mark.parametrize("n_skip", [1, 2])
def test_skip_counts_scores_and_quality(line, n_skip):
    ctx, g, wl, L = line
    de = dict(wl["de"], np_lo=16, np_hi=16, ng_f=10, n_bucket=8, n_skip=n_skip)
    bounds = base_bounds(wl)
    out = ctx.search(bounds, de, seed=13, t_begin=40, t_end=280)
    # 240 samples per trace: a multiple of N_skip + 1, so the paper's count is exact
    assert out["n_evals"] == evals_ens(16 * 240, 16, 10, 5, 1, 1, n_skip)
    cmp, t = _grid(16, 40, 280)
    p, S = _scores_match(out, L, cmp, t, f"skip {n_skip}")
    p_or, S_run, ev = L.search(bounds, de, 13, t_begin=40, t_end=280)
    assert ev == out["n_evals"]
    same = np.all(p == p_or.reshape(-1, 3), axis=1).mean()
    print(f"skip {n_skip}: identical {same:.4f}; mean S gpu {S.mean():.5f} oracle {S_run.mean():.5f}")
    assert abs(S.mean() - S_run.mean()) < 2e-3


def test_skip_ragged_grid_counts_match_oracle(line):
    # 241 samples: the last stride is partial; counts come from the oracle run
    ctx, g, wl, L = line
    de = dict(wl["de"], np_lo=12, np_hi=12, ng_f=4, n_bucket=5, n_skip=2)
    bounds = base_bounds(wl)
    out = ctx.search(bounds, de, seed=21, t_begin=30, t_end=271)
    _, _, ev = L.search(bounds, de, 21, t_begin=30, t_end=271)
    assert out["n_evals"] == ev
    cmp, t = _grid(16, 30, 271)
    _scores_match(out, L, cmp, t, "skip ragged")


def test_first_sweep_skipped_samples_are_interpolated(line):
    # stage 0 only: a skipped sample is the clamped binary32 point at
    # (t - ta)/(tb - ta) between this trace's estimated samples ta, tb
    ctx, g, wl, L = line
    de = dict(wl["de"], np_lo=16, np_hi=16, ng_f=6, n_bucket=8, n_cycle=0, n_skip=2)
    bounds = base_bounds(wl)
    t0, t1 = 40, 200
    out = ctx.search(bounds, de, seed=3, t_begin=t0, t_end=t1)
    p = out["params"].cpu().numpy().reshape(16, t1 - t0, 3)
    n_t = t1 - t0
    boxes = [L.sample_bounds(bounds, t0 + tt) for tt in range(n_t)]
    n_checked = 0
    for tt in range(n_t):
        if tt % 3 == 0:
            continue
        ta = tt - tt % 3
        tb = ta + 3
        lo, hi = boxes[tt]
        if tb < n_t:
            w = np.float32(tt - ta) / np.float32(tb - ta)
            ref = p[:, ta] + w * (p[:, tb] - p[:, ta])
        else:
            ref = p[:, ta].copy()
        ref = np.minimum(np.maximum(ref, lo), hi)
        np.testing.assert_array_equal(p[:, tt], ref)
        n_checked += 16
    assert n_checked == 16 * (n_t - (n_t + 2) // 3)


def test_skip_cycles_never_lower_a_sample(line):
    ctx, g, wl, L = line
    base = dict(wl["de"], np_lo=12, np_hi=12, ng_f=5, n_bucket=6, n_skip=2)
    bounds = base_bounds(wl)
    s0 = ctx.search(bounds, dict(base, n_cycle=0), seed=9, t_begin=60, t_end=240)["S"]
    s1 = ctx.search(bounds, dict(base, n_cycle=1), seed=9, t_begin=60, t_end=240)["S"]
    s2 = ctx.search(bounds, dict(base, n_cycle=2), seed=9, t_begin=60, t_end=240)["S"]
    assert torch.all(s1 >= s0) and torch.all(s2 >= s1)
    assert (s1 > s0).float().mean() > 0.2


def test_skip_graph_replay_matches_eager(ens, line):
    _, g, wl, _ = line
    de = dict(wl["de"], np_lo=16, np_hi=16, ng_f=6, n_bucket=8, n_skip=2)
    bounds = base_bounds(wl)

    def make(stream=None):
        c = ens.Context(stream)
        c.bind(torch.from_numpy(g.traces).cuda(), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"],
               wl["window"], wl["ap_lo"], wl["ap_hi"])
        return c

    eager = make()
    eager.set_tuning(waves_per_sample_group=2, item_order=2)
    ref = eager.search(bounds, de, seed=17)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        gctx = make(s)
        gctx.set_tuning(waves_per_sample_group=2, item_order=2, use_graph=1)
        for rep in range(3):
            out = gctx.search(bounds, de, seed=17)
            torch.cuda.synchronize()
            assert torch.equal(out["params"], ref["params"]), rep
            assert torch.equal(out["S"], ref["S"]), rep
            assert out["n_evals"] == ref["n_evals"]
            x = torch.randn(1 << 20, device="cuda")
            (x * 2).sum().item()


def test_skip_requires_ens_and_range(line):
    ctx, g, wl, L = line
    bounds = base_bounds(wl)
    with pytest.raises(RuntimeError):
        ctx.search(bounds, dict(wl["de"], n_skip=3), seed=1)
    with pytest.raises(RuntimeError):
        ctx.search(bounds, dict(wl["de"], ens_enabled=0, n_skip=1), seed=1)
