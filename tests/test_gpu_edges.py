"""Edge cases of the GPU search against the oracle: one-sample grids, buckets
larger than the line, line ends, the smallest and largest populations and
windows, the CMP operator under ENS, the record's first and last samples."""
import numpy as np
import pytest

import oracle
from synth import base_bounds, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_S = 1e-5


@pytest.fixture(scope="module")
def ens():
    import paper_2304_11399_amd as e
    assert torch.cuda.is_available()
    return e


def _run(ens, name, de_over, grid, seed, min_same=0.9, **wl_over):
    g, wl = make_workload(name, **wl_over)
    ctx = ens.Context()
    ctx.bind(torch.from_numpy(g.traces).cuda(), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"],
             wl["window"], wl["ap_lo"], wl["ap_hi"])
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"])
    de = dict(wl["de"], **de_over)
    bounds = base_bounds(wl)
    cmp_out, t0, t1 = grid
    out = ctx.search(bounds, de, seed=seed, cmp_out=cmp_out, t_begin=t0, t_end=t1)
    p_or, S_run, ev = L.search(bounds, de, seed, cmp_out=None if cmp_out is None else
                               np.asarray(cmp_out, np.int32), t_begin=t0, t_end=t1)
    assert out["n_evals"] == ev
    outs = np.arange(g.n_cmp) if cmp_out is None else np.asarray(cmp_out)
    cmp = np.repeat(outs, t1 - t0).astype(np.int32)
    t = np.tile(np.arange(t0, t1), len(outs)).astype(np.int32)
    P = wl["op"]
    p = out["params"].cpu().numpy().reshape(-1, P)
    S = out["S"].cpu().numpy().reshape(-1).astype(np.float64)
    S_or, _, margin = L.semblance(cmp, t, p.astype(np.float64))
    ok = margin >= 0.05
    if ok.any():
        assert np.abs(S - S_or)[ok].max() <= TOL_S
    same = np.all(p == p_or.reshape(-1, P), axis=1).mean()
    print(f"{name} {de_over} grid={grid}: identical {same:.3f}, evals {ev}")
    assert same >= min_same
    return out


def test_single_time_sample_and_bucket_larger_than_the_line(ens):
    _run(ens, "crs_ens", dict(np_lo=16, np_hi=16, ng_f=3, n_bucket=8), ([2, 3, 4], 150, 151), 1,
         n_cmp=12, nt=300)


def test_line_ends_with_truncated_apertures(ens):
    _run(ens, "crs_ens", dict(np_lo=16, np_hi=16, ng_f=3, n_bucket=2), ([0, 1, 10, 11], 40, 90), 2,
         n_cmp=12, nt=300)


@pytest.mark.parametrize("np_", [4, 64])
def test_smallest_and_largest_population(ens, np_):
    # NP 4 cannot run the backward/forward stages (NP_bf >= 5 is a separate knob)
    _run(ens, "crs_ens", dict(np_lo=np_, np_hi=np_, ng_f=2, n_bucket=4, ens_enabled=int(np_ == 64)),
         (None, 60, 100), 3, n_cmp=8, nt=200)


@pytest.mark.parametrize("window", [3, 15])
def test_smallest_and_largest_window(ens, window):
    _run(ens, "crs_ens", dict(np_lo=16, np_hi=16, ng_f=3, n_bucket=4), (None, 30, 90), 4,
         n_cmp=8, nt=200, window=window)


def test_cmp_operator_under_ens_with_two_cycles(ens):
    _run(ens, "cmp_small", dict(np_lo=16, np_hi=16, ng_f=3, ens_enabled=1, n_cycle=2, n_bucket=4,
                                np_bf=6, ng_bf=1), (None, 0, 256), 5)


def test_first_and_last_record_samples(ens):
    # n0 = 0 (zero t0: the moveout guard) and n0 = nt - 1 (most traces past the record)
    g_nt = 200
    out = _run(ens, "crs_ens", dict(np_lo=16, np_hi=16, ng_f=3, n_bucket=4), (None, 0, 3), 6,
               n_cmp=8, nt=g_nt)
    assert torch.isfinite(out["S"]).all()
    out = _run(ens, "crs_ens", dict(np_lo=16, np_hi=16, ng_f=3, n_bucket=4), (None, g_nt - 3, g_nt), 7,
               n_cmp=8, nt=g_nt)
    assert torch.isfinite(out["S"]).all()
