"""Edge cases of the GPU search against the oracle: one-sample grids, buckets
larger than the line, line ends, the smallest and largest populations and
windows, the CMP operator under ENS, the record's first and last samples, and
the longest records binary16 windows take."""
import numpy as np
import pytest

import oracle
from synth import base_bounds, make_workload, random_candidates
from tests._tol import s_tol

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


@pytest.mark.parametrize("nt", [4080, 6000, 12000, 16368])
def test_long_records_in_binary16(ens, nt):
    # the binary16 windows' traveltime grid coarsens with the record (2^-11
    # samples up to 4080 samples, 2^-10 up to 8176, 2^-9 up to the limit of
    # 16368); candidates over the whole record hold the tolerance of its grid
    g, wl = make_workload("crs_ens", n_cmp=8, nt=nt)
    ctx = ens.Context()
    ctx.bind(torch.from_numpy(g.traces).cuda(), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"],
             wl["window"], wl["ap_lo"], wl["ap_hi"], store="f16")
    q, s = oracle.quantize(g.traces, "f16")
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"],
                                traces=oracle.dequantize(q, s, "f16"))
    cmp, t, p = random_candidates(4000, g.n_cmp, g.nt, g.dt, 3, base_bounds(wl), seed=nt)
    S, M = ctx.semblance_eval(torch.from_numpy(cmp).cuda(), torch.from_numpy(t).cuda(),
                              torch.from_numpy(p).cuda(), with_M=True)
    S, M = S.cpu().numpy().astype(np.float64), M.cpu().numpy()
    S_or, M_or, margin = L.semblance(cmp, t, p.astype(np.float64))
    flip = M != M_or
    assert np.all(margin[flip] < 0.05) and flip.mean() < 1e-3
    ok = ~flip
    err = np.abs(S - S_or)[ok]
    bound = s_tol("f16", L, cmp[ok], t[ok], p[ok])
    print(f"nt={nt}: {cmp.size} candidates, {np.sum(t > 4096)} past sample 4096, max|dS| "
          f"{err.max():.2e} ({np.max(err / bound):.3f} of the bound)")
    assert np.all(err <= bound)


def test_binary16_record_limit(ens):
    g, wl = make_workload("crs_ens", n_cmp=2, nt=ens.MAX_NT_F16 + 1)
    args = (torch.from_numpy(g.traces).cuda(), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"],
            wl["window"], wl["ap_lo"], wl["ap_hi"])
    ctx = ens.Context()
    with pytest.raises(ens.EnsError, match="binary16 windows take records of at most 16368"):
        ctx.bind(*args, store="f16")
    # bfloat16 and binary32 windows take exact traveltimes: no such limit
    for store in ("bf16", "f32"):
        ctx.bind(*args, store=store)
        S = ctx.semblance_eval(torch.tensor([0, 1], dtype=torch.int32).cuda(),
                               torch.tensor([100, g.nt - 1], dtype=torch.int32).cuda(),
                               torch.zeros(2, 3).cuda())
        assert torch.isfinite(S).all()
