"""Packed exploration workgroups (ens_tuning.packing): the populations of
consecutive samples laid end to end over 2, 4 or 8 waves give the same
search as one population per lane group, bit for bit, on uneven populations
(NP 16 -> 64 with t, so that populations straddle waves), for the plain
search, ENS stage 0 with exchange and with time-sample skipping (N_skip 1
and 2), on binary32, binary16 and bfloat16 rows, and
through the measured launch shape (against the fixed shape it picks)."""
import numpy as np
import pytest

from synth import base_bounds, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ens():
    import paper_2304_11399_amd as e
    assert torch.cuda.is_available()
    return e


def _ctx(ens, g, wl, store="f32"):
    ctx = ens.Context()
    ctx.bind(torch.from_numpy(g.traces).cuda(), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"],
             wl["window"], wl["ap_lo"], wl["ap_hi"], store=store)
    return ctx


def _same(a, b):
    assert torch.equal(a["params"], b["params"])
    assert torch.equal(a["S"], b["S"])
    assert a["n_evals"] == b["n_evals"] and a["sum_m"] == b["sum_m"]


@pytest.mark.parametrize("store", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("mode", ["plain", "ens", "ens_skip1", "ens_skip2"])
def test_packed_exploration_equals_one_population_per_lane_group(ens, mode, store):
    g, wl = make_workload("crs_uneven", n_cmp=20, nt=400)
    ctx = _ctx(ens, g, wl, store)
    de = dict(wl["de"], np_lo=16, np_hi=64, ng_f=4, ng_bf=1, n_bucket=6)
    if mode == "plain":
        de["ens_enabled"] = 0
    if mode.startswith("ens_skip"):
        de["n_skip"] = int(mode[-1])
    # t from 37 (a ragged start) to 391: populations of 17..63 members
    kw = dict(seed=11, t_begin=37, t_end=391)
    ctx.set_tuning(waves_per_sample_group=1, item_order=1, occupancy=1, packing=1)
    ref = ctx.search(base_bounds(wl), de, **kw)
    assert ctx.stats()["explore"]["packed"] == 0
    for waves in (2, 4, 8):
        for occ in (1, 2):
            # the slices and order apply to the exploitation launches only
            ctx.set_tuning(waves_per_sample_group=1, item_order=1, occupancy=occ, packing=waves)
            out = ctx.search(base_bounds(wl), de, **kw)
            assert ctx.stats()["explore"]["packed"] == waves
            _same(ref, out)
    for order in (2, 3):   # costliest items first; the same within XCD shares
        ctx.set_tuning(waves_per_sample_group=1, item_order=order, occupancy=1, packing=4)
        out = ctx.search(base_bounds(wl), de, **kw)
        assert ctx.stats()["explore"]["item_order"] == order
        _same(ref, out)
    # the measured shapes: slices change the order of the window sums, so
    # the search is compared bit for bit with the one population per lane
    # group run only where no launch uses slices, else with a run of the
    # fixed shape it picked (plain search: one launch kind)
    ctx.set_tuning(0)
    out = ctx.search(base_bounds(wl), de, **kw)
    st = ctx.stats()
    ex = st["explore"]
    assert out["n_evals"] == ref["n_evals"] and out["sum_m"] == ref["sum_m"]
    if ex["packed"] and (mode == "plain" or st["exploit"]["waves"] == 1):
        _same(ref, out)
    elif mode == "plain":
        ctx.set_tuning(waves_per_sample_group=ex["waves"], item_order=ex["item_order"],
                       occupancy=1 + ex["dense"], packing=max(1, ex["packed"]))
        _same(ctx.search(base_bounds(wl), de, **kw), out)


def test_packing_is_not_used_with_adaptation_or_fixed_slices(ens):
    g, wl = make_workload("crs_ens", n_cmp=12, nt=200)
    ctx = _ctx(ens, g, wl)
    de = dict(wl["de"], np_lo=16, np_hi=16, ng_f=3, n_bucket=6, adapt=1)
    ctx.set_tuning(packing=4)
    ctx.search(base_bounds(wl), de, seed=3)
    assert ctx.stats()["explore"]["packed"] == 0
    ctx.set_tuning(waves_per_sample_group=2)
    ctx.search(base_bounds(wl), dict(de, adapt=0), seed=3)
    assert ctx.stats()["explore"]["packed"] == 0


def test_packed_lanes_cover_a_line_end_and_single_samples(ens):
    # a grid of one sample and a grid whose last item holds one population
    g, wl = make_workload("crs_uneven", n_cmp=8, nt=300)
    ctx = _ctx(ens, g, wl)
    de = dict(wl["de"], np_lo=60, np_hi=64, ng_f=3, n_bucket=4)
    for t0, t1 in ((150, 151), (0, 300), (290, 300)):
        ctx.set_tuning(waves_per_sample_group=1, item_order=1, packing=1)
        ref = ctx.search(base_bounds(wl), de, seed=5, t_begin=t0, t_end=t1)
        ctx.set_tuning(waves_per_sample_group=1, item_order=1, packing=2)
        _same(ref, ctx.search(base_bounds(wl), de, seed=5, t_begin=t0, t_end=t1))
        assert ctx.stats()["explore"]["packed"] == 2
