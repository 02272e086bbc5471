"""LDS-staged binary32 windows (ens_tuning.gather = 1): the staged samples
and the arithmetic are those of the direct reads, so every search result is
bit for bit the same (plain search, ENS with time skipping, JADE, the CMP
operator, every slice count)."""
import pytest

from synth import base_bounds, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ens():
    import paper_2304_11399_amd as e
    assert torch.cuda.is_available()
    return e


def _ctx(ens, g, wl):
    ctx = ens.Context()
    ctx.bind(torch.from_numpy(g.traces).cuda(), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"],
             wl["window"], wl["ap_lo"], wl["ap_hi"], store="f32")
    return ctx


@pytest.mark.parametrize("name,extra", [
    ("crs_ens", dict(np_lo=16, np_hi=16, ng_f=4, n_bucket=6)),
    ("crs_ens", dict(np_lo=16, np_hi=16, ng_f=4, n_bucket=6, n_skip=1)),
    ("crs_ens", dict(np_lo=16, np_hi=16, ng_f=4, n_bucket=6, adapt=1, CR=0.5)),
    ("crs_uneven", dict(ng_f=3, n_bucket=6)),
    ("crs_ens", dict(np_lo=24, np_hi=24, ng_f=5, ens_enabled=0)),
    ("cmp_small", dict(ng_f=6)),
])
def test_staged_windows_equal_direct_reads(ens, name, extra):
    g, wl = make_workload(name, n_cmp=20, nt=300) if name != "cmp_small" else make_workload(name)
    ctx = _ctx(ens, g, wl)
    de = dict(wl["de"], **extra)
    for nsl in (1, 2, 4):
        ctx.set_tuning(waves_per_sample_group=nsl, item_order=1, occupancy=1, packing=1)
        ref = ctx.search(base_bounds(wl), de, seed=9)
        ctx.set_tuning(waves_per_sample_group=nsl, item_order=1, occupancy=1, packing=1, gather=1)
        out = ctx.search(base_bounds(wl), de, seed=9)
        assert torch.equal(ref["params"], out["params"]), nsl
        assert torch.equal(ref["S"], out["S"]), nsl
        assert ref["n_evals"] == out["n_evals"] and ref["sum_m"] == out["sum_m"]
