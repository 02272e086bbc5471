"""ens_stack_noalloc (the entry point that allocates nothing, for callers that
cannot allocate device memory) against ens_stack through the C-ABI: the same
stack and coherence RMS bitwise, on two calls in a row, the second smaller."""
import numpy as np
import pytest

from synth import base_bounds, make_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bound():
    import paper_2304_11399_amd as ens
    assert torch.cuda.is_available()
    g, wl = make_workload("crs_ens", n_cmp=20, nt=300)
    ctx = ens.Context()
    ctx.bind(torch.from_numpy(g.traces).cuda(), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"],
             wl["window"], wl["ap_lo"], wl["ap_hi"], store="f16")
    de = dict(wl["de"], np_lo=12, np_hi=12, ng_f=5, n_bucket=10)
    return ens, ctx, g, wl, de


def _pair(ctx, out, cmp_out, t0, t1):
    ref, rms_ref = ctx.stack(out["params"], out["S"], cmp_out=cmp_out, t_begin=t0, t_end=t1)
    # a caller tensor filled with garbage: every element must be written
    dst = torch.full_like(ref, float("nan"))
    got, rms = ctx.stack(out["params"], out["S"], cmp_out=cmp_out, t_begin=t0, t_end=t1, out=dst,
                         noalloc=True)
    torch.cuda.synchronize()
    assert got.data_ptr() == dst.data_ptr()
    assert torch.equal(got, ref)
    assert rms == rms_ref
    return ref


def test_noalloc_stack_equals_stack_on_two_calls_the_second_smaller(bound):
    ens, ctx, g, wl, de = bound
    big = ctx.search(base_bounds(wl), de, seed=3, t_begin=10, t_end=290)
    _pair(ctx, big, None, 10, 290)                         # every CMP, 280 times
    cmp_small = [2, 3, 4, 5, 6, 7, 8, 9]
    small = ctx.search(base_bounds(wl), de, seed=4, cmp_out=cmp_small, t_begin=50, t_end=120)
    ref = _pair(ctx, small, cmp_small, 50, 120)            # 8 CMPs, 70 times
    assert ref.shape == (8, 70) and torch.isfinite(ref).all()
    # and without the coherence panel
    a, _ = ctx.stack(small["params"], cmp_out=cmp_small, t_begin=50, t_end=120)
    b, rms = ctx.stack(small["params"], cmp_out=cmp_small, t_begin=50, t_end=120, noalloc=True)
    assert rms is None and torch.equal(a, b)


def test_noalloc_stack_rejects_more_output_cmps_than_its_array_holds(bound):
    ens, ctx, g, wl, de = bound
    n = 65537
    cmp_out = np.zeros(n, np.int32)
    params = torch.zeros((n, 1, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(ens.EnsError) as e:
        ctx.stack(params, cmp_out=cmp_out, t_begin=0, t_end=1, noalloc=True)
    assert e.value.status == -2 and "at most 65536" in str(e.value)
