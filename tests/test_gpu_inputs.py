"""The boundary's input forms (through the C-ABI): caller-quantised 16-bit
traces with power-of-two scales and an optional binary32 master, 16-bit data
kept as binary32, and the one-call ens_search against ens_bind followed by
ens_search_bound (section "Traveltime parameter search": f(p) = S(p; #data,
#config), eq. Sf)."""
import numpy as np
import pytest

import oracle
from synth import base_bounds, make_workload, random_candidates

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_S = 1e-5
MARGIN = 0.05


@pytest.fixture(scope="module")
def ens():
    import paper_2304_11399_amd as e
    assert torch.cuda.is_available()
    return e


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _small():
    g, wl = make_workload("crs_precision", n_cmp=24, nt=300)
    de = dict(wl["de"], np_lo=12, np_hi=12, ng_f=6, n_bucket=8)
    return g, wl, de


def _same(a, b):
    for k in ("params", "S", "S64"):
        np.testing.assert_array_equal(a[k].cpu().numpy(), b[k].cpu().numpy(), err_msg=k)
    assert a["n_evals"] == b["n_evals"] and a["sum_m"] == b["sum_m"]


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_caller_quantised_traces_search_like_the_library_quantiser(ens, dtype):
    g, wl, de = _small()
    tr = _dev(g.traces)
    args = (g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"], wl["window"], wl["ap_lo"], wl["ap_hi"])
    ref_ctx = ens.Context()
    ref_ctx.bind(tr, *args, store=dtype)
    ref = ref_ctx.search(base_bounds(wl), de, 5)
    q, s = ref_ctx.quantize(tr, dtype)
    # the caller's q and scales with the binary32 samples as master: the same bits
    ctx = ens.Context()
    ctx.bind(q, *args, scale=s, master=tr, data_dtype=dtype)
    _same(ref, ctx.search(base_bounds(wl), de, 5))
    # without a master the binary64 re-score reads the dequantised samples
    ctx2 = ens.Context()
    ctx2.bind(q, *args, scale=s, data_dtype=dtype)
    out = ctx2.search(base_bounds(wl), de, 5)
    np.testing.assert_array_equal(out["params"].cpu().numpy(), ref["params"].cpu().numpy())
    qn, sn = oracle.quantize(g.traces, dtype)
    Lq = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"],
                                 traces=oracle.dequantize(qn, sn, dtype))
    n_out, n_t = out["S"].shape
    cmp = np.repeat(np.arange(n_out), n_t).astype(np.int32)
    t = np.tile(np.arange(n_t), n_out).astype(np.int32)
    S_or, _, margin = Lq.semblance(cmp, t, out["params"].cpu().numpy().reshape(-1, 3).astype(np.float64))
    ok = margin > 1e-6
    assert np.abs(out["S64"].cpu().numpy().reshape(-1) - S_or)[ok].max() < 1e-11


def test_sixteen_bit_data_stored_as_binary32_are_the_dequantised_samples(ens):
    g, wl, _ = _small()
    q, s = oracle.quantize(g.traces, "f16")
    deq = oracle.dequantize(q, s, "f16")
    ctx = ens.Context()
    ctx.bind(_dev(q.view(np.int16)), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"], wl["window"],
             wl["ap_lo"], wl["ap_hi"], store="f32", scale=_dev(s), data_dtype="f16")
    Lq = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"], traces=deq)
    cmp, t, p = random_candidates(6000, g.n_cmp, g.nt, g.dt, 3, base_bounds(wl), seed=4)
    S, M = ctx.semblance_eval(_dev(cmp), _dev(t), _dev(p), with_M=True)
    S_or, M_or, margin = Lq.semblance(cmp, t, p.astype(np.float64))
    ok = margin >= MARGIN
    assert np.abs(S.cpu().numpy() - S_or)[ok].max() <= TOL_S
    np.testing.assert_array_equal(M.cpu().numpy()[ok], M_or[ok])


def test_scales_that_are_not_powers_of_two_are_rejected(ens):
    g, wl, _ = _small()
    q, s = oracle.quantize(g.traces, "f16")
    s = s.copy()
    s[3] *= 1.5
    ctx = ens.Context()
    with pytest.raises(ens.EnsError) as e:
        ctx.bind(_dev(q.view(np.int16)), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"], wl["window"],
                 wl["ap_lo"], wl["ap_hi"], scale=_dev(s), data_dtype="f16")
    assert e.value.status == -2 and "power of two" in str(e.value)


@pytest.mark.parametrize("store", ["f32", "f16"])
def test_one_call_search_equals_bind_then_search_bound(ens, store):
    g, wl, de = _small()
    tr = _dev(g.traces)
    ctx = ens.Context()
    ctx.bind(tr, g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"], wl["window"], wl["ap_lo"], wl["ap_hi"],
             store=store)
    a = ctx.search(base_bounds(wl), de, 9, cmp_out=[3, 4, 5, 6, 7, 8, 9, 10, 11], t_begin=40,
                   t_end=260)
    b = ens.ens_search(tr, (g.cmp_ptr, g.offset, g.dt, g.dx), ([3, 4, 5, 6, 7, 8, 9, 10, 11], 40, 260),
                       base_bounds(wl), de, 9, op=wl["op"], window=wl["window"], ap_lo=wl["ap_lo"],
                       ap_hi=wl["ap_hi"], store=store)
    _same(a, b)
