"""The hand-written adjoint (semblance_backward) and the gradient polish
against the oracle, through the C-ABI.

The objective is eq. Sf's semblance (section "Traveltime parameter search");
its derivative through the interpolated gather (held M, right derivative at
whole samples) is compared per element with the oracle's binary64 gradient on
the same stored traces, in box-normalised units (dS/dz = dS/dp (hi - lo)):

    |g_gpu - g_64| <= 1e-3 max(|g_64|, median over the batch of |g_64|)

for every pair except those the definition makes ill-conditioned, which are
excluded and counted: a trace within 0.05 samples of a participation edge (M
itself may differ), or a traveltime within the binary32 error (4e-6 of the
moveout) of a whole sample, where the interpolation's derivative jumps."""
import numpy as np
import pytest

import oracle
from tests._tol import s_tol
from synth import base_bounds, make_workload, random_candidates

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EDGE = 0.05      # samples
KINK = 4e-6      # relative to 1 + moveout (samples)
REL = 1e-3


@pytest.fixture(scope="module")
def ens():
    import paper_2304_11399_amd as e
    assert torch.cuda.is_available()
    return e


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _setup(ens, name, store, n_cmp):
    g, wl = make_workload(name, n_cmp=n_cmp)
    ctx = ens.Context()
    ctx.bind(_dev(g.traces), g.cmp_ptr, g.offset, g.dt, g.dx, wl["op"], wl["window"], wl["ap_lo"],
             wl["ap_hi"], store=store)
    traces = None
    if store != "f32":
        q, s = oracle.quantize(g.traces, store)
        traces = oracle.dequantize(q, s, store)
    L = oracle.Line.from_gather(g, wl["window"], wl["op"], wl["ap_lo"], wl["ap_hi"], traces=traces)
    return ctx, g, wl, L


# crs_ens: binary32 traces at the C2 geometry; crs_diff: binary16 traces at the
# C5 geometry (2 ms, 96 offsets to 2400 m, 40 Hz, aperture +-8: up to 1632 traces)
@pytest.mark.parametrize("name,store,n_cmp", [("crs_ens", "f32", 48), ("crs_diff", "f16", 40)])
def test_adjoint_matches_oracle_gradient_per_element(ens, name, store, n_cmp):
    ctx, g, wl, L = _setup(ens, name, store, n_cmp)
    bounds = base_bounds(wl)
    # at the C5 geometry about half the candidates have one of their up to
    # 1632 traces at a whole-sample kink, so draw enough to compare >= 1000
    cmp, t, p = random_candidates(3200, g.n_cmp, g.nt, g.dt, 3, bounds, seed=19,
                                  t_range=(20, g.nt))
    dS = np.ones(cmp.size, np.float32)
    gr = ctx.semblance_backward(_dev(cmp), _dev(t), _dev(p), _dev(dS)).cpu().numpy()
    p64 = p.astype(np.float64)
    _, g_or = L.semblance_grad(cmp, t, p64)
    _, _, margin = L.semblance(cmp, t, p64)
    kink = L.kink_margin(cmp, t, p64)
    span = np.stack([np.subtract(*L.sample_bounds(bounds, tt)[::-1]) for tt in t])
    gz, gz_or = gr.astype(np.float64) * span, g_or * span
    edge, at_kink = margin < EDGE, kink < KINK
    keep = ~edge & ~at_kink
    print(f"{name} {store}: {cmp.size} pairs, excluded {edge.sum()} at a participation edge, "
          f"{(at_kink & ~edge).sum()} at a whole-sample kink; {keep.sum()} compared")
    assert keep.sum() >= 1000
    for d in range(3):
        scale = np.maximum(np.abs(gz_or[keep, d]), np.median(np.abs(gz_or[keep, d])))
        rel = np.abs(gz[keep, d] - gz_or[keep, d]) / scale
        print(f"  d={d}: max rel {rel.max():.2e}, 99% {np.quantile(rel, 0.99):.2e}")
        assert rel.max() <= REL, f"d={d}: worst pair {np.argmax(rel)} rel {rel.max():.3e}"


@pytest.mark.parametrize("name,store,n_cmp", [("crs_diff", "f16", 24), ("crs_ens", "f32", 24)])
def test_polish_matches_oracle_polish_from_the_same_start(ens, name, store, n_cmp):
    ctx, g, wl, L = _setup(ens, name, store, n_cmp)
    bounds = base_bounds(wl)
    t0, t1 = 100, min(g.nt, 700)
    de = dict(wl["de"], np_lo=12, np_hi=12, ng_f=6, n_bucket=12, polish_steps=0)
    start = ctx.search(bounds, de, seed=6, t_begin=t0, t_end=t1)
    post = ctx.search(bounds, dict(de, polish_steps=10, polish_lr=0.01), seed=6, t_begin=t0,
                      t_end=t1, keep_pre_polish=True)
    # the evolution is deterministic: the polish starts from the unpolished result
    assert torch.equal(post["S_pre_polish"], start["S"])
    assert torch.all(post["S"] >= post["S_pre_polish"])
    cmp = np.repeat(np.arange(n_cmp), t1 - t0).astype(np.int32)
    tt = np.tile(np.arange(t0, t1), n_cmp).astype(np.int32)
    p0 = start["params"].cpu().numpy().reshape(-1, 3)
    p_or, S_or = L.polish(bounds, cmp, tt, p0, 0.01, 10)
    S_gpu_at, _, _ = L.semblance(cmp, tt, post["params"].cpu().numpy().reshape(-1, 3).astype(np.float64))
    S0_or, _, _ = L.semblance(cmp, tt, p0.astype(np.float64))
    assert np.all(S_or >= S0_or)
    gain_gpu, gain_or = S_gpu_at - S0_or, S_or - S0_or
    # the polish keeps the step with the best score in the store's arithmetic:
    # between two points whose exact S differ by less than the sum of their
    # score errors it may keep either, so a sample's bound adds both
    # points' per-candidate tolerances (binary32 stores: 1e-5 each)
    p_gpu = post["params"].cpu().numpy().reshape(-1, 3)
    bound = 1e-4 + s_tol(store, L, cmp, tt, p_gpu) + s_tol(store, L, cmp, tt, p_or)
    same_acc = np.mean(np.abs(S_gpu_at - S_or) <= bound)
    print(f"{name} {store}: mean S start {S0_or.mean():.6f}, after GPU polish {S_gpu_at.mean():.6f}, "
          f"after oracle polish {S_or.mean():.6f}; mean gain GPU {gain_gpu.mean():.3e} oracle "
          f"{gain_or.mean():.3e}; within the bound of the oracle's polish: {same_acc:.3f}")
    # the same Adam steps from the same start: the two polished panels agree in
    # mean to 2% of the oracle's mean gain (plus 1e-6), and sample by sample
    # within the bound in the large majority (a binary32 gradient may take a
    # step the binary64 one does not)
    assert abs(S_gpu_at.mean() - S_or.mean()) <= 0.02 * gain_or.mean() + 1e-6
    assert same_acc >= 0.9


def test_adjoint_matches_central_differences_of_the_device_objective(ens):
    """semblance_backward against central differences of the device's own
    binary64 re-score of the same binary32 traces.  The interpolated
    semblance has a kink wherever a trace's traveltime crosses a whole sample,
    and with up to 816 traces per candidate a step of 1e-4 of the box span
    straddles one in 96% of the candidates (the oracle's quotients); the
    quotient also divides the re-score's rounding (up to about 1e-11) by the
    step, which rules out steps much below 1e-5.  The step is 1e-5 of the
    span, and a quotient counts as a derivative only where S is smooth over
    [p - h, p + h]: pairs where the oracle's own quotient departs from its
    analytic gradient by more than 1e-5 are excluded and counted, as are the
    pairs the per-element test excludes (a trace within the binary32
    traveltime error of a whole sample, where the adjoint may take the other
    side's slope, or within 0.05 samples of a participation edge)."""
    ctx, g, wl, L = _setup(ens, "crs_ens", "f32", 48)
    bounds = base_bounds(wl)
    cmp, t, p = random_candidates(2000, g.n_cmp, g.nt, g.dt, 3, bounds, seed=23, t_range=(20, g.nt))
    span = np.stack([np.subtract(*L.sample_bounds(bounds, tt)[::-1]) for tt in t]).astype(np.float64)
    dS = np.ones(cmp.size, np.float32)
    g_gpu = ctx.semblance_backward(_dev(cmp), _dev(t), _dev(p), _dev(dS)).cpu().numpy().astype(np.float64)
    _, g_or = L.semblance_grad(cmp, t, p.astype(np.float64))
    keep = np.ones(cmp.size, bool)
    fd_gpu = np.zeros((cmp.size, 3))
    for d in range(3):
        h = (1e-5 * span[:, d]).astype(np.float32)
        pp, pm = p.copy(), p.copy()
        pp[:, d] = p[:, d] + h
        pm[:, d] = p[:, d] - h
        step = pp[:, d].astype(np.float64) - pm[:, d].astype(np.float64)
        Sp = ctx.semblance_eval64(_dev(cmp), _dev(t), _dev(pp)).cpu().numpy()
        Sm = ctx.semblance_eval64(_dev(cmp), _dev(t), _dev(pm)).cpu().numpy()
        fd_gpu[:, d] = (Sp - Sm) / step
        Sp_or, _, _ = L.semblance(cmp, t, pp.astype(np.float64))
        Sm_or, _, _ = L.semblance(cmp, t, pm.astype(np.float64))
        fd_or = (Sp_or - Sm_or) / step
        scale_or = np.maximum(np.abs(g_or[:, d]), np.median(np.abs(g_or[:, d])))
        keep &= np.abs(fd_or - g_or[:, d]) <= 1e-5 * scale_or
    smooth = keep.copy()
    _, _, margin = L.semblance(cmp, t, p.astype(np.float64))
    keep &= (margin >= EDGE) & (L.kink_margin(cmp, t, p.astype(np.float64)) >= KINK)
    print(f"central differences: {cmp.size} pairs, {(~smooth).sum()} excluded where S is not smooth "
          f"over the step, {(smooth & ~keep).sum()} at an edge or within rounding of a kink; "
          f"{keep.sum()} compared")
    assert keep.sum() >= 1000
    for d in range(3):
        gz, fz = g_gpu[keep, d] * span[keep, d], fd_gpu[keep, d] * span[keep, d]
        scale = np.maximum(np.abs(fz), np.median(np.abs(fz)))
        rel = np.abs(gz - fz) / scale
        print(f"  d={d}: max rel {rel.max():.2e}, 99% {np.quantile(rel, 0.99):.2e}")
        assert rel.max() <= REL, f"d={d}: worst pair {np.argmax(rel)} rel {rel.max():.3e}"
