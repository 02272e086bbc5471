"""MI355X-native windowed-semblance traveltime-parameter search with evolution
by neighbourhood similarity (arXiv 2304.11399).

Thin ctypes binding over ``libens.so`` (include/ens.h).  Every step of the
search runs in the library's HIP kernels; this module only marshals torch
device tensors (memory and the current stream) into the C calls.  There is
no fallback: if the library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .counts import evals_ens, evals_jade  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libens.so")

DTYPES = {"f32": 0, "f16": 1, "bf16": 2}
OPS = {"cmp": 1, "crs": 3, 1: 1, 3: 3}

MAX_NT_F16 = 16368   # longest record searched in binary16 (ens.h ENS_MAX_NT_F16)

ENS_OK = 0
STATUS = {0: "ENS_OK", -1: "ENS_E_INVALID", -2: "ENS_E_RANGE", -3: "ENS_E_HIP", -4: "ENS_E_OOM",
          -5: "ENS_E_UNSUPPORTED", -6: "ENS_E_STATE"}


class EnsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


# ----------------------------------------------------------------- structs
class Traces(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("data", C.c_void_p), ("n_traces", C.c_int64),
                ("nt", C.c_int32), ("ld", C.c_int64), ("dt", C.c_float), ("store_dtype", C.c_int32),
                ("data_dtype", C.c_int32), ("scale", C.c_void_p), ("master", C.c_void_p)]


class Geometry(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("cmp_ptr", C.c_void_p), ("n_cmp", C.c_int32),
                ("dx", C.c_float), ("offset", C.c_void_p)]


class SemCfg(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("op", C.c_int32), ("window", C.c_int32),
                ("ap_lo", C.c_int32), ("ap_hi", C.c_int32)]


class T0Grid(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("cmp_out", C.c_void_p), ("n_cmp_out", C.c_int32),
                ("t_begin", C.c_int32), ("t_end", C.c_int32)]


class Bounds(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("lo", C.c_float * 3), ("hi", C.c_float * 3),
                ("inv_t0_mask", C.c_uint32)]


class DeCfg(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("np_lo", C.c_int32), ("np_hi", C.c_int32),
                ("ng_f", C.c_int32), ("np_bf", C.c_int32), ("ng_bf", C.c_int32),
                ("n_cycle", C.c_int32), ("n_skip", C.c_int32), ("n_bucket", C.c_int32),
                ("ens_enabled", C.c_int32), ("inject", C.c_int32), ("F", C.c_float),
                ("CR", C.c_float), ("polish_steps", C.c_int32), ("polish_lr", C.c_float),
                ("rescore_fp64", C.c_int32), ("adapt", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("params", C.c_void_p), ("S", C.c_void_p),
                ("S64", C.c_void_p), ("S_pre_polish", C.c_void_p), ("n_evals", C.c_int64),
                ("sum_m", C.c_int64)]


class Candidates(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n", C.c_int64), ("cmp", C.c_void_p),
                ("t", C.c_void_p), ("params", C.c_void_p)]


class Tuning(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("waves_per_sample_group", C.c_int32),
                ("use_graph", C.c_int32), ("collect_timing", C.c_int32), ("item_order", C.c_int32),
                ("occupancy", C.c_int32), ("packing", C.c_int32), ("gather", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("launches", C.c_int64 * 4),
                ("evals", C.c_int64 * 4), ("sum_m", C.c_int64 * 4),
                ("device_ms", C.c_double * 4), ("waves_used", C.c_int32 * 2),
                ("order_used", C.c_int32 * 2), ("dense_used", C.c_int32 * 2),
                ("tune_ms", C.c_double), ("packed_used", C.c_int32)]


STAT_KINDS = ("explore", "exploit", "polish", "rescore64")


def _sized(cls, **kw):
    s = cls(**kw)
    s.struct_size = C.sizeof(cls)
    return s


# ----------------------------------------------------------------- library
_lib = None

# name -> (restype, argtypes); mirrors include/ens.h
_P = C.c_void_p
_SIGS = {
    "ens_version": (C.c_char_p, []),
    "ens_ctx_create": (C.c_int, [C.POINTER(C.c_void_p), _P]),
    "ens_ctx_destroy": (None, [_P]),
    "ens_last_error": (C.c_char_p, [_P]),
    "ens_set_tuning": (C.c_int, [_P, C.POINTER(Tuning)]),
    "ens_last_stats": (C.c_int, [_P, C.POINTER(Stats)]),
    "ens_bind": (C.c_int, [_P, C.POINTER(Traces), C.POINTER(Geometry), C.POINTER(SemCfg)]),
    "ens_quantize": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.c_int64, C.c_int32, _P, _P]),
    "ens_search_bound": (C.c_int, [_P, C.POINTER(T0Grid), C.POINTER(Bounds), C.POINTER(DeCfg),
                                   C.c_uint64, C.POINTER(Result)]),
    "ens_search": (C.c_int, [_P, C.POINTER(Traces), C.POINTER(Geometry), C.POINTER(SemCfg),
                             C.POINTER(T0Grid), C.POINTER(Bounds), C.POINTER(DeCfg), C.c_uint64,
                             C.POINTER(Result)]),
    "ens_stack": (C.c_int, [_P, C.POINTER(T0Grid), _P, _P, _P, C.POINTER(C.c_double)]),
    "ens_stack_noalloc": (C.c_int, [_P, C.POINTER(T0Grid), _P, _P, _P, C.POINTER(C.c_double)]),
    "ens_jade_draws": (C.c_int, [_P, C.c_int64, _P, C.c_double, C.c_double, C.c_int32, _P, _P, _P]),
    "semblance_eval": (C.c_int, [_P, C.POINTER(Candidates), _P, _P]),
    "semblance_eval64": (C.c_int, [_P, C.POINTER(Candidates), _P]),
    "semblance_backward": (C.c_int, [_P, C.POINTER(Candidates), _P, _P]),
    "ens_philox": (C.c_int, [_P, C.c_int64, _P, _P, _P]),
    "ens_de_trial": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, _P, _P, _P, C.c_float,
                               C.c_float, _P, _P, _P]),
}


def load():
    """Load libens.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _require_cuda(*tensors):
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libens needs a ROCm GPU; none is visible")
    for t in tensors:
        if t is not None and (not isinstance(t, torch.Tensor) or not t.is_cuda):
            raise TypeError("expected a device tensor")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """An ens_ctx bound to a torch stream (default: the current stream)."""

    def __init__(self, stream=None):
        import torch
        _require_cuda()
        self._lib = load()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        self._check(self._lib.ens_ctx_create(C.byref(h), C.c_void_p(self.stream.cuda_stream)), None)
        self._h = h
        self.nparam = None
        self._keep = []

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ens_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, h="self"):
        if st != ENS_OK:
            msg = self._lib.ens_last_error(self._h if h == "self" else h)
            raise EnsError(st, msg.decode() if msg else "")

    def last_error(self):
        return self._lib.ens_last_error(self._h).decode()

    def set_tuning(self, waves_per_sample_group=0, use_graph=0, collect_timing=0, item_order=0,
                   occupancy=0, packing=0, gather=0):
        """Launch shape of the search kernels (ens_tuning): slices, HIP-graph
        replay, per-launch timing, item order, register budget, packed
        exploration width (1: off) and LDS-staged binary32 windows (gather=1);
        0 = chosen by measurement (gather: direct reads)."""
        t = _sized(Tuning, waves_per_sample_group=waves_per_sample_group, use_graph=use_graph,
                   collect_timing=collect_timing, item_order=item_order, occupancy=occupancy,
                   packing=packing, gather=gather)
        self._check(self._lib.ens_set_tuning(self._h, C.byref(t)))

    def stats(self):
        """Per-kind launches, evaluations, participating traces and device ms of
        the last search."""
        st = _sized(Stats)
        self._check(self._lib.ens_last_stats(self._h, C.byref(st)))
        d = {k: dict(launches=int(st.launches[i]), evals=int(st.evals[i]),
                     sum_m=int(st.sum_m[i]), device_ms=float(st.device_ms[i]))
             for i, k in enumerate(STAT_KINDS)}
        for i, k in enumerate(STAT_KINDS[:2]):
            d[k]["waves"] = int(st.waves_used[i])
            d[k]["item_order"] = int(st.order_used[i])
            d[k]["dense"] = int(st.dense_used[i])
        d["tune_ms"] = float(st.tune_ms)
        d["explore"]["packed"] = int(st.packed_used)
        return d

    # -------------------------------------------------------------- data
    def _data_structs(self, traces, cmp_ptr, offset, dt, dx, op, window, ap_lo, ap_hi, store, scale,
                      master, data_dtype):
        import torch
        _require_cuda(traces, scale, master)
        assert traces.dim() == 2 and traces.stride(1) == 1
        if traces.dtype == torch.float32:
            data_dtype = "f32"
        elif traces.dtype == torch.float16:
            data_dtype = "f16"
        elif traces.dtype == torch.bfloat16:
            data_dtype = "bf16"
        else:
            assert traces.dtype in (torch.int16, torch.uint16) and data_dtype in ("f16", "bf16"), \
                "16-bit bit patterns need data_dtype 'f16' or 'bf16'"
        if data_dtype != "f32":
            assert scale is not None and scale.dtype == torch.float32 and scale.is_contiguous()
            assert scale.numel() == traces.shape[0]
            if master is not None:
                assert master.dtype == torch.float32 and master.stride() == traces.stride()
            store = data_dtype if store is None else store
        store = "f32" if store is None else store
        cmp_ptr = np.ascontiguousarray(cmp_ptr, dtype=np.int64)
        offset = np.ascontiguousarray(offset, dtype=np.float32)
        tr = _sized(Traces, data=traces.data_ptr(), n_traces=traces.shape[0], nt=traces.shape[1],
                    ld=traces.stride(0), dt=float(dt), store_dtype=DTYPES[store],
                    data_dtype=DTYPES[data_dtype], scale=None if scale is None else scale.data_ptr(),
                    master=None if master is None else master.data_ptr())
        geo = _sized(Geometry, cmp_ptr=cmp_ptr.ctypes.data, n_cmp=cmp_ptr.size - 1, dx=float(dx),
                     offset=offset.ctypes.data)
        sem = _sized(SemCfg, op=OPS[op], window=int(window), ap_lo=int(ap_lo),
                     ap_hi=int(ap_lo if ap_hi is None else ap_hi))
        return tr, geo, sem, (cmp_ptr, offset)

    def _bound_as(self, traces, cmp_ptr, op):
        self.nparam = OPS[op]
        self.nt = traces.shape[1]
        self.n_cmp = np.asarray(cmp_ptr).size - 1

    def bind(self, traces, cmp_ptr, offset, dt, dx, op, window, ap_lo=0, ap_hi=None,
             store=None, scale=None, master=None, data_dtype=None):
        """traces: device [n_traces, nt] (row stride taken from the tensor): float32
        samples, or 16-bit samples (float16 / bfloat16, or int16 bit patterns with
        data_dtype 'f16'/'bf16') with per-trace power-of-two scales and an
        optional float32 master.  store: the library's storage ('f32', 'f16',
        'bf16'; default: binary32 for binary32 data, else the data's type)."""
        tr, geo, sem, keep = self._data_structs(traces, cmp_ptr, offset, dt, dx, op, window, ap_lo,
                                                ap_hi, store, scale, master, data_dtype)
        self._check(self._lib.ens_bind(self._h, C.byref(tr), C.byref(geo), C.byref(sem)))
        self._bound_as(traces, cmp_ptr, op)

    def quantize(self, data, dtype):
        import torch
        _require_cuda(data)
        n_tr, nt = data.shape
        q = torch.empty((n_tr, nt), dtype=torch.int16, device=data.device)
        s = torch.empty(n_tr, dtype=torch.float32, device=data.device)
        self._check(self._lib.ens_quantize(self._h, _ptr(data), n_tr, nt, data.stride(0),
                                           DTYPES[dtype], _ptr(q), _ptr(s)))
        return q, s

    # -------------------------------------------------------------- search
    def _search_structs(self, P, nt, n_cmp, bounds, de, cmp_out, t_begin, t_end, rescore_fp64,
                        keep_pre_polish):
        import torch
        t_end = nt if t_end is None else int(t_end)
        n_out = n_cmp if cmp_out is None else len(cmp_out)
        n_t = t_end - t_begin
        dev = torch.device("cuda", torch.cuda.current_device())
        outs = dict(params=torch.empty((n_out, n_t, P), dtype=torch.float32, device=dev),
                    S=torch.empty((n_out, n_t), dtype=torch.float32, device=dev),
                    S64=torch.empty((n_out, n_t), dtype=torch.float64, device=dev)
                    if rescore_fp64 else None,
                    S_pre_polish=torch.empty((n_out, n_t), dtype=torch.float32, device=dev)
                    if keep_pre_polish else None)
        co = None if cmp_out is None else np.ascontiguousarray(cmp_out, dtype=np.int32)
        grid = _sized(T0Grid, cmp_out=None if co is None else co.ctypes.data, n_cmp_out=n_out,
                      t_begin=int(t_begin), t_end=t_end)
        lo, hi, mask = bounds
        b = _sized(Bounds, inv_t0_mask=int(mask))
        for d in range(3):
            b.lo[d] = float(lo[d]) if d < len(lo) else 0.0
            b.hi[d] = float(hi[d]) if d < len(hi) else 0.0
        cfg = de_cfg(de, rescore_fp64=rescore_fp64)
        res = _sized(Result, params=outs["params"].data_ptr(), S=outs["S"].data_ptr(),
                     S64=None if outs["S64"] is None else outs["S64"].data_ptr(),
                     S_pre_polish=None if outs["S_pre_polish"] is None
                     else outs["S_pre_polish"].data_ptr())
        return grid, b, cfg, res, outs, co

    def search(self, bounds, de, seed, cmp_out=None, t_begin=0, t_end=None, rescore_fp64=True,
               keep_pre_polish=False):
        """Search the bound data (ens_search_bound); returns a dict of device
        tensors and host counters."""
        grid, b, cfg, res, outs, keep = self._search_structs(
            self.nparam, self.nt, self.n_cmp, bounds, de, cmp_out, t_begin, t_end, rescore_fp64,
            keep_pre_polish)
        self._check(self._lib.ens_search_bound(self._h, C.byref(grid), C.byref(b), C.byref(cfg),
                                               C.c_uint64(int(seed)), C.byref(res)))
        return dict(outs, n_evals=int(res.n_evals), sum_m=int(res.sum_m))

    def search_traces(self, traces, geometry, sem, bounds, de, seed, cmp_out=None, t_begin=0,
                      t_end=None, rescore_fp64=True, keep_pre_polish=False, store=None, scale=None,
                      master=None, data_dtype=None):
        """The one-call search (ens_search): bind (traces, geometry, sem) and
        search.  geometry = (cmp_ptr, offset, dt, dx); sem = (op, window, ap_lo, ap_hi)."""
        cmp_ptr, offset, dt, dx = geometry
        op, window, ap_lo, ap_hi = sem
        tr, geo, sc, keep = self._data_structs(traces, cmp_ptr, offset, dt, dx, op, window, ap_lo,
                                               ap_hi, store, scale, master, data_dtype)
        grid, b, cfg, res, outs, keep2 = self._search_structs(
            OPS[op], traces.shape[1], np.asarray(cmp_ptr).size - 1, bounds, de, cmp_out, t_begin,
            t_end, rescore_fp64, keep_pre_polish)
        self._check(self._lib.ens_search(self._h, C.byref(tr), C.byref(geo), C.byref(sc),
                                         C.byref(grid), C.byref(b), C.byref(cfg),
                                         C.c_uint64(int(seed)), C.byref(res)))
        self._bound_as(traces, cmp_ptr, op)
        return dict(outs, n_evals=int(res.n_evals), sum_m=int(res.sum_m))

    def stack(self, params, S=None, cmp_out=None, t_begin=0, t_end=None, out=None, noalloc=False):
        """Zero-offset stack along each sample's operator (device [n_out, n_t]),
        and the RMS of the coherence panel S when S is given (else None).
        noalloc: through ens_stack_noalloc (no device allocation in the
        library; out, a caller tensor, receives the stack)."""
        import torch
        _require_cuda(params, S)
        t_end = self.nt if t_end is None else int(t_end)
        n_out = self.n_cmp if cmp_out is None else len(cmp_out)
        n_t = t_end - t_begin
        assert params.dtype == torch.float32 and params.is_contiguous()
        assert params.numel() == n_out * n_t * self.nparam
        if S is not None:
            assert S.dtype == torch.float32 and S.is_contiguous() and S.numel() == n_out * n_t
        co = None if cmp_out is None else np.ascontiguousarray(cmp_out, dtype=np.int32)
        grid = _sized(T0Grid, cmp_out=None if co is None else co.ctypes.data, n_cmp_out=n_out,
                      t_begin=int(t_begin), t_end=t_end)
        if out is None:
            out = torch.empty((n_out, n_t), dtype=torch.float32, device=params.device)
        assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() == n_out * n_t
        rms = C.c_double(0.0)
        fn = self._lib.ens_stack_noalloc if noalloc else self._lib.ens_stack
        self._check(fn(self._h, C.byref(grid), _ptr(params), _ptr(out), _ptr(S),
                       None if S is None else C.byref(rms)))
        return out, (None if S is None else rms.value)

    # -------------------------------------------------------------- objective
    def _cands(self, cmp, t, params):
        import torch
        _require_cuda(cmp, t, params)
        assert cmp.dtype == torch.int32 and t.dtype == torch.int32 and params.dtype == torch.float32
        assert cmp.is_contiguous() and t.is_contiguous() and params.is_contiguous()
        n = cmp.numel()
        assert t.numel() == n and params.numel() == n * self.nparam
        return _sized(Candidates, n=n, cmp=cmp.data_ptr(), t=t.data_ptr(),
                      params=params.data_ptr())

    def semblance_eval(self, cmp, t, params, with_M=False):
        import torch
        c = self._cands(cmp, t, params)
        S = torch.empty(cmp.numel(), dtype=torch.float32, device=cmp.device)
        M = torch.empty(cmp.numel(), dtype=torch.int32, device=cmp.device) if with_M else None
        self._check(self._lib.semblance_eval(self._h, C.byref(c), _ptr(S), _ptr(M)))
        return (S, M) if with_M else S

    def semblance_eval64(self, cmp, t, params):
        import torch
        c = self._cands(cmp, t, params)
        S = torch.empty(cmp.numel(), dtype=torch.float64, device=cmp.device)
        self._check(self._lib.semblance_eval64(self._h, C.byref(c), _ptr(S)))
        return S

    def semblance_backward(self, cmp, t, params, dS):
        import torch
        c = self._cands(cmp, t, params)
        dS = dS.contiguous().to(torch.float32)
        g = torch.empty_like(params)
        self._check(self._lib.semblance_backward(self._h, C.byref(c), _ptr(dS), _ptr(g)))
        return g

    # -------------------------------------------------------------- checks
    def philox(self, counters, key):
        import torch
        _require_cuda(counters, key)
        out = torch.empty_like(counters)
        self._check(self._lib.ens_philox(self._h, counters.shape[0], _ptr(counters), _ptr(key),
                                         _ptr(out)))
        return out

    def jade_draws(self, words, mu_cr, mu_f, np_):
        """JADE's draws for adaptation blocks words [n, 4] (uint64 as int64):
        device int32 tensors k_cr, k_f, a_idx."""
        import torch
        _require_cuda(words)
        n = words.shape[0]
        outs = [torch.empty(n, dtype=torch.int32, device=words.device) for _ in range(3)]
        self._check(self._lib.ens_jade_draws(self._h, n, _ptr(words), float(mu_cr), float(mu_f),
                                             int(np_), *[_ptr(o) for o in outs]))
        return tuple(outs)

    def de_trial(self, pop, S, words, F, CR, lo, hi):
        """pop [n_pop, np, P], S [n_pop, np], words [n_pop, np, 4], lo/hi [n_pop, P]."""
        import torch
        _require_cuda(pop, S, words, lo, hi)
        n_pop, np_, P = pop.shape
        out = torch.empty_like(pop)
        self._check(self._lib.ens_de_trial(self._h, n_pop, np_, P, _ptr(pop), _ptr(S), _ptr(words),
                                           float(F), float(CR), _ptr(lo), _ptr(hi), _ptr(out)))
        return out


def de_cfg(de, rescore_fp64=True):
    return _sized(DeCfg, np_lo=int(de["np_lo"]), np_hi=int(de["np_hi"]), ng_f=int(de["ng_f"]),
                  np_bf=int(de.get("np_bf", 5)), ng_bf=int(de.get("ng_bf", 1)),
                  n_cycle=int(de.get("n_cycle", 0)), n_skip=int(de.get("n_skip", 0)),
                  n_bucket=int(de.get("n_bucket", 1)), ens_enabled=int(de.get("ens_enabled", 0)),
                  inject=int(de.get("inject", 1)), F=float(de["F"]), CR=float(de["CR"]),
                  polish_steps=int(de.get("polish_steps", 0)),
                  polish_lr=float(de.get("polish_lr", 0.01)), rescore_fp64=int(bool(rescore_fp64)),
                  adapt=int(de.get("adapt", 0)))


def ens_search(traces, geometry, t0_grid, bounds, de_cfg_, seed, *, op, window, ap_lo=0,
               ap_hi=None, store=None, scale=None, master=None, data_dtype=None, ctx=None):
    """One-call search through the C entry point ens_search: bind (traces,
    geometry) and search the t0 grid.

    geometry = (cmp_ptr, offset, dt, dx); t0_grid = (cmp_out or None, t_begin, t_end).
    """
    ctx = ctx or Context()
    cmp_out, t_begin, t_end = t0_grid
    return ctx.search_traces(traces, geometry, (op, window, ap_lo, ap_hi), bounds, de_cfg_, seed,
                             cmp_out, t_begin, t_end, store=store, scale=scale, master=master,
                             data_dtype=data_dtype)


def _semblance_fn():
    import torch

    class SemblanceFn(torch.autograd.Function):
        """S = f(p) per candidate; backward through the hand-written adjoint."""

        @staticmethod
        def forward(fctx, ctx, cmp, t, params):
            fctx.ens = ctx
            fctx.save_for_backward(cmp, t, params)
            return ctx.semblance_eval(cmp, t, params.contiguous())

        @staticmethod
        def backward(fctx, grad_out):
            cmp, t, params = fctx.saved_tensors
            g = fctx.ens.semblance_backward(cmp, t, params.contiguous(), grad_out.contiguous())
            return None, None, None, g

    return SemblanceFn


def semblance(ctx, cmp, t, params):
    """Differentiable semblance of candidates (torch.autograd)."""
    return _semblance_fn().apply(ctx, cmp, t, params)
