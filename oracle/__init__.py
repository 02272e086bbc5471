"""FP64 CPU oracle (ctypes wrapper over ``liboracle.so``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
library (``paper_2304_11399_amd``) never imports, links or runs it, and this
package never touches the product.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = ["philox.c", "semblance.c", "search.c", "refine.c", "quant.c", "stack.c"]

_lib = None


class _Line(C.Structure):
    _fields_ = [("u", C.c_void_p), ("n_tr", C.c_int64), ("nt", C.c_int32), ("dt", C.c_double),
                ("cmp_ptr", C.c_void_p), ("n_cmp", C.c_int32), ("dx", C.c_double),
                ("offset", C.c_void_p), ("half_w", C.c_int32), ("op", C.c_int32),
                ("ap_lo", C.c_int32), ("ap_hi", C.c_int32)]


class _Bounds(C.Structure):
    _fields_ = [("lo", C.c_float * 3), ("hi", C.c_float * 3), ("inv_t0_mask", C.c_uint32)]


class _DeCfg(C.Structure):
    _fields_ = [("np_lo", C.c_int32), ("np_hi", C.c_int32), ("ng_f", C.c_int32),
                ("np_bf", C.c_int32), ("ng_bf", C.c_int32), ("n_cycle", C.c_int32),
                ("n_bucket", C.c_int32), ("ens_enabled", C.c_int32), ("inject", C.c_int32),
                ("F", C.c_float), ("CR", C.c_float), ("objective", C.c_int32),
                ("n_skip", C.c_int32), ("adapt", C.c_int32)]


def build(verbose=False):
    """Compile liboracle.so with gcc (plain C, OpenMP, no FMA contraction)."""
    import subprocess
    srcs = [os.path.join(_HERE, s) for s in SOURCES]
    cmd = ["gcc", "-std=gnu11", "-O3", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", LIB_PATH + ".tmp", *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.or_philox4x64_10.argtypes = [P, P, P]
        L.or_num_threads.restype = C.c_int32
        L.or_set_num_threads.argtypes = [C.c_int32]
        L.or_aperture.argtypes = [C.POINTER(_Line), C.c_int32]
        L.or_aperture.restype = C.c_int32
        L.or_pop_size.argtypes = [C.POINTER(_DeCfg), C.c_int32, C.c_int32]
        L.or_pop_size.restype = C.c_int32
        L.or_sample_bounds.argtypes = [C.POINTER(_Line), C.POINTER(_Bounds), C.c_int32, P, P]
        L.or_semblance_batch.argtypes = [C.POINTER(_Line), C.c_int64, P, P, P, P, P, P]
        L.or_semblance_grad_batch.argtypes = [C.POINTER(_Line), C.c_int64, P, P, P, P, P]
        L.or_semblance_tau_l1_batch.argtypes = [C.POINTER(_Line), C.c_int64, P, P, P, P]
        L.or_kink_margin_batch.argtypes = [C.POINTER(_Line), C.c_int64, P, P, P, P]
        L.or_de_trial.argtypes = [C.c_int32, C.c_int32, P, P, P, C.c_float, C.c_float, P, P, P]
        L.or_search.argtypes = [C.POINTER(_Line), C.POINTER(_Bounds), C.POINTER(_DeCfg),
                                C.c_uint64, P, C.c_int32, C.c_int32, C.c_int32, P, P]
        L.or_search.restype = C.c_int64
        L.or_polish.argtypes = [C.POINTER(_Line), C.POINTER(_Bounds), C.c_int64, P, P, P,
                                C.c_double, C.c_int32, P, P]
        L.or_quantize.argtypes = [P, C.c_int64, C.c_int32, C.c_int32, P, P]
        L.or_half_to_double.argtypes = [C.c_uint16]
        L.or_half_to_double.restype = C.c_double
        L.or_bf16_to_double.argtypes = [C.c_uint16]
        L.or_bf16_to_double.restype = C.c_double
        L.or_sref.argtypes = [C.POINTER(_Line), C.POINTER(_Bounds), C.c_int64, P, P, P,
                              C.c_int32, P, P]
        L.or_stack_batch.argtypes = [C.POINTER(_Line), C.c_int64, P, P, P, P, P]
        L.or_jade_draws.argtypes = [P, C.c_double, C.c_double, C.c_int32, P, P, P]
        L.or_jade_trial.argtypes = [C.c_int32, C.c_int32, P, P, P, C.c_int32, P, P, P, P, P, P]
        for name in ("or_jade_ln", "or_jade_cos_turns", "or_jade_tan_half_turn"):
            getattr(L, name).argtypes = [C.c_double]
            getattr(L, name).restype = C.c_double
        L.or_jade_series_batch.argtypes = [C.c_int32, C.c_int64, P, P]
        L.or_jade_run.argtypes = [C.c_int32, C.c_int32, P, P, C.c_int32, P, P, P, P, C.c_float,
                                  C.c_float, P, P, P, P, P, P]
        L.or_rms.argtypes = [P, C.c_int64]
        L.or_rms.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Line:
    """A line plus semblance configuration, held in binary64 for the oracle."""

    def __init__(self, traces, cmp_ptr, offset, dt, dx, window, op, ap_lo=0, ap_hi=None):
        self.u = np.ascontiguousarray(traces, dtype=np.float64)
        self.n_tr, self.nt = self.u.shape
        self.cmp_ptr = np.ascontiguousarray(cmp_ptr, dtype=np.int64)
        self.offset = np.ascontiguousarray(offset, dtype=np.float64)
        # the device path receives binary32 dt/dx: use exactly those values
        self.dt = float(np.float32(dt))
        self.dx = float(np.float32(dx))
        assert window % 2 == 1
        self.window = window
        self.op = int(op)
        self.ap_lo = int(ap_lo)
        self.ap_hi = int(ap_lo if ap_hi is None else ap_hi)
        self.n_cmp = self.cmp_ptr.size - 1
        self._s = _Line(self.u.ctypes.data, self.n_tr, self.nt, self.dt, self.cmp_ptr.ctypes.data,
                        self.n_cmp, self.dx, self.offset.ctypes.data, window // 2, self.op,
                        self.ap_lo, self.ap_hi)

    @classmethod
    def from_gather(cls, g, window, op, ap_lo=0, ap_hi=None, traces=None):
        return cls(g.traces if traces is None else traces, g.cmp_ptr, g.offset, g.dt, g.dx,
                   window, op, ap_lo, ap_hi)

    @property
    def nparam(self):
        return self.op

    def aperture(self, n0):
        return lib().or_aperture(C.byref(self._s), int(n0))

    def sample_bounds(self, bounds, n0):
        lo = np.zeros(3, np.float32)
        hi = np.zeros(3, np.float32)
        lib().or_sample_bounds(C.byref(self._s), C.byref(_bounds(bounds)), int(n0), _ptr(lo),
                               _ptr(hi))
        return lo[: self.op], hi[: self.op]

    def semblance(self, cmp, t, params):
        """S (float64), M (int32) and participation margin (samples) per candidate."""
        cmp = np.ascontiguousarray(cmp, dtype=np.int32)
        t = np.ascontiguousarray(t, dtype=np.int32)
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, self.op))
        n = cmp.size
        S = np.zeros(n)
        M = np.zeros(n, np.int32)
        mg = np.zeros(n)
        lib().or_semblance_batch(C.byref(self._s), n, _ptr(cmp), _ptr(t), _ptr(p), _ptr(S),
                                 _ptr(M), _ptr(mg))
        return S, M, mg

    def stack(self, cmp, t, params):
        """Zero-offset stack (float64) and participating traces M per sample."""
        cmp = np.ascontiguousarray(cmp, dtype=np.int32)
        t = np.ascontiguousarray(t, dtype=np.int32)
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, self.op))
        n = cmp.size
        out = np.zeros(n)
        M = np.zeros(n, np.int32)
        lib().or_stack_batch(C.byref(self._s), n, _ptr(cmp), _ptr(t), _ptr(p), _ptr(out), _ptr(M))
        return out, M

    def semblance_grad(self, cmp, t, params):
        cmp = np.ascontiguousarray(cmp, dtype=np.int32)
        t = np.ascontiguousarray(t, dtype=np.int32)
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, self.op))
        n = cmp.size
        S = np.zeros(n)
        g = np.zeros((n, self.op))
        lib().or_semblance_grad_batch(C.byref(self._s), n, _ptr(cmp), _ptr(t), _ptr(p), _ptr(S),
                                      _ptr(g))
        return S, g

    def tau_sensitivity(self, cmp, t, params):
        """Sum over participating traces of |dS/dtau_i| (tau in samples) per candidate."""
        cmp = np.ascontiguousarray(cmp, dtype=np.int32)
        t = np.ascontiguousarray(t, dtype=np.int32)
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, self.op))
        out = np.zeros(cmp.size)
        lib().or_semblance_tau_l1_batch(C.byref(self._s), cmp.size, _ptr(cmp), _ptr(t), _ptr(p),
                                        _ptr(out))
        return out

    def kink_margin(self, cmp, t, params):
        """min over participating traces of |tau_i - round(tau_i)| / (1 + |tau_i - n0|)."""
        cmp = np.ascontiguousarray(cmp, dtype=np.int32)
        t = np.ascontiguousarray(t, dtype=np.int32)
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1, self.op))
        out = np.zeros(cmp.size)
        lib().or_kink_margin_batch(C.byref(self._s), cmp.size, _ptr(cmp), _ptr(t), _ptr(p), _ptr(out))
        return out

    def search(self, bounds, de, seed, cmp_out=None, t_begin=0, t_end=None, objective=0,
               inject=1):
        cmp_out = np.arange(self.n_cmp, dtype=np.int32) if cmp_out is None else \
            np.ascontiguousarray(cmp_out, dtype=np.int32)
        t_end = self.nt if t_end is None else t_end
        n_t = t_end - t_begin
        params = np.zeros((cmp_out.size, n_t, self.op), np.float32)
        S = np.zeros((cmp_out.size, n_t))
        cfg = de_cfg(de, objective=objective, inject=inject)
        ev = lib().or_search(C.byref(self._s), C.byref(_bounds(bounds)), C.byref(cfg),
                             C.c_uint64(seed), _ptr(cmp_out), cmp_out.size, t_begin, t_end,
                             _ptr(params), _ptr(S))
        return params, S, int(ev)

    def polish(self, bounds, cmp, t, params, lr, steps):
        cmp = np.ascontiguousarray(cmp, dtype=np.int32)
        t = np.ascontiguousarray(t, dtype=np.int32)
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1, self.op))
        n = cmp.size
        out = np.zeros((n, self.op))
        S = np.zeros(n)
        lib().or_polish(C.byref(self._s), C.byref(_bounds(bounds)), n, _ptr(cmp), _ptr(t), _ptr(p),
                        float(lr), int(steps), _ptr(out), _ptr(S))
        return out, S

    def sref(self, bounds, cmp, t, grid, n_refine=8):
        cmp = np.ascontiguousarray(cmp, dtype=np.int32)
        t = np.ascontiguousarray(t, dtype=np.int32)
        g = np.ascontiguousarray(list(grid) + [1] * (3 - len(grid)), dtype=np.int32)
        n = cmp.size
        S = np.zeros(n)
        p = np.zeros((n, self.op))
        lib().or_sref(C.byref(self._s), C.byref(_bounds(bounds)), n, _ptr(cmp), _ptr(t), _ptr(g),
                      int(n_refine), _ptr(S), _ptr(p))
        return S, p


def _bounds(bounds):
    lo, hi, mask = bounds
    b = _Bounds()
    for d in range(3):
        b.lo[d] = float(lo[d]) if d < len(lo) else 0.0
        b.hi[d] = float(hi[d]) if d < len(hi) else 0.0
    b.inv_t0_mask = int(mask)
    return b


def de_cfg(de, objective=0, inject=1):
    return _DeCfg(int(de["np_lo"]), int(de["np_hi"]), int(de["ng_f"]), int(de["np_bf"]),
                  int(de["ng_bf"]), int(de["n_cycle"]), int(de["n_bucket"]),
                  int(de["ens_enabled"]), int(inject), float(de["F"]), float(de["CR"]),
                  int(objective), int(de.get("n_skip", 0)), int(de.get("adapt", 0)))


def pop_size(de, nt, n0):
    return lib().or_pop_size(C.byref(de_cfg(de)), int(nt), int(n0))


def philox4x64_10(counter, key):
    ctr = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib().or_philox4x64_10(_ptr(ctr), _ptr(k), _ptr(out))
    return out


def de_trial(pop, S, words, F, CR, lo, hi):
    pop = np.ascontiguousarray(pop, dtype=np.float32)
    npop, P = pop.shape
    S = np.ascontiguousarray(S, dtype=np.float64)
    words = np.ascontiguousarray(words, dtype=np.uint64).reshape(npop, 4)
    lo = np.ascontiguousarray(lo, dtype=np.float32)
    hi = np.ascontiguousarray(hi, dtype=np.float32)
    out = np.zeros_like(pop)
    lib().or_de_trial(npop, P, _ptr(pop), _ptr(S), _ptr(words), float(F), float(CR), _ptr(lo),
                      _ptr(hi), _ptr(out))
    return out


def rms(x):
    """Root mean square of a panel (binary64)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    return float(lib().or_rms(_ptr(x), x.size))


def jade_draws(words, mu_cr, mu_f, np_):
    """JADE's per-slot draws for blocks words [n][4]: (k_cr, k_f, a_idx) arrays."""
    words = np.ascontiguousarray(words, dtype=np.uint64).reshape(-1, 4)
    n = words.shape[0]
    k_cr = np.zeros(n, np.int32)
    k_f = np.zeros(n, np.int32)
    a_idx = np.zeros(n, np.int32)
    one_cr, one_f, one_a = C.c_int32(), C.c_int32(), C.c_int32()
    for i in range(n):
        lib().or_jade_draws(_ptr(words[i]), float(mu_cr), float(mu_f), int(np_), C.byref(one_cr),
                            C.byref(one_f), C.byref(one_a))
        k_cr[i], k_f[i], a_idx[i] = one_cr.value, one_f.value, one_a.value
    return k_cr, k_f, a_idx


def jade_series(name, x):
    """The oracle's written-out series ('ln', 'cos_turns' or 'tan_half_turn')
    at every point of x (binary64)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    y = np.zeros_like(x)
    which = {"ln": 0, "cos_turns": 1, "tan_half_turn": 2}[name]
    lib().or_jade_series_batch(which, x.size, _ptr(x), _ptr(y))
    return y


def jade_run(pop, S, de_words, St, F0, CR0, lo, hi, jade_words=None, draws=None):
    """ng JADE generations of one population with explicit generator words and
    trial scores (see or_jade_run).  Returns the final (pop, S) and per
    generation the trials, (mu_CR, mu_F), archive sizes and archives."""
    pop = np.ascontiguousarray(pop, dtype=np.float32).copy()
    np_, P = pop.shape
    S = np.ascontiguousarray(S, dtype=np.float64).copy()
    de_words = np.ascontiguousarray(de_words, dtype=np.uint64).reshape(-1, np_, 4)
    ng = de_words.shape[0]
    St = np.ascontiguousarray(St, dtype=np.float64).reshape(ng, np_)
    if jade_words is not None:
        jade_words = np.ascontiguousarray(jade_words, dtype=np.uint64).reshape(ng, np_, 4)
    else:
        draws = np.ascontiguousarray(draws, dtype=np.int32).reshape(ng, np_, 3)
    lo = np.ascontiguousarray(lo, dtype=np.float32)
    hi = np.ascontiguousarray(hi, dtype=np.float32)
    trials = np.zeros((ng, np_, P), np.float32)
    mu = np.zeros((ng, 2))
    n_arch = np.zeros(ng, np.int32)
    arch = np.zeros((ng, np_, P), np.float32)
    lib().or_jade_run(np_, P, _ptr(pop), _ptr(S), ng, _ptr(de_words),
                      None if jade_words is None else _ptr(jade_words),
                      None if draws is None else _ptr(draws), _ptr(St), float(F0), float(CR0),
                      _ptr(lo), _ptr(hi), _ptr(trials), _ptr(mu), _ptr(n_arch), _ptr(arch))
    return dict(pop=pop, S=S, trials=trials, mu=mu, n_arch=n_arch, archive=arch)


def jade_trial(pop, S, archive, words, k_f, k_cr, lo, hi):
    """One JADE generation's trials (binary32) for population pop [np][P]."""
    pop = np.ascontiguousarray(pop, dtype=np.float32)
    np_, P = pop.shape
    archive = np.ascontiguousarray(archive, dtype=np.float32).reshape(-1, P)
    S = np.ascontiguousarray(S, dtype=np.float64)
    words = np.ascontiguousarray(words, dtype=np.uint64).reshape(np_, 4)
    k_f = np.ascontiguousarray(k_f, dtype=np.int32)
    k_cr = np.ascontiguousarray(k_cr, dtype=np.int32)
    lo = np.ascontiguousarray(lo, dtype=np.float32)
    hi = np.ascontiguousarray(hi, dtype=np.float32)
    trial = np.zeros_like(pop)
    lib().or_jade_trial(np_, P, _ptr(pop), _ptr(S), _ptr(archive), archive.shape[0], _ptr(words),
                        _ptr(k_f), _ptr(k_cr), _ptr(lo), _ptr(hi), _ptr(trial))
    return trial


def quantize(u, dtype):
    """dtype 'f16' or 'bf16' -> (q uint16 [n_tr, nt], scale float32 [n_tr])."""
    u = np.ascontiguousarray(u, dtype=np.float32)
    n_tr, nt = u.shape
    q = np.zeros((n_tr, nt), np.uint16)
    s = np.zeros(n_tr, np.float32)
    lib().or_quantize(_ptr(u), n_tr, nt, 1 if dtype == "f16" else 2, _ptr(q), _ptr(s))
    return q, s


def dequantize(q, scale, dtype):
    """Exact binary64 value of scale_i * q_i[n]."""
    q = np.ascontiguousarray(q, dtype=np.uint16)
    if dtype == "f16":
        f = lib().or_half_to_double
    else:
        f = lib().or_bf16_to_double
    table = np.array([f(i) for i in range(65536)], dtype=np.float64)
    return table[q] * np.asarray(scale, dtype=np.float64)[:, None]
