"""The C-ABI library loads, exports every declared entry point and rejects bad
arguments on the host before touching a device (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2304_11399_amd as ens

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ens.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M))


def test_every_declared_symbol_is_exported():
    lib = ens.load()
    names = _declared()
    assert {"ens_search", "semblance_eval", "semblance_backward", "ens_bind"} <= names
    for n in names:
        assert hasattr(lib, n), n
    # and the binding wraps each of them
    assert names == set(ens._SIGS)


def _ctx():
    lib = ens.load()
    h = C.c_void_p()
    assert lib.ens_ctx_create(C.byref(h), None) == 0
    return lib, h


def test_struct_sizes_match_header_layout():
    # int64 members force 8-byte alignment; the Python mirrors must agree
    assert C.sizeof(ens.Traces) == 72
    assert C.sizeof(ens.DeCfg) == 68
    assert C.sizeof(ens.Result) == 56
    assert C.sizeof(ens.Stats) == 176
    assert C.sizeof(ens.Tuning) == 32


def test_struct_sizes_match_the_c_compiler(tmp_path):
    # the header compiled by the host C compiler gives the same sizes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    names = ["ens_traces", "ens_de_cfg", "ens_result", "ens_stats", "ens_tuning",
             "ens_geometry", "ens_sem_cfg", "ens_t0_grid", "ens_bounds", "ens_candidates"]
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include "ens.h"\nint main(void){\n' +
                   "".join(f'printf("%zu\\n", sizeof({n}));\n' for n in names) + "return 0;}\n")
    exe = tmp_path / "sizes"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    mirrors = [ens.Traces, ens.DeCfg, ens.Result, ens.Stats, ens.Tuning, ens.Geometry, ens.SemCfg,
               ens.T0Grid, ens.Bounds, ens.Candidates]
    assert got == [C.sizeof(m) for m in mirrors]


def test_null_and_state_errors():
    lib, h = _ctx()
    try:
        assert lib.ens_bind(h, None, None, None) == -1
        assert b"null" in lib.ens_last_error(h)
        assert lib.ens_search_bound(h, None, None, None, 0, None) == -6
        assert lib.ens_search(h, None, None, None, None, None, None, 0, None) == -1
        c = ens._sized(ens.Candidates, n=0)
        assert lib.semblance_eval(h, C.byref(c), None, None) == -6
        assert lib.semblance_backward(h, C.byref(c), None, None) == -6
        assert lib.ens_ctx_create(None, None) == -1
    finally:
        lib.ens_ctx_destroy(h)


def _bind_args(**kw):
    cmp_ptr = np.array([0, 2, 4], np.int64)
    off = np.array([100, 200, 100, 200], np.float32)
    tr = ens._sized(ens.Traces, data=0x1000, n_traces=4, nt=64, ld=64, dt=0.004, store_dtype=0)
    geo = ens._sized(ens.Geometry, cmp_ptr=cmp_ptr.ctypes.data, n_cmp=2, dx=12.5,
                     offset=off.ctypes.data)
    sem = ens._sized(ens.SemCfg, op=3, window=7, ap_lo=1, ap_hi=1)
    for k, v in kw.items():
        for s in (tr, geo, sem):
            if hasattr(s, k) and k != "struct_size":
                setattr(s, k, v)
    return tr, geo, sem, (cmp_ptr, off)


@pytest.mark.parametrize("field,value,status", [
    ("window", 6, -2), ("window", 17, -2), ("op", 2, -1), ("store_dtype", 7, -1),
    ("nt", 1, -1), ("dt", 0.0, -2), ("dx", -1.0, -2), ("ap_lo", -1, -2), ("ld", 10, -1),
    ("data_dtype", 5, -1),
])
def test_bind_rejects_bad_arguments_before_any_device_call(field, value, status):
    lib, h = _ctx()
    try:
        tr, geo, sem, keep = _bind_args(**{field: value})
        assert lib.ens_bind(h, C.byref(tr), C.byref(geo), C.byref(sem)) == status
        assert len(lib.ens_last_error(h)) > 0
    finally:
        lib.ens_ctx_destroy(h)


def test_bind_rejects_bad_geometry_and_struct_size():
    lib, h = _ctx()
    try:
        tr, geo, sem, keep = _bind_args()
        bad = np.array([0, 3, 2], np.int64)
        geo.cmp_ptr = bad.ctypes.data
        assert lib.ens_bind(h, C.byref(tr), C.byref(geo), C.byref(sem)) == -1
        tr, geo, sem, keep = _bind_args()
        tr.struct_size = 8
        assert lib.ens_bind(h, C.byref(tr), C.byref(geo), C.byref(sem)) == -1
    finally:
        lib.ens_ctx_destroy(h)


def test_sixteen_bit_data_need_scales_and_a_compatible_store():
    lib, h = _ctx()
    try:
        tr, geo, sem, keep = _bind_args(data_dtype=1, store_dtype=1)
        assert lib.ens_bind(h, C.byref(tr), C.byref(geo), C.byref(sem)) == -1     # no scale
        assert b"scale" in lib.ens_last_error(h)
        tr, geo, sem, keep = _bind_args(data_dtype=1, store_dtype=2)
        tr.scale = 0x2000
        assert lib.ens_bind(h, C.byref(tr), C.byref(geo), C.byref(sem)) == -5     # f16 into bf16
    finally:
        lib.ens_ctx_destroy(h)


def test_tuning_and_building_block_validation():
    lib, h = _ctx()
    try:
        t = ens._sized(ens.Tuning, waves_per_sample_group=9)
        assert lib.ens_set_tuning(h, C.byref(t)) == -2
        t.waves_per_sample_group = 4
        assert lib.ens_set_tuning(h, C.byref(t)) == 0
        t.use_graph, t.collect_timing = 1, 1
        assert lib.ens_set_tuning(h, C.byref(t)) == -1
        t.use_graph, t.collect_timing, t.packing = 0, 0, 3
        assert lib.ens_set_tuning(h, C.byref(t)) == -2
        t.packing = 8
        assert lib.ens_set_tuning(h, C.byref(t)) == 0
        st = ens._sized(ens.Stats)
        assert lib.ens_last_stats(h, C.byref(st)) == 0 and st.launches[0] == 0
        assert lib.ens_de_trial(h, 1, 3, 3, 1, 1, 1, 0.5, 0.9, 1, 1, 1) == -2   # np < 4
        assert lib.ens_de_trial(h, 1, 8, 2, 1, 1, 1, 0.5, 0.9, 1, 1, 1) == -1   # P = 2
        assert lib.ens_de_trial(h, 1, 8, 3, 1, 1, 1, 0.5, 1.5, 1, 1, 1) == -2   # CR > 1
        assert lib.ens_philox(h, -1, None, None, None) == -1
        assert lib.ens_quantize(h, None, 1, 1, 1, 1, None, None) == -1
    finally:
        lib.ens_ctx_destroy(h)


def test_binary16_record_limit_is_checked_on_the_host():
    # ens.h ENS_MAX_NT_F16, the binding's MAX_NT_F16 and the record length at
    # which the binary16 traveltime grid would pass 2^-9 samples agree; a longer
    # record searched in binary16 is refused before any device call
    import re
    src = open(os.path.join(ROOT, "include", "ens.h")).read()
    limit = int(re.search(r"ENS_MAX_NT_F16\s*=\s*(\d+)", src).group(1))
    assert limit == ens.MAX_NT_F16 == (1 << 14) - 16
    from tests._tol import tau_err_f16
    assert tau_err_f16(4080) == 1e-3 and tau_err_f16(4081) == 2e-3 and tau_err_f16(limit) == 4e-3
    lib, h = _ctx()
    try:
        tr, geo, sem, keep = _bind_args(nt=limit + 1, ld=limit + 1, store_dtype=1)
        assert lib.ens_bind(h, C.byref(tr), C.byref(geo), C.byref(sem)) == -5
        assert b"binary16 windows take records of at most 16368" in lib.ens_last_error(h)
    finally:
        lib.ens_ctx_destroy(h)
