"""CPU-only checks of the C-ABI library: it loads, exports every symbol the
header declares, agrees with the binding's constants, and rejects bad
arguments before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np

from paper_2211_14212_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kct.h")


def _header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kct_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    assert lib is not None
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    names = set(re.findall(r"\bT (kct_\w+)", out))
    declared = _header_functions()
    assert len(declared) >= 14
    missing = [f for f in declared if f not in names]
    assert not missing, missing
    assert set(_lib.EXPORTED) <= set(declared)


def test_header_constants_match_binding():
    src = open(HEADER).read()
    vals = dict(re.findall(r"\b(KCT_[A-Z0-9_]+)\s*=\s*(\d+)", src))
    assert int(vals["KCT_F32"]) == _lib.KCT_F32 and int(vals["KCT_BF16"]) == _lib.KCT_BF16
    assert int(vals["KCT_F16"]) == _lib.KCT_F16
    assert int(vals["KCT_CGLS"]) == _lib.KCT_CGLS and int(vals["KCT_LSMR"]) == _lib.KCT_LSMR
    assert int(vals["KCT_HYBRID_LSQR"]) == _lib.KCT_HYBRID_LSQR
    assert int(vals["KCT_IRN_TV_CGLS"]) == _lib.KCT_IRN_TV_CGLS
    assert int(vals["KCT_LAMBDA_FIXED"]) == _lib.KCT_LAMBDA_FIXED and int(vals["KCT_LAMBDA_GCV"]) == _lib.KCT_LAMBDA_GCV
    assert int(vals["KCT_LAMBDA_DP"]) == _lib.KCT_LAMBDA_DP
    assert int(vals["KCT_AB_GMRES"]) == _lib.KCT_AB_GMRES and int(vals["KCT_BA_GMRES"]) == _lib.KCT_BA_GMRES
    assert int(vals["KCT_BP_MATCHED"]) == _lib.KCT_BP_MATCHED and int(vals["KCT_BP_INTERP"]) == _lib.KCT_BP_INTERP
    assert int(vals["KCT_SIRT"]) == _lib.KCT_SIRT and int(vals["KCT_OS_SART"]) == _lib.KCT_OS_SART
    assert int(vals["KCT_HYBRID_FLSQR_TV"]) == _lib.KCT_HYBRID_FLSQR_TV
    assert int(re.search(r"#define KCT_HIST_COLS (\d+)", src).group(1)) == _lib.KCT_HIST_COLS
    for name, code in _lib.STATUS_NAMES.items():
        assert int(vals[code]) == name
    # struct layouts: ctypes sizes equal the C sizes under the x86-64 ABI
    assert ctypes.sizeof(_lib.KctGeometry) == 4 * 3 + 4 + 8 * 6 + 4 * 2 + 8 * 2 + 8 * 2 + 8 + 8
    assert ctypes.sizeof(_lib.KctSolveParams) == 4 + 4 + 8 + 4 + 4 + 8 + 4 + 4 + 8 + 4 + 4 + 4 + 4
    assert int(re.search(r"#define KCT_FLAG_STOP_ON_RESIDUAL_INCREASE (\d+)u", src).group(1)) == \
        _lib.KCT_FLAG_STOP_ON_RESIDUAL_INCREASE
    assert int(re.search(r"#define KCT_FLAG_EXPLICIT_RESIDUAL (\d+)u", src).group(1)) == _lib.KCT_FLAG_EXPLICIT_RESIDUAL
    assert int(re.search(r"#define KCT_FLAG_X0_GIVEN (\d+)u", src).group(1)) == _lib.KCT_FLAG_X0_GIVEN


def test_status_strings_and_version():
    lib = _lib.load()
    assert lib.kct_version().startswith(b"kct")
    assert lib.kct_status_str(0) == b"ok"
    assert lib.kct_status_str(2) == b"unsupported geometry"


def _geom(**kw):
    ang = np.linspace(0, 2 * np.pi, 8, endpoint=False)
    d = dict(nx=8, ny=8, nz=8, vx=1.0, vy=1.0, vz=1.0, ox=0.0, oy=0.0, oz=0.0, nu=16, nv=16, du=1.0, dv=1.0,
             dso=100.0, dsd=150.0, n_angles=8)
    d.update(kw)
    a = np.asarray(d.pop("angles", ang), dtype=np.float64)
    g = _lib.KctGeometry(**{k: v for k, v in d.items()}, angles=a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return g, a


def test_invalid_geometry_rejected_without_device():
    lib = _lib.load()
    h = ctypes.c_void_p()
    cases = [dict(nx=0), dict(vx=-1.0), dict(du=0.0), dict(dso=0.0), dict(dsd=50.0), dict(n_angles=0),
             dict(vx=30.0),  # volume reaches the source orbit
             dict(dso=100.0, dsd=101.0)]  # volume crosses the detector
    for kw in cases:
        g, _keep = _geom(**kw)
        assert lib.kct_plan_create(ctypes.byref(g), 0, ctypes.byref(h)) == 2, kw
        assert lib.kct_last_error()
    g, _keep = _geom(angles=[0.0, float("nan")] + [0.0] * 6)
    assert lib.kct_plan_create(ctypes.byref(g), 0, ctypes.byref(h)) == 2
    assert lib.kct_plan_create(None, 0, ctypes.byref(h)) == 1
    g, _keep = _geom()
    assert lib.kct_plan_create(ctypes.byref(g), 0, None) == 1


def test_null_arguments_rejected():
    lib = _lib.load()
    n = ctypes.c_size_t()
    p = _lib.KctSolveParams(0, 10, 0.0, 0, 0, 1e-3, 0, 0, 0.0, 0, 0, 0, 0)
    assert lib.kct_solve_workspace_bytes(None, ctypes.byref(p), ctypes.byref(n)) == 1
    assert lib.kct_forward(None, None, 0, None, 0, None) == 1
    assert lib.kct_backproject(None, None, 0, None, 0, None) == 1
    assert lib.kct_backproject_interp(None, None, 0, None, 0, None) == 1
    assert lib.kct_state_step(None, 1) == 1
    assert lib.kct_plan_destroy(None) == 0
    assert lib.kct_state_destroy(None) == 0


def test_server_statistics_host_logic():
    """Nearest-rank percentiles and the summary used for p50/p99 (CPU only)."""
    from paper_2211_14212_amd import serve

    assert serve.percentile([5, 1, 4, 2, 3], 50) == 3
    assert serve.percentile(list(range(1, 101)), 99) == 99
    assert serve.percentile([7.0], 99) == 7.0
    rs = [serve.Result(i, float(i), float(i), float(i) + 1.0 + i, None, None) for i in range(4)]
    s = serve.summarize(rs)
    assert s["n"] == 4 and s["p50_s"] == 2.0 and s["p99_s"] == 4.0
    assert abs(s["makespan_s"] - 7.0) < 1e-12 and abs(s["throughput_req_per_s"] - 4 / 7.0) < 1e-12
