"""C-ABI checks that need no GPU: the built library loads, exports every entry point declared in
include/md.h, and rejects host-checkable bad arguments synchronously with the documented codes
before touching the device."""
import ctypes
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1408_4599_amd import md
    if not os.path.exists(md.LIB_PATH):
        from paper_1408_4599_amd import build
        build.build()
    return md.lib()


def _declared():
    text = open(os.path.join(ROOT, "include", "md.h")).read()
    return sorted(set(re.findall(r"^(?:int|int64_t|const char \*)\s*(md_[a-z_]+)\(", text, flags=re.M)))


def test_exports_every_declared_symbol(L):
    from paper_1408_4599_amd import md
    names = _declared()
    assert len(names) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", md.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (md_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(L, n)


def _desc(n_lj=1, eps=1.0, sig=1.0, mass=1.0):
    from paper_1408_4599_amd import md
    d = (md.ComponentDesc * 1)()
    keep = [(ctypes.c_double * 12)(*([0.0] * 12)), (ctypes.c_double * 4)(*([eps] * 4)), (ctypes.c_double * 4)(*([sig] * 4))]
    d[0].n_lj = n_lj
    d[0].lj_pos = ctypes.cast(keep[0], md._dp)
    d[0].lj_eps = ctypes.cast(keep[1], md._dp)
    d[0].lj_sigma = ctypes.cast(keep[2], md._dp)
    d[0].mass = mass
    return d, keep


@pytest.mark.parametrize("case,code", [
    ("null_out", -1), ("null_comps", -1), ("ncomp0", -1), ("ncomp_big", -3), ("rc_neg", -1), ("rc_nan", -4),
    ("eps_rf_neg", -1), ("too_many_lj", -3), ("eps_zero", -1), ("mass_zero", -1), ("bad_flag", -1)])
def test_model_create_rejects(L, case, code):
    d, keep = _desc(n_lj={"too_many_lj": 5}.get(case, 1), eps=0.0 if case == "eps_zero" else 1.0,
                    mass=0.0 if case == "mass_zero" else 1.0)
    h = ctypes.c_void_p()
    args = dict(comps=d, ncomp=1, rc=2.5, eps_rf=math.inf, flags=0, out=ctypes.byref(h))
    if case == "null_out":
        args["out"] = None
    if case == "null_comps":
        args["comps"] = None
    if case == "ncomp0":
        args["ncomp"] = 0
    if case == "ncomp_big":
        args["ncomp"] = 5
    if case == "rc_neg":
        args["rc"] = -1.0
    if case == "rc_nan":
        args["rc"] = math.nan
    if case == "eps_rf_neg":
        args["eps_rf"] = -2.0
    if case == "bad_flag":
        args["flags"] = 0x100
    rc = L.md_model_create(args["comps"], args["ncomp"], None, None, args["rc"], args["eps_rf"], args["flags"],
                           args["out"])
    assert rc == code
    assert len(L.md_last_error()) > 0
    assert not h.value


def test_calls_on_null_handles_are_rejected(L):
    box = (ctypes.c_double * 3)(10.0, 10.0, 10.0)
    assert L.md_build_cells(None, None, None, None, None, 10, box, None) == -1
    assert L.md_forces(None, None, 0, None, None, None, None, None, None, None, None) == -1
    assert L.md_step(None, None, None, None, None, None, None, 10, box, 0.001, 1, 0, None, None) == -1
    assert L.md_forces_adjoint(None, None, 0, 1.0, None, None, None, None) == -1
    assert L.md_cells_view(None, None) == -1
    assert L.md_profile(None, 1) == -1
    v = ctypes.c_int32()
    assert L.md_status(None, ctypes.byref(v)) == -1
    assert L.md_model_destroy(None) == 0
    assert L.md_cells_destroy(None) == 0
    assert L.md_param_count(None) == -1


def test_cells_handle_lifecycle_needs_no_device(L):
    h = ctypes.c_void_p()
    assert L.md_cells_create(ctypes.byref(h)) == 0
    from paper_1408_4599_amd import md
    info = md.CellsInfo()
    assert L.md_cells_view(h, ctypes.byref(info)) == -1  # not built yet
    assert b"not built" in L.md_last_error()
    assert L.md_cells_destroy(h) == 0


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1408_4599_amd import md
    monkeypatch.setattr(md, "_lib", None)
    monkeypatch.setattr(md, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        md.lib()


@pytest.mark.parametrize("case", ["lj", "ljts", "mixture_xi_eta", "2cljq"])
def test_long_range_correction_matches_oracle(L, oracle, case):
    """md_long_range_correction (host only) against the oracle's cut-off corrections."""
    from paper_1408_4599_amd import md, workloads as W
    box = [11.0, 12.0, 13.0]
    if case in ("lj", "ljts"):
        m, counts = W.lj_model(3.0, shift=case == "ljts"), [1500]
    elif case == "mixture_xi_eta":
        m = dict(W.mixture_model(rc=3.0), lj_shift=False, xi=[[1.0, 0.93], [0.93, 1.0]], eta=[[1.0, 1.07], [1.07, 1.0]])
        counts = [700, 900]
    else:
        m, counts = dict(W.twoclj_q_model(rc=3.0), lj_shift=False), [1200]
    u, w = md.long_range_correction(m, counts, box)
    uo, wo = oracle.long_range_correction(m, counts, box)
    assert u == pytest.approx(uo, rel=1e-14, abs=0.0)
    assert w == pytest.approx(wo, rel=1e-14, abs=0.0)
    if case == "ljts":
        assert (u, w) == (0.0, 0.0)


@pytest.mark.parametrize("case,code", [("null_out", -1), ("rc_neg", -1), ("box_nan", -4), ("count_neg", -1),
                                       ("ncomp_big", -3), ("eps_zero", -1)])
def test_long_range_correction_rejects(L, case, code):
    d, keep = _desc(eps=0.0 if case == "eps_zero" else 1.0)
    counts = (ctypes.c_int64 * 1)(-5 if case == "count_neg" else 100)
    box = (ctypes.c_double * 3)(float("nan") if case == "box_nan" else 10.0, 10.0, 10.0)
    u, w = ctypes.c_double(), ctypes.c_double()
    rc = L.md_long_range_correction(d, 5 if case == "ncomp_big" else 1, None, None, -1.0 if case == "rc_neg" else 2.5, 0,
                                    counts, box, None if case == "null_out" else ctypes.byref(u), ctypes.byref(w))
    assert rc == code
    assert L.md_last_error()


def test_set_thermostat_rejects(L):
    assert L.md_set_thermostat(None, 1.0) == -1
