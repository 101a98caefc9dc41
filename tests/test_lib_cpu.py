"""CPU checks of the C ABI library: it loads, exports every symbol that
include/pawfe.h declares, and rejects bad arguments on the host before any
device work (no compute call is made here)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2604_26037_amd import pawfe as pw
from workloads import make_system

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(pw.LIB_PATH):
        pytest.skip("libpawfe.so not built")
    return pw.load()


def test_exports_match_header():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "pawfe.h")).read()
    declared = sorted(set(re.findall(r"\b(pawfe_[a-zA-Z0-9_]+)\s*\(", hdr)))
    assert sorted(pw.EXPORTS) == declared
    for name in declared:
        assert hasattr(lib, name), name


def _desc(s, **over):
    keep = dict(veff=np.ascontiguousarray(s.veff_q).ravel(), pos=s.pos.ravel().copy(),
                rcut=s.rcut.copy(), nproj=s.nproj.astype(np.int32), l=s.proj_l.astype(np.int32),
                m=s.proj_m.astype(np.int32), sig=s.proj_sigma.copy(), dH=s.dH.copy(), dS=s.dS.copy())
    for k, v in over.items():
        if k in keep:
            keep[k] = v
    d = pw.Desc()
    d.ncell[:] = over.get("ncell", list(s.ncell))
    d.box[:] = list(s.box)
    d.degree = over.get("degree", s.degree)
    d.nq1d = over.get("nq", s.nq)
    d.kpoint[:] = over.get("kpoint", [0.0, 0.0, 0.0])
    d.is_complex = over.get("is_complex", 0)
    d.veff_q = pw._dptr(keep["veff"])
    d.natoms = len(keep["rcut"])
    d.pos = pw._dptr(keep["pos"])
    d.rcut = pw._dptr(keep["rcut"])
    d.nproj = pw._iptr(keep["nproj"])
    d.proj_l = pw._iptr(keep["l"])
    d.proj_m = pw._iptr(keep["m"])
    d.proj_sigma = pw._dptr(keep["sig"])
    d.dH = pw._dptr(keep["dH"])
    d.dS = pw._dptr(keep["dS"])
    d.sinv_mode = over.get("sinv_mode", 0)
    return d, keep


@pytest.mark.parametrize("over,code", [
    (dict(ncell=[1, 4, 4]), pw.PAWFE_EINVAL),
    (dict(ncell=[4, 1025, 4]), pw.PAWFE_EINVAL),
    (dict(degree=7, nq=9), pw.PAWFE_EUNSUPPORTED),
    (dict(degree=4, nq=5), pw.PAWFE_EUNSUPPORTED),
    (dict(is_complex=2), pw.PAWFE_EINVAL),
    (dict(is_complex=1, kpoint=[np.nan, 0.0, 0.0]), pw.PAWFE_ENONFINITE),
    (dict(kpoint=[0.1, 0.0, 0.0]), pw.PAWFE_EINVAL),
    (dict(sinv_mode=7), pw.PAWFE_EINVAL),
    (dict(rcut=np.array([6.0, 1.5])), pw.PAWFE_EINVAL),
    (dict(l=np.full(16, 3, dtype=np.int32)), pw.PAWFE_EINVAL),
    (dict(sig=np.full(16, -1.0)), pw.PAWFE_EINVAL),
    (dict(veff=np.full(64 * 216, np.nan)), pw.PAWFE_ENONFINITE),
    (dict(dH=np.full(128, np.inf)), pw.PAWFE_ENONFINITE),
])
def test_build_rejects_bad_descriptor(over, code):
    lib = _lib()
    s = make_system("tiny", veff=False)
    d, keep = _desc(s, **over)
    h = C.c_void_p()
    st = lib.pawfe_build_operator(C.byref(d), None, C.byref(h))
    assert st == code, lib.pawfe_last_error()
    assert not h.value
    assert len(lib.pawfe_last_error()) > 0


def test_null_operator_rejected():
    lib = _lib()
    x = C.c_void_p(1)
    assert lib.pawfe_apply_H(None, x, 4, x, 4, 4, 0, None) == pw.PAWFE_EINVAL
    assert lib.pawfe_apply_S(None, x, 4, x, 4, 4, 0, None) == pw.PAWFE_EINVAL
    assert lib.pawfe_apply_Sinv(None, x, 4, x, 4, 4, 0, None) == pw.PAWFE_EINVAL
    b = C.c_size_t()
    assert lib.pawfe_cheb_filter_workspace(None, 4, 4, 0, C.byref(b)) == pw.PAWFE_EINVAL
    assert lib.pawfe_rayleigh_ritz_workspace(None, 4, C.byref(b)) == pw.PAWFE_EINVAL
    assert lib.pawfe_cheb_filter(None, x, 4, x, 4, 4, 4, None, 10, 0.0, 1.0, 2.0, 0, x, 1, None) \
        == pw.PAWFE_EINVAL
    assert lib.pawfe_rayleigh_ritz(None, x, 4, 4, x, x, 0, x, 1, None) == pw.PAWFE_EINVAL
    assert lib.pawfe_band_energy_grad(None, x, 4, 4, None, None, None, None, None) == pw.PAWFE_EINVAL
    a = C.c_double()
    assert lib.pawfe_lanczos_bounds(None, 10, 1, C.byref(a), C.byref(a), C.byref(a), None) \
        == pw.PAWFE_EINVAL
    assert lib.pawfe_chfsi_solve(None, x, 4, 4, 0, 10, 4, 0, 0.0, 20, 1e-6, 10, x, x, None, x, 1, None) \
        == pw.PAWFE_EINVAL
    assert lib.pawfe_destroy_operator(None) == pw.PAWFE_OK


def test_batch_rejects_bad_jobs():
    lib = _lib()
    h = C.c_void_p()
    assert lib.pawfe_batch_create(None, 0, 0, 1, 0, None, C.byref(h)) == pw.PAWFE_EINVAL
    jobs = (pw.FilterJob * 1)()
    jobs[0] = pw.FilterJob(None, 1, 4, 1, 4, 4, 0, 1, 5, -1.0, 0.0, 1.0)
    assert lib.pawfe_batch_create(jobs, 1, 0, 1, 0, None, C.byref(h)) == pw.PAWFE_EINVAL
    assert b"op is NULL" in lib.pawfe_last_error()
    assert lib.pawfe_batch_create(jobs, 1, 2, 1, 0, None, C.byref(h)) == pw.PAWFE_EUNSUPPORTED
    assert h.value is None


def test_tune_cache_file_round_trip(tmp_path):
    """The autotuner's cache file: entries load, merge and save unchanged;
    a wrong first line or a malformed entry is refused and leaves the table
    as it was (host only, no GPU call)."""
    _lib()
    pw.tune_cache_clear()
    assert pw.tune_cache_size() == 0
    src = tmp_path / "a.cache"
    src.write_text("pawfe-tune-cache 1\n"
                   "job/gfx950/n6x6x6/p5/q7/a8/j144/c0/g0/v0/s20000/N128/m25/P1 64 12.5\n"
                   "batch/16384+job/gfx950/n6x6x6/p5/q7/a8/j144/c0/g0/v0/s20000/N128/m25/P1 2 0\n")
    pw.tune_cache_load(str(src))
    assert pw.tune_cache_size() == 2
    out = tmp_path / "b.cache"
    pw.tune_cache_save(str(out))
    lines = out.read_text().splitlines()
    assert lines[0] == "pawfe-tune-cache 1"
    assert sorted(l.split()[:2] for l in lines[1:]) == sorted(l.split()[:2] for l in src.read_text().splitlines()[1:])
    assert float([l for l in lines if l.startswith("job/")][0].split()[2]) == 12.5
    # a second file merges (same key replaced, new key added)
    more = tmp_path / "c.cache"
    more.write_text("pawfe-tune-cache 1\n"
                    "job/gfx950/n6x6x6/p5/q7/a8/j144/c0/g0/v0/s20000/N128/m25/P1 128 9\n"
                    "job/gfx950/n8x8x8/p5/q7/a8/j144/c0/g0/v0/s30000/N64/m25/P1 64 3\n")
    pw.tune_cache_load(str(more))
    assert pw.tune_cache_size() == 3
    for bad in ("not a cache\n", "pawfe-tune-cache 1\nkey-only\n", "pawfe-tune-cache 1\nk 0 1.0\n",
                "pawfe-tune-cache 1\nk 4 1.0 extra\n"):
        f = tmp_path / "bad.cache"
        f.write_text(bad)
        with pytest.raises(pw.PawfeError):
            pw.tune_cache_load(str(f))
        assert pw.tune_cache_size() == 3
    with pytest.raises(pw.PawfeError):
        pw.tune_cache_load(str(tmp_path / "missing.cache"))
    pw.tune_cache_clear()
    assert pw.tune_cache_size() == 0
