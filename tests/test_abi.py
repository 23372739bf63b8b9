"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before launching anything (no GPU needed)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "bip.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bip_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2607_00756_amd import bip
    lib = ctypes.CDLL(bip.library_path())
    syms = declared_symbols()
    assert "bip_build_smatrix" in syms and "bip_eels_signal" in syms
    for s in syms:
        assert hasattr(lib, s), s
    assert set(bip.EXPORTS) <= set(syms)


@pytest.mark.parametrize("kw,msg", [
    (dict(ny=100), "powers of two"),
    (dict(ny=2048), "powers of two"),
    (dict(nz=0), "nz"),
    (dict(dz=0.0), "> 0"),
    (dict(alpha=-1.0), "> 0"),
    (dict(partition=0), "partition"),
    (dict(win=30), "multiple of 4"),
    (dict(win=256), "multiple of 4"),
    (dict(recon=7), "recon_mode"),
])
def test_plan_create_rejects_bad_arguments(kw, msg):
    from paper_2607_00756_amd import bip
    a = dict(ny=128, nx=128, nz=4, ly=16.0, lx=16.0, dz=2.0, energy=200e3, alpha=0.02, theta=0.04,
             partition=4, win=32, recon=0)
    a.update(kw)
    with pytest.raises(bip.BipError) as ei:
        bip.Plan(a["ny"], a["nx"], a["nz"], a["ly"], a["lx"], a["dz"], a["energy"], a["alpha"],
                 a["theta"], a["partition"], [[1.0, 1.0, 1.0]], [a["win"]], [[0, 0]],
                 recon_mode=a["recon"], stream=0)
    assert ei.value.code == bip.EINVAL
    assert msg in str(ei.value)


def test_null_plan_calls_fail_cleanly():
    from paper_2607_00756_amd import bip
    lib = bip._lib
    assert lib.bip_build_smatrix(None, None, None) == bip.EINVAL
    assert lib.bip_eels_signal(None, 1, None, None, None, 0, 1, 1, 0, 0, None, None) == bip.EINVAL
    assert lib.bip_reconstruct_local(None, 0, None, None, None) == bip.EINVAL
    assert lib.bip_query(None, 0, None) == bip.EINVAL
    assert b"NULL" in lib.bip_last_error()
    lib.bip_plan_destroy(None)


def test_allocator_needs_both_callbacks():
    """A bip_alloc with a missing callback is rejected before anything runs."""
    from paper_2607_00756_amd import bip
    half = bip.BipAlloc(bip._ALLOC_FN(lambda n, s, c: None), bip._RELEASE_FN(), None)
    grid = bip.BipGrid(128, 128, 4, 16.0, 16.0, 2.0)
    opt = bip.BipOptics(200e3, 0.02, 0.04, 4, 0, 0, 0.0, 0, 4, 6, 0, 0)
    tau = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    win = (ctypes.c_int32 * 1)(32)
    org = (ctypes.c_int32 * 2)(0, 0)
    h = ctypes.c_void_p()
    rc = bip._lib.bip_plan_create(ctypes.byref(grid), ctypes.byref(opt), 1, tau, win, org,
                                  ctypes.byref(half), None, ctypes.byref(h))
    assert rc == bip.EINVAL and b"alloc" in bip._lib.bip_last_error()
    assert not h.value
    rc = bip._lib.bip_potential_build(ctypes.byref(grid), 1, tau, 1, tau, tau, None, None, None)
    assert rc == bip.EINVAL

