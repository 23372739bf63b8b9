"""Degenerate and extreme inputs of the signal, against the FP64 oracle:
an empty atom subset (zero map), scan rasters of one position, one row or one
column up to the largest supported raster (256 x 256), a specimen in vacuum
at partition factor 1 (BiP reduces to exact PRISM), and a single channel.
Bar: rel-L2 <= 1e-4 (FP32 and split)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import eels as E
from tests._tiny import as_oracle_problem, tiny_cfg, tiny_problem
from tests.gpu_helpers import gpu_run, make_plan, rel_l2, torch_dev

pytestmark = pytest.mark.gpu

FP32, SPLIT = 0, 1
MAP, QEELS, BEAMS = 0, 1, 2


def test_empty_atom_subset_gives_a_zero_map():
    cfg = tiny_cfg(ny=64, nx=64, nz=3, ly=16.0, lx=16.0, alpha=0.02, theta=0.03, s=2, scan=(5, 4))
    tp = tiny_problem(cfg, n_atoms=2, n_ch=2, W=8, seed=2)
    for mode in (MAP, QEELS):
        got, plan = gpu_run(cfg, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off, tp.n_ch,
                            mode, SPLIT, atom_subset=[])
        assert got.size > 0 and np.all(got == 0.0)
        plan.close()


@pytest.mark.parametrize("scan", [(1, 1), (1, 7), (6, 1), (256, 256)])
def test_scan_rasters(scan):
    """One position, one row, one column, and the largest raster (the probe
    sum's DFTs of length 1 and 256)."""
    cfg = tiny_cfg(ny=64, nx=64, nz=3, ly=16.0, lx=16.0, alpha=0.02, theta=0.03, s=2, scan=scan)
    tp = tiny_problem(cfg, n_atoms=2, n_ch=2, W=12, seed=4, planes=[0, 2])
    prob = as_oracle_problem(tp)
    want = E.BiP(prob).run(mode=E.OUT_MAP)
    for prec in (FP32, SPLIT):
        got, plan = gpu_run(cfg, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off, tp.n_ch,
                            MAP, prec)
        err = rel_l2(got, want)
        print(f"[raster {scan} prec {prec}] rel-L2 {err:.2e}")
        assert err < 1e-4
        plan.close()


def test_vacuum_at_partition_one_is_exact_prism():
    """V = 0 and s = 1: no scattering, parents = beams; the map equals the
    oracle's exact dual-matrix map, beams and qEELS too."""
    cfg = tiny_cfg(ny=64, nx=64, nz=4, ly=16.0, lx=16.0, alpha=0.02, theta=0.03, s=1, scan=(6, 6))
    tp = tiny_problem(cfg, n_atoms=3, n_ch=1, W=8, seed=6, zero_v=True, planes=[0, 3, 1],
                      win_sizes=[8, 16, 4])
    prob = as_oracle_problem(tp)
    for mode, omode in ((MAP, E.OUT_MAP), (BEAMS, E.OUT_BEAMS), (QEELS, E.OUT_QEELS)):
        want = E.exact_dual(prob, mode=omode)
        got, plan = gpu_run(cfg, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off, tp.n_ch,
                            mode, FP32)
        err = rel_l2(got, want)
        print(f"[vacuum s=1 mode {mode}] rel-L2 {err:.2e}")
        assert err < 1e-4
        plan.close()


def test_one_atom_per_workspace_chunk():
    """A workspace budget too small for two atoms makes every atom a chunk of
    its own, each chunk reusing the operand buffers of the one before.  Map,
    beams and the direct map agree with the oracle and with the single-chunk
    run; a second build and signal on the same plan repeat the result
    exactly."""
    import os
    cfg = tiny_cfg(ny=64, nx=64, nz=5, ly=16.0, lx=16.0, alpha=0.02, theta=0.03, s=2, scan=(5, 7))
    tp = tiny_problem(cfg, n_atoms=5, n_ch=2, W=8, seed=11, vscale=25.0, planes=[0, 4, 2, 2, 1],
                      win_sizes=[4, 12, 16, 24, 8])
    prob = as_oracle_problem(tp)
    from paper_2607_00756_amd import bip
    for mode, omode in ((MAP, E.OUT_MAP), (BEAMS, E.OUT_BEAMS), (bip.OUT_MAP_DIRECT, E.OUT_MAP)):
        want = E.BiP(prob).run(mode=omode)
        for prec in (FP32, SPLIT):
            one, plan = gpu_run(cfg, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off,
                                tp.n_ch, mode, prec)
            os.environ["BIP_WORKSPACE_GB"] = "1e-9"
            try:
                many, _ = gpu_run(cfg, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off,
                                  tp.n_ch, mode, prec, plan=plan)
                again, _ = gpu_run(cfg, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off,
                                   tp.n_ch, mode, prec, plan=plan)
            finally:
                os.environ.pop("BIP_WORKSPACE_GB", None)
            e1, e2, d = rel_l2(many, want), rel_l2(one, want), rel_l2(many, one)
            print(f"[chunks mode {mode} prec {prec}] per-atom {e1:.2e} single {e2:.2e} apart {d:.2e}")
            assert e1 < 1e-4 and e2 < 1e-4 and d < 1e-5
            assert np.array_equal(many, again)
            plan.close()


def test_parent_beyond_nyquist_is_unsupported():
    """A detector that fills the grid puts parents past the signed index range
    (beam 31 of a 64-pixel axis has parents 28 and 32 at s = 4), which would
    alias: plan creation returns BIP_EUNSUPPORTED."""
    from paper_2607_00756_amd import bip
    torch_dev()
    with pytest.raises(bip.BipError) as ei:
        bip.Plan(64, 64, 2, 8.0, 8.0, 2.0, 200e3, 0.02, 0.45, 4, [[1.0, 1.0, 1.0]], [8], [[0, 0]])
    assert ei.value.code == bip.EUNSUPPORTED and "outside the grid" in str(ei.value)
