"""bip_eels_signal_noalloc (the entry point for callers that cannot allocate)
against bip_eels_signal on the same plan: two calls in a row, the second with
a smaller input (fewer atoms, a smaller raster), every output mode, FP32 and
split precision; and a request beyond its fixed workspace is refused."""
from __future__ import annotations

import numpy as np
import pytest

from tests._tiny import tiny_cfg, tiny_problem
from tests.gpu_helpers import rel_l2, torch_dev

pytestmark = pytest.mark.gpu


def _run(plan, tp, scan, mode, prec, subset, noalloc):
    from paper_2607_00756_amd import bip
    torch, dev = torch_dev()
    P = scan[0] * scan[1]
    shape = {bip.OUT_MAP: (P,), bip.OUT_QEELS: (P, plan.nq), bip.OUT_BEAMS: (P, plan.ndet)}[mode]
    out = torch.full(shape, float("nan"), dtype=torch.float32, device=dev)
    plan.eels_signal(tp.n_ch, torch.from_numpy(tp.H).to(dev), tp.H_off, scan, mode, prec, out,
                     atom_subset=subset, noalloc=noalloc)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_signal_matches_the_allocating_entry_point():
    from paper_2607_00756_amd import bip
    torch, dev = torch_dev()
    cfg = tiny_cfg(ny=64, nx=64, nz=5, ly=16.0, lx=16.0, alpha=0.02, theta=0.03, s=2, scan=(6, 5))
    tp = tiny_problem(cfg, n_atoms=5, n_ch=2, W=8, seed=31, vscale=25.0, planes=[0, 4, 2, 2, 1],
                      win_sizes=[4, 12, 16, 24, 32])
    plan = bip.Plan.from_config(cfg, tp.tau, tp.win_size, tp.win_origin)
    plan.build_smatrix(torch.from_numpy(tp.V).to(dev))
    for mode in (bip.OUT_MAP, bip.OUT_QEELS, bip.OUT_BEAMS):
        for prec in (bip.PREC_FP32, bip.PREC_SPLIT_BF16):
            # first call: all atoms, 6 x 5 raster; second: two atoms, 3 x 4 raster
            for scan, subset in (((6, 5), None), ((3, 4), [3, 1])):
                want = _run(plan, tp, scan, mode, prec, subset, False)
                got = _run(plan, tp, scan, mode, prec, subset, True)
                err = rel_l2(got, want)
                print(f"[noalloc mode {mode} prec {prec} scan {scan}] rel-L2 {err:.2e}")
                assert np.all(np.isfinite(got)) and err < 1e-6
    plan.close()


def test_noalloc_refuses_requests_beyond_its_workspace():
    from paper_2607_00756_amd import bip
    torch, dev = torch_dev()
    cfg = tiny_cfg(ny=256, nx=256, nz=2, ly=32.0, lx=32.0, alpha=0.01, theta=0.06, s=4, scan=(64, 64))
    tp = tiny_problem(cfg, n_atoms=1, n_ch=2, W=64, seed=3, planes=[1])
    plan = bip.Plan.from_config(cfg, tp.tau, tp.win_size, tp.win_origin)
    plan.build_smatrix(torch.from_numpy(tp.V).to(dev))
    P = 64 * 64
    out = torch.empty((P, plan.ndet), dtype=torch.float32, device=dev)
    with pytest.raises(bip.BipError) as ei:
        plan.eels_signal(tp.n_ch, torch.from_numpy(tp.H).to(dev), tp.H_off, (64, 64), bip.OUT_BEAMS,
                         bip.PREC_FP32, out, noalloc=True)
    assert ei.value.code == bip.EUNSUPPORTED and "allocation-free" in str(ei.value)
    assert bip._lib.bip_noalloc_scratch_bytes() == 64 << 20
    plan.close()
