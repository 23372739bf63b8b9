"""The energy-filtered 4D cube of Alg. 3 (partitioned S1, exact exit side)
on the GPU: BIP_OUT_CUBE on a plan whose S2 covers every detector beam,
against the oracle's per-scan exit multislice (oracle.eels.partitioned_cube),
with lattice, hex-ring and focal S1.  Bar: rel-L2 1e-4 (FP32, split)."""
from __future__ import annotations

import dataclasses

import pytest

from oracle import eels as E
from tests._tiny import as_oracle_problem, tiny_cfg, tiny_problem
from tests.gpu_helpers import gpu_run, make_plan, rel_l2, torch_dev

pytestmark = pytest.mark.gpu
CUBE = 4


@pytest.mark.parametrize("kw", [dict(), dict(parents="hex", n_radial=3), dict(focal=True)])
def test_cube_against_per_scan_exit_multislice(kw):
    cfg = dataclasses.replace(tiny_cfg(ny=64, nx=64, nz=5, ly=16.0, lx=16.0, alpha=0.03, theta=0.04, s=2,
                                       scan=(4, 5)), s2_exact=True, **kw)
    tp = tiny_problem(cfg, n_atoms=3, n_ch=2, W=8, seed=91, vscale=25.0, planes=[4, 0, 2],
                      win_sizes=[8, 12, 16])
    want = E.partitioned_cube(as_oracle_problem(tp))
    for prec in (0, 1):
        got, plan = gpu_run(cfg, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off, tp.n_ch, CUBE, prec)
        assert plan.Bp2 == plan.ndet
        err = rel_l2(got, want)
        print(f"[cube {kw} prec {prec}] rel-L2 vs per-scan exit multislice {err:.2e}")
        assert err < 1e-4
        plan.close()


def test_cube_needs_the_exact_detector_matrix():
    from paper_2607_00756_amd import bip
    torch, dev = torch_dev()
    cfg = tiny_cfg(ny=64, nx=64, nz=3, ly=16.0, lx=16.0, alpha=0.03, theta=0.04, s=2, scan=(2, 2))
    tp = tiny_problem(cfg, n_atoms=1, W=8, planes=[1])
    plan = make_plan(cfg, tp.tau, tp.win_size, tp.win_origin)
    plan.build_smatrix(torch.from_numpy(tp.V).to(dev))
    out = torch.empty((4, plan.ndet), dtype=torch.float32, device=dev)
    with pytest.raises(bip.BipError) as ei:
        plan.eels_signal(tp.n_ch, torch.from_numpy(tp.H).to(dev), tp.H_off, cfg.scan, CUBE, 0, out)
    assert ei.value.code == bip.EINVAL
    plan.close()
