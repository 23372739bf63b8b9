"""PRISM interpolation factor f > 1 with the crop mask on the GPU (section
"Exact PRISM-EELS", Alg. 2 beam subsampling; Alg. 4 subsampled detector and
crop mask) against the oracle's Alg. 5 with the same f: beam and parent
counts, then maps (Gram and direct), qEELS and per-beam outputs in FP32 and
split precision, lattice and hex parents, ragged windows, rasters that f
divides and one it does not, with and without focal back-propagation of
S1; outputs off every atom's crop mask are exactly zero.  Bars: counts exact, outputs
rel-L2 1e-4."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from oracle import eels as E
from tests._tiny import as_oracle_problem, tiny_cfg, tiny_problem
from tests.gpu_helpers import gpu_run, rel_l2, torch_dev

pytestmark = pytest.mark.gpu


def _case(f, parents, scan, focal=False):
    cfg = dataclasses.replace(tiny_cfg(ny=64, nx=64, nz=5, ly=16.0, lx=16.0, alpha=0.03, theta=0.035,
                                       s=2, scan=scan),
                              parents=parents, n_radial=3, n_angular=6, interp_f=f, focal=focal)
    tp = tiny_problem(cfg, n_atoms=4, n_ch=2, W=8, seed=83 + f, vscale=25.0, planes=[0, 4, 2, 1],
                      win_sizes=[8, 12, 16, 24])
    return cfg, tp


@pytest.mark.parametrize("f,parents,scan,focal", [(2, "lattice", (8, 8), False), (4, "lattice", (8, 12), False),
                                                  (2, "hex", (6, 10), False), (2, "lattice", (7, 9), False),
                                                  (2, "lattice", (8, 8), True), (4, "hex", (6, 10), True)])
def test_prism_f_outputs_against_oracle(f, parents, scan, focal):
    from paper_2607_00756_amd import bip
    cfg, tp = _case(f, parents, scan, focal)
    prob = as_oracle_problem(tp)
    b = E.BiP(prob)
    I_beams = b.run(mode=E.OUT_BEAMS)
    wants = {bip.OUT_MAP: I_beams.sum(axis=1), bip.OUT_MAP_DIRECT: I_beams.sum(axis=1),
             bip.OUT_QEELS: E.reduce_output(cfg, I_beams.T, b.det, E.OUT_QEELS), bip.OUT_BEAMS: I_beams}
    union = np.zeros(cfg.scan[0] * cfg.scan[1], bool)
    for a in range(len(tp.tau)):
        union |= E.crop_mask(cfg, tp.tau[a], f)
    assert not union.all()  # some scans lie off every mask
    for mode, want in wants.items():
        for prec in (bip.PREC_FP32, bip.PREC_SPLIT_BF16):
            got, plan = gpu_run(cfg, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off, tp.n_ch,
                                mode, prec)
            assert (plan.B, plan.ndet, plan.Bp1, plan.Bp2) == \
                (len(b.beams), len(b.det), b.part1.n_parents, b.part2.n_parents)
            err = rel_l2(got, want)
            print(f"[f {f} {parents} scan {scan} focal {focal} mode {mode} prec {prec}] B {plan.B} n_det {plan.ndet} "
                  f"Bp {plan.Bp1}+{plan.Bp2} rel-L2 {err:.2e}")
            assert err < 1e-4
            assert np.all(got.reshape(len(union), -1)[~union] == 0.0)
            plan.close()


def test_prism_f_one_is_the_plain_plan_and_guards():
    from paper_2607_00756_amd import bip
    torch_dev()
    cfg, tp = _case(1, "lattice", (5, 7))
    a, pa = gpu_run(cfg, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off, tp.n_ch, bip.OUT_MAP, 0)
    cfg0 = dataclasses.replace(cfg, interp_f=0)  # 0 reads as 1
    b, pb = gpu_run(cfg0, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off, tp.n_ch, bip.OUT_MAP, 0)
    assert np.array_equal(a, b)
    pa.close()
    pb.close()
    for kw, code in ((dict(interp_f=3), bip.EINVAL), (dict(interp_f=2, s2_exact=True), bip.EUNSUPPORTED),
                     (dict(interp_f=2, ckpt_stride=1), bip.EUNSUPPORTED)):
        with pytest.raises(bip.BipError) as ei:
            bip.Plan.from_config(cfg, tp.tau, tp.win_size, tp.win_origin, **kw)
        assert ei.value.code == code, kw
