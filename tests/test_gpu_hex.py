"""The paper's own parent geometry on the GPU: hex-ring parents (DC plus
n_radial rings of n_angular (1 + i) samples, snapped to beams) and Sibson
weights against that finite set with the hull rule, computed in FP64 on the
GPU, against the oracle (oracle/sibson.py: hex_ring_parents, HexPartition);
then maps and per-beam outputs of BiP with those parents against the oracle's
Alg. 5.  Bars: parents exact, weights 1e-12, outputs rel-L2 1e-4."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

from oracle import eels as E
from oracle import physics as ph
from oracle import sibson as sb
from paper_2607_00756_amd import specimen
from tests._tiny import as_oracle_problem, tiny_cfg, tiny_problem
from tests.gpu_helpers import gpu_run, rel_l2, torch_dev

pytestmark = pytest.mark.gpu


def _csr_dense(plan, which, n_rows, n_cols):
    from paper_2607_00756_amd import bip
    rp, col, w = plan.query(bip.Q_WEIGHTS1 if which == 1 else bip.Q_WEIGHTS2)
    D = np.zeros((n_rows, n_cols))
    for r in range(n_rows):
        D[r, col[rp[r]:rp[r + 1]]] = w[rp[r]:rp[r + 1]]
    return D


@pytest.mark.parametrize("n_radial,n_angular", [(2, 6), (4, 6), (3, 5)])
def test_hex_parents_and_weights_against_oracle(n_radial, n_angular):
    from paper_2607_00756_amd import bip
    torch_dev()
    cfg = dataclasses.replace(tiny_cfg(ny=64, nx=64, nz=3, ly=16.0, lx=16.0, alpha=0.03, theta=0.05),
                              parents="hex", n_radial=n_radial, n_angular=n_angular)
    tp = tiny_problem(cfg, n_atoms=1, W=8, planes=[1])
    plan = bip.Plan.from_config(cfg, tp.tau, tp.win_size, tp.win_origin)
    prob = as_oracle_problem(tp)
    b = E.BiP(prob)
    for which, part in ((1, b.part1), (2, b.part2)):
        got = plan.query(bip.Q_PARENTS1 if which == 1 else bip.Q_PARENTS2)
        assert np.array_equal(got, part.parents)
        D = _csr_dense(plan, which, part.W.shape[0], part.n_parents)
        err = np.abs(D - part.W.toarray()).max()
        print(f"[hex ({n_radial}, {n_angular}) side {which}] {part.n_parents} parents, "
              f"{part.W.shape[0]} beams, max |w - w_oracle| {err:.1e}")
        assert err < 1e-12
    plan.close()


def test_hex_weights_full_size_sampled():
    """The medium workload's aperture and detector (8,093 and 32,417 beams) with
    hex rings (4, 6): parents exact, and the weights of 600 seeded beams of each
    set against the oracle's general construction."""
    from paper_2607_00756_amd import bip
    torch_dev()
    cfg = dataclasses.replace(specimen.WORKLOADS[1], parents="hex", n_radial=4, n_angular=6)
    plan = bip.Plan.from_config(cfg, [[20.0, 20.0, 50.0]], [24], [[116, 116]])
    lam = ph.wavelength(cfg.energy_ev)
    r = np.random.default_rng(9)
    for which, beams, ang in ((1, ph.aperture_beams(cfg), cfg.alpha), (2, ph.detector_beams(cfg), cfg.theta)):
        par = sb.hex_ring_parents(beams, 4, 6, ang / lam * cfg.ly, ang / lam * cfg.lx)
        got = plan.query(bip.Q_PARENTS1 if which == 1 else bip.Q_PARENTS2)
        assert np.array_equal(got, par)
        rp, col, w = plan.query(bip.Q_WEIGHTS1 if which == 1 else bip.Q_WEIGHTS2)
        hull = sb.convex_hull(par)
        worst = 0.0
        for bi in r.choice(len(beams), size=600, replace=False):
            want = sb.general_weights(beams[bi], par, hull)
            have = {tuple(par[c]): v for c, v in zip(col[rp[bi]:rp[bi + 1]], w[rp[bi]:rp[bi + 1]])}
            assert set(have) == set(want), (which, bi)
            worst = max(worst, max(abs(have[k] - want[k]) for k in want))
        print(f"[hex full size side {which}] {len(par)} parents; 600 sampled rows, max |dw| {worst:.1e}")
        assert worst < 1e-12
    plan.close()


@pytest.mark.parametrize("out_mode", [0, 1, 2])
def test_hex_bip_outputs_against_oracle(out_mode):
    """Map, qEELS and beams with hex-ring parents on ragged windows (FP32 and
    split) against the oracle's Alg. 5 with the same parents."""
    cfg = dataclasses.replace(tiny_cfg(ny=64, nx=64, nz=5, ly=16.0, lx=16.0, alpha=0.03, theta=0.04,
                                       scan=(5, 7)), parents="hex", n_radial=3, n_angular=6)
    tp = tiny_problem(cfg, n_atoms=4, n_ch=2, W=8, seed=71, vscale=25.0, planes=[0, 4, 2, 1],
                      win_sizes=[8, 12, 16, 24])
    prob = as_oracle_problem(tp)
    want = E.BiP(prob).run(mode={0: E.OUT_MAP, 1: E.OUT_QEELS, 2: E.OUT_BEAMS}[out_mode])
    for prec in (0, 1):
        got, plan = gpu_run(cfg, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off, tp.n_ch,
                            out_mode, prec)
        err = rel_l2(got, want)
        print(f"[hex BiP mode {out_mode} prec {prec}] Bp {plan.Bp1}+{plan.Bp2} rel-L2 {err:.2e}")
        assert err < 1e-4
        plan.close()
