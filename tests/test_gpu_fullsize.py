"""Parity at the full size of the benchmark workload (medium workload: 256^2 grid,
50 slices, 112 atoms x 9 channels, 64 x 64 scan), in the launch configuration
bench.py times: the plan holds every atom, the contraction runs for a sample
of atoms (those ionized in the deepest plane, which keeps the oracle's parent
sweeps short), and the oracle computes the map at a sample of scan
positions.  Bar: rel-L2 <= 1e-4 for FP32 and split; plain FP16 reported
(bounded at 1e-3)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import eels as E
from paper_2607_00756_amd import specimen
from tests.gpu_helpers import rel_l2, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    sp = specimen.make(1)
    prob = E.Problem.from_specimen(sp)
    deepest = int(prob.planes.max())
    atoms = [int(a) for a in np.nonzero(prob.planes == deepest)[0][:2]]
    scans = np.random.default_rng(5).choice(sp.cfg.scan[0] * sp.cfg.scan[1], 48, replace=False)
    scans.sort()
    print(f"[c1 full size] atoms {atoms} at plane {deepest}, {len(scans)} sampled scans", flush=True)
    want = E.BiP(prob).run(mode=E.OUT_MAP, atoms=atoms, scans=scans)
    return sp, atoms, scans, want


@pytest.mark.parametrize("prec", [0, 1, 3])
def test_c1_full_size_map_sampled(c1, prec):
    from paper_2607_00756_amd import bip
    torch, dev = torch_dev()
    sp, atoms, scans, want = c1
    plan = bip.Plan.from_config(sp.cfg, sp.tau, sp.win_size, sp.win_origin)
    plan.build_smatrix(torch.from_numpy(sp.V).to(dev))
    P = sp.cfg.scan[0] * sp.cfg.scan[1]
    out = torch.empty(P, dtype=torch.float32, device=dev)
    plan.eels_signal(sp.n_ch, torch.from_numpy(sp.H).to(dev), sp.H_off, sp.cfg.scan, bip.OUT_MAP,
                     prec, out, atom_subset=atoms)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)[scans]
    err = rel_l2(got, want)
    print(f"[c1 full size prec {prec}] map rel-L2 vs FP64 oracle on sampled scans {err:.3e}")
    assert err < (1e-3 if prec == 3 else 1e-4)
    plan.close()
