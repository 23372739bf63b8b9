"""Parity on 512^2, 1024^2 and non-square grids (the sizes of the full-map
and qEELS workloads), and at the full size of those workloads.

Small cases (a few parent columns, a few slices) compare the map and every
parent window with the FP64 oracle.  The full-size cases build the plan of
the workload's own geometry (grid, slices, apertures, partition factor,
ragged windows) for a sample of its ionized atoms and check
* sampled parent windows against the oracle's multislice of those parent
  columns alone (the oracle steps one column at a time),
* properties that hold at any size: the qEELS bins summed over q equal the
  map (two independent contraction paths: the per-beam detector product and
  the Gram form), and the Gram-form map equals the direct detector map.
Bars: maps 1e-4; parent windows 1e-5 on the few-slice cases and 3e-5 at
full size, where a window has been through 2 x 65..100 complex64 transform
passes: a pass of N = 512..1024 points rounds at about 6e-8 x log2 N ~ 6e-7
relative, and independent roundings over ~260 passes grow as their square
root, to ~1e-5 (the largest measured: 7.3e-6)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import eels as E
from oracle import multislice as ms
from oracle import physics as ph
from oracle import sibson as sb
from paper_2607_00756_amd import specimen
from tests._tiny import as_oracle_problem, tiny_cfg, tiny_problem
from tests.gpu_helpers import gpu_run, make_plan, rel_l2, torch_dev

pytestmark = pytest.mark.gpu

FP32, SPLIT = 0, 1
MAP, QEELS, BEAMS, MAP_DIRECT = 0, 1, 2, 3


def _bip():
    from paper_2607_00756_amd import bip
    return bip


@pytest.mark.parametrize("ny,nx", [(512, 512), (1024, 1024), (512, 1024), (1024, 256)])
def test_large_grid_windows_and_map(ny, nx):
    """Every parent window of every atom and the map against the oracle on a
    few-slice problem at the large grid sizes (one and two LDS exchanges per
    transform, square and non-square)."""
    torch, dev = torch_dev()
    px = 1.0 / 32  # A per pixel: a small cell keeps the beam counts (and the oracle) small
    cfg = tiny_cfg(ny=ny, nx=nx, nz=3, ly=ny * px, lx=nx * px, alpha=0.006, theta=0.012, s=3,
                   scan=(6, 5))
    tp = tiny_problem(cfg, n_atoms=3, n_ch=2, W=8, seed=5, vscale=25.0, planes=[0, 2, 1],
                      win_sizes=[8, 32, 64])
    prob = as_oracle_problem(tp)
    b = E.BiP(prob)
    print(f"[large grid {ny}x{nx}] B={len(prob.beams)} ndet={len(prob.det)} "
          f"parents {b.part1.n_parents}+{b.part2.n_parents}", flush=True)
    pw = b.parent_windows([0, 1, 2])
    plan = make_plan(cfg, tp.tau, tp.win_size, tp.win_origin)
    plan.build_smatrix(torch.from_numpy(tp.V).to(dev))
    for a in (0, 1, 2):
        y, x = prob.window(a)
        W = int(tp.win_size[a])
        for side, part, sign in ((1, b.part1, -1), (2, b.part2, +1)):
            out = torch.empty((part.n_parents, W, W), dtype=torch.complex64, device=dev)
            plan.parent_windows(a, side, out)
            torch.cuda.synchronize()
            want = pw[a][side - 1] * E.carrier(cfg, part.parents, y, x, sign)
            err = rel_l2(out.cpu().numpy(), want)
            print(f"  atom {a} side {side} windows rel-L2 {err:.2e}")
            assert err < 1e-5, (a, side)
    want = b.run(mode=E.OUT_MAP)
    for prec in (FP32, SPLIT):
        got, _ = gpu_run(cfg, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off, tp.n_ch,
                         MAP, prec, plan=plan)
        err = rel_l2(got, want)
        print(f"  map prec {prec} rel-L2 {err:.2e}")
        assert err < 1e-4
    plan.close()


def test_fp16_gram_with_many_detector_beams():
    """In split precision the Gram matrix runs on FP16 products once the
    detector holds at least 4096 beams; its map against the oracle."""
    cfg = tiny_cfg(ny=256, nx=256, nz=3, ly=32.0, lx=32.0, alpha=0.01, theta=0.06, s=4, scan=(7, 6))
    tp = tiny_problem(cfg, n_atoms=3, n_ch=2, W=8, seed=8, vscale=25.0, planes=[0, 2, 1],
                      win_sizes=[8, 24, 40])
    prob = as_oracle_problem(tp)
    want = E.BiP(prob).run(mode=E.OUT_MAP)
    got, plan = gpu_run(cfg, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off, tp.n_ch,
                        MAP, SPLIT)
    err = rel_l2(got, want)
    print(f"[fp16 Gram] ndet={plan.ndet} split map rel-L2 {err:.2e}")
    assert plan.ndet >= 4096
    assert err < 1e-4
    plan.close()


def _sampled_windows(sp, plan, atoms, picks=2, bar=3e-5):
    """Parent windows of sampled parents of `atoms` against the oracle's
    multislice of those parent columns alone."""
    torch, dev = torch_dev()
    cfg = sp.cfg
    prob = E.Problem.from_specimen(sp)
    parts = (sb.Partition(prob.beams, cfg.partition), sb.Partition(prob.det, cfg.partition))
    for a in atoms:
        plane = int(prob.planes[a])
        y, x = prob.window(a)
        W = int(sp.win_size[a])
        for side, part, sign in ((1, parts[0], -1), (2, parts[1], +1)):
            n = part.n_parents
            idx = np.unique(np.linspace(0, n - 1, picks).astype(int))  # first and last parent
            par = part.parents[idx]
            cols = (ms.s1_at_planes if side == 1 else ms.s2_at_planes)(cfg, par, prob.T, prob.P, [plane])[plane]
            want = cols[:, y[:, None], x[None, :]] * E.carrier(cfg, par, y, x, sign)
            out = torch.empty((n, W, W), dtype=torch.complex64, device=dev)
            plan.parent_windows(a, side, out)
            torch.cuda.synchronize()
            err = rel_l2(out.cpu().numpy()[idx], want)
            print(f"  atom {a} (plane {plane}, W {W}) side {side}: parents {list(idx)} of {n}, "
                  f"windows rel-L2 {err:.2e}", flush=True)
            assert err < bar, (a, side)


def test_qeels_workload_full_size_sampled():
    """The qEELS workload's geometry (1024^2, 75 slices, 200 keV, 25/60 mrad,
    s = 8, 64^2 windows, 96 x 96 scan, five channels) for four of its ionized
    atoms: sampled parent windows against the oracle, and the qEELS bins
    summed over q against the Gram-form map (split precision)."""
    bip = _bip()
    torch, dev = torch_dev()
    sp = specimen.make(3, n_ionized=4)
    cfg = sp.cfg
    plan = bip.Plan.from_config(cfg, sp.tau, sp.win_size, sp.win_origin)
    print(f"[qEELS workload] B={plan.B} ndet={plan.ndet} parents {plan.Bp1}+{plan.Bp2}", flush=True)
    plan.build_smatrix(torch.from_numpy(sp.V).to(dev))
    _sampled_windows(sp, plan, [0])
    P = cfg.scan[0] * cfg.scan[1]
    H = torch.from_numpy(sp.H).to(dev)
    q = torch.empty((P, plan.nq), dtype=torch.float32, device=dev)
    m = torch.empty(P, dtype=torch.float32, device=dev)
    plan.eels_signal(sp.n_ch, H, sp.H_off, cfg.scan, bip.OUT_QEELS, SPLIT, q, atom_subset=[0, 3])
    plan.eels_signal(sp.n_ch, H, sp.H_off, cfg.scan, bip.OUT_MAP, SPLIT, m, atom_subset=[0, 3])
    torch.cuda.synchronize()
    err = rel_l2(q.sum(dim=1).double().cpu().numpy(), m.double().cpu().numpy())
    print(f"  sum_q qEELS vs map rel-L2 {err:.2e}")
    assert err < 1e-4
    plan.close()


def test_fullmap_workload_full_size_sampled():
    """The full-map workload's geometry (512^2, 100 slices, 300 keV, 30/60 mrad,
    s = 6, ragged windows 24^2 .. 64^2, 128 x 128 scan) for six of its ionized
    atoms: sampled parent windows against the oracle, and the Gram-form map
    against the direct detector map (split precision)."""
    bip = _bip()
    torch, dev = torch_dev()
    sp = specimen.make(2, n_ionized=6)
    cfg = sp.cfg
    plan = bip.Plan.from_config(cfg, sp.tau, sp.win_size, sp.win_origin)
    print(f"[full-map workload] B={plan.B} ndet={plan.ndet} parents {plan.Bp1}+{plan.Bp2} "
          f"W {list(sp.win_size)}", flush=True)
    plan.build_smatrix(torch.from_numpy(sp.V).to(dev))
    small = [int(a) for a in np.argsort(sp.win_size, kind="stable")[:2]]
    _sampled_windows(sp, plan, [small[0], int(np.argmax(sp.win_size))])
    P = cfg.scan[0] * cfg.scan[1]
    H = torch.from_numpy(sp.H).to(dev)
    g = torch.empty(P, dtype=torch.float32, device=dev)
    d = torch.empty(P, dtype=torch.float32, device=dev)
    plan.eels_signal(sp.n_ch, H, sp.H_off, cfg.scan, bip.OUT_MAP, SPLIT, g, atom_subset=small)
    plan.eels_signal(sp.n_ch, H, sp.H_off, cfg.scan, bip.OUT_MAP_DIRECT, SPLIT, d, atom_subset=small)
    torch.cuda.synchronize()
    err = rel_l2(g.double().cpu().numpy(), d.double().cpu().numpy())
    print(f"  Gram map vs direct map rel-L2 {err:.2e}")
    assert err < 1e-4
    plan.close()
