"""Full-size parity against stored FP64 oracle outputs (tests/golden/
fullsize_*.npz, written by tests/golden/make_fullsize.py from oracle/ only).

Each workload runs on the GPU in the launch configuration the benchmark
times (whole raster, all atoms of the plan); the comparison is on the seeded
sample of outputs the oracle computed one by one:
  * medium map (256^2, 50 slices, 112 atoms x 9): all atoms, 64 scans, in
    FP32 and split precision, the quadratic form in its job groups;
  * full-map geometry (512^2, 100 slices, s = 6, ragged 24..64 windows): a
    400-atom plan holding the 8 sampled atoms, atom_subset = those 8, a
    32 x 32 block of the 128 x 128 raster;
  * qEELS geometry (1024^2, 75 slices, s = 8, W = 64): the 200-atom plan,
    atom_subset = 8 sampled atoms: per-beam intensities of 2048 sampled beams,
    all qEELS bins and the map at 96 sampled scans;
  * gradient geometry (256^2, 30 slices, 16 atoms x 3): forward map at every
    scan, dL/dV on 32768 sampled voxels and along 4 dense directions, and
    dL/d(x, y) of every atom (slice potentials) and of the ionized atoms
    (transition potentials), for L = sum (I - I_t)^2 with the oracle's target.
Bars: rel-L2 1e-4 for maps, bins and beams (FP32 and split), 1e-3 for the
gradient."""
from __future__ import annotations

import os

import numpy as np
import pytest

from paper_2607_00756_amd import specimen
from tests.golden import make_fullsize as F
from tests.gpu_helpers import rel_l2, torch_dev

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fixture(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (python tests/golden/make_fullsize.py)")
    return np.load(path, allow_pickle=False)


def _bip():
    from paper_2607_00756_amd import bip
    return bip


def _map(plan, sp, H, prec):
    torch, dev = torch_dev()
    bip = _bip()
    out = torch.empty(sp.cfg.scan[0] * sp.cfg.scan[1], dtype=torch.float32, device=dev)
    plan.eels_signal(sp.n_ch, H, sp.H_off, sp.cfg.scan, bip.OUT_MAP, prec, out)
    torch.cuda.synchronize()
    return out


def test_medium_map_all_atoms_against_oracle():
    fx = _fixture("fullsize_c1_map.npz")
    torch, dev = torch_dev()
    bip = _bip()
    sp = specimen.make(1)
    assert np.array_equal(fx["scans"], F.c1_scans())
    plan = bip.Plan.from_config(sp.cfg, sp.tau, sp.win_size, sp.win_origin)
    plan.build_smatrix(torch.from_numpy(sp.V).to(dev))
    H = torch.from_numpy(sp.H).to(dev)
    for prec in (bip.PREC_FP32, bip.PREC_SPLIT_BF16):
        got = _map(plan, sp, H, prec).cpu().numpy()[fx["scans"]]
        err = rel_l2(got, fx["map"])
        print(f"[medium map, 112 atoms, prec {prec}] rel-L2 vs FP64 oracle on 64 scans {err:.2e}")
        assert err < 1e-4
    plan.close()


def test_full_map_geometry_sampled_atoms_against_oracle():
    fx = _fixture("fullsize_c2_map.npz")
    torch, dev = torch_dev()
    bip = _bip()
    sp = specimen.make(2)
    sample = F.c2_atoms()
    assert np.array_equal(fx["atoms"], sample)
    # a 400-atom plan: the 8 sampled atoms among the first others
    others = [a for a in range(len(sp.tau)) if a not in set(sample.tolist())][:392]
    members = np.sort(np.concatenate([sample, others]))
    idx = {a: i for i, a in enumerate(members)}
    offs = np.concatenate([[0], np.cumsum(sp.H_off[members + 1] - sp.H_off[members])]).astype(np.int64)
    Hg = np.concatenate([sp.H[sp.H_off[a]:sp.H_off[a + 1]] for a in members])
    plan = bip.Plan.from_config(sp.cfg, sp.tau[members], sp.win_size[members], sp.win_origin[members])
    plan.build_smatrix(torch.from_numpy(sp.V).to(dev))
    H = torch.from_numpy(Hg).to(dev)
    P = sp.cfg.scan[0] * sp.cfg.scan[1]
    subset = [idx[a] for a in sample]
    for prec in (bip.PREC_FP32, bip.PREC_SPLIT_BF16):
        out = torch.empty(P, dtype=torch.float32, device=dev)
        plan.eels_signal(sp.n_ch, H, offs, sp.cfg.scan, bip.OUT_MAP, prec, out, atom_subset=subset)
        torch.cuda.synchronize()
        got = out.cpu().numpy()[fx["scans"]]
        err = rel_l2(got, fx["map"])
        print(f"[full-map geometry, 8 atoms W {list(sp.win_size[sample])}, prec {prec}] "
              f"rel-L2 vs FP64 oracle on a 32x32 scan block {err:.2e}")
        assert err < 1e-4
    plan.close()


def test_qeels_geometry_sampled_atoms_against_oracle():
    fx = _fixture("fullsize_c3.npz")
    torch, dev = torch_dev()
    bip = _bip()
    sp = specimen.make(3)
    sample = F.c3_atoms()
    assert np.array_equal(fx["atoms"], sample)
    plan = bip.Plan.from_config(sp.cfg, sp.tau, sp.win_size, sp.win_origin)
    plan.build_smatrix(torch.from_numpy(sp.V).to(dev))
    H = torch.from_numpy(sp.H).to(dev)
    P = sp.cfg.scan[0] * sp.cfg.scan[1]
    scans, beams = fx["scans"], fx["beams"]
    sub = [int(a) for a in sample]
    out = torch.empty((P, plan.ndet), dtype=torch.float32, device=dev)
    plan.eels_signal(sp.n_ch, H, sp.H_off, sp.cfg.scan, bip.OUT_BEAMS, bip.PREC_SPLIT_BF16, out,
                     atom_subset=sub)
    torch.cuda.synchronize()
    got = out[torch.from_numpy(scans).to(dev)][:, torch.from_numpy(beams).to(dev)].cpu().numpy()
    del out
    err_b = rel_l2(got, fx["beams_I"])
    q = torch.empty((P, plan.nq), dtype=torch.float32, device=dev)
    plan.eels_signal(sp.n_ch, H, sp.H_off, sp.cfg.scan, bip.OUT_QEELS, bip.PREC_SPLIT_BF16, q,
                     atom_subset=sub)
    torch.cuda.synchronize()
    err_q = rel_l2(q.cpu().numpy()[scans], fx["qeels"])
    errs_m = {}
    for prec in (bip.PREC_FP32, bip.PREC_SPLIT_BF16):
        m = torch.empty(P, dtype=torch.float32, device=dev)
        plan.eels_signal(sp.n_ch, H, sp.H_off, sp.cfg.scan, bip.OUT_MAP, prec, m, atom_subset=sub)
        torch.cuda.synchronize()
        errs_m[prec] = rel_l2(m.cpu().numpy()[scans], fx["map"])
    print(f"[qEELS geometry, 8 atoms] beams {err_b:.2e} qEELS {err_q:.2e} map FP32 "
          f"{errs_m[bip.PREC_FP32]:.2e} split {errs_m[bip.PREC_SPLIT_BF16]:.2e}")
    assert err_b < 1e-4 and err_q < 1e-4 and max(errs_m.values()) < 1e-4
    plan.close()


def test_gradient_geometry_against_oracle_gradient():
    fx = _fixture("fullsize_c4_grad.npz")
    torch, dev = torch_dev()
    bip = _bip()
    sp = specimen.make(4)
    cfg = sp.cfg
    plan = bip.Plan.from_config(cfg, sp.tau, sp.win_size, sp.win_origin, ckpt_stride=1)
    V = torch.from_numpy(sp.V).to(dev)
    forms = specimen._forms(cfg.channels)
    dHx, dHy = [], []
    for k, a in enumerate(sp.ionized):
        _, hx, hy = specimen.transition_potentials(cfg, sp.xyz[a], int(sp.win_size[k]),
                                                   tuple(sp.win_origin[k]), forms, with_grad=True)
        dHx.append(hx.ravel())
        dHy.append(hy.ravel())
    cat = lambda v: torch.from_numpy(np.concatenate(v).astype(np.complex64)).to(dev)
    H = torch.from_numpy(sp.H).to(dev)
    P = cfg.scan[0] * cfg.scan[1]
    I = torch.empty(P, dtype=torch.float32, device=dev)
    plan.build_smatrix(V)
    plan.eels_signal(sp.n_ch, H, sp.H_off, cfg.scan, bip.OUT_MAP, bip.PREC_FP32, I)
    torch.cuda.synchronize()
    err_I = rel_l2(I.cpu().numpy(), fx["I"])
    It = torch.from_numpy(fx["I_target"]).to(dev)
    ibar = (2.0 * (I.double() - It)).float().contiguous()
    dV = torch.empty_like(V)
    tau = plan.eels_backward(sp.n_ch, H, sp.H_off, cfg.scan, ibar, dV, dHdx=cat(dHx), dHdy=cat(dHy),
                             want_tau=True)
    amps = np.array(specimen.POT_AMPS)[None, :] * \
        np.where(sp.species == 1, cfg.species_b_scale, 1.0)[:, None]
    grid = bip.BipGrid(cfg.ny, cfg.nx, cfg.nz, cfg.ly, cfg.lx, cfg.dz)
    g = bip.potential_grad(grid, sp.xyz, amps, np.array(specimen.POT_WIDTHS), dV)
    torch.cuda.synchronize()
    dVh = dV.cpu().numpy().astype(np.float64)
    err_v = rel_l2(dVh.ravel()[fx["voxels"]], fx["dV"])
    proj = np.array([np.sum(dVh * d) for d in F.c4_directions(dVh.shape)])
    err_p = rel_l2(proj, fx["dV_proj"])
    err_n = abs(np.linalg.norm(dVh) / float(fx["dV_norm"]) - 1.0)
    err_x = rel_l2(g.cpu().numpy()[:, :2], fx["dxyz_V"][:, :2])
    err_h = rel_l2(tau.cpu().numpy(), fx["dxy_H"])
    print(f"[gradient geometry] map {err_I:.2e}; dL/dV sampled {err_v:.2e}, projections {err_p:.2e}, "
          f"norm {err_n:.2e}; dL/dxy through V {err_x:.2e}, through H {err_h:.2e}")
    assert err_I < 1e-4
    assert err_v < 1e-3 and err_p < 1e-3 and err_n < 1e-3 and err_x < 1e-3 and err_h < 1e-3
    plan.close()
