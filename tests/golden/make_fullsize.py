"""Write the full-size oracle fixtures of the GPU parity tests.

    python tests/golden/make_fullsize.py c1|c2|c3|c4 [...]

Every stored value comes from the FP64 oracle (oracle/) on the seeded
synthetic specimens (paper_2607_00756_amd/specimen.py, inputs only); nothing
here runs or reads the HIP library.  The workloads are too large for the
oracle to run in a test, so each fixture holds a seeded sample of outputs the
oracle computes one by one:

  c1  medium map (256^2, 50 slices, 112 atoms x 9 channels): the map over all
      112 atoms at 64 seeded scan positions.
  c2  full map geometry (512^2, 100 slices, s = 6, ragged windows): 8 seeded
      ionized atoms, map on a seeded 32 x 32 block of the 128 x 128 raster.
  c3  qEELS / beams geometry (1024^2, 75 slices, s = 8, W = 64): 8 seeded
      ionized atoms at 96 seeded scan positions: map, qEELS bins, and the
      per-beam intensities of 2048 seeded detector beams.
  c4  gradient geometry (256^2, 30 slices, 16 atoms x 3): the oracle map at
      the specimen's positions, the target map at positions perturbed by
      U(-0.05, 0.05) A per coordinate (windows kept at the unperturbed
      origins), and the oracle gradient of L = sum (I - I_t)^2: dL/dV on
      32768 seeded voxels and along 4 seeded dense directions, dL/d(x, y) of
      every atom through the slice potentials, and of the ionized atoms
      through their transition potentials.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import adjoint as A  # noqa: E402
from oracle import eels as E  # noqa: E402
from oracle import potential as pot  # noqa: E402
from paper_2607_00756_amd import specimen  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sample_rng(cid, what):
    """Seeds of the samples (shared with the tests that read the fixtures)."""
    return np.random.default_rng([cid, 100 + what])


def c1_scans():
    return np.sort(sample_rng(1, 0).choice(64 * 64, size=64, replace=False))


def c2_atoms():
    return np.sort(sample_rng(2, 1).choice(2000, size=8, replace=False))


def c2_scans():
    u0, v0 = sample_rng(2, 0).integers(0, 128 - 32, size=2)
    u, v = np.meshgrid(np.arange(u0, u0 + 32), np.arange(v0, v0 + 32), indexing="ij")
    return (u * 128 + v).ravel()


def c3_atoms():
    return np.sort(sample_rng(3, 1).choice(200, size=8, replace=False))


def c3_scans():
    return np.sort(sample_rng(3, 0).choice(96 * 96, size=96, replace=False))


def c3_beams(ndet):
    return np.sort(sample_rng(3, 2).choice(ndet, size=2048, replace=False))


def c4_perturbed(sp):
    d = np.random.default_rng([4, 4]).uniform(-0.05, 0.05, size=sp.xyz.shape)
    xyz = sp.xyz + d
    cfg = sp.cfg
    xyz[:, 0] %= cfg.lx
    xyz[:, 1] %= cfg.ly
    xyz[:, 2] = np.clip(xyz[:, 2], 0.0, np.nextafter(cfg.nz * cfg.dz, 0.0))
    return xyz


def c4_voxels(shape):
    return np.sort(sample_rng(4, 0).choice(int(np.prod(shape)), size=32768, replace=False))


def c4_directions(shape, n=4):
    r = sample_rng(4, 1)
    return [r.normal(size=shape) for _ in range(n)]


def _log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def _progress(tag, n):
    t0 = time.time()
    done = []

    def f(a):
        done.append(a)
        _log(f"{tag}: atom {a} done ({len(done)}/{n}, {time.time() - t0:.0f} s)")
    return f


def make_c1():
    sp = specimen.make(1)
    prob = E.Problem.from_specimen(sp)
    scans = c1_scans()
    _log(f"c1: {len(sp.tau)} atoms, {len(scans)} scans")
    I = E.BiP(prob).run(mode=E.OUT_MAP, scans=scans, rows=8192,
                        progress=_progress("c1", len(sp.tau)))
    np.savez_compressed(os.path.join(HERE, "fullsize_c1_map.npz"), scans=scans, map=I)


def make_c2():
    sp = specimen.make(2)
    prob = E.Problem.from_specimen(sp)
    atoms, scans = c2_atoms(), c2_scans()
    _log(f"c2: atoms {list(atoms)} W {list(sp.win_size[atoms])}, {len(scans)} scans")
    I = E.BiP(prob).run(mode=E.OUT_MAP, atoms=atoms, scans=scans, rows=4096,
                        progress=_progress("c2", len(atoms)))
    np.savez_compressed(os.path.join(HERE, "fullsize_c2_map.npz"), atoms=atoms, scans=scans, map=I)


def make_c3():
    sp = specimen.make(3)
    prob = E.Problem.from_specimen(sp)
    atoms, scans = c3_atoms(), c3_scans()
    beams = c3_beams(len(prob.det))
    _log(f"c3: atoms {list(atoms)}, {len(scans)} scans")
    I = E.BiP(prob).run(mode=E.OUT_BEAMS, atoms=atoms, scans=scans, rows=8192,
                        progress=_progress("c3", len(atoms)))          # [P, n_det]
    q = E.reduce_output(prob.cfg, I.T, prob.det, E.OUT_QEELS)
    m = E.reduce_output(prob.cfg, I.T, prob.det, E.OUT_MAP)
    np.savez_compressed(os.path.join(HERE, "fullsize_c3.npz"), atoms=atoms, scans=scans,
                        beams=beams, map=m, qeels=q, beams_I=I[:, beams])


def make_c4():
    sp = specimen.make(4)
    cfg = sp.cfg
    prob = E.Problem.from_specimen(sp)
    amps = np.array(specimen.POT_AMPS)[None, :] * \
        np.where(sp.species == 1, cfg.species_b_scale, 1.0)[:, None]
    widths = np.array(specimen.POT_WIDTHS)
    xyz_t = c4_perturbed(sp)
    Vt = pot.projected_potential(cfg, xyz_t, amps, widths)
    forms = specimen._forms(cfg.channels)
    Ht, dH = [], {}
    for k, a in enumerate(sp.ionized):
        W, org = int(sp.win_size[k]), tuple(sp.win_origin[k])
        Ht.append(specimen.transition_potentials(cfg, xyz_t[a], W, org, forms).ravel())
        _, hx, hy = specimen.transition_potentials(cfg, sp.xyz[a], W, org, forms, with_grad=True)
        dH[k] = (hx, hy)
    tau_t = xyz_t[sp.ionized]
    prob_t = E.Problem(cfg, Vt, tau_t, sp.win_size, sp.win_origin, np.concatenate(Ht), sp.H_off,
                       sp.n_ch)
    _log("c4: target map")
    It = E.BiP(prob_t).run(mode=E.OUT_MAP)
    _log("c4: gradient")
    res = A.MapGradient(prob).run(It, dH_dtau=dH)
    dV = res["dV"]
    g_pot = pot.potential_grad(cfg, sp.xyz, amps, widths, dV)
    vox = c4_voxels(dV.shape)
    proj = np.array([float(np.sum(dV * d)) for d in c4_directions(dV.shape)])
    dtau_H = np.array([res["dtau"][k] for k in range(len(sp.ionized))])
    np.savez_compressed(os.path.join(HERE, "fullsize_c4_grad.npz"), I=res["I"], I_target=It,
                        L=res["L"], voxels=vox, dV=dV.ravel()[vox], dV_proj=proj,
                        dV_norm=float(np.linalg.norm(dV)), dxyz_V=g_pot, dxy_H=dtau_H)


if __name__ == "__main__":
    jobs = {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c4": make_c4}
    for name in sys.argv[1:] or ["c4", "c1", "c3", "c2"]:
        t = time.time()
        jobs[name]()
        _log(f"{name} written in {time.time() - t:.0f} s")
