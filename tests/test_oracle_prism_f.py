"""Oracle pins of the PRISM interpolation factor f > 1 and the crop mask
(section "Exact PRISM-EELS", Alg. 2 beam subsampling and coefficient
rescaling; Alg. 4 PRISM-subsampled detector beams and crop mask).

* In vacuum with a detector that takes every beam of the grid and windows no
  larger than the alias-free period N/f, the BiP map at f (partition factor
  1, so reconstruction is exact) equals, on each atom's crop mask,
  sum_n sum_{r in window} |H_n(r) psi_f(r, rho)|^2, where psi_f is the sum
  of the f x f copies of the closed-form PRISM probe shifted by N/f
  (Poisson summation of the decimated beam set) and zero off the mask: a
  check of the subsampling, of the f^2 scale on both the probe coefficients
  and the detector sum (decimated Parseval), and of the mask.
* The crop mask holds (S_y/f)(S_x/f) scans when f divides the raster, the
  scans nearest the atom, and every scan at f = 1.
* Subsampling keeps exactly the beams on the f-lattice; lattice parents of
  the subsampled set sit on the (s f)-lattice.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import pytest

from oracle import eels as E
from oracle import physics
from tests._tiny import as_oracle_problem, tiny_cfg, tiny_problem


def _closed_form_probe(cfg, beams, plane, rho):
    """Vacuum PRISM probe at the entrance of slice `plane` for scan rho
    (pixels): c sum_b exp(-i pi lambda z |q_b|^2) exp(2 pi i h_b.(r - rho)/N),
    c = 1/sqrt(G B), z = plane dz [ny, nx]."""
    lam = physics.wavelength(cfg.energy_ev)
    G = cfg.ny * cfg.nx
    y = np.arange(cfg.ny)[:, None]
    x = np.arange(cfg.nx)[None, :]
    out = np.zeros((cfg.ny, cfg.nx), np.complex128)
    z = plane * cfg.dz
    for hy, hx in beams:
        q2 = (hy / cfg.ly) ** 2 + (hx / cfg.lx) ** 2
        out += np.exp(-1j * math.pi * lam * z * q2) * \
            np.exp(2j * math.pi * (hy * (y - rho[0]) / cfg.ny + hx * (x - rho[1]) / cfg.nx))
    return out / math.sqrt(G * len(beams))


@pytest.mark.parametrize("f", [2, 4])
def test_vacuum_full_detector_map_is_the_periodized_probe_on_the_mask(f):
    cfg = tiny_cfg(ny=32, nx=32, nz=3, ly=8.0, lx=8.0, alpha=0.04, theta=0.08, s=1, scan=(8, 8))
    cfg = dataclasses.replace(cfg, interp_f=f)
    W = min(8, 32 // f)
    tp = tiny_problem(cfg, n_atoms=3, n_ch=2, W=W, seed=5, zero_v=True, planes=[0, 2, 1])
    prob = as_oracle_problem(tp)
    assert len(prob.det) == cfg.ny * cfg.nx  # the detector takes every beam
    bip = E.BiP(prob)
    got = bip.run(mode=E.OUT_MAP)

    rho = E.scan_positions(cfg)
    want = np.zeros(len(rho))
    for a in range(len(tp.tau)):
        y, x = prob.window(a)
        H = prob.H_atom(a)
        mask = E.crop_mask(cfg, tp.tau[a], f)
        for p in np.nonzero(mask)[0]:
            psi1 = _closed_form_probe(cfg, prob.beams, int(prob.planes[a]), rho[p])
            psif = sum(np.roll(psi1, (-ky * cfg.ny // f, -kx * cfg.nx // f), axis=(0, 1))
                       for ky in range(f) for kx in range(f))
            w = psif[y[:, None], x[None, :]]
            want[p] += float(np.sum(np.abs(H * w[None]) ** 2))
    assert np.count_nonzero(want) > 0
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-13 * np.max(want))


@pytest.mark.parametrize("f,scan", [(2, (8, 8)), (4, (8, 12)), (1, (5, 7))])
def test_crop_mask_holds_the_nearest_scans(f, scan):
    cfg = tiny_cfg(ny=48, nx=48, ly=12.0, lx=12.0, scan=scan)
    r = np.random.default_rng(3)
    rho = E.scan_positions(cfg)
    for _ in range(20):
        tau = np.array([r.random() * cfg.lx, r.random() * cfg.ly, 0.0])
        m = E.crop_mask(cfg, tau, f)
        if f == 1:
            assert m.all()
            continue
        assert m.sum() == (scan[0] // f) * (scan[1] // f)
        # every kept scan is within half a period of the atom, every other one is not
        t = np.array([tau[1] * cfg.ny / cfg.ly, tau[0] * cfg.nx / cfg.lx])
        N = np.array([cfg.ny, cfg.nx], float)
        d = np.abs((t - rho + N / 2) % N - N / 2)
        assert np.all(d[m] <= N / (2 * f))
        assert np.all(np.any(d[~m] >= N / (2 * f) - 1e-12, axis=1))


def test_subsampled_beams_and_lattice_parents():
    cfg = dataclasses.replace(tiny_cfg(ny=64, nx=64, ly=16.0, lx=16.0, alpha=0.03, theta=0.05, s=2),
                              interp_f=2)
    tp = tiny_problem(cfg, n_atoms=1, W=8, seed=2)
    bip = E.BiP(as_oracle_problem(tp))
    full = physics.aperture_beams(cfg)
    want = {tuple(h) for h in full if h[0] % 2 == 0 and h[1] % 2 == 0}
    assert {tuple(h) for h in bip.beams} == want
    assert np.all(bip.part1.parents % 4 == 0) and np.all(bip.part2.parents % 4 == 0)
    # weights: convex local coordinates of every retained beam
    W1 = bip.part1.W.toarray()
    assert np.allclose(W1.sum(axis=1), 1.0) and np.all(W1 >= 0)
    # a beam on the parent lattice is its own parent with weight 1
    par = {tuple(p): i for i, p in enumerate(bip.part1.parents)}
    for b, h in enumerate(bip.beams):
        if tuple(h) in par:
            assert W1[b, par[tuple(h)]] == pytest.approx(1.0)
