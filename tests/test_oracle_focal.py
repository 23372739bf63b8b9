"""Pins of the oracle's focal back-propagation of S1 (section "Magnitude-
preserving reconstruction and focal back-propagation"): the window Fresnel
step against the continuous Fresnel integral of a Gaussian, the centroid
depth in closed form, the zero-distance limit, and the accuracy gain the
paper reports (the on-atom probe error falls, about 2x)."""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from oracle import eels as E
from oracle import multislice as ms
from oracle import physics as ph
from paper_2607_00756_amd import specimen
from tests._tiny import as_oracle_problem, tiny_cfg, tiny_problem


def test_window_fresnel_step_is_the_continuous_fresnel_integral():
    """A Gaussian exp(-|r|^2/(4 s0^2)) centred in a 128 x 128 window, stepped
    forward by z and back again: forward it equals (s0^2/sc^2) exp(-|r|^2/(4
    sc^2)), sc^2 = s0^2 + i lambda z/(4 pi) (paraxial Fresnel integral); the
    back step undoes it."""
    cfg = tiny_cfg(ny=256, nx=256, ly=32.0, lx=32.0)
    lam = ph.wavelength(cfg.energy_ev)
    M, s0, z = 128, 0.5, 40.0
    d = cfg.lx / cfg.nx
    t = (np.arange(M) - M // 2) * d
    r2 = t[:, None] ** 2 + t[None, :] ** 2
    f = np.exp(-r2 / (4 * s0 * s0)).astype(complex)
    g = E.window_fresnel(cfg, f, z, -1)
    sc2 = s0 * s0 + 1j * lam * z / (4 * math.pi)
    assert np.abs(g - (s0 * s0 / sc2) * np.exp(-r2 / (4 * sc2))).max() < 1e-10
    assert np.abs(E.window_fresnel(cfg, g, z, +1) - f).max() < 1e-12


def test_centroid_depth_closed_form():
    """Slice potentials constant over the window: c_j = 3, 1, 0, 2 on the four
    slices above plane 4 give z_c = sum (j + 1/2) dz c_j / sum c_j; plane 0
    and an empty path give the plane itself."""
    cfg = tiny_cfg(ny=32, nx=32, nz=6, ly=8.0, lx=8.0, dz=2.0)
    V = np.zeros((cfg.nz, cfg.ny, cfg.nx))
    for j, c in enumerate((3.0, 1.0, 0.0, 2.0, 7.0, 5.0)):
        V[j] = c
    H = np.ones(16, np.complex64)
    for plane, want in ((4, (0.5 * 3 + 1.5 * 1 + 3.5 * 2) * 2.0 / 6.0), (0, 0.0)):
        prob = E.Problem(cfg, V, [[1.0, 1.0, (plane + 0.5) * cfg.dz]], [4], [[3, 5]], H,
                         np.array([0, 16]), 1)
        assert abs(E.centroid_depth(prob, 0) - want) < 1e-12
    prob = E.Problem(cfg, np.zeros_like(V), [[1.0, 1.0, 9.0]], [4], [[3, 5]], H, np.array([0, 16]), 1)
    assert E.centroid_depth(prob, 0) == 4 * cfg.dz


def test_zero_distance_reduces_to_plain_bip():
    """Atoms at plane 0 (no path above): the focal steps are the identity and
    the enlarged window only adds pixels that are cropped away."""
    cfg = tiny_cfg(ny=64, nx=64, nz=3, ly=16.0, lx=16.0, alpha=0.03, theta=0.04, s=2, scan=(4, 4))
    tp = tiny_problem(cfg, n_atoms=2, n_ch=2, W=8, planes=[0, 0], win_sizes=[8, 12])
    prob = as_oracle_problem(tp)
    plain = E.BiP(prob).run(mode=E.OUT_BEAMS)
    prob.cfg = dataclasses.replace(cfg, focal=True)
    assert E.rel_l2(E.BiP(prob).run(mode=E.OUT_BEAMS), plain) < 1e-13


def test_focal_step_lowers_the_on_atom_probe_error():
    """On the small workload's specimen (one atom at plane 4 of 10) the probe
    reconstructed through the focal steps is closer to the exact probe on
    the window than the plain reconstruction (the paper reports 2-3x)."""
    sp = specimen.make(0)
    prob = E.Problem.from_specimen(sp)
    cfg = prob.cfg
    i = int(prob.planes[0])
    C = E.illumination(cfg, prob.beams)
    exact = prob.crop(ms.s1_at_planes(cfg, prob.beams, prob.T, prob.P, [i])[i], 0)
    K = exact.shape[1] * exact.shape[2]
    psi_ex = exact.reshape(-1, K).T @ C.T
    b = E.BiP(prob)
    psi0 = b.reconstructed(0, b.parent_windows([0])[0])[0].reshape(-1, K).T @ C.T
    prob.cfg = dataclasses.replace(cfg, focal=True)
    bf = E.BiP(prob)
    psif = bf.focal_probe(0, bf.parent_windows([0])[0], C)
    e0 = np.linalg.norm(psi0 - psi_ex) / np.linalg.norm(psi_ex)
    ef = np.linalg.norm(psif - psi_ex) / np.linalg.norm(psi_ex)
    assert ef < 0.6 * e0, (e0, ef)
