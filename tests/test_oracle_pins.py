"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test names the passage of the paper (or the mathematical fact) it
checks.  Tolerances are FP64 round-off unless stated otherwise."""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

from oracle import eels as E
from oracle import multislice as ms
from oracle import physics as ph
from oracle import sibson as sb
from tests._tiny import as_oracle_problem, tiny_cfg, tiny_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------- P1 constants
def test_wavelength_and_sigma_match_published_tables():
    rows = json.load(open(os.path.join(GOLDEN, "electron_constants.json")))
    for r in rows["rows"]:
        lam = ph.wavelength(r["kv"] * 1e3)
        sig = ph.interaction_constant(r["kv"] * 1e3)
        assert abs(lam - r["lambda_A"]) / r["lambda_A"] < 3e-4
        assert abs(sig - r["sigma_rad_per_VA"]) / r["sigma_rad_per_VA"] < 3e-4
    lim = rows["nonrelativistic_limit"]["lambda_times_sqrt_volt_A"]
    assert abs(ph.wavelength(1.0) * 1.0 - lim) / lim < 1e-4


# ------------------------------------------------------------ P8 Sibson
def test_sibson_hand_derived_values():
    g = json.load(open(os.path.join(GOLDEN, "sibson_square_lattice.json")))
    for case in g["cases"]:
        w = sb.lattice_weights(case["x"], case["s"])
        want = {tuple(p): v for p, v in case["weights"]}
        assert set(w) == set(want), (case, w)
        for p, v in want.items():
            assert abs(w[p] - v) < 1e-13


def _raster_sibson(x, s, n=1200):
    """Brute force: classify sample points of [x-s, x+s]^2 by nearest site."""
    t = (np.arange(n) + 0.5) / n * 2 * s - s
    Y0, Y1 = np.meshgrid(x[0] + t, x[1] + t, indexing="ij")
    c0, c1 = math.floor(x[0] / s), math.floor(x[1] / s)
    sites = [((c0 + i) * s, (c1 + j) * s) for i in range(-2, 4) for j in range(-2, 4)]
    d_lat = np.stack([(Y0 - p[0]) ** 2 + (Y1 - p[1]) ** 2 for p in sites])
    nearest = np.argmin(d_lat, axis=0)
    dx = (Y0 - x[0]) ** 2 + (Y1 - x[1]) ** 2
    mine = dx < d_lat.min(axis=0)
    tot = mine.sum()
    return {sites[k]: float(((nearest == k) & mine).sum()) / tot for k in range(len(sites))
            if ((nearest == k) & mine).any()}


@pytest.mark.parametrize("s,x", [(4, (1, 0)), (4, (1, 1)), (4, (3, 2)), (6, (1, 3)), (8, (1, 4)),
                                 (8, (5, 2)), (6, (0, 5))])
def test_sibson_against_raster_brute_force(s, x):
    w = sb.lattice_weights(x, s)
    wr = _raster_sibson(x, s)
    for p in set(w) | set(wr):
        assert abs(w.get(p, 0.0) - wr.get(p, 0.0)) < 4e-3, (p, w, wr)


@pytest.mark.parametrize("s", [2, 3, 4, 6, 8])
def test_sibson_invariants(s):
    for r0 in range(s):
        for r1 in range(s):
            w = sb.lattice_weights((r0, r1), s)
            tot = sum(w.values())
            assert abs(tot - 1.0) < 1e-13
            assert all(v > 0 for v in w.values())
            # linear precision: sum_p w_p p = x  (Sibson 1981)
            c0 = sum(v * p[0] for p, v in w.items())
            c1 = sum(v * p[1] for p, v in w.items())
            assert abs(c0 - r0) < 1e-12 and abs(c1 - r1) < 1e-12


def test_partition_factor_one_is_identity():
    beams = ph.beams_within(64, 64, 8.0, 8.0, 0.02 / ph.wavelength(200e3))
    part = sb.Partition(beams, 1)
    assert np.array_equal(part.parents, beams)
    assert abs(part.W - np.eye(len(beams))).max() == 0


# ------------------------------------------------------- P2 vacuum sweeps
def test_vacuum_parent_sweeps_closed_form():
    cfg = tiny_cfg(ny=32, nx=32, nz=4, ly=8.0, lx=8.0, s=1)
    beams = np.array([[0, 0], [3, -2], [-5, 7], [16, -16], [-16, 15]])
    T = np.ones((cfg.nz, cfg.ny, cfg.nx), complex)
    P = ph.propagator(cfg)
    lam = ph.wavelength(cfg.energy_ev)
    S1 = ms.s1_at_planes(cfg, beams, T, P, [0, 2, 4])
    S2 = ms.s2_at_planes(cfg, beams, T, P, [0, 1, 3])
    G = cfg.ny * cfg.nx
    for k, h in enumerate(beams):
        q2 = (h[0] / cfg.ly) ** 2 + (h[1] / cfg.lx) ** 2
        ph1 = np.exp(-1j * math.pi * lam * cfg.dz * q2)
        for i in (0, 2, 4):
            want = ph1 ** i * ph.plane_wave(cfg, h, +1)
            assert np.abs(S1[i][k] - want).max() < 1e-12
        for i in (0, 1, 3):
            want = ph1 ** (cfg.nz - i) * ph.plane_wave(cfg, h, -1) / math.sqrt(G)
            assert np.abs(S2[i][k] - want).max() < 1e-12


def test_norm_conservation_random_potential():
    cfg = tiny_cfg(ny=32, nx=32, nz=5, ly=8.0, lx=8.0)
    tp = tiny_problem(cfg, vscale=300.0)
    T = ph.transmissions(cfg, tp.V)
    P = ph.propagator(cfg)
    beams = np.array([[0, 0], [2, 3], [-7, 1]])
    S1 = ms.s1_at_planes(cfg, beams, T, P, [5])[5]
    S2 = ms.s2_at_planes(cfg, beams, T, P, [0])[0]
    G = cfg.ny * cfg.nx
    assert np.allclose(np.sum(np.abs(S1) ** 2, axis=(1, 2)), G, rtol=1e-13)
    assert np.allclose(np.sum(np.abs(S2) ** 2, axis=(1, 2)), 1.0, rtol=1e-13)


# ---------------------------------------------------- P3 Fresnel probe
def test_prism_synthesis_equals_analytic_fresnel_probe():
    cfg = tiny_cfg(ny=32, nx=32, nz=3, ly=8.0, lx=8.0, alpha=60e-3, scan=(4, 2))
    beams = ph.aperture_beams(cfg)
    T = np.ones((cfg.nz, cfg.ny, cfg.nx), complex)
    P = ph.propagator(cfg)
    S1 = ms.s1_at_planes(cfg, beams, T, P, [3])[3]
    C = E.illumination(cfg, beams)
    lam = ph.wavelength(cfg.energy_ev)
    rho = E.scan_positions(cfg)
    y = np.arange(cfg.ny)[:, None]
    x = np.arange(cfg.nx)[None, :]
    G = cfg.ny * cfg.nx
    for p in range(len(rho)):
        psi = np.tensordot(C[p], S1, axes=(0, 0))
        want = np.zeros((cfg.ny, cfg.nx), complex)
        for h in beams:
            q2 = (h[0] / cfg.ly) ** 2 + (h[1] / cfg.lx) ** 2
            want += np.exp(-1j * math.pi * lam * cfg.dz * 3 * q2) * np.exp(
                2j * math.pi * (h[0] * (y - rho[p, 0]) / cfg.ny + h[1] * (x - rho[p, 1]) / cfg.nx))
        want /= math.sqrt(G * len(beams))
        assert np.abs(psi - want).max() < 1e-13
        assert abs(np.sum(np.abs(psi) ** 2) - 1.0) < 1e-12


# ------------------------------------------------------- P4 brute force
def _dense_operators(cfg, V):
    """Dense G x G multislice steps from an explicit DFT matrix."""
    ny, nx = cfg.ny, cfg.nx
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ky, kx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ry, rx, qy, qx = y.ravel(), x.ravel(), ky.ravel(), kx.ravel()
    F = np.exp(-2j * math.pi * (np.outer(qy, ry) / ny + np.outer(qx, rx) / nx))
    Finv = F.conj().T / (ny * nx)
    lam = ph.wavelength(cfg.energy_ev)
    sig = ph.interaction_constant(cfg.energy_ev)
    hy = np.where(qy < ny // 2, qy, qy - ny)
    hx = np.where(qx < nx // 2, qx, qx - nx)
    Pd = np.exp(-1j * math.pi * lam * cfg.dz * ((hy / cfg.ly) ** 2 + (hx / cfg.lx) ** 2))
    steps = [Finv @ np.diag(Pd) @ F @ np.diag(np.exp(1j * sig * V[j].astype(float).ravel()))
             for j in range(cfg.nz)]
    return F, steps, (ry, rx)


def test_brute_force_dense_alg1_and_alg4():
    cfg = tiny_cfg(ny=8, nx=8, nz=3, ly=4.0, lx=4.0, alpha=20e-3, theta=25e-3, scan=(2, 4))
    tp = tiny_problem(cfg, n_atoms=2, n_ch=2, W=4, planes=[0, 2], vscale=200.0)
    prob = as_oracle_problem(tp)
    F, steps, (ry, rx) = _dense_operators(cfg, tp.V)
    G = cfg.ny * cfg.nx
    beams, det = prob.beams, prob.det
    cb = 1.0 / math.sqrt(G * len(beams))
    rho = E.scan_positions(cfg)
    want = np.zeros((len(rho), len(det)))
    for p in range(len(rho)):
        psi = np.zeros(G, complex)
        for h in beams:
            psi += cb * np.exp(2j * math.pi * (h[0] * (ry - rho[p, 0]) / cfg.ny +
                                               h[1] * (rx - rho[p, 1]) / cfg.nx))
        for i in range(cfg.nz):
            for a in range(2):
                if prob.planes[a] != i:
                    continue
                y, x = prob.window(a)
                Hfull = np.zeros((cfg.ny, cfg.nx), complex)
                for n in range(tp.n_ch):
                    Hfull[:] = 0
                    Hfull[y[:, None], x[None, :]] = prob.H_atom(a)[n]
                    phi = Hfull.ravel() * psi
                    for j in range(i, cfg.nz):
                        phi = steps[j] @ phi
                    amp = (F @ phi) / math.sqrt(G)
                    idx = (det[:, 0] % cfg.ny) * cfg.nx + (det[:, 1] % cfg.nx)
                    want[p] += np.abs(amp[idx]) ** 2
            psi = steps[i] @ psi
    assert E.rel_l2(E.conventional(prob, mode=E.OUT_BEAMS), want) < 1e-12
    assert E.rel_l2(E.exact_dual(prob, mode=E.OUT_BEAMS), want) < 1e-12


# ------------------------------------------- P5, P7, P13 exactness chain
def test_alg1_equals_alg4_and_bip_s1_equals_alg4():
    cfg = tiny_cfg(ny=32, nx=32, nz=4, ly=8.0, lx=8.0, alpha=30e-3, theta=40e-3, s=1, scan=(4, 4))
    tp = tiny_problem(cfg, n_atoms=3, n_ch=2, W=8, vscale=100.0)
    prob = as_oracle_problem(tp)
    I1 = E.conventional(prob, mode=E.OUT_BEAMS)
    I4 = E.exact_dual(prob, mode=E.OUT_BEAMS)
    I4m = E.exact_dual(prob, mode=E.OUT_BEAMS, order="m")
    I5 = E.BiP(prob).run(mode=E.OUT_BEAMS)
    I5c = E.BiP(prob, E.RECON_COMPLEX).run(mode=E.OUT_BEAMS)
    assert E.rel_l2(I1, I4) < 1e-12
    assert E.rel_l2(I4m, I4) < 1e-12
    assert E.rel_l2(I5, I4) < 1e-12
    assert E.rel_l2(I5c, I4) < 1e-12


def test_bip_probe_order_equals_m_order_at_s4():
    cfg = tiny_cfg(ny=32, nx=32, nz=3, ly=8.0, lx=8.0, alpha=40e-3, theta=60e-3, s=4, scan=(4, 4))
    tp = tiny_problem(cfg, n_atoms=2, n_ch=2, W=8)
    prob = as_oracle_problem(tp)
    b = E.BiP(prob)
    assert E.rel_l2(b.run(order="m"), b.run()) < 1e-12


# --------------------------------------------------- P6 dot-product test
def test_s2_bilinear_identity():
    cfg = tiny_cfg(ny=16, nx=16, nz=4, ly=4.0, lx=4.0, theta=80e-3)
    tp = tiny_problem(cfg, vscale=200.0)
    T = ph.transmissions(cfg, tp.V)
    P = ph.propagator(cfg)
    det = ph.detector_beams(cfg)
    r = np.random.default_rng(7)
    for i in (0, 1, 3):
        S2 = ms.s2_at_planes(cfg, det, T, P, [i])[i]
        w = r.normal(size=(cfg.ny, cfg.nx)) + 1j * r.normal(size=(cfg.ny, cfg.nx))
        lhs = np.tensordot(S2, w, axes=([1, 2], [0, 1]))
        Fw = ms.fft2(ms.exit_operator(w, T, P, i)) / math.sqrt(cfg.ny * cfg.nx)
        rhs = Fw[det[:, 0] % cfg.ny, det[:, 1] % cfg.nx]
        assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


def test_s2_peeled_equals_rebuilt():
    cfg = tiny_cfg(ny=16, nx=16, nz=5, ly=4.0, lx=4.0)
    tp = tiny_problem(cfg, vscale=200.0)
    T = ph.transmissions(cfg, tp.V)
    P = ph.propagator(cfg)
    det = ph.detector_beams(cfg)
    a = ms.s2_at_planes(cfg, det, T, P, [1, 2, 4])
    b = ms.s2_peeled(cfg, det, T, P, [1, 2, 4])
    for i in (1, 2, 4):
        assert np.abs(a[i] - b[i]).max() < 1e-12


# ------------------------------------------------ P9 reconstruction pins
@pytest.mark.parametrize("s", [2, 4])
def test_recon_vacuum_closed_form(s):
    cfg = tiny_cfg(ny=64, nx=64, nz=6, ly=16.0, lx=16.0, alpha=30e-3, theta=50e-3, s=s)
    tp = tiny_problem(cfg, n_atoms=1, W=8, planes=[4], zero_v=True)
    prob = as_oracle_problem(tp)
    lam = ph.wavelength(cfg.energy_ev)
    for mode in (E.RECON_MAGNITUDE, E.RECON_COMPLEX):
        b = E.BiP(prob, mode)
        pw = b.parent_windows([0])[0]
        s1, s2 = b.reconstructed(0, pw)
        y, x = prob.window(0)
        for side, rec, part, beams, nsl in ((1, s1, b.part1, prob.beams, 4),
                                            (2, s2, b.part2, prob.det, cfg.nz - 4)):
            q2 = (part.parents[:, 0] / cfg.ly) ** 2 + (part.parents[:, 1] / cfg.lx) ** 2
            phase = np.exp(-1j * math.pi * lam * cfg.dz * q2) ** nsl
            z = part.W @ phase
            if mode == E.RECON_MAGNITUDE:
                z = z / np.abs(z)
            sgn = +1 if side == 1 else -1
            scale = 1.0 if side == 1 else 1.0 / math.sqrt(cfg.ny * cfg.nx)
            want = scale * z[:, None, None] * E.carrier(cfg, beams, y, x, sgn)
            assert np.abs(rec - want).max() < 1e-12 * scale


def test_recon_exact_at_parents_and_linear_precision():
    cfg = tiny_cfg(ny=64, nx=64, nz=3, ly=16.0, lx=16.0, alpha=40e-3, theta=40e-3, s=4)
    prob = as_oracle_problem(tiny_problem(cfg, n_atoms=1, W=6))
    part = sb.Partition(prob.beams, 4)
    y, x = prob.window(0)
    r = np.random.default_rng(3)
    alpha = r.normal(size=(6, 6)) + 1j * r.normal(size=(6, 6))
    beta = r.normal(size=(2, 6, 6)) + 1j * r.normal(size=(2, 6, 6))
    # synthetic de-tilted parent windows linear in h_p, carried by their own carrier
    Dp = alpha[None] + np.einsum("pk,kyx->pyx", part.parents.astype(float), beta)
    win = Dp * E.carrier(cfg, part.parents, y, x, +1)
    rec = E.reconstruct(cfg, win, part.parents, part.W, prob.beams, y, x, 1, E.RECON_COMPLEX)
    Db = alpha[None] + np.einsum("bk,kyx->byx", prob.beams.astype(float), beta)
    assert np.abs(rec - Db * E.carrier(cfg, prob.beams, y, x, +1)).max() < 1e-11
    # at parents that are beams, magnitude mode returns the parent column itself
    rec_m = E.reconstruct(cfg, win, part.parents, part.W, prob.beams, y, x, 1, E.RECON_MAGNITUDE)
    pset = {tuple(p): k for k, p in enumerate(part.parents)}
    for bi, h in enumerate(prob.beams):
        if tuple(h) in pset:
            assert np.abs(rec_m[bi] - win[pset[tuple(h)]]).max() < 1e-12


# --------------------------------------- P11 full detector, P12 qEELS sum
def test_full_detector_unitarity():
    cfg = tiny_cfg(ny=16, nx=16, nz=4, ly=4.0, lx=4.0, alpha=40e-3, theta=1.0, s=1, scan=(4, 4))
    tp = tiny_problem(cfg, n_atoms=2, n_ch=2, W=6, vscale=100.0)
    prob = as_oracle_problem(tp)
    assert len(prob.det) == cfg.ny * cfg.nx
    I = E.exact_dual(prob)
    C = E.illumination(cfg, prob.beams)
    want = np.zeros(C.shape[0])
    S1 = ms.s1_at_planes(cfg, prob.beams, prob.T, prob.P, sorted(set(prob.planes.tolist())))
    for a in range(2):
        s1 = prob.crop(S1[int(prob.planes[a])], a)
        psi = np.tensordot(C, s1, axes=(1, 0))      # [P, W, W]
        for n in range(tp.n_ch):
            want += np.sum(np.abs(prob.H_atom(a)[n][None] * psi) ** 2, axis=(1, 2))
    assert E.rel_l2(I, want) < 1e-12


def test_qeels_sums_to_map():
    cfg = tiny_cfg(ny=32, nx=32, nz=3, ly=8.0, lx=8.0, alpha=30e-3, theta=50e-3, s=2)
    prob = as_oracle_problem(tiny_problem(cfg, n_atoms=2, W=6))
    b = E.BiP(prob)
    q = b.run(mode=E.OUT_QEELS)
    m = b.run(mode=E.OUT_MAP)
    assert np.abs(q.sum(axis=1) - m).max() < 1e-14 * np.abs(m).max()
    beams = b.run(mode=E.OUT_BEAMS)
    assert np.abs(beams.sum(axis=1) - m).max() < 1e-14 * np.abs(m).max()


# -------------------------------------------------- P10 locality / on-atom
def test_on_atom_error_vanishes_at_s1_and_bip_converges_to_exact():
    cfg = tiny_cfg(ny=64, nx=64, nz=4, ly=16.0, lx=16.0, alpha=30e-3, theta=40e-3, s=1, scan=(4, 4))
    tp = tiny_problem(cfg, n_atoms=1, W=8, planes=[3], vscale=30.0)
    prob = as_oracle_problem(tp)
    assert E.on_atom_error(prob, E.BiP(prob), 0) < 1e-13
    exact = E.exact_dual(prob)
    errs = []
    for s in (1, 2, 4):
        import dataclasses
        prob.cfg = dataclasses.replace(cfg, partition=s)
        errs.append(E.rel_l2(E.BiP(prob).run(), exact))
    assert errs[0] < 1e-12 and errs[1] < errs[2]


# ------------------------------------ memory-light sweeps and beam chunks
def test_cropped_sweeps_and_row_chunks_match_full_columns():
    """s1_windows / s2_windows crop the same sweep as s1_at_planes /
    s2_at_planes, and BiP.run with detector rows in chunks returns the same
    intensities (each beam is computed alone)."""
    cfg = tiny_cfg(ny=32, nx=32, nz=5, ly=8.0, lx=8.0, alpha=30e-3, theta=50e-3, s=2, scan=(4, 4))
    tp = tiny_problem(cfg, n_atoms=3, n_ch=2, W=6, vscale=100.0, planes=[4, 0, 2])
    prob = as_oracle_problem(tp)
    b = E.BiP(prob)
    planes = [int(i) for i in prob.planes]
    full1 = ms.s1_at_planes(cfg, b.part1.parents, prob.T, prob.P, planes)
    full2 = ms.s2_at_planes(cfg, b.part2.parents, prob.T, prob.P, planes)
    pw = b.parent_windows([0, 1, 2])
    for a in range(3):
        assert np.array_equal(pw[a][0], prob.crop(full1[planes[a]], a))
        assert np.array_equal(pw[a][1], prob.crop(full2[planes[a]], a))
    ref = b.run(mode=E.OUT_BEAMS)
    got = b.run(mode=E.OUT_BEAMS, rows=37)
    assert np.abs(got - ref).max() <= 1e-15 * np.abs(ref).max()
    sc = [3, 7, 12]
    assert np.abs(b.run(scans=sc, rows=50) - ref.sum(axis=1)[sc]).max() <= 1e-14 * np.abs(ref).max()
