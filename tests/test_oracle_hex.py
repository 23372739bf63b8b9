"""Pins of the oracle's hex-ring parents and of its Sibson weights against a
general parent set (section "Partitioned PRISM-EELS": parent selection and
eq. nnw), with the hull rule for beams outside the parents' convex hull."""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import eels as E
from oracle import physics as ph
from oracle import sibson as sb
from tests._tiny import as_oracle_problem, tiny_cfg, tiny_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_general_weights_reproduce_hand_derived_rationals():
    """On a finite patch of the lattice s Z^2 the general construction must
    give the hand-derived area-stealing rationals (no lattice symmetry used)."""
    g = json.load(open(os.path.join(GOLDEN, "sibson_rationals.json")))
    for case in g["cases"]:
        s = case["s"]
        patch = np.array([(s * i, s * j) for i in range(-3, 5) for j in range(-3, 5)])
        w = sb.general_weights(case["x"], patch)
        want = {tuple(p): float(Fraction(v)) for p, v in case["weights"]}
        assert set(w) == set(want), (case, w)
        for p, v in want.items():
            assert abs(w[p] - v) < 1e-13


def _raster(x, parents, n=700, half=12.0):
    """Brute force: classify sample points around x by nearest site."""
    t = (np.arange(n) + 0.5) / n * 2 * half - half
    Y0, Y1 = np.meshgrid(x[0] + t, x[1] + t, indexing="ij")
    d = np.stack([(Y0 - p[0]) ** 2 + (Y1 - p[1]) ** 2 for p in parents])
    nearest = np.argmin(d, axis=0)
    mine = (Y0 - x[0]) ** 2 + (Y1 - x[1]) ** 2 < d.min(axis=0)
    tot = mine.sum()
    assert not mine[0, :].any() and not mine[-1, :].any() and not mine[:, 0].any() and not mine[:, -1].any()
    return {tuple(parents[k]): float(((nearest == k) & mine).sum()) / tot
            for k in range(len(parents)) if ((nearest == k) & mine).any()}


def _hex_set():
    cfg = tiny_cfg(ny=64, nx=64, ly=16.0, lx=16.0, alpha=0.04)
    beams = ph.aperture_beams(cfg)
    R = cfg.alpha / ph.wavelength(cfg.energy_ev) * cfg.lx
    return beams, R, sb.hex_ring_parents(beams, 4, 6, R, R)


def test_hex_ring_parents_geometry():
    """DC plus rings i = 0..3 of 6 (1 + i) samples at radius (i + 1) R / 4: 61
    distinct parents when the rings are more than a pixel apart, each sample
    snapped to a nearest beam of the set (within half a pixel diagonal when
    that lattice point lies in the disc), all inside the beam set."""
    beams, R, par = _hex_set()
    assert R / 4 > 2 and len(par) == 1 + 6 * (1 + 2 + 3 + 4) == 61
    bset = {tuple(b) for b in beams.tolist()}
    assert all(tuple(p) in bset for p in par.tolist()) and (0, 0) in {tuple(p) for p in par.tolist()}
    for i in range(4):
        m = 6 * (1 + i)
        for k in range(m):
            t = 2 * math.pi * k / m
            s = ((i + 1) / 4 * R * math.sin(t), (i + 1) / 4 * R * math.cos(t))
            d = np.hypot(par[:, 0] - s[0], par[:, 1] - s[1]).min()
            assert abs(d - np.hypot(beams[:, 0] - s[0], beams[:, 1] - s[1]).min()) < 1e-12
            if i < 3:
                assert d <= math.sqrt(0.5) + 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_general_weights_against_raster_brute_force(seed):
    beams, R, par = _hex_set()
    hull = sb.convex_hull(par)
    r = np.random.default_rng(seed)
    done = 0
    while done < 3:
        x = tuple(int(v) for v in beams[r.integers(len(beams))])
        inside, _ = sb._hull_projection(np.array(x, float), hull)
        if not inside or x in {tuple(p) for p in par.tolist()} or math.hypot(*x) > 0.6 * R:
            continue  # interior queries: their cells stay inside the raster
        w = sb.general_weights(x, par, hull)
        wr = _raster(x, par)
        for p in set(w) | set(wr):
            assert abs(w.get(p, 0.0) - wr.get(p, 0.0)) < 6e-3, (x, p, w, wr)
        done += 1


def test_general_weights_invariants_and_hull_rule():
    """Sum 1, non-negative; linear precision (sum_p w_p h_p = h) strictly
    inside the hull (Sibson 1981); outside, the weights sit on one hull edge
    and reproduce the nearest boundary point; at parents, delta."""
    beams, R, par = _hex_set()
    hull = sb.convex_hull(par)
    n_out = 0
    for h in beams[::7]:
        w = sb.general_weights(h, par, hull)
        v = np.array(list(w.values()))
        assert abs(v.sum() - 1) < 1e-12 and v.min() > 0
        c = sum(val * np.array(p, float) for p, val in w.items())
        inside, _ = sb._hull_projection(np.array(h, float), hull)
        if inside:
            assert np.abs(c - h).max() < 1e-9
        else:
            n_out += 1
            assert len(w) <= 2
            hv = [tuple(map(int, q)) for q in hull]
            assert all(p in hv for p in w)
            assert np.hypot(*(c - h)) <= min(np.hypot(*(np.array(q) - h)) for q in hv) + 1e-12
    assert n_out > 0
    for p in par[::5]:
        assert sb.general_weights(p, par, hull) == {tuple(int(v) for v in p): 1.0}


def test_full_parent_set_is_exact():
    """Parents = every beam: identity weights, so BiP reduces to exact PRISM."""
    cfg = tiny_cfg(ny=32, nx=32, ly=8.0, lx=8.0, alpha=30e-3)
    beams = ph.aperture_beams(cfg)
    hull = sb.convex_hull(beams)
    for h in beams:
        assert sb.general_weights(h, beams, hull) == {tuple(int(v) for v in h): 1.0}


def test_hex_bip_converges_to_exact():
    """More rings, smaller error against the exact dual-matrix map (the
    full-parent limit is exact)."""
    import dataclasses
    cfg = tiny_cfg(ny=64, nx=64, nz=4, ly=16.0, lx=16.0, alpha=0.03, theta=0.04, s=1, scan=(4, 4))
    tp = tiny_problem(cfg, n_atoms=1, W=8, planes=[3], vscale=30.0)
    prob = as_oracle_problem(tp)
    exact = E.exact_dual(prob)
    errs = []
    for nr in (2, 3, 4, 6):
        prob.cfg = dataclasses.replace(cfg, parents="hex", n_radial=nr)
        errs.append(E.rel_l2(E.BiP(prob).run(), exact))
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
