"""Pins of the oracle's Alg. 3 cube (partitioned S1, per-scan exit
multislice): with the full parent set it is Alg. 1 (the conventional
multislice cube), and at any partition factor it equals Alg. 5 with the exact
detector matrix (every detector beam its own parent), through the bilinear
identity of eq. s2."""
from __future__ import annotations

import dataclasses

from oracle import eels as E
from tests._tiny import as_oracle_problem, tiny_cfg, tiny_problem


def _prob(s, **kw):
    cfg = dataclasses.replace(tiny_cfg(ny=32, nx=32, nz=4, ly=8.0, lx=8.0, alpha=0.04, theta=0.06, s=s,
                                       scan=(3, 4)), **kw)
    tp = tiny_problem(cfg, n_atoms=2, n_ch=2, W=8, vscale=60.0, planes=[1, 3], win_sizes=[8, 12])
    return as_oracle_problem(tp)


def test_cube_at_partition_one_is_alg1():
    prob = _prob(1)
    assert E.rel_l2(E.partitioned_cube(prob), E.conventional(prob, mode=E.OUT_BEAMS)) < 1e-12


def test_cube_equals_alg5_with_the_exact_detector_matrix():
    for kw in (dict(), dict(parents="hex", n_radial=2), dict(focal=True)):
        prob = _prob(2, **kw)
        cube = E.partitioned_cube(prob)
        prob.cfg = dataclasses.replace(prob.cfg, s2_exact=True)
        assert E.rel_l2(E.BiP(prob).run(mode=E.OUT_BEAMS), cube) < 1e-12, kw
