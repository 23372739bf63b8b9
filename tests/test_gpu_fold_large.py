"""The probe fold on an S1 window block beyond 2 GiB.

The fold reads an atom's parent windows through a buffer descriptor with
32-bit offsets, and through 64-bit pointers when the atom's block (parents x
window pixels x 8 bytes) is larger.  At partition factor 1 every aperture
beam is its own parent with weight 1, so the reconstruction is the identity
and focal back-propagation of S1 (section "Magnitude-preserving
reconstruction and focal back-propagation") is an exact Fresnel round trip on
the enlarged window: the focal map equals the plain one.  With about 17,000
parents the focal atom's 128 x 128 windows exceed 2 GiB (pointer path) while
the plain run's 64 x 64 windows do not (buffer path).  Bar: rel-L2 1e-5 in
FP32 (complex64 Fresnel steps)."""
from __future__ import annotations

import dataclasses

import pytest

from oracle import physics
from tests._tiny import tiny_cfg, tiny_problem
from tests.gpu_helpers import gpu_run, rel_l2

pytestmark = pytest.mark.gpu

LIMIT = 2**31 - 1  # bytes addressable by the fold's buffer offsets


def test_focal_map_over_a_window_block_beyond_2gib_equals_the_plain_map():
    from paper_2607_00756_amd import bip
    cfg = tiny_cfg(ny=256, nx=256, nz=2, ly=40.0, lx=40.0, alpha=0.046, theta=0.01, s=1, scan=(4, 4))
    B = len(physics.aperture_beams(cfg))
    assert B * 64 * 64 * 8 <= LIMIT < B * 128 * 128 * 8  # the plain block fits, the focal one does not
    tp = tiny_problem(cfg, n_atoms=1, n_ch=2, W=64, seed=7, planes=[1])
    args = (tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off, tp.n_ch, bip.OUT_MAP, bip.PREC_FP32)
    plain, p0 = gpu_run(cfg, tp.V, *args)
    n0 = p0.Bp1
    p0.close()
    focal, p1 = gpu_run(dataclasses.replace(cfg, focal=True), tp.V, *args)
    n1 = p1.Bp1
    p1.close()
    assert n0 == n1 >= B and n1 * 128 * 128 * 8 > LIMIT
    err = rel_l2(focal, plain)
    print(f"[fold beyond 2 GiB] parents {n1}, focal block {n1 * 128 * 128 * 8 / 2**30:.2f} GiB, "
          f"focal vs plain map rel-L2 {err:.2e}")
    assert plain.max() > 0
    assert err < 1e-5
