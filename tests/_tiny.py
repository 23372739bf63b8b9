"""Small seeded problems for the oracle pins and the GPU parity tests.

Inputs only (random potentials, windows, transition potentials); none of the
method's arithmetic lives here."""
from __future__ import annotations

import dataclasses

import numpy as np

from paper_2607_00756_amd import specimen


def tiny_cfg(ny=16, nx=16, nz=3, ly=4.0, lx=4.0, dz=2.0, energy=200e3, alpha=20e-3,
             theta=40e-3, s=1, scan=(4, 4)):
    return dataclasses.replace(specimen.WORKLOADS[0], name="tiny", ny=ny, nx=nx, nz=nz, ly=ly, lx=lx,
                               dz=dz, energy_ev=energy, alpha=alpha, theta=theta, partition=s,
                               scan=scan)


@dataclasses.dataclass
class TinyProblem:
    cfg: object
    V: np.ndarray
    tau: np.ndarray
    win_size: np.ndarray
    win_origin: np.ndarray
    H: np.ndarray
    H_off: np.ndarray
    n_ch: int


def tiny_problem(cfg, n_atoms=2, n_ch=2, W=4, seed=0, vscale=20.0, planes=None,
                 real_h=False, zero_v=False, win_sizes=None):
    r = np.random.default_rng(seed)
    V = np.zeros((cfg.nz, cfg.ny, cfg.nx), np.float32) if zero_v else \
        (vscale * r.random((cfg.nz, cfg.ny, cfg.nx))).astype(np.float32)
    if planes is None:
        planes = r.integers(0, cfg.nz, size=n_atoms)
    tau = np.zeros((n_atoms, 3))
    tau[:, 0] = r.random(n_atoms) * cfg.lx
    tau[:, 1] = r.random(n_atoms) * cfg.ly
    tau[:, 2] = (np.asarray(planes) + 0.5) * cfg.dz
    ws = np.full(n_atoms, W, np.int32) if win_sizes is None else np.asarray(win_sizes, np.int32)
    origin = np.stack([r.integers(0, cfg.ny, n_atoms), r.integers(0, cfg.nx, n_atoms)], 1).astype(np.int32)
    parts, offs = [], [0]
    for a in range(n_atoms):
        w = int(ws[a])
        h = r.normal(size=(n_ch, w, w))
        if not real_h:
            h = h + 1j * r.normal(size=(n_ch, w, w))
        parts.append(h.astype(np.complex64).ravel())
        offs.append(offs[-1] + parts[-1].size)
    return TinyProblem(cfg, V, tau, ws, origin, np.concatenate(parts), np.array(offs, np.int64), n_ch)


def as_oracle_problem(tp):
    from oracle import eels
    return eels.Problem(tp.cfg, tp.V, tp.tau, tp.win_size, tp.win_origin, tp.H, tp.H_off, tp.n_ch)
