"""Multislice step, its transpose, and parent-column sweeps (FP64).

Oracle (test infrastructure).

* One multislice step through slice j is transmit-then-propagate,
  psi -> P (T_j psi) with P = F^-1 diag(P(q)) F (eq. propagator); the
  scattering-matrix advance applies it to every column
  (eq. smatrix-advance).
* The exit operator M_{i->exit} applies the steps of slices i..N_Z-1.
* The detector matrix S2 is defined by the bilinear identity of eq. s2,
  sum_r S2^d(r) w(r) = [F M_{i->exit} w]_{h_d} with the unitary F, hence
  S2^d = M_{i->exit}^T [G^-1/2 exp(-2 pi i h_d.r/N)].  Because P(q) is even
  in q the transposed step is "propagate, then transmit" (T_j P), applied in
  reverse slice order.

Ionisation reading: an event in slice i happens at the entrance of the
slice, before T_i (Alg. 1 applies H before advancing the wave), so S1 at
plane i has seen slices 0..i-1 and S2 at plane i carries slices i..N_Z-1.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

from . import physics

WORKERS = int(os.environ.get("ORACLE_FFT_WORKERS", os.cpu_count() or 1))


def fft2(a):
    return sfft.fft2(a, axes=(-2, -1), workers=WORKERS)


def ifft2(a):
    return sfft.ifft2(a, axes=(-2, -1), workers=WORKERS)


def step(psi, T_j, P):
    """psi <- F^-1[P * F[T_j * psi]] (batched over leading axes)."""
    return ifft2(P * fft2(T_j * psi))


def transpose_step(v, T_j, P):
    """v <- T_j * F^-1[P * F[v]], the transpose of `step` (P even in q)."""
    return T_j * ifft2(P * fft2(v))


def exit_operator(psi, T, P, i):
    """M_{i->exit} psi: steps through slices i..N_Z-1."""
    for j in range(i, T.shape[0]):
        psi = step(psi, T[j], P)
    return psi


def initial_s1(cfg, beams):
    """Unit plane waves exp(+2 pi i h.r/N), one per beam [n, ny, nx]."""
    return np.stack([physics.plane_wave(cfg, h, +1) for h in beams]) if len(beams) else \
        np.zeros((0, cfg.ny, cfg.nx), np.complex128)


def initial_s2(cfg, beams):
    """Conjugate detector waves G^-1/2 exp(-2 pi i h.r/N) [n, ny, nx]."""
    g = cfg.ny * cfg.nx
    return np.stack([physics.plane_wave(cfg, h, -1) for h in beams]) / np.sqrt(g) if len(beams) else \
        np.zeros((0, cfg.ny, cfg.nx), np.complex128)


def s1_at_planes(cfg, beams, T, P, planes, batch=256):
    """{plane i: S1 columns after slices 0..i-1} for each requested plane."""
    planes = sorted(set(int(i) for i in planes))
    out = {i: np.empty((len(beams), cfg.ny, cfg.nx), np.complex128) for i in planes}
    for b0 in range(0, len(beams), batch):
        S = initial_s1(cfg, beams[b0:b0 + batch])
        j = 0
        for i in planes:
            while j < i:
                S = step(S, T[j], P)
                j += 1
            out[i][b0:b0 + len(S)] = S
    return out


def s2_at_planes(cfg, beams, T, P, planes, batch=256):
    """{plane i: S2 columns = M_{i->exit}^T chi*_d} for each requested plane."""
    planes = sorted(set(int(i) for i in planes), reverse=True)
    out = {i: np.empty((len(beams), cfg.ny, cfg.nx), np.complex128) for i in planes}
    for b0 in range(0, len(beams), batch):
        S = initial_s2(cfg, beams[b0:b0 + batch])
        j = T.shape[0] - 1
        for i in planes:
            while j >= i:
                S = transpose_step(S, T[j], P)
                j -= 1
            out[i][b0:b0 + len(S)] = S
    return out


def _crop(cols, y, x):
    return cols[:, y[:, None], x[None, :]]


def s1_windows(cfg, beams, T, P, wins, batch=64):
    """S1 columns cropped to windows as the sweep passes their planes.

    wins: list of (plane i, y pixels, x pixels); returns one [n, W, W] array
    per window, holding S1 after slices 0..i-1 on that window.  The same
    steps as s1_at_planes, but no full column is kept beyond the batch being
    advanced, so the memory is that of the windows."""
    out = [np.empty((len(beams), len(y), len(x)), np.complex128) for (_, y, x) in wins]
    order = sorted(range(len(wins)), key=lambda k: wins[k][0])
    for b0 in range(0, len(beams), batch):
        S = initial_s1(cfg, beams[b0:b0 + batch])
        j = 0
        for k in order:
            i, y, x = wins[k]
            while j < i:
                S = step(S, T[j], P)
                j += 1
            out[k][b0:b0 + len(S)] = _crop(S, y, x)
    return out


def s2_windows(cfg, beams, T, P, wins, batch=64):
    """S2 columns cropped to windows as the transpose sweep passes their
    planes (counterpart of s1_windows; S2 at plane i carries slices i..N_Z-1)."""
    out = [np.empty((len(beams), len(y), len(x)), np.complex128) for (_, y, x) in wins]
    order = sorted(range(len(wins)), key=lambda k: -wins[k][0])
    for b0 in range(0, len(beams), batch):
        S = initial_s2(cfg, beams[b0:b0 + batch])
        j = T.shape[0] - 1
        for k in order:
            i, y, x = wins[k]
            while j >= i:
                S = transpose_step(S, T[j], P)
                j -= 1
            out[k][b0:b0 + len(S)] = _crop(S, y, x)
    return out


def s2_peeled(cfg, beams, T, P, planes):
    """S2 at each plane obtained by building it at the entrance (plane 0) and
    peeling forward one slice at a time with the inverse transpose step
    (the PeelTo of Algs. 4 and 5).  Used only to cross-check s2_at_planes."""
    planes = sorted(set(int(i) for i in planes))
    S = s2_at_planes(cfg, beams, T, P, [0])[0]
    out = {}
    j = 0
    for i in planes:
        while j < i:
            # undo v <- T_j P v : v <- P^-1 (conj(T_j) v)  (both unitary)
            S = ifft2(np.conj(P) * fft2(np.conj(T[j]) * S))
            j += 1
        out[i] = S.copy()
    return out
