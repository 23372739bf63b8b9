"""Slice potentials from atom positions and their position gradient (FP64).

Oracle (test infrastructure).  Projected potential of an atom (reading of
the forward model's Gaussian-sum potential): v(r) = sum_k A_k exp(-|r -
r_a|^2 / (2 w_k^2)), periodic images out to 10 w_k along each axis, the
whole atom in the slice floor(z / dz).  V_j is the sum over the atoms of
slice j.  The position gradient of a loss with cotangent dL/dV is
dL/dx_a = sum_r dL/dV_j(r) dv_a(r)/dx_a (likewise y; dL/dz = 0 because slice
membership is piecewise constant).
"""
from __future__ import annotations

import math

import numpy as np


def _profile(coord, n, length, width, deriv=False):
    """g(t) = sum_m exp(-(t - c - m L)^2 / 2w^2) on the grid t = i L/n, and
    optionally dg/dc; images with |t - c - m L| <= 10 w."""
    t = np.arange(n) * (length / n)
    cut = 10.0 * width
    g = np.zeros(n)
    dg = np.zeros(n)
    m_lo = int(math.floor((t.min() - coord - cut) / length))
    m_hi = int(math.ceil((t.max() - coord + cut) / length))
    for m in range(m_lo, m_hi + 1):
        d = t - coord - m * length
        inside = np.abs(d) <= cut
        e = np.where(inside, np.exp(-d * d / (2.0 * width * width)), 0.0)
        g += e
        dg += e * d / (width * width)       # d/dc of exp(-(t-c)^2/2w^2)
    return (g, dg) if deriv else g


def slice_of(cfg, z):
    return int(min(max(math.floor(z / cfg.dz), 0), cfg.nz - 1))


def projected_potential(cfg, xyz, amps, widths):
    """V [nz, ny, nx]; amps [n_atoms, K] (A_k per atom), widths [K] (A)."""
    V = np.zeros((cfg.nz, cfg.ny, cfg.nx))
    for a in range(len(xyz)):
        j = slice_of(cfg, xyz[a, 2])
        for k, w in enumerate(widths):
            gy = _profile(xyz[a, 1], cfg.ny, cfg.ly, w)
            gx = _profile(xyz[a, 0], cfg.nx, cfg.lx, w)
            V[j] += amps[a, k] * np.outer(gy, gx)
    return V


def potential_grad(cfg, xyz, amps, widths, dV):
    """dL/dxyz [n_atoms, 3] from dL/dV [nz, ny, nx]; the z column is 0."""
    out = np.zeros((len(xyz), 3))
    for a in range(len(xyz)):
        j = slice_of(cfg, xyz[a, 2])
        for k, w in enumerate(widths):
            gy, dgy = _profile(xyz[a, 1], cfg.ny, cfg.ly, w, deriv=True)
            gx, dgx = _profile(xyz[a, 0], cfg.nx, cfg.lx, w, deriv=True)
            out[a, 0] += amps[a, k] * gy @ dV[j] @ dgx
            out[a, 1] += amps[a, k] * dgy @ dV[j] @ gx
    return out
