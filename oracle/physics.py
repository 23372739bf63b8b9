"""Physical constants, beam sets and the multislice operators (FP64).

Oracle (test infrastructure).  Follows the paper's forward model section
"Grid, probe and specimen": corner-origin DFT grid, integer beam index h with
signed frequency q = h / L, aperture support, transmission exp(i sigma V_j)
and the Fresnel transfer function P(q) = exp(-i pi lambda dz |q|^2)
(eq. propagator).  The paper gives no formula for lambda or sigma; the
relativistic textbook forms are used (CODATA 2018 constants).
"""
from __future__ import annotations

import math

import numpy as np

# CODATA 2018 (exact SI definitions for h, e, c)
H_PLANCK = 6.62607015e-34
E_CHARGE = 1.602176634e-19
C_LIGHT = 299792458.0
M_ELECTRON = 9.1093837015e-31


def wavelength(energy_ev: float) -> float:
    """Relativistic electron wavelength in Angstrom."""
    e = E_CHARGE * energy_ev
    mc2 = M_ELECTRON * C_LIGHT ** 2
    p = math.sqrt(2.0 * M_ELECTRON * e * (1.0 + e / (2.0 * mc2)))
    return H_PLANCK / p * 1e10


def interaction_constant(energy_ev: float) -> float:
    """sigma in rad / (V * Angstrom): (2 pi / (lambda E)) (mc^2 + eE)/(2 mc^2 + eE)."""
    lam = wavelength(energy_ev)
    mc2_ev = M_ELECTRON * C_LIGHT ** 2 / E_CHARGE
    return 2.0 * math.pi / (lam * energy_ev) * (mc2_ev + energy_ev) / (2.0 * mc2_ev + energy_ev)


def signed_index(n: int) -> np.ndarray:
    """Signed integer frequency index of each corner-origin DFT bin, in [-n/2, n/2)."""
    k = np.arange(n)
    return np.where(k < n // 2, k, k - n)


def beams_within(ny: int, nx: int, ly: float, lx: float, qmax: float) -> np.ndarray:
    """All beams h = (h_y, h_x) with |q|^2 <= qmax^2, sorted by (h_y, h_x).

    Inclusive edge; tested in float64 as (h_y/L_y)^2 + (h_x/L_x)^2 <= qmax^2."""
    hy = signed_index(ny)
    hx = signed_index(nx)
    out = []
    for y in sorted(hy):
        for x in sorted(hx):
            if (y / ly) ** 2 + (x / lx) ** 2 <= qmax * qmax:
                out.append((y, x))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def aperture_beams(cfg) -> np.ndarray:
    return beams_within(cfg.ny, cfg.nx, cfg.ly, cfg.lx, cfg.alpha / wavelength(cfg.energy_ev))


def detector_beams(cfg) -> np.ndarray:
    return beams_within(cfg.ny, cfg.nx, cfg.ly, cfg.lx, cfg.theta / wavelength(cfg.energy_ev))


def propagator(cfg) -> np.ndarray:
    """P(q) = exp(-i pi lambda dz |q|^2) on the corner-origin grid."""
    lam = wavelength(cfg.energy_ev)
    qy = signed_index(cfg.ny) / cfg.ly
    qx = signed_index(cfg.nx) / cfg.lx
    q2 = qy[:, None] ** 2 + qx[None, :] ** 2
    return np.exp(-1j * math.pi * lam * cfg.dz * q2)


def transmissions(cfg, V: np.ndarray) -> np.ndarray:
    """T_j = exp(i sigma V_j) for every slice, complex128 [nz, ny, nx]."""
    sigma = interaction_constant(cfg.energy_ev)
    return np.exp(1j * sigma * V.astype(np.float64))


def plane_wave(cfg, h, sign: int = +1) -> np.ndarray:
    """exp(sign * 2 pi i (h_y y / N_y + h_x x / N_x)) on the pixel grid."""
    y = np.arange(cfg.ny)
    x = np.arange(cfg.nx)
    ph = (h[0] * y[:, None]) / cfg.ny + (h[1] * x[None, :]) / cfg.nx
    return np.exp(sign * 2j * math.pi * ph)


def slice_of(cfg, z: float) -> int:
    """Slice containing depth z: floor(z / dz), clamped to the stack."""
    return int(min(max(math.floor(z / cfg.dz), 0), cfg.nz - 1))
