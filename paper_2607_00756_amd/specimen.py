"""Seeded synthetic specimens: the inputs shared by the GPU path and the FP64 oracle.

This module holds no arithmetic of the BiP-PRISM method itself (no beams, no
propagation, no interpolation, no contraction).  It only draws atoms, builds
the projected slice potentials V_j that enter the transmission function
(forward model, "Grid, probe and specimen"), the transition potentials H_n0
sampled on each ionized atom's crop window (eq. inelastic), and the scan
raster.  Both sides read the very same float32 / complex64 arrays.

Readings of the paper that fix these inputs (all stated here so both sides
agree):

* Projected atomic potential: a 4-term Gaussian sum per atom,
  v(r) = sum_k a_k exp(-|r - r_a|^2 / (2 w_k^2)) with a = (10, 5, 2, 1) V*A
  and w = (0.2, 0.5, 1.0, 2.0) A, periodic images summed while |d| <= 10 w_k
  per axis.  The whole atom goes into the slice floor(z / dz).
* Transition potentials: g = exp(-rho^2 / (2 w^2)), w = 0.3 A, amplitude 1,
  rho the minimum-image displacement from the atom.  Dipole-like forms
  {x/rho, y/rho, 1} g; quadrupole-like forms
  {x^2/rho^2, y^2/rho^2, xy/rho^2, x/rho, y/rho, 1} g rho^2/w^2; x/rho := 0 at
  rho = 0.  H is zero outside the W x W crop window.
* Crop window: W x W pixels with origin floor(tau/delta + 1/2) - W/2 (mod N),
  wrapping periodically.
* Scan raster: rho_{u,v} = (u N_y / S_y, v N_x / S_x) pixels, origin 0.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Gaussian-sum projected potential (amplitude V*A, width A)
POT_AMPS = (10.0, 5.0, 2.0, 1.0)
POT_WIDTHS = (0.2, 0.5, 1.0, 2.0)
TP_WIDTH = 0.3  # transition-potential Gaussian width (A)


@dataclasses.dataclass
class Config:
    name: str
    ny: int
    nx: int
    nz: int
    ly: float
    lx: float
    dz: float
    energy_ev: float
    alpha: float          # probe convergence semi-angle (rad)
    theta: float          # EELS collection semi-angle (rad)
    partition: int        # parent lattice factor s
    scan: tuple           # (S_y, S_x)
    lattice: str          # "sc" | "fcc"
    a: float              # lattice constant (A)
    lz_cell: float        # specimen thickness used for sites (A)
    z_offset: float
    sigma_disp: float
    channels: str         # "l1" | "l1l2" | "l2first5"
    win: object           # int, or tuple of choices
    ionize: str           # selection rule
    n_ionized: int = 0
    ionizable_frac: float = 0.0
    vacancy_frac: float = 0.0
    species_b_scale: float = 1.0
    parents: str = "lattice"      # "lattice" (partition factor s) | "hex" (hex rings)
    n_radial: int = 4             # hex rings: ring count and angular samples of ring 0
    n_angular: int = 6
    focal: bool = False           # focal back-propagation of the S1 parent windows
    s2_exact: bool = False        # S2 over every detector beam (the cube of Alg. 3)
    interp_f: int = 1             # PRISM interpolation factor f (beams kept at h = 0 mod f)


WORKLOADS = {
    0: Config("c0-tiny", 128, 128, 10, 16.0, 16.0, 2.0, 200e3, 20e-3, 40e-3, 4, (16, 16),
              "sc", 4.0, 20.0, 1.0, 0.08, "l1", 32, "nearest_centre"),
    1: Config("c1-medium", 256, 256, 50, 40.0, 40.0, 2.0, 300e3, 25e-3, 50e-3, 4, (64, 64),
              "fcc", 3.6, 100.0, 0.5, 0.1, "l1l2", 24, "columns4"),
    2: Config("c2-fullmap", 512, 512, 100, 80.0, 80.0, 2.0, 300e3, 30e-3, 60e-3, 6, (128, 128),
              "fcc", 3.6, 200.0, 0.5, 0.1, "l1", (24, 32, 40, 48, 56, 64), "random_ionizable",
              n_ionized=2000, ionizable_frac=0.3, species_b_scale=2.0),
    3: Config("c3-qeels", 1024, 1024, 75, 60.0, 60.0, 2.0, 200e3, 25e-3, 60e-3, 8, (96, 96),
              "fcc", 3.6, 150.0, 0.5, 0.1, "l2first5", 64, "random_any",
              n_ionized=200, vacancy_frac=0.02),
    4: Config("c4-gradient", 256, 256, 30, 40.0, 40.0, 2.0, 200e3, 20e-3, 40e-3, 4, (48, 48),
              "fcc", 3.6, 60.0, 0.5, 0.1, "l1", 24, "columns4_middepth"),
}


@dataclasses.dataclass
class Specimen:
    cfg: Config
    xyz: np.ndarray          # [n_atoms, 3] float64 (x, y, z) in A, displaced, wrapped
    species: np.ndarray      # [n_atoms] int32 (0 = A, 1 = B)
    ionized: np.ndarray      # [n_ion] int64 indices into xyz
    tau: np.ndarray          # [n_ion, 3] float64 positions of ionized atoms (x, y, z)
    win_size: np.ndarray     # [n_ion] int32
    win_origin: np.ndarray   # [n_ion, 2] int32 (oy, ox)
    n_ch: int
    H: np.ndarray            # flat complex64, ragged [atom][n_ch][W][W]
    H_off: np.ndarray        # [n_ion + 1] int64 offsets into H (complex elements)
    V: np.ndarray            # [nz, ny, nx] float32 projected potential (V*A)

    def H_atom(self, a: int) -> np.ndarray:
        w = int(self.win_size[a])
        return self.H[self.H_off[a]:self.H_off[a + 1]].reshape(self.n_ch, w, w)


def rng(cfg_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([cfg_id, stream])


# --------------------------------------------------------------------- sites
def _sites(cfg: Config):
    """Nominal sites (x, y, z) and a column id per site."""
    if cfg.lattice == "sc":
        step = cfg.a
        ni = int(math.floor(cfg.lx / step - 1e-9)) + 1
        nj = int(math.floor(cfg.ly / step - 1e-9)) + 1
        pts, col = [], []
        for i in range(ni):
            for j in range(nj):
                k = 0
                while cfg.z_offset + k * step < cfg.lz_cell:
                    pts.append((i * step, j * step, cfg.z_offset + k * step))
                    col.append(i * nj + j)
                    k += 1
        return np.array(pts, dtype=np.float64), np.array(col, dtype=np.int64)
    # FCC projected along [001]: columns on an a/2 square grid, alternate
    # columns offset by a/2 in z.
    h = cfg.a / 2.0
    ni = int(math.floor(cfg.lx / h - 1e-9)) + 1
    nj = int(math.floor(cfg.ly / h - 1e-9)) + 1
    xs, ys, zs, cols = [], [], [], []
    for i in range(ni):
        for j in range(nj):
            z0 = cfg.z_offset + ((i + j) % 2) * h
            nk = int(math.floor((cfg.lz_cell - z0) / cfg.a - 1e-9)) + 1 if z0 < cfg.lz_cell else 0
            z = z0 + cfg.a * np.arange(nk)
            xs.append(np.full(nk, i * h))
            ys.append(np.full(nk, j * h))
            zs.append(z)
            cols.append(np.full(nk, i * nj + j))
    pts = np.stack([np.concatenate(xs), np.concatenate(ys), np.concatenate(zs)], axis=1)
    return pts, np.concatenate(cols).astype(np.int64)


def _nearest_columns(nominal, col, centre_xy, n):
    ucol, first = np.unique(col, return_index=True)
    cxy = nominal[first, :2]
    d2 = (cxy[:, 0] - centre_xy[0]) ** 2 + (cxy[:, 1] - centre_xy[1]) ** 2
    order = np.lexsort((cxy[:, 0], cxy[:, 1], np.round(d2, 9)))
    return ucol[order[:n]]


# ----------------------------------------------------------------- potential
def _axis_profiles(pos, n, length, width):
    """[n_atoms, n] periodic Gaussian profile exp(-d^2/2w^2), |d| <= 10 w."""
    delta = length / n
    grid = np.arange(n) * delta
    cut = 10.0 * width
    n_img = int(math.ceil((cut + length) / length))
    out = np.zeros((pos.shape[0], n), dtype=np.float64)
    for m in range(-n_img, n_img + 1):
        d = grid[None, :] - pos[:, None] - m * length
        mask = np.abs(d) <= cut
        out += np.where(mask, np.exp(-d * d / (2.0 * width * width)), 0.0)
    return out


def projected_potential(cfg: Config, xyz: np.ndarray, species: np.ndarray,
                        scale_b: float = 1.0) -> np.ndarray:
    """Slice potentials V_j [nz, ny, nx] in float64 (V*A)."""
    V = np.zeros((cfg.nz, cfg.ny, cfg.nx), dtype=np.float64)
    plane = np.clip(np.floor(xyz[:, 2] / cfg.dz).astype(np.int64), 0, cfg.nz - 1)
    amp_scale = np.where(species == 1, scale_b, 1.0)
    for j in range(cfg.nz):
        sel = np.nonzero(plane == j)[0]
        if sel.size == 0:
            continue
        for ak, wk in zip(POT_AMPS, POT_WIDTHS):
            gy = _axis_profiles(xyz[sel, 1], cfg.ny, cfg.ly, wk) * (ak * amp_scale[sel])[:, None]
            gx = _axis_profiles(xyz[sel, 0], cfg.nx, cfg.lx, wk)
            V[j] += gy.T @ gx
    return V


# ------------------------------------------------------- transition potential
def _forms(kind: str):
    l1 = ["x", "y", "1"]
    l2 = ["xx", "yy", "xy", "x2", "y2", "12"]
    if kind == "l1":
        return l1
    if kind == "l1l2":
        return l1 + l2
    if kind == "l2first5":
        return l2[:5]
    raise ValueError(kind)


def window_origin(tau_xy, W, cfg: Config):
    dy, dx = cfg.ly / cfg.ny, cfg.lx / cfg.nx
    oy = (int(math.floor(tau_xy[1] / dy + 0.5)) - W // 2) % cfg.ny
    ox = (int(math.floor(tau_xy[0] / dx + 0.5)) - W // 2) % cfg.nx
    return oy, ox


def transition_potentials(cfg: Config, tau, W, origin, forms, width=TP_WIDTH,
                          with_grad=False, complex_variant=False):
    """H_n on the window [n_ch, W, W] (complex128); optionally dH/dx, dH/dy
    with respect to the atom position (i.e. minus the spatial gradient)."""
    dy, dx = cfg.ly / cfg.ny, cfg.lx / cfg.nx
    oy, ox = origin
    yy = ((oy + np.arange(W)) % cfg.ny) * dy
    xx = ((ox + np.arange(W)) % cfg.nx) * dx
    ry = yy[:, None] - tau[1]
    rx = xx[None, :] - tau[0]
    ry = ry - cfg.ly * np.round(ry / cfg.ly)
    rx = rx - cfg.lx * np.round(rx / cfg.lx)
    ry, rx = np.broadcast_arrays(ry, rx)
    r2 = rx * rx + ry * ry
    r = np.sqrt(r2)
    w2 = width * width
    g = np.exp(-r2 / (2 * w2))
    safe = np.where(r > 0, r, 1.0)
    ux = np.where(r > 0, rx / safe, 0.0)
    uy = np.where(r > 0, ry / safe, 0.0)
    # polynomial part p (in rx, ry) such that form = p * g
    polys = {
        "x": (ux, None), "y": (uy, None), "1": (np.ones_like(r), None),
        "xx": (rx * rx / w2, None), "yy": (ry * ry / w2, None), "xy": (rx * ry / w2, None),
        "x2": (rx * r / w2, None), "y2": (ry * r / w2, None), "12": (r2 / w2, None),
    }
    H = np.stack([polys[f][0] * g for f in forms]).astype(np.complex128)
    if complex_variant:
        ph = np.exp(1j * np.arctan2(ry, rx))
        H = H * ph[None]
    if not with_grad:
        return H
    # d/d tau = - d/d r ; finite form of the analytic derivative (inputs only)
    eps = 1e-6
    Hp = transition_potentials(cfg, (tau[0] + eps, tau[1]), W, origin, forms, width,
                               complex_variant=complex_variant)
    Hm = transition_potentials(cfg, (tau[0] - eps, tau[1]), W, origin, forms, width,
                               complex_variant=complex_variant)
    dHx = (Hp - Hm) / (2 * eps)
    Hp = transition_potentials(cfg, (tau[0], tau[1] + eps), W, origin, forms, width,
                               complex_variant=complex_variant)
    Hm = transition_potentials(cfg, (tau[0], tau[1] - eps), W, origin, forms, width,
                               complex_variant=complex_variant)
    dHy = (Hp - Hm) / (2 * eps)
    return H, dHx, dHy


# ------------------------------------------------------------------ assemble
def make(cfg_id: int, cfg: Optional[Config] = None, n_ionized: Optional[int] = None,
         positions_override: Optional[np.ndarray] = None,
         win_origin_override: Optional[np.ndarray] = None) -> Specimen:
    """Build the seeded specimen of a configuration.

    cfg may override the geometry (tests shrink grids); positions_override
    replaces the displaced positions (gradient targets); win_origin_override
    pins the windows (held at the unperturbed origins)."""
    cfg = cfg or WORKLOADS[cfg_id]
    nominal, col = _sites(cfg)
    n = nominal.shape[0]
    r_species = rng(cfg_id, 1)
    keep = np.ones(n, dtype=bool)
    species = np.zeros(n, dtype=np.int32)
    if cfg.vacancy_frac > 0:
        keep = r_species.random(n) >= cfg.vacancy_frac
    if cfg.ionizable_frac > 0:
        species = (r_species.random(n) < cfg.ionizable_frac).astype(np.int32)
    disp = rng(cfg_id, 0).normal(0.0, cfg.sigma_disp, size=(n, 3))
    xyz = nominal + disp
    nominal, col, species, xyz = nominal[keep], col[keep], species[keep], xyz[keep]
    n = nominal.shape[0]
    xyz[:, 0] %= cfg.lx
    xyz[:, 1] %= cfg.ly
    xyz[:, 2] = np.clip(xyz[:, 2], 0.0, np.nextafter(cfg.nz * cfg.dz, 0.0))
    if positions_override is not None:
        xyz = np.array(positions_override, dtype=np.float64, copy=True)

    # ionized selection
    r_sel = rng(cfg_id, 2)
    if cfg.ionize == "nearest_centre":
        c = np.array([cfg.lx / 2, cfg.ly / 2, cfg.lz_cell / 2])
        d2 = np.sum((nominal - c) ** 2, axis=1)
        order = np.lexsort((nominal[:, 0], nominal[:, 1], nominal[:, 2], np.round(d2, 9)))
        ionized = order[:1]
    elif cfg.ionize == "columns4":
        cols = _nearest_columns(nominal, col, (cfg.lx / 2, cfg.ly / 2), 4)
        ionized = np.concatenate([np.nonzero(col == c)[0][np.argsort(nominal[col == c, 2])]
                                  for c in cols])
    elif cfg.ionize == "columns4_middepth":
        cols = _nearest_columns(nominal, col, (cfg.lx / 2, cfg.ly / 2), 4)
        parts = []
        for c in cols:
            idx = np.nonzero(col == c)[0]
            dz = np.abs(nominal[idx, 2] - cfg.lz_cell / 2)
            o = np.lexsort((nominal[idx, 2], np.round(dz, 9)))[:4]
            parts.append(np.sort(idx[o]))
        ionized = np.concatenate(parts)
    elif cfg.ionize == "random_ionizable":
        cand = np.nonzero(species == 1)[0]
        ionized = np.sort(r_sel.choice(cand, size=min(cfg.n_ionized, cand.size), replace=False))
    elif cfg.ionize == "random_any":
        ionized = np.sort(r_sel.choice(n, size=cfg.n_ionized, replace=False))
    else:
        raise ValueError(cfg.ionize)
    if n_ionized is not None:
        ionized = ionized[:n_ionized]
    tau = xyz[ionized].copy()

    # windows
    n_ion = ionized.size
    if isinstance(cfg.win, tuple):
        win = rng(cfg_id, 3).choice(np.array(cfg.win), size=n_ion).astype(np.int32)
    else:
        win = np.full(n_ion, int(cfg.win), dtype=np.int32)
    origin = np.zeros((n_ion, 2), dtype=np.int32)
    for a in range(n_ion):
        origin[a] = window_origin(tau[a], int(win[a]), cfg)
    if win_origin_override is not None:
        origin = np.array(win_origin_override, dtype=np.int32, copy=True)

    forms = _forms(cfg.channels)
    H_parts, offs = [], [0]
    for a in range(n_ion):
        Ha = transition_potentials(cfg, tau[a], int(win[a]), tuple(origin[a]), forms)
        H_parts.append(Ha.astype(np.complex64).ravel())
        offs.append(offs[-1] + H_parts[-1].size)
    H = np.concatenate(H_parts) if H_parts else np.zeros(0, np.complex64)

    V = projected_potential(cfg, xyz, species, cfg.species_b_scale).astype(np.float32)
    return Specimen(cfg, xyz, species, ionized.astype(np.int64), tau, win, origin,
                    len(forms), H, np.array(offs, dtype=np.int64), V)


def shrink(cfg_id: int, **kw) -> Config:
    """A copy of a configuration with some fields replaced (small test cases)."""
    return dataclasses.replace(WORKLOADS[cfg_id], **kw)
