"""Conventional, exact dual-matrix and BiP-PRISM EELS (FP64).

Oracle (test infrastructure).  Implements

* Alg. 1 (conventional transition-potential multislice): the ground truth.
* Alg. 4 (exact dual-matrix map, PRISM factor f = 1): S1 over all aperture
  beams, S2 over all detector beams, coupling on the crop window
  (eq. coupling).
* Alg. 5 (BiP-PRISM): S1 and S2 on lattice parents, windowed
  reconstruction (eq. window-recon) in magnitude-preserving
  (eq. magpreserve) or complex mode, then the same coupling.

Conventions (readings of the paper, shared with the GPU path):
* probe coefficients c_b = Psi(h_b) = 1/sqrt(G B) inside the aperture (no
  aberrations), so the probe has unit norm (eq. probe);
* illumination c_b(rho) = c_b exp(-2 pi i h_b.rho/N), rho on the raster
  (u N_y/S_y, v N_x/S_x);
* detector amplitudes use the unitary DFT;
* de-tilt by the column's own carrier and re-tilt by the target beam's:
  S1 carrier exp(+2 pi i h.r/N), S2 carrier exp(-2 pi i h.r/N);
* sgn(0) = 0 in the magnitude-preserving mode;
* outputs: MAP I(rho) (eq. map-sum), QEELS I(q_x, rho) resolving h_x and
  summing h_y, BEAMS I(d, rho); summed over atoms in input order and over
  channels in order.
"""
from __future__ import annotations

import math

import numpy as np

from . import multislice as ms
from . import physics
from .sibson import HexPartition, Partition

RECON_MAGNITUDE = 0
RECON_COMPLEX = 1
OUT_MAP, OUT_QEELS, OUT_BEAMS = 0, 1, 2


# ------------------------------------------------------------------ geometry
def window_pixels(cfg, W, origin):
    """Absolute (y, x) pixel indices of a W x W window at origin (mod N)."""
    y = (origin[0] + np.arange(W)) % cfg.ny
    x = (origin[1] + np.arange(W)) % cfg.nx
    return y, x


def carrier(cfg, h, y, x, sign):
    """exp(sign 2 pi i (h_y y/N_y + h_x x/N_x)) on window pixels [.., W, W]."""
    h = np.atleast_2d(h)
    ph = (h[:, 0, None, None] * y[None, :, None]) / cfg.ny + \
         (h[:, 1, None, None] * x[None, None, :]) / cfg.nx
    return np.exp(sign * 2j * math.pi * ph)


def scan_positions(cfg):
    """Raster positions (rho_y, rho_x) in pixels, p = u S_x + v."""
    sy, sx = cfg.scan
    u, v = np.meshgrid(np.arange(sy), np.arange(sx), indexing="ij")
    return np.stack([u.ravel() * cfg.ny / sy, v.ravel() * cfg.nx / sx], axis=1)


def illumination(cfg, beams, n_aperture=None, scale=1.0):
    """c_b(rho) [P, B] = c_b exp(-2 pi i (h_y u / S_y + h_x v / S_x)).

    c_b = scale / sqrt(G n_aperture), n_aperture the size of the whole
    aperture (default: the beams given); with PRISM subsampling the retained
    beams keep the coefficient of the whole aperture times f_y f_x (section
    "Exact PRISM-EELS", interpolation factor)."""
    sy, sx = cfg.scan
    G = cfg.ny * cfg.nx
    cb = scale / math.sqrt(G * (len(beams) if n_aperture is None else n_aperture))
    u, v = np.meshgrid(np.arange(sy), np.arange(sx), indexing="ij")
    u = u.ravel()[:, None]
    v = v.ravel()[:, None]
    ph = (beams[None, :, 0] * u) / sy + (beams[None, :, 1] * v) / sx
    return cb * np.exp(-2j * math.pi * ph)


def prism_subsample(beams, f):
    """Alg. 2 beam subsampling by the interpolation factor: keep the beams
    with h_y = 0 and h_x = 0 (mod f)."""
    beams = np.asarray(beams)
    keep = (beams[:, 0] % f == 0) & (beams[:, 1] % f == 0)
    return beams[keep]


def crop_mask(cfg, tau, f):
    """PRISM crop mask of one atom [P] (bool): the scan positions whose
    f-periodic probe (period N/f) holds the atom inside its alias-free
    window (section "Exact PRISM-EELS"; the crop mask of Alg. 4).  Reading:
    the minimum-image displacement atom - rho, in pixels per axis, lies in
    [-N/(2f), N/(2f)); tau = (x, y, z) in A.  f = 1 keeps every scan."""
    rho = scan_positions(cfg)                                   # (y, x) pixels
    t = np.array([tau[1] * cfg.ny / cfg.ly, tau[0] * cfg.nx / cfg.lx])
    N = np.array([cfg.ny, cfg.nx], dtype=np.float64)
    d = (t[None, :] - rho + N / 2) % N - N / 2
    return np.all((d >= -N / (2 * f)) & (d < N / (2 * f)), axis=1)


def qeels_bins(cfg):
    """Number of q_x bins and the bin of each detector beam (h_x + floor(r))."""
    lam = physics.wavelength(cfg.energy_ev)
    r = cfg.theta / lam * cfg.lx
    half = int(math.floor(r + 1e-12))
    return 2 * half + 1, half


def reduce_output(cfg, I_dp, det, mode):
    """Reduce per-beam intensities I[d, rho] to the requested output."""
    if mode == OUT_BEAMS:
        return I_dp.T.copy()                     # [P, n_det]
    if mode == OUT_MAP:
        return I_dp.sum(axis=0)                  # [P]
    nq, half = qeels_bins(cfg)
    out = np.zeros((I_dp.shape[1], nq))
    np.add.at(out.T, det[:, 1] + half, I_dp)
    return out                                   # [P, n_q]


# --------------------------------------------- focal back-propagation of S1
def centroid_depth(prob, a):
    """Depth of the scattering centroid of atom a's entrance-to-ionization
    path (section "Magnitude-preserving reconstruction and focal
    back-propagation"; the paper gives no formula).  Reading: the mean depth
    of the slices above the ionization plane, each slice j at its mid-depth
    (j + 1/2) dz and weighted by its projected potential summed over the
    atom's window; with no potential on the path (or at plane 0) the
    ionization plane itself (no back-propagation)."""
    cfg = prob.cfg
    i = int(prob.planes[a])
    y, x = prob.window(a)
    m = np.array([float(np.sum(prob.V[j][y[:, None], x[None, :]], dtype=np.float64)) for j in range(i)])
    if i == 0 or m.sum() <= 0.0:
        return i * cfg.dz
    return float(np.sum((np.arange(i) + 0.5) * cfg.dz * m) / m.sum())


def focal_window(cfg, W, origin):
    """The enlarged ("padded") window of the focal step: M x M pixels, M the
    smallest power of two >= 2W (at most 128), centred on the W x W window:
    (M, margin, y pixels, x pixels).  Reading: "padded" means a margin of
    the column's own field around the window, so that the Fresnel step of
    the window content sees its surroundings; the margin is cropped away
    after the step."""
    M = min(128, 1 << (2 * W - 1).bit_length())
    pad = (M - W) // 2
    y = (origin[0] - pad + np.arange(M)) % cfg.ny
    x = (origin[1] - pad + np.arange(M)) % cfg.nx
    return M, pad, y, x


def window_fresnel(cfg, f, dist, sign):
    """Fresnel step of fields f [..., M, M] on their window, taken as periodic:
    multiply the window's DFT by exp(sign i pi lambda dist |q|^2), q the
    frequencies of the window grid (k / (M delta) per axis, signed k).
    sign = -1 propagates forward by dist (eq. propagator), +1 back."""
    M = f.shape[-1]
    lam = physics.wavelength(cfg.energy_ev)
    qy = physics.signed_index(M) / (M * cfg.ly / cfg.ny)
    qx = physics.signed_index(M) / (M * cfg.lx / cfg.nx)
    E = np.exp(sign * 1j * math.pi * lam * dist * (qy[:, None] ** 2 + qx[None, :] ** 2))
    return np.fft.ifft2(E * np.fft.fft2(f, axes=(-2, -1)), axes=(-2, -1))


# -------------------------------------------------------------- contraction
def contract_probe_order(S1w, S2w, H, C, psi=None):
    """Per-beam intensity of one atom, probe order.

    S1w [B, W, W], S2w [n_det, W, W], H [n_ch, W, W], C [P, B].
    psi(r, rho) = sum_b S1^b(r) c_b(rho); a_d = sum_r S2^d(r) H_n(r) psi(r, rho);
    returns sum_n |a_d|^2 as [n_det, P].  psi [K, P] may be given instead."""
    K = S2w.shape[1] * S2w.shape[2]
    if psi is None:
        psi = S1w.reshape(S1w.shape[0], K).T @ C.T   # [K, P]
    S2 = S2w.reshape(S2w.shape[0], K)
    I = np.zeros((S2.shape[0], C.shape[0]))
    for n in range(H.shape[0]):
        a = S2 @ (H[n].reshape(K, 1) * psi)      # [n_det, P]
        I += a.real ** 2 + a.imag ** 2
    return I


def contract_m_order(S1w, S2w, H, C):
    """Same quantity via the coupling matrix M_{d,b} (Alg. 4 order)."""
    B = S1w.shape[0]
    K = S1w.shape[1] * S1w.shape[2]
    S1 = S1w.reshape(B, K)
    S2 = S2w.reshape(S2w.shape[0], K)
    I = np.zeros((S2.shape[0], C.shape[0]))
    for n in range(H.shape[0]):
        M = (S2 * H[n].reshape(1, K)) @ S1.T     # [n_det, B]
        a = M @ C.T
        I += a.real ** 2 + a.imag ** 2
    return I


# ---------------------------------------------------------- reconstruction
def reconstruct(cfg, win, parents, Wmat, beams, y, x, side, mode=RECON_MAGNITUDE):
    """Windowed reconstruction of all beams of one matrix (eq. window-recon).

    win [Bp, W, W]: parent columns cropped to the window.  side = 1 for S1
    (carrier +), 2 for S2 (carrier -).  Magnitude mode follows eq.
    magpreserve: (sum_p w |D_p|) * sgn(sum_p w D_p), then re-tilt."""
    s = +1 if side == 1 else -1
    D = win * carrier(cfg, parents, y, x, -s)         # de-tilt
    Wd = Wmat.tocsr()
    Bp = D.shape[0]
    K = D.shape[1] * D.shape[2]
    Df = D.reshape(Bp, K)
    z = Wd @ Df                                        # [n_beams, K]
    if mode == RECON_COMPLEX:
        rec = z
    else:
        m = Wd @ np.abs(Df)
        az = np.abs(z)
        sgn = np.where(az > 0, z / np.where(az > 0, az, 1.0), 0.0)
        rec = m * sgn
    rec = rec.reshape(-1, D.shape[1], D.shape[2])
    return rec * carrier(cfg, beams, y, x, +s)        # re-tilt


# ---------------------------------------------------------------- problem
class Problem:
    """Everything the three algorithms share for one specimen."""

    def __init__(self, cfg, V, tau, win_size, win_origin, H, H_off, n_ch):
        self.cfg = cfg
        self.V = np.asarray(V)
        self.T = physics.transmissions(cfg, self.V)
        self.P = physics.propagator(cfg)
        self.beams = physics.aperture_beams(cfg)
        self.det = physics.detector_beams(cfg)
        self.tau = np.asarray(tau, dtype=np.float64)
        self.win_size = np.asarray(win_size)
        self.win_origin = np.asarray(win_origin)
        self.n_ch = n_ch
        self.H_flat = np.asarray(H)
        self.H_off = np.asarray(H_off)
        self.planes = np.array([physics.slice_of(cfg, z) for z in self.tau[:, 2]], dtype=np.int64)

    @classmethod
    def from_specimen(cls, sp):
        return cls(sp.cfg, sp.V, sp.tau, sp.win_size, sp.win_origin, sp.H, sp.H_off, sp.n_ch)

    def H_atom(self, a):
        W = int(self.win_size[a])
        return self.H_flat[self.H_off[a]:self.H_off[a + 1]].reshape(self.n_ch, W, W).astype(np.complex128)

    def window(self, a):
        return window_pixels(self.cfg, int(self.win_size[a]), self.win_origin[a])

    def crop(self, cols, a):
        y, x = self.window(a)
        return cols[:, y[:, None], x[None, :]]


def _atoms(prob, atoms):
    return list(range(len(prob.tau))) if atoms is None else list(atoms)


# -------------------------------------------------------------- Algorithm 1
def conventional(prob: Problem, mode=OUT_MAP, atoms=None, scans=None):
    """Alg. 1: per scan position, form the probe, multislice it, and at each
    slice containing ionized atoms spawn H_n psi and propagate it to the exit.
    H is the window-restricted transition potential (zero off the window)."""
    cfg = prob.cfg
    atoms = _atoms(prob, atoms)
    C = illumination(cfg, prob.beams)                 # [P, B]
    Pn = C.shape[0]
    scans = range(Pn) if scans is None else scans
    S0 = ms.initial_s1(cfg, prob.beams)               # plane waves
    G = cfg.ny * cfg.nx
    I_dp = np.zeros((len(prob.det), Pn))
    by_plane = {}
    for a in atoms:
        by_plane.setdefault(int(prob.planes[a]), []).append(a)
    for p in scans:
        psi = np.tensordot(C[p], S0, axes=(0, 0))     # eq. probe
        for i in range(cfg.nz):
            for a in by_plane.get(i, []):
                y, x = prob.window(a)
                Ha = prob.H_atom(a)
                for n in range(prob.n_ch):
                    phi = np.zeros_like(psi)
                    phi[y[:, None], x[None, :]] = Ha[n] * psi[y[:, None], x[None, :]]
                    phi = ms.exit_operator(phi, prob.T, prob.P, i)
                    F = ms.fft2(phi) / math.sqrt(G)
                    amp = F[prob.det[:, 0] % cfg.ny, prob.det[:, 1] % cfg.nx]
                    I_dp[:, p] += amp.real ** 2 + amp.imag ** 2
            psi = ms.step(psi, prob.T[i], prob.P)
    return reduce_output(cfg, I_dp, prob.det, mode)


# -------------------------------------------------------------- Algorithm 4
def exact_dual(prob: Problem, mode=OUT_MAP, atoms=None, order="probe"):
    """Alg. 4 with f = 1: exact S1 (all aperture beams) and S2 (all detector
    beams) at each ionization plane; coupling on the crop window."""
    cfg = prob.cfg
    atoms = _atoms(prob, atoms)
    planes = sorted(set(int(prob.planes[a]) for a in atoms))
    S1 = ms.s1_at_planes(cfg, prob.beams, prob.T, prob.P, planes)
    S2 = ms.s2_at_planes(cfg, prob.det, prob.T, prob.P, planes)
    C = illumination(cfg, prob.beams)
    contract = contract_probe_order if order == "probe" else contract_m_order
    I_dp = np.zeros((len(prob.det), C.shape[0]))
    for a in atoms:
        i = int(prob.planes[a])
        I_dp += contract(prob.crop(S1[i], a), prob.crop(S2[i], a), prob.H_atom(a), C)
    return reduce_output(cfg, I_dp, prob.det, mode)


# -------------------------------------------------------------- Algorithm 5
def _lattice_partition(beams, s, f):
    """Lattice parents of PRISM-subsampled beams (all multiples of f): the
    partition of h / f with factor s, parents scaled back by f (Sibson
    weights are unchanged by the scaling)."""
    part = Partition(np.asarray(beams) // f, s)
    part.beams = np.asarray(beams)
    part.parents = part.parents * f
    return part


class BiP:
    """Alg. 5: parents, weights, parent sweeps, windowed reconstruction.

    With the PRISM interpolation factor f = cfg.interp_f > 1 (Alg. 2 and
    Alg. 4) the aperture and detector beams are subsampled (prism_subsample),
    the retained illumination coefficients are scaled by f^2, each atom's
    outputs are kept only on the scans of its crop mask (crop_mask), and the
    detector sums are scaled by f^2.  Reading for the last point (the paper
    states the rescaling for the probe side only): by the same decimation
    argument, a retained detector beam stands for the f x f beams of its
    cell, which keeps the map on the scale of f = 1 when the inelastic wave
    fits the alias-free window."""

    def __init__(self, prob: Problem, recon_mode=RECON_MAGNITUDE):
        self.prob = prob
        cfg = prob.cfg
        self.f = f = int(getattr(cfg, "interp_f", 1))
        if f < 1 or cfg.ny % f or cfg.nx % f:
            raise ValueError("the interpolation factor must divide the grid")
        self.beams = prism_subsample(prob.beams, f)
        self.det = prism_subsample(prob.det, f)
        if getattr(cfg, "parents", "lattice") == "hex":
            # hex-ring parents on the aperture and on the detector disc
            lam = physics.wavelength(cfg.energy_ev)
            self.part1 = HexPartition(self.beams, cfg.n_radial, cfg.n_angular,
                                      cfg.alpha / lam * cfg.ly, cfg.alpha / lam * cfg.lx)
            self.part2 = HexPartition(self.det, cfg.n_radial, cfg.n_angular,
                                      cfg.theta / lam * cfg.ly, cfg.theta / lam * cfg.lx)
        else:
            self.part1 = _lattice_partition(self.beams, cfg.partition, f)
            self.part2 = _lattice_partition(self.det, cfg.partition, f)
        if getattr(cfg, "s2_exact", False):
            self.part2 = Partition(self.det, 1)  # every detector beam its own parent
        self.recon_mode = recon_mode
        self.focal = bool(getattr(cfg, "focal", False))

    def parent_windows(self, atoms):
        """{atom: (S1 parent windows [Bp1, W, W], S2 parent windows [Bp2, W, W])};
        in focal mode the S1 windows are the enlarged M x M ones (focal_window).

        The parent columns are propagated in batches and cropped to each
        window as the sweep passes its plane (memory of the windows only)."""
        prob = self.prob
        cfg = prob.cfg
        atoms = list(atoms)
        wins = [(int(prob.planes[a]),) + tuple(prob.window(a)) for a in atoms]
        wins1 = [(int(prob.planes[a]),) + focal_window(cfg, int(prob.win_size[a]), prob.win_origin[a])[2:]
                 for a in atoms] if self.focal else wins
        w1 = ms.s1_windows(cfg, self.part1.parents, prob.T, prob.P, wins1)
        w2 = ms.s2_windows(cfg, self.part2.parents, prob.T, prob.P, wins)
        return {a: [w1[k], w2[k]] for k, a in enumerate(atoms)}

    def focal_probe(self, a, pw, C):
        """psi [K, P] of atom a with focal back-propagation of S1: the parent
        columns on the enlarged window are Fresnel-stepped back by the
        distance from the ionization plane to the scattering centroid,
        interpolated there (eq. nnw, eq. magpreserve), the probe synthesized,
        stepped forward by the same distance, and cropped to the atom's
        window (section "Magnitude-preserving reconstruction and focal
        back-propagation").  pw[0] holds the enlarged S1 windows."""
        prob = self.prob
        cfg = prob.cfg
        W = int(prob.win_size[a])
        M, pad, y, x = focal_window(cfg, W, prob.win_origin[a])
        dist = int(prob.planes[a]) * cfg.dz - centroid_depth(prob, a)
        back = window_fresnel(cfg, pw[0], dist, +1)
        s1 = reconstruct(cfg, back, self.part1.parents, self.part1.W, self.beams, y, x, 1,
                         self.recon_mode)
        psi_c = np.tensordot(C, s1, axes=(1, 0))            # [P, M, M] at the centroid
        psi = window_fresnel(cfg, psi_c, dist, -1)[:, pad:pad + W, pad:pad + W]
        return psi.reshape(psi.shape[0], W * W).T

    def reconstructed(self, a, pw):
        """(S1~ [B, W, W], S2~ [n_det, W, W]) on the window of atom a (without
        focal back-propagation)."""
        if self.focal:
            raise ValueError("focal mode: S1~ exists only at the centroid, on the enlarged window")
        prob = self.prob
        y, x = prob.window(a)
        s1 = reconstruct(prob.cfg, pw[0], self.part1.parents, self.part1.W, self.beams, y, x, 1,
                         self.recon_mode)
        s2 = reconstruct(prob.cfg, pw[1], self.part2.parents, self.part2.W, self.det, y, x, 2,
                         self.recon_mode)
        return s1, s2

    def illumination(self):
        """c_b(rho) [P, B_f] of the retained aperture beams."""
        return illumination(self.prob.cfg, self.beams, n_aperture=len(self.prob.beams),
                            scale=float(self.f * self.f))

    def run(self, mode=OUT_MAP, atoms=None, order="probe", scans=None, per_atom=False,
            rows=None, progress=None):
        """Outputs of Alg. 5 summed over `atoms` (input order) at the scan
        positions `scans` (indices into the raster; None = all).

        rows: when given, the detector beams are reconstructed and contracted
        rows at a time (each beam's intensity is computed alone, so this only
        bounds the memory of S2~)."""
        prob = self.prob
        atoms = _atoms(prob, atoms)
        pw = self.parent_windows(atoms)
        C = self.illumination()
        sel = np.arange(C.shape[0]) if scans is None else np.asarray(scans)
        C = C[sel]
        contract = contract_probe_order if order == "probe" else contract_m_order
        det = self.det
        I_dp = np.zeros((len(det), C.shape[0]))
        parts = {}
        for a in atoms:
            psi = self.focal_probe(a, pw[a], C) if self.focal else None
            if psi is not None and order != "probe":
                raise ValueError("focal back-propagation acts on the probe: probe order only")
            y, x = prob.window(a)
            s1 = None if psi is not None else \
                reconstruct(prob.cfg, pw[a][0], self.part1.parents, self.part1.W, self.beams, y, x, 1,
                            self.recon_mode)
            if rows is None:
                s2 = reconstruct(prob.cfg, pw[a][1], self.part2.parents, self.part2.W, det, y, x,
                                 2, self.recon_mode)
                Ia = contract(s1, s2, prob.H_atom(a), C, psi) if psi is not None else \
                    contract(s1, s2, prob.H_atom(a), C)
            else:
                Ia = np.zeros_like(I_dp)
                for d0 in range(0, len(det), rows):
                    d1 = min(d0 + rows, len(det))
                    s2 = reconstruct(prob.cfg, pw[a][1], self.part2.parents, self.part2.W[d0:d1],
                                     det[d0:d1], y, x, 2, self.recon_mode)
                    Ia[d0:d1] = contract(s1, s2, prob.H_atom(a), C, psi) if psi is not None else \
                        contract(s1, s2, prob.H_atom(a), C)
            if self.f > 1:
                # detector sums over retained beams, on the atom's crop mask only
                Ia = Ia * float(self.f * self.f)
                Ia[:, ~crop_mask(prob.cfg, prob.tau[a], self.f)[sel]] = 0.0
            if per_atom:
                parts[a] = Ia
            I_dp += Ia
            pw[a] = None
            if progress:
                progress(a)
        out = reduce_output(prob.cfg, I_dp, det, mode)
        return (out, parts) if per_atom else out


# -------------------------------------------------------------- Algorithm 3
def partitioned_cube(prob: Problem, recon_mode=RECON_MAGNITUDE, atoms=None, scans=None):
    """Alg. 3, the energy-filtered 4D cube I(q, rho) [P, n_det] for q in the
    detector: the probe from the partitioned S1 (parents, weights,
    reconstruction and, if configured, focal back-propagation exactly as in
    Alg. 5), then, per scan position and channel, the inelastic wave
    H_n psi on the window propagated to the exit by conventional multislice
    and Fourier-transformed (unitary) to the detector beams (eq. cube)."""
    cfg = prob.cfg
    atoms = _atoms(prob, atoms)
    bip = BiP(prob, recon_mode)
    if bip.f != 1:
        raise ValueError("the 4D cube keeps every exit beam: interpolation factor 1 only")
    pw = bip.parent_windows(atoms)
    C = illumination(cfg, prob.beams)
    if scans is not None:
        C = C[np.asarray(scans)]
    G = cfg.ny * cfg.nx
    I = np.zeros((C.shape[0], len(prob.det)))
    for a in atoms:
        i = int(prob.planes[a])
        y, x = prob.window(a)
        W = len(y)
        if bip.focal:
            psi = bip.focal_probe(a, pw[a], C)                     # [K, P]
        else:
            s1 = reconstruct(cfg, pw[a][0], bip.part1.parents, bip.part1.W, prob.beams, y, x, 1,
                             recon_mode)
            psi = s1.reshape(-1, W * W).T @ C.T
        Ha = prob.H_atom(a)
        for p in range(C.shape[0]):
            for n in range(prob.n_ch):
                phi = np.zeros((cfg.ny, cfg.nx), np.complex128)
                phi[y[:, None], x[None, :]] = Ha[n] * psi[:, p].reshape(W, W)
                phi = ms.exit_operator(phi, prob.T, prob.P, i)
                amp = (ms.fft2(phi) / math.sqrt(G))[prob.det[:, 0] % cfg.ny, prob.det[:, 1] % cfg.nx]
                I[p] += amp.real ** 2 + amp.imag ** 2
    return I


# ------------------------------------------------------------- diagnostics
def on_atom_error(prob: Problem, bip: BiP, a: int):
    """eps_on-atom = ||psi^p - psi||_Omega / ||psi||_Omega (eq. onatom),
    aggregated over all scan positions."""
    cfg = prob.cfg
    i = int(prob.planes[a])
    exact = prob.crop(ms.s1_at_planes(cfg, prob.beams, prob.T, prob.P, [i])[i], a)
    pw = bip.parent_windows([a])[a]
    rec, _ = bip.reconstructed(a, pw)
    C = illumination(cfg, prob.beams)
    K = exact.shape[1] * exact.shape[2]
    psi = exact.reshape(-1, K).T @ C.T
    psip = rec.reshape(-1, K).T @ C.T
    return float(np.linalg.norm(psip - psi) / np.linalg.norm(psi))


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))
