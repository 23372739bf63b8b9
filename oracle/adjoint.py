"""Gradient of an EELS map loss through BiP-PRISM (FP64).

Oracle (test infrastructure).  The loss is L = sum_rho (I(rho) - I_t(rho))^2
on the map of Alg. 5.  Its gradient is taken by hand, in reverse through the
forward steps:

* contraction (eq. coupling, eq. map-sum): a_nd(rho) = sum_r S2~^d(r) H_n(r)
  psi(r, rho), I = sum |a|^2;
* probe synthesis: psi(r, rho) = sum_b c_b(rho) S1~^b(r);
* windowed reconstruction (eq. window-recon, eq. magpreserve) and the
  de-tilt of the parent windows;
* the S1 sweep (psi_{j+1} = P(T_j psi_j), eq. smatrix-advance) and the S2
  transpose sweep (v_j = T_j P v_{j+1}, eq. s2), with the transmission
  T_j = exp(i sigma V_j).

Conventions.  For a complex quantity z the cotangent is the Wirtinger
derivative g_z = dL/d conj(z), so that dL = 2 Re sum conj(g_z) dz; for a
real quantity it is the ordinary derivative.  The position gradient of an
ionized atom through its transition potentials is 2 Re sum conj(g_H) dH/dtau
with dH/dtau supplied by the caller (the potentials are inputs).  The
position gradient through the slice potentials uses potential.py.

Only the map output is differentiated (the loss is defined on it).
"""
from __future__ import annotations

import math

import numpy as np

from . import eels as E
from . import multislice as ms
from . import physics


def _forward_states(cfg, parents_s1, parents_s2, T, P, i_max, i_min):
    """Forward sweeps keeping every state the backward needs.

    u1[j] = T_j psi_j (S1 after the transmission of slice j, j < i_max),
    psi1[j] = S1 at plane j (windows of atoms at plane j), v2[j] = S2 at
    plane j, i.e. after T_j (j >= i_min)."""
    nz = cfg.nz
    psi = ms.initial_s1(cfg, parents_s1)
    psi1, u1 = {0: psi}, {}
    for j in range(i_max):
        u1[j] = T[j] * psi
        psi = ms.ifft2(P * ms.fft2(u1[j]))
        psi1[j + 1] = psi
    v = ms.initial_s2(cfg, parents_s2)
    v2 = {}
    for j in range(nz - 1, i_min - 1, -1):
        v = ms.transpose_step(v, T[j], P)
        v2[j] = v
    return psi1, u1, v2


def _recon_forward(cfg, win, parents, Wmat, beams, y, x, side, mode):
    """Windowed reconstruction with the intermediates of its adjoint."""
    s = +1 if side == 1 else -1
    e = E.carrier(cfg, parents, y, x, -s)              # de-tilt carriers
    t = E.carrier(cfg, beams, y, x, +s)                # re-tilt carriers
    D = win * e
    Wd = Wmat.tocsr()
    K = D.shape[1] * D.shape[2]
    Df = D.reshape(D.shape[0], K)
    z = Wd @ Df
    if mode == E.RECON_COMPLEX:
        rec = z
        m = az = None
    else:
        m = Wd @ np.abs(Df)
        az = np.abs(z)
        sgn = np.where(az > 0, z / np.where(az > 0, az, 1.0), 0.0)
        rec = m * sgn
    out = rec.reshape(-1, D.shape[1], D.shape[2]) * t
    return out, dict(e=e, t=t, Df=Df, z=z, m=m, az=az, Wd=Wd)


def _recon_adjoint(g_out, st, mode):
    """Cotangent of the cropped parent columns (before de-tilt) from the
    cotangent of the reconstructed beams.

    s = m z/|z| (magnitude mode) or z (complex mode), out = s t.  With
    phi = z/|z| and g_s = conj(t) g_out:
      g_z = (m / (2|z|)) (g_s - conj(g_s) phi^2),  g_m = 2 Re(conj(g_s) phi),
    and through z = sum_p w D_p, m = sum_p w |D_p|:
      g_D_p = sum_b w_bp (g_z,b + (g_m,b / 2) D_p/|D_p|)."""
    Wd = st["Wd"]
    nb = g_out.shape[0]
    K = g_out.shape[1] * g_out.shape[2]
    g_s = (np.conj(st["t"]) * g_out).reshape(nb, K)
    Df = st["Df"]
    if mode == E.RECON_COMPLEX:
        g_D = Wd.T @ g_s
    else:
        z, m, az = st["z"], st["m"], st["az"]
        nz_ = az > 0
        phi = np.where(nz_, z / np.where(nz_, az, 1.0), 0.0)
        g_z = np.where(nz_, m / (2.0 * np.where(nz_, az, 1.0)), 0.0) * (g_s - np.conj(g_s) * phi * phi)
        half_gm = np.real(np.conj(g_s) * phi)
        aD = np.abs(Df)
        u = np.where(aD > 0, Df / np.where(aD > 0, aD, 1.0), 0.0)
        g_D = Wd.T @ g_z + (Wd.T @ half_gm) * u
    g_D = g_D.reshape(st["e"].shape)
    return np.conj(st["e"]) * g_D                      # undo the de-tilt


class MapGradient:
    """Map, loss and gradients of Alg. 5 for one specimen (FP64)."""

    def __init__(self, prob: E.Problem, recon_mode=E.RECON_MAGNITUDE):
        self.prob = prob
        self.bip = E.BiP(prob, recon_mode)
        self.mode = recon_mode

    def run(self, I_target, dH_dtau=None, atoms=None):
        """Returns dict(I, L, dV [nz, ny, nx], gH {atom: [n_ch, W, W]},
        dtau {atom: (dL/dx, dL/dy)} when dH_dtau = {atom: (dHx, dHy)})."""
        prob, bip, cfg = self.prob, self.bip, self.prob.cfg
        atoms = list(range(len(prob.tau))) if atoms is None else list(atoms)
        sigma = physics.interaction_constant(cfg.energy_ev)
        T, P = prob.T, prob.P
        planes = {a: int(prob.planes[a]) for a in atoms}
        i_max, i_min = max(planes.values()), min(planes.values())
        psi1, u1, v2 = _forward_states(cfg, bip.part1.parents, bip.part2.parents, T, P, i_max, i_min)
        C = E.illumination(cfg, prob.beams)                        # [P, B]
        Pn = C.shape[0]
        # ---- forward map with intermediates
        per = {}
        I = np.zeros(Pn)
        for a in atoms:
            i = planes[a]
            y, x = prob.window(a)
            w1 = psi1[i][:, y[:, None], x[None, :]]
            w2 = v2[i][:, y[:, None], x[None, :]]
            s1, st1 = _recon_forward(cfg, w1, bip.part1.parents, bip.part1.W, prob.beams, y, x, 1, self.mode)
            s2, st2 = _recon_forward(cfg, w2, bip.part2.parents, bip.part2.W, prob.det, y, x, 2, self.mode)
            K = s1.shape[1] * s1.shape[2]
            S1 = s1.reshape(-1, K)
            S2 = s2.reshape(-1, K)
            H = prob.H_atom(a).reshape(prob.n_ch, K)
            psi = S1.T @ C.T                                       # [K, P]
            amp = np.stack([S2 @ (H[n][:, None] * psi) for n in range(prob.n_ch)])  # [n, d, P]
            I += np.sum(amp.real ** 2 + amp.imag ** 2, axis=(0, 1))
            per[a] = (y, x, S1, S2, H, psi, st1, st2)   # amp is recomputed below (memory)
        L = float(np.sum((I - I_target) ** 2))
        Ibar = 2.0 * (I - I_target)                                # dL/dI
        # ---- contraction, probe and reconstruction adjoints per atom
        inj1 = {}   # plane -> cotangent of the S1 state at that plane [Bp1, ny, nx]
        inj2 = {}
        gH_all, dtau = {}, {}
        for a in atoms:
            y, x, S1, S2, H, psi, st1, st2 = per[a]
            per[a] = None
            amp = np.stack([S2 @ (H[n][:, None] * psi) for n in range(prob.n_ch)])  # as above
            W = len(y)
            g_amp = Ibar[None, None, :] * amp                      # dL/d conj(a)
            g_psi = np.zeros_like(psi)
            g_S2 = np.zeros_like(S2)
            g_H = np.zeros_like(H)
            for n in range(prob.n_ch):
                u = H[n][:, None] * psi                            # [K, P]
                g_u = np.conj(S2).T @ g_amp[n]                     # [K, P]
                g_S2 += g_amp[n] @ np.conj(u).T                    # [d, K]
                g_psi += np.conj(H[n])[:, None] * g_u
                g_H[n] = np.sum(np.conj(psi) * g_u, axis=1)
            gH_all[a] = g_H.reshape(prob.n_ch, W, W)
            if dH_dtau is not None and a in dH_dtau:
                dHx, dHy = dH_dtau[a]
                dtau[a] = (2.0 * float(np.real(np.sum(np.conj(gH_all[a]) * dHx))),
                           2.0 * float(np.real(np.sum(np.conj(gH_all[a]) * dHy))))
            g_S1 = (np.conj(C).T @ g_psi.T)                        # [B, K]
            g_w1 = _recon_adjoint(g_S1.reshape(-1, W, W), st1, self.mode)
            g_w2 = _recon_adjoint(g_S2.reshape(-1, W, W), st2, self.mode)
            i = planes[a]
            for inj, g_w, n_par in ((inj1, g_w1, len(bip.part1.parents)),
                                    (inj2, g_w2, len(bip.part2.parents))):
                buf = inj.setdefault(i, np.zeros((n_par, cfg.ny, cfg.nx), np.complex128))
                np.add.at(buf, (slice(None), y[:, None], x[None, :]), g_w)
        # ---- S1 sweep adjoint: psi_{j+1} = P(u_j), u_j = T_j psi_j
        dV = np.zeros((cfg.nz, cfg.ny, cfg.nx))
        Pc = np.conj(P)
        lam = inj1.get(i_max, 0.0) * np.ones_like(psi1[0])
        for j in range(i_max - 1, -1, -1):
            ubar = ms.ifft2(Pc * ms.fft2(lam))                     # cotangent of u_j
            dV[j] += np.sum(2.0 * np.real(np.conj(ubar) * 1j * sigma * u1[j]), axis=0)
            lam = np.conj(T[j]) * ubar
            if j in inj1:
                lam = lam + inj1[j]
        # ---- S2 sweep adjoint: v_j = T_j P v_{j+1}
        lam = inj2.get(i_min, 0.0) * np.ones_like(v2[i_min])
        for j in range(i_min, cfg.nz):
            dV[j] += np.sum(2.0 * np.real(np.conj(lam) * 1j * sigma * v2[j]), axis=0)
            if j + 1 < cfg.nz:
                lam = ms.ifft2(Pc * ms.fft2(np.conj(T[j]) * lam))
                if j + 1 in inj2:
                    lam = lam + inj2[j + 1]
        return dict(I=I, L=L, dV=dV, gH=gH_all, dtau=dtau)


def loss(prob: E.Problem, I_target, recon_mode=E.RECON_MAGNITUDE, atoms=None):
    """L = sum (I - I_t)^2 from the forward map of Alg. 5."""
    I = E.BiP(prob, recon_mode).run(mode=E.OUT_MAP, atoms=atoms)
    return float(np.sum((I - I_target) ** 2))
