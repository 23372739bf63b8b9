"""The FP64 oracle's map-loss gradient against central finite differences.

Pins the hand-written adjoint (oracle/adjoint.py, oracle/potential.py):
directional derivatives along random slice-potential and transition-potential
directions, and the gradient with respect to atom positions through both the
slice potentials and the transition potentials, each compared with a central
difference of the forward loss of Alg. 5.  dL/dz is zero because an atom's
potential lies wholly in its slice."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import adjoint as A
from oracle import eels as E
from oracle import potential as pot
from paper_2607_00756_amd import specimen
from tests._tiny import as_oracle_problem, tiny_cfg, tiny_problem


def _setup(s, mode, seed=3):
    cfg = tiny_cfg(ny=16, nx=16, nz=4, ly=4.0, lx=4.0, s=s, scan=(3, 5), alpha=0.03, theta=0.06)
    tp = tiny_problem(cfg, n_atoms=3, n_ch=2, W=6, seed=seed, vscale=20.0, planes=[1, 3, 1])
    prob = as_oracle_problem(tp)
    r = np.random.default_rng(seed + 100)
    I0 = E.BiP(prob, mode).run(mode=E.OUT_MAP)
    It = I0 * (1.0 + 0.3 * r.normal(size=I0.shape))
    return cfg, tp, prob, It, r


def _problem(cfg, tp, V=None, H=None):
    return E.Problem(cfg, tp.V if V is None else V, tp.tau, tp.win_size, tp.win_origin,
                     tp.H if H is None else H, tp.H_off, tp.n_ch)


@pytest.mark.parametrize("s,mode", [(1, E.RECON_MAGNITUDE), (2, E.RECON_MAGNITUDE),
                                    (2, E.RECON_COMPLEX)])
def test_slice_potential_gradient_matches_central_differences(s, mode):
    cfg, tp, prob, It, r = _setup(s, mode)
    g = A.MapGradient(prob, mode).run(It)
    assert abs(g["L"] - A.loss(prob, It, mode)) <= 1e-12 * g["L"]
    V0 = tp.V.astype(np.float64)
    for _ in range(4):
        d = r.normal(size=V0.shape)
        eps = 1e-4
        fd = (A.loss(_problem(cfg, tp, V=V0 + eps * d), It, mode) -
              A.loss(_problem(cfg, tp, V=V0 - eps * d), It, mode)) / (2 * eps)
        an = float(np.sum(g["dV"] * d))
        scale = float(np.sum(np.abs(g["dV"] * d)))  # size before cancellation
        assert abs(fd - an) <= 1e-6 * max(abs(fd), scale), (fd, an, scale)


@pytest.mark.parametrize("mode", [E.RECON_MAGNITUDE, E.RECON_COMPLEX])
def test_transition_potential_gradient_matches_central_differences(mode):
    cfg, tp, prob, It, r = _setup(2, mode)
    g = A.MapGradient(prob, mode).run(It)
    for a in range(len(tp.tau)):
        W = int(tp.win_size[a])
        d = r.normal(size=(tp.n_ch, W, W)) + 1j * r.normal(size=(tp.n_ch, W, W))

        def L_at(e):
            H = tp.H.astype(np.complex128)
            H[tp.H_off[a]:tp.H_off[a + 1]] += e * d.ravel()
            return A.loss(_problem(cfg, tp, H=H), It, mode)

        eps = 1e-5
        fd = (L_at(eps) - L_at(-eps)) / (2 * eps)
        an = 2.0 * float(np.real(np.sum(np.conj(g["gH"][a]) * d)))
        scale = 2.0 * float(np.sum(np.abs(g["gH"][a] * d)))
        assert abs(fd - an) <= 1e-7 * max(abs(fd), scale), (a, fd, an)


def _position_problem(xyz, cfg, amps, widths, ionized, W, origins, forms):
    """Problem whose V and H are built from the atom positions."""
    V = pot.projected_potential(cfg, xyz, amps, widths)
    H_parts, offs, dH = [], [0], {}
    for k, a in enumerate(ionized):
        Ha, dHx, dHy = specimen.transition_potentials(cfg, xyz[a], W, tuple(origins[k]), forms,
                                                      with_grad=True)
        H_parts.append(Ha.ravel())
        offs.append(offs[-1] + Ha.size)
        dH[k] = (dHx, dHy)
    prob = E.Problem(cfg, V, xyz[ionized], np.full(len(ionized), W), origins,
                     np.concatenate(H_parts), np.array(offs), len(forms))
    return prob, dH


def test_position_gradient_matches_central_differences():
    """dL/d(x, y) of every atom: through V for all atoms, plus through H for
    the ionized ones (windows held at the unperturbed origins)."""
    cfg = tiny_cfg(ny=32, nx=32, nz=4, ly=8.0, lx=8.0, s=2, scan=(4, 4), alpha=0.025, theta=0.05)
    r = np.random.default_rng(7)
    n = 6
    xyz = np.stack([r.random(n) * cfg.lx, r.random(n) * cfg.ly,
                    (r.integers(0, cfg.nz, n) + 0.3 + 0.4 * r.random(n)) * cfg.dz], 1)
    widths = np.array([0.3, 0.6])
    amps = np.abs(r.normal(size=(n, 2))) * 4.0 + 1.0
    ionized = [1, 4]
    W = 8
    forms = ["x", "y", "1"]
    origins = np.array([specimen.window_origin(xyz[a], W, cfg) for a in ionized], np.int32)
    prob, dH = _position_problem(xyz, cfg, amps, widths, ionized, W, origins, forms)
    It = E.BiP(prob).run(mode=E.OUT_MAP) * (1.0 + 0.2 * r.normal(size=cfg.scan[0] * cfg.scan[1]))
    g = A.MapGradient(prob).run(It, dH_dtau=dH)
    an = pot.potential_grad(cfg, xyz, amps, widths, g["dV"])
    for k, a in enumerate(ionized):
        an[a, 0] += g["dtau"][k][0]
        an[a, 1] += g["dtau"][k][1]

    def L_of(x):
        p, _ = _position_problem(x, cfg, amps, widths, ionized, W, origins, forms)
        return A.loss(p, It)

    h = 1e-4
    for a in range(n):
        for c in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[a, c] += h
            xm[a, c] -= h
            fd = (L_of(xp) - L_of(xm)) / (2 * h)
            if c == 2:
                assert fd == 0.0 and an[a, 2] == 0.0
            else:
                assert abs(fd - an[a, c]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(an).max()), (a, c, fd, an[a, c])


def test_oracle_potential_matches_the_input_generator():
    """Two independent evaluations of the same Gaussian-sum reading."""
    cfg = specimen.shrink(4, ny=64, nx=64, nz=3, lx=10.0, ly=10.0)
    r = np.random.default_rng(2)
    xyz = np.stack([r.random(5) * 10.0, r.random(5) * 10.0, r.random(5) * 6.0], 1)
    species = np.zeros(5, np.int32)
    ref = specimen.projected_potential(cfg, xyz, species)
    amps = np.tile(np.array(specimen.POT_AMPS, float), (5, 1))
    V = pot.projected_potential(cfg, xyz, amps, np.array(specimen.POT_WIDTHS))
    assert np.abs(V - ref).max() <= 1e-12 * np.abs(ref).max()
