"""Gradient of the map loss on the GPU (bip_eels_backward, potential helpers).

Parity with the FP64 oracle gradient (oracle/adjoint.py, itself pinned by
central differences) on ragged problems, both reconstruction modes, with and
without column batching of the reverse sweeps; and central differences of
the GPU's own forward map at the full size of the differentiation workload (256^2, 30 slices, 16 atoms x 3).
Both sides take the same dL/dI = 2 (I - I_t) from the oracle's map, so the
comparison isolates the backward.  Bar: rel-L2 <= 1e-3."""
from __future__ import annotations

import os

import numpy as np
import pytest

from oracle import adjoint as A
from oracle import eels as E
from oracle import potential as pot
from paper_2607_00756_amd import specimen
from tests._tiny import as_oracle_problem, tiny_cfg, tiny_problem
from tests.gpu_helpers import rel_l2, torch_dev

pytestmark = pytest.mark.gpu


def _bip():
    from paper_2607_00756_amd import bip
    return bip


def _ragged(s):
    cfg = tiny_cfg(ny=64, nx=64, nz=5, ly=16.0, lx=16.0, alpha=0.02, theta=0.03, s=s, scan=(5, 7))
    tp = tiny_problem(cfg, n_atoms=5, n_ch=2, W=8, seed=11, vscale=25.0, planes=[0, 4, 2, 2, 1],
                      win_sizes=[4, 12, 16, 24, 64])
    return cfg, tp


def _gpu_grad(cfg, tp, ibar, recon, dHx=None, dHy=None, batch=None, prec=0):
    torch, dev = torch_dev()
    bip = _bip()
    if batch is not None:
        os.environ["BIP_COLUMN_BATCH"] = str(batch)
    try:
        plan = bip.Plan.from_config(cfg, tp.tau, tp.win_size, tp.win_origin, recon_mode=recon,
                                    ckpt_stride=1)
        V = torch.from_numpy(np.ascontiguousarray(tp.V, np.float32)).to(dev)
        plan.build_smatrix(V)
    finally:
        os.environ.pop("BIP_COLUMN_BATCH", None)
    H = torch.from_numpy(np.ascontiguousarray(tp.H, np.complex64)).to(dev)
    dV = torch.empty_like(V)
    gH = torch.empty_like(H)
    dx = dy = None
    if dHx is not None:
        dx = torch.from_numpy(np.ascontiguousarray(dHx, np.complex64)).to(dev)
        dy = torch.from_numpy(np.ascontiguousarray(dHy, np.complex64)).to(dev)
    Ib = torch.from_numpy(np.ascontiguousarray(ibar, np.float32)).to(dev)
    tau = plan.eels_backward(tp.n_ch, H, tp.H_off, cfg.scan, Ib, dV, dL_dHconj=gH, dHdx=dx,
                             dHdy=dy, want_tau=dHx is not None, precision=prec)
    torch.cuda.synchronize()
    out = (dV.cpu().numpy().astype(np.float64), gH.cpu().numpy().astype(np.complex128),
           None if tau is None else tau.cpu().numpy())
    plan.close()
    return out


@pytest.mark.parametrize("s,recon,batch,prec", [(2, E.RECON_MAGNITUDE, None, 0), (1, E.RECON_MAGNITUDE, None, 0),
                                                (2, E.RECON_COMPLEX, None, 0), (3, E.RECON_MAGNITUDE, 7, 0),
                                                (2, E.RECON_MAGNITUDE, None, 1), (3, E.RECON_COMPLEX, 7, 1)])
def test_backward_matches_oracle_gradient(s, recon, batch, prec):
    """prec 0: FP32 products; 1: the split precision (FP16 Gram, hi+lo BF16)."""
    cfg, tp = _ragged(s)
    prob = as_oracle_problem(tp)
    r = np.random.default_rng(4)
    I0 = E.BiP(prob, recon).run(mode=E.OUT_MAP)
    It = I0 * (1.0 + 0.3 * r.normal(size=I0.shape))
    dHx = (r.normal(size=tp.H.shape) + 1j * r.normal(size=tp.H.shape))
    dHy = (r.normal(size=tp.H.shape) + 1j * r.normal(size=tp.H.shape))
    dH = {a: (dHx[tp.H_off[a]:tp.H_off[a + 1]].reshape(tp.n_ch, tp.win_size[a], tp.win_size[a]),
              dHy[tp.H_off[a]:tp.H_off[a + 1]].reshape(tp.n_ch, tp.win_size[a], tp.win_size[a]))
          for a in range(len(tp.tau))}
    print(f"[backward s={s} recon={recon} batch={batch} prec={prec}]", flush=True)
    ref = A.MapGradient(prob, recon).run(It, dH_dtau=dH)
    ibar = 2.0 * (ref["I"] - It)
    dV, gH, tau = _gpu_grad(cfg, tp, ibar, recon, dHx, dHy, batch, prec)
    e_v = rel_l2(dV, ref["dV"])
    gH_ref = np.concatenate([ref["gH"][a].ravel() for a in range(len(tp.tau))])
    e_h = float(np.linalg.norm(gH - gH_ref) / np.linalg.norm(gH_ref))
    tau_ref = np.array([ref["dtau"][a] for a in range(len(tp.tau))])
    e_t = rel_l2(tau, tau_ref)
    print(f"  dV {e_v:.2e}  dH {e_h:.2e}  dtau {e_t:.2e}")
    assert e_v < 1e-3 and e_h < 1e-3 and e_t < 1e-3


def test_potential_build_and_gradient_match_oracle():
    torch, dev = torch_dev()
    bip = _bip()
    cfg = tiny_cfg(ny=64, nx=128, nz=4, ly=10.0, lx=20.0, s=2, scan=(4, 4))
    r = np.random.default_rng(9)
    n = 40
    xyz = np.stack([r.random(n) * cfg.lx, r.random(n) * cfg.ly, r.random(n) * cfg.nz * cfg.dz], 1)
    widths = np.array(specimen.POT_WIDTHS)
    amps = np.abs(r.normal(size=(n, 4))) * 5.0
    grid = bip.BipGrid(cfg.ny, cfg.nx, cfg.nz, cfg.ly, cfg.lx, cfg.dz)
    V = torch.empty((cfg.nz, cfg.ny, cfg.nx), dtype=torch.float32, device=dev)
    bip.potential_build(grid, xyz, amps, widths, V)
    Vref = pot.projected_potential(cfg, xyz, amps, widths)
    e = rel_l2(V.cpu().numpy(), Vref)
    dV = r.normal(size=Vref.shape)
    g = bip.potential_grad(grid, xyz, amps, widths, torch.from_numpy(dV.astype(np.float32)).to(dev))
    g = g.cpu().numpy()
    gref = pot.potential_grad(cfg, xyz, amps, widths, dV.astype(np.float32).astype(np.float64))
    eg = rel_l2(g, gref)
    print(f"[potential] V {e:.2e} grad {eg:.2e}")
    assert e < 1e-6 and eg < 1e-9 and np.all(g[:, 2] == 0.0)


def test_autograd_function_matches_direct_backward():
    torch, dev = torch_dev()
    bip = _bip()
    cfg, tp = _ragged(2)
    plan = bip.Plan.from_config(cfg, tp.tau, tp.win_size, tp.win_origin, ckpt_stride=1)
    V = torch.from_numpy(tp.V).to(dev).requires_grad_(True)
    H = torch.from_numpy(tp.H).to(dev).requires_grad_(True)
    I = bip.EELSMap.apply(V, H, plan, tp.n_ch, tp.H_off, cfg.scan, bip.PREC_FP32)
    It = (I.detach() * 1.1).contiguous()
    L = ((I - It) ** 2).sum()
    L.backward()
    Ib = (2.0 * (I.detach() - It)).contiguous()
    dV = torch.empty_like(V)
    gH = torch.empty_like(H)
    plan.build_smatrix(V.detach())
    plan.eels_backward(tp.n_ch, H.detach(), tp.H_off, cfg.scan, Ib, dV, dL_dHconj=gH)
    torch.cuda.synchronize()
    assert torch.equal(V.grad, dV)
    assert torch.equal(H.grad, 2.0 * gH)
    plan.close()


@pytest.fixture(scope="module")
def c4():
    torch, dev = torch_dev()
    bip = _bip()
    sp = specimen.make(4)
    cfg = sp.cfg
    plan = bip.Plan.from_config(cfg, sp.tau, sp.win_size, sp.win_origin, ckpt_stride=1)
    H = torch.from_numpy(sp.H).to(dev)
    V0 = torch.from_numpy(sp.V).to(dev)
    P = cfg.scan[0] * cfg.scan[1]
    out = torch.empty(P, dtype=torch.float32, device=dev)

    def I_of(V):
        plan.build_smatrix(V)
        plan.eels_signal(sp.n_ch, H, sp.H_off, cfg.scan, bip.OUT_MAP, bip.PREC_FP32, out)
        return out.double().clone()

    I0 = I_of(V0)
    r = np.random.default_rng(1)
    It = I0 * torch.from_numpy(1.0 + 0.2 * r.normal(size=P)).to(dev)
    yield dict(sp=sp, cfg=cfg, plan=plan, H=H, V0=V0, I_of=I_of, It=It, r=r)
    plan.close()


def test_config4_slice_potential_gradient_central_differences(c4):
    """dL/dV of the full gradient configuration against central differences
    of the GPU map along smooth random directions (FP32 forward)."""
    torch, dev = torch_dev()
    cfg, plan, I_of, It, r = c4["cfg"], c4["plan"], c4["I_of"], c4["It"], c4["r"]
    sp, H, V0 = c4["sp"], c4["H"], c4["V0"]

    def L_of(V):
        return float(((I_of(V) - It) ** 2).sum())

    I0 = I_of(V0)
    dV = torch.empty_like(V0)
    plan.eels_backward(sp.n_ch, H, sp.H_off, cfg.scan, (2.0 * (I0 - It)).float().contiguous(), dV)
    torch.cuda.synchronize()
    assert torch.isfinite(dV).all()
    for k in range(3):
        # smooth direction: a few random Gaussians per slice
        d = np.zeros((cfg.nz, cfg.ny, cfg.nx))
        yy, xx = np.meshgrid(np.arange(cfg.ny), np.arange(cfg.nx), indexing="ij")
        for j in range(cfg.nz):
            for _ in range(3):
                cy, cx = r.random() * cfg.ny, r.random() * cfg.nx
                d[j] += np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * 12.0 ** 2))
        dt = torch.from_numpy(d.astype(np.float32)).to(dev)
        # a phase change of sigma * eps ~ 0.01 rad: well above FP32 rounding of the map,
        # well inside the linear range
        eps = 16.0
        fd = (L_of(V0 + eps * dt) - L_of(V0 - eps * dt)) / (2 * eps)
        an = float((dV.double() * dt.double()).sum())
        print(f"[c4 dV dir {k}] fd {fd:.6e} an {an:.6e}")
        assert abs(fd - an) <= 5e-3 * abs(fd)


def test_config4_position_gradient_central_differences(c4):
    """dL/d(x, y) of atoms of the gradient configuration through both paths.

    Moving one atom by a fraction of an angstrom changes the loss by about
    1e-5 of itself, which the float32 map cannot resolve, so each link of the
    chain is checked where central differences are well conditioned:
    * V path: the directional derivative of the GPU map along dV/dx_a (the
      potential change of the move, from two GPU potential builds), with a
      large step in V, equals sum dL/dV dV/dx_a, which bip_potential_grad
      returns (itself checked against the oracle);
    * H path: a central difference along dH/dtau (V fixed), with a step that
      moves H by a fraction of a percent, equals the returned dL/dtau."""
    torch, dev = torch_dev()
    bip = _bip()
    sp, cfg, plan, It = c4["sp"], c4["cfg"], c4["plan"], c4["It"]
    amps = np.array(specimen.POT_AMPS)[None, :] * np.where(sp.species == 1, cfg.species_b_scale, 1.0)[:, None]
    widths = np.array(specimen.POT_WIDTHS)
    grid = bip.BipGrid(cfg.ny, cfg.nx, cfg.nz, cfg.ly, cfg.lx, cfg.dz)
    forms = specimen._forms(cfg.channels)
    P = cfg.scan[0] * cfg.scan[1]
    out = torch.empty(P, dtype=torch.float32, device=dev)
    shape = (cfg.nz, cfg.ny, cfg.nx)

    def V_of(xyz):
        V = torch.empty(shape, dtype=torch.float32, device=dev)
        bip.potential_build(grid, xyz, amps, widths, V)
        return V

    def L_of(V, H):
        plan.build_smatrix(V.float().contiguous())
        plan.eels_signal(sp.n_ch, H, sp.H_off, cfg.scan, bip.OUT_MAP, bip.PREC_FP32, out)
        return float(((out.double() - It) ** 2).sum()), out.double().clone()

    xyz = sp.xyz.copy()
    parts, dxs, dys = [], [], []
    for k, a in enumerate(sp.ionized):
        h, hx, hy = specimen.transition_potentials(cfg, xyz[a], int(sp.win_size[k]),
                                                   tuple(sp.win_origin[k]), forms, with_grad=True)
        parts.append(h.ravel())
        dxs.append(hx.ravel())
        dys.append(hy.ravel())
    cat = lambda v: torch.from_numpy(np.concatenate(v).astype(np.complex64)).to(dev)
    H, dHx, dHy = cat(parts), cat(dxs), cat(dys)
    V0 = V_of(xyz)
    L0, I0 = L_of(V0, H)
    dV = torch.empty_like(V0)
    tau = plan.eels_backward(sp.n_ch, H, sp.H_off, cfg.scan, (2.0 * (I0 - It)).float().contiguous(), dV,
                             dHdx=dHx, dHdy=dHy, want_tau=True).cpu().numpy()
    g = bip.potential_grad(grid, xyz, amps, widths, dV).cpu().numpy()
    assert np.all(g[:, 2] == 0.0)
    ion = int(sp.ionized[0])
    d2 = np.sum((xyz[:, :2] - xyz[ion, :2]) ** 2, axis=1)
    d2[sp.ionized] = np.inf
    other = int(np.argmin(d2))
    hstep = 0.01
    for a in (other, ion):
        for c in (0, 1):
            xp, xm = xyz.copy(), xyz.copy()
            xp[a, c] += hstep
            xm[a, c] -= hstep
            dVdx = (V_of(xp).double() - V_of(xm).double()) / (2 * hstep)  # dV/dx_a
            chain = float((dV.double() * dVdx).sum())
            # dV/dx_a differenced from two float32 builds: ~0.2% rounding noise
            assert abs(chain - g[a, c]) <= 5e-3 * abs(g[a, c]), (a, c, chain, g[a, c])
            d = dVdx / dVdx.abs().max()
            # the float32 map rounds the loss to ~1e-7 of itself, which for the
            # smaller of these derivatives needs a step of several tens to sit
            # well under the tolerance; the O(eps^2) truncation stays below
            # 1e-3 up to a step of about 100
            eps = 64.0
            fd = (L_of(V0.double() + eps * d, H)[0] - L_of(V0.double() - eps * d, H)[0]) / (2 * eps)
            an = float((dV.double() * d).sum())
            print(f"[c4 V path atom {a} coord {c}] fd {fd:.6e} an {an:.6e}")
            assert abs(fd - an) <= 5e-3 * abs(fd)
    for k in range(len(sp.ionized)):
        for c, dH in ((0, dHx), (1, dHy)):
            sel = torch.zeros_like(H)
            sel[sp.H_off[k]:sp.H_off[k + 1]] = dH[sp.H_off[k]:sp.H_off[k + 1]]
            eps = 1e-3
            fd = (L_of(V0, H + eps * sel)[0] - L_of(V0, H - eps * sel)[0]) / (2 * eps)
            print(f"[c4 H path ionized {k} coord {c}] fd {fd:.6e} an {tau[k, c]:.6e}")
            # bounded on the scale of the gradient: small components sit at the
            # float32 rounding of the loss
            assert abs(fd - tau[k, c]) <= 1e-3 * max(abs(fd), np.abs(tau).max())


def test_backward_with_one_atom_per_workspace_chunk():
    """A workspace budget too small for two atoms runs the adjoint one atom at
    a time; dV and dL/dH agree with the default (one batch of all atoms)."""
    cfg, tp = _ragged(2)
    r = np.random.default_rng(9)
    ibar = r.normal(size=cfg.scan[0] * cfg.scan[1]) * 1e-3
    dV1, gH1, _ = _gpu_grad(cfg, tp, ibar, E.RECON_MAGNITUDE)
    os.environ["BIP_WORKSPACE_GB"] = "1e-9"
    try:
        dV2, gH2, _ = _gpu_grad(cfg, tp, ibar, E.RECON_MAGNITUDE)
    finally:
        os.environ.pop("BIP_WORKSPACE_GB", None)
    e1, e2 = rel_l2(dV2, dV1), rel_l2(gH2, gH1)
    print(f"[backward chunks] dV {e1:.2e} dH {e2:.2e}")
    assert e1 < 1e-5 and e2 < 1e-5


@pytest.mark.parametrize("stride", [2, 3, 7])
def test_recomputed_checkpoint_segments_match_slice_checkpoints(stride):
    """ckpt_stride k > 1 keeps every k-th slice and recomputes the others of a
    segment per column batch: dV, dL/dH and dL/dtau equal the slice-checkpoint
    gradient bitwise (same kernels on the same data), also with column
    batching, and match the FP64 oracle gradient."""
    cfg, tp = _ragged(2)
    r = np.random.default_rng(4)
    ibar = r.normal(size=cfg.scan[0] * cfg.scan[1]) * 1e-3
    prob = as_oracle_problem(tp)
    dHx = np.concatenate([r.normal(size=(tp.n_ch, w, w)).ravel() for w in tp.win_size]).astype(np.complex64)
    dHy = np.concatenate([r.normal(size=(tp.n_ch, w, w)).ravel() for w in tp.win_size]).astype(np.complex64)
    for batch in (None, 3):
        ref = _gpu_grad(cfg, tp, ibar, E.RECON_MAGNITUDE, dHx, dHy, batch=batch)
        got = _gpu_grad_stride(cfg, tp, ibar, E.RECON_MAGNITUDE, dHx, dHy, batch, stride)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), (stride, batch)
    # against the oracle gradient (the plan's map at the same dL/dI)
    It = E.BiP(prob).run(mode=E.OUT_MAP) - 0.5 * ibar
    want = A.MapGradient(prob).run(It)
    assert rel_l2(got[0], want["dV"]) < 1e-3


def _gpu_grad_stride(cfg, tp, ibar, recon, dHx, dHy, batch, stride):
    torch, dev = torch_dev()
    bip = _bip()
    if batch is not None:
        os.environ["BIP_COLUMN_BATCH"] = str(batch)
    try:
        plan = bip.Plan.from_config(cfg, tp.tau, tp.win_size, tp.win_origin, recon_mode=recon,
                                    ckpt_stride=stride)
        V = torch.from_numpy(np.ascontiguousarray(tp.V, np.float32)).to(dev)
        plan.build_smatrix(V)
    finally:
        os.environ.pop("BIP_COLUMN_BATCH", None)
    H = torch.from_numpy(np.ascontiguousarray(tp.H, np.complex64)).to(dev)
    dV = torch.empty_like(V)
    gH = torch.empty_like(H)
    dx = torch.from_numpy(dHx).to(dev)
    dy = torch.from_numpy(dHy).to(dev)
    Ib = torch.from_numpy(np.ascontiguousarray(ibar, np.float32)).to(dev)
    tau = plan.eels_backward(tp.n_ch, H, tp.H_off, cfg.scan, Ib, dV, dL_dHconj=gH, dHdx=dx, dHdy=dy,
                             want_tau=True)
    torch.cuda.synchronize()
    out = (dV.cpu().numpy().astype(np.float64), gH.cpu().numpy().astype(np.complex128), tau.cpu().numpy())
    plan.close()
    return out
