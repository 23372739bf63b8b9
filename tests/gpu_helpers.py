"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the FP64 oracle on identical inputs."""
from __future__ import annotations

import numpy as np


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


def make_plan(cfg, tau, win_size, win_origin, recon_mode=0):
    from paper_2607_00756_amd import bip
    return bip.Plan.from_config(cfg, tau, win_size, win_origin, recon_mode=recon_mode)


def gpu_run(cfg, V, tau, win_size, win_origin, H, H_off, n_ch, out_mode, precision,
            recon_mode=0, atom_subset=None, plan=None):
    """Build + signal on the GPU; returns (numpy output, plan)."""
    from paper_2607_00756_amd import bip
    torch, dev = torch_dev()
    if plan is None:
        plan = make_plan(cfg, tau, win_size, win_origin, recon_mode)
    Vd = torch.from_numpy(np.ascontiguousarray(V, np.float32)).to(dev)
    Hd = torch.from_numpy(np.ascontiguousarray(H, np.complex64)).to(dev)
    plan.build_smatrix(Vd)
    P = cfg.scan[0] * cfg.scan[1]
    shape = {bip.OUT_MAP: (P,), bip.OUT_MAP_DIRECT: (P,), bip.OUT_QEELS: (P, plan.nq),
             bip.OUT_BEAMS: (P, plan.ndet), bip.OUT_CUBE: (P, plan.ndet)}[out_mode]
    out = torch.empty(shape, dtype=torch.float32, device=dev)
    plan.eels_signal(n_ch, Hd, H_off, cfg.scan, out_mode, precision, out, atom_subset=atom_subset)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), plan


def rel_l2(x, ref):
    """||x - ref|| / ||ref|| over the whole array; complex inputs are compared
    as complex128 (real and imaginary parts both count)."""
    x, ref = np.asarray(x), np.asarray(ref)
    assert x.shape == ref.shape, (x.shape, ref.shape)
    dt = np.complex128 if (np.iscomplexobj(x) or np.iscomplexobj(ref)) else np.float64
    x, ref = x.astype(dt), ref.astype(dt)
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))
