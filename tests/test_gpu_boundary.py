"""The C-ABI boundary on the GPU: device memory through the caller's
allocator (bip_alloc), the library's own stream-ordered pool when none is
given, device-side outputs of the potential helpers, and the autograd
wrappers (EELSMap, SlicePotential)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import eels as E
from paper_2607_00756_amd import specimen
from tests._tiny import as_oracle_problem, tiny_cfg, tiny_problem
from tests.gpu_helpers import rel_l2, torch_dev

pytestmark = pytest.mark.gpu


def _bip():
    from paper_2607_00756_amd import bip
    return bip


def _problem():
    cfg = tiny_cfg(ny=64, nx=64, nz=5, ly=16.0, lx=16.0, alpha=0.02, theta=0.03, s=2, scan=(5, 7))
    tp = tiny_problem(cfg, n_atoms=4, n_ch=2, W=8, seed=21, vscale=25.0, planes=[0, 4, 2, 1],
                      win_sizes=[8, 12, 16, 24])
    return cfg, tp


def test_every_plan_byte_comes_through_the_allocator():
    """A plan made with a counting torch-backed allocator: every block it
    holds (tables, parent columns, windows, checkpoints, workspaces of the
    signal and the backward) is one the allocator handed out, torch's own
    counter sees them, and destroying the plan gives every block back."""
    torch, dev = torch_dev()
    bip = _bip()
    cfg, tp = _problem()
    alloc = bip.TorchAllocator()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    plan = bip.Plan.from_config(cfg, tp.tau, tp.win_size, tp.win_origin, ckpt_stride=1,
                                allocator=alloc)
    V = torch.from_numpy(tp.V).to(dev)
    H = torch.from_numpy(tp.H).to(dev)
    P = cfg.scan[0] * cfg.scan[1]
    out = torch.empty(P, dtype=torch.float32, device=dev)
    plan.build_smatrix(V)
    for mode, shape in ((bip.OUT_MAP, (P,)), (bip.OUT_BEAMS, (P, plan.ndet))):
        o = torch.empty(shape, dtype=torch.float32, device=dev)
        plan.eels_signal(tp.n_ch, H, tp.H_off, cfg.scan, mode, bip.PREC_SPLIT_BF16, o)
    plan.eels_signal(tp.n_ch, H, tp.H_off, cfg.scan, bip.OUT_MAP, bip.PREC_FP32, out)
    dV = torch.empty_like(V)
    plan.eels_backward(tp.n_ch, H, tp.H_off, cfg.scan, torch.ones(P, device=dev), dV)
    torch.cuda.synchronize()
    now, peak, blocks = (int(v) for v in plan.query(bip.Q_MEMORY))
    print(f"[allocator] plan holds {now} B in {blocks} blocks (peak {peak}); "
          f"allocator live {alloc.live_bytes} B, {alloc.n_alloc} allocations")
    assert now > 0 and blocks == len(alloc.live) and now == alloc.live_bytes
    assert alloc.n_alloc >= blocks and alloc.failed == 0
    held = torch.cuda.memory_allocated() - base
    extra = V.numel() * 4 + H.numel() * 8 + 2 * out.numel() * 4 + dV.numel() * 4 + P * 4 * (1 + plan.ndet)
    assert now <= held <= now + extra + (1 << 22)
    plan.close()
    torch.cuda.synchronize()
    assert alloc.live_bytes == 0 and not alloc.live


def test_library_pool_without_allocator_matches():
    """allocator=None: the library takes its blocks from the stream-ordered HIP
    pool; the results equal those of a torch-allocator plan bitwise."""
    torch, dev = torch_dev()
    bip = _bip()
    cfg, tp = _problem()
    P = cfg.scan[0] * cfg.scan[1]
    res = []
    for allocator in ("torch", None):
        plan = bip.Plan.from_config(cfg, tp.tau, tp.win_size, tp.win_origin, allocator=allocator)
        plan.build_smatrix(torch.from_numpy(tp.V).to(dev))
        out = torch.empty(P, dtype=torch.float32, device=dev)
        plan.eels_signal(tp.n_ch, torch.from_numpy(tp.H).to(dev), tp.H_off, cfg.scan, bip.OUT_MAP,
                         bip.PREC_SPLIT_BF16, out)
        torch.cuda.synchronize()
        res.append(out.cpu().numpy())
        assert int(plan.query(bip.Q_MEMORY)[0]) > 0
        plan.close()
    assert np.array_equal(res[0], res[1])
    want = E.BiP(as_oracle_problem(tp)).run(mode=E.OUT_MAP)
    assert rel_l2(res[1], want) < 1e-4


def test_slice_potential_autograd_equals_potential_grad():
    """SlicePotential.apply(xyz).backward(g) returns bip_potential_grad of g
    (device FP64 output, no host round trip)."""
    torch, dev = torch_dev()
    bip = _bip()
    cfg = tiny_cfg(ny=64, nx=128, nz=4, ly=10.0, lx=20.0, dz=2.0)
    r = np.random.default_rng(5)
    n = 37
    xyz = np.stack([r.random(n) * cfg.lx, r.random(n) * cfg.ly, r.random(n) * cfg.nz * cfg.dz], 1)
    amps = np.abs(r.normal(size=(n, 4))) * 5.0
    widths = np.array(specimen.POT_WIDTHS)
    grid = bip.BipGrid(cfg.ny, cfg.nx, cfg.nz, cfg.ly, cfg.lx, cfg.dz)
    x = torch.tensor(xyz, dtype=torch.float64, requires_grad=True)
    V = bip.SlicePotential.apply(x, grid, amps, widths, (cfg.nz, cfg.ny, cfg.nx))
    g = torch.from_numpy(r.normal(size=(cfg.nz, cfg.ny, cfg.nx)).astype(np.float32)).to(dev)
    (V * g).sum().backward()
    want = bip.potential_grad(grid, xyz, amps, widths, g)
    torch.cuda.synchronize()
    assert x.grad.device == x.device
    assert torch.equal(x.grad, want.cpu())
    assert torch.all(x.grad[:, 2] == 0)


def test_eels_map_autograd_reuses_the_build_and_refuses_unsupported_precisions():
    """EELSMap.backward runs bip_eels_backward on the checkpoints of the
    forward's own build (no second sweep when V is unchanged), and a BF16 or
    FP16 forward, whose gradient the backward does not implement, raises."""
    torch, dev = torch_dev()
    bip = _bip()
    cfg, tp = _problem()
    plan = bip.Plan.from_config(cfg, tp.tau, tp.win_size, tp.win_origin, ckpt_stride=1)
    V = torch.from_numpy(tp.V).to(dev).requires_grad_(True)
    H = torch.from_numpy(tp.H).to(dev)
    for prec in (bip.PREC_BF16, bip.PREC_FP16):
        with pytest.raises(ValueError):
            bip.EELSMap.apply(V, H, plan, tp.n_ch, tp.H_off, cfg.scan, prec)
    builds = []
    orig = plan.build_smatrix
    plan.build_smatrix = lambda *a, **k: (builds.append(1), orig(*a, **k))[1]
    I = bip.EELSMap.apply(V, H, plan, tp.n_ch, tp.H_off, cfg.scan, bip.PREC_FP32)
    (I * I).sum().backward()
    assert len(builds) == 1  # the forward's build only
    dV = torch.empty_like(V)
    plan.build_smatrix = orig
    plan.eels_backward(tp.n_ch, H, tp.H_off, cfg.scan, (2.0 * I).detach(), dV)
    torch.cuda.synchronize()
    assert torch.equal(V.grad, dV)
    plan.close()
