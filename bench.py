"""Throughput of the BiP-PRISM EELS map on one MI355X.

    python bench.py [--steps K] [--warmup W] [--precision split|fp32|bf16|fp16] [--config 1]

One step is the whole hot path on the medium synthetic specimen (FCC a = 3.6 A
in a 40 x 40 x 100 A cell, 256^2 grid, 50 slices of 2 A, 300 keV, 25 mrad
convergence, 50 mrad collection, partition factor 4, 112 ionized atoms x 9
transition channels, 64 x 64 scan): parent multislice for S1 and S2 with the
window gathers (bip_build_smatrix), then windowed reconstruction and the
contraction into the elemental map (bip_eels_signal).  Inputs are resident in
HBM before the timed region.  The metric is scan positions x transitions per
second, one unit being one (scan position, atom, channel) triple.

Prints one JSON line.  It carries the roofline of the dominant kernel (device
time from HIP events recorded on the launch stream inside the timed region)
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "split": 2500.0, "bf16": 2500.0, "fp16": 2500.0}  # dense MFMA, MI355X
ALU_PEAK_TFLOPS = 157.3   # FP32 vector FMA, 256 CUs at 2.4 GHz
HBM_PEAK_GBS = 8000.0
PREC = {"fp32": 0, "split": 1, "bf16": 2, "fp16": 3}


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="split", choices=list(PREC))
    ap.add_argument("--config", type=int, default=1,
                    help="specimen (1: the benchmark workload; others for context)")
    ap.add_argument("--atoms", type=int, default=None,
                    help="only the first N ionized atoms of the specimen (context runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the timing of the map-loss gradient on the differentiation specimen")
    ap.add_argument("--grad-only", action="store_true",
                    help="only time the map-loss gradient and print its JSON object")
    ap.add_argument("--output", default="map", choices=["map", "qeels", "beams"],
                    help="output of the context run: the map (the benchmark), or the per-beam "
                         "intensities binned along q_x (qeels) or kept per beam (beams), both "
                         "through the per-beam detector contraction")
    ap.add_argument("--progress", action="store_true",
                    help="synchronize after every step and report it on stderr (long context runs)")
    ap.add_argument("--map-direct", action="store_true",
                    help="map through the per-beam detector contraction instead of the Gram form")
    ap.add_argument("--no-compare", dest="compare", action="store_false",
                    help="skip the other precisions (by default one step of each is timed and its "
                         "map compared with the benchmark precision's)")
    ap.add_argument("--column-batch", type=int, default=None,
                    help="parent columns per sweep batch (sets BIP_COLUMN_BATCH; 0 = all)")
    ap.add_argument("--atom-groups", type=int, default=0, metavar="K",
                    help="context run: split the ionized atoms into K groups, each with a plan of "
                         "its own that sweeps the parents once for its atoms (a workload whose "
                         "window stacks do not fit one plan), maps summed over the groups")
    ap.add_argument("--no-stage-events", action="store_true",
                    help="context runs: time the steps only (no second pass with HIP events around "
                         "every launch, so no per-stage times or rooflines in the output)")
    ap.add_argument("--no-fullmap", action="store_true",
                    help="skip the full-map workload leg (512^2, 100 slices, 2000 atoms x 3)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times and exit: the known "
                         "byte count that scales the FETCH_SIZE / WRITE_SIZE counters")
    return ap.parse_args()


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.mul(src, 1.0, out=dst)  # one read and one write of n floats
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": 4 * n, "bytes_written": 4 * n, "launches": 5,
                                           "kernel": "torch elementwise mul (out=)"}}))


def cpu_baseline(sp):
    """Time the FP64 oracle on a bounded sample of the same workload and
    extrapolate to the whole job (scan positions x transitions per second).

    Sample: (1) parent multislice (S1 to the deepest ionization plane, S2 from
    the exit to the shallowest) for every 40th parent column of each matrix;
    (2) windowed reconstruction plus probe-order contraction of one atom, all
    channels, on 1/16 of the scan positions, fed with random parent windows of
    the true shapes (timing only).  Full-job time = (1) x 40 + (2) x 16 x atoms."""
    from oracle import eels as E
    from oracle import multislice as ms
    cfg = sp.cfg
    prob = E.Problem.from_specimen(sp)
    bip = E.BiP(prob)
    planes = prob.planes
    step1 = 40
    p1 = bip.part1.parents[::step1]
    p2 = bip.part2.parents[::step1]
    t0 = time.perf_counter()
    ms.s1_at_planes(cfg, p1, prob.T, prob.P, [int(planes.max())])
    ms.s2_at_planes(cfg, p2, prob.T, prob.P, [int(planes.min())])
    t_sweep = (time.perf_counter() - t0) * step1
    rng = np.random.default_rng(0)
    a = 0
    W = int(sp.win_size[a])
    y, x = prob.window(a)
    w1 = rng.normal(size=(bip.part1.n_parents, W, W)) + 1j * rng.normal(size=(bip.part1.n_parents, W, W))
    w2 = rng.normal(size=(bip.part2.n_parents, W, W)) + 1j * rng.normal(size=(bip.part2.n_parents, W, W))
    C = E.illumination(cfg, prob.beams)
    step2 = 16
    t0 = time.perf_counter()
    s1 = E.reconstruct(cfg, w1, bip.part1.parents, bip.part1.W, prob.beams, y, x, 1)
    s2 = E.reconstruct(cfg, w2, bip.part2.parents, bip.part2.W, prob.det, y, x, 2)
    E.contract_probe_order(s1, s2, prob.H_atom(a), C[::step2])
    t_atom = (time.perf_counter() - t0) * step2
    n_atoms = len(sp.tau)
    t_full = t_sweep + t_atom * n_atoms
    units = cfg.scan[0] * cfg.scan[1] * n_atoms * sp.n_ch
    cores = int(os.environ.get("ORACLE_FFT_WORKERS", os.cpu_count() or 1))
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        blas = max([i.get("num_threads", 1) for i in info] + [1])
        cores = max(cores, blas)
    except Exception:
        pass
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": units / t_full, "unit": "scan-positions*transitions/s", "cores": cores,
        "cpu_model": model, "os_cpu_count": os.cpu_count(),
        "kind": "oracle",
        "sample": (f"FP64 oracle on config {cfg.name}: parent sweeps of every {step1}th S1/S2 parent "
                   f"({len(p1)}+{len(p2)} of {bip.part1.n_parents}+{bip.part2.n_parents} columns, all "
                   f"slices) x{step1}, plus reconstruction+contraction of 1 atom x {sp.n_ch} channels on "
                   f"1/{step2} of the scans x{step2} x {n_atoms} atoms; extrapolated full-job time "
                   f"{t_full:.0f} s"),
    }


def gradient_leg(steps, warmup):
    """Forward map + map-loss gradient (dL/dV and dL/dxyz of every atom) on the
    differentiation specimen: 256^2 grid, 30 slices, 200 keV, 20 mrad, s = 4,
    16 ionized atoms x 3 channels, scan 48 x 48.  One step is the potential
    build from the positions, the forward sweeps with slice checkpoints, the
    map, the backward (contraction, reconstruction and sweep adjoints) and the
    position gradient reduction, the contraction products in split precision;
    host wall time around synchronized steps."""
    import torch
    from paper_2607_00756_amd import bip, specimen

    dev = torch.device("cuda:0")
    sp = specimen.make(4)
    cfg = sp.cfg
    plan = bip.Plan.from_config(cfg, sp.tau, sp.win_size, sp.win_origin, ckpt_stride=1)
    grid = bip.BipGrid(cfg.ny, cfg.nx, cfg.nz, cfg.ly, cfg.lx, cfg.dz)
    amps = np.array(specimen.POT_AMPS)[None, :] * np.where(sp.species == 1, cfg.species_b_scale, 1.0)[:, None]
    widths = np.array(specimen.POT_WIDTHS)
    H = torch.from_numpy(sp.H).to(dev)
    P = cfg.scan[0] * cfg.scan[1]
    I = torch.empty(P, dtype=torch.float32, device=dev)
    V = torch.empty((cfg.nz, cfg.ny, cfg.nx), dtype=torch.float32, device=dev)
    dV = torch.empty_like(V)
    It = torch.from_numpy(np.random.default_rng(7).uniform(0.5, 1.5, P)).float().to(dev)
    marks = {}

    def step():
        bip.potential_build(grid, sp.xyz, amps, widths, V)
        plan.build_smatrix(V)
        plan.eels_signal(sp.n_ch, H, sp.H_off, cfg.scan, bip.OUT_MAP, bip.PREC_SPLIT_BF16, I)
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        marks["fwd"] = e
        plan.eels_backward(sp.n_ch, H, sp.H_off, cfg.scan, (2.0 * (I - It * I.mean())).contiguous(), dV,
                           precision=bip.PREC_SPLIT_BF16)
        return bip.potential_grad(grid, sp.xyz, amps, widths, dV)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    fwd_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e0.record()
        step()
        torch.cuda.synchronize()
        fwd_ms += e0.elapsed_time(marks["fwd"])
    ms = (time.perf_counter() - t0) * 1e3 / steps
    n_atoms = len(sp.tau)
    plan.close()
    return {"workload": f"{cfg.name}: FCC, {cfg.ny}^2 grid, {cfg.nz} slices, {cfg.energy_ev/1e3:.0f} keV, "
                        f"{cfg.alpha*1e3:.0f} mrad, s={cfg.partition}, {n_atoms} atoms x {sp.n_ch} channels, "
                        f"scan {cfg.scan[0]}x{cfg.scan[1]}, {len(sp.xyz)} atoms in the potential",
            "ms_per_gradient": ms, "ms_forward": fwd_ms / steps, "ms_backward": ms - fwd_ms / steps,
            "steps": steps, "precision": "split (FP16 Gram, hi+lo BF16 products)",
            "outputs": "dL/dV [nz, ny, nx] and dL/dxyz of every atom (FP64 potential reductions)"}


def full_map_leg(precision="split", steps=1, warmup=1):
    """The largest workload on one GPU: 80 x 80 x 200 A two-species FCC, 512^2
    grid, 100 slices, 300 keV, 30/60 mrad, s = 6, 2000 ionized atoms x 3
    channels with 24^2..64^2 windows, scan 128 x 128, map.  One plan: the S1
    windows of every atom stay resident, S2 is swept in plane segments inside
    the signal call (its windows of all atoms would take 187 GB).  Timed steps
    of build + signal after untimed warmups (HIP events on the stream)."""
    import torch
    from paper_2607_00756_amd import bip, specimen

    dev = torch.device("cuda:0")
    t_setup = time.perf_counter()
    log("full-map workload: building the specimen")
    sp = specimen.make(2)
    cfg = sp.cfg
    log("full-map workload: plan")
    plan = bip.Plan.from_config(cfg, sp.tau, sp.win_size, sp.win_origin)
    V = torch.from_numpy(sp.V).to(dev)
    H = torch.from_numpy(sp.H).to(dev)
    P = cfg.scan[0] * cfg.scan[1]
    out = torch.empty(P, dtype=torch.float32, device=dev)
    prec = PREC[precision]
    t_setup = time.perf_counter() - t_setup

    def step():
        plan.build_smatrix(V)
        plan.eels_signal(sp.n_ch, H, sp.H_off, cfg.scan, bip.OUT_MAP, prec, out)

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        log(f"full-map workload: warmup step {i + 1} done")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    sc = plan.query(bip.Q_SCALARS)
    mem = plan.query(bip.Q_MEMORY)
    units = P * len(sp.tau) * sp.n_ch
    res = {"workload": f"{cfg.name}: FCC two-species {cfg.lx:.0f}x{cfg.ly:.0f}x{cfg.lz_cell:.0f} A, "
                       f"{cfg.ny}^2 grid, {cfg.nz} slices, {cfg.energy_ev/1e3:.0f} keV, "
                       f"{cfg.alpha*1e3:.0f}/{cfg.theta*1e3:.0f} mrad, s={cfg.partition}, "
                       f"{len(sp.tau)} atoms x {sp.n_ch} channels (W 24..64), scan "
                       f"{cfg.scan[0]}x{cfg.scan[1]}, map",
           "value": units / (ms / 1e3), "unit": "scan-positions*transitions/s", "ms_per_step": ms,
           "steps": steps, "warmup": warmup, "precision": precision, "units_per_step": units,
           "B": plan.B, "n_det": plan.ndet, "Bp1": plan.Bp1, "Bp2": plan.Bp2,
           "s2_plane_segments": int(sc[3]), "plan_device_GB": float(mem[1]) / 1e9,
           "setup_s": t_setup, "map_sum": float(out.double().sum().item())}
    plan.close()
    return res


def prism_f_leg(precision="split", f=4, steps=3, warmup=1):
    """The medium workload at PRISM interpolation factor f (the paper's
    production setting; the benchmark itself is f = 1): aperture and detector
    beams on the f-lattice, each atom evaluated on the scans of its crop mask
    (P / f^2 of them).  Timed steps of build + signal (HIP events)."""
    import dataclasses
    import torch
    from paper_2607_00756_amd import bip, specimen

    dev = torch.device("cuda:0")
    sp = specimen.make(1)
    cfg = dataclasses.replace(sp.cfg, interp_f=f)
    plan = bip.Plan.from_config(cfg, sp.tau, sp.win_size, sp.win_origin)
    V = torch.from_numpy(sp.V).to(dev)
    H = torch.from_numpy(sp.H).to(dev)
    P = cfg.scan[0] * cfg.scan[1]
    out = torch.empty(P, dtype=torch.float32, device=dev)

    def step():
        plan.build_smatrix(V)
        plan.eels_signal(sp.n_ch, H, sp.H_off, cfg.scan, bip.OUT_MAP, PREC[precision], out)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    res = {"workload": f"{cfg.name} at interpolation factor f={f}: {len(sp.tau)} atoms x {sp.n_ch} "
                       f"channels, scan {cfg.scan[0]}x{cfg.scan[1]}, map; each atom on its crop mask "
                       f"({P // (f * f)} of {P} scans)",
           "ms_per_step": ms, "steps": steps, "precision": precision, "B": plan.B, "n_det": plan.ndet,
           "Bp1": plan.Bp1, "Bp2": plan.Bp2,
           "evaluated_units_per_s": P // (f * f) * len(sp.tau) * sp.n_ch / (ms / 1e3)}
    plan.close()
    return res


def measured_traffic(stage, column_batch):
    """HBM bytes per launch of the stage's kernel from the committed counter
    summary (FETCH_SIZE / WRITE_SIZE scaled by a copy of known size), or None
    when there is none for this stage, it was taken with another column
    batch, or the kernel's sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("stage") != stage or t.get("column_batch") != column_batch:
        return None
    for src, sha in t.get("sources_sha256", {}).items():
        p = os.path.join(ROOT, src)
        if not os.path.exists(p) or hashlib.sha256(open(p, "rb").read()).hexdigest() != sha:
            return None
    return float(t["bytes_per_launch"])


def atom_groups_run(args):
    """The whole ionized-atom set in K groups: per group a plan (created
    untimed), warmup steps, then timed steps of build + signal.  The job time
    is the sum of the groups' step times; the map is the sum of the groups'
    maps (the map is additive over atoms)."""
    import torch
    from paper_2607_00756_amd import bip, specimen

    dev = torch.device("cuda:0")
    sp = specimen.make(args.config, n_ionized=args.atoms)
    cfg = sp.cfg
    P = cfg.scan[0] * cfg.scan[1]
    V = torch.from_numpy(sp.V).to(dev)
    prec = PREC[args.precision]
    total = torch.zeros(P, dtype=torch.float64, device=dev)
    job_ms = 0.0
    groups = np.array_split(np.arange(len(sp.tau)), args.atom_groups)
    for gi, idx in enumerate(groups):
        offs = np.concatenate([[0], np.cumsum(sp.H_off[idx + 1] - sp.H_off[idx])]).astype(np.int64)
        Hg = np.concatenate([sp.H[sp.H_off[a]:sp.H_off[a + 1]] for a in idx])
        plan = bip.Plan.from_config(cfg, sp.tau[idx], sp.win_size[idx], sp.win_origin[idx])
        H = torch.from_numpy(Hg).to(dev)
        out = torch.empty(P, dtype=torch.float32, device=dev)

        def step():
            plan.build_smatrix(V)
            plan.eels_signal(sp.n_ch, H, offs, cfg.scan, bip.OUT_MAP, prec, out)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        job_ms += ms
        total += out.double()
        print(f"[group {gi + 1}/{len(groups)}] {len(idx)} atoms: {ms:.1f} ms per step", file=sys.stderr,
              flush=True)
        plan.close()
        del H, out
    units = P * len(sp.tau) * sp.n_ch
    print(json.dumps({
        "metric": "scan-positions*transitions/s (map)", "value": units / (job_ms / 1e3),
        "unit": "scan-positions*transitions/s", "ms_per_step": job_ms, "steps": args.steps,
        "warmup": args.warmup, "precision": args.precision,
        "config": {"workload": f"{cfg.name}: {len(sp.tau)} atoms x {sp.n_ch} channels in "
                               f"{len(groups)} groups of up to {max(len(g) for g in groups)}, "
                               f"{cfg.ny}^2 grid, {cfg.nz} slices, scan {cfg.scan[0]}x{cfg.scan[1]}",
                   "groups": len(groups)},
        "map_sum": float(total.sum().item())}))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.column_batch is not None:
        os.environ["BIP_COLUMN_BATCH"] = str(args.column_batch)
    if args.atom_groups:
        atom_groups_run(args)
        return
    if args.grad_only:
        print(json.dumps({"gradient": gradient_leg(args.steps, args.warmup)}))
        return
    import torch
    from paper_2607_00756_amd import bip, specimen

    dev = torch.device("cuda:0")
    sp = specimen.make(args.config, n_ionized=args.atoms)
    cfg = sp.cfg
    plan = bip.Plan.from_config(cfg, sp.tau, sp.win_size, sp.win_origin)
    V = torch.from_numpy(sp.V).to(dev)
    H = torch.from_numpy(sp.H).to(dev)
    P = cfg.scan[0] * cfg.scan[1]
    # per-beam contraction for the direct map and the per-beam outputs
    direct = args.map_direct or args.output != "map"
    out_mode = {"qeels": bip.OUT_QEELS, "beams": bip.OUT_BEAMS}.get(
        args.output, bip.OUT_MAP_DIRECT if args.map_direct else bip.OUT_MAP)
    out_shape = {"qeels": (P, plan.nq), "beams": (P, plan.ndet)}.get(args.output, (P,))
    out = torch.empty(out_shape, dtype=torch.float32, device=dev)
    prec = PREC[args.precision]

    n_done = [0]

    def step(p=prec, o=out):
        plan.build_smatrix(V)
        plan.eels_signal(sp.n_ch, H, sp.H_off, cfg.scan, out_mode, p, o)
        if args.progress:
            torch.cuda.synchronize()
            n_done[0] += 1
            print(f"[step {n_done[0]}] done", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the timed steps: no per-stage events inside
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    if args.no_stage_events:
        units = P * len(sp.tau) * sp.n_ch
        print(json.dumps({"metric": f"scan-positions*transitions/s ({args.output})", "value": units / (ms_step / 1e3),
                          "unit": "scan-positions*transitions/s", "ms_per_step": ms_step, "steps": args.steps,
                          "warmup": args.warmup, "precision": args.precision,
                          "config": {"workload": f"{cfg.name}: {len(sp.tau)} atoms x {sp.n_ch} channels, "
                                                 f"{cfg.ny}^2 grid, {cfg.nz} slices, scan {cfg.scan[0]}x{cfg.scan[1]}, "
                                                 f"{args.output}", "B": plan.B, "n_det": plan.ndet,
                                     "Bp1": plan.Bp1, "Bp2": plan.Bp2}}))
        plan.close()
        return
    # the same number of steps again with HIP events around every launch, on
    # the launch stream, for the per-stage times and the kernel rooflines
    plan.set_profiling(True)
    plan.stage_timings(reset=True)
    e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e2.record()
    for _ in range(args.steps):
        step()
    e3.record()
    torch.cuda.synchronize()
    ms_step_profiled = e2.elapsed_time(e3) / args.steps
    stages = plan.stage_timings(reset=True)
    plan.set_profiling(False)

    n_atoms = len(sp.tau)
    units = P * n_atoms * sp.n_ch
    value = units / (ms_step / 1e3)

    # algorithmic work per step of each timed stage: (amount, unit, bound, peak)
    W2 = sp.win_size.astype(np.float64) ** 2
    B, nd = plan.B, plan.ndet
    Sy, Sx = cfg.scan
    G = cfg.ny * cfg.nx
    # bytes per complex element of the S2~ operand: the Gram path stores it in
    # fp16 for the split precision
    if args.precision == "fp32":
        csz = 8
    elif args.precision == "split":
        csz = 8 if direct else 4
    else:
        csz = 4
    mfma_peak = PEAK_TFLOPS[args.precision]
    work = {
        # fold (fused S1~ reconstruction, not counted) + DFT over x, then DFT over y
        "probe_fold": (float(np.sum(8.0 * W2 * P * Sx)) / 1e12, "TFLOP/s", "alu", ALU_PEAK_TFLOPS),
        "probe_dft": (float(np.sum(8.0 * W2 * P * Sy)) / 1e12, "TFLOP/s", "alu", ALU_PEAK_TFLOPS),
        # S2~ written once in the operand planes, parent windows read once
        "recon": (float(np.sum(W2 * (nd * csz + plan.Bp2 * 8))) / 1e9, "GB/s", "hbm", HBM_PEAK_GBS),
    }
    if direct:
        work["det_gemm"] = (float(np.sum(8.0 * nd * W2 * P) * sp.n_ch) / 1e12, "TFLOP/s", "mfma", mfma_peak)
    else:
        work["gram_gemm"] = (float(np.sum(8.0 * W2 * W2 * nd)) / 1e12, "TFLOP/s", "mfma", mfma_peak)
        work["det_gemm"] = (float(np.sum(8.0 * W2 * W2 * P)) / 1e12, "TFLOP/s", "mfma", mfma_peak)
    # parent sweeps: every pass reads and writes the whole state of the columns
    # of its batch; launches_per_step / n_batches passes over all columns
    # algorithmic bytes of a slice step are 16 G per column (the state read once
    # and written once); a step runs as two passes (rows, then columns), so each
    # pass is credited with half of it, 8 G per column of its batch
    batch = int(plan.query(bip.Q_SCALARS)[2])
    for st, ncol in (("s1_row", plan.Bp1), ("s1_col", plan.Bp1), ("s2_row", plan.Bp2), ("s2_col", plan.Bp2)):
        n_batches = -(-ncol // batch)
        work[st] = (8.0 * G * ncol * stages[st][1] / args.steps / n_batches / 1e9, "GB/s", "hbm",
                    HBM_PEAK_GBS)
    names = {"probe_fold": "k_probe_fold_x (S1~ reconstruction + residue fold + DFT over x)",
             "probe_dft": "k_probe_y (DFT over y, operand store)",
             "recon": "k_recon_operand (S2~ reconstruction)",
             "gram_gemm": "k_zgemm Gram matrix + H correlation",
             "det_gemm": "k_zgemm detector contraction" if direct else "k_zgemm quadratic form",
             "s1_row": "k_row_pass (S1)", "s1_col": "k_col_pass (S1)",
             "s2_row": "k_row_pass (S2)", "s2_col": "k_col_pass (S2)"}
    dom = max(work, key=lambda k: stages[k][0])
    dom_ms, dom_n = stages[dom]
    launches_per_step = dom_n / args.steps
    amount, unit, bound, peak = work[dom]
    achieved = amount / launches_per_step / (dom_ms / dom_n / 1e3)
    traffic = measured_traffic(dom, batch)
    per_stage = {k: {"rate": (w[0] / (stages[k][0] / args.steps / 1e3) if stages[k][0] > 0 else None),
                     "unit": w[1], "bound": w[2], "frac": (w[0] / (stages[k][0] / args.steps / 1e3) / w[3]
                                                            if stages[k][0] > 0 else None)}
                 for k, w in work.items()}
    # multislice as a whole: algorithmic 16 G bytes per parent column per slice
    planes = plan.query(bip.Q_PLANES)
    col_slices = plan.Bp1 * int(planes.max()) + plan.Bp2 * (cfg.nz - int(planes.min()))
    ms_bytes = 16.0 * G * col_slices
    ms_time = sum(stages[k][0] for k in ("s1_row", "s1_col", "s2_row", "s2_col")) / args.steps
    res = {
        "metric": f"scan-positions*transitions/s ({args.output}, <=1e-4 rel-L2 vs FP64 oracle)",
        "value": value, "unit": "scan-positions*transitions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "c64 multislice + fp32 MFMA contraction",
                  "split": "c64 multislice + split MFMA contraction: bf16 hi/lo products, "
                           "Gram matrix on fp16 products from 4096 detector beams (f32 accumulate)",
                  "bf16": "c64 multislice + bf16 MFMA contraction (f32 accumulate)",
                  "fp16": "c64 multislice + fp16 MFMA contraction (f32 accumulate)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.lattice.upper()} {cfg.lx:.0f}x{cfg.ly:.0f}x{cfg.lz_cell:.0f} A, {cfg.ny}^2 grid, {cfg.nz} slices, "
                               f"{cfg.energy_ev/1e3:.0f} keV, {cfg.alpha*1e3:.0f}/{cfg.theta*1e3:.0f} mrad, "
                               f"s={cfg.partition}, {n_atoms} atoms x {sp.n_ch} channels, "
                               f"scan {cfg.scan[0]}x{cfg.scan[1]}, {args.output}",
                   "units_per_step": units, "B": plan.B, "n_det": plan.ndet, "Bp1": plan.Bp1,
                   "Bp2": plan.Bp2, "W": int(sp.win_size[0]), "precision": args.precision,
                   "map_contraction": "direct" if direct else "gram",
                   "column_batch": int(plan.query(bip.Q_SCALARS)[2])},
        "roofline": {"bound": bound, "kernel": names[dom], "stage": dom,
                     "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
                     "traffic": traffic, "traffic_unit": "bytes per launch (HBM, counters)",
                     "launches_per_step": launches_per_step,
                     "avg_launch_ms": dom_ms / dom_n,
                     "algorithmic_per_launch": amount / launches_per_step * (1e9 if unit == "GB/s" else 1e12),
                     # the rate of the bytes the counters saw move (both passes move the
                     # whole state), beside the algorithmic rate
                     "counter_rate": (traffic / (dom_ms / dom_n / 1e3) / 1e9 if traffic else None),
                     "counter_frac": (traffic / (dom_ms / dom_n / 1e3) / 1e9 / HBM_PEAK_GBS
                                      if traffic else None)},
        "stage_rooflines": per_stage,
        "stages_ms_per_step": {k: v[0] / args.steps for k, v in stages.items()},
        "ms_per_step_with_stage_events": ms_step_profiled,
        "multislice": {"algorithmic_GB": ms_bytes / 1e9, "ms_per_step": ms_time,
                       "achieved_GBs": ms_bytes / (ms_time / 1e3) / 1e9,
                       "frac_of_hbm": ms_bytes / (ms_time / 1e3) / 1e9 / HBM_PEAK_GBS},
        "wall_s": wall,
    }
    if args.compare:
        ref = out.clone()
        other = {}
        for name, pv in PREC.items():
            if pv == prec:
                continue
            o2 = torch.empty_like(out)
            step(pv, o2)  # warmup (the workspace of this precision)
            torch.cuda.synchronize()
            c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            n_cmp = 3
            c0.record()
            for _ in range(n_cmp):
                step(pv, o2)
            c1.record()
            torch.cuda.synchronize()
            other[name] = {"ms_per_step": c0.elapsed_time(c1) / n_cmp, "steps": n_cmp,
                           "rel_l2_vs_" + args.precision: float(torch.linalg.norm(o2 - ref) / torch.linalg.norm(ref))}
        res["other_precisions"] = other
    plan.close()
    del plan, V, H, out
    log(f"benchmark workload done: {ms_step:.2f} ms per step")
    if not args.no_grad:
        log("gradient leg")
        res["gradient"] = gradient_leg(args.steps, args.warmup)
    if not args.no_fullmap and args.config == 1 and args.atoms is None:
        log("interpolation-factor leg")
        res["prism_f4"] = prism_f_leg(args.precision)
        res["full_map_workload"] = full_map_leg(args.precision)
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        res["cpu_baseline"] = cpu_baseline(sp)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
