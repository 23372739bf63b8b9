"""Thin Python binding of libbip.so (include/bip.h): argument marshalling only.

Device buffers are torch tensors on the current HIP device; the stream is
torch's current stream.  Every computation runs in the HIP library; if the
library is missing this module raises at import.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch first: its bundled HIP runtime (SONAME libamdhip64.so.7) must be the one
# libbip.so binds to, so that the process holds a single HIP/HSA runtime.
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libbip.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2607_00756_amd.build`")
_lib = ctypes.CDLL(_LIB_PATH)

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ESTATE = 0, -1, -2, -3, -4, -5
RECON_MAGNITUDE, RECON_COMPLEX = 0, 1
PARENTS_LATTICE, PARENTS_HEX = 0, 1
OUT_MAP, OUT_QEELS, OUT_BEAMS, OUT_MAP_DIRECT, OUT_CUBE = 0, 1, 2, 3, 4
PREC_FP32, PREC_SPLIT_BF16, PREC_BF16, PREC_FP16 = 0, 1, 2, 3
Q_COUNTS, Q_BEAMS, Q_DETECTOR, Q_PARENTS1, Q_PARENTS2, Q_PLANES, Q_WEIGHTS1, Q_WEIGHTS2, \
    Q_SCALARS, Q_MEMORY = range(10)

EXPORTS = ["bip_plan_create", "bip_build_smatrix", "bip_reconstruct_local", "bip_eels_signal",
           "bip_parent_windows", "bip_query", "bip_set_profiling", "bip_stage_timings",
           "bip_eels_backward", "bip_potential_build", "bip_potential_grad",
           "bip_plan_destroy", "bip_last_error", "bip_eels_signal_noalloc", "bip_eels_signal_edges",
           "bip_noalloc_scratch_bytes"]
STAGES = ["transmit", "s1_row", "s1_col", "s2_row", "s2_col", "init", "recon", "probe_fold",
          "probe_dft", "det_gemm", "reduce", "gram_gemm"]


class BipGrid(ctypes.Structure):
    _fields_ = [("ny", ctypes.c_int32), ("nx", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("ly", ctypes.c_double), ("lx", ctypes.c_double), ("dz", ctypes.c_double)]


class BipOptics(ctypes.Structure):
    _fields_ = [("energy_ev", ctypes.c_double), ("alpha_rad", ctypes.c_double),
                ("theta_rad", ctypes.c_double), ("partition", ctypes.c_int32),
                ("recon_mode", ctypes.c_int32), ("ckpt_stride", ctypes.c_int32),
                ("s2_window_gb", ctypes.c_double), ("parent_set", ctypes.c_int32),
                ("n_radial", ctypes.c_int32), ("n_angular", ctypes.c_int32), ("focal", ctypes.c_int32),
                ("s2_exact", ctypes.c_int32),
                ("interp_f", ctypes.c_int32)]


class BipEdge(ctypes.Structure):
    _fields_ = [("n_ch", ctypes.c_int32), ("H", ctypes.c_void_p), ("H_off", ctypes.c_void_p),
                ("atom_subset", ctypes.c_void_p), ("n_subset", ctypes.c_int32),
                ("out", ctypes.c_void_p)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class BipAlloc(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("release", _RELEASE_FN), ("ctx", ctypes.c_void_p)]


class TorchAllocator:
    """bip_alloc callbacks served by torch's caching allocator on the current
    device, in the order of the stream the library passes.  Counts what goes
    through it (live bytes and blocks, total allocations)."""

    def __init__(self):
        self.device = None  # the current device at the first allocation
        self.live = {}
        self.n_alloc = 0
        self.failed = 0

        def _alloc(nbytes, stream, ctx):
            try:
                if self.device is None:
                    self.device = torch.cuda.current_device()
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0))
            except Exception:  # out of memory: the library returns BIP_ENOMEM
                self.failed += 1
                return None
            self.live[ptr] = int(nbytes)
            self.n_alloc += 1
            return ptr

        def _release(ptr, nbytes, stream, ctx):
            try:
                if ptr:
                    self.live.pop(ptr, None)
                    torch.cuda.caching_allocator_delete(ptr)
            except Exception:  # interpreter shutdown: torch may be gone already
                pass

        self._fns = (_ALLOC_FN(_alloc), _RELEASE_FN(_release))  # kept alive with the object
        self.struct = BipAlloc(self._fns[0], self._fns[1], None)

    @property
    def live_bytes(self):
        return sum(self.live.values())


_default_allocator = None


def default_allocator():
    """One TorchAllocator per process (plans and potential helpers share it)."""
    global _default_allocator
    if _default_allocator is None:
        _default_allocator = TorchAllocator()
    return _default_allocator


def _alloc_arg(allocator):
    """"torch" (default) -> the shared TorchAllocator; None -> the library's own
    stream-ordered HIP pool; or a TorchAllocator instance."""
    if allocator == "torch":
        allocator = default_allocator()
    if allocator is None:
        return None, None
    return allocator, ctypes.byref(allocator.struct)


_p = ctypes.c_void_p
_lib.bip_plan_create.argtypes = [ctypes.POINTER(BipGrid), ctypes.POINTER(BipOptics), ctypes.c_int32,
                                 _p, _p, _p, _p, _p, ctypes.POINTER(_p)]
_lib.bip_build_smatrix.argtypes = [_p, _p, _p]
_lib.bip_reconstruct_local.argtypes = [_p, ctypes.c_int32, _p, _p, _p]
_lib.bip_eels_signal.argtypes = [_p, ctypes.c_int32, _p, _p, _p, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _p, _p]
_lib.bip_eels_signal_edges.argtypes = [_p, ctypes.c_int32, _p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, _p]
_lib.bip_eels_signal_edges.restype = ctypes.c_int
_lib.bip_eels_signal_noalloc.argtypes = _lib.bip_eels_signal.argtypes
_lib.bip_eels_signal_noalloc.restype = ctypes.c_int
_lib.bip_noalloc_scratch_bytes.argtypes = []
_lib.bip_noalloc_scratch_bytes.restype = ctypes.c_size_t
_lib.bip_parent_windows.argtypes = [_p, ctypes.c_int32, ctypes.c_int32, _p, _p]
_lib.bip_query.argtypes = [_p, ctypes.c_int32, _p]
_lib.bip_set_profiling.argtypes = [_p, ctypes.c_int32]
_lib.bip_stage_timings.argtypes = [_p, _p, _p, ctypes.c_int32]
_lib.bip_eels_backward.argtypes = [_p, ctypes.c_int32, _p, _p, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, _p, _p, _p, _p, _p, _p, _p]
_lib.bip_potential_build.argtypes = [ctypes.POINTER(BipGrid), ctypes.c_int32, _p, ctypes.c_int32,
                                     _p, _p, _p, _p, _p]
_lib.bip_potential_grad.argtypes = [ctypes.POINTER(BipGrid), ctypes.c_int32, _p, ctypes.c_int32,
                                    _p, _p, _p, _p, _p, _p]
_lib.bip_plan_destroy.argtypes = [_p]
_lib.bip_plan_destroy.restype = None
_lib.bip_last_error.restype = ctypes.c_char_p
for _f in EXPORTS[:11]:
    getattr(_lib, _f).restype = ctypes.c_int


class BipError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bip error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise BipError(rc, _lib.bip_last_error().decode())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


class Plan:
    """A bip_plan: geometry, parents, Sibson weights and device workspace."""

    def __init__(self, ny, nx, nz, ly, lx, dz, energy_ev, alpha, theta, partition, tau_xyz,
                 win_size, win_origin, recon_mode=RECON_MAGNITUDE, ckpt_stride=0, stream=None,
                 allocator="torch", s2_window_gb=0.0, parents="lattice", n_radial=4, n_angular=6,
                 focal=False, s2_exact=False, interp_f=1):
        self._h = _p()
        self._built_key = None
        self.allocator, alloc_ref = _alloc_arg(allocator)
        grid = BipGrid(ny, nx, nz, ly, lx, dz)
        self.grid = grid
        opt = BipOptics(energy_ev, alpha, theta, partition, recon_mode, ckpt_stride, s2_window_gb,
                        {"lattice": PARENTS_LATTICE, "hex": PARENTS_HEX}[parents], n_radial, n_angular,
                        1 if focal else 0, 1 if s2_exact else 0, int(interp_f))
        tau, tp = _host(tau_xyz, np.float64)
        ws, wp = _host(win_size, np.int32)
        wo, op = _host(win_origin, np.int32)
        _check(_lib.bip_plan_create(ctypes.byref(grid), ctypes.byref(opt), int(tau.shape[0]), tp,
                                    wp, op, alloc_ref, _stream(stream), ctypes.byref(self._h)))
        self.ny, self.nx, self.nz = ny, nx, nz
        self.win_size = ws.copy()
        c = self.query(Q_COUNTS)
        self.B, self.ndet, self.Bp1, self.Bp2, self.nq, self.n_atoms, self.nnz1, self.nnz2 = \
            (int(v) for v in c)

    @classmethod
    def from_config(cls, cfg, tau, win_size, win_origin, **kw):
        kw.setdefault("parents", getattr(cfg, "parents", "lattice"))
        kw.setdefault("n_radial", getattr(cfg, "n_radial", 4))
        kw.setdefault("n_angular", getattr(cfg, "n_angular", 6))
        kw.setdefault("focal", bool(getattr(cfg, "focal", False)))
        kw.setdefault("s2_exact", bool(getattr(cfg, "s2_exact", False)))
        kw.setdefault("interp_f", int(getattr(cfg, "interp_f", 1)))
        return cls(cfg.ny, cfg.nx, cfg.nz, cfg.ly, cfg.lx, cfg.dz, cfg.energy_ev, cfg.alpha,
                   cfg.theta, cfg.partition, tau, win_size, win_origin, **kw)

    def close(self):
        if self._h:
            _lib.bip_plan_destroy(self._h)
            self._h = _p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- entry points
    def build_smatrix(self, V, stream=None):
        """V: float32 device tensor [nz, ny, nx]."""
        assert V.is_contiguous() and V.dtype.itemsize == 4
        self._built_key = None
        _check(_lib.bip_build_smatrix(self._h, _ptr(V), _stream(stream)))
        self._built_key = _tensor_key(V)

    def built_from(self, V):
        """True when the last build_smatrix read this very tensor, unmodified."""
        return self._built_key is not None and self._built_key == _tensor_key(V)

    def reconstruct_local(self, atom, s1_out=None, s2_out=None, stream=None):
        """s1_out: complex64 [B, W, W]; s2_out: complex64 [n_det, W, W] (device)."""
        _check(_lib.bip_reconstruct_local(self._h, atom, _ptr(s1_out), _ptr(s2_out), _stream(stream)))

    def parent_windows(self, atom, which, out, stream=None):
        _check(_lib.bip_parent_windows(self._h, atom, which, _ptr(out), _stream(stream)))

    def eels_signal(self, n_ch, H, H_off, scan, out_mode, precision, out, atom_subset=None,
                    stream=None, noalloc=False):
        """H: complex64 device [ragged]; H_off: host int64 [n_atoms+1].
        noalloc=True calls bip_eels_signal_noalloc (fixed workspace, no allocation)."""
        offs, op = _host(H_off, np.int64)
        if atom_subset is None:
            sp, ns = ctypes.c_void_p(0), 0
        else:
            sub, sp = _host(atom_subset, np.int32)
            ns = int(sub.size)
        fn = _lib.bip_eels_signal_noalloc if noalloc else _lib.bip_eels_signal
        _check(fn(self._h, int(n_ch), _ptr(H), op, sp, ns, int(scan[0]), int(scan[1]), int(out_mode),
                  int(precision), _ptr(out), _stream(stream)))

    def eels_signal_edges(self, edges, scan, out_mode, precision, accumulate=False, weight=1.0,
                          stream=None):
        """Several edges in one call: edges = [(n_ch, H, H_off, atom_subset or None, out), ...];
        out = weight x signal, or out += weight x signal with accumulate."""
        keep = []
        arr = (BipEdge * len(edges))()
        for i, (n_ch, H, H_off, subset, out) in enumerate(edges):
            offs, op = _host(H_off, np.int64)
            keep.append(offs)
            if subset is None:
                sp, ns = None, 0
            else:
                sub, sp = _host(subset, np.int32)
                keep.append(sub)
                ns = int(sub.size)
            arr[i] = BipEdge(int(n_ch), H.data_ptr(), op, sp, ns, out.data_ptr())
        _check(_lib.bip_eels_signal_edges(self._h, len(edges), arr, int(scan[0]), int(scan[1]),
                                          int(out_mode), int(precision), 1 if accumulate else 0,
                                          float(weight), _stream(stream)))

    def eels_backward(self, n_ch, H, H_off, scan, dL_dI, dL_dV, dL_dHconj=None, dHdx=None,
                      dHdy=None, want_tau=False, precision=PREC_FP32, stream=None):
        """Gradient of a map loss (plan made with ckpt_stride >= 1, after build_smatrix).
        dL_dI: float32 device [P]; dL_dV: float32 device [nz, ny, nx] (written);
        dL_dHconj / dHdx / dHdy: complex64 device, ragged like H, or None;
        precision: PREC_FP32 or PREC_SPLIT_BF16 for the contraction products.
        Returns dL/dtau_xy [n_atoms, 2] (float64 device tensor) when want_tau, else None."""
        offs, op = _host(H_off, np.int64)
        tau = torch.empty((self.n_atoms, 2), dtype=torch.float64, device=dL_dV.device) \
            if want_tau else None
        _check(_lib.bip_eels_backward(self._h, int(n_ch), _ptr(H), op, int(scan[0]), int(scan[1]),
                                      int(precision), _ptr(dL_dI), _ptr(dL_dV), _ptr(dL_dHconj),
                                      _ptr(dHdx), _ptr(dHdy), _ptr(tau), _stream(stream)))
        return tau

    def set_profiling(self, enable):
        _check(_lib.bip_set_profiling(self._h, 1 if enable else 0))

    def stage_timings(self, reset=True):
        """{stage: (total ms, launches)} accumulated while profiling was on."""
        ms = np.zeros(len(STAGES), np.float64)
        n = np.zeros(len(STAGES), np.int64)
        _check(_lib.bip_stage_timings(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                      n.ctypes.data_as(ctypes.c_void_p), 1 if reset else 0))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(STAGES)}

    # ------------------------------------------------------------------- query
    def query(self, what):
        if what == Q_COUNTS:
            buf = np.zeros(8, np.int64)
        elif what in (Q_BEAMS, Q_DETECTOR, Q_PARENTS1, Q_PARENTS2):
            n = {Q_BEAMS: self.B, Q_DETECTOR: self.ndet, Q_PARENTS1: self.Bp1,
                 Q_PARENTS2: self.Bp2}[what]
            buf = np.zeros((n, 2), np.int32)
        elif what == Q_PLANES:
            buf = np.zeros(self.n_atoms, np.int32)
        elif what in (Q_WEIGHTS1, Q_WEIGHTS2):
            nb, nnz = (self.B, self.nnz1) if what == Q_WEIGHTS1 else (self.ndet, self.nnz2)
            raw = np.zeros(4 * (nb + 1) + 4 * nnz + 8 * nnz + 8, np.uint8)
            _check(_lib.bip_query(self._h, what, raw.ctypes.data_as(ctypes.c_void_p)))
            rp = raw[:4 * (nb + 1)].view(np.int32)
            col = raw[4 * (nb + 1):4 * (nb + 1) + 4 * nnz].view(np.int32)
            w = raw[4 * (nb + 1) + 4 * nnz:4 * (nb + 1) + 12 * nnz].view(np.float64)
            return rp.copy(), col.copy(), w.copy()
        elif what == Q_SCALARS:
            buf = np.zeros(4, np.float64)
        elif what == Q_MEMORY:
            buf = np.zeros(3, np.int64)
        else:
            raise ValueError(what)
        _check(_lib.bip_query(self._h, what, buf.ctypes.data_as(ctypes.c_void_p)))
        return buf


def _tensor_key(t):
    return (t.data_ptr(), t._version, tuple(t.shape), t.dtype)


def potential_build(grid, xyz, amp, width, V, stream=None, allocator="torch"):
    """Slice potentials V (float32 device [nz, ny, nx]) from atom positions
    xyz [n, 3], amplitudes amp [n, K] and widths [K] (host arrays)."""
    x, xp = _host(xyz, np.float64)
    a, ap = _host(amp, np.float64)
    w, wp = _host(width, np.float64)
    _, alloc_ref = _alloc_arg(allocator)
    _check(_lib.bip_potential_build(ctypes.byref(grid), int(x.shape[0]), xp, int(w.size), ap, wp,
                                    _ptr(V), alloc_ref, _stream(stream)))


def potential_grad(grid, xyz, amp, width, dL_dV, out=None, stream=None, allocator="torch"):
    """dL/dxyz [n, 3] (float64 device tensor, written into `out` when given)
    from dL/dV (float32 device)."""
    x, xp = _host(xyz, np.float64)
    a, ap = _host(amp, np.float64)
    w, wp = _host(width, np.float64)
    if out is None:
        out = torch.empty((x.shape[0], 3), dtype=torch.float64, device=dL_dV.device)
    assert out.is_contiguous() and out.dtype == torch.float64 and out.numel() == 3 * x.shape[0]
    _, alloc_ref = _alloc_arg(allocator)
    _check(_lib.bip_potential_grad(ctypes.byref(grid), int(x.shape[0]), xp, int(w.size), ap, wp,
                                   _ptr(dL_dV), _ptr(out), alloc_ref, _stream(stream)))
    return out


class EELSMap(torch.autograd.Function):
    """I = map(V, H) through bip_build_smatrix + bip_eels_signal; backward
    through bip_eels_backward.  The plan must be made with ckpt_stride >= 1.
    Gradients follow torch's complex convention (2 dL/d conj(H) for H)."""

    @staticmethod
    def forward(ctx, V, H, plan, n_ch, H_off, scan, precision):
        if precision not in (PREC_FP32, PREC_SPLIT_BF16):
            # the backward implements the FP32 and split products only; another
            # forward precision would return the gradient of a different map
            raise ValueError("EELSMap supports PREC_FP32 and PREC_SPLIT_BF16")
        P = int(scan[0]) * int(scan[1])
        out = torch.empty(P, dtype=torch.float32, device=V.device)
        plan.build_smatrix(V.contiguous())
        plan.eels_signal(n_ch, H.contiguous(), H_off, scan, OUT_MAP, precision, out)
        ctx.plan, ctx.n_ch, ctx.H_off, ctx.scan = plan, n_ch, H_off, scan
        ctx.precision = precision
        ctx.save_for_backward(V, H)
        return out

    @staticmethod
    def backward(ctx, grad_I):
        V, H = ctx.saved_tensors
        dV = torch.empty_like(V)
        gH = torch.empty_like(H) if ctx.needs_input_grad[1] else None
        # the checkpoints belong to the last build: rebuild only if another V
        # (or this one, modified) was built since
        Vc = V.contiguous()
        if not ctx.plan.built_from(Vc):
            ctx.plan.build_smatrix(Vc)
        ctx.plan.eels_backward(ctx.n_ch, H.contiguous(), ctx.H_off, ctx.scan,
                               grad_I.contiguous().float(), dV, dL_dHconj=gH,
                               precision=ctx.precision)
        return dV, (2.0 * gH if gH is not None else None), None, None, None, None, None


class SlicePotential(torch.autograd.Function):
    """V = potential(xyz) through bip_potential_build; backward through
    bip_potential_grad.  xyz: float64 tensor [n, 3] (any device; the library
    reads the positions on the host); its gradient comes back on xyz's device."""

    @staticmethod
    def forward(ctx, xyz, grid, amp, width, shape):
        V = torch.empty(shape, dtype=torch.float32, device="cuda")
        x = xyz.detach().cpu().numpy()
        potential_build(grid, x, amp, width, V)
        ctx.grid, ctx.x, ctx.amp, ctx.width = grid, x, amp, width
        ctx.xyz_device = xyz.device
        return V

    @staticmethod
    def backward(ctx, grad_V):
        g = potential_grad(ctx.grid, ctx.x, ctx.amp, ctx.width, grad_V.contiguous().float())
        return g.to(ctx.xyz_device), None, None, None, None


def library_path() -> str:
    return _LIB_PATH
