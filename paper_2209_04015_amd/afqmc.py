"""ctypes binding of the C ABI in ``include/afqmc.h`` (argument marshalling only).

Device arrays are torch tensors on the GPU (PyTorch is used for device memory
and streams only); every step of the method runs in the HIP library
``_lib/libafqmc.so``.  If that library is missing, :func:`load` raises: there
is no fallback path.
"""

from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

__all__ = ["FP64", "FP32", "BF16X3", "FP16X3", "AfqmcError", "load", "Hamiltonian", "Walkers", "Batch", "MSDTrial",
           "population_control_noalloc", "LIB_PATH"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libafqmc.so")

FP64 = 0
FP32 = 1
BF16X3 = 2
FP16X3 = 3
STEP_REUSE = 1
FLAG_ONE_BODY_FP64 = 1  # AFQMC_FLAG_ONE_BODY_FP64
FLAG_UNFUSED_PROPAGATION = 2  # AFQMC_FLAG_UNFUSED_PROPAGATION
# status-word bits (afqmc_get_status)
STATUS_SINGULAR, STATUS_NONFINITE, STATUS_QR_ZERO, STATUS_NO_LIVE = 1, 2, 4, 8
MSD_MAX_RANK = 6  # AFQMC_MSD_MAX_RANK
EXCHANGE_AUTO, EXCHANGE_DIRECT, EXCHANGE_PAIR = 0, 1, 2
_EXCHANGE = {"auto": EXCHANGE_AUTO, "direct": EXCHANGE_DIRECT, "pair": EXCHANGE_PAIR}
_PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "fp16x3": FP16X3,
               FP64: FP64, FP32: FP32, BF16X3: BF16X3, FP16X3: FP16X3}

EXPORTED = (
    "afqmc_init_hamiltonian",
    "afqmc_overlap",
    "afqmc_force_bias",
    "afqmc_propagate",
    "afqmc_local_energy",
    "afqmc_orthogonalise",
    "afqmc_step",
    "afqmc_global_energy",
    "afqmc_population_control",
    "afqmc_population_control_noalloc",
    "afqmc_block",
    "afqmc_green_function",
    "afqmc_s2_mixed",
    "afqmc_weighted_mean",
    "afqmc_get_exchange_algorithm",
    "afqmc_get_status",
    "afqmc_get_setup",
    "afqmc_profile_enable",
    "afqmc_profile_read",
    "afqmc_profile_phases",
    "afqmc_batch_create",
    "afqmc_batch_step",
    "afqmc_autotune",
    "afqmc_get_tuning",
    "afqmc_set_tuning",
    "afqmc_batch_destroy",
    "afqmc_msd_create",
    "afqmc_msd_overlap",
    "afqmc_msd_green_function",
    "afqmc_msd_force_bias",
    "afqmc_msd_propagate",
    "afqmc_msd_set_hamiltonian",
    "afqmc_msd_local_energy",
    "afqmc_msd_get_strings",
    "afqmc_msd_get_status",
    "afqmc_msd_destroy",
    "afqmc_destroy",
    "afqmc_last_error",
    "afqmc_version",
)


# kernel phases of afqmc_profile_read, in header order
PHASES = ("green", "force_bias", "shift", "vhs", "one_body", "taylor", "qr", "weight",
          "exchange", "energy", "split", "control", "estimator", "propagate")


class AfqmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"afqmc error {code}: {msg}")
        self.code = code


class _Tuning(ctypes.Structure):
    _fields_ = [("ex_tile_m", ctypes.c_int), ("ex_tile_n", ctypes.c_int), ("ex_group", ctypes.c_int),
                ("vhs_tile_m", ctypes.c_int), ("vhs_tile_n", ctypes.c_int)]


class _Params(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int),
        ("na", ctypes.c_int),
        ("nb", ctypes.c_int),
        ("K", ctypes.c_int),
        ("dt", ctypes.c_double),
        ("taylor_order", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("max_walkers", ctypes.c_int),
        ("mu", ctypes.c_double),
        ("e_shift", ctypes.c_double),
        ("exchange", ctypes.c_int),
        ("flags", ctypes.c_int),
    ]


class _BatchOpts(ctypes.Structure):
    _fields_ = [("use_graph", ctypes.c_int), ("reserved", ctypes.c_int * 7)]


class _Walkers(ctypes.Structure):
    _fields_ = [
        ("phi_a", ctypes.c_void_p),
        ("phi_b", ctypes.c_void_p),
        ("log_ovlp", ctypes.c_void_p),
        ("log_w", ctypes.c_void_p),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing; build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
    P = ctypes.POINTER
    lib.afqmc_init_hamiltonian.argtypes = [P(_Params), vp, vp, vp, vp, vp, P(vp)]
    lib.afqmc_overlap.argtypes = [vp, P(_Walkers), ip, vp]
    lib.afqmc_force_bias.argtypes = [vp, P(_Walkers), ip, vp, vp]
    lib.afqmc_propagate.argtypes = [vp, P(_Walkers), ip, vp, vp]
    lib.afqmc_local_energy.argtypes = [vp, P(_Walkers), ip, vp, vp]
    lib.afqmc_orthogonalise.argtypes = [vp, P(_Walkers), ip, vp]
    lib.afqmc_step.argtypes = [vp, P(_Walkers), ip, vp, ip, vp, ip, vp]
    lib.afqmc_global_energy.argtypes = [vp, P(_Walkers), ip, vp, vp, vp]
    lib.afqmc_population_control.argtypes = [vp, P(_Walkers), ip, ctypes.c_double, vp, vp]
    lib.afqmc_population_control_noalloc.argtypes = [ip, ip, ip, P(_Walkers), ip, ctypes.c_double, vp, vp, vp]
    lib.afqmc_block.argtypes = [vp, P(_Walkers), ip, vp, ip, ctypes.c_double, vp, vp, vp, ip, vp]
    lib.afqmc_green_function.argtypes = [vp, P(_Walkers), ip, vp, vp]
    lib.afqmc_s2_mixed.argtypes = [vp, P(_Walkers), ip, vp, vp]
    lib.afqmc_weighted_mean.argtypes = [vp, P(_Walkers), ip, vp, ip, vp, vp]
    lib.afqmc_get_exchange_algorithm.argtypes = [vp, P(ip)]
    lib.afqmc_get_status.argtypes = [vp, vp, P(ip)]
    lib.afqmc_get_setup.argtypes = [vp, vp, dp, dp]
    lib.afqmc_profile_enable.argtypes = [vp, ip]
    lib.afqmc_profile_read.argtypes = [vp, vp, vp]
    lib.afqmc_profile_phases.argtypes = [vp, ctypes.c_uint]
    lib.afqmc_batch_create.argtypes = [vp, vp, vp, ip, P(_BatchOpts), P(vp)]
    lib.afqmc_batch_step.argtypes = [vp, vp, vp, ip, ip, vp]
    lib.afqmc_autotune.argtypes = [vp, ctypes.c_char_p]
    lib.afqmc_get_tuning.argtypes = [vp, P(_Tuning)]
    lib.afqmc_set_tuning.argtypes = [vp, P(_Tuning)]
    lib.afqmc_batch_destroy.argtypes = [vp]
    lib.afqmc_batch_destroy.restype = None
    lib.afqmc_msd_create.argtypes = [ip, ip, ip, vp, vp, ip, vp, vp, vp, ip, vp, P(vp)]
    lib.afqmc_msd_overlap.argtypes = [vp, P(_Walkers), ip, vp, vp]
    lib.afqmc_msd_green_function.argtypes = [vp, P(_Walkers), ip, vp, vp]
    lib.afqmc_msd_force_bias.argtypes = [vp, vp, P(_Walkers), ip, vp, vp]
    lib.afqmc_msd_propagate.argtypes = [vp, vp, P(_Walkers), ip, vp, vp]
    lib.afqmc_msd_set_hamiltonian.argtypes = [vp, ip, vp, vp, vp]
    lib.afqmc_msd_local_energy.argtypes = [vp, P(_Walkers), ip, vp, vp]
    lib.afqmc_msd_get_strings.argtypes = [vp, P(ip), P(ip)]
    lib.afqmc_msd_get_status.argtypes = [vp, vp, P(ip)]
    lib.afqmc_msd_destroy.argtypes = [vp]
    lib.afqmc_msd_destroy.restype = None
    lib.afqmc_destroy.argtypes = [vp]
    lib.afqmc_destroy.restype = None
    lib.afqmc_last_error.argtypes = []
    lib.afqmc_last_error.restype = ctypes.c_char_p
    lib.afqmc_version.argtypes = []
    for name in EXPORTED:
        f = getattr(lib, name)
        if name not in ("afqmc_destroy", "afqmc_last_error", "afqmc_batch_destroy", "afqmc_msd_destroy"):
            f.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise AfqmcError(rc, _lib.afqmc_last_error().decode(errors="replace"))


def _stream_ptr(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _host(a, shape, name):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"{name} has shape {a.shape}, expected {shape}")
    return a


def _dev(t, dtype, shape, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Walkers:
    """Walker ensemble on the device: phi_a [W,N,na], phi_b [W,N,nb] complex128,
    log_ovlp [W] complex128, log_w [W] float64 (torch tensors)."""

    def __init__(self, phi_a, phi_b, log_ovlp=None, log_w=None):
        import torch

        self.phi_a = phi_a
        self.phi_b = phi_b
        W = phi_a.shape[0]
        dev = phi_a.device
        self.log_ovlp = log_ovlp if log_ovlp is not None else torch.zeros(W, dtype=torch.complex128, device=dev)
        self.log_w = log_w if log_w is not None else torch.zeros(W, dtype=torch.float64, device=dev)

    @property
    def W(self):
        return self.phi_a.shape[0]

    @classmethod
    def from_numpy(cls, phi_a, phi_b, log_ovlp=None, log_w=None, device="cuda"):
        import torch

        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
        return cls(
            t(phi_a, torch.complex128),
            t(phi_b, torch.complex128),
            None if log_ovlp is None else t(log_ovlp, torch.complex128),
            None if log_w is None else t(log_w, torch.float64),
        )

    def _struct(self, ham, nw):
        import torch

        N, na, nb = ham.N, ham.na, ham.nb
        s = _Walkers()
        s.phi_a = _dev(self.phi_a, torch.complex128, (self.W, N, na), "phi_a").value
        s.phi_b = _dev(self.phi_b, torch.complex128, (self.W, N, nb), "phi_b").value
        s.log_ovlp = _dev(self.log_ovlp, torch.complex128, (self.W,), "log_ovlp").value
        s.log_w = _dev(self.log_w, torch.float64, (self.W,), "log_w").value
        if nw > self.W:
            raise ValueError(f"nw = {nw} exceeds the {self.W} walkers held")
        return s


class _WalkerShape:
    def __init__(self, w):
        _, self.N, self.na = w.phi_a.shape
        self.nb = w.phi_b.shape[2]


def population_control_noalloc(w: Walkers, u: float, parent=None, status=None, nw=None, stream=None):
    """afqmc_population_control_noalloc: the comb on the library's static
    scratch, without a Hamiltonian handle (sizes from the walker arrays).
    parent (device int32 [nw]) and status (device int32 [1]) are optional
    outputs; returns parent."""
    import torch

    load()
    nw = w.W if nw is None else int(nw)
    shape = _WalkerShape(w)
    pptr = _dev(parent, torch.int32, (nw,), "parent") if parent is not None else None
    sptr = _dev(status, torch.int32, (1,), "status") if status is not None else None
    s = w._struct(shape, nw)
    with torch.cuda.device(w.phi_a.device):
        _check(_lib.afqmc_population_control_noalloc(shape.N, shape.na, shape.nb, ctypes.byref(s), nw, float(u),
                                                     pptr, sptr, _stream_ptr(stream)))
    return parent


class Hamiltonian:
    """A Hamiltonian handle (afqmc_init_hamiltonian) and its workspace."""

    def __init__(self, h1, chol, phiT_a, phiT_b=None, *, dt, max_walkers, taylor_order=6,
                 precision="fp64", mu=None, e_shift=None, exchange="auto", one_body_fp64=False,
                 unfused_propagation=False,
                 stream=None):
        lib = load()
        h1 = np.asarray(h1)
        N = h1.shape[0]
        chol = np.asarray(chol)
        K = chol.shape[0]
        phiT_a = np.asarray(phiT_a)
        na = phiT_a.shape[1]
        phiT_b = phiT_a if phiT_b is None else np.asarray(phiT_b)
        nb = phiT_b.shape[1]
        self._h1 = _host(h1, (N, N), "h1")
        self._chol = _host(chol, (K, N, N), "chol")
        self._pa = _host(phiT_a, (N, na), "phiT_a")
        self._pb = _host(phiT_b, (N, nb), "phiT_b")
        self.N, self.na, self.nb, self.K = N, na, nb, K
        self.precision = _PRECISIONS[precision]
        self.max_walkers = int(max_walkers)
        p = _Params(N, na, nb, K, float(dt), int(taylor_order), self.precision, self.max_walkers,
                    math.nan if mu is None else float(mu), math.nan if e_shift is None else float(e_shift),
                    _EXCHANGE[exchange], (FLAG_ONE_BODY_FP64 if one_body_fp64 else 0)
                    | (FLAG_UNFUSED_PROPAGATION if unfused_propagation else 0))
        h = ctypes.c_void_p()
        _check(lib.afqmc_init_hamiltonian(
            ctypes.byref(p), self._h1.ctypes.data, self._chol.ctypes.data, self._pa.ctypes.data,
            self._pb.ctypes.data, _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        # host copies are not needed after init
        self._chol = None
        v = ctypes.c_int()
        _check(lib.afqmc_get_exchange_algorithm(self._h, ctypes.byref(v)))
        self.exchange = {EXCHANGE_DIRECT: "direct", EXCHANGE_PAIR: "pair"}[v.value]

    def close(self):
        if getattr(self, "_h", None):
            _lib.afqmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _nw(self, w, nw):
        return w.W if nw is None else int(nw)

    def overlap(self, w: Walkers, nw=None, stream=None):
        nw = self._nw(w, nw)
        s = w._struct(self, nw)
        _check(_lib.afqmc_overlap(self._h, ctypes.byref(s), nw, _stream_ptr(stream)))

    def force_bias(self, w: Walkers, out=None, nw=None, stream=None):
        import torch

        nw = self._nw(w, nw)
        if out is None:
            out = torch.empty((nw, self.K), dtype=torch.complex128, device=w.phi_a.device)
        ptr = _dev(out, torch.complex128, (nw, self.K), "vbias")
        s = w._struct(self, nw)
        _check(_lib.afqmc_force_bias(self._h, ctypes.byref(s), nw, ptr, _stream_ptr(stream)))
        return out

    def propagate(self, w: Walkers, fields, nw=None, stream=None):
        import torch

        nw = self._nw(w, nw)
        fp = _dev(fields, torch.float64, (nw, self.K), "fields")
        s = w._struct(self, nw)
        _check(_lib.afqmc_propagate(self._h, ctypes.byref(s), nw, fp, _stream_ptr(stream)))

    def local_energy(self, w: Walkers, out=None, nw=None, stream=None):
        import torch

        nw = self._nw(w, nw)
        if out is None:
            out = torch.empty((nw, 3), dtype=torch.complex128, device=w.phi_a.device)
        ptr = _dev(out, torch.complex128, (nw, 3), "energy")
        s = w._struct(self, nw)
        _check(_lib.afqmc_local_energy(self._h, ctypes.byref(s), nw, ptr, _stream_ptr(stream)))
        return out

    def orthogonalise(self, w: Walkers, nw=None, stream=None):
        nw = self._nw(w, nw)
        s = w._struct(self, nw)
        _check(_lib.afqmc_orthogonalise(self._h, ctypes.byref(s), nw, _stream_ptr(stream)))

    def step(self, w: Walkers, fields, do_qr=False, energy_out=None, reuse=False, nw=None,
             stream=None):
        import torch

        nw = self._nw(w, nw)
        fp = _dev(fields, torch.float64, (nw, self.K), "fields")
        eptr = None
        if energy_out is not None:
            eptr = _dev(energy_out, torch.complex128, (nw, 3), "energy")
        s = w._struct(self, nw)
        _check(_lib.afqmc_step(self._h, ctypes.byref(s), nw, fp, int(bool(do_qr)), eptr,
                               STEP_REUSE if reuse else 0, _stream_ptr(stream)))
        return energy_out

    def global_energy(self, w: Walkers, e, out=None, nw=None, stream=None):
        """Device float64 [4]: Re E, Im E, ln sum w, live walkers (E = sum w E_L / sum w)."""
        import torch

        nw = self._nw(w, nw)
        if out is None:
            out = torch.empty(4, dtype=torch.float64, device=w.phi_a.device)
        optr = _dev(out, torch.float64, (4,), "out")
        eptr = _dev(e, torch.complex128, (nw, 3), "energy") if nw else None
        s = w._struct(self, nw)
        _check(_lib.afqmc_global_energy(self._h, ctypes.byref(s), nw, eptr, optr, _stream_ptr(stream)))
        return out

    def population_control(self, w: Walkers, u: float, parent=None, nw=None, stream=None):
        """Comb population control in place; returns the device int32 parent map."""
        import torch

        nw = self._nw(w, nw)
        if parent is None:
            parent = torch.empty(nw, dtype=torch.int32, device=w.phi_a.device)
        pptr = _dev(parent, torch.int32, (nw,), "parent")
        s = w._struct(self, nw)
        _check(_lib.afqmc_population_control(self._h, ctypes.byref(s), nw, float(u), pptr,
                                             _stream_ptr(stream)))
        return parent

    def block(self, w: Walkers, fields, u, energy_out=None, out=None, parent=None, reuse=False,
              nw=None, stream=None):
        """len(fields) steps (QR and energy at the last), global energy, comb (u >= 0).

        Returns (energy [nw, 3], out [4], parent [nw])."""
        import torch

        nw = self._nw(w, nw)
        nsteps = int(fields.shape[0])
        dev = w.phi_a.device
        fp = _dev(fields, torch.float64, (nsteps, nw, self.K), "fields")
        if energy_out is None:
            energy_out = torch.empty((nw, 3), dtype=torch.complex128, device=dev)
        if out is None:
            out = torch.empty(4, dtype=torch.float64, device=dev)
        if parent is None:
            parent = torch.empty(nw, dtype=torch.int32, device=dev)
        s = w._struct(self, nw)
        _check(_lib.afqmc_block(self._h, ctypes.byref(s), nw, fp, nsteps, float(u),
                                _dev(energy_out, torch.complex128, (nw, 3), "energy"),
                                _dev(out, torch.float64, (4,), "out"),
                                _dev(parent, torch.int32, (nw,), "parent"),
                                STEP_REUSE if reuse else 0, _stream_ptr(stream)))
        return energy_out, out, parent

    def green_function(self, w: Walkers, out=None, nw=None, stream=None):
        """Device complex128 [nw, 2, N, N]: G^s_pq of every walker."""
        import torch

        nw = self._nw(w, nw)
        if out is None:
            out = torch.empty((nw, 2, self.N, self.N), dtype=torch.complex128, device=w.phi_a.device)
        ptr = _dev(out, torch.complex128, (nw, 2, self.N, self.N), "G")
        s = w._struct(self, nw)
        _check(_lib.afqmc_green_function(self._h, ctypes.byref(s), nw, ptr, _stream_ptr(stream)))
        return out

    def s2_mixed(self, w: Walkers, out=None, nw=None, stream=None):
        """Device complex128 [nw]: the mixed estimator of S^2 of every walker."""
        import torch

        nw = self._nw(w, nw)
        if out is None:
            out = torch.empty(nw, dtype=torch.complex128, device=w.phi_a.device)
        ptr = _dev(out, torch.complex128, (nw,), "s2")
        s = w._struct(self, nw)
        _check(_lib.afqmc_s2_mixed(self._h, ctypes.byref(s), nw, ptr, _stream_ptr(stream)))
        return out

    def weighted_mean(self, w: Walkers, values, out=None, nw=None, stream=None):
        """values complex128 [nw, m] -> device float64 [2m + 2] (means re/im, ln sum w, live)."""
        import torch

        nw = self._nw(w, nw)
        m = int(values.shape[1]) if values.dim() == 2 else 1
        if out is None:
            out = torch.empty(2 * m + 2, dtype=torch.float64, device=w.phi_a.device)
        vptr = _dev(values, torch.complex128, (nw, m) if values.dim() == 2 else (nw,), "values")
        optr = _dev(out, torch.float64, (2 * m + 2,), "out")
        s = w._struct(self, nw)
        _check(_lib.afqmc_weighted_mean(self._h, ctypes.byref(s), nw, vptr, m, optr, _stream_ptr(stream)))
        return out

    def status(self, stream=None) -> int:
        v = ctypes.c_int()
        _check(_lib.afqmc_get_status(self._h, _stream_ptr(stream), ctypes.byref(v)))
        return v.value

    def tuning(self) -> dict:
        """Kernel tiling (afqmc_get_tuning): exchange and VHS output tile shapes, exchange group size."""
        t = _Tuning()
        _check(_lib.afqmc_get_tuning(self._h, ctypes.byref(t)))
        return {"exchange_tile": (t.ex_tile_m, t.ex_tile_n), "exchange_group": t.ex_group,
                "vhs_tile": (t.vhs_tile_m, t.vhs_tile_n)}

    def set_tuning(self, exchange_tile, exchange_group, vhs_tile):
        """afqmc_set_tuning: shapes as (rows, columns) tuples."""
        t = _Tuning(int(exchange_tile[0]), int(exchange_tile[1]), int(exchange_group), int(vhs_tile[0]),
                    int(vhs_tile[1]))
        _check(_lib.afqmc_set_tuning(self._h, ctypes.byref(t)))

    def profile_enable(self, max_records: int):
        """Bracket every kernel phase with HIP events on its stream (0 turns it off)."""
        _check(_lib.afqmc_profile_enable(self._h, int(max_records)))

    def profile_phases(self, phases=None):
        """Time only the named phases (None: all) from the next call on."""
        mask = 0xFFFFFFFF if phases is None else sum(1 << PHASES.index(p) for p in phases)
        _check(_lib.afqmc_profile_phases(self._h, mask))

    def profile_read(self):
        """{phase: (total ms, launches)} since the last read; synchronises."""
        ms = np.zeros(len(PHASES))
        n = np.zeros(len(PHASES), dtype=np.int32)
        _check(_lib.afqmc_profile_read(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                       n.ctypes.data_as(ctypes.c_void_p)))
        return {p: (float(ms[i]), int(n[i])) for i, p in enumerate(PHASES)}

    def setup(self):
        """(P [N,N], mu, e_shift) as computed at init."""
        P = np.zeros((self.N, self.N))
        mu = ctypes.c_double()
        es = ctypes.c_double()
        _check(_lib.afqmc_get_setup(self._h, P.ctypes.data_as(ctypes.c_void_p), ctypes.byref(mu), ctypes.byref(es)))
        return P, mu.value, es.value


class Batch:
    """Several Hamiltonians (of uneven sizes) advanced together, one hipGraph
    launch per step (afqmc_batch_create / afqmc_batch_step)."""

    def __init__(self, hams, walkers, nw=None, use_graph=True):
        load()
        self.hams = list(hams)
        self.walkers = list(walkers)
        n = len(self.hams)
        self.nw = [w.W for w in self.walkers] if nw is None else [int(x) for x in nw]
        ws = (_Walkers * n)()
        for i, (h, w) in enumerate(zip(self.hams, self.walkers)):
            ws[i] = w._struct(h, self.nw[i])
        hp = (ctypes.c_void_p * n)(*[h._h.value for h in self.hams])
        nwa = (ctypes.c_int * n)(*self.nw)
        opts = _BatchOpts(1 if use_graph else 0)
        b = ctypes.c_void_p()
        _check(_lib.afqmc_batch_create(ctypes.cast(hp, ctypes.c_void_p), ctypes.cast(ws, ctypes.c_void_p),
                                       ctypes.cast(nwa, ctypes.c_void_p), n, ctypes.byref(opts), ctypes.byref(b)))
        self._b = b
        self._keep = (ws, hp, nwa)

    def step(self, fields, energies=None, do_qr=True, stream=None):
        """fields[i]: [nsteps, nw_i, K_i] float64; energies[i]: [nsteps, nw_i, 3] complex128 or None."""
        import torch

        n = len(self.hams)
        nsteps = fields[0].shape[0]
        fp = []
        for i in range(n):
            fp.append(_dev(fields[i], torch.float64, (nsteps, self.nw[i], self.hams[i].K), f"fields[{i}]").value)
        ep = [None] * n
        if energies is not None:
            for i in range(n):
                if energies[i] is not None:
                    ep[i] = _dev(energies[i], torch.complex128, (nsteps, self.nw[i], 3), f"energies[{i}]").value
        fa = (ctypes.c_void_p * n)(*fp)
        ea = (ctypes.c_void_p * n)(*ep)
        _check(_lib.afqmc_batch_step(self._b, ctypes.cast(fa, ctypes.c_void_p), ctypes.cast(ea, ctypes.c_void_p),
                                     int(nsteps), int(bool(do_qr)), _stream_ptr(stream)))

    def autotune(self, cache_path=None):
        _check(_lib.afqmc_autotune(self._b, None if cache_path is None else str(cache_path).encode()))

    def close(self):
        if getattr(self, "_b", None):
            _lib.afqmc_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MSDTrial:
    """A multi-determinant trial handle (afqmc_msd_create): the overlap and
    Green's function of walkers against sum_a c_a t_a |psi_0> (Sec. III.A).

    C_a, C_b: [N, N] orthogonal orbitals (psi_0 = their first na / nb
    columns); coeff [ndet]; rank [ndet, 2]; orbs [ndet, 2, 2, MSD_MAX_RANK]
    (the format of ``inputs.msd_expansion``)."""

    def __init__(self, C_a, C_b, na, nb, coeff, rank, orbs, *, max_walkers, stream=None):
        lib = load()
        C_a = np.asarray(C_a)
        N = C_a.shape[0]
        C_b = C_a if C_b is None else C_b
        coeff = np.asarray(coeff)
        ndet = coeff.shape[0]
        self._ca = _host(C_a, (N, N), "C_a")
        self._cb = _host(C_b, (N, N), "C_b")
        self._coeff = _host(coeff, (ndet,), "coeff")
        self._rank = np.ascontiguousarray(rank, dtype=np.int32)
        self._orbs = np.ascontiguousarray(orbs, dtype=np.int32)
        if self._rank.shape != (ndet, 2) or self._orbs.shape != (ndet, 2, 2, MSD_MAX_RANK):
            raise ValueError("rank must be [ndet, 2] and orbs [ndet, 2, 2, MSD_MAX_RANK]")
        self.N, self.na, self.nb, self.ndet = N, int(na), int(nb), ndet
        self.max_walkers = int(max_walkers)
        h = ctypes.c_void_p()
        _check(lib.afqmc_msd_create(N, self.na, self.nb, self._ca.ctypes.data, self._cb.ctypes.data, ndet,
                                    self._coeff.ctypes.data, self._rank.ctypes.data, self._orbs.ctypes.data,
                                    self.max_walkers, _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib.afqmc_msd_get_strings(self._h, ctypes.byref(a), ctypes.byref(b)))
        self.strings = (a.value, b.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib.afqmc_msd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def overlap(self, w: Walkers, out=None, nw=None, stream=None):
        """Device complex128 [nw]: log <Psi_T|phi_z>."""
        import torch

        nw = w.W if nw is None else int(nw)
        if out is None:
            out = torch.empty((nw,), dtype=torch.complex128, device=w.phi_a.device)
        ptr = _dev(out, torch.complex128, (nw,), "log_ovlp")
        s = w._struct(self, nw)
        _check(_lib.afqmc_msd_overlap(self._h, ctypes.byref(s), nw, ptr, _stream_ptr(stream)))
        return out

    def green_function(self, w: Walkers, out=None, nw=None, stream=None):
        """Device complex128 [nw, 2, N, N]: G^s_pq of every walker for this trial."""
        import torch

        nw = w.W if nw is None else int(nw)
        if out is None:
            out = torch.empty((nw, 2, self.N, self.N), dtype=torch.complex128, device=w.phi_a.device)
        ptr = _dev(out, torch.complex128, (nw, 2, self.N, self.N), "G")
        s = w._struct(self, nw)
        _check(_lib.afqmc_msd_green_function(self._h, ctypes.byref(s), nw, ptr, _stream_ptr(stream)))
        return out

    def force_bias(self, ham: "Hamiltonian", w: Walkers, out=None, nw=None, stream=None):
        """Device complex128 [nw, K]: sum_s sum_pq G^s_pq L_g,pq for this trial (ham: FP64)."""
        import torch

        nw = w.W if nw is None else int(nw)
        if out is None:
            out = torch.empty((nw, ham.K), dtype=torch.complex128, device=w.phi_a.device)
        ptr = _dev(out, torch.complex128, (nw, ham.K), "vbias")
        s = w._struct(self, nw)
        _check(_lib.afqmc_msd_force_bias(self._h, ham._h, ctypes.byref(s), nw, ptr, _stream_ptr(stream)))
        return out

    def propagate(self, ham: "Hamiltonian", w: Walkers, fields, nw=None, stream=None):
        """One phaseless step of w under this trial (ham: FP64); w.log_ovlp must
        hold the expansion's log overlap (see overlap)."""
        import torch

        nw = w.W if nw is None else int(nw)
        fp = _dev(fields, torch.float64, (nw, ham.K), "fields")
        s = w._struct(self, nw)
        _check(_lib.afqmc_msd_propagate(self._h, ham._h, ctypes.byref(s), nw, fp, _stream_ptr(stream)))

    def set_hamiltonian(self, h1, chol, stream=None):
        """Attach h1 [N, N] and the Cholesky vectors [K, N, N] (host arrays) for
        local_energy (afqmc_msd_set_hamiltonian)."""
        h1 = _host(h1, (self.N, self.N), "h1")
        chol = np.asarray(chol)
        K = chol.shape[0]
        chol = _host(chol, (K, self.N, self.N), "chol")
        _check(_lib.afqmc_msd_set_hamiltonian(self._h, K, h1.ctypes.data, chol.ctypes.data, _stream_ptr(stream)))
        self.K = K

    def local_energy(self, w: Walkers, out=None, nw=None, stream=None):
        """E_L of each walker against the expansion: complex [nw, 3] (E1, EJ, EK)."""
        import torch

        nw = w.W if nw is None else int(nw)
        if out is None:
            out = torch.empty((nw, 3), dtype=torch.complex128, device=w.phi_a.device)
        optr = _dev(out, torch.complex128, (nw, 3), "energy")
        s = w._struct(self, nw)
        _check(_lib.afqmc_msd_local_energy(self._h, ctypes.byref(s), nw, optr, _stream_ptr(stream)))
        return out

    def status(self, stream=None):
        v = ctypes.c_int()
        _check(_lib.afqmc_msd_get_status(self._h, _stream_ptr(stream), ctypes.byref(v)))
        return v.value
