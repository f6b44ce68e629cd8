"""ctypes binding of libvgtb.so (the C ABI declared in include/vgtb.h).

Argument marshalling only: every step of the propagation runs in the HIP
library.  PyTorch provides the device arena, output tensors and the stream.
The binding refuses to run without the built library and a GPU.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvgtb.so")

VGTB_OK, VGTB_E_INVAL, VGTB_E_STATE, VGTB_E_NOT_PD, VGTB_E_UNSTABLE, VGTB_E_NOMEM, \
    VGTB_E_DEVICE, VGTB_E_NONFINITE = range(8)
STATUS_NAMES = {0: "VGTB_OK", 1: "VGTB_E_INVAL", 2: "VGTB_E_STATE", 3: "VGTB_E_NOT_PD",
                4: "VGTB_E_UNSTABLE", 5: "VGTB_E_NOMEM", 6: "VGTB_E_DEVICE", 7: "VGTB_E_NONFINITE"}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x3": 3}
COUPLINGS = {"peierls": 0, "momentum": 1}
PROPAGATORS = {"leapfrog": 0, "crank_nicolson": 1}

# Every symbol the header declares (checked by the CPU test suite).
EXPORTED = [
    "vgtb_workspace_size", "vgtb_create", "vgtb_ground_state", "vgtb_set_density",
    "vgtb_set_field_table", "vgtb_set_field", "vgtb_step", "vgtb_synchronize",
    "vgtb_read_observables", "vgtb_get_density", "vgtb_get_reference_charges",
    "vgtb_state_size", "vgtb_save_state", "vgtb_load_state", "vgtb_step_index",
    "vgtb_last_error", "vgtb_destroy", "vgtb_zgemm", "vgtb_profile_enable", "vgtb_profile_read",
    "vgtb_spectrum", "vgtb_autotune", "vgtb_server_create", "vgtb_server_run",
    "vgtb_server_destroy", "vgtb_set_coefficients", "vgtb_num_states", "vgtb_get_coefficients",
    "vgtb_spectrum_noalloc", "vgtb_group_create", "vgtb_group_step", "vgtb_group_destroy",
]
KERNELS = {"observe": 0, "reduce": 1, "spmm": 2, "gemm": 3, "update": 4, "rescale": 5,
           "assemble": 6, "small": 7, "cn_pattern": 8, "cn_solve": 9, "cn_update": 10}


class VgtbError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class VgtbSystem(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int32), ("orbs_per_atom", ctypes.c_int32),
        ("cell", ctypes.c_double * 9), ("n_blocks", ctypes.c_int32),
        ("blk_i", ctypes.c_void_p), ("blk_j", ctypes.c_void_p), ("blk_d", ctypes.c_void_p),
        ("blk_h0", ctypes.c_void_p), ("blk_s", ctypes.c_void_p), ("n_k", ctypes.c_int32),
        ("kpts", ctypes.c_void_p), ("kw", ctypes.c_void_p), ("n_electrons", ctypes.c_double),
        ("z_ref", ctypes.c_void_p), ("gamma", ctypes.c_void_p), ("blk_ds", ctypes.c_void_p),
    ]


OPT_NO_GRAPHS, OPT_NO_SMALL_PATH, OPT_FUSE_UPDATE = 1, 2, 4


class VgtbOptions(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("precision", ctypes.c_int32),
                ("rescale_every", ctypes.c_int32), ("history_capacity", ctypes.c_int32),
                ("coupling", ctypes.c_int32), ("propagator", ctypes.c_int32),
                ("tile_override", ctypes.c_int32), ("spmm_variant", ctypes.c_int32),
                ("spmm_group", ctypes.c_int32), ("flags", ctypes.c_int32)]


class VgtbTuning(ctypes.Structure):
    _fields_ = [("spmm_variant", ctypes.c_int32), ("gemm_tile", ctypes.c_int32),
                ("n_spmm", ctypes.c_int32), ("n_gemm", ctypes.c_int32),
                ("spmm_candidates", ctypes.c_int32 * 8), ("spmm_ms", ctypes.c_double * 8),
                ("gemm_candidates", ctypes.c_int32 * 8), ("gemm_ms", ctypes.c_double * 8)]


class VgtbRequest(ctypes.Structure):
    _fields_ = [("system", ctypes.c_void_p), ("options", VgtbOptions), ("n_steps", ctypes.c_int64),
                ("n_field", ctypes.c_int64), ("field", ctypes.c_void_p),
                ("n_omega", ctypes.c_int32), ("omega", ctypes.c_void_p),
                ("e0", ctypes.c_double), ("tau0", ctypes.c_double), ("arrival_s", ctypes.c_double),
                ("j_out", ctypes.c_void_p), ("sigma_out", ctypes.c_void_p)]


class VgtbRequestStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("slot", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_size_t), ("arrival_s", ctypes.c_double),
                ("admitted_s", ctypes.c_double), ("ready_s", ctypes.c_double),
                ("finished_s", ctypes.c_double), ("message", ctypes.c_char * 128)]


class VgtbServerStats(ctypes.Structure):
    _fields_ = [("makespan_s", ctypes.c_double), ("k_steps", ctypes.c_double),
                ("k_steps_per_s", ctypes.c_double), ("peak_bytes", ctypes.c_size_t),
                ("peak_active", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libvgtb.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2308_09782_amd.build.build()")
    lib = ctypes.CDLL(path)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "vgtb_workspace_size": [vp, vp, ctypes.POINTER(sz)],
        "vgtb_create": [vp, vp, vp, sz, vp, ctypes.POINTER(vp)],
        "vgtb_ground_state": [vp, ctypes.POINTER(ctypes.c_double)],
        "vgtb_set_density": [vp, vp, ctypes.c_int],
        "vgtb_set_field_table": [vp, i64, vp],
        "vgtb_set_field": [vp, vp],
        "vgtb_step": [vp, i64],
        "vgtb_synchronize": [vp],
        "vgtb_read_observables": [vp, i64, i64, vp, vp, vp, vp],
        "vgtb_get_density": [vp, i32, vp, ctypes.c_int],
        "vgtb_get_reference_charges": [vp, vp],
        "vgtb_state_size": [vp, ctypes.POINTER(sz)],
        "vgtb_save_state": [vp, vp, sz],
        "vgtb_load_state": [vp, vp, sz],
        "vgtb_zgemm": [vp, vp, vp, i32, i32, vp],
        "vgtb_profile_enable": [vp, ctypes.c_int],
        "vgtb_profile_read": [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)],
        "vgtb_spectrum": [vp, i64, vp, ctypes.c_double, i64, vp, ctypes.c_double, ctypes.c_double,
                          ctypes.c_int, vp, vp],
        "vgtb_spectrum_noalloc": [i64, vp, ctypes.c_double, i64, vp, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int, vp, vp, vp],
        "vgtb_autotune": [vp, i32, ctypes.POINTER(VgtbTuning)],
        "vgtb_set_coefficients": [vp, vp, vp, i32, ctypes.c_int],
        "vgtb_get_coefficients": [vp, vp, vp, ctypes.c_int],
        "vgtb_server_create": [vp, sz, i32, ctypes.POINTER(vp)],
        "vgtb_group_create": [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)],
        "vgtb_group_step": [vp, i64],
        "vgtb_server_run": [vp, i32, ctypes.POINTER(VgtbRequest), ctypes.POINTER(VgtbRequestStats),
                            ctypes.POINTER(VgtbServerStats)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.vgtb_step_index.argtypes = [vp]
    lib.vgtb_step_index.restype = i64
    lib.vgtb_num_states.argtypes = [vp]
    lib.vgtb_num_states.restype = i32
    lib.vgtb_last_error.argtypes = [vp]
    lib.vgtb_last_error.restype = ctypes.c_char_p
    lib.vgtb_destroy.argtypes = [vp]
    lib.vgtb_destroy.restype = None
    lib.vgtb_server_destroy.argtypes = [vp]
    lib.vgtb_server_destroy.restype = None
    lib.vgtb_group_destroy.argtypes = [vp]
    lib.vgtb_group_destroy.restype = None
    _lib = lib
    return lib


def _check(status: int, ctx=None):
    if status != VGTB_OK:
        msg = load_library().vgtb_last_error(ctx)
        raise VgtbError(status, msg.decode() if msg else "")


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the vgtb library needs a ROCm GPU; none is visible")
    return torch


def make_system_struct(system):
    """Pack a tight-binding system (vgtb_synth.TBSystem or alike) into the C struct.

    Returns (struct, keepalive) - keep the second object alive during the call.
    """
    arrs = {
        "blk_i": np.ascontiguousarray(system.blk_i, dtype=np.int32),
        "blk_j": np.ascontiguousarray(system.blk_j, dtype=np.int32),
        "blk_d": np.ascontiguousarray(system.blk_d, dtype=np.float64),
        "blk_h0": np.ascontiguousarray(system.blk_h0, dtype=np.float64),
        "blk_s": np.ascontiguousarray(system.blk_s, dtype=np.float64),
        "kpts": np.ascontiguousarray(system.kpts, dtype=np.float64),
        "kw": np.ascontiguousarray(system.kw, dtype=np.float64),
        "z_ref": None if system.z_ref is None else np.ascontiguousarray(system.z_ref, np.float64),
        "gamma": None if system.gamma is None else np.ascontiguousarray(system.gamma, np.float64),
        "blk_ds": (None if getattr(system, "blk_ds", None) is None
                   else np.ascontiguousarray(system.blk_ds, dtype=np.float64)),
    }
    s = VgtbSystem()
    s.n_atoms = int(system.pos.shape[0])
    s.orbs_per_atom = int(system.norb)
    cell = np.ascontiguousarray(system.cell, dtype=np.float64).reshape(9)
    for i in range(9):
        s.cell[i] = float(cell[i])
    s.n_blocks = int(arrs["blk_i"].shape[0])
    s.n_k = int(arrs["kpts"].shape[0])
    s.n_electrons = float(system.n_electrons)
    for name in ("blk_i", "blk_j", "blk_d", "blk_h0", "blk_s", "kpts", "kw", "z_ref", "gamma",
                 "blk_ds"):
        setattr(s, name, _ptr(arrs[name]))
    return s, arrs


def make_options(dt: float, precision: str = "fp64", rescale_every: int = 50,
                 history_capacity: int = 1024, coupling: str = "peierls",
                 propagator: str = "leapfrog", tile: int = 0, spmm_variant: int = 0,
                 spmm_group: int = 0, graphs: bool = True, small_path: bool = True,
                 fused_update: bool = False) -> VgtbOptions:
    """vgtb_options; tile, spmm_variant and spmm_group are the header's kernel
    choices (0 = default); graphs / small_path clear the VGTB_OPT_NO_* flags,
    fused_update sets VGTB_OPT_FUSE_UPDATE."""
    o = VgtbOptions()
    o.dt = float(dt)
    o.precision = PRECISIONS[precision]
    o.rescale_every = int(rescale_every)
    o.history_capacity = int(history_capacity)
    o.coupling = COUPLINGS[coupling]
    o.propagator = PROPAGATORS[propagator]
    o.tile_override = int(tile)
    o.spmm_variant = int(spmm_variant)
    o.spmm_group = int(spmm_group)
    o.flags = ((0 if graphs else OPT_NO_GRAPHS) | (0 if small_path else OPT_NO_SMALL_PATH)
               | (OPT_FUSE_UPDATE if fused_update else 0))
    return o


def vgtb_workspace_size(system, options: VgtbOptions) -> int:
    lib = load_library()
    s, keep = make_system_struct(system)
    out = ctypes.c_size_t(0)
    _check(lib.vgtb_workspace_size(ctypes.byref(s), ctypes.byref(options), ctypes.byref(out)))
    del keep
    return int(out.value)


def vgtb_zgemm(a, b, c, stream=None):
    """c[k] = a[k] @ b[k] for complex128 CUDA tensors of shape (batch, n, n)."""
    torch = _torch()
    lib = load_library()
    for t in (a, b, c):
        if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("vgtb_zgemm needs contiguous complex128 device tensors")
    if not (a.shape == b.shape == c.shape and a.dim() == 3 and a.shape[1] == a.shape[2]):
        raise ValueError("vgtb_zgemm needs three (batch, n, n) tensors of one shape")
    st = torch.cuda.current_stream(a.device).cuda_stream if stream is None else stream
    _check(lib.vgtb_zgemm(a.data_ptr(), b.data_ptr(), c.data_ptr(), int(a.shape[1]),
                          int(a.shape[0]), st))


def spectrum_noalloc(j, dt: float, omegas, e0: float, tau0: float = 200.0,
                     subtract_mean: bool = True, stream=None):
    """(sigma, epsilon) of Eqs. 15-16 through vgtb_spectrum_noalloc (no context,
    no allocation: the library's fixed device scratch) on the current device."""
    torch = _torch()
    lib = load_library()
    j = np.ascontiguousarray(j, dtype=np.float64).reshape(-1)
    w = np.ascontiguousarray(omegas, dtype=np.float64).reshape(-1)
    sig = np.zeros(w.size, dtype=np.complex128)
    eps = np.zeros(w.size, dtype=np.complex128)
    st = torch.cuda.current_stream().cuda_stream if stream is None else stream
    _check(lib.vgtb_spectrum_noalloc(j.size, j.ctypes.data, float(dt), w.size, w.ctypes.data,
                                     float(e0), float(tau0), 1 if subtract_mean else 0,
                                     sig.ctypes.data, eps.ctypes.data, st))
    return sig, eps


class Propagator:
    """One propagation context: device arena, stream and the C handle."""

    def __init__(self, system, dt: float, precision: str = "fp64", rescale_every: int = 50,
                 history_capacity: int = 1024, device: str = "cuda:0", coupling: str = "peierls",
                 propagator: str = "leapfrog", **kernel_options):
        """kernel_options: tile, spmm_variant, spmm_group, graphs, small_path, fused_update
        (make_options)."""
        torch = _torch()
        self._torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        self.n_atoms = int(system.pos.shape[0])
        self.norb = int(system.norb)
        self.n = self.n_atoms * self.norb
        self.n_k = int(np.asarray(system.kpts).shape[0])
        self.precision = precision
        self.options = make_options(dt, precision, rescale_every, history_capacity, coupling,
                                    propagator, **kernel_options)
        s, keep = make_system_struct(system)
        with torch.cuda.device(self.device):
            size = ctypes.c_size_t(0)
            _check(self.lib.vgtb_workspace_size(ctypes.byref(s), ctypes.byref(self.options),
                                                ctypes.byref(size)))
            self.arena = torch.empty(int(size.value) + 256, dtype=torch.uint8, device=self.device)
            base = self.arena.data_ptr()
            aligned = (base + 255) & ~255
            self.stream = torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            _check(self.lib.vgtb_create(ctypes.byref(s), ctypes.byref(self.options), aligned,
                                        int(size.value), self.stream.cuda_stream, ctypes.byref(h)))
        del keep
        self.ctx = h

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            self.lib.vgtb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- calls ---------------------------------------------------------------
    def ground_state(self) -> float:
        gap = ctypes.c_double(0.0)
        _check(self.lib.vgtb_ground_state(self.ctx, ctypes.byref(gap)), self.ctx)
        return float(gap.value)

    def set_density(self, d):
        torch = self._torch
        if isinstance(d, torch.Tensor):
            t = d.to(device=self.device, dtype=torch.complex128).contiguous()
            self._check_shape(t.shape)
            _check(self.lib.vgtb_set_density(self.ctx, t.data_ptr(), 1), self.ctx)
        else:
            a = np.ascontiguousarray(d, dtype=np.complex128)
            self._check_shape(a.shape)
            _check(self.lib.vgtb_set_density(self.ctx, a.ctypes.data, 0), self.ctx)

    def set_coefficients(self, c, occ):
        """Crank-Nicolson contexts: n_k x N x n_states coefficients and n_k x n_states occupations."""
        torch = self._torch
        occ = np.ascontiguousarray(occ, dtype=np.float64)
        if isinstance(c, torch.Tensor):
            t = c.to(device=self.device, dtype=torch.complex128).contiguous()
            shape, ptr, on_dev = tuple(t.shape), t.data_ptr(), 1
        else:
            a = np.ascontiguousarray(c, dtype=np.complex128)
            shape, ptr, on_dev = a.shape, a.ctypes.data, 0
        if len(shape) != 3 or shape[:2] != (self.n_k, self.n) or occ.shape != (self.n_k, shape[2]):
            raise ValueError(f"coefficients must be ({self.n_k}, {self.n}, n_states) with occupations "
                             f"({self.n_k}, n_states); got {shape} and {occ.shape}")
        _check(self.lib.vgtb_set_coefficients(self.ctx, ptr, occ.ctypes.data, int(shape[2]), on_dev),
               self.ctx)

    @property
    def num_states(self) -> int:
        return int(self.lib.vgtb_num_states(self.ctx))

    def get_coefficients(self):
        """(coefficients n_k x N x n_states on the device, occupations n_k x n_states)."""
        torch = self._torch
        ns = self.num_states
        out = torch.empty((self.n_k, self.n, max(ns, 1)), dtype=torch.complex128, device=self.device)
        occ = np.zeros((self.n_k, max(ns, 1)))
        _check(self.lib.vgtb_get_coefficients(self.ctx, out.data_ptr(), occ.ctypes.data, 1), self.ctx)
        return out, occ

    def _check_shape(self, shape):
        if tuple(shape) != (self.n_k, self.n, self.n):
            raise ValueError(f"density must have shape {(self.n_k, self.n, self.n)}, got {tuple(shape)}")

    def set_field_table(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1, 3)
        _check(self.lib.vgtb_set_field_table(self.ctx, a.shape[0], a.ctypes.data), self.ctx)

    def set_field(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(3)
        _check(self.lib.vgtb_set_field(self.ctx, a.ctypes.data), self.ctx)

    def step(self, n_steps: int):
        _check(self.lib.vgtb_step(self.ctx, int(n_steps)), self.ctx)

    def synchronize(self):
        _check(self.lib.vgtb_synchronize(self.ctx), self.ctx)

    @property
    def step_index(self) -> int:
        return int(self.lib.vgtb_step_index(self.ctx))

    def read_observables(self, first: int = 0, count: Optional[int] = None) -> dict:
        if count is None:
            count = self.step_index - first
        j = np.zeros((count, 3))
        e = np.zeros(count)
        tr = np.zeros(count)
        q = np.zeros((count, self.n_atoms))
        _check(self.lib.vgtb_read_observables(self.ctx, first, count, j.ctypes.data, e.ctypes.data,
                                              tr.ctypes.data, q.ctypes.data), self.ctx)
        return {"J": j, "E": e, "trace": tr, "q": q}

    def get_density(self, level: int = 0):
        torch = self._torch
        out = torch.empty((self.n_k, self.n, self.n), dtype=torch.complex128, device=self.device)
        _check(self.lib.vgtb_get_density(self.ctx, int(level), out.data_ptr(), 1), self.ctx)
        return out

    def reference_charges(self) -> np.ndarray:
        z = np.zeros(self.n_atoms)
        _check(self.lib.vgtb_get_reference_charges(self.ctx, z.ctypes.data), self.ctx)
        return z

    def save_state(self) -> bytes:
        size = ctypes.c_size_t(0)
        _check(self.lib.vgtb_state_size(self.ctx, ctypes.byref(size)), self.ctx)
        buf = ctypes.create_string_buffer(int(size.value))
        _check(self.lib.vgtb_save_state(self.ctx, buf, size.value), self.ctx)
        return buf.raw

    def profile(self, enable: bool = True):
        """Start (clearing totals) or stop per-kernel event timing inside vgtb_step."""
        _check(self.lib.vgtb_profile_enable(self.ctx, 1 if enable else 0), self.ctx)

    def profile_read(self) -> dict:
        """{kernel: (total_ms, launches)} since profiling was enabled."""
        out = {}
        for name, kid in KERNELS.items():
            ms = ctypes.c_double(0.0)
            cnt = ctypes.c_int64(0)
            _check(self.lib.vgtb_profile_read(self.ctx, kid, ctypes.byref(ms), ctypes.byref(cnt)), self.ctx)
            out[name] = (float(ms.value), int(cnt.value))
        return out

    def spectrum(self, j, dt: float, omegas, e0: float, tau0: float = 200.0,
                 subtract_mean: bool = True):
        """(sigma, epsilon) of one current component on the GPU (Eqs. 15-16)."""
        j = np.ascontiguousarray(j, dtype=np.float64).reshape(-1)
        w = np.ascontiguousarray(omegas, dtype=np.float64).reshape(-1)
        sig = np.zeros(w.size, dtype=np.complex128)
        eps = np.zeros(w.size, dtype=np.complex128)
        _check(self.lib.vgtb_spectrum(self.ctx, j.size, j.ctypes.data, float(dt), w.size, w.ctypes.data,
                                      float(e0), float(tau0), 1 if subtract_mean else 0,
                                      sig.ctypes.data, eps.ctypes.data), self.ctx)
        return sig, eps

    def autotune(self, reps: int = 5) -> dict:
        """Time the kernel variants on this context and keep the fastest (vgtb_autotune)."""
        t = VgtbTuning()
        _check(self.lib.vgtb_autotune(self.ctx, int(reps), ctypes.byref(t)), self.ctx)
        return {"spmm_variant": t.spmm_variant, "gemm_tile": t.gemm_tile,
                "spmm_ms": {int(t.spmm_candidates[i]): float(t.spmm_ms[i]) for i in range(t.n_spmm)},
                "gemm_ms": {int(t.gemm_candidates[i]): float(t.gemm_ms[i]) for i in range(t.n_gemm)}}

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self.lib.vgtb_load_state(self.ctx, buf, len(blob)), self.ctx)


class Group:
    """Several small-system Propagators stepped together, one launch per block
    of steps with a workgroup per (system, k-point) (vgtb_group_*).  The
    propagators must outlive the group; read each one's results as usual."""

    def __init__(self, propagators):
        self.lib = load_library()
        self.members = list(propagators)
        arr = (ctypes.c_void_p * len(self.members))(*[p.ctx for p in self.members])
        h = ctypes.c_void_p()
        _check(self.lib.vgtb_group_create(arr, len(self.members), ctypes.byref(h)))
        self.grp = h

    def step(self, n_steps: int):
        _check(self.lib.vgtb_group_step(self.grp, int(n_steps)))

    def close(self):
        if getattr(self, "grp", None):
            self.lib.vgtb_group_destroy(self.grp)
            self.grp = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """Several propagations overlapped on one GPU (vgtb_server_*): one device
    arena of arena_bytes, max_active slots (streams)."""

    def __init__(self, arena_bytes: int, max_active: int = 8, device: str = "cuda:0"):
        torch = _torch()
        self.lib = load_library()
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=self.device)
            aligned = (self.arena.data_ptr() + 255) & ~255
            h = ctypes.c_void_p()
            _check(self.lib.vgtb_server_create(aligned, int(arena_bytes), int(max_active),
                                               ctypes.byref(h)))
        self.srv = h

    def run(self, requests):
        """requests: dicts with system, dt, n_steps, field (n x 3), arrival_s and optionally
        precision (default fp16x3), rescale_every, coupling, omegas, e0, tau0.  Returns
        (results, summary): per request {status, message, J (n_steps x 3), sigma, slot,
        workspace_bytes, arrival_s, admitted_s, ready_s, finished_s}, and the run's
        {makespan_s, k_steps, k_steps_per_s, peak_bytes, peak_active}."""
        n = len(requests)
        reqs = (VgtbRequest * max(n, 1))()
        stats = (VgtbRequestStats * max(n, 1))()
        summ = VgtbServerStats()
        keep, outs = [], []
        for i, r in enumerate(requests):
            s, arrs = make_system_struct(r["system"])
            field = np.ascontiguousarray(r["field"], dtype=np.float64).reshape(-1, 3)
            om = np.ascontiguousarray(r.get("omegas", np.zeros(0)), dtype=np.float64)
            jo = np.zeros((int(r["n_steps"]), 3))
            so = np.zeros(om.size, dtype=np.complex128)
            keep.append((s, arrs, field, om))
            outs.append((jo, so))
            q = reqs[i]
            q.system = ctypes.cast(ctypes.pointer(s), ctypes.c_void_p)
            q.options = make_options(r["dt"], r.get("precision", "fp16x3"),
                                     r.get("rescale_every", 50), 1, r.get("coupling", "peierls"))
            q.n_steps = int(r["n_steps"])
            q.n_field = field.shape[0]
            q.field = field.ctypes.data
            q.n_omega = om.size
            q.omega = om.ctypes.data if om.size else None
            q.e0 = float(r.get("e0", 1.0))
            q.tau0 = float(r.get("tau0", 200.0))
            q.arrival_s = float(r.get("arrival_s", 0.0))
            q.j_out = jo.ctypes.data
            q.sigma_out = so.ctypes.data if om.size else None
        _check(self.lib.vgtb_server_run(self.srv, n, reqs, stats, ctypes.byref(summ)))
        results = []
        for i in range(n):
            st = stats[i]
            results.append({"status": int(st.status), "message": st.message.decode(errors="replace"),
                            "J": outs[i][0], "sigma": outs[i][1],
                            "slot": int(st.slot), "workspace_bytes": int(st.workspace_bytes),
                            "arrival_s": st.arrival_s, "admitted_s": st.admitted_s,
                            "ready_s": st.ready_s, "finished_s": st.finished_s})
        del keep
        summary = {"makespan_s": summ.makespan_s, "k_steps": summ.k_steps,
                   "k_steps_per_s": summ.k_steps_per_s, "peak_bytes": int(summ.peak_bytes),
                   "peak_active": int(summ.peak_active)}
        return results, summary

    def close(self):
        if getattr(self, "srv", None):
            self.lib.vgtb_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
