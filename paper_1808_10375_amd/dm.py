"""Thin ctypes binding of libdm (include/dm.h) over torch device buffers.

Every function keeps the C name and only marshals arguments: torch tensors
become device pointers, the current torch stream becomes the hipStream_t.
All arithmetic runs in libdm's HIP kernels; when the library is missing this
module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdm.so")

DM_OK = 0
DM_E_ARG = -1
DM_E_UNSUPPORTED = -2
DM_E_BOUNDS = -3
DM_E_WORKSPACE = -4
DM_E_HIP = -5
DM_E_STATE = -6
DM_E_NUMERIC = -7

DM_FP32_FFT = 0
DM_BF16X3_DFT = 1
DM_FLAG_MULTIPASS = 1   # force the three-kernel transform path (always for F = 256)
DM_FLAG_PHASE_TIMING = 2  # HIP events around every phase launch
DM_FLAG_GRAPH = 4         # capture one iteration into a hipGraph and replay it
DM_FLAG_PSI_ERROR_LAST = 8  # eps_psi in the last iteration of a call only (psi-free update)
DM_FLAG_PROBE_FIRST = 16  # probe update before the object update (the order before Section III's swap)
DM_VIEWS_FUSED = 0            # dm_tuning.view_path values
DM_VIEWS_THREE_KERNEL = 1
DM_VIEWS_STREAMED = 2
DM_VIEWS_STREAMED_CACHED = 3
DM_VIEWS_STREAMED_MERGED = 4
DM_VIEWS_STREAMED_WIDE = 5
DM_MAX_MODES = 16
DM_MAX_OBJ_MODES = 4
DM_MAX_PAIRS = 32
DM_MAX_PROBE_CHUNKS = 64
PHASES = ["views", "object", "probe_partial", "probe_final", "errors"]

EXPORTED = [
    "dm_workspace_bytes", "dm_init", "dm_iterate", "dm_get_object", "dm_get_probe",
    "dm_error", "dm_error_history", "dm_iterations", "dm_get_state", "dm_set_state",
    "dm_free", "dm_status_str", "dm_last_error", "dm_phase_times",
    "dm_batch_workspace_bytes", "dm_batch_init", "dm_n_scans", "dm_scan_get_object",
    "dm_scan_get_probe", "dm_scan_error_history", "dm_get_tuning", "dm_set_tuning",
    "dm_autotune", "dm_warm_start", "dm_scan_warm_start", "dm_mode_power",
    "dm_scan_mode_power", "dm_orthogonalize_modes", "dm_scan_orthogonalize_modes",
    "dm_orthogonalize_modes_noalloc",
]


class dm_desc(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("frame", ctypes.c_int32),
                ("n_modes", ctypes.c_int32), ("obj_h", ctypes.c_int32),
                ("obj_w", ctypes.c_int32), ("beta", ctypes.c_float),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("n_obj_modes", ctypes.c_int32)]


class dm_errors(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("eps_psi", ctypes.c_float),
                ("eps_obj", ctypes.c_float), ("eps_probe", ctypes.c_float),
                ("eps_probe_mode", ctypes.c_float * DM_MAX_MODES)]

    def to_dict(self, n_modes: int) -> dict:
        return {"iter": self.iter, "eps_psi": self.eps_psi, "eps_obj": self.eps_obj,
                "eps_probe": self.eps_probe,
                "eps_probe_mode": [self.eps_probe_mode[k] for k in range(n_modes)]}


class dm_tuning(ctypes.Structure):
    _fields_ = [("obj_tile", ctypes.c_int32), ("probe_chunks", ctypes.c_int32),
                ("view_path", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def to_dict(self) -> dict:
        return {"obj_tile": self.obj_tile, "probe_chunks": self.probe_chunks,
                "view_path": self.view_path}


class DMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """The loaded libdm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1808_10375_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    L.dm_workspace_bytes.argtypes = [ctypes.POINTER(dm_desc)]
    L.dm_workspace_bytes.restype = u64
    L.dm_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(dm_desc), vp,
                          ctypes.POINTER(i32), vp, vp, vp, u64, vp]
    L.dm_init.restype = i32
    L.dm_iterate.argtypes = [vp, i32]
    L.dm_iterate.restype = i32
    L.dm_get_object.argtypes = [vp, vp]
    L.dm_get_object.restype = i32
    L.dm_get_probe.argtypes = [vp, vp]
    L.dm_get_probe.restype = i32
    L.dm_error.argtypes = [vp, ctypes.POINTER(dm_errors)]
    L.dm_error.restype = i32
    L.dm_error_history.argtypes = [vp, i32, i32, ctypes.POINTER(dm_errors)]
    L.dm_error_history.restype = i32
    L.dm_iterations.argtypes = [vp]
    L.dm_iterations.restype = i32
    L.dm_get_state.argtypes = [vp, vp, vp, vp, ctypes.POINTER(i32)]
    L.dm_get_state.restype = i32
    L.dm_set_state.argtypes = [vp, vp, vp, vp, i32]
    L.dm_set_state.restype = i32
    L.dm_phase_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]
    L.dm_phase_times.restype = i32
    L.dm_batch_workspace_bytes.argtypes = [i32, ctypes.POINTER(dm_desc)]
    L.dm_batch_workspace_bytes.restype = u64
    L.dm_batch_init.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(dm_desc),
                                ctypes.POINTER(vp), ctypes.POINTER(ctypes.POINTER(i32)),
                                ctypes.POINTER(vp), ctypes.POINTER(vp), vp, u64, vp]
    L.dm_batch_init.restype = i32
    L.dm_n_scans.argtypes = [vp]
    L.dm_n_scans.restype = i32
    L.dm_scan_get_object.argtypes = [vp, i32, vp]
    L.dm_scan_get_object.restype = i32
    L.dm_scan_get_probe.argtypes = [vp, i32, vp]
    L.dm_scan_get_probe.restype = i32
    L.dm_scan_error_history.argtypes = [vp, i32, i32, i32, ctypes.POINTER(dm_errors)]
    L.dm_scan_error_history.restype = i32
    L.dm_mode_power.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.dm_mode_power.restype = i32
    L.dm_scan_mode_power.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
    L.dm_scan_mode_power.restype = i32
    L.dm_orthogonalize_modes.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.dm_orthogonalize_modes.restype = i32
    L.dm_scan_orthogonalize_modes.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
    L.dm_scan_orthogonalize_modes.restype = i32
    L.dm_orthogonalize_modes_noalloc.argtypes = [vp, vp, i32, i32, i32, vp, vp]
    L.dm_orthogonalize_modes_noalloc.restype = i32
    L.dm_get_tuning.argtypes = [vp, ctypes.POINTER(dm_tuning)]
    L.dm_get_tuning.restype = i32
    L.dm_set_tuning.argtypes = [vp, ctypes.POINTER(dm_tuning)]
    L.dm_set_tuning.restype = i32
    L.dm_autotune.argtypes = [vp, i32, ctypes.c_char_p, ctypes.POINTER(dm_tuning)]
    L.dm_autotune.restype = i32
    L.dm_warm_start.argtypes = [vp, vp]
    L.dm_warm_start.restype = i32
    L.dm_scan_warm_start.argtypes = [vp, i32, vp]
    L.dm_scan_warm_start.restype = i32
    L.dm_free.argtypes = [vp]
    L.dm_free.restype = None
    L.dm_status_str.argtypes = [i32]
    L.dm_status_str.restype = ctypes.c_char_p
    L.dm_last_error.argtypes = [vp]
    L.dm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def make_desc(n_frames, frame, n_modes, obj_h, obj_w, beta=0.8, precision=DM_FP32_FFT,
              flags=0, n_obj_modes=0) -> dm_desc:
    return dm_desc(int(n_frames), int(frame), int(n_modes), int(obj_h), int(obj_w),
                   float(beta), int(precision), int(flags), int(n_obj_modes))


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    h = getattr(stream, "cuda_stream", stream)
    return int(h) if h else None


def dm_status_str(status: int) -> str:
    return lib().dm_status_str(int(status)).decode()


def dm_last_error(ctx=None) -> str:
    return lib().dm_last_error(ctx).decode()


def _check(status: int, ctx=None):
    if status != DM_OK:
        raise DMError(status, f"{dm_status_str(status)}: {dm_last_error(ctx)}")


def dm_workspace_bytes(desc: dm_desc) -> int:
    return int(lib().dm_workspace_bytes(ctypes.byref(desc)))


def dm_init(desc: dm_desc, I, pos, probe0, object0, workspace, stream=None):
    """Returns the opaque context handle.  I, probe0, object0 and workspace are
    torch device tensors; pos is a host int32 array [N][2]."""
    pos = np.ascontiguousarray(np.asarray(pos, dtype=np.int32))
    if pos.shape != (desc.n_frames, 2):
        raise ValueError(f"pos must have shape ({desc.n_frames}, 2)")
    ctx = ctypes.c_void_p()
    st = lib().dm_init(ctypes.byref(ctx), ctypes.byref(desc), _ptr(I),
                       pos.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(probe0),
                       _ptr(object0), _ptr(workspace), int(workspace.numel()
                                                            * workspace.element_size()),
                       _stream_handle(stream))
    _check(st, None)
    return ctx


def dm_iterate(ctx, n_iter: int):
    _check(lib().dm_iterate(ctx, int(n_iter)), ctx)


def dm_get_object(ctx, dst):
    _check(lib().dm_get_object(ctx, _ptr(dst)), ctx)


def dm_get_probe(ctx, dst):
    _check(lib().dm_get_probe(ctx, _ptr(dst)), ctx)


def dm_error(ctx) -> dm_errors:
    out = dm_errors()
    _check(lib().dm_error(ctx, ctypes.byref(out)), ctx)
    return out


def dm_error_history(ctx, first: int, count: int):
    arr = (dm_errors * max(count, 1))()
    _check(lib().dm_error_history(ctx, int(first), int(count), arr), ctx)
    return [arr[i] for i in range(count)]


def dm_scan_mode_power(ctx, scan: int, n_modes: int):
    arr = (ctypes.c_double * n_modes)()
    _check(lib().dm_scan_mode_power(ctx, int(scan), arr), ctx)
    return [float(arr[i]) for i in range(n_modes)]


def dm_mode_power(ctx, n_modes: int):
    arr = (ctypes.c_double * n_modes)()
    _check(lib().dm_mode_power(ctx, arr), ctx)
    return [float(arr[i]) for i in range(n_modes)]


def dm_scan_orthogonalize_modes(ctx, scan: int, n_modes: int, want_power: bool = True):
    """Orthogonal probe modes (the views mixed alike); the new modes' powers
    (descending) if want_power, else None without synchronising."""
    arr = (ctypes.c_double * n_modes)() if want_power else None
    _check(lib().dm_scan_orthogonalize_modes(ctx, int(scan), arr), ctx)
    return [float(arr[i]) for i in range(n_modes)] if want_power else None


def dm_orthogonalize_modes(ctx, n_modes: int, want_power: bool = True):
    arr = (ctypes.c_double * n_modes)() if want_power else None
    _check(lib().dm_orthogonalize_modes(ctx, arr), ctx)
    return [float(arr[i]) for i in range(n_modes)] if want_power else None


def dm_orthogonalize_modes_noalloc(probe, psi=None, power=None, stream=None):
    """Context-free orthogonalisation on caller buffers (no allocation in the
    library): probe [M][F][F] and psi [N][M][F][F] complex64 device tensors,
    mixed in place; power: optional float64 device tensor [M]."""
    m, f = int(probe.shape[0]), int(probe.shape[-1])
    n = 0 if psi is None else int(psi.shape[0])
    _check(lib().dm_orthogonalize_modes_noalloc(_ptr(probe), _ptr(psi), n, m, f, _ptr(power),
                                                _stream_handle(stream)), None)


def dm_iterations(ctx) -> int:
    return int(lib().dm_iterations(ctx))


def dm_get_state(ctx, psi_dst=None, probe_dst=None, object_dst=None) -> int:
    it = ctypes.c_int32()
    _check(lib().dm_get_state(ctx, _ptr(psi_dst), _ptr(probe_dst), _ptr(object_dst),
                              ctypes.byref(it)), ctx)
    return int(it.value)


def dm_set_state(ctx, psi, probe, obj, iteration: int = 0):
    _check(lib().dm_set_state(ctx, _ptr(psi), _ptr(probe), _ptr(obj), int(iteration)), ctx)


def dm_phase_times(ctx):
    """(dict phase -> milliseconds, iterations) since the previous call."""
    arr = (ctypes.c_double * len(PHASES))()
    n = ctypes.c_int32()
    _check(lib().dm_phase_times(ctx, arr, ctypes.byref(n)), ctx)
    return {p: arr[i] for i, p in enumerate(PHASES)}, int(n.value)


def dm_batch_workspace_bytes(descs) -> int:
    arr = (dm_desc * len(descs))(*descs)
    return int(lib().dm_batch_workspace_bytes(len(descs), arr))


def dm_batch_init(descs, Is, poss, probe0s, object0s, workspace, stream=None):
    """Context for a batch of scans (same F, M, flags); per-scan lists of
    torch device tensors and host position arrays."""
    n = len(descs)
    arr = (dm_desc * n)(*descs)
    poss = [np.ascontiguousarray(np.asarray(p, dtype=np.int32)) for p in poss]
    for d, p in zip(descs, poss):
        if p.shape != (d.n_frames, 2):
            raise ValueError("positions must have shape (n_frames, 2)")
    vp = ctypes.c_void_p
    I_arr = (vp * n)(*[_ptr(t) for t in Is])
    P_arr = (vp * n)(*[_ptr(t) for t in probe0s])
    O_arr = (vp * n)(*[_ptr(t) for t in object0s])
    pos_arr = (ctypes.POINTER(ctypes.c_int32) * n)(
        *[p.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) for p in poss])
    ctx = ctypes.c_void_p()
    st = lib().dm_batch_init(ctypes.byref(ctx), n, arr, I_arr, pos_arr, P_arr, O_arr,
                             _ptr(workspace), int(workspace.numel() * workspace.element_size()),
                             _stream_handle(stream))
    _check(st, None)
    return ctx


def dm_n_scans(ctx) -> int:
    return int(lib().dm_n_scans(ctx))


def dm_scan_get_object(ctx, scan: int, dst):
    _check(lib().dm_scan_get_object(ctx, int(scan), _ptr(dst)), ctx)


def dm_scan_get_probe(ctx, scan: int, dst):
    _check(lib().dm_scan_get_probe(ctx, int(scan), _ptr(dst)), ctx)


def dm_scan_error_history(ctx, scan: int, first: int, count: int):
    arr = (dm_errors * max(count, 1))()
    _check(lib().dm_scan_error_history(ctx, int(scan), int(first), int(count), arr), ctx)
    return [arr[i] for i in range(count)]


def dm_get_tuning(ctx) -> dm_tuning:
    t = dm_tuning()
    _check(lib().dm_get_tuning(ctx, ctypes.byref(t)), ctx)
    return t


def dm_set_tuning(ctx, obj_tile: int, probe_chunks: int, view_path: int = 0):
    t = dm_tuning(int(obj_tile), int(probe_chunks), int(view_path), 0)
    _check(lib().dm_set_tuning(ctx, ctypes.byref(t)), ctx)


def dm_autotune(ctx, reps: int = 5, cache_path: Optional[str] = None) -> dm_tuning:
    t = dm_tuning()
    _check(lib().dm_autotune(ctx, int(reps), cache_path.encode() if cache_path else None,
                             ctypes.byref(t)), ctx)
    return t


def dm_warm_start(ctx, patches):
    _check(lib().dm_warm_start(ctx, _ptr(patches)), ctx)


def dm_scan_warm_start(ctx, scan: int, patches):
    _check(lib().dm_scan_warm_start(ctx, int(scan), _ptr(patches)), ctx)


def dm_free(ctx):
    if ctx:
        lib().dm_free(ctx)


class DMContext:
    """Owns the torch buffers of one reconstruction and its context handle."""

    def __init__(self, I, pos, probe0, object0, beta=0.8, precision=DM_FP32_FFT, flags=0,
                 stream=None):
        import torch
        if I.dtype != torch.float32 or not I.is_cuda:
            raise TypeError("I must be a float32 CUDA tensor [N][F][F]")
        n, f, f2 = I.shape
        m = probe0.shape[0]
        # object [H][W], or [L][H][W] with L object modes
        n_obj = object0.shape[0] if object0.dim() == 3 else 0
        h, w = object0.shape[-2:]
        self.desc = make_desc(n, f, m, h, w, beta, precision, flags, n_obj)
        nbytes = dm_workspace_bytes(self.desc)
        if nbytes == 0:
            raise DMError(DM_E_ARG, "invalid problem description")
        self.device = I.device
        self.I = I.contiguous()
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._p0 = probe0.to(self.device, torch.complex64).contiguous()
        self._o0 = object0.to(self.device, torch.complex64).contiguous()
        self.pos = np.ascontiguousarray(np.asarray(pos, dtype=np.int32))
        self.stream = stream
        self.ctx = dm_init(self.desc, self.I, self.pos, self._p0, self._o0, self.workspace,
                           stream)

    @property
    def n_obj_modes(self):
        return max(1, self.desc.n_obj_modes)

    def _obj_shape(self):
        d = self.desc
        return ((d.obj_h, d.obj_w) if d.n_obj_modes <= 1
                else (d.n_obj_modes, d.obj_h, d.obj_w))

    @property
    def n_modes(self):
        return self.desc.n_modes

    def iterate(self, n: int = 1):
        dm_iterate(self.ctx, n)

    def object(self):
        import torch
        out = torch.empty(self._obj_shape(), dtype=torch.complex64, device=self.device)
        dm_get_object(self.ctx, out)
        return out

    def probe(self):
        import torch
        f = self.desc.frame
        out = torch.empty((self.desc.n_modes, f, f), dtype=torch.complex64, device=self.device)
        dm_get_probe(self.ctx, out)
        return out

    def errors(self) -> dict:
        return dm_error(self.ctx).to_dict(self.n_modes)

    def error_history(self, first: int = 1, count: Optional[int] = None):
        if count is None:
            count = dm_iterations(self.ctx) - first + 1
        return [e.to_dict(self.n_modes) for e in dm_error_history(self.ctx, first, count)]

    def mode_power(self):
        """sum over pixels of |P_k|^2 for every probe mode (synchronises)"""
        return dm_mode_power(self.ctx, self.n_modes)

    def orthogonalize_modes(self, want_power: bool = True):
        """eigenmodes of the probe modes' overlap matrix, views mixed alike;
        returns their powers (descending) if want_power"""
        return dm_orthogonalize_modes(self.ctx, self.n_modes, want_power)

    def state(self):
        import torch
        d = self.desc
        psi = torch.empty((d.n_frames, d.n_modes * self.n_obj_modes, d.frame, d.frame),
                          dtype=torch.complex64, device=self.device)
        P = torch.empty((d.n_modes, d.frame, d.frame), dtype=torch.complex64, device=self.device)
        O = torch.empty(self._obj_shape(), dtype=torch.complex64, device=self.device)
        it = dm_get_state(self.ctx, psi, P, O)
        return psi, P, O, it

    def set_state(self, psi, P, O, iteration: int = 0):
        import torch
        self._state_keep = [t.to(self.device, torch.complex64).contiguous() for t in (psi, P, O)]
        dm_set_state(self.ctx, *self._state_keep, iteration)

    def phase_times(self):
        return dm_phase_times(self.ctx)

    def warm_start(self, patches):
        """Stitch complex64 patches [N][F][F] (device) into the object."""
        import torch
        self._patches = patches.to(self.device, torch.complex64).contiguous()
        dm_warm_start(self.ctx, self._patches)

    def tuning(self) -> dict:
        return dm_get_tuning(self.ctx).to_dict()

    def set_tuning(self, obj_tile, probe_chunks, view_path=0):
        dm_set_tuning(self.ctx, obj_tile, probe_chunks, view_path)

    def autotune(self, reps=5, cache_path=None) -> dict:
        return dm_autotune(self.ctx, reps, cache_path).to_dict()

    @property
    def iterations(self) -> int:
        return dm_iterations(self.ctx)

    def free(self):
        if getattr(self, "ctx", None):
            dm_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class DMBatch:
    """Many scans (same frame size and mode count) advanced together: one
    launch per phase per iteration for the whole batch."""

    def __init__(self, scans, beta=0.8, flags=0, stream=None, device=None):
        """scans: list of dicts with numpy or torch arrays I, pos, P0, O0."""
        import torch
        self.device = torch.device(device or "cuda:0")
        self.stream = stream
        self._keep = []
        descs, Is, poss, P0s, O0s = [], [], [], [], []
        for sc in scans:
            I = torch.as_tensor(sc["I"], dtype=torch.float32).to(self.device).contiguous()
            P0 = torch.as_tensor(sc["P0"]).to(self.device, torch.complex64).contiguous()
            O0 = torch.as_tensor(sc["O0"]).to(self.device, torch.complex64).contiguous()
            n, f, _ = I.shape
            descs.append(make_desc(n, f, P0.shape[0], O0.shape[0], O0.shape[1],
                                   sc.get("beta", beta), DM_FP32_FFT, flags))
            Is.append(I); P0s.append(P0); O0s.append(O0)
            poss.append(np.asarray(sc["pos"], dtype=np.int32))
        self.descs = descs
        nbytes = dm_batch_workspace_bytes(descs)
        if nbytes == 0:
            raise DMError(DM_E_ARG, "invalid batch description")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._keep = [Is, P0s, O0s]
        self.ctx = dm_batch_init(descs, Is, poss, P0s, O0s, self.workspace, stream)

    @property
    def n_scans(self) -> int:
        return dm_n_scans(self.ctx)

    def iterate(self, n: int = 1):
        dm_iterate(self.ctx, n)

    def object(self, scan: int):
        import torch
        d = self.descs[scan]
        out = torch.empty((d.obj_h, d.obj_w), dtype=torch.complex64, device=self.device)
        dm_scan_get_object(self.ctx, scan, out)
        return out

    def probe(self, scan: int):
        import torch
        d = self.descs[scan]
        out = torch.empty((d.n_modes, d.frame, d.frame), dtype=torch.complex64,
                          device=self.device)
        dm_scan_get_probe(self.ctx, scan, out)
        return out

    def error_history(self, scan: int, first: int = 1, count: Optional[int] = None):
        if count is None:
            count = dm_iterations(self.ctx) - first + 1
        m = self.descs[scan].n_modes
        return [e.to_dict(m) for e in dm_scan_error_history(self.ctx, scan, first, count)]

    def mode_power(self, scan: int):
        return dm_scan_mode_power(self.ctx, scan, self.descs[scan].n_modes)

    def tuning(self) -> dict:
        return dm_get_tuning(self.ctx).to_dict()

    def set_tuning(self, obj_tile, probe_chunks, view_path=0):
        dm_set_tuning(self.ctx, obj_tile, probe_chunks, view_path)

    def autotune(self, reps=5, cache_path=None) -> dict:
        return dm_autotune(self.ctx, reps, cache_path).to_dict()

    def warm_start(self, scan: int, patches):
        """Stitch complex64 patches [N_s][F][F] (device) into scan's object."""
        import torch
        p = patches.to(self.device, torch.complex64).contiguous()
        self._keep.append(p)
        dm_scan_warm_start(self.ctx, scan, p)

    @property
    def iterations(self) -> int:
        return dm_iterations(self.ctx)

    def free(self):
        if getattr(self, "ctx", None):
            dm_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
