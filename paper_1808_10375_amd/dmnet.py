"""Thin ctypes binding of the warm-start network in libdm (include/dmnet.h).

Same rules as dm.py: C names, argument marshalling only, torch tensors for
device memory and the current torch stream as the hipStream_t; the library
must be built, there is no other implementation behind these calls.
"""
from __future__ import annotations

import ctypes
from typing import Optional

from . import dm
from .dm import DMError, DM_OK, _ptr, _stream_handle

DMNET_FLAG_FP32_WEIGHTS = 1

EXPORTED = [
    "dmnet_n_params", "dmnet_workspace_bytes", "dmnet_create", "dmnet_set_params",
    "dmnet_get_params", "dmnet_forward", "dmnet_loss_grad", "dmnet_train_step",
    "dmnet_preprocess", "dmnet_patches", "dmnet_free", "dmnet_last_error",
]


class dmnet_desc(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("size", ctypes.c_int32),
                ("base_ch", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_int32)]


_bound = None


def lib():
    global _bound
    L = dm.lib()
    if _bound is L:
        return L
    vp, i32, u64, fp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_void_p
    pd = ctypes.POINTER(dmnet_desc)
    L.dmnet_n_params.argtypes = [pd]
    L.dmnet_n_params.restype = u64
    L.dmnet_workspace_bytes.argtypes = [pd]
    L.dmnet_workspace_bytes.restype = u64
    L.dmnet_create.argtypes = [ctypes.POINTER(vp), pd, vp, u64, vp]
    L.dmnet_create.restype = i32
    L.dmnet_set_params.argtypes = [vp, fp]
    L.dmnet_set_params.restype = i32
    L.dmnet_get_params.argtypes = [vp, fp]
    L.dmnet_get_params.restype = i32
    L.dmnet_forward.argtypes = [vp, fp, fp, i32]
    L.dmnet_forward.restype = i32
    L.dmnet_loss_grad.argtypes = [vp, fp, fp, i32, fp, ctypes.POINTER(ctypes.c_float)]
    L.dmnet_loss_grad.restype = i32
    L.dmnet_train_step.argtypes = [vp, fp, fp, i32, ctypes.POINTER(ctypes.c_float)]
    L.dmnet_train_step.restype = i32
    L.dmnet_preprocess.argtypes = [vp, fp, i32, i32, fp]
    L.dmnet_preprocess.restype = i32
    L.dmnet_patches.argtypes = [vp, fp, i32, vp]
    L.dmnet_patches.restype = i32
    L.dmnet_free.argtypes = [vp]
    L.dmnet_free.restype = None
    L.dmnet_last_error.argtypes = [vp]
    L.dmnet_last_error.restype = ctypes.c_char_p
    _bound = L
    return L


def make_desc(batch, size=64, base_ch=32, levels=4, lr=1e-3, beta1=0.9, beta2=0.999,
              eps=1e-8, flags=0) -> dmnet_desc:
    return dmnet_desc(int(batch), int(size), int(base_ch), int(levels), float(lr),
                      float(beta1), float(beta2), float(eps), int(flags), 0)


def dmnet_last_error(net) -> str:
    return lib().dmnet_last_error(net).decode()


def _check(status, net=None):
    if status != DM_OK:
        msg = dmnet_last_error(net) if net else ""
        raise DMError(status, f"{dm.dm_status_str(status)}: {msg}")


def dmnet_n_params(desc: dmnet_desc) -> int:
    return int(lib().dmnet_n_params(ctypes.byref(desc)))


def dmnet_workspace_bytes(desc: dmnet_desc) -> int:
    return int(lib().dmnet_workspace_bytes(ctypes.byref(desc)))


def dmnet_create(desc: dmnet_desc, workspace, stream=None):
    net = ctypes.c_void_p()
    st = lib().dmnet_create(ctypes.byref(net), ctypes.byref(desc), _ptr(workspace),
                            int(workspace.numel() * workspace.element_size()),
                            _stream_handle(stream))
    _check(st)
    return net


def dmnet_set_params(net, params):
    _check(lib().dmnet_set_params(net, _ptr(params)), net)


def dmnet_get_params(net, params):
    _check(lib().dmnet_get_params(net, _ptr(params)), net)


def dmnet_forward(net, x, y, n: int):
    _check(lib().dmnet_forward(net, _ptr(x), _ptr(y), int(n)), net)


def dmnet_loss_grad(net, x, target, n: int, grads=None) -> float:
    loss = ctypes.c_float()
    _check(lib().dmnet_loss_grad(net, _ptr(x), _ptr(target), int(n), _ptr(grads),
                                 ctypes.byref(loss)), net)
    return float(loss.value)


def dmnet_train_step(net, x, target, n: int, want_loss: bool = True) -> Optional[float]:
    loss = ctypes.c_float()
    _check(lib().dmnet_train_step(net, _ptr(x), _ptr(target), int(n),
                                  ctypes.byref(loss) if want_loss else None), net)
    return float(loss.value) if want_loss else None


def dmnet_preprocess(net, I, n: int, frame: int, x):
    _check(lib().dmnet_preprocess(net, _ptr(I), int(n), int(frame), _ptr(x)), net)


def dmnet_patches(net, y, n: int, patches):
    _check(lib().dmnet_patches(net, _ptr(y), int(n), _ptr(patches)), net)


def dmnet_free(net):
    if net:
        lib().dmnet_free(net)


class DMNet:
    """Owns the workspace and handle of one network."""

    def __init__(self, batch, size=64, base_ch=32, levels=4, lr=1e-3, flags=0,
                 device=None, stream=None):
        import torch
        self.desc = make_desc(batch, size, base_ch, levels, lr=lr, flags=flags)
        nbytes = dmnet_workspace_bytes(self.desc)
        if nbytes == 0:
            raise DMError(dm.DM_E_ARG, "invalid network description")
        self.device = torch.device(device or "cuda:0")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.n_params = dmnet_n_params(self.desc)
        self.stream = stream
        self.net = dmnet_create(self.desc, self.workspace, stream)

    def set_params(self, flat):
        import torch
        p = torch.as_tensor(flat, dtype=torch.float32).to(self.device).contiguous()
        if p.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        dmnet_set_params(self.net, p)
        torch.cuda.synchronize(self.device)

    def params(self):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        dmnet_get_params(self.net, out)
        return out

    def forward(self, x):
        import torch
        x = x.contiguous()
        n, _, s, _ = x.shape
        y = torch.empty((n, 2, s, s), dtype=torch.float32, device=self.device)
        dmnet_forward(self.net, x, y, n)
        return y

    def loss_grad(self, x, target):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        loss = dmnet_loss_grad(self.net, x.contiguous(), target.contiguous(), x.shape[0], g)
        return loss, g

    def train_step(self, x, target, want_loss=True):
        return dmnet_train_step(self.net, x.contiguous(), target.contiguous(), x.shape[0],
                                want_loss)

    def preprocess(self, I):
        import torch
        I = I.contiguous()
        n, f, _ = I.shape
        x = torch.empty((n, 1, f // 2, f // 2), dtype=torch.float32, device=self.device)
        dmnet_preprocess(self.net, I, n, f, x)
        return x

    def patches(self, y):
        import torch
        y = y.contiguous()
        n, _, s, _ = y.shape
        out = torch.empty((n, 2 * s, 2 * s), dtype=torch.complex64, device=self.device)
        dmnet_patches(self.net, y, n, out)
        return out

    def free(self):
        if getattr(self, "net", None):
            dmnet_free(self.net)
            self.net = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
