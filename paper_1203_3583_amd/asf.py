"""Thin ctypes binding of libasf.so (the C ABI in include/asf.h).

Argument marshalling only: torch tensors supply device memory and the stream,
every step of the computation runs in the library's HIP kernels.  There is no
CPU fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libasf.so")

ASF_OK = 0
ASF_EINVAL = -1
ASF_EDOMAIN = -2
ASF_ENOMEM = -3
ASF_EHIP = -4
ASF_ESIZE = -5
ASF_ENOSYS = -6

ASF_FFT_FP32 = 0
ASF_FFT_SPLIT_FP16 = 1
ASF_INCIDENT_NONE = 2

STAGES = ("bin", "scan", "scatter", "spread", "fft_pass1", "fft_pass2",
          "adj_fft_pass2", "adj_fft_pass1", "interp")

_CODES = {ASF_EINVAL: "EINVAL", ASF_EDOMAIN: "EDOMAIN", ASF_ENOMEM: "ENOMEM", ASF_EHIP: "EHIP",
          ASF_ESIZE: "ESIZE", ASF_ENOSYS: "ENOSYS"}


class AsfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"asf error {code} ({_CODES.get(code, '?')}): {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("z0", ctypes.c_double), ("p2x", ctypes.c_double),
                ("p2y", ctypes.c_double), ("mx", ctypes.c_int32), ("my", ctypes.c_int32),
                ("tol", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("n_src", ctypes.c_int64), ("mx", ctypes.c_int32), ("my", ctypes.c_int32),
                ("nfx", ctypes.c_int32), ("nfy", ctypes.c_int32), ("w", ctypes.c_int32),
                ("beta", ctypes.c_double), ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("ntiles", ctypes.c_int32),
                ("slot_cap", ctypes.c_int64), ("col_batch", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("off_status", ctypes.c_size_t), ("off_tile_start", ctypes.c_size_t),
                ("off_cell", ctypes.c_size_t), ("off_frac", ctypes.c_size_t),
                ("off_phase", ctypes.c_size_t), ("off_perm", ctypes.c_size_t),
                ("off_fine", ctypes.c_size_t), ("off_mid", ctypes.c_size_t),
                ("ws_bytes", ctypes.c_size_t), ("off_cursor", ctypes.c_size_t),
                ("off_slab", ctypes.c_size_t), ("off_split", ctypes.c_size_t),
                ("off_split_meta", ctypes.c_size_t), ("off_slot_owner", ctypes.c_size_t),
                ("split_slots", ctypes.c_uint32), ("off_live", ctypes.c_size_t),
                ("skip_empty", ctypes.c_uint32), ("mid_panel", ctypes.c_int32)]


class LineParams(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("z0", ctypes.c_double), ("p2", ctypes.c_double),
                ("x0", ctypes.c_double), ("m", ctypes.c_int32), ("tol", ctypes.c_double),
                ("flags", ctypes.c_uint32)]


LINE_MAX_POINTS = 16384

_lib = None


def lib():
    """Load libasf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python paper_1203_3583_amd/csrc/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.asf_workspace_bytes.restype = ctypes.c_size_t
        L.asf_workspace_bytes.argtypes = [i64, ctypes.POINTER(Params)]
        L.asf_plan.restype = i32
        L.asf_plan.argtypes = [ctypes.POINTER(vp), i64, vp, vp, vp, ctypes.POINTER(Params), vp,
                               ctypes.c_size_t, vp]
        L.asf_setpts.restype = i32
        L.asf_setpts.argtypes = [vp, vp, vp, vp, vp]
        L.asf_status.restype = i32
        L.asf_status.argtypes = [vp, vp]
        L.asf_forward.restype = i32
        L.asf_forward.argtypes = [vp, vp, vp, vp]
        L.asf_forward_add.restype = i32
        L.asf_forward_add.argtypes = [vp, vp, vp, vp]
        L.asf_forward_static.restype = i32
        L.asf_forward_static.argtypes = [vp, vp, vp, vp]
        L.asf_adjoint.restype = i32
        L.asf_adjoint.argtypes = [vp, vp, vp, vp]
        L.asf_plan_info.restype = i32
        L.asf_plan_info.argtypes = [vp, ctypes.POINTER(Info)]
        L.asf_set_timing.restype = i32
        L.asf_set_timing.argtypes = [vp, i32]
        L.asf_stage_times.restype = i32
        L.asf_stage_times.argtypes = [vp, ctypes.POINTER(dbl), i32]
        L.asf_destroy.restype = i32
        L.asf_destroy.argtypes = [vp]
        L.asf_line_workspace_bytes.restype = ctypes.c_size_t
        L.asf_line_workspace_bytes.argtypes = [i64, ctypes.POINTER(LineParams)]
        L.asf_line_plan.restype = i32
        L.asf_line_plan.argtypes = [ctypes.POINTER(vp), i64, vp, vp, ctypes.POINTER(LineParams), vp,
                                    ctypes.c_size_t, vp]
        L.asf_line_forward.restype = i32
        L.asf_line_forward.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
        L.asf_line_destroy.restype = i32
        L.asf_line_destroy.argtypes = [vp]
        L.asf_last_error.restype = ctypes.c_char_p
        L.asf_last_error.argtypes = []
        _lib = L
    return _lib


def last_error() -> str:
    return lib().asf_last_error().decode()


def _check(rc):
    if rc != ASF_OK:
        raise AsfError(rc, last_error())
    return rc


def make_params(lam, z0, p2x, p2y, mx, my, tol=1e-5, fft="fp32", incident="plane", x0=0.0,
                y0=0.0) -> Params:
    flags = {"fp32": ASF_FFT_FP32, "split_fp16": ASF_FFT_SPLIT_FP16}[fft]
    if incident == "none":
        flags |= ASF_INCIDENT_NONE
    elif incident != "plane":
        raise ValueError(f"incident must be 'plane' or 'none', got {incident!r}")
    return Params(float(lam), float(z0), float(p2x), float(p2y), int(mx), int(my), float(tol), flags,
                  float(x0), float(y0))


def workspace_bytes(n_src, params: Params) -> int:
    b = lib().asf_workspace_bytes(int(n_src), ctypes.byref(params))
    if b == 0:
        raise AsfError(ASF_EINVAL, last_error())
    return int(b)


def _stream_ptr(torch, device, stream):
    s = torch.cuda.current_stream(device) if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(torch, t, name, n, device):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != device:
        raise TypeError(f"{name} must be a float64 tensor on {device}")
    if t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with {n} elements")
    return t


class Plan:
    """A forward plan: geometry binned on the GPU, tables built in FP64.

    x1, y1, d1: float64 device tensors [n] (m); optics lam, z0 (m); destination
    pitch p2x, p2y (m) and size mx x my; tol sets the spreading width; fft is
    "fp32" or "split_fp16"; incident is "plane" (u_I = exp(i k d1)) or "none";
    (x0, y0) centres the destination window off the axis (m).
    """

    def __init__(self, x1, y1, d1, lam, z0, p2x, p2y, mx, my, tol=1e-5, fft="fp32",
                 incident="plane", stream=None, x0=0.0, y0=0.0):
        import torch

        self._torch = torch
        self.device = x1.device
        if self.device.type != "cuda":
            raise TypeError("x1 must be a GPU tensor")
        n = x1.numel()
        for t, name in ((x1, "x1"), (y1, "y1"), (d1, "d1")):
            _dev_f64(torch, t, name, n, self.device)
        self.n = n
        self.mx, self.my = int(mx), int(my)
        self.params = make_params(lam, z0, p2x, p2y, mx, my, tol, fft, incident, x0, y0)
        nbytes = workspace_bytes(n, self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        rc = lib().asf_plan(ctypes.byref(h), n, x1.data_ptr(), y1.data_ptr(), d1.data_ptr(),
                            ctypes.byref(self.params), self.workspace.data_ptr(), nbytes,
                            _stream_ptr(torch, self.device, stream))
        _check(rc)
        self._h = h

    # -- geometry -----------------------------------------------------------------
    def setpts(self, x1, y1, d1, stream=None):
        """Re-bin a new geometry (same n) asynchronously; check with status()."""
        torch = self._torch
        for t, name in ((x1, "x1"), (y1, "y1"), (d1, "d1")):
            _dev_f64(torch, t, name, self.n, self.device)
        _check(lib().asf_setpts(self._h, x1.data_ptr(), y1.data_ptr(), d1.data_ptr(),
                                _stream_ptr(torch, self.device, stream)))

    def status(self, stream=None):
        """Synchronise and raise AsfError(EDOMAIN) if the last geometry had invalid points."""
        _check(lib().asf_status(self._h, _stream_ptr(self._torch, self.device, stream)))

    # -- transforms -----------------------------------------------------------------
    def forward(self, u1, out=None, stream=None, accumulate=False):
        """u2 (complex64 [my, mx]) from u1 (complex64 [n]) on the GPU, asynchronously.

        accumulate=True adds A u1 into ``out`` (asf_forward_add) instead of overwriting it.
        """
        torch = self._torch
        if not isinstance(u1, torch.Tensor) or u1.dtype != torch.complex64 or u1.device != self.device:
            raise TypeError(f"u1 must be a complex64 tensor on {self.device}")
        if u1.numel() != self.n or not u1.is_contiguous():
            raise ValueError(f"u1 must be contiguous with {self.n} elements")
        if accumulate and out is None:
            raise ValueError("accumulate=True needs the out tensor to add into")
        if out is None:
            out = torch.empty((self.my, self.mx), dtype=torch.complex64, device=self.device)
        elif (out.dtype != torch.complex64 or out.device != self.device or out.numel() != self.mx * self.my
              or not out.is_contiguous()):
            raise ValueError("out must be a contiguous complex64 [my, mx] tensor on the plan's device")
        fn = lib().asf_forward_add if accumulate else lib().asf_forward
        _check(fn(self._h, u1.data_ptr(), out.data_ptr(), _stream_ptr(torch, self.device, stream)))
        return out

    def forward_static(self, u1, out, stream=None):
        """asf_forward_static: the forward with the fine grid and column-pass output in the
        library's fixed device scratch (destinations up to 1024 x 1024; calls on one GPU
        must not overlap).  ``out`` must be given (nothing is allocated)."""
        torch = self._torch
        if not isinstance(u1, torch.Tensor) or u1.dtype != torch.complex64 or u1.device != self.device:
            raise TypeError(f"u1 must be a complex64 tensor on {self.device}")
        if u1.numel() != self.n or not u1.is_contiguous():
            raise ValueError(f"u1 must be contiguous with {self.n} elements")
        if (out.dtype != torch.complex64 or out.device != self.device or out.numel() != self.mx * self.my
                or not out.is_contiguous()):
            raise ValueError("out must be a contiguous complex64 [my, mx] tensor on the plan's device")
        _check(lib().asf_forward_static(self._h, u1.data_ptr(), out.data_ptr(),
                                        _stream_ptr(torch, self.device, stream)))
        return out

    def adjoint(self, g2, out=None, stream=None):
        """g1 = A^H g2 (complex64 [n]) from g2 (complex64 [my, mx]) on the GPU, asynchronously."""
        torch = self._torch
        if not isinstance(g2, torch.Tensor) or g2.dtype != torch.complex64 or g2.device != self.device:
            raise TypeError(f"g2 must be a complex64 tensor on {self.device}")
        if g2.numel() != self.mx * self.my or not g2.is_contiguous():
            raise ValueError(f"g2 must be contiguous with {self.my} x {self.mx} elements")
        if out is None:
            out = torch.empty(self.n, dtype=torch.complex64, device=self.device)
        elif (out.dtype != torch.complex64 or out.device != self.device or out.numel() != self.n
              or not out.is_contiguous()):
            raise ValueError("out must be a contiguous complex64 [n] tensor on the plan's device")
        _check(lib().asf_adjoint(self._h, g2.data_ptr(), out.data_ptr(),
                                 _stream_ptr(torch, self.device, stream)))
        return out

    # -- introspection ----------------------------------------------------------------
    def info(self) -> dict:
        inf = Info()
        _check(lib().asf_plan_info(self._h, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in Info._fields_}

    def set_timing(self, enable: bool):
        _check(lib().asf_set_timing(self._h, 1 if enable else 0))

    def stage_times(self) -> dict:
        buf = (ctypes.c_double * len(STAGES))()
        k = lib().asf_stage_times(self._h, buf, len(STAGES))
        if k < 0:
            raise AsfError(k, last_error())
        return {STAGES[i]: buf[i] for i in range(k) if buf[i] >= 0}

    def workspace_view(self, offset, count, dtype):
        """A tensor view of `count` elements of `dtype` at byte `offset` of the workspace."""
        torch = self._torch
        itemsize = torch.empty((), dtype=dtype).element_size()
        return self.workspace[offset:offset + count * itemsize].view(dtype)

    def close(self):
        if getattr(self, "_h", None):
            lib().asf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_line_params(lam, z0, p2, m, tol=1e-5, incident="plane", x0=0.0) -> LineParams:
    if incident not in ("plane", "none"):
        raise ValueError(f"incident must be 'plane' or 'none', got {incident!r}")
    flags = ASF_INCIDENT_NONE if incident == "none" else 0
    return LineParams(float(lam), float(z0), float(p2), float(x0), int(m), float(tol), flags)


def line_workspace_bytes(n_src, params: LineParams) -> int:
    b = lib().asf_line_workspace_bytes(int(n_src), ctypes.byref(params))
    if b == 0:
        raise AsfError(ASF_EINVAL, last_error())
    return int(b)


class LinePlan:
    """A one-dimensional plan (the paper's profiles): a line source x1 with
    displacement d1 onto m destination pixels at X = x0 + p2 (ix - m/2).

    x1, d1: float64 device tensors [n] (m), n <= LINE_MAX_POINTS; optics lam, z0;
    tol sets the spreading width; incident is "plane" or "none".
    """

    def __init__(self, x1, d1, lam, z0, p2, m, tol=1e-5, incident="plane", x0=0.0, stream=None):
        import torch

        self._torch = torch
        self.device = x1.device
        if self.device.type != "cuda":
            raise TypeError("x1 must be a GPU tensor")
        n = x1.numel()
        for t, name in ((x1, "x1"), (d1, "d1")):
            _dev_f64(torch, t, name, n, self.device)
        self.n, self.m = n, int(m)
        self.params = make_line_params(lam, z0, p2, m, tol, incident, x0)
        nbytes = line_workspace_bytes(n, self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check(lib().asf_line_plan(ctypes.byref(h), n, x1.data_ptr(), d1.data_ptr(),
                                   ctypes.byref(self.params), self.workspace.data_ptr(), nbytes,
                                   _stream_ptr(torch, self.device, stream)))
        self._h = h

    def forward(self, u1, out=None, stream=None):
        """u2 (complex64 [m], or [batch, m]) from u1 (complex64 [n] or [batch, n])."""
        torch = self._torch
        if not isinstance(u1, torch.Tensor) or u1.dtype != torch.complex64 or u1.device != self.device:
            raise TypeError(f"u1 must be a complex64 tensor on {self.device}")
        if u1.shape[-1] != self.n or u1.dim() not in (1, 2) or not u1.is_contiguous():
            raise ValueError(f"u1 must be contiguous [n] or [batch, n] with n = {self.n}")
        batch = 1 if u1.dim() == 1 else u1.shape[0]
        shape = (self.m,) if u1.dim() == 1 else (batch, self.m)
        if out is None:
            out = torch.empty(shape, dtype=torch.complex64, device=self.device)
        elif (out.dtype != torch.complex64 or out.device != self.device or tuple(out.shape) != shape
              or not out.is_contiguous()):
            raise ValueError(f"out must be a contiguous complex64 {shape} tensor on the plan's device")
        if batch == 0:
            return out
        _check(lib().asf_line_forward(self._h, batch, u1.data_ptr(), out.data_ptr(),
                                      _stream_ptr(torch, self.device, stream)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().asf_line_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
