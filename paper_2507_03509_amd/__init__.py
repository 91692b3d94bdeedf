"""Split-step Fourier fibre propagation on MI355X: Python binding of libssfm.

The binding only marshals arguments: every step of the propagation runs in
the HIP kernels of ``libssfm.so`` (built in this directory by
``python -m paper_2507_03509_amd.build``).  There is no CPU fallback; if the
library is missing, loading it raises.

Functions with the names of the C ABI (``ssfm_plan``, ``ssfm_forward``, ...)
take and return the same things as their C counterparts, with torch tensors
standing in for device pointers; :class:`Plan` wraps them for convenience.
"""

from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

__all__ = [
    "SsfmLink", "SsfmPlanInfo", "SsfmError", "library_path", "load_library",
    "make_link", "ssfm_plan", "ssfm_plan_destroy", "ssfm_plan_get_info",
    "ssfm_forward", "ssfm_forward_spans", "ssfm_adjoint", "ssfm_adjoint_noalloc", "ssfm_dft",
    "ssfm_batch", "ssfm_status_string", "ssfm_last_error", "ssfm_version", "Plan",
    "ssfm_profile_begin", "ssfm_profile_end", "SsfmKernelStats", "propagate",
    "SsfmTuneInfo", "ssfm_plan_autotune", "ssfm_stream_copy", "ssfm_dft16_rounds",
    "ssfm_orchestration_probe",
    "ssfm_plan_set_state_memory", "ssfm_plan_set_forward_streams",
    "SSFM_OK", "SSFM_EINVAL", "SSFM_ENOMEM", "SSFM_EHIP", "SSFM_EUNSUPPORTED",
    "SSFM_FLAG_FP32_ARITHMETIC",
]

SSFM_OK = 0
SSFM_EINVAL = -1
SSFM_ENOMEM = -2
SSFM_EHIP = -3
SSFM_EUNSUPPORTED = -4
SSFM_FLAG_FP32_ARITHMETIC = 1  # ssfm_link.flags: the FP32-arithmetic variant

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(_HERE, "libssfm.so")


class SsfmLink(ctypes.Structure):
    """Mirror of ``ssfm_link`` in include/ssfm.h."""

    _fields_ = [
        ("n_pol", ctypes.c_int32),
        ("n_spans", ctypes.c_int32),
        ("steps_per_span", ctypes.c_int32),
        ("ase", ctypes.c_int32),
        ("n_samples", ctypes.c_int64),
        ("sample_rate_hz", ctypes.c_double),
        ("span_km", ctypes.c_double),
        ("alpha_db_per_km", ctypes.c_double),
        ("beta2_ps2_per_km", ctypes.c_double),
        ("gamma_per_w_km", ctypes.c_double),
        ("nl_factor", ctypes.c_double),
        ("edfa_gain_db", ctypes.c_double),
        ("edfa_nf_db", ctypes.c_double),
        ("carrier_hz", ctypes.c_double),
        ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class SsfmPlanInfo(ctypes.Structure):
    """Mirror of ``ssfm_plan_info``."""

    _fields_ = [
        ("path", ctypes.c_int32),
        ("n1", ctypes.c_int32),
        ("n2", ctypes.c_int32),
        ("columns_per_tile", ctypes.c_int32),
        ("launches_per_call", ctypes.c_int64),
        ("table_bytes", ctypes.c_int64),
        ("chunk_realisations", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class SsfmKernelStats(ctypes.Structure):
    """Mirror of ``ssfm_kernel_stats``."""

    _fields_ = [
        ("name", ctypes.c_char * 24),
        ("launches", ctypes.c_int64),
        ("total_ms", ctypes.c_double),
        ("field_bytes", ctypes.c_double),
    ]


class SsfmTuneInfo(ctypes.Structure):
    """Mirror of ``ssfm_tune_info``."""

    _fields_ = [
        ("columns", ctypes.c_int32),
        ("row_lanes", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("us_per_step", ctypes.c_double * 4),
    ]

    def as_dict(self) -> dict:
        return {"columns": self.columns, "row_lanes": self.row_lanes,
                "us_per_step": list(self.us_per_step)[: self.candidates]}


class SsfmError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {ssfm_status_string(status)} ({status}): {detail}")


_lib = None


def load_library() -> ctypes.CDLL:
    """Load libssfm.so from the package directory (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is not built; run `python -m paper_2507_03509_amd.build` "
            "(the HIP library is required: there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, I32, I64, U64, VP = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                            ctypes.c_uint64, ctypes.c_void_p)
    lib.ssfm_plan.argtypes = [ctypes.POINTER(SsfmLink), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    lib.ssfm_plan_destroy.argtypes = [P]
    lib.ssfm_plan_get_info.argtypes = [P, ctypes.POINTER(SsfmPlanInfo)]
    lib.ssfm_forward.argtypes = [P, VP, I64, U64, VP]
    lib.ssfm_forward_spans.argtypes = [P, VP, I64, U64, U64, I32, I32, VP]
    lib.ssfm_adjoint.argtypes = [P, VP, VP, I64, U64, VP]
    lib.ssfm_adjoint_noalloc.argtypes = [P, VP, VP, I64, U64, VP]
    lib.ssfm_dft.argtypes = [P, VP, I64, I32, VP]
    lib.ssfm_plan_set_state_memory.argtypes = [P, U64]
    lib.ssfm_plan_set_forward_streams.argtypes = [P, I32]
    lib.ssfm_batch.argtypes = [ctypes.POINTER(SsfmLink), ctypes.POINTER(ctypes.c_void_p), I64,
                               ctypes.POINTER(ctypes.c_uint64), ctypes.c_int, VP]
    lib.ssfm_plan_autotune.argtypes = [P, I64, VP, ctypes.POINTER(SsfmTuneInfo)]
    lib.ssfm_stream_copy.argtypes = [VP, VP, I64, VP]
    lib.ssfm_dft16_rounds.argtypes = [ctypes.c_int, VP, I64, ctypes.c_int, VP]
    lib.ssfm_orchestration_probe.argtypes = [ctypes.c_int, I32, I32, VP,
                                             ctypes.POINTER(ctypes.c_double)]
    lib.ssfm_profile_begin.argtypes = [P]
    lib.ssfm_profile_end.argtypes = [P, ctypes.POINTER(SsfmKernelStats), ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int)]
    lib.ssfm_status_string.argtypes = [ctypes.c_int]
    lib.ssfm_status_string.restype = ctypes.c_char_p
    lib.ssfm_last_error.argtypes = []
    lib.ssfm_last_error.restype = ctypes.c_char_p
    lib.ssfm_version.argtypes = []
    for name in ("ssfm_plan", "ssfm_plan_destroy", "ssfm_plan_get_info", "ssfm_forward",
                 "ssfm_forward_spans", "ssfm_adjoint", "ssfm_batch", "ssfm_version",
                 "ssfm_profile_begin", "ssfm_profile_end", "ssfm_plan_autotune",
                 "ssfm_stream_copy", "ssfm_dft16_rounds", "ssfm_plan_set_state_memory",
                 "ssfm_plan_set_forward_streams", "ssfm_adjoint_noalloc", "ssfm_dft",
                 "ssfm_orchestration_probe"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def ssfm_profile_begin(plan: int) -> None:
    _check(load_library().ssfm_profile_begin(plan), "ssfm_profile_begin")


def ssfm_profile_end(plan: int) -> list:
    """Per-kernel-family stats of the window: list of dicts."""
    out = (SsfmKernelStats * 8)()
    cnt = ctypes.c_int(0)
    _check(load_library().ssfm_profile_end(plan, out, 8, ctypes.byref(cnt)), "ssfm_profile_end")
    return [dict(name=out[i].name.decode(), launches=out[i].launches,
                 total_ms=out[i].total_ms, field_bytes=out[i].field_bytes)
            for i in range(cnt.value)]


def ssfm_status_string(status: int) -> str:
    return load_library().ssfm_status_string(int(status)).decode()


def ssfm_last_error() -> str:
    return load_library().ssfm_last_error().decode()


def ssfm_version() -> int:
    return int(load_library().ssfm_version())


def _check(status: int, where: str) -> None:
    if status != SSFM_OK:
        raise SsfmError(status, where, ssfm_last_error())


def _nan_if_none(v) -> float:
    return float("nan") if v is None else float(v)


def make_link(link, flags: int = 0) -> SsfmLink:
    """``SsfmLink`` from any object with the fields of ``workloads.Link``;
    ``flags``: 0 or SSFM_FLAG_FP32_ARITHMETIC."""
    return SsfmLink(
        n_pol=int(link.n_pol), n_spans=int(link.n_spans),
        steps_per_span=int(link.steps_per_span), ase=1 if link.ase else 0,
        n_samples=int(link.n_samples), sample_rate_hz=float(link.sample_rate_hz),
        span_km=float(link.span_km), alpha_db_per_km=float(link.alpha_db_per_km),
        beta2_ps2_per_km=float(link.beta2_ps2_per_km),
        gamma_per_w_km=float(link.gamma_per_w_km),
        nl_factor=_nan_if_none(getattr(link, "nl_factor", None)),
        edfa_gain_db=float(getattr(link, "edfa_gain_db", 0.0)),
        edfa_nf_db=float(getattr(link, "edfa_nf_db", 0.0)),
        carrier_hz=_nan_if_none(getattr(link, "carrier_hz", None)),
        flags=int(flags), reserved=0)


# ---------------------------------------------------------------------------
# C-ABI mirrors
# ---------------------------------------------------------------------------

def ssfm_plan(link, hip_device: int = 0, flags: int = 0) -> int:
    """Build a plan; returns the opaque handle (an int)."""
    lib = load_library()
    s = link if isinstance(link, SsfmLink) else make_link(link, flags)
    out = ctypes.c_void_p()
    _check(lib.ssfm_plan(ctypes.byref(s), int(hip_device), ctypes.byref(out)), "ssfm_plan")
    return out.value


def ssfm_plan_destroy(plan: int) -> None:
    _check(load_library().ssfm_plan_destroy(plan), "ssfm_plan_destroy")


def ssfm_plan_get_info(plan: int) -> dict:
    info = SsfmPlanInfo()
    _check(load_library().ssfm_plan_get_info(plan, ctypes.byref(info)), "ssfm_plan_get_info")
    return info.as_dict()


def _field_args(field, n_pol: Optional[int] = None, n: Optional[int] = None):
    import torch
    if not isinstance(field, torch.Tensor):
        raise TypeError("field must be a torch tensor")
    if field.dtype != torch.complex64:
        raise TypeError(f"field must be complex64, got {field.dtype}")
    if not field.is_cuda:
        raise ValueError("field must be on a GPU device")
    if not field.is_contiguous():
        raise ValueError("field must be contiguous")
    if field.dim() == 2:
        batch = 1
        shape = (1,) + tuple(field.shape)
    elif field.dim() == 3:
        batch = int(field.shape[0])
        shape = tuple(field.shape)
    else:
        raise ValueError("field must have shape [n_pol, n] or [batch, n_pol, n]")
    if n_pol is not None and (shape[1] != n_pol or shape[2] != n):
        raise ValueError(f"field shape {tuple(field.shape)} does not match the plan "
                         f"(n_pol={n_pol}, n_samples={n})")
    return batch, field.data_ptr()


def _stream_ptr(field, stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(field.device)
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def ssfm_forward(plan: int, field, batch: Optional[int] = None, seed: int = 0,
                 stream=None) -> None:
    """In-place propagation of a complex64 CUDA tensor [batch, n_pol, n]."""
    b, ptr = _field_args(field)
    if batch is not None and batch != b:
        raise ValueError("batch does not match the tensor")
    _check(load_library().ssfm_forward(plan, ptr, b, int(seed) & (2 ** 64 - 1),
                                       _stream_ptr(field, stream)), "ssfm_forward")


def ssfm_forward_spans(plan: int, field, seed: int, realization0: int, span_begin: int,
                       span_end: int, stream=None) -> None:
    b, ptr = _field_args(field)
    _check(load_library().ssfm_forward_spans(plan, ptr, b, int(seed) & (2 ** 64 - 1),
                                             int(realization0), int(span_begin),
                                             int(span_end), _stream_ptr(field, stream)),
           "ssfm_forward_spans")


def ssfm_dft(plan: int, field, inverse: bool = False, stream=None) -> None:
    """The plan's unnormalised DFT of every polarisation, in place (see
    ssfm_dft in ssfm.h for the frequency order of the four-step path)."""
    b, ptr = _field_args(field)
    _check(load_library().ssfm_dft(plan, ptr, b, 1 if inverse else 0, _stream_ptr(field, stream)),
           "ssfm_dft")


def ssfm_adjoint(plan: int, field_in, grad, seed: int = 0, stream=None) -> None:
    """grad (complex64 CUDA tensor shaped like field_in) holds dL/dA_out* on
    entry and dL/dA_in* on exit; field_in is the forward input (read only)."""
    b, ptr = _field_args(field_in)
    bg, gptr = _field_args(grad)
    if bg != b or tuple(grad.shape) != tuple(field_in.shape):
        raise ValueError("grad must have the shape of field_in")
    _check(load_library().ssfm_adjoint(plan, ptr, gptr, b, int(seed) & (2 ** 64 - 1),
                                       _stream_ptr(field_in, stream)), "ssfm_adjoint")


def ssfm_adjoint_noalloc(plan: int, field_in, grad, seed: int = 0, stream=None) -> None:
    """ssfm_adjoint with the library's fixed device scratch instead of
    allocated workspace (no device allocation; calls on one device must not
    overlap)."""
    b, ptr = _field_args(field_in)
    bg, gptr = _field_args(grad)
    if bg != b or tuple(grad.shape) != tuple(field_in.shape):
        raise ValueError("grad must have the shape of field_in")
    _check(load_library().ssfm_adjoint_noalloc(plan, ptr, gptr, b, int(seed) & (2 ** 64 - 1),
                                               _stream_ptr(field_in, stream)),
           "ssfm_adjoint_noalloc")


def ssfm_plan_set_state_memory(plan: int, nbytes: int) -> None:
    """Device memory ssfm_adjoint may keep nonlinear-step inputs in (0: none)."""
    if nbytes < 0:
        raise ValueError("nbytes must be >= 0")
    _check(load_library().ssfm_plan_set_state_memory(plan, int(nbytes)),
           "ssfm_plan_set_state_memory")


def ssfm_plan_set_forward_streams(plan: int, streams: int) -> None:
    """Concurrent parts of each chunk of a four-step call: 0 the library's
    choice (two from 256 column tiles per part), 1..5 that many."""
    _check(load_library().ssfm_plan_set_forward_streams(plan, int(streams)),
           "ssfm_plan_set_forward_streams")


def ssfm_plan_autotune(plan: int, batch: int, stream=None) -> dict:
    """Measure the four-step launch shapes for ``batch`` and record the
    fastest in the plan (see include/ssfm.h)."""
    info = SsfmTuneInfo()
    st = None
    if stream is not None:
        st = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    else:
        import torch
        if torch.cuda.is_available():
            st = torch.cuda.current_stream().cuda_stream
    _check(load_library().ssfm_plan_autotune(plan, int(batch), st, ctypes.byref(info)),
           "ssfm_plan_autotune")
    return info.as_dict()


def ssfm_stream_copy(dst, src, stream=None) -> None:
    """Copy the device tensor ``src`` into ``dst`` (same byte size) with the
    library's plain copy kernel (the bandwidth reference)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("dst and src differ in size")
    _check(load_library().ssfm_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes,
                                           _stream_ptr(src, stream)), "ssfm_stream_copy")


def ssfm_orchestration_probe(method: int, workgroups: int, rounds: int, stream=None) -> float:
    """GPU microseconds per ordering point: 0 graph-replayed dependent
    launches, 1 direct launches, 2 device-wide barriers in one cooperative
    kernel (see include/ssfm.h)."""
    us = ctypes.c_double(0.0)
    st = stream.cuda_stream if stream is not None else None
    _check(load_library().ssfm_orchestration_probe(int(method), int(workgroups), int(rounds), st,
                                                   ctypes.byref(us)),
           "ssfm_orchestration_probe")
    return us.value


def ssfm_dft16_rounds(method: int, data, rounds: int, stream=None) -> None:
    """In place on the device complex128 tensor ``data`` of shape
    (count, 16), count a multiple of 64: each row becomes (F/4)^rounds x with
    the 16-point DFT matrix F; method 0 vector butterfly, 1 matrix cores."""
    if data.dtype != __import__("torch").complex128 or data.dim() != 2 or data.shape[1] != 16:
        raise ValueError("data must be a complex128 tensor of shape (count, 16)")
    if not data.is_contiguous():
        raise ValueError("data must be contiguous")
    _check(load_library().ssfm_dft16_rounds(int(method), data.data_ptr(), data.shape[0],
                                            int(rounds), _stream_ptr(data, stream)),
           "ssfm_dft16_rounds")


def ssfm_batch(links, fields, seeds, hip_device: int = 0, stream=None) -> None:
    n = len(links)
    arr = (SsfmLink * n)(*[l if isinstance(l, SsfmLink) else make_link(l) for l in links])
    ptrs = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fields])
    sd = (ctypes.c_uint64 * n)(*[int(s) for s in seeds])
    st = _stream_ptr(fields[0], stream) if n else None
    _check(load_library().ssfm_batch(arr, ptrs, n, sd, int(hip_device), st), "ssfm_batch")


class Plan:
    """A plan for one link on one device (see ``ssfm_plan``)."""

    def __init__(self, link, device: Optional[int] = None, arithmetic: str = "fp64"):
        """``arithmetic``: "fp64" (the library's path) or "fp32" (the
        FP32-arithmetic variant, SSFM_FLAG_FP32_ARITHMETIC; forward only)."""
        import torch
        if arithmetic not in ("fp64", "fp32"):
            raise ValueError("arithmetic must be 'fp64' or 'fp32'")
        self.link = link
        self.arithmetic = arithmetic
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.n_pol = int(link.n_pol)
        self.n_samples = int(link.n_samples)
        self.handle = ssfm_plan(link, self.device,
                                SSFM_FLAG_FP32_ARITHMETIC if arithmetic == "fp32" else 0)

    @property
    def info(self) -> dict:
        return ssfm_plan_get_info(self.handle)

    def forward(self, field, seed: int = 0, realization0: int = 0,
                span_begin: int = 0, span_end: Optional[int] = None, stream=None):
        """Propagate ``field`` in place (complex64 CUDA tensor [B, P, N] or
        [P, N]); returns it."""
        _field_args(field, self.n_pol, self.n_samples)
        if span_end is None:
            span_end = int(self.link.n_spans)
        ssfm_forward_spans(self.handle, field, seed, realization0, span_begin, span_end,
                           stream)
        return field

    def autotune(self, batch: int, stream=None) -> dict:
        """Choose this plan's launch shape for ``batch`` by measurement."""
        return ssfm_plan_autotune(self.handle, batch, stream)

    def set_forward_streams(self, streams: int) -> None:
        """Concurrent parts of each chunk of a four-step call: 0 the
        library's choice (two from 256 column tiles per part), 1..5 that many."""
        ssfm_plan_set_forward_streams(self.handle, streams)

    def set_state_memory(self, nbytes: int) -> None:
        """Budget for the adjoint's stored nonlinear-step inputs (bytes)."""
        ssfm_plan_set_state_memory(self.handle, nbytes)

    def adjoint(self, field_in, grad, seed: int = 0, stream=None):
        """In-place on ``grad``: dL/dA_out* -> dL/dA_in* (see ssfm_adjoint)."""
        _field_args(field_in, self.n_pol, self.n_samples)
        ssfm_adjoint(self.handle, field_in, grad, seed, stream)
        return grad

    def close(self) -> None:
        if getattr(self, "handle", None):
            ssfm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd_function():
    import torch

    class Propagate(torch.autograd.Function):
        """Differentiable propagation: forward by ssfm_forward, backward by
        ssfm_adjoint (PyTorch's complex-gradient convention, 2 dL/dz*, is
        carried through unchanged: the pullback is real-linear)."""

        @staticmethod
        def forward(ctx, field, plan, seed):
            x = field.detach().contiguous()
            out = x.clone()
            plan.forward(out, seed=seed)
            ctx.save_for_backward(x)
            ctx.plan = plan
            ctx.seed = seed
            return out

        @staticmethod
        def backward(ctx, grad_out):
            (x,) = ctx.saved_tensors
            g = grad_out.detach().to(torch.complex64).contiguous().clone()
            ctx.plan.adjoint(x, g, seed=ctx.seed)
            return g, None, None

    return Propagate


_Propagate = None


def propagate(field, plan: "Plan", seed: int = 0):
    """Autograd-aware propagation of a complex64 CUDA tensor through
    ``plan``'s link (out of place)."""
    global _Propagate
    if _Propagate is None:
        _Propagate = _autograd_function()
    return _Propagate.apply(field, plan, seed)
