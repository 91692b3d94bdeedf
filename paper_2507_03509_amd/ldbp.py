"""Learned digital back-propagation on MI355X: binding of the ``ssfm_ldbp_*``
entry points of libssfm (include/ssfm_ldbp.h).

Argument marshalling only: the forward model, the loss and the gradients run
in the library's HIP kernels.  Tensors stand in for device pointers:

* fields      complex64  [batch, P, N]
* taps        complex128 [K, T]
* xi          float64    [K]
* symbols     complex64  [batch, P, N / sps]
* mf          float64    [2R + 1]

:func:`ldbp_apply` and :func:`ldbp_mse` are autograd functions over them.
"""

from __future__ import annotations

import ctypes
from typing import Optional

from . import SsfmError, _check, _stream_ptr, load_library

__all__ = ["SsfmLdbpDesc", "ssfm_ldbp_create", "ssfm_ldbp_destroy",
           "ssfm_ldbp_checkpoint_bytes", "ssfm_ldbp_forward", "ssfm_ldbp_loss",
           "ssfm_ldbp_backward", "Ldbp", "ldbp_apply", "ldbp_mse", "init_params"]


class SsfmLdbpDesc(ctypes.Structure):
    """Mirror of ``ssfm_ldbp_desc``."""

    _fields_ = [
        ("n_pol", ctypes.c_int32),
        ("n_steps", ctypes.c_int32),
        ("n_taps", ctypes.c_int32),
        ("steps_per_span", ctypes.c_int32),
        ("n_samples", ctypes.c_int64),
        ("sps", ctypes.c_int32),
        ("mf_taps", ctypes.c_int32),
    ]


_ready = False


def _lib() -> ctypes.CDLL:
    global _ready
    lib = load_library()
    if not _ready:
        VP, I64 = ctypes.c_void_p, ctypes.c_int64
        lib.ssfm_ldbp_create.argtypes = [ctypes.POINTER(SsfmLdbpDesc), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_void_p)]
        lib.ssfm_ldbp_destroy.argtypes = [VP]
        lib.ssfm_ldbp_checkpoint_bytes.argtypes = [VP, I64, ctypes.POINTER(ctypes.c_int64)]
        lib.ssfm_ldbp_forward.argtypes = [VP, VP, VP, VP, VP, I64, VP, VP]
        lib.ssfm_ldbp_loss.argtypes = [VP, VP, VP, VP, I64, VP, VP, VP]
        lib.ssfm_ldbp_backward.argtypes = [VP, VP, VP, VP, VP, I64, VP, VP, VP, VP, VP]
        from . import SsfmLink
        lib.ssfm_ldbp_init_params.argtypes = [ctypes.POINTER(SsfmLink), ctypes.c_int32,
                                              ctypes.c_int32, VP, VP]
        for name in ("ssfm_ldbp_create", "ssfm_ldbp_destroy", "ssfm_ldbp_checkpoint_bytes",
                     "ssfm_ldbp_forward", "ssfm_ldbp_loss", "ssfm_ldbp_backward",
                     "ssfm_ldbp_init_params"):
            getattr(lib, name).restype = ctypes.c_int
        _ready = True
    return lib


def _tensor(t, dtype, shape, what):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{what} must be on a GPU device")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


# ---------------------------------------------------------------------------
# C-ABI mirrors (pointers as ints)
# ---------------------------------------------------------------------------

def ssfm_ldbp_create(desc: SsfmLdbpDesc, hip_device: int = 0) -> int:
    out = ctypes.c_void_p()
    _check(_lib().ssfm_ldbp_create(ctypes.byref(desc), int(hip_device), ctypes.byref(out)),
           "ssfm_ldbp_create")
    return out.value


def ssfm_ldbp_destroy(h: int) -> None:
    _check(_lib().ssfm_ldbp_destroy(h), "ssfm_ldbp_destroy")


def ssfm_ldbp_checkpoint_bytes(h: int, batch: int) -> int:
    out = ctypes.c_int64(0)
    _check(_lib().ssfm_ldbp_checkpoint_bytes(h, int(batch), ctypes.byref(out)),
           "ssfm_ldbp_checkpoint_bytes")
    return int(out.value)


def ssfm_ldbp_forward(h: int, field_in: int, field_out: int, taps: int, xi: int, batch: int,
                      checkpoints: Optional[int], stream: Optional[int]) -> None:
    _check(_lib().ssfm_ldbp_forward(h, field_in, field_out, taps, xi, int(batch), checkpoints,
                                    stream), "ssfm_ldbp_forward")


def ssfm_ldbp_loss(h: int, field_out: int, symbols: int, mf: int, batch: int, loss: int,
                   grad_out: Optional[int], stream: Optional[int]) -> None:
    _check(_lib().ssfm_ldbp_loss(h, field_out, symbols, mf, int(batch), loss, grad_out, stream),
           "ssfm_ldbp_loss")


def ssfm_ldbp_backward(h: int, field_in: int, field_out: int, taps: int, xi: int, batch: int,
                       checkpoints: Optional[int], grad: int, grad_taps: int, grad_xi: int,
                       stream: Optional[int]) -> None:
    _check(_lib().ssfm_ldbp_backward(h, field_in, field_out, taps, xi, int(batch), checkpoints,
                                     grad, grad_taps, grad_xi, stream), "ssfm_ldbp_backward")


# ---------------------------------------------------------------------------
# Tensor-level wrapper
# ---------------------------------------------------------------------------

class Ldbp:
    """One LDBP configuration on one device (see include/ssfm_ldbp.h)."""

    def __init__(self, n_pol: int, n_steps: int, n_taps: int, steps_per_span: int,
                 n_samples: int, sps: int, mf_taps: int, device: Optional[int] = None):
        import torch
        self.desc = SsfmLdbpDesc(n_pol=int(n_pol), n_steps=int(n_steps), n_taps=int(n_taps),
                                 steps_per_span=int(steps_per_span), n_samples=int(n_samples),
                                 sps=int(sps), mf_taps=int(mf_taps))
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.handle = ssfm_ldbp_create(self.desc, self.device)

    @property
    def n_spans(self) -> int:
        return self.desc.n_steps // self.desc.steps_per_span

    def _field(self, t, what, batch=None):
        import torch
        d = self.desc
        if t.dim() != 3:
            raise ValueError(f"{what} must be [batch, {d.n_pol}, {d.n_samples}]")
        b = int(t.shape[0]) if batch is None else batch
        _tensor(t, torch.complex64, (b, d.n_pol, d.n_samples), what)
        return b

    def _params(self, taps, xi):
        import torch
        d = self.desc
        _tensor(taps, torch.complex128, (d.n_steps, d.n_taps), "taps")
        _tensor(xi, torch.float64, (d.n_steps,), "xi")

    def new_checkpoints(self, batch: int):
        """A checkpoint buffer for ``batch`` realisations (None when K = S)."""
        import torch
        nbytes = ssfm_ldbp_checkpoint_bytes(self.handle, batch)
        if nbytes == 0:
            return None
        return torch.empty(nbytes // 8, dtype=torch.complex64,
                           device=f"cuda:{self.device}")

    def forward(self, x, taps, xi, checkpoints=None, stream=None):
        """Returns LDBP(x) (new tensor); fills ``checkpoints`` if given."""
        import torch
        b = self._field(x, "field_in")
        self._params(taps, xi)
        out = torch.empty_like(x)
        ck = None
        if checkpoints is not None:
            ck = checkpoints.data_ptr()
        ssfm_ldbp_forward(self.handle, x.data_ptr(), out.data_ptr(), taps.data_ptr(),
                          xi.data_ptr(), b, ck, _stream_ptr(x, stream))
        return out

    def loss(self, z, symbols, mf, want_grad: bool = True, stream=None):
        """(loss as a float64 tensor of one element, gradient w.r.t. z or None)."""
        import torch
        d = self.desc
        b = self._field(z, "field_out")
        _tensor(symbols, torch.complex64, (b, d.n_pol, d.n_samples // d.sps), "symbols")
        _tensor(mf, torch.float64, (d.mf_taps,), "mf")
        loss = torch.empty(1, dtype=torch.float64, device=z.device)
        g = torch.empty_like(z) if want_grad else None
        ssfm_ldbp_loss(self.handle, z.data_ptr(), symbols.data_ptr(), mf.data_ptr(), b,
                       loss.data_ptr(), None if g is None else g.data_ptr(),
                       _stream_ptr(z, stream))
        return loss, g

    def backward(self, x, z, taps, xi, checkpoints, grad, stream=None):
        """grad (gradient w.r.t. z) is overwritten with the gradient w.r.t. x;
        returns (grad, grad_taps, grad_xi)."""
        import torch
        b = self._field(x, "field_in")
        self._field(z, "field_out", b)
        self._field(grad, "grad", b)
        self._params(taps, xi)
        gt = torch.empty_like(taps)
        gx = torch.empty_like(xi)
        ssfm_ldbp_backward(self.handle, x.data_ptr(), z.data_ptr(), taps.data_ptr(),
                           xi.data_ptr(), b,
                           None if checkpoints is None else checkpoints.data_ptr(),
                           grad.data_ptr(), gt.data_ptr(), gx.data_ptr(), _stream_ptr(x, stream))
        return grad, gt, gx

    def close(self) -> None:
        if getattr(self, "handle", None):
            ssfm_ldbp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Initial parameters from the link
# ---------------------------------------------------------------------------

def init_params(link, n_taps: int, steps_per_span: int):
    """Taps (complex128 [K, T]) and Kerr coefficients (float64 [K]) that
    back-propagate ``link`` (any object with the fields of ``ssfm_link``),
    K = n_spans * steps_per_span, last span first: ssfm_ldbp_init_params."""
    import numpy as np
    from . import make_link
    k = int(link.n_spans) * int(steps_per_span)
    taps = np.empty((k, int(n_taps)), dtype=np.complex128)
    xi = np.empty(k, dtype=np.float64)
    s = make_link(link)
    _check(_lib().ssfm_ldbp_init_params(
        ctypes.byref(s), int(n_taps), int(steps_per_span),
        taps.ctypes.data_as(ctypes.c_void_p), xi.ctypes.data_as(ctypes.c_void_p)),
        "ssfm_ldbp_init_params")
    return taps, xi


# ---------------------------------------------------------------------------
# Autograd
# ---------------------------------------------------------------------------

def _functions():
    import torch

    class Apply(torch.autograd.Function):
        """z = LDBP(x; taps, xi); the forward keeps span checkpoints, the
        backward recomputes inside each span (ssfm_ldbp_backward)."""

        @staticmethod
        def forward(ctx, x, taps, xi, model):
            x = x.detach().contiguous()
            taps = taps.detach().contiguous()
            xi = xi.detach().contiguous()
            ck = model.new_checkpoints(int(x.shape[0]))
            z = model.forward(x, taps, xi, ck)
            ctx.model = model
            ctx.ck = ck
            ctx.save_for_backward(x, z, taps, xi)
            return z

        @staticmethod
        def backward(ctx, gz):
            x, z, taps, xi = ctx.saved_tensors
            g = gz.detach().to(torch.complex64).contiguous().clone()
            g, gt, gxi = ctx.model.backward(x, z, taps, xi, ctx.ck, g)
            return g, gt, gxi, None

    class Mse(torch.autograd.Function):
        """Mean |matched filter(z) at the symbol instants - symbols|^2."""

        @staticmethod
        def forward(ctx, z, symbols, mf, model):
            loss, g = model.loss(z.detach().contiguous(), symbols, mf, want_grad=True)
            ctx.save_for_backward(g)
            return loss[0]

        @staticmethod
        def backward(ctx, gl):
            (g,) = ctx.saved_tensors
            return (g * gl.to(torch.float32)).to(torch.complex64), None, None, None

    return Apply, Mse


_fns = None


def ldbp_apply(x, taps, xi, model: Ldbp):
    """Differentiable LDBP forward (w.r.t. x, taps and xi)."""
    global _fns
    if _fns is None:
        _fns = _functions()
    return _fns[0].apply(x, taps, xi, model)


def ldbp_mse(z, symbols, mf, model: Ldbp):
    """Differentiable MSE loss of ``z`` against ``symbols``."""
    global _fns
    if _fns is None:
        _fns = _functions()
    return _fns[1].apply(z, symbols, mf, model)
