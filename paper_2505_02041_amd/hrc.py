"""Python binding of the C ABI: torch tensors in, device pointers and the
current HIP stream out.  Marshalling only; every step runs in libhrc.so.

Functions named like the C entry points (``hrc_forward``, ``hrc_backward``,
``hrc_batch_plan`` ...) take torch tensors; ``fluence`` adds autograd.
"""
from __future__ import annotations

import ctypes
import math
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import check, hrc_scene


def _log2_size(t: torch.Tensor) -> int:
    if t.dim() != 2 or t.shape[0] != t.shape[1]:
        raise ValueError("expected a square [S, S] tensor")
    S = t.shape[0]
    N = S.bit_length() - 1
    if S != 1 << N:
        raise ValueError("grid side must be a power of two")
    return N


def _check_field(t: torch.Tensor, name: str) -> None:
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")


def _check_like(ref: torch.Tensor, **fields: torch.Tensor) -> None:
    """Every field a contiguous float32 tensor of ref's shape on ref's device (a
    tensor of the wrong size would make the kernels read or write out of
    bounds)."""
    for name, t in fields.items():
        _check_field(t, name)
        if t.shape != ref.shape or t.device != ref.device:
            raise ValueError(f"{name} must have shape {tuple(ref.shape)} on {ref.device}, "
                             f"got {tuple(t.shape)} on {t.device}")


def _stream_handle(device: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def hrc_workspace_bytes(log2_size: int, flags: int = 0) -> Tuple[int, int]:
    """(forward, backward) workspace bytes; a pure host query."""
    f = ctypes.c_size_t(0)
    b = ctypes.c_size_t(0)
    check(_lib.load().hrc_workspace_bytes(log2_size, flags, ctypes.byref(f), ctypes.byref(b)),
          "hrc_workspace_bytes")
    return f.value, b.value


class Context:
    """An ``hrc_context`` on one device plus cached workspaces per grid size and
    stream (calls on different streams never share a workspace).  Like the C
    context, it is meant for one host thread at a time."""

    def __init__(self, device: Optional[int] = None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        self._ptr = ctypes.c_void_p(0)
        check(_lib.load().hrc_create(self.device, ctypes.byref(self._ptr)), "hrc_create")
        self._ws: Dict[Tuple[int, bool], torch.Tensor] = {}

    def __del__(self):
        ptr = getattr(self, "_ptr", None)
        if ptr is not None and ptr.value:
            try:
                _lib.load().hrc_destroy(ptr)
            except Exception:
                pass
            self._ptr = ctypes.c_void_p(0)

    def set_environment(self, radiance: Optional[Sequence[float]]) -> None:
        """Light from beyond the grid (``hrc_set_environment``): radiance samples at
        world angles 2 pi k / K from +x (columns) towards +y (rows), or None."""
        if radiance is None or len(radiance) == 0:
            check(_lib.load().hrc_set_environment(self._ptr, None, 0), "hrc_set_environment")
            return
        arr = (ctypes.c_float * len(radiance))(*[float(v) for v in radiance])
        check(_lib.load().hrc_set_environment(self._ptr, arr, len(radiance)),
              "hrc_set_environment")

    def _check_device(self, t: torch.Tensor) -> None:
        if t.device.index != self.device:
            raise ValueError(f"tensors must be on cuda:{self.device} (the context's device)")

    def _stream_key(self) -> int:
        # cached workspaces are per stream: calls on different streams never
        # share one (calls on one stream run in order)
        return torch.cuda.current_stream(self.device).cuda_stream

    def workspace(self, N: int, backward: bool, flags: int = 0) -> torch.Tensor:
        # the forward's size depends on the quadrant grouping and the interval
        # storage, the backward's on neither
        sized = flags & (_lib.HRC_FLAG_HALF_INTERVALS if backward else
                         (_lib.HRC_FLAG_QUADRANTS_MASK | _lib.HRC_FLAG_HALF_INTERVALS))
        key = (N, backward, sized, self._stream_key())
        ws = self._ws.get(key)
        if ws is None:
            f, b = hrc_workspace_bytes(N, sized)
            ws = torch.empty(b if backward else f, dtype=torch.uint8,
                             device=torch.device("cuda", self.device))
            self._ws[key] = ws
        return ws

    def release_workspaces(self) -> None:
        self._ws.clear()

    def reserve(self, N: int, flags: int = 0) -> torch.Tensor:
        """A fresh (uncached) workspace of the backward's size: the reserve space
        a forward with ``HRC_FLAG_KEEP_PYRAMID`` fills and a backward with
        ``HRC_FLAG_REUSE_PYRAMID`` reads."""
        _, b = hrc_workspace_bytes(N, flags & _lib.HRC_FLAG_HALF_INTERVALS)
        return torch.empty(b, dtype=torch.uint8, device=torch.device("cuda", self.device))

    def _workspace_arg(self, ws: torch.Tensor) -> torch.Tensor:
        if ws.dtype != torch.uint8 or not ws.is_cuda or not ws.is_contiguous():
            raise ValueError("reserve must be a contiguous uint8 CUDA tensor")
        self._check_device(ws)
        return ws

    # -- entry points --------------------------------------------------------
    def hrc_forward(self, emission: torch.Tensor, sigma_t: torch.Tensor,
                    out: Optional[torch.Tensor] = None, flags: int = 0,
                    reserve: Optional[torch.Tensor] = None) -> torch.Tensor:
        """With ``HRC_FLAG_KEEP_PYRAMID`` in flags, ``reserve`` (from ``reserve()``)
        is the workspace and keeps what the reverse reads."""
        _check_field(emission, "emission")
        self._check_device(emission)
        N = _log2_size(emission)
        if out is None:
            out = torch.empty_like(emission)
        _check_like(emission, sigma_t=sigma_t, out=out)
        if flags & _lib.HRC_FLAG_KEEP_PYRAMID:
            if reserve is None:
                raise ValueError("HRC_FLAG_KEEP_PYRAMID needs a reserve tensor")
            ws = self._workspace_arg(reserve)
        else:
            ws = self.workspace(N, False, flags)
        check(_lib.load().hrc_forward(self._ptr, N, emission.data_ptr(), sigma_t.data_ptr(),
                                      out.data_ptr(), ws.data_ptr(), ws.numel(),
                                      _stream_handle(emission.device), flags), "hrc_forward")
        return out

    def hrc_forward_static(self, emission: torch.Tensor, sigma_t: torch.Tensor,
                           out: torch.Tensor, flags: int = 0) -> torch.Tensor:
        """``hrc_forward_static``: the forward on the library's own device scratch
        (no workspace; grids up to 512^2), writing into the caller's ``out``."""
        _check_field(emission, "emission")
        self._check_device(emission)
        N = _log2_size(emission)
        _check_like(emission, sigma_t=sigma_t, out=out)
        check(_lib.load().hrc_forward_static(self._ptr, N, emission.data_ptr(),
                                             sigma_t.data_ptr(), out.data_ptr(),
                                             _stream_handle(emission.device), flags),
              "hrc_forward_static")
        return out

    def hrc_backward(self, emission: torch.Tensor, sigma_t: torch.Tensor,
                     grad_fluence: torch.Tensor, flags: int = 0,
                     reserve: Optional[torch.Tensor] = None):
        """With ``HRC_FLAG_REUSE_PYRAMID`` in flags, ``reserve`` is the workspace a
        forward with ``HRC_FLAG_KEEP_PYRAMID`` filled on the same inputs."""
        _check_field(emission, "emission")
        self._check_device(emission)
        N = _log2_size(emission)
        _check_like(emission, sigma_t=sigma_t, grad_fluence=grad_fluence)
        ge = torch.empty_like(emission)
        gs = torch.empty_like(emission)
        if flags & _lib.HRC_FLAG_REUSE_PYRAMID:
            if reserve is None:
                raise ValueError("HRC_FLAG_REUSE_PYRAMID needs the kept forward's reserve tensor")
            ws = self._workspace_arg(reserve)
        else:
            ws = self.workspace(N, True, flags)
        check(_lib.load().hrc_backward(self._ptr, N, emission.data_ptr(), sigma_t.data_ptr(),
                                       grad_fluence.data_ptr(), ge.data_ptr(), gs.data_ptr(),
                                       ws.data_ptr(), ws.numel(),
                                       _stream_handle(emission.device), flags), "hrc_backward")
        return ge, gs


    # -- three radiance channels over one medium ----------------------------
    def _rgb_sizes(self, N: int, flags: int = 0) -> Tuple[int, int]:
        f, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
        check(_lib.load().hrc_workspace_bytes_rgb(N, flags, ctypes.byref(f), ctypes.byref(b)),
              "hrc_workspace_bytes_rgb")
        return f.value, b.value

    def reserve_rgb(self, N: int, flags: int = 0) -> torch.Tensor:
        """A fresh workspace of the RGB reverse's size (for the interval storage
        in ``flags``): the reserve space that hrc_forward_rgb with
        ``HRC_FLAG_KEEP_PYRAMID`` fills and hrc_backward_rgb with
        ``HRC_FLAG_REUSE_PYRAMID`` reads."""
        half = flags & _lib.HRC_FLAG_HALF_INTERVALS
        return torch.empty(self._rgb_sizes(N, half)[1], dtype=torch.uint8,
                           device=torch.device("cuda", self.device))

    def _rgb_workspace(self, N: int, backward: bool, flags: int = 0) -> torch.Tensor:
        half = flags & _lib.HRC_FLAG_HALF_INTERVALS
        key = ("rgb", N, backward, half, self._stream_key())
        ws = self._ws.get(key)
        if ws is None:
            f, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
            check(_lib.load().hrc_workspace_bytes_rgb(N, half, ctypes.byref(f), ctypes.byref(b)),
                  "hrc_workspace_bytes_rgb")
            ws = torch.empty(b.value if backward else f.value, dtype=torch.uint8,
                             device=torch.device("cuda", self.device))
            self._ws[key] = ws
        return ws

    def _rgb_shapes(self, emission: torch.Tensor, sigma_t: torch.Tensor) -> int:
        if emission.dim() != 3 or emission.shape[0] != 3:
            raise ValueError("emission must be a [3, S, S] tensor")
        self._check_device(emission)
        N = _log2_size(sigma_t)
        if tuple(emission.shape[1:]) != tuple(sigma_t.shape) or sigma_t.device != emission.device:
            raise ValueError("emission planes and sigma_t shapes or devices differ")
        return N

    def hrc_forward_rgb(self, emission: torch.Tensor, sigma_t: torch.Tensor,
                        out: Optional[torch.Tensor] = None, flags: int = 0,
                        reserve: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Fluence of the three channels of emission [3, S, S] over one sigma_t [S, S];
        with ``HRC_FLAG_KEEP_PYRAMID``, ``reserve`` (``reserve_rgb()``) is the workspace."""
        _check_field(emission, "emission")
        _check_field(sigma_t, "sigma_t")
        N = self._rgb_shapes(emission, sigma_t)
        if out is None:
            out = torch.empty_like(emission)
        _check_like(emission, out=out)
        if flags & _lib.HRC_FLAG_KEEP_PYRAMID:
            if reserve is None:
                raise ValueError("HRC_FLAG_KEEP_PYRAMID needs a reserve tensor")
            ws = self._workspace_arg(reserve)
        else:
            ws = self._rgb_workspace(N, False, flags)
        check(_lib.load().hrc_forward_rgb(self._ptr, N, emission.data_ptr(), sigma_t.data_ptr(),
                                          out.data_ptr(), ws.data_ptr(), ws.numel(),
                                          _stream_handle(emission.device), flags),
              "hrc_forward_rgb")
        return out

    def hrc_backward_rgb(self, emission: torch.Tensor, sigma_t: torch.Tensor,
                         grad_fluence: torch.Tensor, flags: int = 0,
                         reserve: Optional[torch.Tensor] = None):
        """With ``HRC_FLAG_REUSE_PYRAMID``, ``reserve`` is the kept RGB forward's workspace."""
        for t, n in ((emission, "emission"), (sigma_t, "sigma_t"), (grad_fluence, "grad_fluence")):
            _check_field(t, n)
        N = self._rgb_shapes(emission, sigma_t)
        _check_like(emission, grad_fluence=grad_fluence)
        ge = torch.empty_like(emission)
        gs = torch.empty_like(sigma_t)
        if flags & _lib.HRC_FLAG_REUSE_PYRAMID:
            if reserve is None:
                raise ValueError("HRC_FLAG_REUSE_PYRAMID needs the kept forward's reserve tensor")
            ws = self._workspace_arg(reserve)
        else:
            ws = self._rgb_workspace(N, True, flags)
        check(_lib.load().hrc_backward_rgb(self._ptr, N, emission.data_ptr(), sigma_t.data_ptr(),
                                           grad_fluence.data_ptr(), ge.data_ptr(), gs.data_ptr(),
                                           ws.data_ptr(), ws.numel(),
                                           _stream_handle(emission.device), flags),
              "hrc_backward_rgb")
        return ge, gs

    def _bounce_workspace(self, N: int, bounces: int, backward: bool) -> torch.Tensor:
        key = ("bounces", N, bounces, backward, self._stream_key())
        ws = self._ws.get(key)
        if ws is None:
            f, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
            check(_lib.load().hrc_multibounce_workspace_bytes(N, bounces, 0, ctypes.byref(f),
                                                              ctypes.byref(b)),
                  "hrc_multibounce_workspace_bytes")
            ws = torch.empty(b.value if backward else f.value, dtype=torch.uint8,
                             device=torch.device("cuda", self.device))
            self._ws[key] = ws
        return ws

    def hrc_multibounce_forward(self, emission: torch.Tensor, sigma_t: torch.Tensor,
                                albedo: torch.Tensor, bounces: int,
                                out: Optional[torch.Tensor] = None) -> torch.Tensor:
        _check_field(emission, "emission")
        self._check_device(emission)
        N = _log2_size(emission)
        F = out if out is not None else torch.empty_like(emission)
        _check_like(emission, sigma_t=sigma_t, albedo=albedo, out=F)
        ws = self._bounce_workspace(N, bounces, False)
        check(_lib.load().hrc_multibounce_forward(
            self._ptr, N, emission.data_ptr(), sigma_t.data_ptr(), albedo.data_ptr(), bounces,
            F.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(emission.device), 0),
            "hrc_multibounce_forward")
        return F

    def hrc_multibounce_backward(self, emission: torch.Tensor, sigma_t: torch.Tensor,
                                 albedo: torch.Tensor, bounces: int, grad_fluence: torch.Tensor):
        _check_field(emission, "emission")
        self._check_device(emission)
        N = _log2_size(emission)
        _check_like(emission, sigma_t=sigma_t, albedo=albedo, grad_fluence=grad_fluence)
        ge, gs, ga = (torch.empty_like(emission) for _ in range(3))
        ws = self._bounce_workspace(N, bounces, True)
        check(_lib.load().hrc_multibounce_backward(
            self._ptr, N, emission.data_ptr(), sigma_t.data_ptr(), albedo.data_ptr(), bounces,
            grad_fluence.data_ptr(), ge.data_ptr(), gs.data_ptr(), ga.data_ptr(), ws.data_ptr(),
            ws.numel(), _stream_handle(emission.device), 0), "hrc_multibounce_backward")
        return ge, gs, ga

    def hrc_profile_solve(self, emission: torch.Tensor, sigma_t: torch.Tensor,
                          grad_fluence: Optional[torch.Tensor] = None,
                          return_outputs: bool = False):
        """One forward (or, with grad_fluence, one backward), each pass timed by
        HIP events recorded at its kernel's start and end; returns
        [(pass name, level, milliseconds)], and with return_outputs also the
        fluence (forward) or (d emission, d sigma_t) (backward)."""
        _check_field(emission, "emission")
        self._check_device(emission)
        N = _log2_size(emission)
        _check_like(emission, sigma_t=sigma_t)
        if grad_fluence is not None:
            _check_like(emission, grad_fluence=grad_fluence)
        bwd = grad_fluence is not None
        ws = self.workspace(N, bwd)
        F = torch.empty_like(emission)
        ge = torch.empty_like(emission) if bwd else None
        gs = torch.empty_like(emission) if bwd else None
        cap = 128
        ms = (ctypes.c_float * cap)()
        kind = (ctypes.c_int * cap)()
        lvl = (ctypes.c_int * cap)()
        count = ctypes.c_int(0)
        check(_lib.load().hrc_profile_solve(
            self._ptr, N, emission.data_ptr(), sigma_t.data_ptr(), F.data_ptr(),
            grad_fluence.data_ptr() if bwd else None, ge.data_ptr() if bwd else None,
            gs.data_ptr() if bwd else None, ws.data_ptr(), ws.numel(),
            _stream_handle(emission.device), ms, kind, lvl, cap, ctypes.byref(count)),
            "hrc_profile_solve")
        passes = [(_lib.PASS_NAMES[kind[i]], lvl[i], ms[i]) for i in range(min(count.value, cap))]
        if return_outputs:
            return passes, ((ge, gs) if bwd else F)
        return passes


_contexts: Dict[int, Context] = {}


def default_context(device: Optional[int] = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    ctx = _contexts.get(device)
    if ctx is None:
        ctx = Context(device)
        _contexts[device] = ctx
    return ctx


class HRCFunction(torch.autograd.Function):
    """F = HRC(emission, sigma_t) with the hand-written adjoint as backward.
    When a gradient is needed the forward keeps the interval pyramid and the
    cascade levels in a reserve tensor (``HRC_FLAG_KEEP_PYRAMID``: the
    backward's workspace size, held until the graph is freed) and the backward
    reads them instead of recomputing them (``HRC_FLAG_REUSE_PYRAMID``);
    ``keep=False`` saves only the inputs and lets ``hrc_backward`` recompute."""

    @staticmethod
    def forward(ctx, emission, sigma_t, blur=False, keep=True):
        emission = emission.contiguous()
        sigma_t = sigma_t.contiguous()
        c = default_context(emission.device.index)
        ctx.flags = _lib.HRC_FLAG_BLUR if blur else 0
        ctx.reserve = None
        if keep and (ctx.needs_input_grad[0] or ctx.needs_input_grad[1]):
            ctx.reserve = c.reserve(_log2_size(emission), ctx.flags)
            F = c.hrc_forward(emission, sigma_t, flags=ctx.flags | _lib.HRC_FLAG_KEEP_PYRAMID,
                              reserve=ctx.reserve)
        else:
            F = c.hrc_forward(emission, sigma_t, flags=ctx.flags)
        ctx.save_for_backward(emission, sigma_t)
        return F

    @staticmethod
    def backward(ctx, grad_F):
        emission, sigma_t = ctx.saved_tensors
        c = default_context(emission.device.index)
        if ctx.reserve is not None:
            ge, gs = c.hrc_backward(emission, sigma_t, grad_F.contiguous(),
                                    flags=ctx.flags | _lib.HRC_FLAG_REUSE_PYRAMID,
                                    reserve=ctx.reserve)
        else:
            ge, gs = c.hrc_backward(emission, sigma_t, grad_F.contiguous(), flags=ctx.flags)
        return ge, gs, None, None


def fluence(emission: torch.Tensor, sigma_t: torch.Tensor, blur: bool = False,
            keep: bool = True) -> torch.Tensor:
    """Per-pixel fluence of a square power-of-two scene (differentiable); with
    ``blur`` the cross blur of Eq. 21 follows the gather.  ``keep=False``
    trades the reverse's recomputation for not holding the reserve tensor
    between forward and backward."""
    return HRCFunction.apply(emission, sigma_t, blur, keep)


class RGBFunction(torch.autograd.Function):
    """F[3, S, S] = HRC of three emission channels over one sigma_t, with the
    hand-written RGB reverse (``hrc_backward_rgb``) as backward; as for
    ``HRCFunction``, the forward keeps what the reverse reads in a reserve
    tensor when a gradient is needed (``keep=False``: the reverse recomputes)."""

    @staticmethod
    def forward(ctx, emission, sigma_t, blur=False, keep=True):
        emission = emission.contiguous()
        sigma_t = sigma_t.contiguous()
        c = default_context(emission.device.index)
        ctx.flags = _lib.HRC_FLAG_BLUR if blur else 0
        ctx.reserve = None
        ctx.save_for_backward(emission, sigma_t)
        if keep and (ctx.needs_input_grad[0] or ctx.needs_input_grad[1]):
            ctx.reserve = c.reserve_rgb(_log2_size(sigma_t), ctx.flags)
            return c.hrc_forward_rgb(emission, sigma_t,
                                     flags=ctx.flags | _lib.HRC_FLAG_KEEP_PYRAMID,
                                     reserve=ctx.reserve)
        return c.hrc_forward_rgb(emission, sigma_t, flags=ctx.flags)

    @staticmethod
    def backward(ctx, grad_F):
        emission, sigma_t = ctx.saved_tensors
        c = default_context(emission.device.index)
        if ctx.reserve is not None:
            ge, gs = c.hrc_backward_rgb(emission, sigma_t, grad_F.contiguous(),
                                        flags=ctx.flags | _lib.HRC_FLAG_REUSE_PYRAMID,
                                        reserve=ctx.reserve)
        else:
            ge, gs = c.hrc_backward_rgb(emission, sigma_t, grad_F.contiguous(), flags=ctx.flags)
        return ge, gs, None, None


def fluence_rgb(emission: torch.Tensor, sigma_t: torch.Tensor, blur: bool = False,
                keep: bool = True) -> torch.Tensor:
    """Fluence [3, S, S] of three emission channels [3, S, S] over one attenuation
    sigma_t [S, S] (differentiable in both)."""
    return RGBFunction.apply(emission, sigma_t, blur, keep)


class MultibounceFunction(torch.autograd.Function):
    """F after several diffuse bounces (``hrc_multibounce_forward``) with the
    hand-written reverse (``hrc_multibounce_backward``) as backward."""

    @staticmethod
    def forward(ctx, emission, sigma_t, albedo, bounces):
        emission, sigma_t, albedo = (t.contiguous() for t in (emission, sigma_t, albedo))
        c = default_context(emission.device.index)
        ctx.bounces = int(bounces)
        ctx.save_for_backward(emission, sigma_t, albedo)
        return c.hrc_multibounce_forward(emission, sigma_t, albedo, ctx.bounces)

    @staticmethod
    def backward(ctx, grad_F):
        emission, sigma_t, albedo = ctx.saved_tensors
        c = default_context(emission.device.index)
        ge, gs, ga = c.hrc_multibounce_backward(emission, sigma_t, albedo, ctx.bounces,
                                                grad_F.contiguous())
        return ge, gs, ga, None


def fluence_multibounce(emission: torch.Tensor, sigma_t: torch.Tensor, albedo: torch.Tensor,
                        bounces: int) -> torch.Tensor:
    """Fluence after ``bounces`` diffuse bounces (differentiable in all three fields)."""
    return MultibounceFunction.apply(emission, sigma_t, albedo, bounces)


class Batch:
    """A planned batch (``hrc_batch_plan``): one persistent-kernel graph launch
    computes every scene's fluence and, where a grad_fluence is given, its
    gradients.  The tensors passed in are the ones every launch reads/writes."""

    def __init__(self, scenes: Sequence[dict], context: Optional[Context] = None,
                 flags: int = 0):
        self.ctx = context or default_context()
        self.scenes = list(scenes)
        arr = (hrc_scene * len(self.scenes))()
        for i, sc in enumerate(self.scenes):
            e, s, F = sc["emission"], sc["sigma_t"], sc["fluence"]
            _check_field(e, "emission")
            _check_like(e, sigma_t=s, fluence=F)
            arr[i].log2_size = _log2_size(e)
            arr[i].emission = e.data_ptr()
            arr[i].sigma_t = s.data_ptr()
            arr[i].fluence = F.data_ptr()
            if sc.get("grad_fluence") is not None:
                _check_like(e, **{n: sc[n] for n in ("grad_fluence", "grad_emission",
                                                     "grad_sigma_t")})
                arr[i].grad_fluence = sc["grad_fluence"].data_ptr()
                arr[i].grad_emission = sc["grad_emission"].data_ptr()
                arr[i].grad_sigma_t = sc["grad_sigma_t"].data_ptr()
        self._ptr = ctypes.c_void_p(0)
        dev = self.scenes[0]["emission"].device
        check(_lib.load().hrc_batch_plan(self.ctx._ptr, arr, len(self.scenes), flags,
                                         _stream_handle(dev), ctypes.byref(self._ptr)),
              "hrc_batch_plan")
        self._device = dev

    def launch(self) -> None:
        check(_lib.load().hrc_batch_launch(self._ptr, _stream_handle(self._device)),
              "hrc_batch_launch")

    def status(self) -> None:
        """Wait for the launches so far and raise (``HRC_ERR_TIMEOUT``) if one of
        them left a pass incomplete (``hrc_batch_status``)."""
        check(_lib.load().hrc_batch_status(self._ptr, _stream_handle(self._device)),
              "hrc_batch_status")

    def debug_waits(self, spins: int) -> None:
        """Failure testing (``hrc_batch_debug_waits``): with spins > 0 every
        dependency wait of later launches gives up after that many polls."""
        torch.cuda.synchronize(self._device)
        check(_lib.load().hrc_batch_debug_waits(self._ptr, int(spins)), "hrc_batch_debug_waits")

    @property
    def workspace_bytes(self) -> int:
        return int(_lib.load().hrc_batch_workspace_bytes(self._ptr))

    def describe(self) -> dict:
        """The autotuner's choice (``hrc_batch_describe``)."""
        v, g, t, c, d = (ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(),
                         ctypes.c_int())
        check(_lib.load().hrc_batch_describe(self._ptr, ctypes.byref(v), ctypes.byref(g),
                                             ctypes.byref(t), ctypes.byref(c), ctypes.byref(d)),
              "hrc_batch_describe")
        nq, xl, sl, br = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(_lib.load().hrc_batch_queues(self._ptr, ctypes.byref(nq), ctypes.byref(xl),
                                           ctypes.byref(sl), ctypes.byref(br)), "hrc_batch_queues")
        return {"variant": v.value, "grid": g.value, "target_tiles": t.value,
                "chunk_groups": c.value, "direct_scenes": d.value, "queues": nq.value,
                "xcd_local": xl.value, "slots_per_queue": sl.value, "direct_branches": br.value}

    def candidates(self) -> List[dict]:
        """Every candidate the autotuner timed (``hrc_batch_candidates``)."""
        n = ctypes.c_int(0)
        check(_lib.load().hrc_batch_candidates(self._ptr, 0, ctypes.byref(n), None, None),
              "hrc_batch_candidates")
        cap = n.value
        F = 8  # fields per candidate
        desc = (ctypes.c_int * (F * max(cap, 1)))()
        ms = (ctypes.c_float * max(cap, 1))()
        check(_lib.load().hrc_batch_candidates(self._ptr, cap, ctypes.byref(n), desc, ms),
              "hrc_batch_candidates")
        keys = ("direct_from_log2", "queues", "xcd_local", "slots_per_queue", "variant",
                "target_tiles", "chunk_groups", "direct_branches")
        return [dict(zip(keys, desc[F * i:F * i + F]), ms=ms[i]) for i in range(cap)]

    def __del__(self):
        ptr = getattr(self, "_ptr", None)
        if ptr is not None and ptr.value:
            try:
                _lib.load().hrc_batch_destroy(ptr)
            except Exception:
                pass
            self._ptr = ctypes.c_void_p(0)
