"""WR3L deblurring on MI355X (gfx950): Wiener initialisation followed by
robust and regularised Richardson-Lucy iterations (Welk et al., "Fast and
Robust Linear Motion Deblurring", Sec. 2.1, 2.3, 3.2).

The compute runs in hand-written HIP kernels behind the C ABI of
include/deblur.h (libdeblur.so).  This module only marshals arguments:
PyTorch provides device memory and the current stream.  The binding
functions carry the C names (deblur_wiener, deblur_rrrl_iterate, ...);
`wr3l` chains them.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import (BC_PERIODIC, BC_REPLICATE, CONV_AUTO, CONV_FFT, CONV_RUNSUM, CONV_STENCIL, PSF_BOX_H, PSF_BOX_V,
                   PSF_TAPS, PSI_PERONA_MALIK, PSI_TV, START_FLAT, START_OBSERVED, DeblurError)

__all__ = ["Psf", "Params", "deblur_workspace_bytes", "deblur_wiener", "deblur_rrrl_iterate", "wr3l",
           "DeblurError", "BC_REPLICATE", "BC_PERIODIC", "PSF_BOX_H", "PSF_BOX_V", "PSF_TAPS",
           "CONV_AUTO", "CONV_RUNSUM", "CONV_STENCIL", "CONV_FFT", "PSI_TV", "PSI_PERONA_MALIK", "START_FLAT",
           "START_OBSERVED", "deblur_rrrl_start", "rrrl", "library_path", "deblur_rrrl_iterate_noalloc"]


def library_path() -> str:
    return _lib.LIB_PATH


@dataclass
class Psf:
    """Point-spread function: a box along x or y (uniform linear motion of
    length n + frac, Sec. 4.3), or a general odd-sized tap array (device
    float32, row-major, normalised)."""
    kind: int
    length: int = 0
    taps: torch.Tensor | None = None
    frac: float = 0.0

    @staticmethod
    def box(length: float, axis: str = "h") -> "Psf":
        """Box of length L >= 1; a non-integer L adds one pixel of weight
        (frac/2)/L at each end of the floor(L) pixels of weight 1/L."""
        n = int(math.floor(length))
        return Psf(PSF_BOX_H if axis == "h" else PSF_BOX_V, n, None, float(length) - n)

    def array_shape(self) -> tuple[int, int]:
        """(ph, pw) of the PSF array (for boxes: the odd array holding the taps)."""
        if self.kind == PSF_TAPS:
            return (int(self.taps.shape[0]), int(self.taps.shape[1]))
        P = self.length + (1 - self.length % 2) + (2 if self.frac > 0.0 else 0)
        return (1, P) if self.kind == PSF_BOX_H else (P, 1)

    @staticmethod
    def from_taps(taps: torch.Tensor) -> "Psf":
        if taps.dim() != 2 or taps.dtype != torch.float32 or not taps.is_cuda:
            raise ValueError("taps must be a 2D float32 device tensor")
        return Psf(PSF_TAPS, 0, taps.contiguous())

    def c(self) -> _lib.deblur_psf:
        if self.kind == PSF_TAPS:
            return _lib.deblur_psf(PSF_TAPS, 0, self.taps.shape[0], self.taps.shape[1], self.taps.data_ptr())
        return _lib.deblur_psf(self.kind, self.length, 0, 0, None, self.frac)


@dataclass
class Params:
    """RRRL parameters (eq. (9)) and the conventions the paper leaves open."""
    alpha: float = 0.003
    iters: int = 10
    eps_data: float = 0.1
    eps_tv: float = 0.1
    s_min: float = 1e-12
    robust: bool = True
    boundary: int = BC_REPLICATE
    conv: int = CONV_AUTO
    tile: int = 0
    psi: int = PSI_TV   # regulariser: PSI_TV, or PSI_PERONA_MALIK (non-convex, lambda = eps_tv)
    rf_lut: bool = False  # r_f through the lookup table of Sec. 4.1 instead of exactly
    bwd_tile: int = 0   # tile rows of the backward kernels: 0 default (by batch size), 1: 8, 2: 4, 3: 16, 4: 32

    def c(self) -> _lib.deblur_params:
        return _lib.deblur_params(self.alpha, self.eps_data, self.eps_tv, self.s_min, int(self.iters),
                                  int(bool(self.robust)), int(self.boundary), int(self.conv), int(self.tile),
                                  int(self.psi), int(bool(self.rf_lut)), int(self.bwd_tile))


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def _image(t: torch.Tensor, name: str) -> tuple[int, int, int]:
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or t.dim() != 2:
        raise ValueError(f"{name} must be a 2D float32 device tensor")
    if t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    return t.shape[0], t.shape[1], t.stride(0)


def _same_layout(a, b, na, nb):
    if a != b:
        raise ValueError(f"{na} and {nb} must have the same shape and row pitch")


def _workspace(nbytes: int, ref: torch.Tensor, ws: torch.Tensor | None) -> torch.Tensor:
    if ws is not None:
        return ws
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=ref.device)


def deblur_workspace_bytes(op: int, H: int, W: int, pitch: int, psf: Psf, params: Params | None = None) -> int:
    cpsf = psf.c()
    cpar = params.c() if params is not None else None
    return int(_lib.load().deblur_workspace_bytes(op, H, W, pitch, ctypes.byref(cpsf),
                                                  ctypes.byref(cpar) if cpar is not None else None))


def deblur_wiener(f: torch.Tensor, u0: torch.Tensor, psf: Psf, K: float = 0.01, pos_floor: float = 1.0,
                  ws: torch.Tensor | None = None, fp64: bool = False) -> torch.Tensor:
    """u0 <- max(Re IDFT(DFT(f) conj(h^)/(|h^|^2+K)), pos_floor), on f's stream.
    fp64=True: deblur_wiener_fp64 (transforms in FP64, output rounded once)."""
    lib = _lib.load()
    H, W, pitch = _image(f, "f")
    _same_layout((H, W, pitch), _image(u0, "u0"), "f", "u0")
    cpsf = psf.c()
    op = _lib.OP_WIENER_FP64 if fp64 else _lib.OP_WIENER
    need = lib.deblur_workspace_bytes(op, H, W, pitch, ctypes.byref(cpsf), None)
    wst = _workspace(need, f, ws)
    fn, name = (lib.deblur_wiener_fp64, "deblur_wiener_fp64") if fp64 else (lib.deblur_wiener, "deblur_wiener")
    st = fn(f.data_ptr(), u0.data_ptr(), H, W, pitch, ctypes.byref(cpsf), float(K), float(pos_floor),
            wst.data_ptr(), wst.numel(), _stream(f))
    _lib.check(st, name)
    return u0


def deblur_rrrl_start(f: torch.Tensor, u0: torch.Tensor, mode: int = _lib.START_FLAT,
                      pos_floor: float = 1.0) -> torch.Tensor:
    """Starting image of RRRL without the Wiener step: START_FLAT gives
    max(mean(f), pos_floor) everywhere, START_OBSERVED max(f, pos_floor)."""
    lib = _lib.load()
    H, W, pitch = _image(f, "f")
    _same_layout((H, W, pitch), _image(u0, "u0"), "f", "u0")
    st = lib.deblur_rrrl_start(f.data_ptr(), u0.data_ptr(), H, W, pitch, int(mode), float(pos_floor), _stream(f))
    _lib.check(st, "deblur_rrrl_start")
    return u0


def rrrl(f: torch.Tensor, psf: Psf, params: Params | None = None, start: int = _lib.START_FLAT,
         pos_floor: float = 1.0, out: torch.Tensor | None = None) -> torch.Tensor:
    """RRRL alone (Sec. 2.3, the RRRL columns of Table 1): a flat or observed
    start, then params.iters iterations.  With params.alpha = 0 and
    robust = False this is Richardson-Lucy."""
    params = params or Params()
    u = out if out is not None else torch.empty_like(f)
    deblur_rrrl_start(f, u, start, pos_floor)
    return deblur_rrrl_iterate(f, u, u, psf, params)


def deblur_rrrl_iterate(f: torch.Tensor, u_in: torch.Tensor, u_out: torch.Tensor, psf: Psf, params: Params,
                        ckpt: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """params.iters RRRL iterations u_in -> u_out (u_in may be u_out).  ckpt
    (optional, [iters, H, pitch] float32) receives u^0 .. u^{iters-1}."""
    lib = _lib.load()
    H, W, pitch = _image(f, "f")
    _same_layout((H, W, pitch), _image(u_in, "u_in"), "f", "u_in")
    _same_layout((H, W, pitch), _image(u_out, "u_out"), "f", "u_out")
    if ckpt is not None:
        if (not ckpt.is_cuda or ckpt.dtype != torch.float32 or not ckpt.is_contiguous()
                or ckpt.numel() < params.iters * H * pitch):
            raise ValueError("ckpt must be a contiguous float32 device tensor of iters*H*pitch elements")
    cpsf, cpar = psf.c(), params.c()
    need = lib.deblur_workspace_bytes(_lib.OP_ITERATE, H, W, pitch, ctypes.byref(cpsf), ctypes.byref(cpar))
    wst = _workspace(need, f, ws)
    st = lib.deblur_rrrl_iterate(f.data_ptr(), u_in.data_ptr(), u_out.data_ptr(), H, W, pitch,
                                 ctypes.byref(cpsf), ctypes.byref(cpar),
                                 ckpt.data_ptr() if ckpt is not None else None,
                                 wst.data_ptr(), wst.numel(), _stream(f))
    _lib.check(st, "deblur_rrrl_iterate")
    return u_out


def deblur_rrrl_iterate_noalloc(f: torch.Tensor, u_in: torch.Tensor, u_out: torch.Tensor, psf: Psf,
                                params: Params, ckpt: torch.Tensor | None = None) -> torch.Tensor:
    """deblur_rrrl_iterate on the library's static device scratch: allocates
    nothing.  Calls that overlap in time on one GPU share that scratch and
    race; problems needing more than 64 MiB of workspace raise DeblurError."""
    lib = _lib.load()
    H, W, pitch = _image(f, "f")
    _same_layout((H, W, pitch), _image(u_in, "u_in"), "f", "u_in")
    _same_layout((H, W, pitch), _image(u_out, "u_out"), "f", "u_out")
    if ckpt is not None:
        if (not ckpt.is_cuda or ckpt.dtype != torch.float32 or not ckpt.is_contiguous()
                or ckpt.numel() < params.iters * H * pitch):
            raise ValueError("ckpt must be a contiguous float32 device tensor of iters*H*pitch elements")
    cpsf, cpar = psf.c(), params.c()
    st = lib.deblur_rrrl_iterate_noalloc(f.data_ptr(), u_in.data_ptr(), u_out.data_ptr(), H, W, pitch,
                                         ctypes.byref(cpsf), ctypes.byref(cpar),
                                         ckpt.data_ptr() if ckpt is not None else None, _stream(f))
    _lib.check(st, "deblur_rrrl_iterate_noalloc")
    return u_out


def wr3l(f: torch.Tensor, psf: Psf, K: float = 0.01, params: Params | None = None,
         pos_floor: float = 1.0, out: torch.Tensor | None = None, wiener_fp64: bool = False) -> torch.Tensor:
    """WR3L (Sec. 3.2): Wiener initialisation, then params.iters RRRL steps
    (wiener_fp64: the Wiener step through deblur_wiener_fp64)."""
    params = params or Params()
    u = out if out is not None else torch.empty_like(f)
    deblur_wiener(f, u, psf, K, pos_floor, fp64=wiener_fp64)
    return deblur_rrrl_iterate(f, u, u, psf, params)


# ----------------------------------------------------------- stage level
__all__ += ["deblur_taps_bytes", "deblur_compile_taps", "deblur_rrrl_weights", "deblur_rrrl_update"]


def deblur_taps_bytes(psf: Psf) -> int:
    return int(_lib.load().deblur_taps_bytes(ctypes.byref(psf.c())))


def deblur_compile_taps(psf: Psf, out: torch.Tensor | None = None, device=None) -> torch.Tensor:
    """Compiled non-zero tap list of `psf` in a device byte buffer."""
    lib = _lib.load()
    cpsf = psf.c()
    n = lib.deblur_taps_bytes(ctypes.byref(cpsf))
    if n == 0:
        raise DeblurError(_lib.DEBLUR_EINVAL, "deblur_taps_bytes")
    if out is None:
        dev = device if device is not None else (psf.taps.device if psf.taps is not None else "cuda")
        out = torch.empty(n, dtype=torch.uint8, device=dev)
    st = lib.deblur_compile_taps(ctypes.byref(cpsf), out.data_ptr(), out.numel(), _stream(out))
    _lib.check(st, "deblur_compile_taps")
    return out


def deblur_rrrl_weights(f: torch.Tensor, u: torch.Tensor, qw: torch.Tensor, psf: Psf, taps: torch.Tensor,
                        params: Params) -> torch.Tensor:
    """Stage 1 of one RRRL step: qw[..., 0] = q, qw[..., 1] = W ([H, W, 2] float32)."""
    lib = _lib.load()
    H, W, pitch = _image(f, "f")
    _same_layout((H, W, pitch), _image(u, "u"), "f", "u")
    if qw.shape != (H, W, 2) or not qw.is_contiguous() or qw.dtype != torch.float32:
        raise ValueError("qw must be a contiguous [H, W, 2] float32 device tensor")
    cpsf, cpar = psf.c(), params.c()
    st = lib.deblur_rrrl_weights(f.data_ptr(), u.data_ptr(), qw.data_ptr(), H, W, pitch, ctypes.byref(cpsf),
                                 taps.data_ptr(), ctypes.byref(cpar), _stream(f))
    _lib.check(st, "deblur_rrrl_weights")
    return qw


def deblur_rrrl_update(qw: torch.Tensor, u: torch.Tensor, u_out: torch.Tensor, psf: Psf, taps: torch.Tensor,
                       params: Params, u_copy: torch.Tensor | None = None) -> torch.Tensor:
    """Stage 2 of one RRRL step: correlation, diffusion term and update."""
    lib = _lib.load()
    H, W, pitch = _image(u, "u")
    _same_layout((H, W, pitch), _image(u_out, "u_out"), "u", "u_out")
    if u_copy is not None:
        _same_layout((H, W, pitch), _image(u_copy, "u_copy"), "u", "u_copy")
    if qw.shape != (H, W, 2) or not qw.is_contiguous() or qw.dtype != torch.float32:
        raise ValueError("qw must be a contiguous [H, W, 2] float32 device tensor")
    cpsf, cpar = psf.c(), params.c()
    st = lib.deblur_rrrl_update(qw.data_ptr(), u.data_ptr(), u_out.data_ptr(),
                                u_copy.data_ptr() if u_copy is not None else None, H, W, pitch,
                                ctypes.byref(cpsf), taps.data_ptr(), ctypes.byref(cpar), _stream(u))
    _lib.check(st, "deblur_rrrl_update")
    return u_out


# -------------------------------------------------------------- backward
__all__ += ["deblur_rrrl_backward", "WR3LFunction", "wr3l_autograd"]


def deblur_rrrl_backward(f: torch.Tensor, ckpt: torch.Tensor | None, grad_uK: torch.Tensor, psf: Psf,
                         params: Params, through_wiener: bool = True, K: float = 0.01, pos_floor: float = 1.0,
                         grad_taps: bool = True, grad_alpha: bool = True, grad_u0: bool = False,
                         ws: torch.Tensor | None = None) -> dict:
    """Gradients of L(u^K) given dL/du^K = grad_uK: returns a dict with
    'f' (dL/df), 'taps' (dL/dh for every PSF entry), 'alpha', 'u0'."""
    lib = _lib.load()
    H, W, pitch = _image(f, "f")
    _same_layout((H, W, pitch), _image(grad_uK, "grad_uK"), "f", "grad_uK")
    if params.iters > 0 and (ckpt is None or not ckpt.is_contiguous() or ckpt.numel() < params.iters * H * pitch):
        raise ValueError("ckpt must hold iters * H * pitch floats")
    cpsf, cpar = psf.c(), params.c()
    op = _lib.OP_BACKWARD_WIENER if through_wiener else _lib.OP_BACKWARD
    need = lib.deblur_workspace_bytes(op, H, W, pitch, ctypes.byref(cpsf), ctypes.byref(cpar))
    wst = _workspace(need, f, ws)
    out = {"f": torch.empty_strided((H, W), (pitch, 1), dtype=torch.float32, device=f.device)}
    ph, pw = psf.array_shape()
    if grad_taps:
        out["taps"] = torch.empty((ph, pw), dtype=torch.float32, device=f.device)
    if grad_alpha:
        out["alpha"] = torch.empty((), dtype=torch.float32, device=f.device)
    if grad_u0:
        out["u0"] = torch.empty_strided((H, W), (pitch, 1), dtype=torch.float32, device=f.device)
    st = lib.deblur_rrrl_backward(f.data_ptr(), ckpt.data_ptr() if ckpt is not None else None, grad_uK.data_ptr(),
                                  H, W, pitch, ctypes.byref(cpsf), ctypes.byref(cpar), int(bool(through_wiener)),
                                  float(K), float(pos_floor), out["f"].data_ptr(),
                                  out["taps"].data_ptr() if grad_taps else None,
                                  out["alpha"].data_ptr() if grad_alpha else None,
                                  out["u0"].data_ptr() if grad_u0 else None, wst.data_ptr(), wst.numel(), _stream(f))
    _lib.check(st, "deblur_rrrl_backward")
    return out


__all__ += ["deblur_wiener_batch", "deblur_rrrl_iterate_batch", "deblur_rrrl_backward_batch"]


def _batch_images(t: torch.Tensor, name: str) -> tuple[int, int, int, int, int]:
    """(B, H, W, pitch, image stride) of a [B, H, W] float32 device tensor."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or t.dim() != 3:
        raise ValueError(f"{name} must be a [B, H, W] float32 device tensor")
    if t.stride(2) != 1:
        raise ValueError(f"{name} must have unit column stride")
    return t.shape[0], t.shape[1], t.shape[2], t.stride(1), t.stride(0)


def _batch_psf(taps, B: int):
    """(deblur_psf, taps stride, (ph, pw), tensor kept alive) of the PSFs of a
    batch: a Psf (any kind) or [ph, pw] taps shared by the batch, or [B, ph,
    pw] taps, one PSF per image."""
    if isinstance(taps, Psf):
        return taps.c(), 0, taps.array_shape(), taps.taps
    if taps.dim() == 2:
        tb, tstride = taps.contiguous(), 0
    elif taps.dim() == 3 and taps.shape[0] == B:
        tb = taps.contiguous()
        tstride = tb.stride(0)
    else:
        raise ValueError("taps must be [ph, pw], [B, ph, pw] or a Psf")
    return Psf.from_taps(tb if tb.dim() == 2 else tb[0]).c(), tstride, (int(tb.shape[-2]), int(tb.shape[-1])), tb


def _batch_alpha(alpha, B: int):
    if alpha is None:
        return None
    if not isinstance(alpha, torch.Tensor) or not alpha.is_cuda or alpha.dtype != torch.float32 or alpha.numel() != B:
        raise ValueError("alpha must be a [B] float32 device tensor")
    return alpha.contiguous()


def deblur_wiener_batch(f: torch.Tensor, u0: torch.Tensor, taps, K: float = 0.01, pos_floor: float = 1.0,
                        fp64: bool = False, ws: torch.Tensor | None = None) -> torch.Tensor:
    """deblur_wiener for a batch: f, u0 [B, H, W] (same layout); taps as in
    deblur_rrrl_backward_batch (a Psf, [ph, pw] or [B, ph, pw])."""
    lib = _lib.load()
    B, H, W, pitch, istride = _batch_images(f, "f")
    if _batch_images(u0, "u0") != (B, H, W, pitch, istride):
        raise ValueError("f and u0 must have the same shape and strides")
    cpsf, tstride, _, _keep = _batch_psf(taps, B)
    op = _lib.OP_WIENER_FP64 if fp64 else _lib.OP_WIENER
    need = lib.deblur_workspace_bytes_batch(op, B, H, W, pitch, ctypes.byref(cpsf), None)
    wst = _workspace(need, f, ws)
    st = lib.deblur_wiener_batch(B, f.data_ptr(), u0.data_ptr(), H, W, pitch, istride, ctypes.byref(cpsf), tstride,
                                 float(K), float(pos_floor), int(bool(fp64)), wst.data_ptr(), wst.numel(), _stream(f))
    _lib.check(st, "deblur_wiener_batch")
    return u0


def deblur_rrrl_iterate_batch(f: torch.Tensor, u_in: torch.Tensor, u_out: torch.Tensor, taps, params: Params,
                              alpha: torch.Tensor | None = None, ckpt: torch.Tensor | None = None,
                              ws: torch.Tensor | None = None) -> torch.Tensor:
    """deblur_rrrl_iterate for a batch: f, u_in, u_out [B, H, W] (same
    layout; u_out may be u_in); taps as in deblur_rrrl_backward_batch;
    alpha: [B] device float32 weights (None: params.alpha); ckpt (optional):
    [B, iters, H, W] with each image's iterates as consecutive H x pitch
    planes."""
    lib = _lib.load()
    B, H, W, pitch, istride = _batch_images(f, "f")
    for t, n in ((u_in, "u_in"), (u_out, "u_out")):
        if _batch_images(t, n) != (B, H, W, pitch, istride):
            raise ValueError(f"f and {n} must have the same shape and strides")
    cstride = 0
    if ckpt is not None:
        if ckpt.dim() != 4 or tuple(ckpt.shape) != (B, params.iters, H, W) or ckpt.dtype != torch.float32:
            raise ValueError("ckpt must be a [B, iters, H, W] float32 tensor")
        if ckpt.stride(3) != 1 or ckpt.stride(2) != pitch or ckpt.stride(1) != H * pitch:
            raise ValueError("ckpt must hold each image's iterates as consecutive H x pitch planes")
        cstride = ckpt.stride(0)
    cpsf, tstride, _, _keep = _batch_psf(taps, B)
    alpha = _batch_alpha(alpha, B)
    cpar = params.c()
    need = lib.deblur_workspace_bytes_batch(_lib.OP_ITERATE, B, H, W, pitch, ctypes.byref(cpsf), ctypes.byref(cpar))
    if need == 0:
        raise ValueError("invalid or unsupported iterate batch arguments")
    wst = _workspace(need, f, ws)
    st = lib.deblur_rrrl_iterate_batch(B, f.data_ptr(), u_in.data_ptr(), u_out.data_ptr(), H, W, pitch, istride,
                                       ctypes.byref(cpsf), tstride, alpha.data_ptr() if alpha is not None else None,
                                       ctypes.byref(cpar), ckpt.data_ptr() if ckpt is not None else None, cstride,
                                       wst.data_ptr(), wst.numel(), _stream(f))
    _lib.check(st, "deblur_rrrl_iterate_batch")
    return u_out


def deblur_rrrl_backward_batch(f: torch.Tensor, ckpt: torch.Tensor | None, grad_uK: torch.Tensor,
                               taps, params: Params, alpha: torch.Tensor | None = None,
                               through_wiener: bool = True, K: float = 0.01, pos_floor: float = 1.0,
                               grad_taps: bool = True, grad_alpha: bool = True, grad_u0: bool = False,
                               ws: torch.Tensor | None = None) -> dict:
    """deblur_rrrl_backward for a batch of B equally sized images in one
    launch per kernel.  f, grad_uK: [B, H, W] (same layout); ckpt:
    [B, iters, H, W] (contiguous per image, None when iters == 0); taps:
    [B, ph, pw] one PSF per image, [ph, pw] or a Psf (any kind) shared by
    the batch; alpha: [B] device
    float32 weights (None: params.alpha for all).  Returns a dict of batched
    gradients: 'f' [B, H, W], 'taps' [B, ph, pw], 'alpha' [B], 'u0'."""
    lib = _lib.load()
    B, H, W, pitch, istride = _batch_images(f, "f")
    if _batch_images(grad_uK, "grad_uK") != (B, H, W, pitch, istride):
        raise ValueError("f and grad_uK must have the same shape and strides")
    cstride = 0
    if params.iters > 0:
        if ckpt is None or ckpt.dim() != 4 or tuple(ckpt.shape) != (B, params.iters, H, W) or ckpt.dtype != torch.float32:
            raise ValueError("ckpt must be a [B, iters, H, W] float32 tensor")
        if ckpt.stride(3) != 1 or ckpt.stride(2) != pitch or ckpt.stride(1) != H * pitch:
            raise ValueError("ckpt must hold each image's iterates as consecutive H x pitch planes")
        cstride = ckpt.stride(0)
    cpsf, tstride, (ph, pw), _keep = _batch_psf(taps, B)
    alpha = _batch_alpha(alpha, B)
    cpar = params.c()
    op = _lib.OP_BACKWARD_WIENER if through_wiener else _lib.OP_BACKWARD
    need = lib.deblur_workspace_bytes_batch(op, B, H, W, pitch, ctypes.byref(cpsf), ctypes.byref(cpar))
    if need == 0:
        raise ValueError("invalid backward batch arguments")
    wst = _workspace(need, f, ws)
    out = {"f": torch.empty_strided((B, H, W), (istride, pitch, 1), dtype=torch.float32, device=f.device)}
    if grad_taps:
        out["taps"] = torch.empty((B, ph, pw), dtype=torch.float32, device=f.device)
    if grad_alpha:
        out["alpha"] = torch.empty((B,), dtype=torch.float32, device=f.device)
    if grad_u0:
        out["u0"] = torch.empty_strided((B, H, W), (istride, pitch, 1), dtype=torch.float32, device=f.device)
    st = lib.deblur_rrrl_backward_batch(B, f.data_ptr(), ckpt.data_ptr() if ckpt is not None else None,
                                        grad_uK.data_ptr(), H, W, pitch, istride, cstride, ctypes.byref(cpsf),
                                        tstride, alpha.data_ptr() if alpha is not None else None,
                                        ctypes.byref(cpar), int(bool(through_wiener)), float(K), float(pos_floor),
                                        out["f"].data_ptr(), out["taps"].data_ptr() if grad_taps else None,
                                        out["alpha"].data_ptr() if grad_alpha else None,
                                        out["u0"].data_ptr() if grad_u0 else None, wst.data_ptr(), wst.numel(),
                                        _stream(f))
    _lib.check(st, "deblur_rrrl_backward_batch")
    return out


class WR3LFunction(torch.autograd.Function):
    """u = WR3L(f; h, alpha) with the hand-written adjoint as backward.

    forward(f, taps, alpha, K, iters, template, pos_floor):
      f      [H, W] or a batch [B, H, W] (device float32);
      taps   [ph, pw] shared by the batch, or [B, ph, pw] one PSF per image;
      alpha  a scalar or a [B] tensor (one regulariser weight per image).  Its
             values are launch parameters read on the host: a device tensor
             costs one synchronisation per forward (pass it on the CPU to
             avoid it);
      template: the other RRRL parameters (penalisers, boundary, tile, ...),
             all carried over; the lookup mode of r_f is not differentiable
             here and is rejected;
      pos_floor: the Wiener positivity floor (Sec. 3.2).
    The Wiener step runs in FP64 (deblur_wiener_fp64): the gradient of the
    unrolled iteration is ill-conditioned near the border ringing of the
    periodic Wiener filter, and a correctly rounded u^0 keeps the GPU
    gradient within 1e-3 of the FP64 one.  The per-iteration checkpoints u^k
    are stored; the backward recomputes every other quantity from them.  The
    forward and the backward cover a batch with one launch per kernel
    (deblur_wiener_batch, deblur_rrrl_iterate_batch,
    deblur_rrrl_backward_batch)."""

    @staticmethod
    def forward(ctx, f, taps, alpha, K: float, iters: int, template: Params | None = None, pos_floor: float = 1.0):
        base = template or Params()
        if base.rf_lut:
            raise ValueError("WR3LFunction differentiates the exact r_f: template.rf_lut must be False")
        batched = f.dim() == 3
        fb = (f if batched else f.unsqueeze(0)).contiguous()
        B, H, W = fb.shape
        tb = taps.detach()
        if tb.dim() == 2:
            tb = tb.unsqueeze(0).expand(B, -1, -1)
        tb = tb.contiguous()
        if tb.shape[0] != B:
            raise ValueError("taps must be [ph, pw] or [B, ph, pw]")
        a = torch.as_tensor(alpha).detach().to("cpu", torch.float64).reshape(-1)
        if a.numel() not in (1, B):
            raise ValueError("alpha must be a scalar or hold one value per image")
        alphas = [float(a[i if a.numel() > 1 else 0]) for i in range(B)]
        u = torch.empty_like(fb)
        ck = torch.empty((B, max(iters, 1), H, W), dtype=torch.float32, device=f.device)
        plist = [dataclasses.replace(base, alpha=alphas[i], iters=int(iters)) for i in range(B)]
        # one upload of the weights (pinned, without blocking the host), kept for the backward
        ad = torch.tensor(alphas, dtype=torch.float32).pin_memory().to(f.device, non_blocking=True)
        deblur_wiener_batch(fb, u, tb, K, pos_floor, fp64=True)
        deblur_rrrl_iterate_batch(fb, u, u, tb, plist[0], alpha=ad, ckpt=ck if iters > 0 else None)
        ctx.save_for_backward(fb, tb, ck)
        ctx.plist, ctx.K, ctx.pos_floor, ctx.alpha_dev = plist, K, pos_floor, ad
        ctx.batched, ctx.shared_taps = batched, taps.dim() == 2
        ctx.alpha_shape = a.numel()
        ctx.alpha_like = alpha if isinstance(alpha, torch.Tensor) else None
        return u if batched else u[0]

    @staticmethod
    def backward(ctx, grad_u):
        fb, tb, ck = ctx.saved_tensors
        gb = (grad_u if ctx.batched else grad_u.unsqueeze(0)).contiguous()
        p0 = ctx.plist[0]
        g = deblur_rrrl_backward_batch(fb, ck if p0.iters > 0 else None, gb, tb, p0, alpha=ctx.alpha_dev,
                                       through_wiener=True, K=ctx.K, pos_floor=ctx.pos_floor)
        gf, gt, ga = g["f"], g["taps"], g["alpha"]
        if ctx.shared_taps:
            gt = gt.sum(0)
        if ctx.alpha_shape == 1:
            ga = ga.sum()
        if ctx.alpha_like is not None:
            ga = ga.reshape(ctx.alpha_like.shape).to(device=ctx.alpha_like.device, dtype=ctx.alpha_like.dtype)
        return (gf if ctx.batched else gf[0]), gt, ga, None, None, None, None


def wr3l_autograd(f: torch.Tensor, taps: torch.Tensor, alpha: torch.Tensor, K: float = 0.01, iters: int = 10,
                  template: Params | None = None, pos_floor: float = 1.0) -> torch.Tensor:
    """Differentiable WR3L (w.r.t. f, taps, alpha) through the library's
    forward and backward kernels; f is [H, W] or a batch [B, H, W] (see
    WR3LFunction)."""
    return WR3LFunction.apply(f, taps, alpha, K, iters, template, pos_floor)


# --------------------------------------------------------------- batched
__all__ += ["BatchPlan"]


class BatchPlan:
    """Many WR3L problems (f_i, psf_i, params_i, K_i) run by one graph launch.

    `items`: sequence of (f, psf, params, K, pos_floor) with f a 2D float32
    device tensor; outputs are allocated here (self.outputs).  All params
    must have the same `iters`.  group_size > 0 runs consecutive groups of
    that many images one after another.  `tiles`: None (library defaults),
    "auto" (the tuned shapes of autotune.best_batch_tiles for this batch, the
    defaults when none are cached) or the five variants (stencil, box_h,
    box_v, box_h_large, box_v_large): box images up to 512 x 512 pixels and
    larger ones have their own tile classes."""

    STENCIL, BOX = 0, 1                 # tile families
    NTILES = 5
    TILE_NAMES = ("stencil", "box_h", "box_v", "box_h_large", "box_v_large")
    CLASS_NAMES = ("stencil_r4", "stencil_r8", "stencil_r16", "stencil_r32", "box_h", "box_v", "box_h_large",
                   "box_v_large")

    def __init__(self, items, group_size: int = 0, tiles=None):
        lib = _lib.load()
        self._keep = []
        self.outputs = []
        arr = (_lib.deblur_batch_item * len(items))()
        for k, (f, psf, params, K, floor) in enumerate(items):
            H, W, pitch = _image(f, "f")
            u = torch.empty_strided((H, W), (pitch, 1), dtype=torch.float32, device=f.device)
            self._keep += [f, psf.taps]
            self.outputs.append(u)
            arr[k] = _lib.deblur_batch_item(f.data_ptr(), u.data_ptr(), H, W, pitch, psf.c(), params.c(), float(K),
                                            float(floor))
        if isinstance(tiles, str):
            if tiles != "auto":
                raise ValueError("tiles: None, 'auto' or five variants")
            from . import autotune
            tiles = autotune.best_batch_tiles(items)
        self.tiles = tuple(int(t) for t in tiles) if tiles is not None else (0,) * self.NTILES
        if len(self.tiles) != self.NTILES:
            raise ValueError("tiles: " + ", ".join(self.TILE_NAMES))
        self._plan = ctypes.c_void_p()
        tt = (ctypes.c_int32 * self.NTILES)(*self.tiles)
        st = lib.deblur_batch_plan_create_tiled(arr, len(items), int(group_size), tt, ctypes.byref(self._plan))
        _lib.check(st, "deblur_batch_plan_create_tiled")
        self.n = len(items)
        self.device = items[0][0].device

    @staticmethod
    def tile_variants(family: int) -> int:
        return int(_lib.load().deblur_batch_tile_variants(int(family)))

    def class_of(self, image: int) -> int:
        c = _lib.load().deblur_batch_class_of(self._plan, int(image))
        _lib.check(min(c, 0), "deblur_batch_class_of")
        return int(c)

    def class_tiles(self, cls: int) -> int:
        c = _lib.load().deblur_batch_class_tiles(self._plan, int(cls))
        _lib.check(min(c, 0), "deblur_batch_class_tiles")
        return int(c)

    def launch_class(self, cls: int, stage: int = 1, stream=None):
        """One launch of one class kernel over the first group's tiles,
        outside the graph (for per-kernel timing); outputs unchanged."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _lib.check(_lib.load().deblur_batch_launch_class(self._plan, int(cls), int(stage), s.cuda_stream),
                   "deblur_batch_launch_class")

    def run(self):
        st = _lib.load().deblur_batch_run(self._plan, torch.cuda.current_stream(self.device).cuda_stream)
        _lib.check(st, "deblur_batch_run")
        return self.outputs

    def latencies_us(self):
        import numpy as np
        out = (ctypes.c_double * self.n)()
        _lib.check(_lib.load().deblur_batch_latencies(self._plan, out), "deblur_batch_latencies")
        return np.array(out[:])

    def close(self):
        if getattr(self, "_plan", None) and self._plan.value:
            _lib.load().deblur_batch_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
