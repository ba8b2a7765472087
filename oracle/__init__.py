"""FP64 CPU oracle of WR3L (Wiener init + robust, regularised Richardson-Lucy).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.
It shares no code with the GPU path (it has its own C library, liborc.so,
built from oracle.c by `build()`).

Passages followed (Welk et al., "Fast and Robust Linear Motion Deblurring"):
  * blur model and adjoint PSF: Sec. 2, eq. (1) and the definition of h*;
  * Wiener filter: Sec. 2.1, eq. (2), with periodic continuation (Sec. 4.2);
  * replacement of non-positive Wiener values by a small positive value
    before RRRL: Sec. 3.2 (WR3L);
  * RRRL iteration: Sec. 2.3, eqs. (6)-(12), multiplicative in u^k;
  * diffusion term by central differences: Sec. 4.1; the non-convex
    (Perona-Malik) penaliser as the variant Sec. 2.3 mentions;
  * the lookup-table evaluation of r_f: Sec. 4.1;
  * starting images of RRRL without the Wiener step (Table 1's RRRL
    columns): flat or observed.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc.so")
BC_REPLICATE = 0
BC_PERIODIC = 1


def build(force: bool = True) -> str:
    """Compile oracle.c into liborc.so (gcc, -O2, no fast-math, no FMA contraction)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", src, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("eps_data", ctypes.c_double),
                ("eps_tv", ctypes.c_double), ("s_min", ctypes.c_double),
                ("robust", ctypes.c_int), ("bc", ctypes.c_int), ("psi", ctypes.c_int), ("rf_lut", ctypes.c_int)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        for name in ("orc_blur", "orc_corr"):
            fn = getattr(lib, name)
            fn.argtypes = [dp, i, i, dp, i, i, i, dp, i]
            fn.restype = None
        lib.orc_rf.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_rf.restype = ctypes.c_double
        lib.orc_rf_lut.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_rf_lut.restype = ctypes.c_double
        lib.orc_tv.argtypes = [dp, i, i, ctypes.c_double, i, dp, i]
        lib.orc_tv.restype = None
        lib.orc_rrrl_step.argtypes = [dp, dp, dp, i, i, dp, i, i, ctypes.POINTER(_Params), dp, i]
        lib.orc_rrrl_step.restype = None
        lib.orc_rrrl.argtypes = [dp, dp, dp, i, i, dp, i, i, ctypes.POINTER(_Params), i, dp, i]
        lib.orc_rrrl.restype = None
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def default_threads() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return max(1, min(16, os.cpu_count() or 1))


@dataclass
class Params:
    """RRRL parameters (eq. (9)) and the conventions the paper leaves open."""
    alpha: float = 0.003
    eps_data: float = 0.1
    eps_tv: float = 0.1
    s_min: float = 1e-12
    robust: bool = True
    bc: int = BC_REPLICATE
    psi: int = 0   # regulariser: 0 regularised TV, 1 Perona-Malik (lambda = eps_tv)
    rf_lut: bool = False   # r_f by the lookup of Sec. 4.1 (forward only)

    def c(self) -> _Params:
        return _Params(self.alpha, self.eps_data, self.eps_tv, self.s_min,
                       int(bool(self.robust)), int(self.bc), int(self.psi), int(bool(self.rf_lut)))


# ---------------------------------------------------------------- operators
def blur(v, h, bc: int = BC_REPLICATE, threads: int | None = None) -> np.ndarray:
    """A v(x) = sum_d h(d) E(v)(x-d) (eq. (1))."""
    v, h = _f64(v), _f64(h)
    out = np.empty_like(v)
    _load().orc_blur(_ptr(v), v.shape[0], v.shape[1], _ptr(h), h.shape[0], h.shape[1],
                     int(bc), _ptr(out), threads or default_threads())
    return out


def corr(v, h, bc: int = BC_REPLICATE, threads: int | None = None) -> np.ndarray:
    """B v(x) = sum_d h(d) E(v)(x+d): convolution with h*(x) = h(-x) (Sec. 2)."""
    v, h = _f64(v), _f64(h)
    out = np.empty_like(v)
    _load().orc_corr(_ptr(v), v.shape[0], v.shape[1], _ptr(h), h.shape[0], h.shape[1],
                     int(bc), _ptr(out), threads or default_threads())
    return out


def rf(f: float, s: float) -> float:
    """Information divergence r_f(s) = s - f - f ln(s/f) (eq. (7)); r_0(s) = s."""
    return _load().orc_rf(float(f), float(s))


def rf_lut(f: float, s: float) -> float:
    """r_f(s) by the lookup of Sec. 4.1 (r_1 sampled at k/64 up to 65, linear
    interpolation, tangent beyond 65)."""
    return _load().orc_rf_lut(float(f), float(s))


def tv(u, eps_tv: float, threads: int | None = None, psi: int = 0) -> np.ndarray:
    """D(u) = div(Psi'(|grad u|^2) grad u) by central differences (eq. (11), Sec. 4.1);
    psi = 1 selects the non-convex Perona-Malik penaliser with lambda = eps_tv."""
    u = _f64(u)
    out = np.empty_like(u)
    _load().orc_tv(_ptr(u), u.shape[0], u.shape[1], float(eps_tv), int(psi), _ptr(out),
                   threads or default_threads())
    return out


def rrrl_step(f, u, h, p: Params, threads: int | None = None, parts: bool = False):
    """One RRRL step (eqs. (9)-(12)).  With parts=True also returns the
    intermediate planes (s, W, q, Bq, BW, D) as a dict."""
    f, u, h = _f64(f), _f64(u), _f64(h)
    out = np.empty_like(u)
    pp = p.c()
    buf = np.empty((6,) + u.shape) if parts else None
    _load().orc_rrrl_step(_ptr(f), _ptr(u), _ptr(out), u.shape[0], u.shape[1], _ptr(h),
                          h.shape[0], h.shape[1], ctypes.byref(pp),
                          _ptr(buf) if parts else None, threads or default_threads())
    if parts:
        return out, dict(zip(("s", "W", "q", "N1", "N2", "D"), buf))
    return out


def rrrl(f, u0, h, p: Params, iters: int, threads: int | None = None,
         checkpoints: bool = False):
    """`iters` RRRL steps from u0.  With checkpoints=True also returns the
    iterates u^0..u^{iters-1} stacked."""
    f, u0, h = _f64(f), _f64(u0), _f64(h)
    out = np.empty_like(u0)
    pp = p.c()
    ck = np.empty((iters,) + u0.shape) if checkpoints else None
    _load().orc_rrrl(_ptr(f), _ptr(u0), _ptr(out), u0.shape[0], u0.shape[1], _ptr(h),
                     h.shape[0], h.shape[1], ctypes.byref(pp), int(iters),
                     _ptr(ck) if checkpoints else None, threads or default_threads())
    return (out, ck) if checkpoints else out


# ------------------------------------------------------------------- Wiener
def psf_spectrum(h, H: int, W: int) -> np.ndarray:
    """h^(k) = sum_d h(d) exp(-2 pi i (k_y d_y / H + k_x d_x / W)): the DFT of
    the PSF placed with its centre at index (0,0) under periodic wrap."""
    h = _f64(h)
    Py, Px = h.shape
    cy, cx = (Py - 1) // 2, (Px - 1) // 2
    pad = np.zeros((H, W))
    for j in range(Py):
        for i in range(Px):
            pad[(j - cy) % H, (i - cx) % W] += h[j, i]
    return np.fft.fft2(pad)


def wiener_multiplier(h, H: int, W: int, K: float) -> np.ndarray:
    """M = conj(h^) / (|h^|^2 + K) (eq. (2))."""
    hh = psf_spectrum(h, H, W)
    return np.conj(hh) / (np.abs(hh) ** 2 + K)


def wiener(f, h, K: float) -> np.ndarray:
    """Wiener filter, eq. (2): u = Re IDFT(DFT(f) * conj(h^)/(|h^|^2+K)),
    periodic continuation (Sec. 4.2).  FP64."""
    f = _f64(f)
    M = wiener_multiplier(h, f.shape[0], f.shape[1], K)
    return np.real(np.fft.ifft2(np.fft.fft2(f) * M))


def wiener_init(f, h, K: float, pos_floor: float) -> np.ndarray:
    """WR3L initialisation (Sec. 3.2): Wiener output with values below the
    positive floor replaced, u^0 = max(u_pre, pos_floor)."""
    return np.maximum(wiener(f, h, K), pos_floor)


def rrrl_start(f, mode: int, pos_floor: float) -> np.ndarray:
    """Starting image of RRRL without the Wiener step (the paper does not
    state one): mode 0 (flat) max(mean f, pos_floor) everywhere, mode 1
    (observed) max(f, pos_floor); positive as the multiplicative update needs."""
    f = _f64(f)
    if mode == 0:
        return np.full_like(f, max(float(f.mean()), pos_floor))
    return np.maximum(f, pos_floor)


def wr3l(f, h, K: float, p: Params, iters: int, pos_floor: float = 1.0,
         threads: int | None = None) -> np.ndarray:
    """WR3L (Sec. 3.2): Wiener initialisation followed by `iters` RRRL steps."""
    u0 = wiener_init(f, h, K, pos_floor)
    return rrrl(f, u0, h, p, iters, threads=threads)


# ------------------------------------------------------------------ adjoint
def _load_adjoint():
    lib = _load()
    if not hasattr(lib, "_adj_ready"):
        dp = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        lib.orc_rrrl_step_adjoint.argtypes = [dp, dp, i, i, dp, i, i, ctypes.POINTER(_Params), dp, dp, dp, dp, dp, i]
        lib.orc_rrrl_step_adjoint.restype = None
        lib._adj_ready = True
    return lib


def rrrl_step_adjoint(f, u, h, p: Params, lam, threads: int | None = None):
    """Reverse-mode derivative of one RRRL step at u: given lam = dL/du',
    returns (dL/du, dL/df, dL/dh, dL/dalpha) of that step."""
    f, u, h, lam = _f64(f), _f64(u), _f64(h), _f64(lam)
    du = np.empty_like(u)
    df = np.zeros_like(u)
    dh = np.zeros_like(h)
    da = ctypes.c_double(0.0)
    pp = p.c()
    _load_adjoint().orc_rrrl_step_adjoint(_ptr(f), _ptr(u), u.shape[0], u.shape[1], _ptr(h), h.shape[0], h.shape[1],
                                          ctypes.byref(pp), _ptr(lam), _ptr(du), _ptr(df), _ptr(dh),
                                          ctypes.byref(da), threads or default_threads())
    return du, df, dh, da.value


def rrrl_adjoint(f, checkpoints, h, p: Params, lam_K, threads: int | None = None):
    """Backward through the unrolled iterations u^0 -> ... -> u^K given the
    iterates u^0..u^{K-1} and lam_K = dL/du^K.  Returns (dL/du^0, dL/df,
    dL/dh, dL/dalpha) with f entering every step."""
    lam = _f64(lam_K)
    df = np.zeros_like(lam)
    dh = np.zeros(np.shape(h))
    da = 0.0
    for k in range(len(checkpoints) - 1, -1, -1):
        lam, dfk, dhk, dak = rrrl_step_adjoint(f, checkpoints[k], h, p, lam, threads)
        df += dfk
        dh += dhk
        da += dak
    return lam, df, dh, da


def wiener_adjoint(f, h, K: float, pos_floor: float, lam0):
    """Reverse-mode derivative of the WR3L initialisation u0 = max(u_pre,
    pos_floor), u_pre = Re IDFT(DFT(f) M), M = conj(h^)/(|h^|^2 + K).
    Returns (dL/df, dL/dh) given lam0 = dL/du0.

    u_pre is linear in f with transpose Re IDFT(DFT(.) conj(M)).  For h:
    dL = (1/N) sum_k F(k) dM(k) conj(G^(k)) with G = dL/du_pre, and
    dM/dh(d) = [K e^{+i w.d} - conj(h^)^2 e^{-i w.d}] / (|h^|^2 + K)^2,
    evaluated tap by tap."""
    f, h, lam0 = _f64(f), _f64(h), _f64(lam0)
    H, W = f.shape
    hh = psf_spectrum(h, H, W)
    M = np.conj(hh) / (np.abs(hh) ** 2 + K)
    u_pre = np.real(np.fft.ifft2(np.fft.fft2(f) * M))
    G = lam0 * (u_pre > pos_floor)
    Gh = np.fft.fft2(G)
    df = np.real(np.fft.ifft2(Gh * np.conj(M)))
    Z = np.fft.fft2(f) * np.conj(Gh) / (H * W)
    den2 = (np.abs(hh) ** 2 + K) ** 2
    c1 = K / den2
    c2 = -np.conj(hh) ** 2 / den2
    ky = np.arange(H)[:, None] / H
    kx = np.arange(W)[None, :] / W
    Py, Px = h.shape
    cy, cx = (Py - 1) // 2, (Px - 1) // 2
    dh = np.zeros_like(h)
    for j in range(Py):
        for i in range(Px):
            ph = np.exp(2j * np.pi * (ky * (j - cy) + kx * (i - cx)))
            dh[j, i] = np.real(np.sum(Z * (c1 * ph + c2 * np.conj(ph))))
    return df, dh


def wr3l_loss_and_grad(f, h, K: float, p: Params, iters: int, g, pos_floor: float = 1.0,
                       threads: int | None = None):
    """L = sum (u^K - g)^2 of WR3L and its gradients (dL/df, dL/dh, dL/dalpha)
    through the Wiener initialisation and the unrolled RRRL iterations."""
    f = _f64(f)
    u0 = wiener_init(f, h, K, pos_floor)
    uK, ck = rrrl(f, u0, h, p, iters, threads=threads, checkpoints=True)
    r = uK - _f64(g)
    loss = float(np.sum(r * r))
    lam0, df, dh, da = rrrl_adjoint(f, ck, h, p, 2.0 * r, threads)
    dfw, dhw = wiener_adjoint(f, h, K, pos_floor, lam0)
    return loss, df + dfw, dh + dhw, da
