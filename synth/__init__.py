"""Seeded synthetic inputs shaped like the paper's deblurring workloads.

The paper evaluates on photographs that are not available (a test image and
industrial photos, Sec. 3.1 and 3.3); these generators stand in for them with
seeded, reproducible images of the same size class, grey range [0, 255] and
the same blur types (uniform axis-aligned motion, oblique linear motion,
general 2D blur), blurred in the spatial domain with constant continuation at
the border as the paper does for its synthetic tests (Sec. 3.1).

This module serves both the FP64 oracle tests and the GPU path.  It holds
input generation only (ground truth, PSFs, the forward blur used to *make*
observations, noise): nothing of the deblurring method itself.

Seeds: numpy Generator(PCG64(SeedSequence([2245, config, image]))).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage, signal

KIND_BOX_H = 0
KIND_BOX_V = 1
KIND_TAPS = 2

SIZES_BATCHED = (128, 192, 256, 384, 512, 768, 1024)


def rng_for(config: int, image: int = 0, stream: int = 0) -> np.random.Generator:
    """Seeded generator for (config, image); `stream` separates sub-draws."""
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([2245, int(config), int(image), int(stream)])))


# --------------------------------------------------------------------------
# ground truth images
# --------------------------------------------------------------------------
def ground_truth(rng: np.random.Generator, H: int, W: int,
                 n_rect: int = 20, texture_std: float = 0.0) -> np.ndarray:
    """Piecewise-constant rectangles on a linear background gradient.

    background b0 + gx*(x/(W-1)-1/2) + gy*(y/(H-1)-1/2), b0 ~ U[60,190],
    gx, gy ~ U[-60,60]; then `n_rect` rectangles with height in
    [ceil(H/16), floor(H/3)], width in [ceil(W/16), floor(W/3)], uniform
    top-left corner, uniform grey in [0,255], painted in order.  Optional
    band-limited Gaussian texture (white noise low-passed by a Gaussian of
    sigma 2 px, rescaled to std `texture_std`).  Clipped to [0,255], FP64.
    """
    b0 = rng.uniform(60.0, 190.0)
    gx, gy = rng.uniform(-60.0, 60.0, size=2)
    xs = np.arange(W, dtype=np.float64) / max(W - 1, 1) - 0.5
    ys = np.arange(H, dtype=np.float64) / max(H - 1, 1) - 0.5
    g = b0 + gx * xs[None, :] + gy * ys[:, None]
    hmin, hmax = math.ceil(H / 16), max(math.ceil(H / 16), H // 3)
    wmin, wmax = math.ceil(W / 16), max(math.ceil(W / 16), W // 3)
    for _ in range(n_rect):
        rh = int(rng.integers(hmin, hmax + 1))
        rw = int(rng.integers(wmin, wmax + 1))
        y0 = int(rng.integers(0, H))
        x0 = int(rng.integers(0, W))
        grey = rng.uniform(0.0, 255.0)
        g[y0:y0 + rh, x0:x0 + rw] = grey
    if texture_std > 0.0:
        t = ndimage.gaussian_filter(rng.standard_normal((H, W)), 2.0, mode="wrap")
        t *= texture_std / max(t.std(), 1e-300)
        g = g + t
    return np.clip(g, 0.0, 255.0)


# --------------------------------------------------------------------------
# point-spread functions (odd-sized arrays, centre at ((Py-1)/2, (Px-1)/2))
# --------------------------------------------------------------------------
def box_psf(L: float, axis: str = "h") -> np.ndarray:
    """Uniform linear motion of length L >= 1 along a coordinate axis.

    n = floor(L) taps at offsets d in [-floor((n-1)/2), floor(n/2)], weight
    1/L each (one extra tap on the + side for even n), stored in an odd-length
    array of n + (n even) entries.  A non-integer L adds one tap of weight
    (frac/2)/L, frac = L - n, just outside each end (two more entries).
    """
    n = int(math.floor(L))
    if n < 1:
        raise ValueError("box length must be >= 1")
    frac = float(L) - n
    P = n + (1 - n % 2) + (2 if frac > 0.0 else 0)
    c = (P - 1) // 2
    row = np.zeros(P, dtype=np.float64)
    lo, hi = -((n - 1) // 2), n // 2
    row[c + lo:c + hi + 1] = 1.0 / L
    if frac > 0.0:
        row[c + lo - 1] = row[c + hi + 1] = 0.5 * frac / L
    return row[None, :] if axis == "h" else row[:, None]


def line_psf(L: int, theta: float, drop: float = 1e-9) -> np.ndarray:
    """Oblique linear motion blur of length L at angle theta (radians).

    L samples at t_k = k - (L-1)/2 along direction (cos theta, -sin theta)
    (x right, y down, theta counter-clockwise from +x), each of weight 1/L,
    bilinearly splatted to its 4 neighbouring pixels; splat weights below
    `drop` are discarded and the result renormalised to sum 1 (FP64).
    Array size P = 2*ceil((L-1)/2) + 1.
    """
    R = math.ceil((L - 1) / 2)
    P = 2 * R + 1
    h = np.zeros((P, P), dtype=np.float64)
    c, s = math.cos(theta), -math.sin(theta)
    for k in range(L):
        t = k - (L - 1) / 2.0
        px, py = t * c, t * s
        ix, iy = math.floor(px), math.floor(py)
        fx, fy = px - ix, py - iy
        for oy, wy in ((0, 1.0 - fy), (1, fy)):
            for ox, wx in ((0, 1.0 - fx), (1, fx)):
                w = wy * wx / L
                if w <= drop:
                    continue
                jy, jx = R + iy + oy, R + ix + ox
                if not (0 <= jy < P and 0 <= jx < P):
                    raise AssertionError("line PSF splat left its support")
                h[jy, jx] += w
    return h / h.sum()


def gauss_mixture_psf(rng: np.random.Generator, P: int = 31, n: int = 3) -> np.ndarray:
    """Random smooth PSF: sum of `n` anisotropic Gaussians on a PxP grid.

    Each component: sigmas ~ U[1,6] px, orientation ~ U[0,pi), centre ~
    U[-5,5]^2 px; each normalised to unit sum on the grid (equal weights);
    the sum renormalised to 1.  Non-negative by construction.
    """
    c = (P - 1) // 2
    yy, xx = np.mgrid[-c:c + 1, -c:c + 1].astype(np.float64)
    h = np.zeros((P, P))
    for _ in range(n):
        sa, sb = rng.uniform(1.0, 6.0, size=2)
        phi = rng.uniform(0.0, math.pi)
        my, mx = rng.uniform(-5.0, 5.0, size=2)
        ca, sn = math.cos(phi), math.sin(phi)
        X, Y = xx - mx, yy - my
        a = ca * X + sn * Y
        b = -sn * X + ca * Y
        comp = np.exp(-0.5 * ((a / sa) ** 2 + (b / sb) ** 2))
        h += comp / comp.sum()
    return h / h.sum()


def camera_shake_psf(rng: np.random.Generator, P: int = 25, steps: int = 60, step_len: float = 0.45) -> np.ndarray:
    """Irregular "camera-shake" PSF (the kind of Fig. 1(a)): a random walk with
    momentum from the centre (`steps` steps of `step_len` px, heading turning
    by N(0, 0.35) rad per step), recentred on its mean, each visited point
    bilinearly splatted with equal weight; PxP array, normalised to 1."""
    pts = np.zeros((steps + 1, 2))
    heading = rng.uniform(0.0, 2.0 * math.pi)
    for k in range(steps):
        heading += rng.normal(0.0, 0.35)
        pts[k + 1] = pts[k] + step_len * np.array([math.sin(heading), math.cos(heading)])
    pts -= pts.mean(axis=0)
    R = (P - 1) // 2
    if np.abs(pts).max() > R - 1:
        pts *= (R - 1) / np.abs(pts).max()
    h = np.zeros((P, P))
    for py, px in pts:
        iy, ix = math.floor(py), math.floor(px)
        fy, fx = py - iy, px - ix
        for oy, wy in ((0, 1.0 - fy), (1, fy)):
            for ox, wx in ((0, 1.0 - fx), (1, fx)):
                h[R + iy + oy, R + ix + ox] += wy * wx
    return h / h.sum()


def add_impulse_noise(rng: np.random.Generator, f: np.ndarray, density: float) -> np.ndarray:
    """Replaces a fraction `density` of the pixels by values uniform on [0, 255]
    (the impulse noise of Fig. 2(i)); float32."""
    out = np.array(f, dtype=np.float32, copy=True)
    mask = rng.uniform(size=f.shape) < density
    out[mask] = rng.uniform(0.0, 255.0, size=int(mask.sum())).astype(np.float32)
    return out


def table1_scenarios(size: int = 256, seed: int = 0) -> list[dict]:
    """Synthetic stand-ins for the four test images of Table 1 (the
    cameraman image is not available): one seeded ground truth with texture,
    degraded as (a) camera shake, no noise beyond 8-bit quantisation;
    (b) 21 px motion at 45 degrees; (c) (a) plus Gaussian noise sigma 5;
    (d) (a) with 15 % impulse noise.  Blur with constant continuation (no
    inverse crime).  Each: name, f, g, psf, Wiener K of Table 1."""
    rng = rng_for(10, seed)
    g = ground_truth(rng, size, size, texture_std=10.0)
    shake = camera_shake_psf(rng)
    motion = line_psf(21, math.pi / 4)
    blurred = np.round(np.clip(blur_replicate(g, shake), 0.0, 255.0))
    out = [
        dict(name="camera_shake", f=blurred.astype(np.float32), psf=shake, K=0.006),
        dict(name="motion21_45deg", f=np.round(np.clip(blur_replicate(g, motion), 0.0, 255.0)).astype(np.float32),
             psf=motion, K=0.006),
        dict(name="shake_gauss5", f=np.clip(blurred + rng.normal(0.0, 5.0, size=g.shape), 0.0, 255.0)
             .astype(np.float32), psf=shake, K=0.06),
        dict(name="shake_impulse15", f=add_impulse_noise(rng, blurred, 0.15), psf=shake, K=0.16),
    ]
    for d in out:
        d["g"] = g.astype(np.float32)
    return out


# --------------------------------------------------------------------------
# forward model used to make observations (data generation only)
# --------------------------------------------------------------------------
def blur_replicate(g: np.ndarray, h: np.ndarray) -> np.ndarray:
    """(g * h) with constant continuation at the border, FP64.

    Edge-pads g by the PSF radius and takes the valid part of a linear
    convolution (FFT-based, round-off ~1e-13 relative: irrelevant for data
    generation).
    """
    Py, Px = h.shape
    cy, cx = (Py - 1) // 2, (Px - 1) // 2
    gp = np.pad(g, ((cy, cy), (cx, cx)), mode="edge")
    return signal.fftconvolve(gp, h, mode="valid")


def observe(rng: np.random.Generator, g: np.ndarray, h: np.ndarray,
            sigma: float) -> np.ndarray:
    """f = clip(g*h + N(0, sigma^2), 0, 255) as float32."""
    f = blur_replicate(g, h) + rng.normal(0.0, sigma, size=g.shape)
    return np.clip(f, 0.0, 255.0).astype(np.float32)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------
@dataclass
class Case:
    """One deblurring problem: observation, PSF and method parameters."""
    f: np.ndarray                 # float32 HxW observed image
    g: np.ndarray                 # float32 HxW ground truth
    psf: np.ndarray               # float32 PyxPx taps (odd dims), sum ~ 1
    kind: int                     # KIND_BOX_H / KIND_BOX_V / KIND_TAPS
    length: int                   # box length (box kinds), else 0
    K: float = 0.01               # Wiener noise-to-signal parameter
    alpha: float = 0.003          # regulariser weight
    iters: int = 10               # RRRL iterations
    sigma: float = 2.0            # noise std used to make f
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.f.shape


def _case(rng, H, W, h, kind, length, sigma, texture_std=0.0, **kw) -> Case:
    g = ground_truth(rng, H, W, texture_std=texture_std)
    h32 = h.astype(np.float32)
    f = observe(rng, g, h32.astype(np.float64), sigma)
    return Case(f=f, g=g.astype(np.float32), psf=h32, kind=kind, length=length,
                sigma=sigma, **kw)


def make_case(config: int, image: int = 0, size: int | None = None) -> Case:
    """The seeded synthetic workload `config` (0..4), image index `image`.

    0: 256^2, uniform horizontal motion L=15, sigma 2, K=0.01, alpha=0.003,
       10 iterations.
    1: 1024^2 + Gaussian texture (std 10), oblique line L=31 at a random
       angle, sigma 3, alpha=0.002, 20 iterations.
    2: 2048^2, random smooth 31x31 Gaussian-mixture PSF, sigma 2,
       alpha=0.003, 30 iterations.
    3: one image of the batched workload: side from SIZES_BATCHED, 50% box
       (H/V, L in 5..41), 50% line (L in 9..31), sigma ~ U[1,4], alpha=0.003,
       15 iterations.
    4: 512^2, oblique line L=31, sigma 2, alpha=0.002, 10 iterations.
    `size` overrides the side length (smaller parity cases).
    """
    rng = rng_for(config, image)
    if config == 0:
        n = size or 256
        return _case(rng, n, n, box_psf(15, "h"), KIND_BOX_H, 15, 2.0,
                     K=0.01, alpha=0.003, iters=10)
    if config == 1:
        n = size or 1024
        theta = rng.uniform(0.0, math.pi)
        c = _case(rng, n, n, line_psf(31, theta), KIND_TAPS, 0, 3.0,
                  texture_std=10.0, K=0.01, alpha=0.002, iters=20)
        c.meta["theta"] = theta
        return c
    if config == 2:
        n = size or 2048
        h = gauss_mixture_psf(rng, 31)
        return _case(rng, n, n, h, KIND_TAPS, 0, 2.0, K=0.01, alpha=0.003, iters=30)
    if config == 3:
        n = size or int(rng.choice(SIZES_BATCHED))
        sigma = rng.uniform(1.0, 4.0)
        if rng.uniform() < 0.5:
            axis = "h" if rng.uniform() < 0.5 else "v"
            L = int(rng.integers(5, 42))
            kind = KIND_BOX_H if axis == "h" else KIND_BOX_V
            c = _case(rng, n, n, box_psf(L, axis), kind, L, sigma,
                      K=0.01, alpha=0.003, iters=15)
        else:
            L = int(rng.integers(9, 32))
            theta = rng.uniform(0.0, math.pi)
            c = _case(rng, n, n, line_psf(L, theta), KIND_TAPS, 0, sigma,
                      K=0.01, alpha=0.003, iters=15)
            c.meta["theta"] = theta
            c.meta["L"] = L
        return c
    if config == 4:
        n = size or 512
        theta = rng.uniform(0.0, math.pi)
        c = _case(rng, n, n, line_psf(31, theta), KIND_TAPS, 0, 2.0,
                  K=0.01, alpha=0.002, iters=10)
        c.meta["theta"] = theta
        return c
    raise ValueError(f"unknown workload {config}")


def random_image(rng: np.random.Generator, H: int, W: int, lo=1.0, hi=255.0) -> np.ndarray:
    """Uniform random positive FP64 image (for operator-level tests)."""
    return rng.uniform(lo, hi, size=(H, W))


def random_psf(rng: np.random.Generator, Py: int, Px: int, density: float = 1.0) -> np.ndarray:
    """Random non-negative, asymmetric PSF normalised to sum 1 (FP64)."""
    h = rng.uniform(0.0, 1.0, size=(Py, Px))
    if density < 1.0:
        h *= rng.uniform(size=(Py, Px)) < density
        if h.sum() == 0.0:
            h[(Py - 1) // 2, (Px - 1) // 2] = 1.0
    return h / h.sum()
