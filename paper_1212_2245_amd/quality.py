"""Restoration quality of the methods the library runs (Sec. 3.1, Table 1):
the SNR measure and a harness that runs Wiener, RL, RRRL and WR3L on one
degraded image."""
from __future__ import annotations

import math

import numpy as np
import torch


def snr(u, u0, border: int = 0) -> float:
    """SNR(u, u0) = 10 log10(var(u) / var(u - u0)) dB (Sec. 3.1), for a
    restored or degraded image u and the unperturbed image u0 (FP64); with
    `border` > 0 over the interior only (a band of that width left out)."""
    u = np.asarray(u, dtype=np.float64)
    u0 = np.asarray(u0, dtype=np.float64)
    if border > 0:
        u, u0 = u[border:-border, border:-border], u0[border:-border, border:-border]
    d = u - u0
    vd = float(d.var())
    return math.inf if vd == 0.0 else 10.0 * math.log10(float(u.var()) / vd)


def method_snrs(f: np.ndarray, g: np.ndarray, psf: np.ndarray, K: float, alpha: float = 0.003,
                rrrl_iters=(5, 30, 100), rl_iters: int = 30, wr3l_iters: int = 5, border: int = 0) -> dict:
    """SNRs against g of: the degraded image, the Wiener filter (K), RL
    (rl_iters), RRRL (each of rrrl_iters; robust data term, TV, alpha) and
    WR3L (wr3l_iters), the columns of Table 1.  RL and RRRL start from the
    observed image; every method runs in the library's kernels.  `border`:
    as in snr()."""
    from . import Params, Psf, START_OBSERVED, deblur_wiener, rrrl, wr3l

    dev = torch.device("cuda")
    fd = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).to(dev)
    p = Psf.from_taps(torch.from_numpy(np.ascontiguousarray(psf, dtype=np.float32)).to(dev))
    out = {"degraded": snr(f, g, border)}
    u = torch.empty_like(fd)
    deblur_wiener(fd, u, p, K, 1.0)
    out["wiener"] = snr(u.cpu().numpy(), g, border)
    u = rrrl(fd, p, Params(alpha=0.0, robust=False, iters=rl_iters), start=START_OBSERVED)
    out[f"rl{rl_iters}"] = snr(u.cpu().numpy(), g, border)
    for it in rrrl_iters:
        u = rrrl(fd, p, Params(alpha=alpha, iters=it), start=START_OBSERVED)
        out[f"rrrl{it}"] = snr(u.cpu().numpy(), g, border)
    u = wr3l(fd, p, K, Params(alpha=alpha, iters=wr3l_iters))
    out[f"wr3l{wr3l_iters}"] = snr(u.cpu().numpy(), g, border)
    return out
