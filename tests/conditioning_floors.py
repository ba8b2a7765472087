"""Conditioning floors of the 2048x2048 Gaussian-mixture workload (31x31
PSF, Wiener + 30 iterations), computed with the FP64 oracle alone.

The GPU iterates in FP32: every iteration rounds its state to FP32.  The
oracle can do the same (its own FP64 iteration, the state rounded to FP32
after every step), which gives the error that FP32 state storage alone
causes, whatever the kernels' arithmetic.  A second figure is the oracle's
response to a random perturbation of one FP32 rounding unit of the start
image.  Both are relative L2 (and largest pixel error) against the plain
FP64 result, on the constant (replicate) and periodic continuations.

Usage: python tests/conditioning_floors.py [--threads N] [--iters K]
(not collected by pytest; about two minutes per continuation on 8 threads).
"""
import argparse
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
import synth  # noqa: E402


def err(a, b):
    d = a - b
    return float(np.linalg.norm(d) / np.linalg.norm(b)), float(np.abs(d).max() / np.abs(b).max())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    ap.add_argument("--iters", type=int, default=0, help="0: the workload's 30")
    a = ap.parse_args()
    c = synth.make_case(2)
    iters = a.iters or c.iters
    h = c.psf.astype(np.float64)
    u0 = oracle.wiener_init(c.f, h, c.K, 1.0)
    for bc, name in ((oracle.BC_REPLICATE, "replicate"), (oracle.BC_PERIODIC, "periodic")):
        p = oracle.Params(alpha=c.alpha, bc=bc)
        t0 = time.perf_counter()
        want = oracle.rrrl(c.f, u0, h, p, iters, threads=a.threads)
        u = u0.astype(np.float32).astype(np.float64)
        for _ in range(iters):
            u = oracle.rrrl(c.f, u, h, p, 1, threads=a.threads).astype(np.float32).astype(np.float64)
        rng = np.random.default_rng(1)
        up = u0 * (1.0 + rng.uniform(-6e-8, 6e-8, u0.shape))
        pert = oracle.rrrl(c.f, up, h, p, iters, threads=a.threads)
        fl, flp = err(u, want)
        pe, pep = err(pert, want)
        print(f"{name}: {iters} iterations, FP32-state floor rel_l2 {fl:.3e} (largest pixel {flp:.3e} of max), "
              f"response to 1-roundoff start noise rel_l2 {pe:.3e} (largest pixel {pep:.3e} of max); "
              f"{time.perf_counter() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
