"""Tile-shape autotuner for the stencil kernels of the RRRL iteration.

The stencil stages run on 64-column tiles whose height and workgroup size
are selectable (deblur_params.tile, 1..deblur_tile_variants(); 0 = the
library's default for the image size, which may differ between the two
stages; it is timed as a candidate too).  Every shape sums the taps of a pixel
in the same order, so all give bitwise-identical results; only speed differs.
`tune` times every shape on the caller's problem with HIP events, checks the
outputs are identical, and records the fastest in a JSON cache keyed by GPU
architecture, ROCm version, image size class and PSF radius class.
`best_tile` looks a key up (0 when unknown).

Cache file: $DEBLUR_TUNE_CACHE, else ~/.cache/deblur_mi355x/tiles.json.
"""
from __future__ import annotations

import json
import os

CACHE_ENV = "DEBLUR_TUNE_CACHE"


def cache_path() -> str:
    p = os.environ.get(CACHE_ENV)
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "deblur_mi355x", "tiles.json")


def radius_class(ph: int, pw: int) -> int:
    r = max((ph - 1) // 2, (pw - 1) // 2)
    for c in (4, 8, 16, 32):
        if r <= c:
            return c
    raise ValueError("PSF radius above 32")


def size_class(H: int, W: int) -> int:
    """Pixels rounded up to a power of two (tile counts, hence the best shape,
    change with the image area)."""
    n = H * W
    c = 1
    while c < n:
        c <<= 1
    return c


def key(arch: str, rocm: str, H: int, W: int, ph: int, pw: int) -> str:
    return f"{arch}|{rocm}|px{size_class(H, W)}|r{radius_class(ph, pw)}"


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as fh:
            d = json.load(fh)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(d: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def choose(timings: dict[int, float]) -> int:
    """Fastest variant; ties go to the smaller index."""
    return min(sorted(timings), key=lambda v: timings[v])


def _device_ids():
    import torch
    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", props.name), str(torch.version.hip)


def best_tile(H: int, W: int, ph: int, pw: int, path: str | None = None) -> int:
    arch, rocm = _device_ids()
    entry = load_cache(path).get(key(arch, rocm, H, W, ph, pw))
    return int(entry["tile"]) if entry else 0


def tune(f, psf, params, iters: int = 3, reps: int = 5, path: str | None = None, store: bool = True) -> dict:
    """Time every tile shape of the stencil path on (f, psf, params) and
    record the fastest.  Returns {"tile", "timings_us", "key"}; raises if two
    shapes disagree bitwise."""
    import dataclasses

    import torch

    from . import Psf, _lib, deblur_rrrl_iterate

    lib = _lib.load()
    H, W = f.shape
    ph, pw = psf.array_shape()
    u0 = torch.clamp(f, min=1.0)
    ref = None
    timings = {}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for v in range(0, lib.deblur_tile_variants() + 1):   # 0: the library's per-stage default
        p = dataclasses.replace(params, iters=iters, tile=v, conv=2)  # stencil path
        out = torch.empty_like(f)
        deblur_rrrl_iterate(f, u0, out, psf, p)
        torch.cuda.synchronize()
        if ref is None:
            ref = out.clone()
        elif not torch.equal(out, ref):
            raise AssertionError(f"tile shape {v} changed the result")
        ev0.record()
        for _ in range(reps):
            deblur_rrrl_iterate(f, u0, out, psf, p)
        ev1.record()
        torch.cuda.synchronize()
        timings[v] = ev0.elapsed_time(ev1) * 1e3 / (reps * iters)
    arch, rocm = _device_ids()
    k = key(arch, rocm, H, W, ph, pw)
    best = choose(timings)
    if store:
        d = load_cache(path)
        d[k] = {"tile": best, "timings_us": {str(a): round(b, 3) for a, b in timings.items()}}
        save_cache(d, path)
    return {"tile": best, "timings_us": timings, "key": k}
