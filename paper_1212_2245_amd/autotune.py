"""Tile-shape autotuner of the RRRL kernels.

Three families of kernels have selectable tile shapes, and within a family
every shape gives bitwise-identical results (the shapes only change which
workgroup computes a pixel, never the order of its arithmetic):

* "stencil": the single-image stencil stages (deblur_params.tile,
  1..deblur_tile_variants(); 0 = the library's per-size default);
* "box_h" / "box_v": the single-image running-sum kernel of a horizontal or
  vertical box (deblur_params.tile, 1..deblur_box_tile_variants());
* "batch": the tile shapes of a batch plan, the (stencil, box_h, box_v,
  box_h_large, box_v_large) variants of deblur_batch_plan_create_tiled;
* "backward": the tile rows of the backward's iteration kernels
  (deblur_params.bwd_tile, 1..deblur_backward_tile_variants()).

Each `tune_*` times every shape of its family on the caller's problem with
HIP events, checks that the outputs are bitwise identical (AssertionError
otherwise), and records the fastest in a JSON cache keyed by family, GPU
architecture, ROCm version, an image-size class and a PSF-radius class;
`best_*` looks a key up (the library default when the key is unknown).

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
    """Key of the stencil family (the family name is implicit)."""
    return f"{arch}|{rocm}|px{size_class(H, W)}|r{radius_class(ph, pw)}"


def length_class(L: float) -> int:
    """Box length rounded up to a power of two, at least 8 (the halo of a box
    tile grows with the length)."""
    c = 8
    while c < L:
        c <<= 1
    return c


def family_key(family: str, arch: str, rocm: str, size: int, radius: int) -> str:
    return f"{family}|{arch}|{rocm}|px{size}|r{radius}"


def batch_class(items) -> tuple[int, int]:
    """(total pixels, largest PSF radius or box length) classes of a batch."""
    from . import PSF_BOX_H, PSF_BOX_V
    px = sum(int(it[0].shape[0]) * int(it[0].shape[1]) for it in items)
    rad = 1
    for it in items:
        psf = it[1]
        if psf.kind in (PSF_BOX_H, PSF_BOX_V):
            rad = max(rad, length_class(psf.length + psf.frac))
        else:
            ph, pw = psf.array_shape()
            rad = max(rad, radius_class(ph, pw))
    return size_class(px, 1), rad


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


def _time(fn, reps):
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) * 1e3 / reps


def _store(family_k: str, entry: dict, path: str | None) -> None:
    d = load_cache(path)
    d[family_k] = entry
    save_cache(d, path)


def best_box_tile(H: int, W: int, length: float, axis: str, path: str | None = None) -> int:
    arch, rocm = _device_ids()
    k = family_key(f"box_{axis}", arch, rocm, size_class(H, W), length_class(length))
    entry = load_cache(path).get(k)
    return int(entry["tile"]) if entry else 0


def tune_box(f, psf, params, iters: int = 3, reps: int = 5, path: str | None = None, store: bool = True) -> dict:
    """Time every running-sum tile shape on (f, box psf, params), bitwise
    check, record the fastest under the box_h / box_v family."""
    import dataclasses

    import torch

    from . import PSF_BOX_H, PSF_BOX_V, _lib, deblur_rrrl_iterate

    if psf.kind not in (PSF_BOX_H, PSF_BOX_V):
        raise ValueError("tune_box needs a box PSF")
    axis = "h" if psf.kind == PSF_BOX_H else "v"
    lib = _lib.load()
    H, W = f.shape
    u0 = torch.clamp(f, min=1.0)
    ref, timings = None, {}
    for v in range(0, lib.deblur_box_tile_variants() + 1):
        p = dataclasses.replace(params, iters=iters, tile=v, conv=1)   # running sums
        out = torch.empty_like(f)
        deblur_rrrl_iterate(f, u0, out, psf, p)
        torch.cuda.synchronize()
        if ref is None:
            ref = out.clone()
        elif not torch.equal(out, ref):
            raise AssertionError(f"box tile shape {v} changed the result")
        timings[v] = _time(lambda: deblur_rrrl_iterate(f, u0, out, psf, p), reps) / iters
    arch, rocm = _device_ids()
    k = family_key(f"box_{axis}", arch, rocm, size_class(H, W), length_class(psf.length + psf.frac))
    best = choose(timings)
    if store:
        _store(k, {"tile": best, "timings_us": {str(a): round(b, 3) for a, b in timings.items()}}, path)
    return {"tile": best, "timings_us": timings, "key": k}


BatchPlan_NTILES = 5     # tile entries of a batch plan


def best_batch_tiles(items, path: str | None = None):
    """Cached tile variants (BatchPlan.TILE_NAMES order) for a batch like
    `items`, or None (library defaults)."""
    arch, rocm = _device_ids()
    px, rad = batch_class(items)
    entry = load_cache(path).get(family_key("batch", arch, rocm, px, rad))
    if not entry or len(entry["tiles"]) != BatchPlan_NTILES:
        return None
    return tuple(int(t) for t in entry["tiles"])


def tune_batch(items, reps: int = 10, path: str | None = None, store: bool = True) -> dict:
    """Tile shapes of a batch plan over `items`: every variant of one tile
    entry (stencil, box_h, box_v, box_h_large, box_v_large) is tried with the
    others at their defaults, each plan's outputs must equal the default
    plan's bitwise, and each entry is timed by launching its classes' kernels
    alone (the plan's per-class launch hook): after one full run of the plan,
    the best of three rounds of `reps` launches.  Entries whose classes hold
    no image keep the default (0)."""
    import torch

    from . import BatchPlan

    def class_time(plan, classes):
        t = 0.0
        for c in classes:
            for stage in ((1, 2) if c < 4 else (1,)):
                plan.launch_class(c, stage)
                torch.cuda.synchronize()
                t += _time(lambda: plan.launch_class(c, stage), reps)
        return t

    n = BatchPlan.NTILES
    ref_plan = BatchPlan(items, tiles=(0,) * n)
    ref = [o.clone() for o in ref_plan.run()]
    torch.cuda.synchronize()
    classes = sorted({ref_plan.class_of(i) for i in range(ref_plan.n)})
    ref_plan.close()
    # tile entry -> its classes: 0 the stencil classes 0..3, 1..4 the box classes 4..7
    fams = {0: [c for c in classes if c < 4]}
    for e in range(1, n):
        fams[e] = [c for c in classes if c == e + 3]
    best, timings = [0] * n, {}
    for fam in range(n):
        if not fams[fam]:
            continue
        tf = {}
        for v in range(1, BatchPlan.tile_variants(BatchPlan.STENCIL if fam == 0 else BatchPlan.BOX) + 1):
            tiles = [0] * n
            tiles[fam] = v
            plan = BatchPlan(items, tiles=tuple(tiles))
            outs = plan.run()
            torch.cuda.synchronize()
            for i, (a, b) in enumerate(zip(outs, ref)):
                if not torch.equal(a, b):
                    plan.close()
                    raise AssertionError(f"batch tiles {tiles} changed image {i}")
            tf[v] = min(class_time(plan, fams[fam]) for _ in range(3))
            plan.close()
        best[fam] = choose(tf)
        timings[BatchPlan.TILE_NAMES[fam]] = tf
    arch, rocm = _device_ids()
    px, rad = batch_class(items)
    k = family_key("batch", arch, rocm, px, rad)
    if store:
        _store(k, {"tiles": best, "timings_us": {f: {str(a): round(b, 3) for a, b in t.items()}
                                                 for f, t in timings.items()}}, path)
    return {"tiles": tuple(best), "timings_us": timings, "key": k}


def best_backward_tile(H: int, W: int, ph: int, pw: int, path: str | None = None) -> int:
    arch, rocm = _device_ids()
    entry = load_cache(path).get(family_key("backward", arch, rocm, size_class(H, W), radius_class(ph, pw)))
    return int(entry["tile"]) if entry else 0


def tune_backward(f, psf, params, reps: int = 3, path: str | None = None, store: bool = True,
                  through_wiener: bool = True, K: float = 0.01) -> dict:
    """Time every backward tile-row shape on a checkpointed forward of
    (f, psf, params); every shape must give the same gradients bit for bit."""
    import dataclasses

    import torch

    from . import _lib, deblur_rrrl_backward, deblur_rrrl_iterate, deblur_wiener

    lib = _lib.load()
    H, W = f.shape
    ph, pw = psf.array_shape()
    iters = max(int(params.iters), 1)
    u = torch.empty_like(f)
    ck = torch.empty((iters, H, W), dtype=torch.float32, device=f.device)
    p0 = dataclasses.replace(params, iters=iters)
    deblur_wiener(f, u, psf, K, 1.0, fp64=True)
    deblur_rrrl_iterate(f, u, u, psf, p0, ckpt=ck)
    gu = torch.clamp(u, max=1.0) - 0.5
    ref, timings = None, {}
    for v in range(0, lib.deblur_backward_tile_variants() + 1):
        p = dataclasses.replace(p0, bwd_tile=v)

        def run():
            return deblur_rrrl_backward(f, ck, gu, psf, p, through_wiener=through_wiener, K=K)
        g = run()
        torch.cuda.synchronize()
        if ref is None:
            ref = {k: t.clone() for k, t in g.items()}
        elif any(not torch.equal(g[k], ref[k]) for k in ref):
            raise AssertionError(f"backward tile shape {v} changed the gradients")
        timings[v] = _time(run, reps)
    arch, rocm = _device_ids()
    k = family_key("backward", arch, rocm, size_class(H, W), radius_class(ph, pw))
    best = choose(timings)
    if store:
        _store(k, {"tile": best, "timings_us": {str(a): round(b, 3) for a, b in timings.items()}}, path)
    return {"tile": best, "timings_us": timings, "key": k}
