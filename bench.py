#!/usr/bin/env python3
"""WR3L benchmark on one MI355X.

Headline workload: the batched form, 512 float32 images with sides drawn from
{128, 192, 256, 384, 512, 768, 1024}, each with its own PSF (half uniform
axis-aligned motion blur of length 5..41, half oblique line blur of length
9..31), noise sigma 1..4, Wiener initialisation then 15 RRRL iterations each.
One step = one launch of the batch plan (one hipGraph: every image's Wiener
step and all iterations), inputs resident in HBM.  value = RRRL megapixel-
iterations per second over the whole batch (sum of H*W*iters / step time,
Wiener time included).  The JSON line also carries:
  * batched: images/s, per-image latency p50/p99 (completion time stamped by
    each image's last tile), for the one-group plan and for 64-image groups;
  * roofline: the batch's dominant kernel (largest time per batch), each
    class kernel timed alone with HIP events on its launch stream, against
    the MI355X peak for its bound (ALU for the stencil classes, HBM for the
    running-sum classes); roofline_classes: every class;
  * ceilings: the HBM fraction each path could reach if it ran at its ALU
    roofline (the paths are ALU-bound per the instruction counts);
  * cpu_baseline: the FP64 oracle on the host cores on a sample of the batch's
    images, with the GPU's error against it on those images;
  * configs: the single-image workloads (256^2 box, 1024^2 oblique line,
    2048^2 Gaussian mixture against the full-size oracle on both
    continuations, the 64 x 512^2 differentiation workload).

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
       python bench.py --ingest-pmc DIR --kernels FRAG...   (rocprofv3 --pmc CSVs -> profiles/kernel_traffic.json)
       python bench.py --summarize-trace CSV OUT [--solo-calls N]   (rocprofv3 kernel trace -> markdown + JSON)
       python bench.py --summarize-counters CSV... OUT --kernels FRAG...
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X fp32 vector (packed FMA), TFLOP/s
FP32_UNPACKED_TFLOPS = 78.6      # the same without packed FP32 (the code is built without it)
CSRC = os.path.join(ROOT, "paper_1212_2245_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")
METRIC = "RRRL megapixel-iterations/s + % HBM peak at ≤1e-4 rel-L2 vs FP64; batched images/s"

# the sources each kernel family is compiled from (its include closure):
# counter figures stay valid while these are unchanged
KERNEL_SOURCES = {
    "stencil": ("rrrl_taps.hip", "stencil_tiles.hpp", "launch.hpp", "psf.hpp", "common.hpp"),
    "box": ("rrrl_box.hip", "box_seg.hpp", "launch.hpp", "common.hpp"),
    "batch": ("batch.hip", "box_seg.hpp", "stencil_tiles.hpp", "launch.hpp", "psf.hpp", "common.hpp"),
}


def family_of(kernel: str) -> str:
    if "batch_" in kernel:
        return "batch"
    if "rrrl_box_iter" in kernel:
        return "box"
    return "stencil"


def kernel_source_hash(family: str) -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[family]:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kernel-reps", type=int, default=50, help="solo launches per class kernel for the roofline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the single-image and differentiation figures")
    ap.add_argument("--no-config2-oracle", action="store_true",
                    help="skip the full-size FP64 oracle of the 2048^2 workload (about a minute of host time)")
    ap.add_argument("--grad-images", type=int, default=64, help="images of the differentiation workload")
    ap.add_argument("--batch-images", type=int, default=512)
    ap.add_argument("--latency-group", type=int, default=64,
                    help="group size of the second plan whose per-image latencies are reported")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="host time budget of the oracle sample")
    ap.add_argument("--tile", default="auto",
                    help="batch tile shapes: auto (tuned here), default, or five variants S,BH,BV,BHL,BVL")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="also copy 256 MiB device-to-device (the scale of the HBM byte counters)")
    ap.add_argument("--ingest-pmc", metavar="DIR", help="parse rocprofv3 --pmc CSVs (DIR/fetch, DIR/write) and exit")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("CSV", "OUT"),
                    help="summarize a rocprofv3 kernel-trace CSV into OUT (.md) and OUT's .json, then exit")
    ap.add_argument("--summarize-counters", nargs="+", metavar="CSV_OR_OUT",
                    help="per-wavefront SQ counters of --kernels from rocprofv3 --pmc CSVs; last argument = OUT")
    ap.add_argument("--kernels", nargs="+", default=[], help="kernel name fragments for --ingest-pmc / counters")
    ap.add_argument("--solo-calls", type=int, default=0,
                    help="with --summarize-trace: launches per class kernel on the bench's timing stream")
    ap.add_argument("--command", default="", help="command line recorded in summaries")
    ap.add_argument("--only-grad", action="store_true",
                    help="run only the differentiation workload (forward + backward timings) and print its JSON")
    ap.add_argument("--quality", action="store_true",
                    help="print the SNR table of the methods on the Table 1 stand-ins (one JSON line) and exit")
    return ap.parse_args()


# ------------------------------------------------------------- profiles
def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").replace("deblur::", "")


def _csv_rows(path: str):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def summarize_trace(path: str, out: str, command: str, solo_calls: int = 0) -> None:
    """Per-kernel, per-stream summary (calls, total, average duration) of a
    rocprofv3 --kernel-trace CSV as markdown (OUT) and JSON (OUT with .json).
    Rows on a stream where a kernel has exactly solo_calls launches are the
    bench's solo timing launches (marked solo)."""
    agg: dict = {}
    for r in _csv_rows(path):
        k = (_short(r["Kernel_Name"]), r.get("Stream_Id", "?"))
        d = agg.setdefault(k, [0, 0.0])
        d[0] += 1
        d[1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
    total = sum(v[1] for v in agg.values()) or 1.0
    rows = sorted(agg.items(), key=lambda kv: -kv[1][1])
    lines = [f"# rocprofv3 kernel trace: {os.path.basename(out)}", "", "Command:", "", "```", command, "```", "",
             "Durations per kernel and stream" + (f"; solo = the {solo_calls} launches per class kernel of the "
                                                   "bench's timing stream" if solo_calls else "") + ".", "",
             "| kernel | stream | calls | total us | avg us | % |", "|---|---|---|---|---|---|"]
    js = {"command": command, "solo_calls": solo_calls,
          "source_hash": {f: kernel_source_hash(f) for f in KERNEL_SOURCES}, "kernels": []}
    for (name, stream), (calls, tot) in rows:
        solo = bool(solo_calls) and calls == solo_calls
        lines.append(f"| `{name}` | {stream}{' (solo)' if solo else ''} | {calls} | {tot:.1f} | {tot / calls:.3f} | "
                     f"{100 * tot / total:.1f} |")
        js["kernels"].append({"kernel": name, "stream": stream, "calls": calls, "total_us": round(tot, 3),
                              "avg_us": round(tot / calls, 3), "solo": solo})
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(os.path.splitext(out)[0] + ".json", "w") as fh:
        json.dump(js, fh, indent=1)
    print("\n".join(lines))


def rocprof_solo_avg(kernel: str, trace_json: str):
    """Average duration (us) of a kernel's solo launches in a committed trace
    summary, or None (no summary, or the kernel's sources changed since)."""
    try:
        d = json.load(open(trace_json))
    except (OSError, ValueError):
        return None
    fam = family_of(kernel)
    if d.get("source_hash", {}).get(fam) != kernel_source_hash(fam):
        return None
    for r in d.get("kernels", []):
        if r["solo"] and r["kernel"] == kernel:
            return r["avg_us"]
    return None


def summarize_counters(paths, out: str, command: str, frags) -> None:
    """Per-wavefront figures of the kernels matching `frags` from rocprofv3
    --pmc CSVs (SQ_* counters, averaged over each kernel's dispatches of its
    largest grid; cycle counters in units of 4 cycles)."""
    vals: dict = {}
    for path in paths:
        acc: dict = {}
        rows = _csv_rows(path)
        top: dict = {}      # per kernel, the dispatches of its largest grid
        for r in rows:
            name = _short(r["Kernel_Name"])
            if any(f in name for f in frags):
                top[name] = max(top.get(name, 0), int(r["Grid_Size"]))
        for r in rows:
            name = _short(r["Kernel_Name"])
            if name not in top or int(r["Grid_Size"]) != top[name]:
                continue
            acc.setdefault((name, r["Counter_Name"]), []).append(float(r["Counter_Value"]))
        for (name, ctr), v in acc.items():
            vals.setdefault(name, {})[ctr] = sum(v) / len(v)
    lines = [f"# rocprofv3 counters: {os.path.basename(out)}", "", "Command (one pass per counter set):", "",
             "```", command, "```", "",
             "Per dispatch (each kernel's dispatches of its largest grid), divided by SQ_WAVES (cycle counters "
             "are in units of 4 cycles).", ""]
    for name, c in sorted(vals.items()):
        w = c.get("SQ_WAVES", 0.0) or 1.0
        lines += [f"## `{name}`", "", "| counter | per dispatch | per wavefront |", "|---|---|---|"]
        for n in sorted(c):
            lines.append(f"| {n} | {c[n]:.0f} | {c[n] / w:.1f} |")
        lines.append("")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


TRAFFIC_JSON = os.path.join(PROFILES, "kernel_traffic.json")
PMC_COPY_BYTES = 256 << 20      # the device copy of --pmc-calibrate


def ingest_pmc(d: str, command: str, frags) -> None:
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the kernels matching
    `frags`, from two rocprofv3 --pmc CSVs under d/fetch and d/write, scaled
    by what the same counters read for the largest plain device copy of the
    run (bench.py --pmc-calibrate copies 256 MiB); merged into
    profiles/kernel_traffic.json with each kernel's source hash."""
    try:
        res = json.load(open(TRAFFIC_JSON))
    except (OSError, ValueError):
        res = {"kernels": {}}
    scale, per, calib = {}, {}, {}
    for ctr, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        paths = glob.glob(os.path.join(d, sub, "**", "*counter_collection.csv"), recursive=True)
        if not paths:
            raise SystemExit(f"no counter CSV under {os.path.join(d, sub)}")
        rows = [r for r in _csv_rows(paths[0]) if r["Counter_Name"] == ctr]
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"]]
        # the calibration copy is the run's last device operation
        last = max(copies, key=lambda r: int(r["Dispatch_Id"]))
        scale[ctr] = PMC_COPY_BYTES / (float(last["Counter_Value"]) * 1024.0)
        calib[ctr] = {"dispatch": int(last["Dispatch_Id"]), "KiB": float(last["Counter_Value"])}
        # per kernel, the dispatches of its largest grid (a batch kernel also
        # runs over the smaller tile lists of 64-image groups)
        top: dict = {}
        for r in rows:
            name = _short(r["Kernel_Name"])
            if any(f in name for f in frags):
                top[name] = max(top.get(name, 0), int(r["Grid_Size"]))
        for r in rows:
            name = _short(r["Kernel_Name"])
            if name in top and int(r["Grid_Size"]) == top[name]:
                per.setdefault(name, {}).setdefault(ctr, []).append(float(r["Counter_Value"]))
    for name, c in per.items():
        e = {k + "_KiB": sum(v) / len(v) for k, v in c.items()}
        e["traffic_bytes"] = (e["FETCH_SIZE_KiB"] * scale["FETCH_SIZE"] + e["WRITE_SIZE_KiB"] * scale["WRITE_SIZE"]) * 1024.0
        e["scale"] = scale
        e["calibration"] = calib
        e["source_hash"] = kernel_source_hash(family_of(name))
        e["command"] = command
        res["kernels"][name] = e
    os.makedirs(PROFILES, exist_ok=True)
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))


def load_traffic(kernel: str):
    """Counted HBM bytes per launch of a kernel, or None (not counted, or its
    sources changed since the counters were taken)."""
    try:
        e = json.load(open(TRAFFIC_JSON))["kernels"].get(kernel)
    except (OSError, ValueError, KeyError):
        return None
    if not e or e.get("source_hash") != kernel_source_hash(family_of(kernel)):
        return None
    return e["traffic_bytes"]


# ------------------------------------------------------------------- batched
CLASS_NAMES = ("stencil_r4", "stencil_r8", "stencil_r16", "stencil_r32", "box_h", "box_v", "box_h_large",
               "box_v_large")
STENCIL_SHAPES = {1: (32, 512), 2: (16, 256), 3: (32, 256)}           # batch stencil variants (rows, threads)
BOX_SHAPES = {False: {1: (256, 8), 2: (128, 16), 3: (64, 32), 4: (64, 8), 5: (64, 4)},   # (along, across)
              True: {1: (128, 16), 2: (256, 8), 3: (64, 32), 4: (64, 8), 5: (64, 4)}}
BATCH_DEFAULT_TILES = (1, 5, 5, 1, 1)   # stencil; box h, v up to 512^2; box h, v above
# algorithmic operations per pixel-iteration beyond the blur taps: the
# robust weight and quotient (~20), the diffusivity (~12) and the diffusion
# term and update (~20) of eqs. (9)-(12), plus the two window sums of each
# running-sum pass (~8 with re-basing) for a box
STENCIL_EXTRA_FLOPS = 40       # per stage, as counted for the roofline (1 FMA = 2 flops)
BOX_OPS_PER_PX = 80            # VALU operations per pixel-iteration of the fused box iteration
BYTES_PER_PX_IT = 12.0         # read u and f, write u'


def class_kernel(cls: int, stage: int, tiles) -> str:
    """The class kernel's name as the kernel trace prints it."""
    if cls >= 4:
        vert, large = cls in (5, 7), cls >= 6
        ta, tc = BOX_SHAPES[vert][tiles[cls - 3]]
        return f"batch_box<{'true' if vert else 'false'}, {ta}, {tc}, {'true' if large else 'false'}>"
    th, nt = STENCIL_SHAPES[tiles[0]]
    return f"batch_stage{stage}<{4 << cls}, {th}, {nt}>"


def batch_workload(dev, n):
    import torch

    import paper_1212_2245_amd as dbl
    import synth

    cases = [synth.make_case(3, image=i) for i in range(n)]

    def gpu_psf(c):
        if c.kind == synth.KIND_BOX_H:
            return dbl.Psf.box(c.length, "h")
        if c.kind == synth.KIND_BOX_V:
            return dbl.Psf.box(c.length, "v")
        return dbl.Psf.from_taps(torch.from_numpy(c.psf).to(dev))

    items = [(torch.from_numpy(c.f).to(dev), gpu_psf(c), dbl.Params(alpha=c.alpha, iters=c.iters), c.K, 1.0)
             for c in cases]
    return cases, items


def time_classes(plan, cases, tiles, reps: int):
    """Every class kernel of the plan launched alone reps times (after one
    warm launch) on a dedicated stream, timed with HIP events on that stream;
    algorithmic work per launch and the rate against the class's roofline."""
    import numpy as np
    import torch

    iters = cases[0].iters
    solo = torch.cuda.Stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cls_of = [plan.class_of(i) for i in range(plan.n)]
    out = []
    for cls in sorted(set(cls_of)):
        imgs = [i for i in range(plan.n) if cls_of[i] == cls]
        px = float(sum(cases[i].f.size for i in imgs))
        for stage in ((1, 2) if cls < 4 else (1,)):
            plan.launch_class(cls, stage, solo)
            ev0.record(solo)
            for _ in range(reps):
                plan.launch_class(cls, stage, solo)
            ev1.record(solo)
            solo.synchronize()
            us = ev0.elapsed_time(ev1) * 1e3 / reps
            name = class_kernel(cls, stage, tiles)
            e = {"class": CLASS_NAMES[cls], "kernel": name, "images": len(imgs), "megapixels": round(px / 1e6, 3),
                 "tiles": plan.class_tiles(cls), "avg_launch_us": round(us, 3), "launches_per_batch": iters,
                 "time_per_batch_us": round(us * iters, 1)}
            if cls < 4:
                taps = [int(np.count_nonzero(cases[i].psf)) for i in imgs]
                per_tap = 2 if stage == 1 else 4        # A: T FMA; B on two channels: 2T FMA
                flops = float(sum((per_tap * t + STENCIL_EXTRA_FLOPS) * cases[i].f.size for t, i in zip(taps, imgs)))
                ach = flops / (us * 1e-6) / 1e12
                e.update({"bound": "alu", "flops_per_launch": flops, "achieved": round(ach, 3), "unit": "TFLOP/s",
                          "peak": FP32_VECTOR_PEAK_TFLOPS, "frac": round(ach / FP32_VECTOR_PEAK_TFLOPS, 4),
                          "frac_of_unpacked": round(ach / FP32_UNPACKED_TFLOPS, 4),
                          "mean_taps": round(float(np.mean(taps)), 1)})
            else:
                nbytes = BYTES_PER_PX_IT * px
                ach = nbytes / (us * 1e-6) / 1e9
                e.update({"bound": "hbm", "bytes_per_launch": nbytes, "achieved": round(ach, 1), "unit": "GB/s",
                          "peak": HBM_PEAK_GBS, "frac": round(ach / HBM_PEAK_GBS, 4)})
            out.append(e)
    return out


def hbm_ceilings(classes):
    """HBM fraction each class could reach at its ALU roofline: the time of
    its algorithmic operations at the unpacked FP32 rate (78.6 TFLOP/s, i.e.
    39.3 T lane-operations/s) against the time of its 12 B per
    pixel-iteration at 8 TB/s."""
    t_hbm = BYTES_PER_PX_IT / (HBM_PEAK_GBS * 1e9)
    ops_rate = FP32_UNPACKED_TFLOPS * 1e12 / 2
    out = {}
    for e in classes:
        if e["bound"] == "alu":
            if not e["kernel"].startswith("batch_stage1"):
                continue
            # both stages: 3T FMA + 2 x 40 extra flops, each extra flop one operation
            ops = 3 * e["mean_taps"] + 2 * STENCIL_EXTRA_FLOPS
        else:
            ops = BOX_OPS_PER_PX
        out[e["class"]] = {"ops_per_px_it": round(ops, 1), "hbm_frac_ceiling": round(min(1.0, t_hbm / (ops / ops_rate)), 3)}
    return out


def percentiles(lat):
    import numpy as np
    return round(float(np.percentile(lat, 50)), 1), round(float(np.percentile(lat, 99)), 1)


# ------------------------------------------------------------ other configs
def _events_ms(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _err(got, want):
    import numpy as np
    got = got.astype(np.float64)
    return {"rel_l2": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
            "max_abs": float(np.abs(got - want).max()),
            "max_abs_rel_to_max": float(np.abs(got - want).max() / np.abs(want).max())}


def config0(dev, args):
    """256^2, horizontal box L=15: Wiener + 10 iterations per solve."""
    import torch

    import paper_1212_2245_amd as dbl
    import synth
    c = synth.make_case(0)
    H, W = c.f.shape
    f = torch.from_numpy(c.f).to(dev)
    psf = dbl.Psf.box(c.length, "h")
    p = dbl.Params(alpha=c.alpha, iters=c.iters)
    u = torch.empty_like(f)
    wsw = torch.empty(dbl.deblur_workspace_bytes(0, H, W, W, psf), dtype=torch.uint8, device=dev)
    wsi = torch.empty(dbl.deblur_workspace_bytes(1, H, W, W, psf, p), dtype=torch.uint8, device=dev)

    def solve0():
        dbl.deblur_wiener(f, u, psf, c.K, 1.0, ws=wsw)
        dbl.deblur_rrrl_iterate(f, u, u, psf, p, ws=wsi)
    ms = _events_ms(solve0, 50)
    msw = _events_ms(lambda: dbl.deblur_wiener(f, u, psf, c.K, 1.0, ws=wsw), 50)
    solve0()
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    e = None
    if not args.no_cpu_baseline:
        import oracle
        e = _err(got, oracle.wr3l(c.f, c.psf, c.K, oracle.Params(alpha=c.alpha), c.iters))
    it_us = (ms - msw) * 1e3 / c.iters
    res = {"workload": "256x256, horizontal box L=15, Wiener K=0.01 + 10 RRRL iterations alpha=0.003",
           "us_per_solve": round(ms * 1e3, 2), "wiener_us": round(msw * 1e3, 2), "iteration_us": round(it_us, 2),
           "mpx_it_per_s": round(H * W / it_us, 1),
           "hbm_frac": round((8 * H * W + 12 * H * W * c.iters) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
           "parity": e}
    it = {}
    for L in (c.length, c.length - 0.5):     # and a non-integer length (fractional end pixels)
        pL = dbl.Psf.box(L, "h")
        wsL = torch.empty(dbl.deblur_workspace_bytes(1, H, W, W, pL, p), dtype=torch.uint8, device=dev)
        it[str(L)] = round(_events_ms(lambda: dbl.deblur_rrrl_iterate(f, f, u, pL, p, ws=wsL), 50) * 1e3 / c.iters, 2)
    res["iteration_us_by_length"] = it
    return res


def config1(dev, args):
    """1024^2, oblique line L=31 (31x31 bilinear PSF): Wiener + 20 iterations,
    the stencil path with autotuned tiles; both stage kernels timed alone."""
    import numpy as np
    import torch

    import paper_1212_2245_amd as dbl
    import synth
    from paper_1212_2245_amd import autotune
    case = synth.make_case(1)
    H, W = case.f.shape
    iters = case.iters
    f = torch.from_numpy(case.f).to(dev)
    psf = dbl.Psf.from_taps(torch.from_numpy(case.psf).to(dev))
    tune = autotune.tune(f, psf, dbl.Params(alpha=case.alpha, iters=iters), store=False)
    tile = int(tune["tile"])
    params = dbl.Params(alpha=case.alpha, iters=iters, tile=tile)
    u = torch.empty_like(f)
    ws_w = torch.empty(dbl.deblur_workspace_bytes(0, H, W, W, psf), dtype=torch.uint8, device=dev)
    ws_i = torch.empty(dbl.deblur_workspace_bytes(1, H, W, W, psf, params), dtype=torch.uint8, device=dev)

    def step():
        dbl.deblur_wiener(f, u, psf, case.K, 1.0, ws=ws_w)
        dbl.deblur_rrrl_iterate(f, u, u, psf, params, ws=ws_i)
    ms = _events_ms(step, 20)
    step()
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    ms_w = _events_ms(lambda: dbl.deblur_wiener(f, u, psf, case.K, 1.0, ws=ws_w), 20)
    taps = dbl.deblur_compile_taps(psf)
    qw = torch.empty((H, W, 2), dtype=torch.float32, device=dev)
    u2 = torch.empty_like(u)
    p1 = dbl.Params(alpha=case.alpha, iters=1, tile=tile)
    T = int(np.count_nonzero(case.psf))
    kt = {}
    for name, fn, per_tap in (("stage1", lambda: dbl.deblur_rrrl_weights(f, u, qw, psf, taps, p1), 2),
                              ("stage2", lambda: dbl.deblur_rrrl_update(qw, u, u2, psf, taps, p1), 4)):
        us = _events_ms(fn, args.kernel_reps) * 1e3
        fl = (per_tap * T + STENCIL_EXTRA_FLOPS) * H * W
        kt[name] = {"avg_launch_us": round(us, 3), "flops_per_launch": fl,
                    "achieved_tflops": round(fl / (us * 1e-6) / 1e12, 3),
                    "frac": round(fl / (us * 1e-6) / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4)}
    res = {"workload": "1024x1024, oblique line blur L=31 (31x31 bilinear PSF, %d taps), Wiener K=0.01 + "
                       "20 RRRL iterations alpha=0.002, replicate border" % T,
           "ms_per_solve": round(ms, 4), "wiener_ms": round(ms_w, 4),
           "iteration_us": round((ms - ms_w) * 1e3 / iters, 3),
           "mpx_it_per_s": round(H * W * iters / (ms * 1e-3) / 1e6, 1),
           "hbm_frac": round((12.0 * H * W * iters + 8.0 * H * W) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
           "tile": tile, "tile_timings_us": {str(k): round(v, 2) for k, v in tune["timings_us"].items()},
           "stage_kernels": kt}
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        want = oracle.wr3l(case.f, case.psf, case.K, oracle.Params(alpha=case.alpha), iters,
                           threads=oracle.default_threads())
        res["parity"] = _err(got, want)
        res["parity"]["oracle_s"] = round(time.perf_counter() - t0, 2)
    return res


def config2(dev, args):
    """2048^2, 31x31 Gaussian mixture, Wiener + 30 iterations: the stencil path
    on both continuations and the FFT path (periodic), each against the
    full-size FP64 oracle on its continuation (Sec. 4.2)."""
    import numpy as np
    import torch

    import paper_1212_2245_amd as dbl
    import synth
    c = synth.make_case(2)
    H, W = c.f.shape
    f = torch.from_numpy(c.f).to(dev)
    psf = dbl.Psf.from_taps(torch.from_numpy(c.psf).to(dev))
    u0 = torch.empty_like(f)
    wsw = torch.empty(dbl.deblur_workspace_bytes(0, H, W, W, psf), dtype=torch.uint8, device=dev)
    msw = _events_ms(lambda: dbl.deblur_wiener(f, u0, psf, c.K, 1.0, ws=wsw), 5)
    T = int(np.count_nonzero(c.psf))
    res = {"workload": "2048x2048, 31x31 Gaussian-mixture PSF (%d taps), Wiener K=0.01 + 30 RRRL iterations "
                       "alpha=0.002" % T, "wiener_us": round(msw * 1e3, 1)}
    outs = {}
    for name, bc, conv in (("stencil_replicate", dbl.BC_REPLICATE, dbl.CONV_STENCIL),
                           ("stencil_periodic", dbl.BC_PERIODIC, dbl.CONV_STENCIL),
                           ("fft_periodic", dbl.BC_PERIODIC, dbl.CONV_FFT)):
        p = dbl.Params(alpha=c.alpha, iters=c.iters, boundary=bc, conv=conv)
        ws = torch.empty(dbl.deblur_workspace_bytes(1, H, W, W, psf, p), dtype=torch.uint8, device=dev)
        uo = torch.empty_like(f)
        ms = _events_ms(lambda: dbl.deblur_rrrl_iterate(f, u0, uo, psf, p, ws=ws), 2)
        outs[name] = uo.cpu().numpy()
        it_us = ms * 1e3 / c.iters
        res[name] = {"iteration_us": round(it_us, 1), "mpx_it_per_s": round(H * W / it_us, 1)}
        if conv == dbl.CONV_STENCIL:
            tflops = (6 * T + 2 * STENCIL_EXTRA_FLOPS) * H * W / (it_us * 1e-6) / 1e12
            res[name]["roofline"] = {"bound": "alu", "achieved_tflops": round(tflops, 2),
                                     "peak": FP32_VECTOR_PEAK_TFLOPS, "frac": round(tflops / FP32_VECTOR_PEAK_TFLOPS, 4)}
    a, b = outs["stencil_periodic"], outs["fft_periodic"]
    res["fft_vs_stencil_periodic_rel_l2"] = float(np.linalg.norm(a - b) / np.linalg.norm(a))
    if not (args.no_cpu_baseline or args.no_config2_oracle):
        import oracle
        threads = oracle.default_threads()
        for bc, names in ((oracle.BC_REPLICATE, ("stencil_replicate",)),
                          (oracle.BC_PERIODIC, ("stencil_periodic", "fft_periodic"))):
            print(f"[bench] 2048^2 FP64 oracle, {'periodic' if bc else 'replicate'} continuation", file=sys.stderr,
                  flush=True)
            t0 = time.perf_counter()
            want = oracle.wr3l(c.f, c.psf, c.K, oracle.Params(alpha=c.alpha, bc=bc), c.iters, threads=threads)
            dt = time.perf_counter() - t0
            for n in names:
                res[n]["vs_oracle"] = _err(outs[n], want)
                res[n]["vs_oracle"]["oracle_s"] = round(dt, 1)
                res[n]["vs_oracle"]["oracle_threads"] = threads
    return res


def config4(dev, args):
    """64 x 512^2 oblique lines (31-tap PSFs): the batch through the autograd
    function (Wiener with FP64 transforms + 10 iterations with per-iteration
    checkpoints, one launch per kernel over all images), then the backward
    through the iterations and the Wiener step (dL/df, dL/dh, dL/dalpha) of
    the L2 loss against the ground truth, batched the same way."""
    import numpy as np
    import torch

    import paper_1212_2245_amd as dbl
    import synth
    cases = [synth.make_case(4, image=i) for i in range(args.grad_images)]
    H, W = cases[0].f.shape
    iters = cases[0].iters
    f = torch.from_numpy(np.stack([c.f for c in cases])).to(dev)
    taps = torch.from_numpy(np.stack([c.psf for c in cases])).to(dev)
    g = torch.from_numpy(np.stack([c.g for c in cases])).to(dev)
    alpha = torch.tensor([c.alpha for c in cases], dtype=torch.float32)      # host: no synchronisation
    K = cases[0].K

    def fwd():
        with torch.no_grad():
            dbl.wr3l_autograd(f, taps, alpha, K, iters)

    def fwd_bwd():
        fr, tr, ar = f.clone().requires_grad_(), taps.clone().requires_grad_(), alpha.clone().requires_grad_()
        u = dbl.wr3l_autograd(fr, tr, ar, K, iters)
        ((u - g) ** 2).sum().backward()

    ms_f = _events_ms(fwd, 2)
    ms_fb = _events_ms(fwd_bwd, 2)
    npx = len(cases) * H * W
    return {"workload": f"{len(cases)} x 512x512, oblique line PSFs (31x31), Wiener (FP64 transforms) + 10 RRRL "
                        "iterations with checkpoints, backward through both, one launch per kernel over the 64 images",
            "images": len(cases), "ms_forward": round(ms_f, 3), "ms_forward_backward": round(ms_fb, 3),
            "images_per_s_fwd_bwd": round(len(cases) / (ms_fb * 1e-3), 1),
            "mpx_it_per_s_fwd_bwd": round(npx * iters / (ms_fb * 1e-3) / 1e6, 1),
            "note": "gradient parity: tests/test_gpu_backward.py"}


def cpu_sample(cases, outputs, budget_s: float):
    """The FP64 oracle on the batch's images in order until budget_s of host
    time is spent (at least one image); throughput and the GPU's error on
    those images."""
    import numpy as np

    import oracle
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    done, errs = [], []
    for i, c in enumerate(cases):
        want = oracle.wr3l(c.f, c.psf, c.K, oracle.Params(alpha=c.alpha), c.iters, threads=threads)
        errs.append(_err(outputs[i], want))
        done.append(i)
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    pxit = sum(cases[i].f.size * cases[i].iters for i in done)
    sizes = sorted({cases[i].f.shape[0] for i in done})
    base = {"value": round(pxit / dt / 1e6, 4), "unit": "Mpx-it/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {len(done)} images of the batch (sides {sizes}, {pxit / 1e6:.1f} Mpx-it), "
                      f"FP64 oracle Wiener + 15 RRRL iterations each, {dt:.1f} s wall on {threads} threads"}
    parity = {"images": len(done), "max_rel_l2": max(e["rel_l2"] for e in errs),
              "max_abs_rel_to_max": max(e["max_abs_rel_to_max"] for e in errs),
              "median_rel_l2": float(np.median([e["rel_l2"] for e in errs])), "tol_rel_l2": 1e-4}
    return base, parity


# ------------------------------------------------------------------- bench
def main():
    args = parse_args()
    if args.ingest_pmc:
        ingest_pmc(args.ingest_pmc, args.command, args.kernels)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters[:-1], args.summarize_counters[-1], args.command, args.kernels)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace[0], args.summarize_trace[1], args.command, args.solo_calls)
        return
    if args.quality:
        import synth
        from paper_1212_2245_amd import quality
        rows = {}
        for sc in synth.table1_scenarios(256, 0):
            rows[sc["name"]] = {
                "full": {k: round(v, 2) for k, v in quality.method_snrs(sc["f"], sc["g"], sc["psf"], sc["K"]).items()},
                "interior24": {k: round(v, 2) for k, v in
                               quality.method_snrs(sc["f"], sc["g"], sc["psf"], sc["K"], border=24).items()}}
        print(json.dumps({"snr_db": rows, "data": "synthetic stand-ins, 256x256, seed 0"}), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (images are independent, "
              "so several GPUs would each take their own share of the images). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1212_2245_amd as dbl

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only_grad:
        print(json.dumps({"grad512x64": config4(dev, args)}), flush=True)
        return

    t0 = time.perf_counter()
    cases, items = batch_workload(dev, args.batch_images)
    gen_s = time.perf_counter() - t0
    iters = cases[0].iters
    npx = sum(c.f.size for c in cases)
    tune = None
    if args.tile == "auto":
        from paper_1212_2245_amd import autotune
        print("[bench] tuning the batch tile shapes", file=sys.stderr, flush=True)
        tune = autotune.tune_batch(items, store=False)
        tiles = tuple(tune["tiles"])
    elif args.tile == "default":
        tiles = (0,) * len(BATCH_DEFAULT_TILES)
    else:
        tiles = tuple(int(t) for t in args.tile.split(","))
    resolved = tuple(t if t > 0 else d for t, d in zip(tiles, BATCH_DEFAULT_TILES))
    t0 = time.perf_counter()
    plan = dbl.BatchPlan(items, tiles=tiles)
    plan_ms = (time.perf_counter() - t0) * 1e3
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps), timing {args.steps} steps of {len(cases)} images",
          file=sys.stderr, flush=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        plan.run()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = max(ev0.elapsed_time(ev1) / args.steps, 1e3 * wall / args.steps)
    lat1 = plan.latencies_us()
    outputs = [o.cpu().numpy() for o in plan.outputs]

    print("[bench] class kernels alone", file=sys.stderr, flush=True)
    classes = time_classes(plan, cases, resolved, args.kernel_reps)
    plan.close()
    dom = max(classes, key=lambda e: e["time_per_batch_us"])
    rp = rocprof_solo_avg(dom["kernel"], os.path.join(PROFILES, "bench_default_kernel_trace.json"))
    roofline = {"bound": dom["bound"], "achieved": dom["achieved"], "peak": dom["peak"], "unit": dom["unit"],
                "frac": dom["frac"], "traffic": load_traffic(dom["kernel"]), "kernel": dom["kernel"],
                "class": dom["class"], "avg_launch_us": dom["avg_launch_us"],
                "work_per_launch": dom.get("flops_per_launch", dom.get("bytes_per_launch")),
                "rocprof_avg_us": rp,
                "frac_rocprof": (round(dom["frac"] * dom["avg_launch_us"] / rp, 4) if rp else None)}

    lat_plan = dbl.BatchPlan(items, group_size=args.latency_group, tiles=tiles)
    lat_plan.run()
    torch.cuda.synchronize()
    lat64 = lat_plan.latencies_us()
    lat_plan.close()
    p50, p99 = percentiles(lat1)
    g50, g99 = percentiles(lat64)
    alg = BYTES_PER_PX_IT * npx * iters + 8.0 * npx
    out = {
        "metric": METRIC, "value": round(npx * iters / (ms_step * 1e-3) / 1e6, 1), "unit": "Mpx-it/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched RRRL: {len(cases)} images, sides from {{128,...,1024}}, half uniform "
                               "axis-aligned motion blur L 5..41, half oblique line blur L 9..31, noise sigma 1..4, "
                               "Wiener + 15 RRRL iterations each, one hipGraph launch per batch",
                   "images": len(cases), "megapixels": round(npx / 1e6, 2), "iters": iters,
                   "tiles": list(resolved), "tile_timings_us": tune["timings_us"] if tune else None},
        "roofline": roofline,
        "batched": {"images_per_s": round(len(cases) / (ms_step * 1e-3), 1),
                    "latency_p50_us": p50, "latency_p99_us": p99,
                    "latency_group": args.latency_group, "group_latency_p50_us": g50, "group_latency_p99_us": g99,
                    "plan_create_ms": round(plan_ms, 1), "generate_s": round(gen_s, 1),
                    "kinds": {"box_h": sum(c.kind == 0 for c in cases), "box_v": sum(c.kind == 1 for c in cases),
                              "line": sum(c.kind == 2 for c in cases)}},
        "hbm": {"algorithmic_bytes_per_step": alg, "achieved_GBs": round(alg / (ms_step * 1e-3) / 1e9, 1),
                "peak_GBs": HBM_PEAK_GBS, "frac": round(alg / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "roofline_classes": classes,
        "ceilings": hbm_ceilings(classes),
    }
    if not args.no_configs:
        print("[bench] single-image and differentiation workloads", file=sys.stderr, flush=True)
        out["configs"] = {"box256": config0(dev, args), "line1024": config1(dev, args),
                          "gauss2048": config2(dev, args), "grad512x64": config4(dev, args)}
    if not args.no_cpu_baseline:
        print("[bench] FP64 oracle on a sample of the batch", file=sys.stderr, flush=True)
        out["cpu_baseline"], out["parity"] = cpu_sample(cases, outputs, args.cpu_seconds)
    if args.pmc_calibrate:
        nbytes = PMC_COPY_BYTES
        a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["pmc_calibration_copy_bytes"] = nbytes
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
