#!/usr/bin/env python3
"""WR3L benchmark on one MI355X.

Workload (default): one 1024x1024 float32 image (rectangles on a gradient plus
band-limited texture), oblique linear motion blur of length 31 px at a seeded
random angle (31x31 bilinear line PSF), noise sigma 3; Wiener initialisation
(K = 0.01) followed by 20 RRRL iterations with alpha = 0.002.

One step = the whole hot path on that image: deblur_wiener + 20 iterations of
deblur_rrrl_iterate, inputs resident in HBM.  value = RRRL megapixel-
iterations per second of the whole step (H*W*iters / step time, Wiener time
included).  The JSON line also carries:
  * roofline: the dominant kernel's algorithmic rate (timed alone with HIP
    events on its launch stream) against the MI355X peak for its bound;
  * hbm: the iteration's algorithmic bytes (12 B per pixel-iteration read u, f,
    write u; 8 B per pixel for Wiener) per second against 8 TB/s;
  * cpu_baseline: the FP64 oracle on the host cores for the same workload.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
       python bench.py --ingest-pmc DIR   (rocprofv3 --pmc databases -> profiles/)
       python bench.py --summarize-trace DB OUT   (rocprofv3 kernel trace -> markdown)
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X fp32 vector (packed FMA), TFLOP/s
CSRC = os.path.join(ROOT, "paper_1212_2245_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")
METRIC = "RRRL megapixel-iterations/s + % HBM peak at ≤1e-4 rel-L2 vs FP64; batched images/s"

# kernel name fragments as they appear in rocprofv3 traces
KERNELS = {"stage1": "rrrl_taps_stage1", "stage2": "rrrl_taps_stage2"}


# the sources the two stage kernels are compiled from (their include closure):
# the HBM-traffic counters stay valid while these are unchanged
STAGE_SOURCES = ("rrrl_taps.hip", "stencil_tiles.hpp", "launch.hpp", "psf.hpp", "common.hpp")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in STAGE_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kernel-reps", type=int, default=50, help="launches per stage kernel for the roofline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 512-image measurement")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the per-configuration figures (256^2 box, 2048^2 Gaussian stencil/FFT, "
                         "64 x 512^2 forward + backward)")
    ap.add_argument("--grad-images", type=int, default=64, help="images of the differentiation workload")
    ap.add_argument("--batch-images", type=int, default=512)
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--latency-group", type=int, default=64,
                    help="group size of the latency plan (images run group after group)")
    ap.add_argument("--cpu-iters", type=int, default=20, help="RRRL iterations in the oracle sample")
    ap.add_argument("--tile", default="auto",
                    help="stencil tile shape: 'auto' (autotuner, not cached), 0 (library default) or 1..n")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    ap.add_argument("--ingest-pmc", metavar="DIR", help="parse rocprofv3 --pmc databases and exit")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("DB", "OUT"),
                    help="write a markdown summary of a rocprofv3 --kernel-trace database and exit")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DB_OR_OUT",
                    help="rocprofv3 --pmc databases of the stencil stages, then the output markdown file")
    ap.add_argument("--command", default="", help="command line recorded in summaries")
    ap.add_argument("--quality", action="store_true",
                    help="print the SNR table of the methods on the Table 1 stand-ins (one JSON line) and exit")
    return ap.parse_args()


# ------------------------------------------------------------- profiles
def _rocpd_rows(db: str, sql: str):
    import sqlite3
    con = sqlite3.connect(db)
    try:
        return list(con.execute(sql))
    finally:
        con.close()


def summarize_trace(db: str, out: str, command: str) -> None:
    """Per-kernel summary (calls, total, average duration) of a rocprofv3
    --kernel-trace database, as a short markdown file."""
    rows = _rocpd_rows(db, "select name, total_calls, total_duration, average, percentage from top_kernels")
    lines = [f"# rocprofv3 kernel trace: {os.path.basename(out)}", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | total us | avg us | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in rows:
        short = name.split("(")[0].replace("void ", "")
        lines.append(f"| `{short}` | {calls} | {tot:.1f} | {avg:.3f} | {pct:.1f} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_counters(dbs, out: str, command: str) -> None:
    """Per-wavefront figures of the stencil stage kernels from rocprofv3 --pmc
    databases (SQ_* counters; cycle counters in units of 4 cycles)."""
    vals: dict = {}
    for db in dbs:
        for kname, ctr, v in _rocpd_rows(db, "select kernel_name, counter_name, avg(value) from counters_collection "
                                             "group by kernel_name, counter_name"):
            for k, frag in KERNELS.items():
                if frag in kname:
                    vals.setdefault(k, {"name": kname.split("(")[0].replace("void ", "")})[ctr] = v
    lines = [f"# rocprofv3 counters: {os.path.basename(out)}", "", "Command (one pass per counter set):", "",
             "```", command, "```", "",
             "Per dispatch, divided by SQ_WAVES (cycle counters are in units of 4 cycles).", ""]
    for k, c in sorted(vals.items()):
        w = c.get("SQ_WAVES", 0.0) or 1.0
        lines += [f"## {k}: `{c['name']}`", "", "| counter | per dispatch | per wavefront |", "|---|---|---|"]
        for n in sorted(c):
            if n == "name":
                continue
            lines.append(f"| {n} | {c[n]:.0f} | {c[n] / w:.1f} |")
        lines.append("")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def ingest_pmc(d: str, command: str = "") -> None:
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the kernels from two
    rocprofv3 --pmc databases under d/fetch and d/write, scaled by what the
    same counters read for the largest plain device copy in the same run
    (bench.py --pmc-calibrate copies 256 MiB), into
    profiles/stage_kernels_traffic.json."""
    res = {"source_hash": kernel_source_hash(), "command": command, "kernels": {}}
    scale = {}
    for ctr, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        dbs = glob.glob(os.path.join(d, sub, "**", "*.db"), recursive=True)
        if not dbs:
            raise SystemExit(f"no database under {os.path.join(d, sub)}")
        rows = _rocpd_rows(dbs[0], "select kernel_name, value, grid_size from counters_collection "
                                   f"where counter_name = '{ctr}'")
        copies = [r for r in rows if "copyBuffer" in r[0]]
        big = max(copies, key=lambda r: r[2])
        copy_bytes = json.load(open(os.path.join(d, "calib.json")))["copy_bytes"]
        scale[ctr] = copy_bytes / (big[1] * 1024.0)
        for k, frag in KERNELS.items():
            vals = [r[1] for r in rows if frag in r[0]]
            if vals:
                res["kernels"].setdefault(k, {})[ctr + "_KiB"] = sum(vals) / len(vals)
    res["scale"] = scale
    for k, v in res["kernels"].items():
        v["traffic_bytes"] = (v["FETCH_SIZE_KiB"] * scale["FETCH_SIZE"] + v["WRITE_SIZE_KiB"] * scale["WRITE_SIZE"]) * 1024.0
    os.makedirs(PROFILES, exist_ok=True)
    with open(os.path.join(PROFILES, "stage_kernels_traffic.json"), "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))


def load_traffic(kernel: str):
    p = os.path.join(PROFILES, "stage_kernels_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("source_hash") != kernel_source_hash():
        return None  # kernels changed since the counters were taken
    return (d.get("kernels", {}).get(kernel) or {}).get("traffic_bytes")


# ------------------------------------------------------------------- batched
def bench_batched(dev, args):
    """512 images, sides from {128,...,1024}, half uniform axis-aligned motion
    (L 5..41), half oblique lines (L 9..31), 15 iterations each, in one graph
    launch (one group); per-image latency from a second plan whose images run
    in consecutive groups."""
    import torch

    import paper_1212_2245_amd as dbl
    import synth

    t0 = time.perf_counter()
    cases = [synth.make_case(3, image=i) for i in range(args.batch_images)]
    gen_s = time.perf_counter() - t0

    def gpu_psf(c):
        if c.kind == synth.KIND_BOX_H:
            return dbl.Psf.box(c.length, "h")
        if c.kind == synth.KIND_BOX_V:
            return dbl.Psf.box(c.length, "v")
        return dbl.Psf.from_taps(torch.from_numpy(c.psf).to(dev))

    items = [(torch.from_numpy(c.f).to(dev), gpu_psf(c), dbl.Params(alpha=c.alpha, iters=c.iters), c.K, 1.0)
             for c in cases]
    iters = cases[0].iters
    npx = sum(c.f.size for c in cases)
    t0 = time.perf_counter()
    plan = dbl.BatchPlan(items)
    plan_ms = (time.perf_counter() - t0) * 1e3
    plan.run()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.batch_reps):
        plan.run()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.batch_reps
    plan.close()
    lat_plan = dbl.BatchPlan(items, group_size=args.latency_group)
    lat_plan.run()
    torch.cuda.synchronize()
    lat = lat_plan.latencies_us()
    lat_plan.close()
    import numpy as np
    alg = 12.0 * npx * iters + 8.0 * npx
    return {"images": len(cases), "megapixels": round(npx / 1e6, 2), "iters": iters, "ms_per_batch": round(ms, 3),
            "images_per_s": round(len(cases) / (ms * 1e-3), 1),
            "mpx_it_per_s": round(npx * iters / (ms * 1e-3) / 1e6, 1),
            "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "latency_group": args.latency_group,
            "latency_p50_us": round(float(np.percentile(lat, 50)), 1),
            "latency_p99_us": round(float(np.percentile(lat, 99)), 1),
            "plan_create_ms": round(plan_ms, 1), "generate_s": round(gen_s, 1),
            "kinds": {"box_h": sum(c.kind == 0 for c in cases), "box_v": sum(c.kind == 1 for c in cases),
                      "line": sum(c.kind == 2 for c in cases)}}


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


def bench_configs(dev, args):
    """Per-configuration figures beside the headline: the 256^2 box workload
    (Wiener + 10 iterations, parity vs the oracle), the 2048^2 Gaussian-mixture
    workload (30 iterations; stencil with constant and periodic continuation,
    FFT path periodic) and the differentiation workload (64 x 512^2 line PSF,
    Wiener + 10 iterations with checkpoints, then the backward through both)."""
    import numpy as np
    import torch

    import paper_1212_2245_amd as dbl
    import synth
    out = {}

    # config 0: 256^2, horizontal box L=15
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
        t0 = time.perf_counter()
        want = oracle.wr3l(c.f, c.psf, c.K, oracle.Params(alpha=c.alpha), c.iters, threads=1)
        t_cpu = time.perf_counter() - t0
        e = {"rel_l2": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
             "max_abs": float(np.abs(got - want).max()), "oracle_ms_1core": round(t_cpu * 1e3, 2)}
    it_us = (ms - msw) * 1e3 / c.iters
    out["config0_box256"] = {"us_per_solve": round(ms * 1e3, 2), "wiener_us": round(msw * 1e3, 2),
                             "iteration_us": round(it_us, 2),
                             "mpx_it_per_s": round(H * W / it_us, 1),
                             "hbm_frac": round((8 * H * W + 12 * H * W * c.iters) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                             "parity": e}
    # the same image with a box of non-integer length (fractional end pixels)
    # and the integer length next to it, iterations only
    it = {}
    for L in (c.length, c.length - 0.5):
        pL = dbl.Psf.box(L, "h")
        wsL = torch.empty(dbl.deblur_workspace_bytes(1, H, W, W, pL, p), dtype=torch.uint8, device=dev)
        it[str(L)] = round(_events_ms(lambda: dbl.deblur_rrrl_iterate(f, f, u, pL, p, ws=wsL), 50) * 1e3 / c.iters, 2)
    out["config0_box256"]["iteration_us_by_length"] = it

    # config 2: 2048^2, 31x31 Gaussian mixture, 30 iterations
    c = synth.make_case(2)
    H, W = c.f.shape
    f = torch.from_numpy(c.f).to(dev)
    psf = dbl.Psf.from_taps(torch.from_numpy(c.psf).to(dev))
    u0 = torch.empty_like(f)
    wsw = torch.empty(dbl.deblur_workspace_bytes(0, H, W, W, psf), dtype=torch.uint8, device=dev)
    msw = _events_ms(lambda: dbl.deblur_wiener(f, u0, psf, c.K, 1.0, ws=wsw), 5)
    res = {"wiener_us": round(msw * 1e3, 1), "nonzero_taps": int(np.count_nonzero(c.psf))}
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
            # both stencil stages: A (2T flops) and B on two channels (4T), plus ~80 per pixel
            tflops = (6 * res["nonzero_taps"] + 80) * H * W / (it_us * 1e-6) / 1e12
            res[name]["roofline"] = {"bound": "alu", "achieved_tflops": round(tflops, 2),
                                     "peak": FP32_VECTOR_PEAK_TFLOPS, "frac": round(tflops / FP32_VECTOR_PEAK_TFLOPS, 4)}
    a, b = outs["stencil_periodic"], outs["fft_periodic"]
    res["fft_vs_stencil_rel_l2"] = float(np.linalg.norm(a - b) / np.linalg.norm(a))
    out["config2_gauss2048"] = res

    # config 4: forward with checkpoints + backward through Wiener and iterations
    cases = [synth.make_case(4, image=i) for i in range(args.grad_images)]
    H, W = cases[0].f.shape
    iters = cases[0].iters
    data = []
    for c in cases:
        fd = torch.from_numpy(c.f).to(dev)
        psf = dbl.Psf.from_taps(torch.from_numpy(c.psf).to(dev))
        data.append((fd, psf, torch.from_numpy(c.g).to(dev), dbl.Params(alpha=c.alpha, iters=iters), c.K))
    p0 = data[0][3]
    wsw = torch.empty(dbl.deblur_workspace_bytes(0, H, W, W, data[0][1]), dtype=torch.uint8, device=dev)
    wsi = torch.empty(dbl.deblur_workspace_bytes(1, H, W, W, data[0][1], p0), dtype=torch.uint8, device=dev)
    wsb = torch.empty(dbl.deblur_workspace_bytes(3, H, W, W, data[0][1], p0), dtype=torch.uint8, device=dev)
    ck = torch.empty((iters, H, W), dtype=torch.float32, device=dev)
    u = torch.empty((H, W), dtype=torch.float32, device=dev)

    def fwd(i):
        fd, psf, g, p, K = data[i]
        dbl.deblur_wiener(fd, u, psf, K, 1.0, ws=wsw)
        dbl.deblur_rrrl_iterate(fd, u, u, psf, p, ckpt=ck, ws=wsi)

    def fwd_bwd(i):
        fwd(i)
        fd, psf, g, p, K = data[i]
        dbl.deblur_rrrl_backward(fd, ck, 2.0 * (u - g), psf, p, through_wiener=True, K=K, ws=wsb)

    ms_f = _events_ms(lambda: [fwd(i) for i in range(len(data))], 2)
    ms_fb = _events_ms(lambda: [fwd_bwd(i) for i in range(len(data))], 2)
    npx = len(data) * H * W
    out["config4_grad512"] = {"images": len(data), "ms_forward": round(ms_f, 3), "ms_forward_backward": round(ms_fb, 3),
                              "images_per_s_fwd_bwd": round(len(data) / (ms_fb * 1e-3), 1),
                              "mpx_it_per_s_fwd_bwd": round(npx * iters / (ms_fb * 1e-3) / 1e6, 1),
                              "note": "gradient parity: tests/test_gpu_backward.py"}
    return out


# ------------------------------------------------------------------- bench
def main():
    args = parse_args()
    if args.ingest_pmc:
        ingest_pmc(args.ingest_pmc, args.command)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters[:-1], args.summarize_counters[-1], args.command)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace[0], args.summarize_trace[1], args.command)
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

    import numpy as np
    import torch

    import paper_1212_2245_amd as dbl
    import synth

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    case = synth.make_case(1)
    H, W = case.f.shape
    iters = case.iters
    f = torch.from_numpy(case.f).to(dev)
    psf = dbl.Psf.from_taps(torch.from_numpy(case.psf).to(dev))
    tune = None
    if args.tile == "auto":
        from paper_1212_2245_amd import autotune
        tune = autotune.tune(f, psf, dbl.Params(alpha=case.alpha, iters=iters), store=False)
        tile = int(tune["tile"])
    else:
        tile = int(args.tile)
    params = dbl.Params(alpha=case.alpha, iters=iters, tile=tile)
    u = torch.empty_like(f)
    ws_w = torch.empty(dbl.deblur_workspace_bytes(0, H, W, W, psf), dtype=torch.uint8, device=dev)
    ws_i = torch.empty(dbl.deblur_workspace_bytes(1, H, W, W, psf, params), dtype=torch.uint8, device=dev)

    def step():
        dbl.deblur_wiener(f, u, psf, case.K, 1.0, ws=ws_w)
        dbl.deblur_rrrl_iterate(f, u, u, psf, params, ws=ws_i)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps), timing {args.steps} steps", file=sys.stderr, flush=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    ms_step = max(ms_step, 1e3 * wall / args.steps)
    mpxit = H * W * iters / (ms_step * 1e-3) / 1e6
    result_gpu = u.cpu().numpy()

    # Wiener alone and one iteration alone (context)
    ev0.record()
    for _ in range(args.kernel_reps):
        dbl.deblur_wiener(f, u, psf, case.K, 1.0, ws=ws_w)
    ev1.record()
    torch.cuda.synchronize()
    ms_wiener = ev0.elapsed_time(ev1) / args.kernel_reps

    # per-kernel timing of the two stage kernels, each launched alone
    taps = dbl.deblur_compile_taps(psf)
    qw = torch.empty((H, W, 2), dtype=torch.float32, device=dev)
    u2 = torch.empty_like(u)
    p1 = dbl.Params(alpha=case.alpha, iters=1, tile=tile)
    dbl.deblur_rrrl_weights(f, u, qw, psf, taps, p1)
    dbl.deblur_rrrl_update(qw, u, u2, psf, taps, p1)
    torch.cuda.synchronize()
    kt = {}
    for name, fn in (("stage1", lambda: dbl.deblur_rrrl_weights(f, u, qw, psf, taps, p1)),
                     ("stage2", lambda: dbl.deblur_rrrl_update(qw, u, u2, psf, taps, p1))):
        ev0.record()
        for _ in range(args.kernel_reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        kt[name] = ev0.elapsed_time(ev1) / args.kernel_reps * 1e-3   # seconds per launch
    T = int(np.count_nonzero(case.psf))
    # algorithmic flops per pixel: stage 1 = A (T FMA) + robust weight and
    # quotient (~40); stage 2 = B on two channels (2T FMA) + diffusion term and
    # update (~40).  One FMA = 2 flops.
    flops = {"stage1": (2 * T + 40) * H * W, "stage2": (4 * T + 40) * H * W}
    dom = max(kt, key=lambda k: kt[k])
    ach = flops[dom] / kt[dom] / 1e12
    traffic = load_traffic(dom)
    roofline = {"bound": "alu", "achieved": round(ach, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": KERNELS[dom], "avg_launch_us": round(kt[dom] * 1e6, 3),
                "flops_per_launch": flops[dom], "nonzero_taps": T,
                "other_kernel": {"name": KERNELS["stage1" if dom == "stage2" else "stage2"],
                                 "avg_launch_us": round(kt["stage1" if dom == "stage2" else "stage2"] * 1e6, 3)}}
    alg_bytes = 12.0 * H * W * iters + 8.0 * H * W
    hbm_gbs = alg_bytes / (ms_step * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(mpxit, 3), "unit": "Mpx-it/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "oblique line blur L=31 (31x31 bilinear PSF), 1024x1024, Wiener K=0.01 + "
                               "20 RRRL iterations alpha=0.002, robust, TV, replicate border",
                   "H": H, "W": W, "iters": iters, "psf_theta_rad": round(case.meta["theta"], 6),
                   "tile": tile, "tile_timings_us": ({str(k): round(v, 2) for k, v in tune["timings_us"].items()}
                                                     if tune else None)},
        "roofline": roofline,
        "hbm": {"algorithmic_bytes_per_step": alg_bytes, "achieved_GBs": round(hbm_gbs, 2),
                "peak_GBs": HBM_PEAK_GBS, "frac": round(hbm_gbs / HBM_PEAK_GBS, 5)},
        "wiener_ms": round(ms_wiener, 5),
        "iteration_us": round((ms_step - ms_wiener) * 1e3 / iters, 3),
    }
    # the same iterations with r_f through the lookup table of Sec. 4.1
    # (speed only; its accuracy cost is measured by the parity tests)
    p_lut = dbl.Params(alpha=case.alpha, iters=iters, tile=tile, rf_lut=True)
    ws_l = torch.empty(dbl.deblur_workspace_bytes(1, H, W, W, psf, p_lut), dtype=torch.uint8, device=dev)
    us_it = {}
    u_it = torch.empty_like(u)
    for name, pp, wsx in (("exact", params, ws_i), ("lookup", p_lut, ws_l)):
        dbl.deblur_rrrl_iterate(f, u, u_it, psf, pp, ws=wsx)
        ev0.record()
        for _ in range(max(1, args.kernel_reps // 4)):
            dbl.deblur_rrrl_iterate(f, u, u_it, psf, pp, ws=wsx)
        ev1.record()
        torch.cuda.synchronize()
        us_it[name] = round(ev0.elapsed_time(ev1) / max(1, args.kernel_reps // 4) * 1e3 / iters, 3)
    out["rf_iteration_us"] = us_it

    if not args.no_batched:
        print(f"[bench] batched workload: {args.batch_images} images", file=sys.stderr, flush=True)
        out["batched"] = bench_batched(dev, args)

    if not args.no_configs:
        print("[bench] per-configuration figures", file=sys.stderr, flush=True)
        out["configs"] = bench_configs(dev, args)

    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.default_threads()
        t0 = time.perf_counter()
        want = oracle.wr3l(case.f, case.psf, case.K, oracle.Params(alpha=case.alpha), args.cpu_iters,
                           threads=threads)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(H * W * args.cpu_iters / dt / 1e6, 4), "unit": "Mpx-it/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"the full workload image (1024x1024), FP64 oracle Wiener + "
                                         f"{args.cpu_iters} RRRL iterations, {dt:.2f} s wall"}
        if args.cpu_iters == iters:
            e = float(np.linalg.norm(result_gpu.astype(np.float64) - want) / np.linalg.norm(want))
            out["parity"] = {"rel_l2": e, "max_abs": float(np.abs(result_gpu - want).max()), "tol": 1e-4}

    if args.pmc_calibrate:
        nbytes = 256 << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["pmc_calibration_copy_bytes"] = nbytes
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
