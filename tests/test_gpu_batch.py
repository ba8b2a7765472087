"""Batched WR3L (one graph launch: the Wiener steps, then per iteration one
launch per tile class, each over a flat tile list of many images of mixed
sizes and PSFs): bitwise equal to the single-image entry points whatever the
tile shapes, within the parity bar of the FP64 oracle, with per-image
completion times."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1212_2245_amd as dbl  # noqa: E402


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def gpu_psf(c):
    if c.kind == synth.KIND_BOX_H:
        return dbl.Psf.box(c.length, "h")
    if c.kind == synth.KIND_BOX_V:
        return dbl.Psf.box(c.length, "v")
    return dbl.Psf.from_taps(dev(c.psf))


def batch_cases(n, sizes=(128, 192, 256)):
    cases = []
    for i in range(n):
        c = synth.make_case(3, image=i, size=sizes[i % len(sizes)])
        c.iters = 4
        cases.append(c)
    return cases


def test_batch_equals_single_image_calls():
    cases = batch_cases(14)
    items = [(dev(c.f), gpu_psf(c), dbl.Params(alpha=c.alpha, iters=c.iters), c.K, 1.0) for c in cases]
    kinds = {c.kind for c in cases}
    assert kinds == {synth.KIND_BOX_H, synth.KIND_BOX_V, synth.KIND_TAPS}
    plan = dbl.BatchPlan(items)
    outs = plan.run()
    torch.cuda.synchronize()
    for (f, psf, p, K, fl), out in zip(items, outs):
        ref = dbl.wr3l(f, psf, K, p, fl)
        assert torch.equal(out, ref)
    # running again gives the same result (plan buffers are reused)
    first = [o.clone() for o in outs]
    plan.run()
    torch.cuda.synchronize()
    for a, b in zip(first, plan.outputs):
        assert torch.equal(a, b)
    lat = plan.latencies_us()
    # one completion time per image, stamped by its last tile
    assert lat.shape == (14,) and np.all(lat > 0) and len(set(lat.tolist())) > 1
    plan.close()


def test_batch_tile_shapes_bitwise_and_class_launches():
    """Every tile shape of every family gives the default plan's outputs bit
    for bit; the per-class launches (for kernel timing) run each class's
    kernels alone and leave the outputs unchanged."""
    cases = batch_cases(14) + batch_cases(4, sizes=(768,))     # box images up to 512^2 and above
    items = [(dev(c.f), gpu_psf(c), dbl.Params(alpha=c.alpha, iters=c.iters), c.K, 1.0) for c in cases]
    ref_plan = dbl.BatchPlan(items)
    ref = [o.clone() for o in ref_plan.run()]
    torch.cuda.synchronize()
    classes = {ref_plan.class_of(i) for i in range(ref_plan.n)}
    assert {4, 5, 6, 7} <= classes and any(c < 4 for c in classes)
    for c in sorted(classes):
        assert ref_plan.class_tiles(c) > 0
        for stage in ((1, 2) if c < 4 else (1,)):
            ref_plan.launch_class(c, stage)
    torch.cuda.synchronize()
    for a, b in zip(ref, ref_plan.outputs):
        assert torch.equal(a, b)
    with pytest.raises(dbl.DeblurError):
        ref_plan.launch_class(4, 2)            # a box class has one kernel
    for c in range(8):
        if c not in classes:
            assert ref_plan.class_tiles(c) == 0
            with pytest.raises(dbl.DeblurError):
                ref_plan.launch_class(c, 1)
    with pytest.raises(dbl.DeblurError):
        ref_plan.class_of(len(items))
    ref_plan.close()
    for fam in range(dbl.BatchPlan.NTILES):
        nv = dbl.BatchPlan.tile_variants(dbl.BatchPlan.STENCIL if fam == 0 else dbl.BatchPlan.BOX)
        for v in range(1, nv + 1):
            t = [0] * dbl.BatchPlan.NTILES
            t[fam] = v
            print(f"[batch] tiles {t}", flush=True)
            plan = dbl.BatchPlan(items, tiles=tuple(t))
            outs = plan.run()
            torch.cuda.synchronize()
            for i, (a, b) in enumerate(zip(outs, ref)):
                assert torch.equal(a, b), (t, i)
            plan.close()


def test_autotune_box_and_batch_families(tmp_path, monkeypatch):
    """The box and batch families of the autotuner: bitwise-checked timings,
    the choice cached and read back (a plan built with tiles='auto' takes it)."""
    from paper_1212_2245_amd import autotune
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tiles.json"))
    c = synth.make_case(0)
    res = autotune.tune_box(dev(c.f), dbl.Psf.box(c.length, "h"), dbl.Params(alpha=c.alpha), iters=2, reps=2)
    assert 0 <= res["tile"] <= 5 and len(res["timings_us"]) == 6
    assert autotune.best_box_tile(256, 256, c.length, "h") == res["tile"]
    assert autotune.best_box_tile(256, 256, c.length, "v") == 0          # not tuned
    cases = batch_cases(8)
    items = [(dev(c.f), gpu_psf(c), dbl.Params(alpha=c.alpha, iters=c.iters), c.K, 1.0) for c in cases]
    r = autotune.tune_batch(items, reps=2)
    assert autotune.best_batch_tiles(items) == r["tiles"]
    plan = dbl.BatchPlan(items, tiles="auto")
    assert plan.tiles == r["tiles"]
    plan.close()


def test_batch_against_oracle_and_groups():
    cases = batch_cases(6, sizes=(96, 144))
    items = [(dev(c.f), gpu_psf(c), dbl.Params(alpha=c.alpha, iters=c.iters), c.K, 1.0) for c in cases]
    plan = dbl.BatchPlan(items, group_size=2)
    outs = plan.run()
    torch.cuda.synchronize()
    for c, out in zip(cases, outs):
        want = oracle.wr3l(c.f, c.psf, c.K, oracle.Params(alpha=c.alpha), c.iters)
        e = float(np.linalg.norm(out.cpu().numpy() - want) / np.linalg.norm(want))
        print(f"[parity] batch image {c.shape} kind {c.kind}: rel_l2={e:.3e}", flush=True)
        assert e <= 1e-4
    lat = plan.latencies_us()
    assert np.all(lat > 0)
    # waves of 2 images enter one iteration apart: the last wave ends last
    assert max(lat[4], lat[5]) > max(lat[0], lat[1])
    plan.close()


def test_batch_fractional_boxes():
    """Boxes of non-integer length in the batched graph: bitwise equal to the
    single-image calls and within the parity bar of the oracle."""
    rng = np.random.default_rng(77)
    specs = [(96, 128, 14.5, "h"), (128, 96, 7.25, "v"), (64, 144, 1.5, "h"), (162, 64, 30.75, "v")]
    items, want = [], []
    for H, W, L, axis in specs:
        h = synth.box_psf(L, axis)
        f = synth.observe(rng, synth.ground_truth(rng, H, W), h, 2.0).astype(np.float32)
        p = dbl.Params(alpha=0.003, iters=4)
        items.append((dev(f), dbl.Psf.box(L, axis), p, 0.01, 1.0))
        want.append(oracle.wr3l(f, h.astype(np.float32), 0.01, oracle.Params(alpha=0.003), 4))
    plan = dbl.BatchPlan(items)
    outs = plan.run()
    torch.cuda.synchronize()
    for (f, psf, p, K, fl), out, w, spec in zip(items, outs, want, specs):
        assert torch.equal(out, dbl.wr3l(f, psf, K, p, fl)), spec
        e = float(np.linalg.norm(out.cpu().numpy() - w) / np.linalg.norm(w))
        print(f"[parity] batch fractional box {spec}: rel_l2={e:.3e}", flush=True)
        assert e <= 1e-4
    plan.close()


def test_batch_method_variants():
    """Per-item method variants in one graph (Perona-Malik regulariser, the
    lookup mode of r_f, plain RL) next to the default method: bitwise equal
    to the single-image calls."""
    rng = np.random.default_rng(5)
    specs = [(96, 128, synth.line_psf(15, 0.4), dbl.Params(alpha=0.02, iters=4, psi=dbl.PSI_PERONA_MALIK, eps_tv=15.0)),
             (128, 96, synth.line_psf(9, 2.0), dbl.Params(alpha=0.003, iters=4, rf_lut=True)),
             (64, 144, None, dbl.Params(alpha=0.0, robust=False, iters=4)),
             (96, 96, synth.line_psf(11, 1.0), dbl.Params(alpha=0.003, iters=4))]
    items = []
    for H, W, h, p in specs:
        psf_arr = h if h is not None else synth.box_psf(9, "h")
        f = synth.observe(rng, synth.ground_truth(rng, H, W), psf_arr, 2.0)
        psf = dbl.Psf.from_taps(dev(psf_arr)) if h is not None else dbl.Psf.box(9, "h")
        items.append((dev(f), psf, p, 0.01, 1.0))
    plan = dbl.BatchPlan(items)
    outs = plan.run()
    torch.cuda.synchronize()
    for (f, psf, p, K, fl), out in zip(items, outs):
        assert torch.equal(out, dbl.wr3l(f, psf, K, p, fl))
    plan.close()


def test_batch_small_images_large_psfs():
    """Images barely larger than their PSFs (halos clamp on both sides of
    every tile) in one graph with a larger image: bitwise equal to the
    single-image calls, for every stencil radius class and both box axes."""
    rng = np.random.default_rng(11)
    specs = [(32, 32, synth.line_psf(31, 0.9)), (36, 48, synth.line_psf(17, 2.3)), (16, 24, synth.line_psf(9, 0.2)),
             (24, 16, synth.random_psf(np.random.default_rng(4), 7, 5)), (16, 48, None), (48, 16, "v"),
             (256, 256, synth.line_psf(31, 1.7))]
    items = []
    for H, W, h in specs:
        if h is None or isinstance(h, str):
            axis = "v" if h == "v" else "h"
            psf_arr, psf = synth.box_psf(13, axis), dbl.Psf.box(13, axis)
        else:
            psf_arr, psf = h, dbl.Psf.from_taps(dev(h))
        f = synth.observe(rng, synth.ground_truth(rng, H, W), psf_arr, 2.0)
        items.append((dev(f), psf, dbl.Params(alpha=0.003, iters=5), 0.01, 1.0))
    plan = dbl.BatchPlan(items)
    outs = plan.run()
    torch.cuda.synchronize()
    for (f, psf, p, K, fl), out in zip(items, outs):
        assert torch.equal(out, dbl.wr3l(f, psf, K, p, fl))
    plan.close()


def test_batch_workload_images_against_oracle():
    """Real images of the 512-image batched workload at their own sizes
    (the largest box and line images among its first 40, 15 iterations),
    run in one plan: each against the FP64 oracle, rel-L2 <= 1e-4 and the
    largest pixel error within 1e-3 of the reference maximum (the per-pixel
    bar of the parity tests)."""
    cases = [synth.make_case(3, image=i) for i in range(40)]
    box = sorted([c for c in cases if c.kind != synth.KIND_TAPS], key=lambda c: -c.shape[0] * c.shape[1])[:2]
    line = sorted([c for c in cases if c.kind == synth.KIND_TAPS], key=lambda c: -c.shape[0] * c.shape[1])[:2]
    chosen = box + line
    items = [(dev(c.f), gpu_psf(c), dbl.Params(alpha=c.alpha, iters=c.iters), c.K, 1.0) for c in chosen]
    plan = dbl.BatchPlan(items)
    outs = plan.run()
    torch.cuda.synchronize()
    for c, out in zip(chosen, outs):
        want = oracle.wr3l(c.f, c.psf, c.K, oracle.Params(alpha=c.alpha), c.iters)
        got = out.cpu().numpy()
        e = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        px = float(np.abs(got - want).max() / np.abs(want).max())
        print(f"[parity] batch workload image {c.shape} kind {c.kind} L {c.length or c.meta.get('L')}: "
              f"rel_l2={e:.3e} max_abs/max|ref|={px:.3e}", flush=True)
        assert e <= 1e-4 and px <= 1e-3
    assert np.all(plan.latencies_us() > 0)
    plan.close()
