"""The batched forward entry points (deblur_wiener_batch,
deblur_rrrl_iterate_batch: one launch per kernel for B equally sized images,
image index = blockIdx.z) against one deblur_wiener / deblur_rrrl_iterate call
per image: outputs and checkpoints equal bit for bit.  The single-image calls
are checked against the FP64 oracle in test_gpu_parity.py; equality here
carries that parity over to the batch."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1212_2245_amd as dbl  # noqa: E402


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def images(rng, B, H, W, pitch):
    buf = torch.zeros((B, H, pitch), dtype=torch.float32, device="cuda")
    buf[:, :, :W] = dev(rng.uniform(1.0, 255.0, (B, H, W)))
    return buf[:, :, :W]


def psfs_for(kind, rng, B):
    """(argument for the batched call, per-image Psf list)."""
    if kind == "box_h":
        p = dbl.Psf.box(15, "h")
        return p, [p] * B
    if kind == "box_v_frac":
        p = dbl.Psf.box(9.5, "v")
        return p, [p] * B
    if kind == "shared_random":
        t = dev(synth.random_psf(rng, 5, 7))
        return t, [dbl.Psf.from_taps(t)] * B
    if kind == "row_taps":
        tb = torch.stack([dev(synth.random_psf(rng, 1, 9)) for _ in range(B)])
        return tb, [dbl.Psf.from_taps(tb[b]) for b in range(B)]
    tb = torch.stack([dev(synth.line_psf(21, 0.3 + 0.5 * b)) for b in range(B)])
    return tb, [dbl.Psf.from_taps(tb[b]) for b in range(B)]


@pytest.mark.parametrize("kind,fp64,H,W,pitch", [("lines", True, 48, 96, 104), ("lines", False, 64, 64, 64),
                                                 ("row_taps", False, 36, 72, 72), ("box_h", True, 48, 64, 64)],
                         ids=["lines_fp64_pitch", "lines_fp32", "rowwise", "box_fp64"])
def test_wiener_batch_equals_single_calls(kind, fp64, H, W, pitch):
    print(f"[fwd-batch] wiener {kind} fp64={fp64} {H}x{W}", flush=True)
    rng = np.random.default_rng(3)
    B = 5
    f = images(rng, B, H, W, pitch)
    arg, psfs = psfs_for(kind, rng, B)
    u = torch.full((B, H, pitch), -7.0, dtype=torch.float32, device="cuda")[:, :, :W]
    dbl.deblur_wiener_batch(f, u, arg, 0.01, 1.5, fp64=fp64)
    for b in range(B):
        ref = torch.empty_strided((H, W), (pitch, 1), dtype=torch.float32, device="cuda")
        dbl.deblur_wiener(f[b], ref, psfs[b], 0.01, 1.5, fp64=fp64)
        assert torch.equal(u[b], ref), (kind, b)


# (name, PSF kind, B, H, W, pitch, iters, in place, checkpoints, per-image alpha, boundary, conv)
ITER_CASES = [
    ("lines_inplace_odd", "lines", 5, 48, 96, 104, 3, True, True, True, dbl.BC_REPLICATE, dbl.CONV_AUTO),
    ("shared_periodic", "shared_random", 3, 36, 72, 72, 4, False, False, False, dbl.BC_PERIODIC, dbl.CONV_AUTO),
    ("box_runsum", "box_h", 4, 48, 64, 72, 2, True, True, True, dbl.BC_REPLICATE, dbl.CONV_AUTO),
    ("box_frac_stencil", "box_v_frac", 3, 40, 64, 64, 3, False, True, True, dbl.BC_REPLICATE, dbl.CONV_STENCIL),
    ("no_iterations", "lines", 3, 32, 64, 64, 0, False, False, True, dbl.BC_REPLICATE, dbl.CONV_AUTO),
    # 16 x 512^2: the batch's default stencil tile switches to 32 rows (the one-image calls take 16)
    ("large_batch", "lines", 16, 512, 512, 512, 2, True, True, True, dbl.BC_REPLICATE, dbl.CONV_AUTO),
]


@pytest.mark.parametrize("name,kind,B,H,W,pitch,iters,inplace,ckpt,per_alpha,bc,conv", ITER_CASES,
                         ids=[c[0] for c in ITER_CASES])
def test_iterate_batch_equals_single_calls(name, kind, B, H, W, pitch, iters, inplace, ckpt, per_alpha, bc, conv):
    print(f"[fwd-batch] iterate {name} B={B} {H}x{W} pitch {pitch}", flush=True)
    rng = np.random.default_rng(5)
    f = images(rng, B, H, W, pitch)
    u0 = images(rng, B, H, W, pitch)
    arg, psfs = psfs_for(kind, rng, B)
    alphas = [0.002 + 0.0015 * b if per_alpha else 0.003 for b in range(B)]
    base = dbl.Params(alpha=0.003, iters=iters, boundary=bc, conv=conv)
    plist = [dbl.Params(alpha=a, iters=iters, boundary=bc, conv=conv) for a in alphas]
    ad = torch.tensor(alphas, dtype=torch.float32, device="cuda") if per_alpha else None
    u_in = torch.empty_strided(u0.shape, u0.stride(), dtype=torch.float32, device="cuda").copy_(u0) if inplace else u0
    if inplace:
        u_out = u_in
    else:
        u_out = torch.full((B, H, pitch), -3.0, dtype=torch.float32, device="cuda")[:, :, :W]
    ckb = torch.full((B, max(iters, 1), H, pitch), -5.0, dtype=torch.float32, device="cuda") if ckpt else None
    ck = ckb[:, :, :, :W] if ckpt else None
    dbl.deblur_rrrl_iterate_batch(f, u_in, u_out, arg, base, alpha=ad, ckpt=ck)
    for b in range(B):
        ref = torch.empty_strided((H, W), (pitch, 1), dtype=torch.float32, device="cuda")
        rck = torch.full((max(iters, 1), H, pitch), -5.0, dtype=torch.float32, device="cuda") if ckpt else None
        dbl.deblur_rrrl_iterate(f[b], u0[b], ref, psfs[b], plist[b], ckpt=rck)
        assert torch.equal(u_out[b], ref), (name, b)
        if ckpt:
            assert torch.equal(ckb[b, :, :, :W], rck[:, :, :W]), (name, b)
