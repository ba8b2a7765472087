"""The batched backward (deblur_rrrl_backward_batch: one launch per kernel for
B equally sized images, image index = blockIdx.z) against one
deblur_rrrl_backward call per image: every gradient equal bit for bit.  The
single-image calls are checked against the FP64 oracle adjoint in
test_gpu_backward.py; equality here carries that parity over to the batch."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1212_2245_amd as dbl  # noqa: E402


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


# (name, B, H, W, pitch, PSF maker, shared PSF, per-image alpha, boundary, iters, through Wiener)
CASES = [
    ("line16_wiener", 5, 48, 96, 96, "line", False, True, dbl.BC_REPLICATE, 3, True),
    ("ragged_pitch_periodic", 3, 36, 72, 80, "random", True, False, dbl.BC_PERIODIC, 2, False),
    ("no_iterations", 4, 64, 64, 64, "random", False, True, dbl.BC_REPLICATE, 0, True),
    ("box_shared", 3, 48, 64, 72, "box", True, True, dbl.BC_REPLICATE, 2, True),
    ("dense_r32", 2, 96, 96, 96, "dense", False, True, dbl.BC_REPLICATE, 2, False),
    # 32 x 512^2: the batch's default tile rows switch to 16 (the one-image calls keep 8) and dL/dh
    # runs on the matrix cores over two column tiles per image
    ("large_batch_default_rows", 32, 512, 512, 512, "line", False, True, dbl.BC_REPLICATE, 2, True),
]


def make_psf(kind, rng, b):
    if kind == "line":
        return synth.line_psf(21, 0.3 + 0.4 * b)
    if kind == "random":
        return synth.random_psf(rng, 5, 7)
    if kind == "dense":
        return synth.random_psf(rng, 41, 33)
    raise ValueError(kind)


@pytest.mark.parametrize("name,B,H,W,pitch,kind,shared,per_alpha,bc,iters,tw", CASES, ids=[c[0] for c in CASES])
def test_backward_batch_equals_single_calls(name, B, H, W, pitch, kind, shared, per_alpha, bc, iters, tw):
    print(f"[batch-bwd] {name} B={B} {H}x{W} pitch {pitch}", flush=True)
    rng = np.random.default_rng(11)
    K = 0.01
    fbuf = torch.zeros((B, H, pitch), dtype=torch.float32, device="cuda")
    fbuf[:, :, :W] = dev(rng.uniform(1.0, 255.0, (B, H, W)))
    f = fbuf[:, :, :W]
    goal = dev(rng.uniform(0.0, 255.0, (B, H, W)))
    if kind == "box":
        psfs = [dbl.Psf.box(9.5, "v")] * B
        taps = psfs[0]
    else:
        hs = [make_psf(kind, rng, 0 if shared else b) for b in range(B)]
        tb = torch.stack([dev(h) for h in hs])
        psfs = [dbl.Psf.from_taps(tb[b]) for b in range(B)]
        taps = tb[0] if shared else tb
        if shared:
            psfs = [dbl.Psf.from_taps(tb[0])] * B
    alphas = [0.002 + 0.001 * b if per_alpha else 0.003 for b in range(B)]
    plist = [dbl.Params(alpha=a, iters=iters, boundary=bc) for a in alphas]
    ckbuf = torch.zeros((B, max(iters, 1), H, pitch), dtype=torch.float32, device="cuda")
    gbuf = torch.zeros((B, H, pitch), dtype=torch.float32, device="cuda")
    for b in range(B):
        u = torch.empty_strided((H, W), (pitch, 1), dtype=torch.float32, device="cuda")
        dbl.deblur_wiener(f[b], u, psfs[b], K, 1.0, fp64=True)
        if iters > 0:
            dbl.deblur_rrrl_iterate(f[b], u, u, psfs[b], plist[b], ckpt=ckbuf[b])
        gbuf[b, :, :W] = 2.0 * (u - goal[b])
    g = gbuf[:, :, :W]
    ck = ckbuf[:, :, :, :W] if iters > 0 else None
    alpha = torch.tensor(alphas, dtype=torch.float32, device="cuda") if per_alpha else None
    got = dbl.deblur_rrrl_backward_batch(f, ck, g, taps, plist[0], alpha=alpha, through_wiener=tw, K=K,
                                         grad_u0=True)
    for b in range(B):
        ref = dbl.deblur_rrrl_backward(f[b], ckbuf[b] if iters > 0 else None, g[b], psfs[b], plist[b],
                                       through_wiener=tw, K=K, grad_u0=True)
        for k in ref:
            assert torch.equal(got[k][b], ref[k]), (name, b, k)
        assert torch.isfinite(ref["f"]).all()
