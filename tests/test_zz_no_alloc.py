"""deblur_rrrl_iterate_noalloc (the entry point for callers that cannot
allocate): through the C ABI, its output must equal deblur_rrrl_iterate's bit
for bit (same kernels; the workspace is the library's static scratch instead
of the caller's), on consecutive calls that reuse the scratch, the second
with a smaller image, on the stencil, running-sum and Fourier paths."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1212_2245_amd as dbl  # noqa: E402


def _pitched(H, W, pitch, value):
    """H x W view with row pitch `pitch` of a device buffer filled with value."""
    return torch.full((H, pitch), value, dtype=torch.float32, device="cuda")[:, :W]


def _inputs(rng, H, W, pitch):
    f, u = _pitched(H, W, pitch, 0.0), _pitched(H, W, pitch, 0.0)
    f.copy_(torch.from_numpy(synth.random_image(rng, H, W, 0.0, 255.0)))
    u.copy_(torch.from_numpy(synth.random_image(rng, H, W, 1.0, 255.0)))
    return f, u


def _psf(kind, rng):
    if kind == "line":
        return dbl.Psf.from_taps(torch.from_numpy(synth.line_psf(21, 0.7)).float().cuda())
    if kind == "dense":
        return dbl.Psf.from_taps(torch.from_numpy(synth.random_psf(rng, 9, 7)).float().cuda())
    if kind == "box_h":
        return dbl.Psf.box(13.5, "h")
    return dbl.Psf.box(9, "v")


# (psf, conv, boundary, first (H, W, pitch), second smaller (H, W, pitch))
CASES = [
    ("line", dbl.CONV_AUTO, dbl.BC_REPLICATE, (384, 512, 520), (136, 200, 200)),
    ("dense", dbl.CONV_STENCIL, dbl.BC_PERIODIC, (256, 320, 320), (96, 160, 168)),
    ("box_h", dbl.CONV_AUTO, dbl.BC_REPLICATE, (300, 700, 704), (64, 90, 96)),
    ("box_v", dbl.CONV_RUNSUM, dbl.BC_PERIODIC, (512, 256, 256), (128, 72, 80)),
    ("line", dbl.CONV_FFT, dbl.BC_PERIODIC, (256, 384, 384), (96, 128, 128)),
]


@pytest.mark.parametrize("kind,conv,bc,first,second", CASES, ids=[f"{c[0]}-conv{c[1]}-bc{c[2]}" for c in CASES])
def test_noalloc_matches_workspace_entry(kind, conv, bc, first, second):
    rng = synth.rng_for(97, conv * 10 + bc)
    psf = _psf(kind, rng)
    for call, (H, W, pitch) in enumerate((first, second)):
        iters = 5 - call   # odd, then even: both ping-pong parities
        p = dbl.Params(alpha=0.003, iters=iters, conv=conv, boundary=bc)
        f, u0 = _inputs(rng, H, W, pitch)
        ck_ref = torch.full((iters, H, pitch), -1.0, device="cuda")
        ck_na = torch.full((iters, H, pitch), -1.0, device="cuda")
        ref = _pitched(H, W, pitch, -1.0)
        dbl.deblur_rrrl_iterate(f, u0, ref, psf, p, ckpt=ck_ref)
        got = _pitched(H, W, pitch, -2.0)
        dbl.deblur_rrrl_iterate_noalloc(f, u0, got, psf, p, ckpt=ck_na)
        # in place (u_in == u_out), as the other entry point allows
        inplace = _pitched(H, W, pitch, 0.0)
        inplace.copy_(u0)
        dbl.deblur_rrrl_iterate_noalloc(f, inplace, inplace, psf, p)
        torch.cuda.synchronize()
        print(f"[noalloc] {kind} conv={conv} bc={bc} call {call}: {H}x{W} pitch {pitch}, {iters} iterations",
              flush=True)
        assert torch.equal(got, ref), (kind, call, (got - ref).abs().max().item())
        assert torch.equal(inplace, ref), (kind, call)
        assert torch.equal(ck_na[:, :, :W], ck_ref[:, :, :W])
        assert np.isfinite(ref.cpu().numpy()).all() and float(ref.min()) > 0.0


def test_noalloc_rejects_oversize_before_enqueue():
    """A stencil problem needing more than the 64 MiB scratch is refused and
    its output stays untouched."""
    H = W = 2048
    rng = synth.rng_for(97, 99)
    psf = dbl.Psf.from_taps(torch.from_numpy(synth.random_psf(rng, 5, 5)).float().cuda())
    f = torch.ones(H, W, device="cuda")
    u = torch.ones(H, W, device="cuda")
    out = torch.full_like(f, 7.0)
    with pytest.raises(dbl.DeblurError, match="scratch"):
        dbl.deblur_rrrl_iterate_noalloc(f, u, out, psf, dbl.Params(iters=2))
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
