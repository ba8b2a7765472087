"""Method variants in the same kernels (Sec. 2.2-2.3, Table 1): Richardson-Lucy
(alpha = 0, W = 1), RRRL without the Wiener step from a flat or observed
start, and the non-convex Perona-Malik regulariser, against the FP64 oracle
(relative L2 <= 1e-4)."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1212_2245_amd as dbl  # noqa: E402

RTOL_ITER = 1e-4


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def report(name, got, want):
    e = rel_l2(got, want)
    print(f"[parity] {name}: rel_l2={e:.3e}", flush=True)
    return e


def observed(H, W, h, seed):
    rng = np.random.default_rng(seed)
    return synth.observe(rng, synth.ground_truth(rng, H, W), h.astype(np.float64), 2.0).astype(np.float32)


@pytest.mark.parametrize("mode", [dbl.START_FLAT, dbl.START_OBSERVED])
def test_start_images(mode):
    f = observed(77, 130, synth.line_psf(9, 0.5), 5)
    f[:5, :] = 0.0   # below the floor
    u = torch.empty((77, 130), dtype=torch.float32, device="cuda")
    dbl.deblur_rrrl_start(dev(f), u, mode, 1.5)
    want = oracle.rrrl_start(f, mode, 1.5)
    got = u.cpu().numpy()
    if mode == dbl.START_OBSERVED:
        np.testing.assert_array_equal(got, want.astype(np.float32))
    else:
        np.testing.assert_allclose(got, want, rtol=2e-7)
        assert np.all(got == got[0, 0])


@pytest.mark.parametrize("name,H,W,mk,kind,L,iters,kw", [
    # Richardson-Lucy: no regulariser, unit weights (eq. (3) with the adjoint blur)
    ("rl_line11", 64, 80, lambda: synth.line_psf(11, 0.5), synth.KIND_TAPS, 0, 8, dict(alpha=0.0, robust=False)),
    ("rl_box_h9", 64, 96, lambda: synth.box_psf(9, "h"), synth.KIND_BOX_H, 9, 8, dict(alpha=0.0, robust=False)),
    # pure RRRL from a flat start, Table 1's "RRRL 30 it." shape
    ("rrrl_flat_line15_30", 96, 96, lambda: synth.line_psf(15, 2.0), synth.KIND_TAPS, 0, 30, dict(alpha=0.003)),
    ("rrrl_flat_box_v7.5", 80, 64, lambda: synth.box_psf(7.5, "v"), synth.KIND_BOX_V, 7.5, 10, dict(alpha=0.003)),
    # non-convex Perona-Malik regulariser on every convolution path
    ("pm_line13_stencil", 96, 112, lambda: synth.line_psf(13, 1.0), synth.KIND_TAPS, 0, 8,
     dict(alpha=0.02, psi=1, eps_tv=20.0)),
    ("pm_box_h11", 96, 128, lambda: synth.box_psf(11, "h"), synth.KIND_BOX_H, 11, 8,
     dict(alpha=0.02, psi=1, eps_tv=15.0)),
    ("pm_gauss_fft_periodic", 96, 96, lambda: synth.gauss_mixture_psf(synth.rng_for(2), 15), synth.KIND_TAPS, 0, 6,
     dict(alpha=0.02, psi=1, eps_tv=20.0, bc=oracle.BC_PERIODIC, conv=dbl.CONV_FFT)),
])
def test_variant_parity(name, H, W, mk, kind, L, iters, kw):
    h = mk().astype(np.float32)
    f = observed(H, W, h, H + W)
    alpha, robust = kw.get("alpha", 0.003), kw.get("robust", True)
    psi, eps_tv, bc = kw.get("psi", 0), kw.get("eps_tv", 0.1), kw.get("bc", oracle.BC_REPLICATE)
    start = dbl.START_FLAT if name.startswith("rrrl_flat") else dbl.START_OBSERVED
    u0 = oracle.rrrl_start(f, start, 1.0)
    want = oracle.rrrl(f, u0, h, oracle.Params(alpha=alpha, robust=robust, bc=bc, psi=psi, eps_tv=eps_tv), iters)
    if kind == synth.KIND_TAPS:
        psf = dbl.Psf.from_taps(dev(h))
    else:
        psf = dbl.Psf.box(L, "h" if kind == synth.KIND_BOX_H else "v")
    gp = dbl.Params(alpha=alpha, iters=iters, robust=robust, boundary=bc, psi=psi, eps_tv=eps_tv,
                    conv=kw.get("conv", dbl.CONV_AUTO))
    got = dbl.rrrl(dev(f), psf, gp, start=start, pos_floor=1.0).cpu().numpy()
    assert np.all(np.isfinite(got))
    assert report(name, got, want) <= RTOL_ITER


def test_perona_malik_differs_from_tv():
    """The regulariser switch reaches the kernels: at alpha > 0 the two
    penalisers give different iterates, at alpha = 0 identical ones."""
    h = synth.line_psf(9, 0.3).astype(np.float32)
    f = dev(observed(64, 64, h, 3))
    psf = dbl.Psf.from_taps(dev(h))
    outs = {}
    for alpha in (0.0, 0.05):
        for psi in (0, 1):
            outs[alpha, psi] = dbl.rrrl(f, psf, dbl.Params(alpha=alpha, iters=4, psi=psi, eps_tv=10.0))
    assert torch.equal(outs[0.0, 0], outs[0.0, 1])
    assert not torch.equal(outs[0.05, 0], outs[0.05, 1])


@pytest.mark.parametrize("name,H,W,mk,kind,L,kw", [
    ("lut_line17_stencil", 96, 128, lambda: synth.line_psf(17, 0.8), synth.KIND_TAPS, 0, {}),
    ("lut_box_v13", 128, 80, lambda: synth.box_psf(13, "v"), synth.KIND_BOX_V, 13, {}),
    ("lut_line9_fft", 96, 96, lambda: synth.line_psf(9, 2.4), synth.KIND_TAPS, 0,
     dict(bc=oracle.BC_PERIODIC, conv=dbl.CONV_FFT)),
])
def test_rf_lookup_mode_parity(name, H, W, mk, kind, L, kw):
    """r_f by the lookup table of Sec. 4.1 on every iteration path, against the
    oracle's lookup mode; and the lookup's own cost: its distance from the
    exact iteration, on the GPU and in the oracle."""
    h = mk().astype(np.float32)
    f = observed(H, W, h, H * 3 + W)
    bc = kw.get("bc", oracle.BC_REPLICATE)
    u0 = oracle.rrrl_start(f, 1, 1.0)
    want_lut = oracle.rrrl(f, u0, h, oracle.Params(alpha=0.003, bc=bc, rf_lut=True), 10)
    want_exact = oracle.rrrl(f, u0, h, oracle.Params(alpha=0.003, bc=bc), 10)
    psf = dbl.Psf.from_taps(dev(h)) if kind == synth.KIND_TAPS else dbl.Psf.box(L, "v")
    outs = {}
    for lut in (True, False):
        gp = dbl.Params(alpha=0.003, iters=10, boundary=bc, conv=kw.get("conv", dbl.CONV_AUTO), rf_lut=lut)
        outs[lut] = dbl.rrrl(dev(f), psf, gp, start=dbl.START_OBSERVED).cpu().numpy()
    assert report(name + " lut vs oracle lut", outs[True], want_lut) <= RTOL_ITER
    cost_oracle = rel_l2(want_lut, want_exact)
    cost_gpu = report(name + " lut vs exact (gpu)", outs[True], outs[False])
    print(f"[lut] {name}: lookup vs exact: oracle {cost_oracle:.3e}, gpu {cost_gpu:.3e}", flush=True)
    assert cost_oracle > 0.0
    assert abs(cost_gpu - cost_oracle) <= 0.1 * cost_oracle + 2 * RTOL_ITER


def test_rf_lookup_mode_rejected_by_backward():
    h = synth.line_psf(5, 0.3).astype(np.float32)
    f = dev(observed(32, 32, h, 1))
    ck = torch.empty((2, 32, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(dbl.DeblurError):
        dbl.deblur_rrrl_backward(f, ck, f, dbl.Psf.from_taps(dev(h)), dbl.Params(iters=2, rf_lut=True))
