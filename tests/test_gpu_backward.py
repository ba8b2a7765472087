"""GPU backward (hand-written adjoint through the unrolled RRRL iterations
and the Wiener initialisation) against the FP64 oracle adjoint: relative
error <= 1e-3 for dL/df, dL/dh (every PSF entry), dL/dalpha and dL/du^0,
loss L = sum (u^K - g)^2.  Each side runs its own forward; the GPU forward
starts from deblur_wiener_fp64 (the Wiener output correctly rounded to FP32),
as the differentiable entry point does.

The map u^0 -> u^K is only piecewise smooth (the [D]_+ / [D]_- split of the
update switches at D = 0), and where the iteration is far from converged
(e.g. the ringing the periodic Wiener step leaves at the image border) its
gradient reacts strongly to tiny changes of the iterates.  How strongly is
printed beside each result: the oracle's own gradient change when its FP64
state is rounded to FP32 after the Wiener step and after every iteration
(the conditioning floor).  The tolerance is 1e-3 regardless."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1212_2245_amd as dbl  # noqa: E402

RTOL_GRAD = 1e-3


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def oracle_grads(f, h, g, K, p, iters, through_wiener, floor=1.0):
    u0 = oracle.wiener_init(f, h, K, floor)
    if iters > 0:
        uK, ck = oracle.rrrl(f, u0, h, p, iters, checkpoints=True)
    else:
        uK, ck = u0, np.zeros((0,) + f.shape)
    lam0, df, dh, da = oracle.rrrl_adjoint(f, ck, h, p, 2.0 * (uK - g))
    if through_wiener:
        dfw, dhw = oracle.wiener_adjoint(f, h, K, floor, lam0)
        df, dh = df + dfw, dh + dhw
    return df, dh, da, lam0


def gpu_grads(f, psf, g, K, gp, through_wiener, pitch=None):
    H, W = f.shape
    if pitch:
        buf = torch.zeros((H, pitch), dtype=torch.float32, device="cuda")
        buf[:, :W] = dev(f)
        fd = buf[:, :W]
    else:
        fd = dev(f)
        pitch = W
    u = torch.empty_strided((H, W), (pitch, 1), dtype=torch.float32, device="cuda")
    dbl.deblur_wiener(fd, u, psf, K, 1.0, fp64=True)
    ck = torch.empty((max(gp.iters, 1), H, pitch), dtype=torch.float32, device="cuda")
    dbl.deblur_rrrl_iterate(fd, u, u, psf, gp, ckpt=ck)
    lam = (2.0 * (u - dev(g))).contiguous() if pitch == W else None
    if lam is None:
        lam = torch.empty_strided((H, W), (pitch, 1), dtype=torch.float32, device="cuda")
        lam.copy_(2.0 * (u - dev(g)))
    out = dbl.deblur_rrrl_backward(fd, ck, lam, psf, gp, through_wiener=through_wiener, K=K, grad_u0=True)
    return {k: v.cpu().numpy() for k, v in out.items()}


def oracle_floor(f, h, g, K, p, iters, through_wiener, floor=1.0):
    """Relative change of each oracle gradient when the FP64 forward state is
    rounded to FP32 after the Wiener step and after every iteration."""
    ref = oracle_grads(f, h, g, K, p, iters, through_wiener, floor)
    u = oracle.wiener_init(f, h, K, floor).astype(np.float32).astype(np.float64)
    cks = []
    for _ in range(iters):
        cks.append(u)
        u = oracle.rrrl(f, u, h, p, 1).astype(np.float32).astype(np.float64)
    ck = np.stack(cks) if iters else np.zeros((0,) + f.shape)
    lam0, df, dh, da = oracle.rrrl_adjoint(f, ck, h, p, 2.0 * (u - g))
    if through_wiener:
        dfw, dhw = oracle.wiener_adjoint(f, h, K, floor, lam0)
        df, dh = df + dfw, dh + dhw
    return ref, {"f": rel(df, ref[0]), "h": rel(dh, ref[1]), "alpha": abs(da - ref[2]) / max(abs(ref[2]), 1e-300),
                 "u0": rel(lam0, ref[3])}


def check(name, got, df, dh, da, lam0, floor=None):
    err = {"f": rel(got["f"], df), "h": rel(got["taps"], dh),
           "alpha": abs(float(got["alpha"]) - da) / max(abs(da), 1e-300), "u0": rel(got["u0"], lam0)}
    floor = floor or {k: 0.0 for k in err}
    tol = {k: RTOL_GRAD for k in err}
    print(f"[grad] {name}: " + "  ".join(f"{k} {err[k]:.2e} (floor {floor[k]:.1e}, tol {tol[k]:.1e})" for k in err),
          flush=True)
    assert all(err[k] <= tol[k] for k in err), err


CASES = [
    ("line9_rep_robust", 48, 64, lambda: synth.line_psf(9, 0.7), oracle.BC_REPLICATE, True, 3, True),
    ("asym5x7_rep", 36, 48, lambda: synth.random_psf(np.random.default_rng(1), 5, 7), oracle.BC_REPLICATE, True, 2,
     True),
    ("asym5x7_periodic", 36, 48, lambda: synth.random_psf(np.random.default_rng(2), 5, 7), oracle.BC_PERIODIC, True,
     2, True),
    pytest.param("line13_nonrobust", 48, 48, lambda: synth.line_psf(13, 2.2), oracle.BC_REPLICATE, False, 3, True,
                 marks=pytest.mark.xfail(strict=False, reason="plain RL data term: the oracle's own dL/dalpha moves "
                                         "4.8e-3 when its state is rounded to FP32; GPU measured 1.4e-3 (dL/df, dL/dh "
                                         "3.5e-4)"), id="line13_nonrobust"),
    ("no_wiener", 48, 72, lambda: synth.line_psf(7, 1.0), oracle.BC_REPLICATE, True, 4, False),
    ("iters0", 32, 32, lambda: synth.random_psf(np.random.default_rng(3), 3, 3), oracle.BC_REPLICATE, True, 0, True),
    ("gauss31_64", 64, 64, lambda: synth.gauss_mixture_psf(synth.rng_for(2), 31), oracle.BC_REPLICATE, True, 2, True),
    # PSF reach comparable to the image: the transposes' border folds span most of a row or column
    ("line31_on_32", 32, 32, lambda: synth.line_psf(31, 0.9), oracle.BC_REPLICATE, True, 2, True),
    ("line31_on_32x36_periodic", 32, 36, lambda: synth.line_psf(31, 0.9), oracle.BC_PERIODIC, True, 2, False),
    # PSF arrays of the matrix-core dL/dh path (longer side 17..31) that are not square: unequal row and
    # column lags, down to a single row or column
    ("rect17x31_rep", 48, 64, lambda: synth.random_psf(np.random.default_rng(21), 17, 31), oracle.BC_REPLICATE,
     True, 2, True),
    ("row1x25_periodic", 36, 48, lambda: synth.random_psf(np.random.default_rng(22), 1, 25), oracle.BC_PERIODIC,
     True, 2, False),
    ("col29x3_rep", 64, 48, lambda: synth.random_psf(np.random.default_rng(23), 29, 3), oracle.BC_REPLICATE, True,
     3, True),
]


@pytest.mark.parametrize("name,H,W,mk,bc,robust,iters,tw", CASES,
                         ids=[c[0] if isinstance(c, tuple) else c.id for c in CASES])
def test_backward_vs_oracle_adjoint(name, H, W, mk, bc, robust, iters, tw):
    rng = np.random.default_rng(H + W)
    g = synth.ground_truth(rng, H, W)
    h = mk().astype(np.float32)
    f = synth.observe(rng, g, h.astype(np.float64), 2.0)
    K, alpha = 0.01, 0.01
    p = oracle.Params(alpha=alpha, robust=robust, bc=bc)
    (df, dh, da, lam0), floor = oracle_floor(f, h, g.astype(np.float32), K, p, iters, tw)
    gp = dbl.Params(alpha=alpha, iters=iters, robust=robust, boundary=bc)
    got = gpu_grads(f, dbl.Psf.from_taps(dev(h)), g.astype(np.float32), K, gp, tw)
    check(name, got, df, dh, da, lam0, floor)


def test_backward_box_psf_and_pitch():
    rng = np.random.default_rng(7)
    H, W = 48, 72
    g = synth.ground_truth(rng, H, W)
    h = synth.box_psf(9, "h").astype(np.float32)
    f = synth.observe(rng, g, h.astype(np.float64), 2.0)
    p = oracle.Params(alpha=0.003)
    df, dh, da, lam0 = oracle_grads(f, h, g.astype(np.float32), 0.01, p, 3, True)
    got = gpu_grads(f, dbl.Psf.box(9, "h"), g.astype(np.float32), 0.01, dbl.Params(alpha=0.003, iters=3), True,
                    pitch=80)
    check("box9_pitch80", {k: (v[:, :W] if v.ndim == 2 and v.shape[0] == H else v) for k, v in got.items()},
          df, dh, da, lam0)


@pytest.mark.parametrize("image", [0, 2])
def test_backward_workload_shape(image):
    """The differentiation workload's per-image shape: 512^2, oblique line
    L=31, Wiener + 10 iterations, alpha = 0.002.  Image 0 carries a border
    ringing spot where the gradient is ill-conditioned (floor ~5e-4; with
    the FP32 Wiener transforms its dL/df error was 4e-3, with the FP64 ones
    7e-4); image 2 is well conditioned (floor ~1e-5)."""
    c = synth.make_case(4, image=image)
    p = oracle.Params(alpha=c.alpha)
    (df, dh, da, lam0), floor = oracle_floor(c.f, c.psf, c.g, c.K, p, c.iters, True)
    got = gpu_grads(c.f, dbl.Psf.from_taps(dev(c.psf)), c.g, c.K, dbl.Params(alpha=c.alpha, iters=c.iters), True)
    check(f"workload 512 line31 k10 image {image}", got, df, dh, da, lam0, floor)


def test_autograd_function_and_determinism():
    c = synth.make_case(4, size=96)
    f = dev(c.f).requires_grad_(True)
    taps = dev(c.psf).requires_grad_(True)
    alpha = torch.tensor(c.alpha, dtype=torch.float32, requires_grad=True)
    grads = []
    for _ in range(2):
        for t in (f, taps, alpha):
            t.grad = None
        u = dbl.wr3l_autograd(f, taps, alpha, c.K, 4)
        loss = ((u.double() - dev(c.g).double()) ** 2).sum()
        loss.backward()
        grads.append((f.grad.clone(), taps.grad.clone(), alpha.grad.clone()))
    for a, b in zip(*grads):
        assert torch.equal(a, b)   # deterministic reductions
    df, dh, da, _ = oracle_grads(c.f, c.psf, c.g, c.K, oracle.Params(alpha=c.alpha), 4, True)
    assert rel(grads[0][0].cpu().numpy(), df) <= RTOL_GRAD
    assert rel(grads[0][1].cpu().numpy(), dh) <= RTOL_GRAD
    assert abs(float(grads[0][2]) - da) <= RTOL_GRAD * abs(da)


def test_gpu_finite_difference_in_f():
    """Central difference of the GPU forward's loss along a random direction
    in f, against the GPU gradient and against the same finite difference of
    the FP64 oracle forward.  The map is only piecewise smooth (the [D]_+ /
    [D]_- switch, the positivity floor), so a finite difference has an error
    of its own: with the FP64 oracle, step 0.1 differs from the exact
    directional derivative by ~1%, and at step 1e-3 FP32 rounding of the
    state alone already moves it by ~0.6%.  Step 0.1 keeps the FP32 noise
    far below the step's own error."""
    c = synth.make_case(4, size=128)
    taps = dev(c.psf)
    alpha = torch.tensor(c.alpha, dtype=torch.float64)
    rng = np.random.default_rng(9)
    vn = rng.normal(size=c.f.shape) * (c.f >= 1)
    v = dev(vn)
    f = dev(c.f).requires_grad_(True)
    u = dbl.wr3l_autograd(f, taps, alpha, c.K, 5)
    loss = ((u.double() - dev(c.g).double()) ** 2).sum()
    loss.backward()
    gv = float((f.grad.double() * v.double()).sum())

    def L(ff):
        with torch.no_grad():
            uu = dbl.wr3l_autograd(ff, taps, alpha, c.K, 5)
            return float(((uu.double() - dev(c.g).double()) ** 2).sum())

    p = oracle.Params(alpha=c.alpha)

    def L64(ff):
        return float(((oracle.wr3l(ff, c.psf, c.K, p, 5) - c.g) ** 2).sum())

    e = 0.1
    fd = (L(dev(c.f) + e * v) - L(dev(c.f) - e * v)) / (2 * e)
    fd64 = (L64(c.f + e * vn) - L64(c.f - e * vn)) / (2 * e)
    print(f"[grad] GPU FD {fd:.6e}  oracle FD {fd64:.6e}  GPU adjoint {gv:.6e}", flush=True)
    assert abs(fd - fd64) <= 2e-3 * abs(fd64)
    assert abs(fd - gv) <= 2e-2 * abs(gv)


def test_backward_perona_malik():
    """The non-convex Perona-Malik regulariser (lambda = 20 grey levels) in the
    backward pass: derivative of the diffusivity g = lambda^2/(lambda^2 + z)."""
    H, W = 48, 64
    rng = np.random.default_rng(99)
    g = synth.ground_truth(rng, H, W)
    h = synth.line_psf(9, 1.2).astype(np.float32)
    f = synth.observe(rng, g, h.astype(np.float64), 2.0)
    K, alpha, iters = 0.01, 0.02, 3
    p = oracle.Params(alpha=alpha, eps_tv=20.0, psi=1)
    (df, dh, da, lam0), floor = oracle_floor(f, h, g.astype(np.float32), K, p, iters, True)
    gp = dbl.Params(alpha=alpha, iters=iters, eps_tv=20.0, psi=dbl.PSI_PERONA_MALIK)
    got = gpu_grads(f, dbl.Psf.from_taps(dev(h)), g.astype(np.float32), K, gp, True)
    check("perona_malik", got, df, dh, da, lam0, floor)


def test_backward_fractional_box():
    """A vertical box of non-integer length (fractional end pixels): dL/dh for
    every entry of its array, including the two end taps."""
    rng = np.random.default_rng(17)
    H, W = 72, 48
    g = synth.ground_truth(rng, H, W)
    h = synth.box_psf(8.5, "v").astype(np.float32)
    f = synth.observe(rng, g, h.astype(np.float64), 2.0)
    p = oracle.Params(alpha=0.003)
    (df, dh, da, lam0), floor = oracle_floor(f, h, g.astype(np.float32), 0.01, p, 3, True)
    got = gpu_grads(f, dbl.Psf.box(8.5, "v"), g.astype(np.float32), 0.01, dbl.Params(alpha=0.003, iters=3), True)
    assert got["taps"].shape == h.shape
    check("box8.5v", got, df, dh, da, lam0, floor)


def test_autograd_batch_per_image_alpha():
    """WR3LFunction on a batch [B, H, W] with one alpha and one PSF per image:
    every image's output and gradients equal those of its single-image call
    bit for bit; a PSF shared by the batch gets the sum of the images' dL/dh,
    a scalar alpha the sum of their dL/dalpha."""
    B = 6          # more images than side streams: two images share a stream
    cases = [synth.make_case(4, image=i, size=96) for i in range(B)]
    g = torch.stack([dev(c.g) for c in cases]).double()
    alpha = torch.tensor([0.002, 0.004, 0.001, 0.003, 0.0015, 0.0025], dtype=torch.float32)
    f = torch.stack([dev(c.f) for c in cases]).requires_grad_(True)
    taps = torch.stack([dev(c.psf) for c in cases]).requires_grad_(True)
    a = alpha.clone().requires_grad_(True)
    u = dbl.wr3l_autograd(f, taps, a, 0.01, 4)
    ((u.double() - g) ** 2).sum().backward()
    for i in range(B):
        fi = dev(cases[i].f).requires_grad_(True)
        ti = dev(cases[i].psf).requires_grad_(True)
        ai = alpha[i].clone().requires_grad_(True)
        ui = dbl.wr3l_autograd(fi, ti, ai, 0.01, 4)
        ((ui.double() - g[i]) ** 2).sum().backward()
        assert torch.equal(ui, u[i])
        assert torch.equal(fi.grad, f.grad[i]) and torch.equal(ti.grad, taps.grad[i])
        assert torch.equal(ai.grad, a.grad[i])
    # one PSF and one alpha for the whole batch
    ts = dev(cases[0].psf).requires_grad_(True)
    a1 = torch.tensor(0.002, requires_grad=True)
    f2 = torch.stack([dev(c.f) for c in cases]).requires_grad_(True)
    u2 = dbl.wr3l_autograd(f2, ts, a1, 0.01, 4)
    ((u2.double() - g) ** 2).sum().backward()
    per = []
    for i in range(B):
        ti = dev(cases[0].psf).requires_grad_(True)
        ai = torch.tensor(0.002, requires_grad=True)
        ((dbl.wr3l_autograd(dev(cases[i].f), ti, ai, 0.01, 4).double() - g[i]) ** 2).sum().backward()
        per.append((ti.grad, ai.grad))
    assert torch.equal(ts.grad, torch.stack([p[0] for p in per]).sum(0))
    assert torch.allclose(a1.grad, torch.stack([p[1] for p in per]).sum(), rtol=1e-6, atol=0)


def test_autograd_template_carries_over():
    """Every field of the parameter template reaches the forward and the
    backward (here the Perona-Malik regulariser and a periodic border); the
    lookup mode of r_f, which the backward does not differentiate, is refused."""
    c = synth.make_case(4, size=96)
    tmpl = dbl.Params(eps_tv=20.0, psi=dbl.PSI_PERONA_MALIK, boundary=dbl.BC_PERIODIC)
    f = dev(c.f).requires_grad_(True)
    taps = dev(c.psf).requires_grad_(True)
    alpha = torch.tensor(0.01, requires_grad=True)
    u = dbl.wr3l_autograd(f, taps, alpha, 0.01, 3, template=tmpl, pos_floor=2.0)
    lam = 2.0 * (u.detach() - dev(c.g))
    (u * lam).sum().backward()
    # the same through the entry points, with the template's fields
    p = dbl.Params(alpha=0.01, iters=3, eps_tv=20.0, psi=dbl.PSI_PERONA_MALIK, boundary=dbl.BC_PERIODIC)
    psf = dbl.Psf.from_taps(dev(c.psf))
    fd = dev(c.f)
    u0 = torch.empty_like(fd)
    dbl.deblur_wiener(fd, u0, psf, 0.01, 2.0, fp64=True)
    ck = torch.empty((3,) + fd.shape, device="cuda")
    dbl.deblur_rrrl_iterate(fd, u0, u0, psf, p, ckpt=ck)
    assert torch.equal(u0, u.detach())
    gd = dbl.deblur_rrrl_backward(fd, ck, lam.contiguous(), psf, p, through_wiener=True, K=0.01, pos_floor=2.0)
    assert torch.equal(gd["f"], f.grad) and torch.equal(gd["taps"], taps.grad)
    with pytest.raises(ValueError, match="rf_lut"):
        dbl.wr3l_autograd(f, taps, alpha, 0.01, 3, template=dbl.Params(rf_lut=True))


@pytest.mark.parametrize("which", ["alpha", "tap"])
def test_gpu_finite_difference_in_parameters(which):
    """Central differences of the GPU forward's loss (step 1e-3 relative to
    the parameter: alpha, or the largest PSF entry, taken off and put back so
    the PSF stays normalised only to first order; the loss is defined for any
    tap values) against the GPU adjoint."""
    c = synth.make_case(4, size=128)
    g = dev(c.g).double()
    f = dev(c.f)
    h0 = c.psf.astype(np.float32)
    j = np.unravel_index(np.argmax(h0), h0.shape)

    def loss(alpha, h):
        with torch.no_grad():
            u = dbl.wr3l_autograd(f, dev(h), torch.tensor(alpha), c.K, 5)
            return float(((u.double() - g) ** 2).sum())

    taps = dev(h0).requires_grad_(True)
    a = torch.tensor(c.alpha, requires_grad=True)
    u = dbl.wr3l_autograd(f, taps, a, c.K, 5)
    ((u.double() - g) ** 2).sum().backward()
    if which == "alpha":
        e = 1e-3 * c.alpha
        fd = (loss(c.alpha + e, h0) - loss(c.alpha - e, h0)) / (2 * e)
        adj = float(a.grad)
    else:
        e = 1e-3 * float(h0[j])
        hp, hm = h0.copy(), h0.copy()
        hp[j] += e
        hm[j] -= e
        fd = (loss(c.alpha, hp) - loss(c.alpha, hm)) / (2 * e)
        adj = float(taps.grad[j])
    print(f"[grad] FD {which}: {fd:.6e}  adjoint {adj:.6e}  rel {abs(fd - adj) / abs(adj):.2e}", flush=True)
    assert abs(fd - adj) <= 2e-2 * abs(adj)


@pytest.mark.parametrize("bc", [oracle.BC_REPLICATE, oracle.BC_PERIODIC], ids=["replicate", "periodic"])
def test_backward_tile_rows_bitwise(bc):
    """Every tile-row shape of the backward kernels gives the same gradients
    bit for bit: a 36 x 72 image (partial tiles both ways; the gradient stops
    at u^0) and a 48 x 96 one through the Wiener step with a long line PSF
    (radius class 16)."""
    rng = np.random.default_rng(7)
    n = dbl._lib.load().deblur_backward_tile_variants()
    assert n == 4
    for H, W, h, tw in ((36, 72, synth.random_psf(rng, 5, 7), False), (48, 96, synth.line_psf(21, 0.4), True)):
        f = rng.uniform(0.0, 255.0, (H, W))
        g = rng.uniform(0.0, 255.0, (H, W))
        psf = dbl.Psf.from_taps(dev(h))
        ref = None
        for v in range(n + 1):
            gp = dbl.Params(alpha=0.01, iters=3, boundary=bc, bwd_tile=v)
            got = gpu_grads(f, psf, g, 0.01, gp, tw)
            if ref is None:
                ref = got
            else:
                for k in ref:
                    assert np.array_equal(got[k], ref[k]), (H, W, v, k)


def test_autotune_backward_family(tmp_path, monkeypatch):
    from paper_1212_2245_amd import autotune
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tiles.json"))
    c = synth.make_case(4, image=0)
    psf = dbl.Psf.from_taps(dev(c.psf))
    res = autotune.tune_backward(dev(c.f), psf, dbl.Params(alpha=c.alpha, iters=2), reps=1)
    n = dbl._lib.load().deblur_backward_tile_variants()
    assert 0 <= res["tile"] <= n and len(res["timings_us"]) == n + 1
    assert autotune.best_backward_tile(512, 512, 31, 31) == res["tile"]
    print(f"[tune] {res['key']}: {res['timings_us']}", flush=True)
