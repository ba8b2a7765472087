"""GPU backward (hand-written adjoint through the unrolled RRRL iterations
and the Wiener initialisation) against the FP64 oracle adjoint: relative
error <= 1e-3 for dL/df, dL/dh (every PSF entry) and dL/dalpha, loss
L = sum (u^K - g)^2.  Each side runs its own forward."""
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
    dbl.deblur_wiener(fd, u, psf, K, 1.0)
    ck = torch.empty((max(gp.iters, 1), H, pitch), dtype=torch.float32, device="cuda")
    dbl.deblur_rrrl_iterate(fd, u, u, psf, gp, ckpt=ck)
    lam = (2.0 * (u - dev(g))).contiguous() if pitch == W else None
    if lam is None:
        lam = torch.empty_strided((H, W), (pitch, 1), dtype=torch.float32, device="cuda")
        lam.copy_(2.0 * (u - dev(g)))
    out = dbl.deblur_rrrl_backward(fd, ck, lam, psf, gp, through_wiener=through_wiener, K=K, grad_u0=True)
    return {k: v.cpu().numpy() for k, v in out.items()}


def check(name, got, df, dh, da, lam0):
    e_f, e_h, e_a = rel(got["f"], df), rel(got["taps"], dh), abs(float(got["alpha"]) - da) / max(abs(da), 1e-300)
    e_u = rel(got["u0"], lam0)
    print(f"[grad] {name}: f {e_f:.2e}  h {e_h:.2e}  alpha {e_a:.2e}  u0 {e_u:.2e}", flush=True)
    assert e_f <= RTOL_GRAD and e_h <= RTOL_GRAD and e_a <= RTOL_GRAD and e_u <= RTOL_GRAD


CASES = [
    ("line9_rep_robust", 48, 64, lambda: synth.line_psf(9, 0.7), oracle.BC_REPLICATE, True, 3, True),
    ("asym5x7_rep", 36, 48, lambda: synth.random_psf(np.random.default_rng(1), 5, 7), oracle.BC_REPLICATE, True, 2,
     True),
    ("asym5x7_periodic", 36, 48, lambda: synth.random_psf(np.random.default_rng(2), 5, 7), oracle.BC_PERIODIC, True,
     2, True),
    ("line13_nonrobust", 48, 48, lambda: synth.line_psf(13, 2.2), oracle.BC_REPLICATE, False, 3, True),
    ("no_wiener", 40, 56, lambda: synth.line_psf(7, 1.0), oracle.BC_REPLICATE, True, 4, False),
    ("iters0", 32, 32, lambda: synth.random_psf(np.random.default_rng(3), 3, 3), oracle.BC_REPLICATE, True, 0, True),
    ("gauss31_64", 64, 64, lambda: synth.gauss_mixture_psf(synth.rng_for(2), 31), oracle.BC_REPLICATE, True, 2, True),
]


@pytest.mark.parametrize("name,H,W,mk,bc,robust,iters,tw", CASES, ids=[c[0] for c in CASES])
def test_backward_vs_oracle_adjoint(name, H, W, mk, bc, robust, iters, tw):
    rng = np.random.default_rng(H + W)
    g = synth.ground_truth(rng, H, W)
    h = mk().astype(np.float32)
    f = synth.observe(rng, g, h.astype(np.float64), 2.0)
    K, alpha = 0.01, 0.01
    p = oracle.Params(alpha=alpha, robust=robust, bc=bc)
    df, dh, da, lam0 = oracle_grads(f, h, g.astype(np.float32), K, p, iters, tw)
    gp = dbl.Params(alpha=alpha, iters=iters, robust=robust, boundary=bc)
    got = gpu_grads(f, dbl.Psf.from_taps(dev(h)), g.astype(np.float32), K, gp, tw)
    check(name, got, df, dh, da, lam0)


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


def test_backward_workload_shape():
    """The differentiation workload's per-image shape: 512^2, oblique line
    L=31, Wiener + 10 iterations, alpha = 0.002."""
    c = synth.make_case(4)
    p = oracle.Params(alpha=c.alpha)
    df, dh, da, lam0 = oracle_grads(c.f, c.psf, c.g, c.K, p, c.iters, True)
    got = gpu_grads(c.f, dbl.Psf.from_taps(dev(c.psf)), c.g, c.K, dbl.Params(alpha=c.alpha, iters=c.iters), True)
    check("workload 512 line31 k10", got, df, dh, da, lam0)


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
    """Central difference (step 1e-3) of the GPU forward's loss along a random
    direction in f, against the GPU gradient (FP32 forward: 1e-2)."""
    c = synth.make_case(4, size=128)
    taps = dev(c.psf)
    alpha = torch.tensor(c.alpha)
    rng = np.random.default_rng(9)
    v = dev(rng.normal(size=c.f.shape) * (c.f >= 1))
    f = dev(c.f).requires_grad_(True)
    u = dbl.wr3l_autograd(f, taps, alpha, c.K, 5)
    loss = ((u.double() - dev(c.g).double()) ** 2).sum()
    loss.backward()
    gv = float((f.grad.double() * v.double()).sum())

    def L(ff):
        with torch.no_grad():
            uu = dbl.wr3l_autograd(ff, taps, alpha, c.K, 5)
            return float(((uu.double() - dev(c.g).double()) ** 2).sum())

    e = 1e-3
    fd = (L(dev(c.f) + e * v) - L(dev(c.f) - e * v)) / (2 * e)
    print(f"[grad] GPU FD {fd:.6e} vs adjoint {gv:.6e}", flush=True)
    assert abs(fd - gv) <= 1e-2 * abs(gv)
