"""Pins of the oracle's hand-written adjoint (backward through Wiener + the
unrolled RRRL iterations): central finite differences of the oracle's own
forward, and an independent forward written with torch FP64 CPU operations
(pad + conv2d for the blurs, slicing for the diffusion term, torch.fft for
the Wiener filter) differentiated by autograd."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
import synth


@pytest.fixture(autouse=True)
def _float64_default():
    """FP64 as torch's default dtype for this module's tests only."""
    prev = torch.get_default_dtype()
    torch.set_default_dtype(torch.float64)
    yield
    torch.set_default_dtype(prev)


def rng(i):
    return np.random.default_rng(3000 + i)


# ---------------------------------------------------- independent forward
def t_blur(v, h, bc, adjoint=False):
    """A (or B if adjoint) with constant / periodic continuation, torch ops."""
    Py, Px = h.shape
    cy, cx = (Py - 1) // 2, (Px - 1) // 2
    mode = "replicate" if bc == oracle.BC_REPLICATE else "circular"
    vp = F.pad(v[None, None], (cx, cx, cy, cy), mode=mode)
    # conv2d is a correlation: B uses h as is, A uses h flipped
    k = h if adjoint else torch.flip(h, (0, 1))
    return F.conv2d(vp, k[None, None])[0, 0]


def t_tv(u, eps, psi=0):
    up = F.pad(u[None, None], (1, 1, 1, 1), mode="replicate")[0, 0]
    gx = 0.5 * (up[1:-1, 2:] - up[1:-1, :-2])
    gy = 0.5 * (up[2:, 1:-1] - up[:-2, 1:-1])
    z = gx * gx + gy * gy
    # regularised TV, or the non-convex Perona-Malik penaliser (lambda = eps)
    g = eps * eps / (eps * eps + z) if psi else 1.0 / torch.sqrt(z + eps * eps)
    D = torch.zeros_like(u)
    # vertical fluxes between rows y and y+1, horizontal between x and x+1
    fy = 0.5 * (g[:-1] + g[1:]) * (u[1:] - u[:-1])
    fx = 0.5 * (g[:, :-1] + g[:, 1:]) * (u[:, 1:] - u[:, :-1])
    D = D + F.pad(fy, (0, 0, 0, 1)) - F.pad(fy, (0, 0, 1, 0))
    D = D + F.pad(fx, (0, 1, 0, 0)) - F.pad(fx, (1, 0, 0, 0))
    return D


def t_step(f, u, h, alpha, p: oracle.Params):
    s = torch.clamp(t_blur(u, h, p.bc), min=p.s_min)
    fpos = f > 0
    fs = torch.where(fpos, f, torch.ones_like(f))
    r = torch.where(fpos, s - f - fs * torch.log(s / fs), s)
    if p.robust:
        W = 1.0 / torch.sqrt(torch.clamp(r, min=0.0) + p.eps_data ** 2)
    else:
        W = torch.ones_like(s)
    # max(f, 0) with the derivative taken as 0 at f = 0 (the branch f <= 0)
    q = W * torch.where(fpos, f, torch.zeros_like(f)) / s
    N1 = t_blur(q, h, p.bc, adjoint=True)
    N2 = t_blur(W, h, p.bc, adjoint=True)
    D = t_tv(u, p.eps_tv, p.psi)
    return u * (N1 + alpha * torch.clamp(D, min=0.0)) / (N2 - alpha * torch.clamp(D, max=0.0))


def t_wiener_init(f, h, K, floor):
    H, W = f.shape
    Py, Px = h.shape
    cy, cx = (Py - 1) // 2, (Px - 1) // 2
    pad = torch.zeros((H, W))
    ys = [(j - cy) % H for j in range(Py)]
    xs = [(i - cx) % W for i in range(Px)]
    pad = pad.index_put((torch.tensor(ys)[:, None].expand(Py, Px).reshape(-1),
                         torch.tensor(xs)[None, :].expand(Py, Px).reshape(-1)), h.reshape(-1), accumulate=True)
    hh = torch.fft.fft2(pad)
    M = torch.conj(hh) / (hh.abs() ** 2 + K)
    u_pre = torch.real(torch.fft.ifft2(torch.fft.fft2(f) * M))
    return torch.clamp(u_pre, min=floor)


# ----------------------------------------------------------------- tests
CASES = [(oracle.BC_REPLICATE, True, 0), (oracle.BC_PERIODIC, True, 0), (oracle.BC_REPLICATE, False, 0),
         (oracle.BC_REPLICATE, True, 1)]


def case_params(alpha, robust, bc, psi):
    # Perona-Malik with lambda = 20 grey levels: both diffusion regimes occur
    return oracle.Params(alpha=alpha, robust=robust, bc=bc, psi=psi, eps_tv=20.0 if psi else 0.1)


@pytest.mark.parametrize("bc,robust,psi", CASES)
def test_step_adjoint_matches_torch_autograd(bc, robust, psi):
    r = rng(bc * 2 + robust + 5 * psi)
    H, W = 11, 13
    h = synth.random_psf(r, 5, 3, density=0.7)
    f = r.uniform(0, 255, (H, W))
    f[2, 3:6] = 0.0
    u = r.uniform(3, 255, (H, W))
    lam = r.normal(size=(H, W))
    p = case_params(0.07, robust, bc, psi)
    du, df, dh, da = oracle.rrrl_step_adjoint(f, u, h, p, lam)

    tf, tu, th = (torch.tensor(x, requires_grad=True) for x in (f, u, h))
    ta = torch.tensor(0.07, requires_grad=True)
    out = t_step(tf, tu, th, ta, p)
    np.testing.assert_allclose(out.detach().numpy(), oracle.rrrl_step(f, u, h, p), rtol=1e-12)
    (out * torch.tensor(lam)).sum().backward()
    np.testing.assert_allclose(du, tu.grad.numpy(), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(df, tf.grad.numpy(), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(dh, th.grad.numpy(), rtol=1e-9, atol=1e-9)
    assert abs(da - ta.grad.item()) <= 1e-9 * abs(da) + 1e-12


@pytest.mark.parametrize("bc,robust,psi", CASES)
def test_step_adjoint_finite_differences(bc, robust, psi):
    """Central differences of the oracle forward along random directions, for
    u, f (directions on pixels with f >= 1), every tap (zero or not) and alpha."""
    r = rng(10 + bc * 2 + robust + 5 * psi)
    H, W = 10, 12
    h = synth.line_psf(5, 0.6)
    f = r.uniform(0, 255, (H, W))
    f[0, :4] = 0.0
    u = r.uniform(3, 255, (H, W))
    lam = r.normal(size=(H, W))
    p = case_params(0.05, robust, bc, psi)
    du, df, dh, da = oracle.rrrl_step_adjoint(f, u, h, p, lam)

    def L(ff=f, uu=u, hh=h, a=0.05):
        q = case_params(a, robust, bc, psi)
        return float((oracle.rrrl_step(ff, uu, hh, q) * lam).sum())

    e = 1e-6
    v = r.normal(size=(H, W))
    fd = (L(uu=u + e * v) - L(uu=u - e * v)) / (2 * e)
    assert abs(fd - (du * v).sum()) <= 1e-6 * abs(fd) + 1e-6
    v = r.normal(size=(H, W)) * (f >= 1)
    fd = (L(ff=f + e * v) - L(ff=f - e * v)) / (2 * e)
    assert abs(fd - (df * v).sum()) <= 1e-6 * abs(fd) + 1e-6
    for j in range(h.shape[0]):
        for i in range(h.shape[1]):
            d = np.zeros_like(h)
            d[j, i] = 1.0
            fd = (L(hh=h + e * d) - L(hh=h - e * d)) / (2 * e)
            assert abs(fd - dh[j, i]) <= 1e-5 * abs(fd) + 1e-4, (j, i)
    fd = (L(a=0.05 + e) - L(a=0.05 - e)) / (2 * e)
    assert abs(fd - da) <= 1e-6 * abs(fd) + 1e-6


def test_wiener_adjoint_matches_torch_autograd():
    r = rng(20)
    H, W = 12, 18
    h = synth.random_psf(r, 3, 5)
    f = r.uniform(0, 255, (H, W))
    lam0 = r.normal(size=(H, W))
    K, floor = 0.02, 40.0
    df, dh = oracle.wiener_adjoint(f, h, K, floor, lam0)
    tf, th = torch.tensor(f, requires_grad=True), torch.tensor(h, requires_grad=True)
    u0 = t_wiener_init(tf, th, K, floor)
    np.testing.assert_allclose(u0.detach().numpy(), oracle.wiener_init(f, h, K, floor), rtol=1e-12, atol=1e-9)
    (u0 * torch.tensor(lam0)).sum().backward()
    np.testing.assert_allclose(df, tf.grad.numpy(), rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(dh, th.grad.numpy(), rtol=1e-9, atol=1e-8)


def test_wr3l_gradient_finite_differences():
    """Whole WR3L (Wiener + 3 iterations), L = sum (u^K - g)^2: taps with
    h(d) > 2e-3, alpha, and f along a random direction supported on pixels
    with f >= 1 (central differences; the step is small enough that the
    O(step^2) truncation stays below the tolerance)."""
    c = synth.make_case(4, size=48)
    h = c.psf.astype(np.float64)
    f = c.f.astype(np.float64)
    g = c.g.astype(np.float64)
    p = oracle.Params(alpha=c.alpha)
    iters = 3
    loss, df, dh, da = oracle.wr3l_loss_and_grad(f, h, c.K, p, iters, g)

    def L(ff=f, hh=h, a=c.alpha):
        u = oracle.wr3l(ff, hh, c.K, oracle.Params(alpha=a), iters)
        return float(((u - g) ** 2).sum())

    assert abs(L() - loss) <= 1e-9 * loss
    e = 1e-4
    r = rng(30)
    v = r.normal(size=f.shape) * (f >= 1)
    fd = (L(ff=f + e * v) - L(ff=f - e * v)) / (2 * e)
    assert abs(fd - (df * v).sum()) <= 1e-4 * abs(fd) + 1e-6
    for (j, i) in list(zip(*np.nonzero(h > 2e-3)))[:6]:
        d = np.zeros_like(h)
        d[j, i] = 1.0
        fd = (L(hh=h + 1e-5 * d) - L(hh=h - 1e-5 * d)) / 2e-5
        assert abs(fd - dh[j, i]) <= 1e-4 * abs(fd) + 1e-3, (j, i)
    fd = (L(a=c.alpha + 1e-5) - L(a=c.alpha - 1e-5)) / 2e-5
    assert abs(fd - da) <= 1e-4 * abs(fd) + 1e-6
