"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: a library
routine for a special case, a closed form, an invariant of the iteration, a
hand-worked value, or brute force.  Chosen so that a dropped term, a wrong
sign or index, or swapped operands in the oracle fails at least one.
"""
import math
import os

import numpy as np
import pytest
from scipy import ndimage, special

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
BCS = [(oracle.BC_REPLICATE, "nearest"), (oracle.BC_PERIODIC, "wrap")]


def rng(i=0):
    return np.random.default_rng(1000 + i)


# ------------------------------------------------------------------ A and B
@pytest.mark.parametrize("bc,mode", BCS)
@pytest.mark.parametrize("shape,pshape", [((12, 10), (5, 3)), ((7, 16), (3, 7)),
                                          ((9, 9), (9, 9)), ((16, 5), (1, 5)),
                                          ((6, 11), (5, 1))])
def test_blur_corr_match_scipy(bc, mode, shape, pshape):
    """A = convolution, B = correlation with the centred PSF (eq. (1), h*),
    constant or periodic continuation: scipy.ndimage with mode nearest/wrap."""
    r = rng(shape[0] * 31 + pshape[1])
    v = r.uniform(0, 255, size=shape)
    h = synth.random_psf(r, *pshape)  # asymmetric
    np.testing.assert_allclose(oracle.blur(v, h, bc), ndimage.convolve(v, h, mode=mode),
                               rtol=1e-13, atol=1e-10)
    np.testing.assert_allclose(oracle.corr(v, h, bc), ndimage.correlate(v, h, mode=mode),
                               rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("L", [1, 2, 3, 4, 7, 8, 15, 16, 27])
@pytest.mark.parametrize("axis", ["h", "v"])
def test_box_blur_is_window_mean(L, axis):
    """Uniform motion blur of integer length L: the mean over L consecutive
    pixels, window [x - floor(L/2), x + floor((L-1)/2)] (brute force)."""
    r = rng(L)
    v = r.uniform(0, 255, size=(9, 33) if axis == "h" else (33, 9))
    h = synth.box_psf(L, axis)
    got = oracle.blur(v, h, oracle.BC_REPLICATE)
    vv = v if axis == "h" else v.T
    want = np.empty_like(vv)
    n = vv.shape[1]
    for x in range(n):
        idx = [min(max(j, 0), n - 1) for j in range(x - L // 2, x + (L - 1) // 2 + 1)]
        want[:, x] = vv[:, idx].mean(axis=1)
    want = want if axis == "h" else want.T
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-11)


@pytest.mark.parametrize("L", [1.5, 2.25, 4.5, 7.75, 14.5, 15.25, 40.9])
@pytest.mark.parametrize("axis", ["h", "v"])
def test_fractional_box_blur(L, axis):
    """Uniform motion of non-integer length L = n + frac (Sec. 4.3): the
    integer window of n pixels with weight 1/L plus one pixel of weight
    (frac/2)/L at each end (brute force); and successive window values differ
    by two additions and two subtractions, as the paper states for its box
    filter update."""
    r = rng(int(L * 8))
    v = r.uniform(0, 255, size=(7, 80) if axis == "h" else (80, 7))
    h = synth.box_psf(L, axis)
    got = oracle.blur(v, h, oracle.BC_REPLICATE)
    vv = v if axis == "h" else v.T
    gg = got if axis == "h" else got.T
    n, frac = int(math.floor(L)), L - math.floor(L)
    e = 0.5 * frac
    N = vv.shape[1]
    cl = lambda j: min(max(j, 0), N - 1)  # noqa: E731
    for x in range(N):
        inner = sum(vv[:, cl(j)] for j in range(x - n // 2, x + (n - 1) // 2 + 1))
        ends = vv[:, cl(x - n // 2 - 1)] + vv[:, cl(x + (n - 1) // 2 + 1)]
        np.testing.assert_allclose(gg[:, x], (inner + e * ends) / L, rtol=1e-13, atol=1e-11)
    lo, hi = n // 2 + 2, N - (n - 1) // 2 - 3   # interior: no clamping
    for x in range(lo, hi):
        upd = ((1 - e) * vv[:, x + 1 + (n - 1) // 2] + e * vv[:, x + 2 + (n - 1) // 2]
               - (1 - e) * vv[:, x - n // 2] - e * vv[:, x - n // 2 - 1]) / L
        np.testing.assert_allclose(gg[:, x + 1] - gg[:, x], upd, rtol=1e-9, atol=1e-9)


def test_fractional_box_limits():
    """frac -> 0 gives the integer box (continuity in L); weights sum to one."""
    for n in (1, 2, 5, 16, 31):
        a = synth.box_psf(n + 1e-12, "h")[0]
        b = np.pad(synth.box_psf(n, "h")[0], 1)
        np.testing.assert_allclose(a, b, atol=1e-12)
        for frac in (0.1, 0.5, 0.9):
            h = synth.box_psf(n + frac, "v")
            assert h.shape == (n + (1 - n % 2) + 2, 1)
            assert abs(h.sum() - 1.0) < 1e-14


def test_blur_preserves_mass_periodic():
    """Normalised PSF: periodic blur preserves total mass (sum_d h(d) = 1)."""
    r = rng(5)
    v = r.uniform(0, 255, size=(20, 24))
    h = synth.random_psf(r, 7, 5)
    assert abs(oracle.blur(v, h, oracle.BC_PERIODIC).sum() - v.sum()) < 1e-9 * v.sum()
    assert abs(oracle.corr(v, h, oracle.BC_PERIODIC).sum() - v.sum()) < 1e-9 * v.sum()


def test_corr_is_transpose_of_blur_periodic():
    """<A v, w> = <v, B w> under periodic continuation (h* is the adjoint)."""
    r = rng(6)
    v, w = r.normal(size=(11, 13)), r.normal(size=(11, 13))
    h = synth.random_psf(r, 5, 7)
    lhs = (oracle.blur(v, h, oracle.BC_PERIODIC) * w).sum()
    rhs = (v * oracle.corr(w, h, oracle.BC_PERIODIC)).sum()
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


# ---------------------------------------------------------------------- r_f
def test_rf_is_kl_divergence():
    """r_f(s) = s - f - f ln(s/f) equals scipy.special.kl_div(f, s), including
    the f = 0 limit r_0(s) = s."""
    r = rng(7)
    for f, s in zip(np.r_[0.0, r.uniform(0, 255, 200)], np.r_[3.0, r.uniform(1e-3, 300, 200)]):
        assert math.isclose(oracle.rf(f, s), float(special.kl_div(f, s)), rel_tol=1e-12,
                            abs_tol=1e-10)


def test_rf_closed_forms():
    rows = np.loadtxt(os.path.join(GOLD, "rf_closed_forms.txt"))
    for f, s, want in rows:
        assert math.isclose(oracle.rf(f, s), want, rel_tol=1e-13, abs_tol=1e-14)
    # non-negative, zero only at s = f, homogeneous of degree 1
    for f, s, c in [(3.0, 7.0, 2.5), (100.0, 40.0, 0.1), (0.5, 0.51, 8.0)]:
        assert oracle.rf(f, s) > 0.0
        assert math.isclose(oracle.rf(c * f, c * s), c * oracle.rf(f, s), rel_tol=1e-12)
    # quadratic near s = f: r_f(f + e) ~ e^2 / (2 f)
    f, e = 80.0, 1e-3
    assert math.isclose(oracle.rf(f, f + e), e * e / (2 * f), rel_tol=1e-4)


def test_rf_lookup_mode():
    """The lookup mode of Sec. 4.1 against the exact r_f: equal at the table
    samples s = f k/64; between samples above it by at most the linear
    interpolation bound f h^2/8 max r_1'' (h = 1/64, r_1''(x) = 1/x^2, convex);
    beyond x = 65 the tangent, below r_f by at most f (x-65)^2 / (2 65^2);
    r_0(s) = s."""
    r = rng(17)
    for f in (0.5, 7.0, 100.0, 240.0):
        for k in (1, 2, 63, 64, 65, 100, 1000, 4159, 4160):
            s = f * k / 64.0
            assert math.isclose(oracle.rf_lut(f, s), oracle.rf(f, s), rel_tol=1e-12, abs_tol=1e-12 * f)
        for x in r.uniform(1.0 / 64.0, 65.0, 300):
            lo = math.floor(x * 64.0) / 64.0
            bound = f * (1.0 / 64.0) ** 2 / 8.0 / lo ** 2
            d = oracle.rf_lut(f, f * x) - oracle.rf(f, f * x)
            assert -1e-12 * f <= d <= bound * (1 + 1e-9) + 1e-12 * f, (f, x, d, bound)
        for x in (65.5, 80.0, 200.0):
            d = oracle.rf(f, f * x) - oracle.rf_lut(f, f * x)
            assert -1e-9 * f <= d <= f * (x - 65.0) ** 2 / (2 * 65.0 ** 2) * (1 + 1e-9)
    assert oracle.rf_lut(0.0, 3.5) == 3.5
    assert math.isclose(oracle.rf_lut(10.0, 0.01), 10.0 * (1 / 64 - 1 - math.log(1 / 64)), rel_tol=1e-12)


def test_rrrl_start_images():
    """Starting images of RRRL without the Wiener step: flat = the mean,
    floored; observed = the image, floored."""
    c = np.full((5, 7), 42.5)
    np.testing.assert_array_equal(oracle.rrrl_start(c, 0, 1.0), c)
    H, W = 6, 9
    ramp = np.add.outer(np.arange(H, dtype=np.float64), 10.0 * np.arange(W))
    np.testing.assert_allclose(oracle.rrrl_start(ramp, 0, 1.0), np.full((H, W), (H - 1) / 2 + 10 * (W - 1) / 2))
    np.testing.assert_array_equal(oracle.rrrl_start(np.zeros((3, 3)), 0, 1.5), np.full((3, 3), 1.5))
    f = np.array([[0.0, 0.5, 3.0], [-2.0, 1.0, 7.0]])
    np.testing.assert_array_equal(oracle.rrrl_start(f, 1, 1.0), [[1.0, 1.0, 3.0], [1.0, 1.0, 7.0]])


# ----------------------------------------------------------------------- TV
def test_tv_hand_worked_profile():
    rows = np.loadtxt(os.path.join(GOLD, "tv_profile_1x5.txt"))
    D = oracle.tv(rows[:, 0][None, :], 0.1)
    np.testing.assert_allclose(D[0], rows[:, 1], rtol=1e-14, atol=1e-14)
    # the same profile as a column: the operator is symmetric in x and y
    np.testing.assert_allclose(oracle.tv(rows[:, 0][:, None], 0.1)[:, 0], rows[:, 1],
                               rtol=1e-14, atol=1e-14)


def test_perona_malik_hand_worked_profile():
    """Non-convex Perona-Malik regulariser (lambda = 2) on a hand-worked 1x5
    profile; as a row and as a column."""
    rows = np.loadtxt(os.path.join(GOLD, "tv_perona_malik_1x5.txt"))
    np.testing.assert_allclose(oracle.tv(rows[:, 0][None, :], 2.0, psi=1)[0], rows[:, 1], rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(oracle.tv(rows[:, 0][:, None], 2.0, psi=1)[:, 0], rows[:, 1], rtol=1e-14,
                               atol=1e-14)


def test_perona_malik_limits():
    """lambda -> infinity: diffusivity 1, D = the zero-flux 5-point Laplacian;
    small lambda: edges (|grad u| >> lambda) stop diffusing; fluxes still
    telescope to zero."""
    u = rng(18).uniform(0, 255, size=(13, 17))
    np.testing.assert_allclose(oracle.tv(u, 1e9, psi=1), ndimage.laplace(u, mode="nearest"), rtol=1e-9, atol=1e-7)
    step = np.zeros((6, 12))
    step[:, 6:] = 100.0
    D = oracle.tv(step, 1.0, psi=1)
    # only the two columns at the jump have a flux: (g + g)/2 * 100 with g = 1/(1 + 50^2)
    g = 1.0 / (1.0 + 50.0 ** 2)
    np.testing.assert_allclose(D[:, 5], g * 100.0, rtol=1e-12)
    np.testing.assert_allclose(D[:, 6], -g * 100.0, rtol=1e-12)
    assert np.all(D[:, :5] == 0.0) and np.all(D[:, 7:] == 0.0)
    assert abs(oracle.tv(u, 30.0, psi=1).sum()) < 1e-9 * np.abs(u).sum()


def test_tv_constant_diffusivity_is_neumann_laplacian():
    """With Psi' constant (eps_tv huge), eps_tv * D is the 5-point Laplacian
    with reflecting (zero-flux) boundary: scipy.ndimage.laplace, mode nearest."""
    u = rng(8).uniform(0, 255, size=(13, 17))
    eps = 1e9
    np.testing.assert_allclose(eps * oracle.tv(u, eps), ndimage.laplace(u, mode="nearest"),
                               rtol=1e-9, atol=1e-7)


def test_tv_invariants():
    r = rng(9)
    u = r.uniform(0, 255, size=(15, 12))
    D = oracle.tv(u, 0.3)
    assert abs(D.sum()) < 1e-9 * np.abs(D).sum()           # zero flux: telescoping
    assert np.all(oracle.tv(np.full((6, 7), 42.0), 0.1) == 0.0)
    # a linear ramp has zero divergence away from the border
    y, x = np.mgrid[0:12, 0:14].astype(float)
    ramp = 3.0 * x - 2.0 * y + 5.0
    assert np.abs(oracle.tv(ramp, 0.1)[2:-2, 2:-2]).max() < 1e-12
    # transpose symmetry
    np.testing.assert_allclose(oracle.tv(u.T, 0.3), D.T, rtol=1e-13, atol=1e-12)


# --------------------------------------------------------------------- RRRL
def P(**kw):
    return oracle.Params(**kw)


def test_rrrl_reduces_to_textbook_rl():
    """robust = 0, alpha = 0: u' = u * ((f / (u*h)) * h*), the RL method
    (eq. (3) with the adjoint convolution); built from scipy.ndimage."""
    r = rng(10)
    h = synth.random_psf(r, 5, 3)
    u = r.uniform(1, 255, size=(14, 11))
    f = r.uniform(1, 255, size=(14, 11))
    for bc, mode in BCS:
        want = u * ndimage.correlate(f / ndimage.convolve(u, h, mode=mode), h, mode=mode)
        got = oracle.rrrl_step(f, u, h, P(alpha=0.0, robust=False, bc=bc))
        np.testing.assert_allclose(got, want, rtol=1e-12)


def test_rl_flux_preservation_periodic():
    """Unregularised, non-robust RRRL = RL preserves total flux: sum u^{k+1} =
    sum f for every k (periodic continuation, normalised PSF)."""
    r = rng(11)
    h = synth.random_psf(r, 7, 5)
    f = r.uniform(0, 255, size=(16, 18))
    u = r.uniform(1, 255, size=(16, 18))
    p = P(alpha=0.0, robust=False, bc=oracle.BC_PERIODIC)
    for _ in range(4):
        u = oracle.rrrl_step(f, u, h, p)
        assert abs(u.sum() - f.sum()) < 1e-10 * f.sum()


def test_data_term_is_negative_energy_gradient():
    """N1 - N2 = B(W f/s) - B(W) equals -grad E_data(u) with
    E_data(u) = sum_x 2 sqrt(r_f(u*h) + eps^2)  (eq. (6) with regularised L1
    Phi; W = 2 Phi'), periodic continuation, by central finite differences
    of an energy built from scipy.ndimage.convolve and scipy.special.kl_div."""
    r = rng(12)
    h = synth.random_psf(r, 3, 5)
    f = r.uniform(0, 255, size=(8, 9))
    f[0, :3] = 0.0                    # the f = 0 limit of r_f
    u = r.uniform(5, 255, size=(8, 9))
    eps = 0.7
    p = P(alpha=0.0, robust=True, eps_data=eps, bc=oracle.BC_PERIODIC)

    def energy(v):
        s = ndimage.convolve(v, h, mode="wrap")
        return np.sum(2.0 * np.sqrt(special.kl_div(f, s) + eps * eps))

    u1, parts = oracle.rrrl_step(f, u, h, p, parts=True)
    neg_grad = parts["N1"] - parts["N2"]
    # alpha = 0: u'/u - 1 = (N1 - N2)/N2
    np.testing.assert_allclose((u1 / u - 1.0) * parts["N2"], neg_grad, rtol=1e-9, atol=1e-12)
    for k in range(5):
        v = r.normal(size=u.shape)
        d = 1e-4
        fd = (energy(u + d * v) - energy(u - d * v)) / (2 * d)
        assert math.isclose(-fd, (neg_grad * v).sum(), rel_tol=1e-6, abs_tol=1e-9)


def test_identity_psf_one_step():
    """h = delta, alpha = 0: s = u, q = W f/u, so u' = f after one step
    (robust or not)."""
    r = rng(13)
    f = r.uniform(1, 255, size=(7, 8))
    u = r.uniform(1, 255, size=(7, 8))
    for robust in (False, True):
        np.testing.assert_allclose(oracle.rrrl_step(f, u, np.ones((1, 1)), P(alpha=0.0, robust=robust)),
                                   f, rtol=1e-13)


def test_regulariser_step_direction():
    """h = delta, f = u, W = 1: u' = u (1 + a[D]_+)/(1 - a[D]_-), so
    (u'-u)/(a u) -> D as a -> 0; with Psi' constant D is the Neumann
    Laplacian / eps_tv (scipy.ndimage.laplace)."""
    r = rng(14)
    u = r.uniform(20, 200, size=(9, 10))
    eps = 1e6
    a = 1e-3
    got = oracle.rrrl_step(u, u, np.ones((1, 1)), P(alpha=a, robust=False, eps_tv=eps))
    want = ndimage.laplace(u, mode="nearest") / eps
    np.testing.assert_allclose((got - u) / (a * u), want, rtol=1e-6, atol=1e-12)
    # and for one sign of D the update multiplies, for the other it divides
    D = oracle.tv(u, 0.2)
    a = 0.5
    got = oracle.rrrl_step(u, u, np.ones((1, 1)), P(alpha=a, robust=False, eps_tv=0.2))
    pos = D > 0
    np.testing.assert_allclose(got[pos], u[pos] * (1 + a * D[pos]), rtol=1e-13)
    np.testing.assert_allclose(got[~pos], u[~pos] / (1 - a * D[~pos]), rtol=1e-13)


@pytest.mark.parametrize("bc", [oracle.BC_REPLICATE, oracle.BC_PERIODIC])
@pytest.mark.parametrize("robust", [False, True])
def test_fixed_point_exact_blur(bc, robust):
    """f = u* h exactly, alpha = 0: u* is a fixed point (W is uniform)."""
    r = rng(15)
    h = synth.random_psf(r, 5, 7)
    ustar = r.uniform(10, 250, size=(12, 13))
    f = oracle.blur(ustar, h, bc)
    got = oracle.rrrl(f, ustar, h, P(alpha=0.0, robust=robust, bc=bc), 3)
    np.testing.assert_allclose(got, ustar, rtol=1e-12)


def test_constant_fixed_point_with_regulariser():
    h = synth.random_psf(rng(16), 3, 3)
    c = np.full((10, 11), 77.0)
    got = oracle.rrrl(c, c, h, P(alpha=0.7), 4)
    np.testing.assert_allclose(got, c, rtol=1e-13)


def test_positivity_and_finiteness():
    """The multiplicative RL-style update keeps u > 0 when f > 0; where a
    whole PSF window of f is 0 the quotient vanishes and u becomes exactly 0
    (never negative), and the s_min guard keeps everything finite."""
    r = rng(17)
    h = synth.line_psf(9, 0.7)
    f = r.uniform(0.5, 255, size=(20, 22))
    u = oracle.rrrl(f, np.ones_like(f), h, P(alpha=0.003), 25)
    assert np.all(np.isfinite(u)) and np.all(u > 0)
    f[3:12, 4:15] = 0.0
    u = oracle.rrrl(f, np.ones_like(f), h, P(alpha=0.003), 25)
    assert np.all(np.isfinite(u)) and np.all(u >= 0)
    assert np.all(u[0:2] > 0)


def test_symmetries():
    """Transposing (f, h) transposes u (both continuations); under periodic
    continuation a cyclic shift of f shifts u."""
    r = rng(18)
    h = synth.random_psf(r, 5, 3)
    f = r.uniform(0, 255, size=(12, 15))
    u0 = r.uniform(1, 255, size=(12, 15))
    for bc in (oracle.BC_REPLICATE, oracle.BC_PERIODIC):
        p = P(alpha=0.05, bc=bc)
        a = oracle.rrrl(f, u0, h, p, 3)
        b = oracle.rrrl(f.T, u0.T, h.T, p, 3)
        np.testing.assert_allclose(b, a.T, rtol=1e-12)
    p = P(alpha=0.0, bc=oracle.BC_PERIODIC)
    a = oracle.rrrl(f, u0, h, p, 3)
    b = oracle.rrrl(np.roll(f, (3, -4), (0, 1)), np.roll(u0, (3, -4), (0, 1)), h, p, 3)
    np.testing.assert_allclose(b, np.roll(a, (3, -4), (0, 1)), rtol=1e-12)


def test_resume():
    r = rng(19)
    h = synth.box_psf(6, "v")
    f = r.uniform(0, 255, size=(16, 9))
    u0 = r.uniform(1, 255, size=(16, 9))
    p = P(alpha=0.01)
    full, ck = oracle.rrrl(f, u0, h, p, 5, checkpoints=True)
    half = oracle.rrrl(f, u0, h, p, 2)
    np.testing.assert_array_equal(oracle.rrrl(f, half, h, p, 3), full)
    np.testing.assert_array_equal(ck[0], u0)
    np.testing.assert_array_equal(ck[2], half)


# ------------------------------------------------------------------- Wiener
def test_psf_spectrum_is_dft_definition():
    """h^(k) = sum_d h(d) exp(-2 pi i k.d/N), evaluated term by term."""
    r = rng(20)
    h = synth.random_psf(r, 3, 5)
    H, W = 6, 8
    got = oracle.psf_spectrum(h, H, W)
    want = np.zeros((H, W), complex)
    for ky in range(H):
        for kx in range(W):
            for j in range(3):
                for i in range(5):
                    dy, dx = j - 1, i - 2
                    want[ky, kx] += h[j, i] * np.exp(-2j * np.pi * (ky * dy / H + kx * dx / W))
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14)


def test_wiener_constant_image():
    """Constant image c: only the DC term, h^(0) = 1, so u = c/(1+K)."""
    h = synth.line_psf(15, 0.4)
    for K in (0.01, 0.3):
        u = oracle.wiener(np.full((16, 24), 90.0), h, K)
        np.testing.assert_allclose(u, 90.0 / (1.0 + K), rtol=1e-12)


def test_wiener_cosine_box():
    """Box of odd length L along x, input cos(2 pi k x/N): output M_k cos(...)
    with h^_k = sin(pi k L/N)/(L sin(pi k/N)), M_k = h^_k/(h^_k^2 + K)."""
    N, L, K = 64, 9, 0.02
    x = np.arange(N)
    for k in (1, 5, 7, 20):
        f = np.tile(np.cos(2 * np.pi * k * x / N), (4, 1))
        hk = math.sin(math.pi * k * L / N) / (L * math.sin(math.pi * k / N))
        Mk = hk / (hk * hk + K)
        np.testing.assert_allclose(oracle.wiener(f, synth.box_psf(L, "h"), K), Mk * f,
                                   atol=1e-12)


def test_wiener_2d_equals_rowwise_1d():
    """A PSF supported on one row: the 2D Wiener filter equals a 1D Wiener
    filter applied to every row (Sec. 4.3, non-uniform linear motion)."""
    r = rng(21)
    f = r.uniform(0, 255, size=(10, 32))
    h = synth.random_psf(r, 1, 7)
    K = 0.05
    hk = np.zeros(32)
    for i in range(7):
        hk[(i - 3) % 32] += h[0, i]
    H1 = np.fft.fft(hk)
    want = np.real(np.fft.ifft(np.fft.fft(f, axis=1) * np.conj(H1) / (np.abs(H1) ** 2 + K), axis=1))
    np.testing.assert_allclose(oracle.wiener(f, h, K), want, atol=1e-10)


def test_wiener_inverts_periodic_blur_as_K_vanishes():
    """With |h^| bounded away from 0, Wiener with K -> 0 inverts periodic blur."""
    r = rng(22)
    g = r.uniform(0, 255, size=(12, 16))
    h = np.array([[0.05, 0.1, 0.05], [0.1, 0.4, 0.1], [0.05, 0.1, 0.05]])  # h^ >= 0.04
    f = ndimage.convolve(g, h, mode="wrap")
    np.testing.assert_allclose(oracle.wiener(f, h, 1e-14), g, rtol=1e-8, atol=1e-8)


def test_wiener_init_floor():
    r = rng(23)
    f = r.uniform(0, 255, size=(16, 16))
    f[:, 8] = 0.0
    u = oracle.wiener_init(f, synth.box_psf(5, "h"), 0.001, 1.0)
    assert u.min() >= 1.0
    pre = oracle.wiener(f, synth.box_psf(5, "h"), 0.001)
    np.testing.assert_array_equal(u, np.maximum(pre, 1.0))


# ------------------------------------------------------------ inputs (sanity)
def test_synthetic_psfs():
    for L in (9, 10, 31):
        for th in (0.0, 0.3, math.pi / 4, 1.2, math.pi / 2):
            h = synth.line_psf(L, th)
            assert h.shape[0] == h.shape[1] == 2 * math.ceil((L - 1) / 2) + 1
            assert abs(h.sum() - 1.0) < 1e-14 and h.min() >= 0.0
            np.testing.assert_allclose(h, h[::-1, ::-1], atol=1e-15)  # point-symmetric
    # odd L at 0 degrees is the horizontal box
    np.testing.assert_allclose(synth.line_psf(9, 0.0)[4], synth.box_psf(9, "h")[0], atol=1e-15)
    np.testing.assert_allclose(synth.line_psf(9, math.pi / 2)[:, 4], synth.box_psf(9, "v")[:, 0],
                               atol=1e-12)
    g = synth.gauss_mixture_psf(synth.rng_for(2), 31)
    assert g.shape == (31, 31) and abs(g.sum() - 1) < 1e-13 and g.min() >= 0
