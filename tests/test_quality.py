"""Restoration quality (Sec. 3.1, Table 1): the SNR measure, the synthetic
stand-ins for the paper's degraded test images, and Table 1's trends (not
its numbers: the cameraman image is not available) on the GPU."""
import math

import numpy as np
import pytest

import synth
from paper_1212_2245_amd import quality


def test_snr_closed_forms():
    r = np.random.default_rng(0)
    u0 = r.uniform(0, 255, (40, 50))
    assert math.isclose(quality.snr(2.0 * u0, u0), 10 * math.log10(4.0), rel_tol=1e-12)   # var(2u0)/var(u0)
    ui = r.integers(0, 256, (40, 50)).astype(np.float64)
    assert quality.snr(ui + 7.0, ui) == math.inf                                             # offset: no variance
    n = r.normal(0, 1, u0.shape)
    u = u0 + n
    want = 10 * math.log10(u.var() / n.var())
    assert math.isclose(quality.snr(u, u0), want, rel_tol=1e-12)
    # interior: the border band is left out of both variances
    uc, nc = u[3:-3, 3:-3], n[3:-3, 3:-3]
    assert math.isclose(quality.snr(u, u0, border=3), 10 * math.log10(uc.var() / nc.var()), rel_tol=1e-12)


def test_table1_scenarios():
    sc = synth.table1_scenarios(128, 0)
    assert [s["name"] for s in sc] == ["camera_shake", "motion21_45deg", "shake_gauss5", "shake_impulse15"]
    for s in sc:
        h = s["psf"]
        assert h.shape[0] % 2 == 1 and h.shape[1] % 2 == 1 and abs(h.sum() - 1) < 1e-12 and h.min() >= 0
        assert s["f"].dtype == np.float32 and s["f"].min() >= 0 and s["f"].max() <= 255
    # no noise beyond quantisation in the first two; impulse: about 15 % of pixels replaced
    assert np.all(sc[0]["f"] == np.round(sc[0]["f"]))
    changed = np.mean(sc[3]["f"] != sc[0]["f"])
    assert 0.13 < changed < 0.17
    # the camera-shake PSF is irregular: neither a line nor symmetric
    h = sc[0]["psf"]
    assert not np.allclose(h, h[::-1, ::-1]) and np.count_nonzero(h) > 30


@pytest.mark.gpu
@pytest.mark.parametrize("seed", [0, 1])
def test_table1_trends(seed):
    """Table 1's trends with the paper's SNR over the whole image, and over the
    interior (a 24 px band left out), where the periodic Wiener step's border
    ringing on data blurred with constant continuation does not count (the
    paper notes the Wiener filter's sensitivity to boundary artifacts)."""
    pytest.importorskip("torch")
    for sc in synth.table1_scenarios(256, seed):
        full = quality.method_snrs(sc["f"], sc["g"], sc["psf"], sc["K"])
        inner = quality.method_snrs(sc["f"], sc["g"], sc["psf"], sc["K"], border=24)
        print(f"[snr] seed {seed} {sc['name']}: full "
              + " ".join(f"{k} {v:.2f}" for k, v in full.items()) + " | interior "
              + " ".join(f"{k} {v:.2f}" for k, v in inner.items()), flush=True)
        for s in (full, inner):
            assert s["rrrl5"] < s["rrrl30"] < s["rrrl100"]          # more iterations, sharper
        assert inner["wiener"] > inner["degraded"]
        assert inner["wr3l5"] > inner["rrrl5"]                      # the Wiener start pays off
        assert inner["wr3l5"] > inner["rrrl30"] - 3.0               # comparable to 30 RRRL iterations
        if sc["name"] == "shake_impulse15":                          # the robust data term
            assert full["rl30"] < full["degraded"]
            assert full["rrrl30"] > full["wiener"] + 3.0 and full["rrrl30"] > full["rl30"] + 3.0
        if sc["name"] == "shake_gauss5":
            assert all(v > full["degraded"] for k, v in full.items() if k != "degraded")
