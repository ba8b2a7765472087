"""Device PSF compiler (deblur_compile_taps): bit-exact check of the tap list,
the column groups and their packed copy against the layout documented in
deblur.h, for
sparse, dense, gapped and boundary-size PSFs."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1212_2245_amd as dbl  # noqa: E402


def expected_groups(h):
    """Column runs of non-zero taps, split every 8 rows, ordered by length
    descending, then column, then first row."""
    ph, pw = h.shape
    cy, cx = (ph - 1) // 2, (pw - 1) // 2
    out = []
    for i in range(pw):
        j = 0
        while j < ph:
            if h[j, i] == 0:
                j += 1
                continue
            j0 = j
            while j < ph and h[j, i] != 0 and j - j0 < 8:
                j += 1
            out.append((j - j0, i - cx, j0 - cy, [float(v) for v in h[j0:j, i]]))
    out.sort(key=lambda g: (-g[0], g[1], g[2]))
    return out


def decode(buf, ph, pw):
    b = buf.cpu().numpy().tobytes()
    hdr = np.frombuffer(b[:44], dtype=np.int32)
    T, G = int(hdr[0]), int(hdr[1])
    taps = np.frombuffer(b[256:256 + 16 * T], dtype=np.int32).reshape(T, 4)
    goff = 256 + 16 * ph * pw
    groups = []
    for k in range(G):
        rec = b[goff + 48 * k: goff + 48 * (k + 1)]
        dx, dy0, S, _ = np.frombuffer(rec[:16], dtype=np.int32)
        w = np.frombuffer(rec[16:48], dtype=np.float32)
        groups.append((int(S), int(dx), int(dy0), [float(v) for v in w[:S]]))
    poff = goff + 48 * ph * pw
    words = np.frombuffer(b[poff:poff + 4 * int(hdr[10])], dtype=np.int32)
    packed, k = [], 0
    while k < len(words):
        h = int(words[k])
        dx, dy0 = ((h & 0xFFFF) ^ 0x8000) - 0x8000, h >> 16
        S = next(g[0] for g in groups if g[1] == dx and g[2] == dy0)
        w = words[k + 1:k + 1 + S].view(np.float32)
        packed.append((S, dx, dy0, [float(v) for v in w]))
        k += 1 + S
    return hdr, taps, groups, packed


def psfs():
    rng = np.random.default_rng(5)
    yield "line31", synth.line_psf(31, 2.095)
    yield "gauss31", synth.gauss_mixture_psf(synth.rng_for(2), 31)
    gap = np.zeros((21, 5), np.float32)
    gap[0:3, 0] = 1
    gap[4:17, 2] = 1      # a run of 13: 8 + 5
    gap[18, 2] = 1
    gap[::2, 4] = 1       # isolated taps
    yield "gapped", gap / gap.sum()
    d = rng.random((65, 65)).astype(np.float32) + 0.01
    yield "dense65", d / d.sum()
    yield "one", np.ones((1, 1), np.float32)
    r = rng.random((9, 13)).astype(np.float32)
    r[r < 0.6] = 0
    yield "sparse9x13", r / r.sum()


@pytest.mark.parametrize("name,h", list(psfs()), ids=[n for n, _ in psfs()])
def test_compiled_taps_bit_exact(name, h):
    h = np.ascontiguousarray(h, dtype=np.float32)
    ph, pw = h.shape
    psf = dbl.Psf.from_taps(torch.from_numpy(h).cuda())
    buf = dbl.deblur_compile_taps(psf)
    torch.cuda.synchronize()
    hdr, taps, groups, packed = decode(buf, ph, pw)
    nz = np.argwhere(h != 0)
    assert int(hdr[0]) == len(nz)
    cy, cx = (ph - 1) // 2, (pw - 1) // 2
    want_taps = np.array([[j - cy, i - cx, np.float32(h[j, i]).view(np.int32), 0] for j, i in nz], dtype=np.int32)
    assert np.array_equal(taps, want_taps.reshape(-1, 4))
    want = expected_groups(h)
    assert groups == want
    for S in range(1, 9):
        assert int(hdr[1 + S]) == sum(g[0] == S for g in want)
    assert int(hdr[1]) == len(want)
    assert int(hdr[10]) == len(want) + len(nz) and packed == want
    print(f"[taps] {name}: {len(nz)} taps, {len(want)} groups", flush=True)
