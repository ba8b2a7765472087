"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/deblur.h declares, and rejects invalid arguments
before touching the device.  Only error paths are exercised here (every
call below fails validation, so nothing is enqueued)."""
import ctypes
import os
import re

import pytest

from paper_1212_2245_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "deblur.h")

# fake, far-apart device addresses: only used on paths that fail validation
F, U, V, CK, WS = 0x10000000, 0x20000000, 0x30000000, 0x40000000, 0x50000000


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(deblur_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1212_2245_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert {"deblur_wiener", "deblur_rrrl_iterate", "deblur_workspace_bytes"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert {n for n, _, _ in _lib.SIGNATURES} == set(names)


def test_status_strings(lib):
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.deblur_status_string(s)
    assert lib.deblur_status_string(7) == b"unknown status"
    assert lib.deblur_version() >= 100


def box(L=15, kind=_lib.PSF_BOX_H, frac=0.0):
    return _lib.deblur_psf(kind, L, 0, 0, None, frac)


def taps(ph, pw, ptr=0x60000000):
    return _lib.deblur_psf(_lib.PSF_TAPS, 0, ph, pw, ptr)


def params(**kw):
    d = dict(alpha=0.003, eps_data=0.1, eps_tv=0.1, s_min=1e-12, iters=3, robust=1, boundary=0, conv=0, tile=0,
             psi=0, rf_lut=0, bwd_tile=0)
    d.update(kw)
    return _lib.deblur_params(*[d[k] for k, _ in _lib.deblur_params._fields_])


def wiener(lib, f=F, u=U, H=256, W=256, pitch=256, psf=None, K=0.01, floor=1.0, ws=None, wsb=0):
    psf = psf if psf is not None else box()
    return lib.deblur_wiener(f, u, H, W, pitch, ctypes.byref(psf), K, floor, ws, wsb, None)


def iterate(lib, f=F, ui=U, uo=V, H=64, W=64, pitch=64, psf=None, p=None, ck=None, ws=None, wsb=0):
    psf = psf if psf is not None else box()
    p = p if p is not None else params()
    return lib.deblur_rrrl_iterate(f, ui, uo, H, W, pitch, ctypes.byref(psf), ctypes.byref(p), ck, ws, wsb,
                                   None)


def test_workspace_bytes(lib):
    p = params()
    assert lib.deblur_workspace_bytes(0, 256, 256, 256, ctypes.byref(box()), None) > 0
    assert lib.deblur_workspace_bytes(1, 256, 256, 256, ctypes.byref(box(14, frac=0.5)), ctypes.byref(p)) > 0
    assert lib.deblur_workspace_bytes(1, 256, 256, 256, ctypes.byref(box(14, frac=1.5)), ctypes.byref(p)) == 0
    assert lib.deblur_workspace_bytes(0, 256, 256, 256, ctypes.byref(taps(31, 31)), None) > 0
    assert lib.deblur_workspace_bytes(1, 100, 77, 80, ctypes.byref(taps(31, 31)), ctypes.byref(p)) > 0
    assert lib.deblur_workspace_bytes(0, 256, 250, 256, ctypes.byref(box()), None) == 0   # 250 = 2 * 5^3
    assert lib.deblur_workspace_bytes(2, 256, 256, 256, ctypes.byref(box()), None) == 0   # unknown op
    assert lib.deblur_workspace_bytes(1, 64, 64, 63, ctypes.byref(box()), ctypes.byref(p)) == 0


def test_wiener_validation(lib):
    E, U_, W_ = _lib.DEBLUR_EINVAL, _lib.DEBLUR_EUNSUPPORTED, _lib.DEBLUR_EWORKSPACE
    assert wiener(lib, f=None) == E
    assert wiener(lib, u=None) == E
    assert wiener(lib, H=0) == E
    assert wiener(lib, pitch=255) == E
    assert wiener(lib, K=0.0) == E
    assert wiener(lib, K=float("nan")) == E
    assert wiener(lib, floor=0.0) == E
    assert wiener(lib, psf=box(0)) == E
    assert wiener(lib, psf=box(0, frac=0.5)) == E                # length 0.5 < 1
    for bad in (-0.25, 1.0, 1.5, float("nan"), float("inf")):
        assert wiener(lib, psf=box(14, frac=bad)) == E           # fractional part outside [0, 1)
    assert wiener(lib, psf=box(63, _lib.PSF_BOX_V, frac=0.5)) == W_  # 65 entries: supported
    assert wiener(lib, psf=box(64, _lib.PSF_BOX_V, frac=0.5)) == U_  # 67 entries: beyond the tap limit
    assert wiener(lib, psf=_lib.deblur_psf(9, 3, 0, 0, None)) == E
    assert wiener(lib, psf=taps(4, 5)) == E                      # even dims
    assert wiener(lib, psf=_lib.deblur_psf(_lib.PSF_TAPS, 0, 3, 3, None)) == E
    assert wiener(lib, psf=taps(67, 3)) == U_                    # beyond the tap limit
    assert wiener(lib, W=250, pitch=256) == U_                   # prime factor 5
    assert wiener(lib, H=250, psf=taps(3, 3)) == U_              # 2D path needs H = 2^a 3^b
    assert wiener(lib, H=250) == W_                              # row-wise path: H free
    assert wiener(lib, W=8192, pitch=8192) == U_
    assert wiener(lib, u=F + 100) == E                           # overlapping f and u0
    assert wiener(lib) == W_
    assert wiener(lib, ws=WS, wsb=16) == W_


def test_iterate_validation(lib):
    E, U_, W_ = _lib.DEBLUR_EINVAL, _lib.DEBLUR_EUNSUPPORTED, _lib.DEBLUR_EWORKSPACE
    assert iterate(lib, f=None) == E
    assert iterate(lib, ui=None) == E
    assert iterate(lib, uo=None) == E
    assert iterate(lib, W=0) == E
    assert iterate(lib, pitch=10) == E
    assert iterate(lib, p=params(alpha=-1.0)) == E
    assert iterate(lib, p=params(eps_data=0.0)) == E
    assert iterate(lib, p=params(eps_tv=-1.0)) == E
    assert iterate(lib, p=params(s_min=0.0)) == E
    assert iterate(lib, p=params(iters=-1)) == E
    assert iterate(lib, p=params(robust=2)) == E
    assert iterate(lib, p=params(psi=2)) == E
    assert iterate(lib, p=params(psi=-1)) == E
    assert iterate(lib, p=params(psi=1)) == W_                      # Perona-Malik: valid
    assert iterate(lib, p=params(rf_lut=2)) == E
    assert iterate(lib, p=params(boundary=5)) == E
    assert iterate(lib, p=params(conv=9)) == E
    assert iterate(lib, p=params(tile=-1)) == E
    assert iterate(lib, p=params(tile=lib.deblur_tile_variants() + 1)) == E
    assert iterate(lib, p=params(tile=lib.deblur_tile_variants()), psf=taps(5, 5)) == W_
    assert iterate(lib, psf=taps(3, 3), p=params(conv=_lib.CONV_RUNSUM)) == E
    assert iterate(lib, psf=taps(67, 1)) == U_
    assert iterate(lib, uo=F) == E                                # u_out overlaps f
    assert iterate(lib, ui=V + 4) == E                            # partial overlap u_in / u_out
    assert iterate(lib, ck=F) == E                                # ckpt overlaps f
    assert iterate(lib, ui=V) == W_                               # u_in == u_out is allowed
    assert iterate(lib) == W_
    assert iterate(lib, ws=WS, wsb=64) == W_


def test_iterate_noalloc_validation(lib):
    """Error paths of the no-allocation variant: rejected before the static
    scratch is looked up or anything is enqueued."""
    E, U_, S_ = _lib.DEBLUR_EINVAL, _lib.DEBLUR_EUNSUPPORTED, _lib.DEBLUR_ESCRATCH

    def call(f=F, ui=U, uo=V, H=64, W=64, pitch=64, psf=None, p=None, ck=None):
        psf = psf if psf is not None else box()
        p = p if p is not None else params()
        return lib.deblur_rrrl_iterate_noalloc(f, ui, uo, H, W, pitch, ctypes.byref(psf), ctypes.byref(p), ck, None)

    assert call(f=None) == E
    assert call(uo=F) == E
    assert call(p=params(alpha=-1.0)) == E
    assert call(p=params(rf_lut=1)) == U_                        # the lookup mode would allocate its table
    assert lib.deblur_rrrl_iterate_noalloc(F, U, V, 64, 64, 64, ctypes.byref(box()), None, None, None) == E
    # stencil path at 2048 x 2048: 16 B/px of workspace plus the tap list > 64 MiB
    need = lib.deblur_workspace_bytes(1, 2048, 2048, 2048, ctypes.byref(taps(5, 5)), ctypes.byref(params()))
    assert need > _lib.NOALLOC_SCRATCH_BYTES
    far = 0x1000000000
    assert call(f=far, ui=2 * far, uo=3 * far, H=2048, W=2048, pitch=2048, psf=taps(5, 5)) == S_
    assert lib.deblur_status_string(S_) and b"scratch" in lib.deblur_status_string(S_)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        _lib.load()


def batch_item(f=F, u=U, H=128, W=128, pitch=128, psf=None, iters=3, K=0.01, floor=1.0):
    return _lib.deblur_batch_item(f, u, H, W, pitch, psf if psf is not None else box(), params(iters=iters), K, floor)


def test_batch_validation(lib):
    E = _lib.DEBLUR_EINVAL
    plan = ctypes.c_void_p()
    arr = (_lib.deblur_batch_item * 2)(batch_item(), batch_item(f=0x70000000, u=0x78000000))
    assert lib.deblur_batch_plan_create(arr, 0, 0, ctypes.byref(plan)) == E
    assert lib.deblur_batch_plan_create(arr, 2, -1, ctypes.byref(plan)) == E
    assert lib.deblur_batch_plan_create(None, 2, 0, ctypes.byref(plan)) == E
    bad = (_lib.deblur_batch_item * 2)(batch_item(), batch_item(f=0x70000000, u=0x78000000, iters=4))
    assert lib.deblur_batch_plan_create(bad, 2, 0, ctypes.byref(plan)) == E          # different iters
    bad = (_lib.deblur_batch_item * 1)(batch_item(u=F + 64))
    assert lib.deblur_batch_plan_create(bad, 1, 0, ctypes.byref(plan)) == E          # f and u overlap
    bad = (_lib.deblur_batch_item * 1)(batch_item(W=250, pitch=256))
    assert lib.deblur_batch_plan_create(bad, 1, 0, ctypes.byref(plan)) == _lib.DEBLUR_EUNSUPPORTED
    bad = (_lib.deblur_batch_item * 1)(batch_item(K=0.0))
    assert lib.deblur_batch_plan_create(bad, 1, 0, ctypes.byref(plan)) == E
    assert lib.deblur_batch_run(None, None) == E
    assert lib.deblur_batch_latencies(None, None) == E
    assert lib.deblur_batch_size(None) == 0
    lib.deblur_batch_plan_destroy(None)


def test_backward_tile_validation(lib):
    assert lib.deblur_backward_tile_variants() == 4
    assert iterate(lib, p=params(bwd_tile=5)) == _lib.DEBLUR_EINVAL
    assert iterate(lib, p=params(bwd_tile=-1)) == _lib.DEBLUR_EINVAL


def test_batch_tiles_validation(lib):
    """Tile shapes of a plan: variant counts per family; out-of-range shapes
    and FFT-path items are rejected before any device work."""
    E = _lib.DEBLUR_EINVAL
    assert lib.deblur_batch_tile_variants(0) == 3
    assert lib.deblur_batch_tile_variants(1) == lib.deblur_box_tile_variants() == 5
    assert lib.deblur_batch_tile_variants(2) == 0
    plan = ctypes.c_void_p()
    arr = (_lib.deblur_batch_item * 1)(batch_item())
    for t in ((4, 0, 0, 0, 0), (0, 6, 0, 0, 0), (0, 0, 6, 0, 0), (0, 0, 0, 6, 0), (0, 0, 0, 0, 6), (-1, 0, 0, 0, 0)):
        t5 = (ctypes.c_int32 * 5)(*t)
        assert lib.deblur_batch_plan_create_tiled(arr, 1, 0, t5, ctypes.byref(plan)) == E
    fft = batch_item()
    fft.p.conv = _lib.CONV_FFT
    fft.p.boundary = _lib.BC_PERIODIC
    arr = (_lib.deblur_batch_item * 1)(fft)
    assert lib.deblur_batch_plan_create(arr, 1, 0, ctypes.byref(plan)) == _lib.DEBLUR_EUNSUPPORTED
    t5 = (ctypes.c_int32 * 5)(1, 2, 3, 4, 5)
    assert lib.deblur_batch_plan_create_tiled(arr, 1, 0, t5, ctypes.byref(plan)) == _lib.DEBLUR_EUNSUPPORTED
    assert lib.deblur_batch_class_of(None, 0) == E
    assert lib.deblur_batch_class_tiles(None, 0) == E
    assert lib.deblur_batch_launch_class(None, 0, 1, None) == E


def test_backward_validation(lib):
    E = _lib.DEBLUR_EINVAL
    p = params(iters=2)

    def bw(f=F, ck=CK, g=V, H=64, W=64, pitch=64, psf=None, tw=1, K=0.01, gf=0x58000000, ws=None, wsb=0, pp=None):
        psf = psf if psf is not None else taps(5, 5)
        return lib.deblur_rrrl_backward(f, ck, g, H, W, pitch, ctypes.byref(psf), ctypes.byref(pp or p), tw, K, 1.0,
                                        gf, None, None, None, ws, wsb, None)
    assert bw(f=None) == E
    assert bw(gf=None) == E
    assert bw(ck=None) == E                      # iters > 0 needs checkpoints
    assert bw(tw=2) == E
    assert bw(K=0.0) == E
    assert bw(gf=F) == E                         # grad_f overlaps f
    assert bw(H=100) == _lib.DEBLUR_EUNSUPPORTED  # through the Wiener step: 2^a 3^b
    assert bw(H=100, tw=0) == _lib.DEBLUR_EWORKSPACE
    assert bw() == _lib.DEBLUR_EWORKSPACE
    assert lib.deblur_workspace_bytes(3, 64, 64, 64, ctypes.byref(taps(5, 5)), ctypes.byref(p)) > \
        lib.deblur_workspace_bytes(2, 64, 64, 64, ctypes.byref(taps(5, 5)), ctypes.byref(p)) > 0


def test_backward_batch_validation(lib):
    E = _lib.DEBLUR_EINVAL
    p = params(iters=2)
    img = 64 * 64

    def bb(B=4, f=F, ck=CK, g=V, H=64, W=64, pitch=64, istr=img, cstr=2 * img, psf=None, tstr=25, tw=1, K=0.01,
           gf=0x58000000, ws=None, wsb=0, pp=None):
        psf = psf if psf is not None else taps(5, 5)
        return lib.deblur_rrrl_backward_batch(B, f, ck, g, H, W, pitch, istr, cstr, ctypes.byref(psf), tstr, None,
                                              ctypes.byref(pp or p), tw, K, 1.0, gf, None, None, None, ws, wsb, None)
    assert bb(B=0) == E
    assert bb(B=65536) == E
    assert bb(f=None) == E
    assert bb(gf=None) == E
    assert bb(ck=None) == E                      # iters > 0 needs checkpoints
    assert bb(tw=2) == E
    assert bb(K=0.0) == E
    assert bb(istr=img - 1) == E                 # images would overlap
    assert bb(cstr=2 * img - 1) == E             # checkpoints of consecutive images would overlap
    assert bb(tstr=24) == E                      # PSFs would overlap
    assert bb(psf=box(), tstr=1) == E            # box PSFs are shared: stride 0
    assert bb(gf=F + 4 * 3 * img) == E           # grad_f overlaps image 3 of f
    assert bb(H=100) == _lib.DEBLUR_EUNSUPPORTED  # through the Wiener step: 2^a 3^b
    assert bb() == _lib.DEBLUR_EWORKSPACE
    assert bb(tstr=0) == _lib.DEBLUR_EWORKSPACE   # one shared PSF is valid
    one = lib.deblur_workspace_bytes(3, 64, 64, 64, ctypes.byref(taps(5, 5)), ctypes.byref(p))
    four = lib.deblur_workspace_bytes_batch(3, 4, 64, 64, 64, ctypes.byref(taps(5, 5)), ctypes.byref(p))
    assert four >= 4 * one and four % (4 * 256) == 0
    assert bb(ws=WS, wsb=four - 1) == _lib.DEBLUR_EWORKSPACE
    assert lib.deblur_workspace_bytes_batch(3, 0, 64, 64, 64, ctypes.byref(taps(5, 5)), ctypes.byref(p)) == 0
    assert lib.deblur_workspace_bytes_batch(3, 4, 64, 64, 64, ctypes.byref(taps(5, 5)), None) == 0


def test_wiener_and_iterate_batch_validation(lib):
    E = _lib.DEBLUR_EINVAL
    img = 64 * 64

    def wb(B=4, f=F, u=U, H=64, W=64, pitch=64, istr=img, psf=None, tstr=25, K=0.01, floor=1.0, fp64=0, ws=None,
           wsb=0):
        psf = psf if psf is not None else taps(5, 5)
        return lib.deblur_wiener_batch(B, f, u, H, W, pitch, istr, ctypes.byref(psf), tstr, K, floor, fp64, ws, wsb,
                                       None)
    assert wb(B=0) == E
    assert wb(f=None) == E
    assert wb(fp64=2) == E
    assert wb(K=0.0) == E
    assert wb(floor=0.0) == E
    assert wb(istr=img - 1) == E
    assert wb(tstr=24) == E
    assert wb(psf=box(), tstr=25) == E
    assert wb(u=F + 4 * 3 * img) == E              # u0 overlaps image 3 of f
    assert wb(H=100) == _lib.DEBLUR_EUNSUPPORTED
    assert wb() == _lib.DEBLUR_EWORKSPACE
    need = lib.deblur_workspace_bytes_batch(4, 4, 64, 64, 64, ctypes.byref(taps(5, 5)), None)
    assert need >= 4 * lib.deblur_workspace_bytes(4, 64, 64, 64, ctypes.byref(taps(5, 5)), None) > 0
    assert wb(fp64=1, ws=WS, wsb=need - 1) == _lib.DEBLUR_EWORKSPACE

    p = params(iters=3)

    def ib(B=4, f=F, ui=U, uo=U, H=64, W=64, pitch=64, istr=img, psf=None, tstr=25, pp=None, ck=None, cstr=0,
           ws=None, wsb=0):
        psf = psf if psf is not None else taps(5, 5)
        return lib.deblur_rrrl_iterate_batch(B, f, ui, uo, H, W, pitch, istr, ctypes.byref(psf), tstr, None,
                                             ctypes.byref(pp or p), ck, cstr, ws, wsb, None)
    assert ib(B=65536) == E
    assert ib(uo=None) == E
    assert ib(istr=img - 1) == E
    assert ib(tstr=24) == E
    assert ib(psf=box(), tstr=1) == E
    assert ib(uo=F) == E                            # output overlaps f
    assert ib(ck=CK, cstr=3 * img - 1) == E         # checkpoints of consecutive images overlap
    assert ib(ck=U + 4 * img, cstr=3 * img) == E    # checkpoints overlap image 1 of u
    assert ib(pp=params(iters=3, conv=_lib.CONV_FFT, boundary=_lib.BC_PERIODIC)) == _lib.DEBLUR_EUNSUPPORTED
    assert lib.deblur_workspace_bytes_batch(1, 4, 64, 64, 64, ctypes.byref(taps(5, 5)),
                                            ctypes.byref(params(conv=_lib.CONV_FFT, boundary=_lib.BC_PERIODIC))) == 0
    assert ib() == _lib.DEBLUR_EWORKSPACE
    assert ib(psf=box(), tstr=0) == _lib.DEBLUR_EWORKSPACE
    need = lib.deblur_workspace_bytes_batch(1, 4, 64, 64, 64, ctypes.byref(taps(5, 5)), ctypes.byref(p))
    assert need >= 4 * lib.deblur_workspace_bytes(1, 64, 64, 64, ctypes.byref(taps(5, 5)), ctypes.byref(p)) > 0
    assert ib(ws=WS, wsb=need - 1) == _lib.DEBLUR_EWORKSPACE
