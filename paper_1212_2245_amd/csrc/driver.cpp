// RRRL iteration driver: ping-pong between the caller's output and a
// workspace buffer so that the last iteration lands in u_out.
#include "launch.hpp"

namespace deblur {

static size_t round256(size_t n) { return (n + 255) & ~(size_t)255; }

size_t iterate_ws_bytes(int H, int W, int pitch, const PsfDev& psf, bool use_box)
{
    const size_t plane = round256((size_t)H * pitch * sizeof(float));
    if (use_box) return 2 * plane;
    return round256(tap_list_bytes(psf)) + round256((size_t)H * W * 2 * sizeof(float)) + 2 * plane;
}

int launch_rrrl_iterate(const float* f, const float* u_in, float* u_out, int H, int W, int pitch,
                        const PsfDev& psf, const IterParams& p, int iters, float* ckpt, bool use_box, void* ws,
                        hipStream_t st)
{
    return launch_rrrl_iterate_batch(1, f, u_in, u_out, H, W, pitch, 0, psf, 0, nullptr, p, iters, ckpt, 0, use_box,
                                     ws, 0, st);
}

static const float* adv(const float* p, size_t bytes, int b)
{
    return reinterpret_cast<const float*>(reinterpret_cast<const unsigned char*>(p) + (size_t)b * bytes);
}

int launch_rrrl_iterate_batch(int B, const float* f, const float* u_in, float* u_out, int H, int W, int pitch,
                              size_t img_stride, const PsfDev& psf, size_t taps_stride, const float* alpha,
                              const IterParams& p, int iters, float* ckpt, size_t ck_stride, bool use_box, void* ws,
                              size_t ws_stride, hipStream_t st)
{
    unsigned char* w8 = reinterpret_cast<unsigned char*>(ws);
    const size_t plane = round256((size_t)H * pitch * sizeof(float));
    void* list = nullptr;
    float* qw = nullptr;
    if (!use_box) {
        list = w8;
        w8 += round256(tap_list_bytes(psf));
        qw = reinterpret_cast<float*>(w8);
        w8 += round256((size_t)H * W * 2 * sizeof(float));
        launch_compile_taps(psf, list, st, ZBatch{B, taps_stride, ws_stride});
    }
    float* t0 = reinterpret_cast<float*>(w8);
    float* t1 = reinterpret_cast<float*>(w8 + plane);
    const size_t rowb = (size_t)pitch * sizeof(float);
    auto copy = [&](float* dst, size_t dz, const float* src, size_t sz) {
        for (int b = 0; b < B; ++b)
            (void)hipMemcpy2DAsync(const_cast<float*>(adv(dst, dz, b)), rowb, adv(src, sz, b), rowb, W * sizeof(float),
                                   H, hipMemcpyDeviceToDevice, st);
    };
    if (iters == 0) {
        if (u_out != u_in) copy(u_out, img_stride, u_in, img_stride);
        return hipGetLastError() == hipSuccess ? 0 : -4;
    }
    // iteration k writes u_out when (iters-1-k) is even, t0 otherwise; if
    // u_in aliases u_out and the first write would land there, start from a copy
    const float* src = u_in;
    size_t src_z = img_stride;
    if (u_in == u_out && (iters - 1) % 2 == 0) {
        copy(t1, ws_stride, u_in, img_stride);
        src = t1;
        src_z = ws_stride;
    }
    for (int k = 0; k < iters; ++k) {
        const bool out = (iters - 1 - k) % 2 == 0;
        float* dst = out ? u_out : t0;
        IterZ z;
        z.f = img_stride;
        z.u = src_z;
        z.un = out ? img_stride : ws_stride;
        z.ck = ck_stride;
        z.ws = ws_stride;
        z.alpha = alpha;
        float* ck = ckpt ? ckpt + (size_t)k * H * pitch : nullptr;
        int s;
        if (use_box) {
            s = launch_rrrl_box_iter(f, src, dst, ck, H, W, pitch, psf.length, psf.frac, psf.kind == PSF_BOX_V, p, st,
                                     B, z);
        } else {
            s = launch_taps_stage1(f, src, qw, H, W, pitch, psf, list, p, p.tile, st, nullptr, B, z);
            if (!s) s = launch_taps_stage2(qw, src, dst, ck, H, W, pitch, psf, list, p, p.tile, st, B, z);
        }
        if (s) return s;
        src = dst;
        src_z = z.un;
    }
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace deblur
