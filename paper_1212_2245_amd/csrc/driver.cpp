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
    unsigned char* w8 = reinterpret_cast<unsigned char*>(ws);
    const size_t plane = round256((size_t)H * pitch * sizeof(float));
    void* list = nullptr;
    float* qw = nullptr;
    if (!use_box) {
        list = w8;
        w8 += round256(tap_list_bytes(psf));
        qw = reinterpret_cast<float*>(w8);
        w8 += round256((size_t)H * W * 2 * sizeof(float));
        launch_compile_taps(psf, list, st);
    }
    float* t0 = reinterpret_cast<float*>(w8);
    float* t1 = reinterpret_cast<float*>(w8 + plane);
    const size_t rowb = (size_t)pitch * sizeof(float);
    if (iters == 0) {
        if (u_out != u_in)
            (void)hipMemcpy2DAsync(u_out, rowb, u_in, rowb, W * sizeof(float), H, hipMemcpyDeviceToDevice, st);
        return hipGetLastError() == hipSuccess ? 0 : -4;
    }
    // iteration k writes u_out when (iters-1-k) is even, t0 otherwise; if
    // u_in aliases u_out and the first write would land there, start from a copy
    const float* src = u_in;
    if (u_in == u_out && (iters - 1) % 2 == 0) {
        (void)hipMemcpy2DAsync(t1, rowb, u_in, rowb, W * sizeof(float), H, hipMemcpyDeviceToDevice, st);
        src = t1;
    }
    for (int k = 0; k < iters; ++k) {
        float* dst = ((iters - 1 - k) % 2 == 0) ? u_out : t0;
        float* ck = ckpt ? ckpt + (size_t)k * H * pitch : nullptr;
        int s;
        if (use_box) {
            s = launch_rrrl_box_iter(f, src, dst, ck, H, W, pitch, psf.length, psf.frac, psf.kind == PSF_BOX_V, p, st);
        } else {
            s = launch_taps_stage1(f, src, qw, H, W, pitch, psf, list, p, p.tile, st);
            if (!s) s = launch_taps_stage2(qw, src, dst, ck, H, W, pitch, psf, list, p, p.tile, st);
        }
        if (s) return s;
        src = dst;
    }
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace deblur
