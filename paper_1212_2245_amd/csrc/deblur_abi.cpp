// Host side of the C ABI declared in include/deblur.h: argument validation,
// workspace sizing and dispatch to the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

#include "deblur.h"
#include "psf.hpp"

#include "launch.hpp"

using namespace deblur;

namespace {

constexpr int kMaxFft = 2048;
constexpr int kMaxTapDim = 65;

bool is_2a3b(int n)
{
    if (n < 1) return false;
    while (n % 3 == 0) n /= 3;
    while (n % 2 == 0) n /= 2;
    return n == 1;
}

// Validates a PSF descriptor and converts it; DEBLUR_OK or an error code.
int convert_psf(const deblur_psf* psf, PsfDev* out)
{
    if (!psf) return DEBLUR_EINVAL;
    PsfDev d{};
    d.kind = psf->kind;
    d.taps = psf->taps;
    if (psf->kind == DEBLUR_PSF_BOX_H || psf->kind == DEBLUR_PSF_BOX_V) {
        if (psf->length < 1) return DEBLUR_EINVAL;
        if (!(psf->frac >= 0.0f && psf->frac < 1.0f)) return DEBLUR_EINVAL;   // also rejects NaN
        const int P = psf->length + (psf->length % 2 == 0 ? 1 : 0) + (psf->frac > 0.0f ? 2 : 0);
        if (P > kMaxTapDim) return DEBLUR_EUNSUPPORTED;
        d.length = psf->length;
        d.frac = psf->frac;
        d.ph = psf->kind == DEBLUR_PSF_BOX_H ? 1 : P;
        d.pw = psf->kind == DEBLUR_PSF_BOX_H ? P : 1;
    } else if (psf->kind == DEBLUR_PSF_TAPS) {
        if (!psf->taps || psf->ph < 1 || psf->pw < 1 || psf->ph % 2 == 0 || psf->pw % 2 == 0)
            return DEBLUR_EINVAL;
        if (psf->ph > kMaxTapDim || psf->pw > kMaxTapDim) return DEBLUR_EUNSUPPORTED;
        d.length = 0;
        d.frac = 0.0f;
        d.ph = psf->ph;
        d.pw = psf->pw;
    } else {
        return DEBLUR_EINVAL;
    }
    *out = d;
    return DEBLUR_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + nb && y < x + na;
}

int check_image(int32_t H, int32_t W, int32_t pitch)
{
    if (H < 1 || W < 1 || pitch < W) return DEBLUR_EINVAL;
    if ((int64_t)H * pitch > (int64_t)1 << 31) return DEBLUR_EUNSUPPORTED;
    return DEBLUR_OK;
}

bool wiener_rowwise(const PsfDev& d) { return d.ph == 1; }

int check_wiener(int32_t H, int32_t W, int32_t pitch, const deblur_psf* psf, PsfDev* d)
{
    int s = check_image(H, W, pitch);
    if (s) return s;
    if ((s = convert_psf(psf, d))) return s;
    if (d->ph > H || d->pw > W) return DEBLUR_EINVAL;
    if (!is_2a3b(W) || W > kMaxFft) return DEBLUR_EUNSUPPORTED;
    if (!wiener_rowwise(*d) && (!is_2a3b(H) || H > kMaxFft)) return DEBLUR_EUNSUPPORTED;
    return DEBLUR_OK;
}

// Device table of r_1 for the lookup mode of r_f, built on first use on
// each device (host FP64, rounded once) and kept until the process ends.
const float* r1_table()
{
    static std::mutex mu;
    static std::vector<float*> tables;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)tables.size() <= dev) tables.resize(dev + 1, nullptr);
    if (tables[dev]) return tables[dev];
    std::vector<float> h(RF_LUT_WORDS);
    for (int k = 1; k <= RF_LUT_N; ++k) {
        const double x = (double)k / RF_LUT_PER_UNIT;
        h[k] = (float)((x - 1.0) - std::log(x));
    }
    h[0] = h[1];
    h[RF_LUT_N + 1] = (float)(1.0 - 1.0 / 65.0);
    float* d = nullptr;
    if (hipMalloc(&d, sizeof(float) * RF_LUT_WORDS) != hipSuccess) return nullptr;
    if (hipMemcpy(d, h.data(), sizeof(float) * RF_LUT_WORDS, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return nullptr;
    }
    tables[dev] = d;
    return d;
}

int check_iterate(int32_t H, int32_t W, int32_t pitch, const deblur_psf* psf, const deblur_params* p, PsfDev* d)
{
    int s = check_image(H, W, pitch);
    if (s) return s;
    if ((s = convert_psf(psf, d))) return s;
    if (!p) return DEBLUR_EINVAL;
    if (!(p->alpha >= 0.0f) || !std::isfinite(p->alpha)) return DEBLUR_EINVAL;
    if (!(p->eps_data > 0.0f) || !std::isfinite(p->eps_data)) return DEBLUR_EINVAL;
    if (!(p->eps_tv > 0.0f) || !std::isfinite(p->eps_tv)) return DEBLUR_EINVAL;
    if (!(p->s_min > 0.0f) || !std::isfinite(p->s_min)) return DEBLUR_EINVAL;
    if (p->iters < 0 || (p->robust != 0 && p->robust != 1)) return DEBLUR_EINVAL;
    if (p->psi != 0 && p->psi != 1) return DEBLUR_EINVAL;
    if (p->rf_lut != 0 && p->rf_lut != 1) return DEBLUR_EINVAL;
    if (p->bwd_tile < 0 || p->bwd_tile > backward_tile_variants()) return DEBLUR_EINVAL;
    if (p->rf_lut && !r1_table()) return DEBLUR_EDEVICE;
    if (p->boundary != DEBLUR_BC_REPLICATE && p->boundary != DEBLUR_BC_PERIODIC) return DEBLUR_EINVAL;
    if (p->conv < DEBLUR_CONV_AUTO || p->conv > DEBLUR_CONV_FFT) return DEBLUR_EINVAL;
    if (p->conv == DEBLUR_CONV_FFT) {
        if (p->boundary != DEBLUR_BC_PERIODIC) return DEBLUR_EINVAL;  // Fourier domain: periodic only
        if (!is_2a3b(H) || !is_2a3b(W) || H > kMaxFft || W > kMaxFft) return DEBLUR_EUNSUPPORTED;
        if (d->ph > H || d->pw > W) return DEBLUR_EINVAL;
        if (p->tile < 0 || p->tile > taps_num_variants()) return DEBLUR_EINVAL;
        return DEBLUR_OK;
    }
    if (p->conv == DEBLUR_CONV_RUNSUM && d->kind == DEBLUR_PSF_TAPS) return DEBLUR_EINVAL;
    if (p->tile < 0 || p->tile > taps_num_variants()) return DEBLUR_EINVAL;
    if (d->kind != DEBLUR_PSF_TAPS && p->conv != DEBLUR_CONV_STENCIL && p->tile > box_num_variants())
        return DEBLUR_EINVAL;
    const int rad = (d->ph - 1) / 2 > (d->pw - 1) / 2 ? (d->ph - 1) / 2 : (d->pw - 1) / 2;
    if (tap_radius_class(rad) < 0) return DEBLUR_EUNSUPPORTED;
    if ((d->ph - 1) / 2 > H || (d->pw - 1) / 2 > W) return DEBLUR_EINVAL;
    return DEBLUR_OK;
}

int check_backward(int32_t H, int32_t W, int32_t pitch, const deblur_psf* psf, const deblur_params* p,
                   bool through_wiener, PsfDev* d)
{
    int s = check_iterate(H, W, pitch, psf, p, d);
    if (s) return s;
    if (p->rf_lut) return DEBLUR_EUNSUPPORTED;   // the adjoint differentiates the exact r_f
    if (through_wiener && (!is_2a3b(H) || !is_2a3b(W) || H > kMaxFft || W > kMaxFft)) return DEBLUR_EUNSUPPORTED;
    if (through_wiener && (d->ph > H || d->pw > W)) return DEBLUR_EINVAL;
    return DEBLUR_OK;
}

bool use_box(const PsfDev& d, const deblur_params* p)
{
    return d.kind != DEBLUR_PSF_TAPS && p->conv != DEBLUR_CONV_STENCIL;
}

IterParams iter_params(const deblur_params* p)
{
    IterParams q;
    q.alpha = p->alpha;
    q.eps_d2 = p->eps_data * p->eps_data;
    q.eps_t2 = p->eps_tv * p->eps_tv;
    q.s_min = p->s_min;
    q.robust = p->robust;
    q.psi = p->psi;
    q.bwd_tile = p->bwd_tile;
    q.r1_lut = p->rf_lut ? r1_table() : nullptr;
    q.bc = p->boundary;
    q.tile = p->tile;
    return q;
}

// deblur_rrrl_iterate and its no-allocation variant: validation, then the
// iteration driver on the caller's workspace or, when use_static, on the
// library's static scratch (after checking that the need fits in it).
int iterate_impl(const float* f, const float* u_in, float* u_out, int32_t H, int32_t W, int32_t pitch,
                 const deblur_psf* psf, const deblur_params* p, float* ckpt, void* ws, size_t ws_bytes,
                 bool use_static, void* stream)
{
    PsfDev d;
    if (!f || !u_in || !u_out) return DEBLUR_EINVAL;
    int s = check_iterate(H, W, pitch, psf, p, &d);
    if (s) return s;
    const size_t img = (size_t)H * pitch * sizeof(float);
    if (overlaps(f, img, u_out, img) || (u_in != u_out && overlaps(u_in, img, u_out, img))) return DEBLUR_EINVAL;
    if (ckpt) {
        const size_t ck = img * (size_t)p->iters;
        if (overlaps(ckpt, ck, f, img) || overlaps(ckpt, ck, u_in, img) || overlaps(ckpt, ck, u_out, img))
            return DEBLUR_EINVAL;
    }
    const bool fft = p->conv == DEBLUR_CONV_FFT;
    const bool box = !fft && use_box(d, p);
    const size_t need = fft ? fft_iter_ws_bytes(H, W, pitch) : iterate_ws_bytes(H, W, pitch, d, box);
    if (use_static) {
        if (need > NOALLOC_SCRATCH_BYTES) return DEBLUR_ESCRATCH;
        hipError_t e = hipSuccess;
        ws = noalloc_scratch(&e);
        if (!ws) return DEBLUR_EDEVICE;
        ws_bytes = NOALLOC_SCRATCH_BYTES;
    }
    if (!ws || ws_bytes < need) return DEBLUR_EWORKSPACE;
    const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (fft) {
        s = launch_rrrl_fft(f, u_in, u_out, H, W, pitch, d, iter_params(p), p->iters, ckpt, ws, st);
        return s == 0 ? DEBLUR_OK : DEBLUR_EDEVICE;
    }
    s = launch_rrrl_iterate(f, u_in, u_out, H, W, pitch, d, iter_params(p), p->iters, ckpt, box, ws, st);
    return s == 0 ? DEBLUR_OK : (s == -2 ? DEBLUR_EUNSUPPORTED : DEBLUR_EDEVICE);
}

}  // namespace

struct deblur_batch_plan {
    deblur::BatchPlan* impl;
};

extern "C" {

const char* deblur_status_string(int status)
{
    switch (status) {
        case DEBLUR_OK: return "ok";
        case DEBLUR_EINVAL: return "invalid argument";
        case DEBLUR_EUNSUPPORTED: return "unsupported configuration";
        case DEBLUR_EWORKSPACE: return "workspace missing or too small";
        case DEBLUR_EDEVICE: return "HIP device or launch failure";
        case DEBLUR_ESCRATCH: return "problem exceeds the static scratch of the no-allocation entry point";
        default: return "unknown status";
    }
}

int deblur_version(void) { return 100; }

int deblur_tile_variants(void) { return taps_num_variants(); }

int deblur_box_tile_variants(void) { return box_num_variants(); }

int deblur_backward_tile_variants(void) { return backward_tile_variants(); }

size_t deblur_workspace_bytes(int32_t op, int32_t H, int32_t W, int32_t pitch, const deblur_psf* psf,
                              const deblur_params* p)
{
    PsfDev d;
    if (op == 0 || op == 4) {
        if (check_wiener(H, W, pitch, psf, &d)) return 0;
        return wiener_ws_bytes(H, W, wiener_rowwise(d), op == 4);
    }
    if (op == 1) {
        if (check_iterate(H, W, pitch, psf, p, &d)) return 0;
        if (p->conv == DEBLUR_CONV_FFT) return fft_iter_ws_bytes(H, W, pitch);
        return iterate_ws_bytes(H, W, pitch, d, use_box(d, p));
    }
    if (op == 2 || op == 3) {
        if (check_backward(H, W, pitch, psf, p, op == 3, &d)) return 0;
        return backward_ws_bytes(H, W, d, op == 3);
    }
    return 0;
}

static int wiener_impl(const float* f, float* u0, int32_t H, int32_t W, int32_t pitch, const deblur_psf* psf,
                       double K, float pos_floor, void* ws, size_t ws_bytes, bool fp64, void* stream)
{
    PsfDev d;
    if (!f || !u0) return DEBLUR_EINVAL;
    int s = check_wiener(H, W, pitch, psf, &d);
    if (s) return s;
    if (!(K > 0.0) || !std::isfinite(K) || !(pos_floor > 0.0f) || !std::isfinite(pos_floor)) return DEBLUR_EINVAL;
    const size_t img = (size_t)H * pitch * sizeof(float);
    if (overlaps(f, img, u0, img)) return DEBLUR_EINVAL;
    const size_t need = wiener_ws_bytes(H, W, wiener_rowwise(d), fp64);
    if (!ws || ws_bytes < need) return DEBLUR_EWORKSPACE;
    return launch_wiener(f, u0, H, W, pitch, d, K, pos_floor, ws, wiener_rowwise(d), fp64,
                         reinterpret_cast<hipStream_t>(stream)) == 0
               ? DEBLUR_OK
               : DEBLUR_EDEVICE;
}

int deblur_wiener(const float* f, float* u0, int32_t H, int32_t W, int32_t pitch, const deblur_psf* psf,
                  double K, float pos_floor, void* ws, size_t ws_bytes, void* stream)
{
    return wiener_impl(f, u0, H, W, pitch, psf, K, pos_floor, ws, ws_bytes, false, stream);
}

int deblur_wiener_fp64(const float* f, float* u0, int32_t H, int32_t W, int32_t pitch, const deblur_psf* psf,
                       double K, float pos_floor, void* ws, size_t ws_bytes, void* stream)
{
    return wiener_impl(f, u0, H, W, pitch, psf, K, pos_floor, ws, ws_bytes, true, stream);
}

int deblur_rrrl_start(const float* f, float* u0, int32_t H, int32_t W, int32_t pitch, int32_t mode,
                      float pos_floor, void* stream)
{
    if (!f || !u0) return DEBLUR_EINVAL;
    int s = check_image(H, W, pitch);
    if (s) return s;
    if (mode != DEBLUR_START_FLAT && mode != DEBLUR_START_OBSERVED) return DEBLUR_EINVAL;
    if (!(pos_floor > 0.0f) || !std::isfinite(pos_floor)) return DEBLUR_EINVAL;
    const size_t img = (size_t)H * pitch * sizeof(float);
    if (overlaps(f, img, u0, img)) return DEBLUR_EINVAL;
    return launch_rrrl_start(f, u0, H, W, pitch, mode, pos_floor, reinterpret_cast<hipStream_t>(stream)) == 0
               ? DEBLUR_OK
               : DEBLUR_EDEVICE;
}

int deblur_rrrl_iterate(const float* f, const float* u_in, float* u_out, int32_t H, int32_t W, int32_t pitch,
                        const deblur_psf* psf, const deblur_params* p, float* ckpt, void* ws, size_t ws_bytes,
                        void* stream)
{
    return iterate_impl(f, u_in, u_out, H, W, pitch, psf, p, ckpt, ws, ws_bytes, false, stream);
}

int deblur_rrrl_iterate_noalloc(const float* f, const float* u_in, float* u_out, int32_t H, int32_t W,
                                int32_t pitch, const deblur_psf* psf, const deblur_params* p, float* ckpt,
                                void* stream)
{
    // the lookup mode would allocate its table on first use
    if (p && p->rf_lut) return DEBLUR_EUNSUPPORTED;
    return iterate_impl(f, u_in, u_out, H, W, pitch, psf, p, ckpt, nullptr, 0, true, stream);
}

int deblur_rrrl_backward(const float* f, const float* ckpt, const float* grad_uK, int32_t H, int32_t W,
                         int32_t pitch, const deblur_psf* psf, const deblur_params* p, int32_t through_wiener,
                         double K, float pos_floor, float* grad_f, float* grad_taps, float* grad_alpha,
                         float* grad_u0, void* ws, size_t ws_bytes, void* stream)
{
    PsfDev d;
    if (!f || !grad_uK || !grad_f) return DEBLUR_EINVAL;
    if (through_wiener != 0 && through_wiener != 1) return DEBLUR_EINVAL;
    int s = check_backward(H, W, pitch, psf, p, through_wiener == 1, &d);
    if (s) return s;
    if (p->iters > 0 && !ckpt) return DEBLUR_EINVAL;
    if (through_wiener && (!(K > 0.0) || !std::isfinite(K) || !std::isfinite(pos_floor))) return DEBLUR_EINVAL;
    const size_t img = (size_t)H * pitch * sizeof(float);
    const size_t ck = img * (size_t)p->iters;
    if (overlaps(grad_f, img, f, img) || overlaps(grad_f, img, grad_uK, img) || (ckpt && overlaps(grad_f, img, ckpt, ck)))
        return DEBLUR_EINVAL;
    if (grad_u0 && (overlaps(grad_u0, img, grad_f, img) || overlaps(grad_u0, img, f, img) ||
                    overlaps(grad_u0, img, grad_uK, img) || (ckpt && overlaps(grad_u0, img, ckpt, ck))))
        return DEBLUR_EINVAL;
    const size_t need = backward_ws_bytes(H, W, d, through_wiener == 1);
    if (!ws || ws_bytes < need) return DEBLUR_EWORKSPACE;
    s = launch_rrrl_backward(f, ckpt, grad_uK, H, W, pitch, d, iter_params(p), p->iters, through_wiener == 1, K,
                             pos_floor, grad_f, grad_taps, grad_alpha, grad_u0, ws,
                             reinterpret_cast<hipStream_t>(stream));
    return s == 0 ? DEBLUR_OK : (s == -2 ? DEBLUR_EUNSUPPORTED : DEBLUR_EDEVICE);
}

namespace {

// Shared checks of the batched entry points: batch size, image stride and
// PSF stride (in floats).
int check_batch_common(int32_t B, int32_t H, int32_t pitch, const PsfDev& d, int64_t img_stride, int64_t taps_stride)
{
    if (B < 1 || B > 65535) return DEBLUR_EINVAL;
    if (img_stride < (int64_t)H * pitch || taps_stride < 0) return DEBLUR_EINVAL;
    if (d.kind == PSF_TAPS) {
        if (taps_stride != 0 && taps_stride < (int64_t)d.ph * d.pw) return DEBLUR_EINVAL;
    } else if (taps_stride != 0) {
        return DEBLUR_EINVAL;
    }
    return DEBLUR_OK;
}

// Validates the shared arguments of a backward batch; DEBLUR_OK or an error.
int check_backward_batch(int32_t B, int32_t H, int32_t W, int32_t pitch, const deblur_psf* psf,
                         const deblur_params* p, int32_t through_wiener, int64_t img_stride, int64_t ckpt_stride,
                         int64_t taps_stride, PsfDev* d)
{
    if (B < 1 || B > 65535) return DEBLUR_EINVAL;
    if (through_wiener != 0 && through_wiener != 1) return DEBLUR_EINVAL;
    int s = check_backward(H, W, pitch, psf, p, through_wiener == 1, d);
    if (s) return s;
    if ((s = check_batch_common(B, H, pitch, *d, img_stride, taps_stride))) return s;
    if (ckpt_stride < 0 || (p->iters > 0 && ckpt_stride < (int64_t)H * pitch * p->iters)) return DEBLUR_EINVAL;
    return DEBLUR_OK;
}

size_t round256(size_t n) { return (n + 255) & ~(size_t)255; }

}  // namespace

size_t deblur_workspace_bytes_batch(int32_t op, int32_t B, int32_t H, int32_t W, int32_t pitch,
                                    const deblur_psf* psf, const deblur_params* p)
{
    if (B < 1 || B > 65535) return 0;
    if (op == 1 && p && p->conv == DEBLUR_CONV_FFT) return 0;   // the Fourier-domain iteration has no batched form
    // one workspace per image, each starting on a 256-byte boundary
    const size_t one = deblur_workspace_bytes(op, H, W, pitch, psf, p);
    return one ? (size_t)B * round256(one) : 0;
}

int deblur_wiener_batch(int32_t B, const float* f, float* u0, int32_t H, int32_t W, int32_t pitch, int64_t img_stride,
                        const deblur_psf* psf, int64_t taps_stride, double K, float pos_floor, int32_t fp64,
                        void* ws, size_t ws_bytes, void* stream)
{
    PsfDev d;
    if (!f || !u0) return DEBLUR_EINVAL;
    if (fp64 != 0 && fp64 != 1) return DEBLUR_EINVAL;
    int s = check_wiener(H, W, pitch, psf, &d);
    if (s) return s;
    if ((s = check_batch_common(B, H, pitch, d, img_stride, taps_stride))) return s;
    if (!(K > 0.0) || !std::isfinite(K) || !(pos_floor > 0.0f) || !std::isfinite(pos_floor)) return DEBLUR_EINVAL;
    const size_t img = ((size_t)(B - 1) * img_stride + (size_t)H * pitch) * sizeof(float);
    if (overlaps(f, img, u0, img)) return DEBLUR_EINVAL;
    const size_t stride = round256(wiener_ws_bytes(H, W, wiener_rowwise(d), fp64 == 1));
    if (!ws || ws_bytes / B < stride) return DEBLUR_EWORKSPACE;
    return launch_wiener_z(B, f, u0, H, W, pitch, (size_t)img_stride * sizeof(float), d,
                           (size_t)taps_stride * sizeof(float), K, pos_floor, ws, stride, wiener_rowwise(d), fp64 == 1,
                           reinterpret_cast<hipStream_t>(stream)) == 0
               ? DEBLUR_OK
               : DEBLUR_EDEVICE;
}

int deblur_rrrl_iterate_batch(int32_t B, const float* f, const float* u_in, float* u_out, int32_t H, int32_t W,
                              int32_t pitch, int64_t img_stride, const deblur_psf* psf, int64_t taps_stride,
                              const float* alpha, const deblur_params* p, float* ckpt, int64_t ckpt_stride, void* ws,
                              size_t ws_bytes, void* stream)
{
    PsfDev d;
    if (!f || !u_in || !u_out) return DEBLUR_EINVAL;
    int s = check_iterate(H, W, pitch, psf, p, &d);
    if (s) return s;
    if (p->conv == DEBLUR_CONV_FFT) return DEBLUR_EUNSUPPORTED;
    if ((s = check_batch_common(B, H, pitch, d, img_stride, taps_stride))) return s;
    if (ckpt && (ckpt_stride < 0 || ckpt_stride < (int64_t)H * pitch * p->iters)) return DEBLUR_EINVAL;
    const size_t img = ((size_t)(B - 1) * img_stride + (size_t)H * pitch) * sizeof(float);
    if (overlaps(f, img, u_out, img) || (u_in != u_out && overlaps(u_in, img, u_out, img))) return DEBLUR_EINVAL;
    if (ckpt && p->iters > 0) {
        const size_t ck = ((size_t)(B - 1) * ckpt_stride + (size_t)p->iters * H * pitch) * sizeof(float);
        if (overlaps(ckpt, ck, f, img) || overlaps(ckpt, ck, u_in, img) || overlaps(ckpt, ck, u_out, img))
            return DEBLUR_EINVAL;
    }
    const bool box = use_box(d, p);
    const size_t stride = round256(iterate_ws_bytes(H, W, pitch, d, box));
    if (!ws || ws_bytes / B < stride) return DEBLUR_EWORKSPACE;
    s = launch_rrrl_iterate_batch(B, f, u_in, u_out, H, W, pitch, (size_t)img_stride * sizeof(float), d,
                                  (size_t)taps_stride * sizeof(float), alpha, iter_params(p), p->iters, ckpt,
                                  ckpt ? (size_t)ckpt_stride * sizeof(float) : 0, box, ws, stride,
                                  reinterpret_cast<hipStream_t>(stream));
    return s == 0 ? DEBLUR_OK : (s == -2 ? DEBLUR_EUNSUPPORTED : DEBLUR_EDEVICE);
}

int deblur_rrrl_backward_batch(int32_t B, const float* f, const float* ckpt, const float* grad_uK, int32_t H,
                               int32_t W, int32_t pitch, int64_t img_stride, int64_t ckpt_stride,
                               const deblur_psf* psf, int64_t taps_stride, const float* alpha,
                               const deblur_params* p, int32_t through_wiener, double K, float pos_floor,
                               float* grad_f, float* grad_taps, float* grad_alpha, float* grad_u0, void* ws,
                               size_t ws_bytes, void* stream)
{
    PsfDev d;
    if (!f || !grad_uK || !grad_f) return DEBLUR_EINVAL;
    int s = check_backward_batch(B, H, W, pitch, psf, p, through_wiener, img_stride, ckpt_stride, taps_stride, &d);
    if (s) return s;
    if (p->iters > 0 && !ckpt) return DEBLUR_EINVAL;
    if (through_wiener && (!(K > 0.0) || !std::isfinite(K) || !std::isfinite(pos_floor))) return DEBLUR_EINVAL;
    // extents over the whole batch
    const size_t img = ((size_t)(B - 1) * img_stride + (size_t)H * pitch) * sizeof(float);
    const size_t ck = p->iters > 0 ? ((size_t)(B - 1) * ckpt_stride + (size_t)p->iters * H * pitch) * sizeof(float) : 0;
    if (overlaps(grad_f, img, f, img) || overlaps(grad_f, img, grad_uK, img) || (ckpt && overlaps(grad_f, img, ckpt, ck)))
        return DEBLUR_EINVAL;
    if (grad_u0 && (overlaps(grad_u0, img, grad_f, img) || overlaps(grad_u0, img, f, img) ||
                    overlaps(grad_u0, img, grad_uK, img) || (ckpt && overlaps(grad_u0, img, ckpt, ck))))
        return DEBLUR_EINVAL;
    const size_t stride = backward_batch_stride(H, W, d, through_wiener == 1);
    if (!ws || ws_bytes / B < stride) return DEBLUR_EWORKSPACE;
    s = launch_rrrl_backward_batch(B, f, ckpt, grad_uK, H, W, pitch, (size_t)img_stride * sizeof(float),
                                   (size_t)ckpt_stride * sizeof(float), d, (size_t)taps_stride * sizeof(float), alpha,
                                   iter_params(p), p->iters, through_wiener == 1, K, pos_floor, grad_f, grad_taps,
                                   grad_alpha, grad_u0, ws, stride, reinterpret_cast<hipStream_t>(stream));
    return s == 0 ? DEBLUR_OK : (s == -2 ? DEBLUR_EUNSUPPORTED : DEBLUR_EDEVICE);
}

int deblur_batch_plan_create(const deblur_batch_item* items, int32_t n, int32_t group_size,
                             deblur_batch_plan** plan)
{
    return deblur_batch_plan_create_tiled(items, n, group_size, nullptr, plan);
}

int32_t deblur_batch_tile_variants(int32_t family)
{
    return family == DEBLUR_BATCH_STENCIL || family == DEBLUR_BATCH_BOX ? batch_num_variants(family) : 0;
}

int deblur_batch_plan_create_tiled(const deblur_batch_item* items, int32_t n, int32_t group_size,
                                   const int32_t* tiles, deblur_batch_plan** plan)
{
    if (!items || n < 1 || !plan || group_size < 0) return DEBLUR_EINVAL;
    *plan = nullptr;
    int t5[DEBLUR_BATCH_NTILES] = {0, 0, 0, 0, 0};
    if (tiles) {
        for (int k = 0; k < DEBLUR_BATCH_NTILES; ++k) {
            const int lim = batch_num_variants(k == 0 ? DEBLUR_BATCH_STENCIL : DEBLUR_BATCH_BOX);
            if (tiles[k] < 0 || tiles[k] > lim) return DEBLUR_EINVAL;
            t5[k] = tiles[k];
        }
    }
    std::vector<BatchItemDev> dev(n);
    for (int i = 0; i < n; ++i) {
        const deblur_batch_item& it = items[i];
        PsfDev d;
        if (!it.f || !it.u) return DEBLUR_EINVAL;
        int s = check_wiener(it.H, it.W, it.pitch, &it.psf, &d);
        if (s) return s;
        if ((s = check_iterate(it.H, it.W, it.pitch, &it.psf, &it.p, &d))) return s;
        if (!(it.K > 0.0) || !std::isfinite(it.K) || !(it.pos_floor > 0.0f) || !std::isfinite(it.pos_floor))
            return DEBLUR_EINVAL;
        if (it.p.iters != items[0].p.iters) return DEBLUR_EINVAL;
        if (it.p.conv == DEBLUR_CONV_FFT) return DEBLUR_EUNSUPPORTED;   // plans run the direct paths only
        const size_t img = (size_t)it.H * it.pitch * sizeof(float);
        if (overlaps(it.f, img, it.u, img)) return DEBLUR_EINVAL;
        BatchItemDev& b = dev[i];
        b.f = it.f;
        b.u = it.u;
        b.H = it.H;
        b.W = it.W;
        b.pitch = it.pitch;
        b.psf = d;
        b.p = iter_params(&it.p);
        b.iters = it.p.iters;
        b.K = it.K;
        b.pos_floor = it.pos_floor;
        b.stencil = it.p.conv == DEBLUR_CONV_STENCIL;
    }
    BatchPlan* impl = nullptr;
    const int s = batch_plan_create(dev.data(), n, group_size, t5, &impl);
    if (s) return s == -3 ? DEBLUR_EWORKSPACE : DEBLUR_EDEVICE;
    *plan = new deblur_batch_plan{impl};
    return DEBLUR_OK;
}

int deblur_batch_run(deblur_batch_plan* plan, void* stream)
{
    if (!plan) return DEBLUR_EINVAL;
    return batch_run(plan->impl, reinterpret_cast<hipStream_t>(stream)) == 0 ? DEBLUR_OK : DEBLUR_EDEVICE;
}

int32_t deblur_batch_size(const deblur_batch_plan* plan) { return plan ? batch_size(plan->impl) : 0; }

int32_t deblur_batch_class_of(const deblur_batch_plan* plan, int32_t image)
{
    if (!plan || image < 0 || image >= batch_size(plan->impl)) return DEBLUR_EINVAL;
    return batch_class_of(plan->impl, image);
}

int32_t deblur_batch_class_tiles(const deblur_batch_plan* plan, int32_t cls)
{
    if (!plan || cls < 0 || cls >= DEBLUR_BATCH_NCLASS) return DEBLUR_EINVAL;
    return batch_class_tiles(plan->impl, cls);
}

int deblur_batch_launch_class(deblur_batch_plan* plan, int32_t cls, int32_t stage, void* stream)
{
    if (!plan || cls < 0 || cls >= DEBLUR_BATCH_NCLASS) return DEBLUR_EINVAL;
    const int s = batch_launch_class(plan->impl, cls, stage, reinterpret_cast<hipStream_t>(stream));
    return s == 0 ? DEBLUR_OK : (s == -2 ? DEBLUR_EINVAL : DEBLUR_EDEVICE);
}

int deblur_batch_latencies(deblur_batch_plan* plan, double* us_out)
{
    if (!plan || !us_out) return DEBLUR_EINVAL;
    return batch_latencies(plan->impl, us_out) == 0 ? DEBLUR_OK : DEBLUR_EDEVICE;
}

void deblur_batch_plan_destroy(deblur_batch_plan* plan)
{
    if (!plan) return;
    batch_plan_destroy(plan->impl);
    delete plan;
}

size_t deblur_taps_bytes(const deblur_psf* psf)
{
    PsfDev d;
    if (convert_psf(psf, &d)) return 0;
    return tap_list_bytes(d);
}

int deblur_compile_taps(const deblur_psf* psf, void* taps_out, size_t taps_bytes, void* stream)
{
    PsfDev d;
    int s = convert_psf(psf, &d);
    if (s) return s;
    if (!taps_out || taps_bytes < tap_list_bytes(d)) return DEBLUR_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(taps_out) % 256 != 0) return DEBLUR_EINVAL;
    launch_compile_taps(d, taps_out, reinterpret_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? DEBLUR_OK : DEBLUR_EDEVICE;
}

int deblur_rrrl_weights(const float* f, const float* u, float* qw, int32_t H, int32_t W, int32_t pitch,
                        const deblur_psf* psf, const void* taps, const deblur_params* p, void* stream)
{
    PsfDev d;
    if (!f || !u || !qw || !taps) return DEBLUR_EINVAL;
    int s = check_iterate(H, W, pitch, psf, p, &d);
    if (s) return s;
    const size_t img = (size_t)H * pitch * sizeof(float), q = (size_t)H * W * 2 * sizeof(float);
    if (overlaps(qw, q, f, img) || overlaps(qw, q, u, img)) return DEBLUR_EINVAL;
    s = launch_taps_stage1(f, u, qw, H, W, pitch, d, taps, iter_params(p), p->tile,
                           reinterpret_cast<hipStream_t>(stream));
    if (s) return DEBLUR_EUNSUPPORTED;
    return hipGetLastError() == hipSuccess ? DEBLUR_OK : DEBLUR_EDEVICE;
}

int deblur_rrrl_update(const float* qw, const float* u, float* u_out, float* u_copy, int32_t H, int32_t W,
                       int32_t pitch, const deblur_psf* psf, const void* taps, const deblur_params* p,
                       void* stream)
{
    PsfDev d;
    if (!qw || !u || !u_out || !taps) return DEBLUR_EINVAL;
    int s = check_iterate(H, W, pitch, psf, p, &d);
    if (s) return s;
    const size_t img = (size_t)H * pitch * sizeof(float), q = (size_t)H * W * 2 * sizeof(float);
    if (overlaps(u, img, u_out, img) || overlaps(qw, q, u_out, img)) return DEBLUR_EINVAL;
    if (u_copy && (overlaps(u_copy, img, u, img) || overlaps(u_copy, img, u_out, img) || overlaps(u_copy, img, qw, q)))
        return DEBLUR_EINVAL;
    s = launch_taps_stage2(qw, u, u_out, u_copy, H, W, pitch, d, taps, iter_params(p), p->tile,
                           reinterpret_cast<hipStream_t>(stream));
    if (s) return DEBLUR_EUNSUPPORTED;
    return hipGetLastError() == hipSuccess ? DEBLUR_OK : DEBLUR_EDEVICE;
}

}  // extern "C"
