// Host-side launchers of the gfx950 kernels, called by the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "psf.hpp"

namespace deblur {

// Per-iteration constants of the RRRL update (squares of the penaliser
// epsilons are precomputed).
struct IterParams {
    float alpha, eps_d2, eps_t2, s_min;
    int robust, bc;
    int tile;  // tile-shape variant (0 = default)
    int bwd_tile;   // backward tile rows variant (0 = default)
    int psi;   // regulariser: 0 regularised TV, 1 Perona-Malik (lambda^2 = eps_t2)
    const float* r1_lut;   // device table of r_1 (lookup mode of r_f), or null: exact r_f
};

// Image z of an iteration launch over a batch of equally shaped images
// (blockIdx.z = image): byte strides from image 0 of f, of the iterate read
// (u), of the iterate written (un), of the checkpoints and of the workspace
// (tap lists, the (q, W) plane); alpha: the images' weights (device array;
// nullptr: the IterParams value).  All zero: one image.
struct IterZ {
    size_t f = 0, u = 0, un = 0, ck = 0, ws = 0;
    const float* alpha = nullptr;
};

// Lookup mode of the information divergence (Sec. 4.1): r_1(x) = x - 1 - ln x
// tabulated at x = k / RF_LUT_PER_UNIT, k = 1 .. RF_LUT_N (x up to 65), read
// with linear interpolation; r_f(s) = f r_1(s/f); beyond 65 the tangent of
// r_1 at 65; below the first sample the first sample.  Table layout:
// [0] unused (= [1]), [1..RF_LUT_N] samples, [RF_LUT_N + 1] the slope
// r_1'(65) = 1 - 1/65.
constexpr int RF_LUT_PER_UNIT = 64;
constexpr int RF_LUT_N = 65 * RF_LUT_PER_UNIT;
constexpr int RF_LUT_WORDS = RF_LUT_N + 2;

DEBLUR_DEV float rf_lookup(float f, float s, const float* __restrict__ lut)
{
    if (!(f > 0.0f)) return s;   // r_0(s) = s
    const float x = s * rcp(f);
    const float t = fminf(fmaxf(x * (float)RF_LUT_PER_UNIT, 1.0f), (float)RF_LUT_N);
    const int k = min((int)t, RF_LUT_N - 1);
    const float a = lut[k], b = lut[k + 1];
    float r1 = fmaf(t - (float)k, b - a, a);
    if (x > 65.0f) r1 = fmaf(x - 65.0f, lut[RF_LUT_N + 1], lut[RF_LUT_N]);
    return f * r1;
}

// r_f(s) (eq. (7)) as the iteration's data weight uses it: exact, or the
// lookup mode.
DEBLUR_DEV float rf_eval(float f, float s, const IterParams& p)
{
    return p.r1_lut ? rf_lookup(f, s, global_ptr(p.r1_lut)) : info_div(f, s);
}

// Diffusivity g = 2 Psi'(z), z = |grad u|^2, in the scaling of the data
// weight (the factor 1/2 cancels in the quotient of eq. (9)): regularised TV
// (z + eps^2)^(-1/2), or the non-convex Perona-Malik penaliser
// (Sec. 2.3) lambda^2 / (lambda^2 + z).
DEBLUR_DEV float tv_diffusivity(float z, const IterParams& p)
{
    return p.psi ? p.eps_t2 * rcp(p.eps_t2 + z) : pen_deriv(z, p.eps_t2);
}

// -2 dg/dz through g (backward): g^3 (TV) or 2 g^2 / lambda^2 (Perona-Malik).
DEBLUR_DEV float tv_slope(float g, const IterParams& p)
{
    return p.psi ? 2.0f * g * g * rcp(p.eps_t2) : g * g * g;
}

// Compiled PSF ("tap list" buffer), built on the device by launch_compile_taps:
//   bytes [0, 256)        header: int count of non-zero taps T, int count of
//                         column groups G, counts of groups of length 1..8,
//                         int count of packed words (G + T)
//   bytes [256, ...)      non-zero taps {dy, dx, weight bits, 0}, row-major
//   bytes [groups_off..)  column groups: runs of up to 8 vertically adjacent
//                         non-zero taps of one PSF column, ordered by length
//                         (longest first), then column, then row
//   bytes [packed_off..)  the same groups packed for the stencil kernels:
//                         per group one word (dx & 0xffff) | (dy0 << 16),
//                         then its S weights
struct TapGroup {
    int dx, dy0, S, pad;  // taps (dy0 + s, dx), s < S
    float w[8];
};
static_assert(sizeof(TapGroup) == 48, "three 16-byte words per group");
constexpr int TAP_GROUP_MAX = 8;
inline size_t tap_groups_offset(int ph, int pw) { return 256 + 16 * (size_t)ph * pw; }
inline size_t tap_packed_offset(int ph, int pw) { return tap_groups_offset(ph, pw) + 48 * (size_t)ph * pw; }

// Wiener step; fp64: M, spectra and transforms in FP64 (output rounded once).
size_t wiener_ws_bytes(int H, int W, bool rowwise, bool fp64 = false);
// Raises the LDS limit of the Wiener kernels (once per process; a plan calls
// it before capturing a graph).
void prepare_wiener_kernels();
// One image's Wiener step in a batched launch: input, output (H x pitch),
// PSF, K, positivity floor and its own workspace (wiener_ws_bytes, FP32).
struct WienerJob {
    const float* f;
    float* u;
    int pitch;
    float pos_floor;
    double K;
    PsfDev psf;
    void* ws;
};
int launch_wiener_batch(const WienerJob* jobs, int n, int H, int W, bool rowwise, hipStream_t st);
int launch_wiener(const float* f, float* u, int H, int W, int pitch, const PsfDev& psf, double K,
                  float pos_floor, void* ws, bool rowwise, bool fp64, hipStream_t st);
// The Wiener step of B images of one size at once (blockIdx.z = image):
// image z's f and u0 at z img_stride bytes, its PSF taps at z taps_stride
// bytes (0: shared), its workspace of wiener_ws_bytes at z ws_stride bytes.
int launch_wiener_z(int B, const float* f, float* u, int H, int W, int pitch, size_t img_stride, const PsfDev& psf,
                    size_t taps_stride, double K, float pos_floor, void* ws, size_t ws_stride, bool rowwise, bool fp64,
                    hipStream_t st);

// A launch over n images of one shape at once (blockIdx.z = image): image z's
// planes are the first image's advanced by z times the byte strides s0, s1,
// s2 of the pointer arguments in order (0: shared by all images).
struct ZBatch {
    int n = 1;
    size_t s0 = 0, s1 = 0, s2 = 0;
};

// 2D transform building blocks on half spectra H x (W/2+1) (complex64); the
// ZBatch strides follow the pointer arguments (for the multiplier: the PSF
// taps, M, h^).
void launch_wiener_mult(const PsfDev& psf, int H, int W, double K, float2* M, float2* hh, hipStream_t st,
                        ZBatch zb = {});
void launch_fft2_forward(const float* x, int pitch, int H, int W, float2* S, hipStream_t st, ZBatch zb = {});
void launch_fft2_inverse(float2* S, int H, int W, float* out, int pitch, float floor_, bool accumulate,
                         hipStream_t st, ZBatch zb = {});
void launch_rows_fwd(const float* x, int pitch, int H, int W, float2* S, hipStream_t st);
void launch_cols(float2* S, const float2* mult, bool conj_mult, int mode, int H, int W, hipStream_t st);
int fft_row_batch(int W);
void launch_spectral_mul(const float2* Sin, const float2* M, bool conjM, float2* Sout, size_t n, hipStream_t st,
                         ZBatch zb = {});
// (one stride, s0, for all four spectra)
void launch_wiener_dh_prep(const float2* Fh, const float2* Gh, const float2* hh, float2* Y, size_t n, double K,
                           hipStream_t st, ZBatch zb = {});

int tap_radius_class(int rad);
size_t tap_list_bytes(const PsfDev& psf);
// (ZBatch: n PSFs; strides of the taps and of the lists)
void launch_compile_taps(const PsfDev& psf, void* list, hipStream_t st, ZBatch zb = {});
// `variant`: 0 = default tile shape for the image size, 1..taps_num_variants()
// = an explicit tile shape (all give bitwise-identical results).
int taps_num_variants();
// (B images at once with the strides of z; the default tile shape then goes
// by the tiles of the whole batch)
int launch_taps_stage1(const float* f, const float* u, float* qw, int H, int W, int pitch, const PsfDev& psf,
                       const void* list, const IterParams& p, int variant, hipStream_t st, float* s_out = nullptr,
                       int B = 1, const IterZ& z = IterZ{});
int launch_taps_stage2(const float* qw, const float* u, float* un, float* ckpt, int H, int W, int pitch,
                       const PsfDev& psf, const void* list, const IterParams& p, int variant, hipStream_t st,
                       int B = 1, const IterZ& z = IterZ{});

// One fused RRRL iteration for a box PSF of length L along x (vert = false)
// or y (vert = true).
// Starting image of RRRL without the Wiener step: mode 0 flat (mean of f),
// 1 the observed image; both floored at pos_floor.
int launch_rrrl_start(const float* f, float* u0, int H, int W, int pitch, int mode, float pos_floor, hipStream_t st);

// Box tile shapes: count of explicit variants (deblur_params.tile for the
// running-sum path) and the default for an image.
int box_num_variants();
int backward_tile_variants();
int box_default_variant(int H, int W, bool vert);
int launch_rrrl_box_iter(const float* f, const float* u, float* un, float* ckpt, int H, int W, int pitch, int L,
                         float frac, bool vert, const IterParams& p, hipStream_t st, int B = 1,
                         const IterZ& z = IterZ{});

// Iteration driver: `iters` iterations u_in -> u_out with ping-pong buffers
// in the workspace; box kinds use the fused running-sum kernel when use_box.
size_t iterate_ws_bytes(int H, int W, int pitch, const PsfDev& psf, bool use_box);
int launch_rrrl_iterate(const float* f, const float* u_in, float* u_out, int H, int W, int pitch,
                        const PsfDev& psf, const IterParams& p, int iters, float* ckpt, bool use_box, void* ws,
                        hipStream_t st);
// B images of one size at once: image z's f, u_in, u_out at z img_stride
// bytes, its checkpoints at z ck_stride, its PSF taps at z taps_stride (0:
// shared), its workspace (iterate_ws_bytes) at z ws_stride; alpha: device
// array of the images' weights or nullptr for p.alpha.
int launch_rrrl_iterate_batch(int B, const float* f, const float* u_in, float* u_out, int H, int W, int pitch,
                              size_t img_stride, const PsfDev& psf, size_t taps_stride, const float* alpha,
                              const IterParams& p, int iters, float* ckpt, size_t ck_stride, bool use_box, void* ws,
                              size_t ws_stride, hipStream_t st);

// Backward through WR3L (iterations from checkpoints, optionally the Wiener
// initialisation).
size_t backward_ws_bytes(int H, int W, const PsfDev& psf, bool through_wiener);
// The same for B images of one size and PSF box at once (blockIdx.z = image):
// image z's planes at the first image's plus z times the byte strides
// (img_stride: f, grad_uK, grad_f, grad_u0; ck_stride: checkpoints;
// taps_stride: PSF taps; ws_stride: workspaces of backward_batch_stride bytes;
// grad_taps + z ph pw, grad_alpha + z); alpha: device array of the images'
// weights, or nullptr for p.alpha.
size_t backward_batch_stride(int H, int W, const PsfDev& psf, bool through_wiener);
int launch_rrrl_backward_batch(int B, const float* f, const float* ckpt, const float* grad_uK, int H, int W,
                               int pitch, size_t img_stride, size_t ck_stride, const PsfDev& psf, size_t taps_stride,
                               const float* alpha, const IterParams& p, int iters, bool through_wiener, double K,
                               float pos_floor, float* grad_f, float* grad_taps, float* grad_alpha, float* grad_u0,
                               void* ws, size_t ws_stride, hipStream_t st);
int launch_rrrl_backward(const float* f, const float* ckpt, const float* grad_uK, int H, int W, int pitch,
                         const PsfDev& psf, const IterParams& p, int iters, bool through_wiener, double K,
                         float pos_floor, float* grad_f, float* grad_taps, float* grad_alpha, float* grad_u0,
                         void* ws, hipStream_t st);

// Fourier-domain RRRL iterations (periodic continuation), rrrl_fft.hip
size_t fft_iter_ws_bytes(int H, int W, int pitch);
int launch_rrrl_fft(const float* f, const float* u_in, float* u_out, int H, int W, int pitch, const PsfDev& psf,
                    const IterParams& p, int iters, float* ckpt, void* ws, hipStream_t st);

// Static scratch of the no-allocation iterate entry point (noalloc.hip): its
// size, and the device address of the calling device's copy (looked up once
// per device; nullptr and *err set on failure).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
void* noalloc_scratch(hipError_t* err);

// Batched plans (batch.hip)
struct BatchPlan;
struct BatchItemDev {
    const float* f;
    float* u;
    int H, W, pitch;
    PsfDev psf;
    IterParams p;
    int iters;
    double K;
    float pos_floor;
    bool stencil;  // run a box PSF through the stencil classes
};

int batch_plan_create(const BatchItemDev* items, int n, int group_size, const int* tiles, BatchPlan** out);
int batch_class_of(const BatchPlan* P, int img);
int batch_class_tiles(const BatchPlan* P, int cls);
int batch_launch_class(const BatchPlan* P, int cls, int stage, hipStream_t st);
int batch_num_variants(int family);
int batch_run(BatchPlan* P, hipStream_t st);
int batch_latencies(BatchPlan* P, double* us);
int batch_size(const BatchPlan* P);
void batch_plan_destroy(BatchPlan* P);

}  // namespace deblur
