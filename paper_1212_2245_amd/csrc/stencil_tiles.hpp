// Per-tile bodies of the two RRRL stages for general PSFs (spatial stencil on
// LDS tiles), shared by the single-image and the batched launches.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace deblur {

template <int RAD, int TH>
constexpr int stage1_lds_floats() { return (TH + 2 * RAD) * (64 + 2 * RAD); }

// Stage 1 on the tile with top-left output (x0, y0): tile = LDS scratch of
// stage1_lds_floats() floats.
template <int RAD, int TH, int NT>
DEBLUR_DEV void stage1_tile(float* __restrict__ tile, const float* __restrict__ u, const float* __restrict__ f,
                            float2* __restrict__ qw, float* __restrict__ s_out, int H, int W, int pitch, int x0,
                            int y0, const int4* __restrict__ taps, int n, const IterParams& p)
{
    constexpr int TW = 64, LW = TW + 2 * RAD, LH = TH + 2 * RAD, R = TH / (NT / 64);
    static_assert(R >= 1 && TH % (NT / 64) == 0, "rows per thread");
    const int tid = threadIdx.x;
    for (int idx = tid; idx < LH * LW; idx += NT) {
        const int ly = idx / LW, lx = idx - ly * LW;
        const int gy = ext_index(y0 - RAD + ly, H, p.bc), gx = ext_index(x0 - RAD + lx, W, p.bc);
        tile[idx] = u[(size_t)gy * pitch + gx];
    }
    __syncthreads();
    const int tx = tid & 63, ty = tid >> 6;
    float acc[R];
#pragma unroll
    for (int i = 0; i < R; ++i) acc[i] = 0.0f;
    const float* base = tile + (ty * R + RAD) * LW + tx + RAD;
    for (int t = 0; t < n; ++t) {
        const int4 e = taps[t];
        const float w = __int_as_float(e.z);
        const float* s = base - e.x * LW - e.y;   // A: E(u)(x - d)
#pragma unroll
        for (int i = 0; i < R; ++i) acc[i] = fmaf(w, s[i * LW], acc[i]);
    }
    const int x = x0 + tx;
    if (x >= W) return;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int y = y0 + ty * R + i;
        if (y >= H) break;
        if (s_out) s_out[(size_t)y * W + x] = acc[i];   // unclamped A u (backward pass)
        const float s = fmaxf(acc[i], p.s_min);
        const float fv = f[(size_t)y * pitch + x];
        const float wt = p.robust ? pen_deriv(fmaxf(info_div(fv, s), 0.0f), p.eps_d2) : 1.0f;
        const float q = wt * fmaxf(fv, 0.0f) / s;
        qw[(size_t)y * W + x] = make_float2(q, wt);
    }
}

template <int RAD, int TH, int NT>
__global__ void __launch_bounds__(NT) rrrl_taps_stage1(const float* __restrict__ u, const float* __restrict__ f,
                                                       float2* __restrict__ qw, float* __restrict__ s_out, int H,
                                                       int W, int pitch, const int4* __restrict__ taps,
                                                       const int* __restrict__ ntaps, IterParams p)
{
    __shared__ float tile[stage1_lds_floats<RAD, TH>()];
    stage1_tile<RAD, TH, NT>(tile, u, f, qw, s_out, H, W, pitch, blockIdx.x * 64, blockIdx.y * TH, taps, ntaps[0],
                             p);
}

template <int RAD, int TH>
struct Stage2Smem {
    float2 qt[(TH + 2 * RAD) * (64 + 2 * RAD)];
    float ut[(TH + 4) * (64 + 4)];
    float gt[(TH + 2) * (64 + 2)];
};

// Stage 2 on the tile with top-left output (x0, y0).
template <int RAD, int TH, int NT>
DEBLUR_DEV void stage2_tile(Stage2Smem<RAD, TH>& sm, const float2* __restrict__ qw, const float* __restrict__ u,
                            float* __restrict__ u_next, float* __restrict__ ckpt, int H, int W, int pitch, int x0,
                            int y0, const int4* __restrict__ taps, int n, const IterParams& p)
{
    constexpr int TW = 64, LW = TW + 2 * RAD, LH = TH + 2 * RAD, R = TH / (NT / 64);
    static_assert(R >= 1 && TH % (NT / 64) == 0, "rows per thread");
    constexpr int UW = TW + 4, UH = TH + 4, GW = TW + 2, GH = TH + 2;
    float2* __restrict__ qt = sm.qt;
    float* __restrict__ ut = sm.ut;
    float* __restrict__ gt = sm.gt;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < LH * LW; idx += NT) {
        const int ly = idx / LW, lx = idx - ly * LW;
        const int gy = ext_index(y0 - RAD + ly, H, p.bc), gx = ext_index(x0 - RAD + lx, W, p.bc);
        qt[idx] = qw[(size_t)gy * W + gx];
    }
    for (int idx = tid; idx < UH * UW; idx += NT) {
        const int ly = idx / UW, lx = idx - ly * UW;
        ut[idx] = u[(size_t)clampi(y0 - 2 + ly, H) * pitch + clampi(x0 - 2 + lx, W)];
    }
    __syncthreads();
    // diffusivity g = Psi'(|grad u|^2) by central differences at pixels
    for (int idx = tid; idx < GH * GW; idx += NT) {
        const int a = idx / GW, b = idx - a * GW;
        const float gx = 0.5f * (ut[(a + 1) * UW + b + 2] - ut[(a + 1) * UW + b]);
        const float gy = 0.5f * (ut[(a + 2) * UW + b + 1] - ut[a * UW + b + 1]);
        gt[idx] = pen_deriv(gx * gx + gy * gy, p.eps_t2);
    }
    const int tx = tid & 63, ty = tid >> 6;
    float n1[R], n2[R];
#pragma unroll
    for (int i = 0; i < R; ++i) n1[i] = n2[i] = 0.0f;
    const float2* base = qt + (ty * R + RAD) * LW + tx + RAD;
    for (int t = 0; t < n; ++t) {
        const int4 e = taps[t];
        const float w = __int_as_float(e.z);
        const float2* s = base + e.x * LW + e.y;   // B: E(q, W)(x + d)
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const float2 v = s[i * LW];
            n1[i] = fmaf(w, v.x, n1[i]);
            n2[i] = fmaf(w, v.y, n2[i]);
        }
    }
    __syncthreads();   // gt complete
    const int x = x0 + tx;
    if (x >= W) return;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int ry = ty * R + i;
        const int y = y0 + ry;
        if (y >= H) break;
        const int c = (ry + 2) * UW + tx + 2;
        const int cg = (ry + 1) * GW + tx + 1;
        const float up = ut[c], gp = gt[cg];
        // neighbours outside the image read the clamped value u_p: zero flux
        const float D = 0.5f * (gp + gt[cg - GW]) * (ut[c - UW] - up)
                      + 0.5f * (gp + gt[cg + GW]) * (ut[c + UW] - up)
                      + 0.5f * (gp + gt[cg - 1]) * (ut[c - 1] - up)
                      + 0.5f * (gp + gt[cg + 1]) * (ut[c + 1] - up);
        const float num = n1[i] + p.alpha * fmaxf(D, 0.0f);
        const float den = n2[i] - p.alpha * fminf(D, 0.0f);
        const size_t o = (size_t)y * pitch + x;
        if (ckpt) ckpt[o] = up;
        u_next[o] = up * num / den;
    }
}

template <int RAD, int TH, int NT>
__global__ void __launch_bounds__(NT) rrrl_taps_stage2(const float2* __restrict__ qw, const float* __restrict__ u,
                                                       float* __restrict__ u_next, float* __restrict__ ckpt,
                                                       int H, int W, int pitch, const int4* __restrict__ taps,
                                                       const int* __restrict__ ntaps, IterParams p)
{
    __shared__ Stage2Smem<RAD, TH> sm;
    stage2_tile<RAD, TH, NT>(sm, qw, u, u_next, ckpt, H, W, pitch, blockIdx.x * 64, blockIdx.y * TH, taps,
                             ntaps[0], p);
}

}  // namespace deblur
