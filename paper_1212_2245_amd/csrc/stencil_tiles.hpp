// Per-tile bodies of the two RRRL stages for general PSFs (spatial stencil on
// LDS tiles), shared by the single-image and the batched launches.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace deblur {

// One column group applied to R consecutive output rows of one column.
// A (blur, E(u)(x - d)): p points at tile row (first output row - dy0 - S + 1),
// column (x - dx); v[k] = p[k LW] serves output i, tap s at k = i + S - 1 - s.
template <int R, int S, int LW>
DEBLUR_DEV void group_fma_a(const float* __restrict__ p, const float* w, float (&acc)[R])
{
    float v[R + S - 1];
#pragma unroll
    for (int k = 0; k < R + S - 1; ++k) v[k] = p[k * LW];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int i = 0; i < R; ++i) acc[i] = fmaf(w[s], v[i + S - 1 - s], acc[i]);
}

// B (correlation, E(q, W)(x + d)) on the two-channel tile: p points at tile
// row (first output row + dy0), column (x + dx); output i, tap s at k = i + s.
template <int R, int S, int LW>
DEBLUR_DEV void group_fma_b(const float2* __restrict__ p, const float* w, float (&n1)[R], float (&n2)[R])
{
    float2 v[R + S - 1];
#pragma unroll
    for (int k = 0; k < R + S - 1; ++k) v[k] = p[k * LW];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int i = 0; i < R; ++i) {
            n1[i] = fmaf(w[s], v[i + s].x, n1[i]);
            n2[i] = fmaf(w[s], v[i + s].y, n2[i]);
        }
}

// Sum over all column groups, in list order (column-major, dy ascending
// within a column): the order is the same for every tile shape, so the
// result of a pixel does not depend on the tiling.  The descriptor of the
// next group is fetched while the current one is processed.
template <int R, int LW>
DEBLUR_DEV void blur_groups(const float* __restrict__ base, const TapGroup* __restrict__ grp, int ng,
                            float (&acc)[R])
{
    TapGroup cur = grp[0];
    for (int g = 0; g < ng; ++g) {
        const TapGroup nxt = grp[g + 1 < ng ? g + 1 : g];
        const float* p = base - (cur.dy0 + cur.S - 1) * LW - cur.dx;
        switch (cur.S) {
            case 1: group_fma_a<R, 1, LW>(p, cur.w, acc); break;
            case 2: group_fma_a<R, 2, LW>(p, cur.w, acc); break;
            case 3: group_fma_a<R, 3, LW>(p, cur.w, acc); break;
            case 4: group_fma_a<R, 4, LW>(p, cur.w, acc); break;
            case 5: group_fma_a<R, 5, LW>(p, cur.w, acc); break;
            case 6: group_fma_a<R, 6, LW>(p, cur.w, acc); break;
            case 7: group_fma_a<R, 7, LW>(p, cur.w, acc); break;
            case 8: group_fma_a<R, 8, LW>(p, cur.w, acc); break;
            default: break;
        }
        cur = nxt;
    }
}

template <int R, int LW>
DEBLUR_DEV void corr_groups(const float2* __restrict__ base, const TapGroup* __restrict__ grp, int ng,
                            float (&n1)[R], float (&n2)[R])
{
    TapGroup cur = grp[0];
    for (int g = 0; g < ng; ++g) {
        const TapGroup nxt = grp[g + 1 < ng ? g + 1 : g];
        const float2* p = base + cur.dy0 * LW + cur.dx;
        switch (cur.S) {
            case 1: group_fma_b<R, 1, LW>(p, cur.w, n1, n2); break;
            case 2: group_fma_b<R, 2, LW>(p, cur.w, n1, n2); break;
            case 3: group_fma_b<R, 3, LW>(p, cur.w, n1, n2); break;
            case 4: group_fma_b<R, 4, LW>(p, cur.w, n1, n2); break;
            case 5: group_fma_b<R, 5, LW>(p, cur.w, n1, n2); break;
            case 6: group_fma_b<R, 6, LW>(p, cur.w, n1, n2); break;
            case 7: group_fma_b<R, 7, LW>(p, cur.w, n1, n2); break;
            case 8: group_fma_b<R, 8, LW>(p, cur.w, n1, n2); break;
            default: break;
        }
        cur = nxt;
    }
}

template <int RAD, int TH>
constexpr int stage1_lds_floats() { return (TH + 2 * RAD) * (64 + 2 * RAD); }

// Stage 1 on the tile with top-left output (x0, y0): tile = LDS scratch of
// stage1_lds_floats() floats.
template <int RAD, int TH, int NT>
DEBLUR_DEV void stage1_tile(float* __restrict__ tile, const float* __restrict__ u, const float* __restrict__ f,
                            float2* __restrict__ qw, float* __restrict__ s_out, int H, int W, int pitch, int x0,
                            int y0, const TapGroup* __restrict__ grp, int ng, const IterParams& p)
{
    // With s_out (the backward recompute) the pair written is (e, W) with
    // e = q - W = W (f - s) / s, formed without cancellation, instead of (q, W).
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
    blur_groups<R, LW>(tile + (ty * R + RAD) * LW + tx + RAD, grp, ng, acc);   // A: E(u)(x - d)
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
        const float fp = fmaxf(fv, 0.0f);
        const float q = s_out ? wt * (fp - s) / s : wt * fp / s;
        qw[(size_t)y * W + x] = make_float2(q, wt);
    }
}

template <int RAD, int TH, int NT>
__global__ void __launch_bounds__(NT) rrrl_taps_stage1(const float* __restrict__ u, const float* __restrict__ f,
                                                       float2* __restrict__ qw, float* __restrict__ s_out, int H,
                                                       int W, int pitch, const TapGroup* __restrict__ grp,
                                                       const int* __restrict__ hdr, IterParams p)
{
    __shared__ float tile[stage1_lds_floats<RAD, TH>()];
    stage1_tile<RAD, TH, NT>(tile, u, f, qw, s_out, H, W, pitch, blockIdx.x * 64, blockIdx.y * TH, grp, hdr[1], p);
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
                            int y0, const TapGroup* __restrict__ grp, int ng, const IterParams& p)
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
    corr_groups<R, LW>(qt + (ty * R + RAD) * LW + tx + RAD, grp, ng, n1, n2);   // B: E(q, W)(x + d)
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
                                                       int H, int W, int pitch, const TapGroup* __restrict__ grp,
                                                       const int* __restrict__ hdr, IterParams p)
{
    __shared__ Stage2Smem<RAD, TH> sm;
    stage2_tile<RAD, TH, NT>(sm, qw, u, u_next, ckpt, H, W, pitch, blockIdx.x * 64, blockIdx.y * TH, grp, hdr[1],
                             p);
}

}  // namespace deblur
