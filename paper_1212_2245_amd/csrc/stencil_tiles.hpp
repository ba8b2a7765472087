// Per-tile bodies of the two RRRL stages for general PSFs (spatial stencil on
// LDS tiles), shared by the single-image and the batched launches.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace deblur {

// One column group applied to R consecutive output rows of one column.
// A (blur, E(u)(x - d)): p points at tile row (first output row - dy0 - S + 1),
// column (x - dx); v[k] = p[k LW] serves output i, tap s at k = i + S - 1 - s.
// Column groups of at least GROUP_PARTIAL taps are summed into a partial of
// their own that is then added to the pixel's total: a dense PSF's total then
// takes one rounded addition per group instead of one per tap (the 961 taps of
// a 31 x 31 PSF: 124 additions), which bounds its rounding error ~7x lower.
// Shorter groups (sparse line PSFs) accumulate directly.
constexpr int GROUP_PARTIAL = 4;

template <int R, int S, int LW>
DEBLUR_DEV void group_fma_a(const float* __restrict__ p, const float* w, float (&acc)[R])
{
    float v[R + S - 1];
#pragma unroll
    for (int k = 0; k < R + S - 1; ++k) v[k] = p[k * LW];
    if constexpr (S >= GROUP_PARTIAL) {
        float part[R];
#pragma unroll
        for (int i = 0; i < R; ++i) part[i] = w[0] * v[i + S - 1];
#pragma unroll
        for (int s = 1; s < S; ++s)
#pragma unroll
            for (int i = 0; i < R; ++i) part[i] = fmaf(w[s], v[i + S - 1 - s], part[i]);
#pragma unroll
        for (int i = 0; i < R; ++i) acc[i] += part[i];
    } else {
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int i = 0; i < R; ++i) acc[i] = fmaf(w[s], v[i + S - 1 - s], acc[i]);
    }
}

// B (correlation, E(q, W)(x + d)) on the two-channel tile: p points at tile
// row (first output row + dy0), column (x + dx); output i, tap s at k = i + s.
template <int R, int S, int LW>
DEBLUR_DEV void group_fma_b(const float2* __restrict__ p, const float* w, float (&n1)[R], float (&n2)[R])
{
    float2 v[R + S - 1];
#pragma unroll
    for (int k = 0; k < R + S - 1; ++k) v[k] = p[k * LW];
    if constexpr (S >= GROUP_PARTIAL) {
        float p1[R], p2[R];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            p1[i] = w[0] * v[i].x;
            p2[i] = w[0] * v[i].y;
        }
#pragma unroll
        for (int s = 1; s < S; ++s)
#pragma unroll
            for (int i = 0; i < R; ++i) {
                p1[i] = fmaf(w[s], v[i + s].x, p1[i]);
                p2[i] = fmaf(w[s], v[i + s].y, p2[i]);
            }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            n1[i] += p1[i];
            n2[i] += p2[i];
        }
    } else {
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int i = 0; i < R; ++i) {
                n1[i] = fmaf(w[s], v[i + s].x, n1[i]);
                n2[i] = fmaf(w[s], v[i + s].y, n2[i]);
            }
    }
}

// Sum over all column groups in list order (by run length, longest first,
// then column-major): the order is the same for every tile shape, so the
// result of a pixel does not depend on the tiling.  The groups are read in
// place from the compiled tap list (pk: per group one word (dx & 0xffff) |
// (dy0 << 16) and its S weights; the addresses are the same for every lane,
// so they are scalar loads and take no LDS); cnt[S - 1] = number of groups of
// length S.  Each length has its own loop (no per-group dispatch).
DEBLUR_DEV void unpack_offsets(const float* d, int& dx, int& dy0)
{
    const int h = __builtin_amdgcn_readfirstlane(__float_as_int(d[0]));
    dx = (int)(short)(h & 0xffff);
    dy0 = h >> 16;
}

template <int S, int R, int LW>
DEBLUR_DEV const float* blur_class(const float* __restrict__ base, const float* __restrict__ pk, int n,
                                   float (&acc)[R])
{
    for (int k = 0; k < n; ++k) {
        const float* d = pk + k * (S + 1);
        int dx, dy0;
        unpack_offsets(d, dx, dy0);
        float w[S];
#pragma unroll
        for (int s = 0; s < S; ++s) w[s] = d[1 + s];
        group_fma_a<R, S, LW>(base - (dy0 + S - 1) * LW - dx, w, acc);
    }
    return pk + n * (S + 1);
}

template <int S, int R, int LW>
DEBLUR_DEV const float* corr_class(const float2* __restrict__ base, const float* __restrict__ pk, int n,
                                   float (&n1)[R], float (&n2)[R])
{
    for (int k = 0; k < n; ++k) {
        const float* d = pk + k * (S + 1);
        int dx, dy0;
        unpack_offsets(d, dx, dy0);
        float w[S];
#pragma unroll
        for (int s = 0; s < S; ++s) w[s] = d[1 + s];
        group_fma_b<R, S, LW>(base + dy0 * LW + dx, w, n1, n2);
    }
    return pk + n * (S + 1);
}

// The per-thread tile address, hidden from constant folding: the compiler
// would otherwise fold the tile's LDS offset into the immediate offsets of the
// group loads, and re-materialise the large offsets with a VALU add for
// every paired LDS read inside the group loops.
template <typename T>
DEBLUR_DEV const T* opaque_lds(const T* p)
{
    using LT = __attribute__((address_space(3))) const T;
    LT* q = (LT*)p;
    asm("" : "+v"(q));
    return (const T*)q;
}

template <int R, int LW>
DEBLUR_DEV void blur_groups(const float* __restrict__ base, const float* __restrict__ pk, const int* cnt,
                            float (&acc)[R])
{
    base = opaque_lds(base);
    pk = blur_class<8, R, LW>(base, pk, cnt[7], acc);
    pk = blur_class<7, R, LW>(base, pk, cnt[6], acc);
    pk = blur_class<6, R, LW>(base, pk, cnt[5], acc);
    pk = blur_class<5, R, LW>(base, pk, cnt[4], acc);
    pk = blur_class<4, R, LW>(base, pk, cnt[3], acc);
    pk = blur_class<3, R, LW>(base, pk, cnt[2], acc);
    pk = blur_class<2, R, LW>(base, pk, cnt[1], acc);
    blur_class<1, R, LW>(base, pk, cnt[0], acc);
}

template <int R, int LW>
DEBLUR_DEV void corr_groups(const float2* __restrict__ base, const float* __restrict__ pk, const int* cnt,
                            float (&n1)[R], float (&n2)[R])
{
    base = opaque_lds(base);
    pk = corr_class<8, R, LW>(base, pk, cnt[7], n1, n2);
    pk = corr_class<7, R, LW>(base, pk, cnt[6], n1, n2);
    pk = corr_class<6, R, LW>(base, pk, cnt[5], n1, n2);
    pk = corr_class<5, R, LW>(base, pk, cnt[4], n1, n2);
    pk = corr_class<4, R, LW>(base, pk, cnt[3], n1, n2);
    pk = corr_class<3, R, LW>(base, pk, cnt[2], n1, n2);
    pk = corr_class<2, R, LW>(base, pk, cnt[1], n1, n2);
    corr_class<1, R, LW>(base, pk, cnt[0], n1, n2);
}

// The eight per-length group counts of a compiled PSF (registers, uniform).
DEBLUR_DEV void group_counts(const int* __restrict__ hdr, int (&cnt)[TAP_GROUP_MAX])
{
#pragma unroll
    for (int q = 0; q < TAP_GROUP_MAX; ++q) cnt[q] = hdr[2 + q];
}

// The forward stage tiles read a sparse PSF's packed groups in place (scalar
// loads) and stage a dense one's in LDS, where its many weights are read
// faster (31x31 Gaussian at 2048^2: 357-361 us per iteration from LDS,
// 395-402 us in place; the 31-pixel lines, about 100 words, gain in place).
constexpr int DIRECT_TAP_WORDS = 512;
template <int RAD>
constexpr int packed_words_max() { return 2 * (2 * RAD + 1) * (2 * RAD + 1); }

// Copies the packed groups (hdr[10] words at pkg) into LDS (at most pk's
// capacity for the radius class).
template <int RAD>
DEBLUR_DEV void stage_groups(float* __restrict__ pk, const float* __restrict__ pkg, const int* __restrict__ hdr)
{
    const int nw = min(hdr[10], packed_words_max<RAD>());
    stage_to_lds_n<4>(pk, nw, [&](int i) { return pkg[i]; });
}

// Generic form for one or two channels (T = float or float2), used by the
// adjoint stencils.  DIR = +1: out(z) = sum h(d) V(z + d) (taps visited as in
// B); DIR = -1: out(z) = sum h(d) V(z - d) (as in A).
DEBLUR_DEV void fma_t(float w, float v, float& a) { a = fmaf(w, v, a); }
DEBLUR_DEV void fma_t(float w, float2 v, float2& a)
{
    a.x = fmaf(w, v.x, a.x);
    a.y = fmaf(w, v.y, a.y);
}

template <int DIR, int S, int R, int LW, typename T>
DEBLUR_DEV const float* stencil_class(const T* __restrict__ base, const float* __restrict__ pk, int n, T (&acc)[R])
{
    for (int k = 0; k < n; ++k) {
        const float* d = pk + k * (S + 1);
        int dx, dy0;
        unpack_offsets(d, dx, dy0);
        float w[S];
#pragma unroll
        for (int s = 0; s < S; ++s) w[s] = d[1 + s];
        const T* p = DIR > 0 ? base + dy0 * LW + dx : base - (dy0 + S - 1) * LW - dx;
        T v[R + S - 1];
#pragma unroll
        for (int q = 0; q < R + S - 1; ++q) v[q] = p[q * LW];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int i = 0; i < R; ++i) fma_t(w[s], v[DIR > 0 ? i + s : i + S - 1 - s], acc[i]);
    }
    return pk + n * (S + 1);
}

template <int DIR, int R, int LW, typename T>
DEBLUR_DEV void stencil_groups(const T* __restrict__ base, const float* __restrict__ pk, const int* cnt, T (&acc)[R])
{
    base = opaque_lds(base);
    pk = stencil_class<DIR, 8, R, LW>(base, pk, cnt[7], acc);
    pk = stencil_class<DIR, 7, R, LW>(base, pk, cnt[6], acc);
    pk = stencil_class<DIR, 6, R, LW>(base, pk, cnt[5], acc);
    pk = stencil_class<DIR, 5, R, LW>(base, pk, cnt[4], acc);
    pk = stencil_class<DIR, 4, R, LW>(base, pk, cnt[3], acc);
    pk = stencil_class<DIR, 3, R, LW>(base, pk, cnt[2], acc);
    pk = stencil_class<DIR, 2, R, LW>(base, pk, cnt[1], acc);
    stencil_class<DIR, 1, R, LW>(base, pk, cnt[0], acc);
}

template <int RAD, int TH>
constexpr int stage1_lds_floats() { return (TH + 2 * RAD) * (64 + 2 * RAD); }

// Stage 1 on the tile with top-left output (x0, y0): tile = LDS scratch of
// stage1_lds_floats() floats.
template <int RAD, int TH, int NT>
DEBLUR_DEV void stage1_tile(float* __restrict__ tile, float* __restrict__ pk, const float* __restrict__ u,
                            const float* __restrict__ f, float2* __restrict__ qw, float* __restrict__ s_out, int H,
                            int W, int pitch, int x0, int y0, const float* __restrict__ pkg,
                            const int* __restrict__ hdr, const IterParams& p)
{
    // With s_out (the backward recompute) the pair written is (e, W) with
    // e = q - W = W (f - s) / s, formed without cancellation, instead of (q, W).
    constexpr int TW = 64, LW = TW + 2 * RAD, LH = TH + 2 * RAD, R = TH / (NT / 64);
    static_assert(R >= 1 && TH % (NT / 64) == 0, "rows per thread");
    const int tid = threadIdx.x;
    const int tx = tid & 63, ty = tid >> 6;
    const int x = x0 + tx;
    // f of the thread's pixels, fetched first so these loads are in flight
    // together with the tile's
    float fr[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int y = y0 + ty * R + i;
        fr[i] = (x < W && y < H) ? f[(size_t)y * pitch + x] : 0.0f;
    }
    int cnt[TAP_GROUP_MAX];
    group_counts(hdr, cnt);
    const bool direct = hdr[10] <= DIRECT_TAP_WORDS;   // uniform: taps in place or staged
    if (!direct) stage_groups<RAD>(pk, pkg, hdr);
    const bool inner = x0 >= RAD && y0 >= RAD && x0 + TW + RAD <= W && y0 + TH + RAD <= H;
    if (inner && pitch % 4 == 0 && ((uintptr_t)u & 15) == 0) {
        // rows start at x0 - RAD, a multiple of 4: 16-byte loads
        copy_rows_f4<NT, LH, LW>(tile, u + (size_t)(y0 - RAD) * pitch + (x0 - RAD), pitch);
    } else if (inner) {
        const float* src = u + (size_t)(y0 - RAD) * pitch + (x0 - RAD);
        stage_to_lds<NT, LH * LW>(tile, [&](int idx) {
            const int ly = idx / LW;
            return src[(size_t)ly * pitch + (idx - ly * LW)];
        });
    } else if (p.bc == BC_REPLICATE) {
        stage_to_lds<NT, LH * LW>(tile, [&](int idx) {
            const int ly = idx / LW, lx = idx - ly * LW;
            return u[(size_t)clampi(y0 - RAD + ly, H) * pitch + clampi(x0 - RAD + lx, W)];
        });
    } else {
        stage_to_lds<NT, LH * LW>(tile, [&](int idx) {
            const int ly = idx / LW, lx = idx - ly * LW;
            const int gy = ext_index(y0 - RAD + ly, H, BC_PERIODIC), gx = ext_index(x0 - RAD + lx, W, BC_PERIODIC);
            return u[(size_t)gy * pitch + gx];
        });
    }
    __syncthreads();
    float acc[R];
#pragma unroll
    for (int i = 0; i < R; ++i) acc[i] = 0.0f;
    if (direct)
        blur_groups<R, LW>(tile + (ty * R + RAD) * LW + tx + RAD, pkg, cnt, acc);
    else
        blur_groups<R, LW>(tile + (ty * R + RAD) * LW + tx + RAD, pk, cnt, acc);   // A: E(u)(x - d)
    if (x >= W) return;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int y = y0 + ty * R + i;
        if (y >= H) break;
        if (s_out) s_out[(size_t)y * W + x] = acc[i];   // unclamped A u (backward pass)
        const float s = fmaxf(acc[i], p.s_min);
        const float fv = fr[i];
        const float wt = p.robust ? pen_deriv(fmaxf(rf_eval(fv, s, p), 0.0f), p.eps_d2) : 1.0f;
        const float fp = fmaxf(fv, 0.0f);
        const float q = (s_out ? wt * (fp - s) : wt * fp) * rcp(s);
        qw[(size_t)y * W + x] = make_float2(q, wt);
    }
}

// Tile (column, row) of this workgroup on a 2D grid of tiles, remapped so
// that the workgroups of one XCD take a contiguous range of tiles in raster
// order: vertically adjacent tiles, which share halo rows, then mostly share
// an L2.
DEBLUR_DEV int2 xcd_tile()
{
    const int n = gridDim.x * gridDim.y;
    const int w = xcd_group(blockIdx.y * gridDim.x + blockIdx.x, n);
    const int ty = w / gridDim.x;
    return make_int2(w - ty * gridDim.x, ty);
}

template <int RAD, int TH, int NT>
__global__ void __launch_bounds__(NT) rrrl_taps_stage1(const float* __restrict__ u, const float* __restrict__ f,
                                                       float2* __restrict__ qw, float* __restrict__ s_out, int H,
                                                       int W, int pitch, const float* __restrict__ pkg,
                                                       const int* __restrict__ hdr, IterParams p, IterZ z)
{
    __shared__ float tile[stage1_lds_floats<RAD, TH>()];
    __shared__ float pk[packed_words_max<RAD>()];
    const int2 t = xcd_tile();
    stage1_tile<RAD, TH, NT>(tile, pk, zadv(u, z.u), zadv(f, z.f), zadv(qw, z.ws), s_out ? zadv(s_out, z.ws) : nullptr,
                             H, W, pitch, t.x * 64, t.y * TH, zadv(pkg, z.ws), zadv(hdr, z.ws), p);
}

template <int RAD, int TH>
struct Stage2Smem {
    float2 qt[(TH + 2 * RAD) * (64 + 2 * RAD)];
    float ut[(TH + 4) * (64 + 4)];
    float gt[(TH + 2) * (64 + 2)];
    float pk[packed_words_max<RAD>()];
};

// Stage 2 on the tile with top-left output (x0, y0).
template <int RAD, int TH, int NT>
DEBLUR_DEV void stage2_tile(Stage2Smem<RAD, TH>& sm, const float2* __restrict__ qw, const float* __restrict__ u,
                            float* __restrict__ u_next, float* __restrict__ ckpt, int H, int W, int pitch, int x0,
                            int y0, const float* __restrict__ pkg, const int* __restrict__ hdr, const IterParams& p)
{
    constexpr int TW = 64, LW = TW + 2 * RAD, LH = TH + 2 * RAD, R = TH / (NT / 64);
    static_assert(R >= 1 && TH % (NT / 64) == 0, "rows per thread");
    constexpr int UW = TW + 4, UH = TH + 4, GW = TW + 2, GH = TH + 2;
    float2* __restrict__ qt = sm.qt;
    float* __restrict__ ut = sm.ut;
    float* __restrict__ gt = sm.gt;
    const int tid = threadIdx.x;
    int cnt[TAP_GROUP_MAX];
    group_counts(hdr, cnt);
    const bool direct = hdr[10] <= DIRECT_TAP_WORDS;   // uniform: taps in place or staged
    if (!direct) stage_groups<RAD>(sm.pk, pkg, hdr);
    const bool inner = x0 >= RAD && y0 >= RAD && x0 + TW + RAD <= W && y0 + TH + RAD <= H;
    if (inner && W % 2 == 0 && ((uintptr_t)qw & 15) == 0) {
        // (q, W) pairs from an even column: 16-byte loads of two pairs
        copy_rows_f4<NT, LH, 2 * LW>(reinterpret_cast<float*>(qt),
                                     reinterpret_cast<const float*>(qw + (size_t)(y0 - RAD) * W + (x0 - RAD)),
                                     2 * (size_t)W);
    } else if (inner) {
        const float2* src = qw + (size_t)(y0 - RAD) * W + (x0 - RAD);
        stage_to_lds<NT, LH * LW>(qt, [&](int idx) {
            const int ly = idx / LW;
            return src[(size_t)ly * W + (idx - ly * LW)];
        });
    } else if (p.bc == BC_REPLICATE) {
        stage_to_lds<NT, LH * LW>(qt, [&](int idx) {
            const int ly = idx / LW, lx = idx - ly * LW;
            return qw[(size_t)clampi(y0 - RAD + ly, H) * W + clampi(x0 - RAD + lx, W)];
        });
    } else {
        stage_to_lds<NT, LH * LW>(qt, [&](int idx) {
            const int ly = idx / LW, lx = idx - ly * LW;
            const int gy = ext_index(y0 - RAD + ly, H, BC_PERIODIC), gx = ext_index(x0 - RAD + lx, W, BC_PERIODIC);
            return qw[(size_t)gy * W + gx];
        });
    }
    stage_to_lds<NT, UH * UW>(ut, [&](int idx) {
        const int ly = idx / UW, lx = idx - ly * UW;
        return u[(size_t)clampi(y0 - 2 + ly, H) * pitch + clampi(x0 - 2 + lx, W)];
    });
    __syncthreads();
    // diffusivity g = Psi'(|grad u|^2) by central differences at pixels
    for (int idx = tid; idx < GH * GW; idx += NT) {
        const int a = idx / GW, b = idx - a * GW;
        const float gx = 0.5f * (ut[(a + 1) * UW + b + 2] - ut[(a + 1) * UW + b]);
        const float gy = 0.5f * (ut[(a + 2) * UW + b + 1] - ut[a * UW + b + 1]);
        gt[idx] = tv_diffusivity(gx * gx + gy * gy, p);
    }
    const int tx = tid & 63, ty = tid >> 6;
    float n1[R], n2[R];
#pragma unroll
    for (int i = 0; i < R; ++i) n1[i] = n2[i] = 0.0f;
    if (direct)
        corr_groups<R, LW>(qt + (ty * R + RAD) * LW + tx + RAD, pkg, cnt, n1, n2);   // B: E(q, W)(x + d)
    else
        corr_groups<R, LW>(qt + (ty * R + RAD) * LW + tx + RAD, sm.pk, cnt, n1, n2);
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
        u_next[o] = up * num * rcp(den);
    }
}

template <int RAD, int TH, int NT>
__global__ void __launch_bounds__(NT) rrrl_taps_stage2(const float2* __restrict__ qw, const float* __restrict__ u,
                                                       float* __restrict__ u_next, float* __restrict__ ckpt,
                                                       int H, int W, int pitch, const float* __restrict__ pkg,
                                                       const int* __restrict__ hdr, IterParams p, IterZ z)
{
    __shared__ Stage2Smem<RAD, TH> sm;
    const int2 t = xcd_tile();
    if (z.alpha) p.alpha = z.alpha[blockIdx.z];
    stage2_tile<RAD, TH, NT>(sm, zadv(qw, z.ws), zadv(u, z.u), zadv(u_next, z.un), ckpt ? zadv(ckpt, z.ck) : nullptr, H,
                             W, pitch, t.x * 64, t.y * TH, zadv(pkg, z.ws), zadv(hdr, z.ws), p);
}

}  // namespace deblur
