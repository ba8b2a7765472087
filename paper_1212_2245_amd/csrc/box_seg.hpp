// Box tiles of the RRRL iteration (Sec. 2.3, eqs. (9)-(12)) for uniform linear
// motion blur along a coordinate axis (box PSF of length L = n + frac), one
// fused kernel per iteration, FP32 throughout.
//
// Window sums follow the paper's fast box filter (Sec. 4.3, uniform linear
// motion): a window sum is updated by one addition and one subtraction per
// position.  Long chains of such updates drift, so the chain is re-based
// every BOX_SEG positions of the blur axis: at every position whose
// coordinate is a multiple of BOX_SEG the window sum is formed afresh by a
// direct sum of its n terms, and between two such positions it slides
// (windows of at most BOX_SEG terms are always summed directly, and so is
// every window of an image of at most 512 x 512 pixels: such images are bound
// by the latency of a tile, and direct sums have no serial chain).  The
// re-basing points are absolute image coordinates, so the value at a pixel
// does not depend on the tile that computes it: every tile shape gives
// bitwise-identical results.  A non-integer length adds the two end pixels
// with weight frac/2 (relative to 1) outside the slid sum.
//
// Per tile (TA outputs along the blur axis x TC lines across it), 256 threads:
//   A. u on the tile plus a halo along (the A window of every q position B
//      reads, and the re-basing lead-in) and 2 lines across (diffusion term);
//      f at the q positions.
//   B. s = A u at the TA + n - 1 (+2) positions B reads (sliding: each thread
//      aligned blocks of BOX_SEG positions of one line; direct sums: one
//      position per thread and step); diffusivity g on the tile + 1; then W
//      and q at those positions (one position per thread and step).
//   C. N1 = B q, N2 = B W (re-based every BOX_SEG outputs), D(u), and the
//      update u' = u (N1 + a[D]_+) / (N2 - a[D]_-).
// A: window [x - floor(n/2), x + floor((n-1)/2)]; B: [x - floor((n-1)/2),
// x + floor(n/2)], weight 1/L; end pixels just outside each window.
// Orientation: VERT = false for horizontal motion (along = x, LDS lines are
// image rows), true for vertical motion (along = y, LDS rows are image rows
// so that global accesses stay coalesced along x).
#pragma once

#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace deblur {

constexpr int BOX_SEG = 8;    // re-basing period of the slid window sums
constexpr int BOX_NT = 256;   // threads per box tile

struct BoxGeom {
    int N, M;            // image extent along / across the blur axis
    int n, aL, bL, fr;   // integer length n, floor((n-1)/2), floor(n/2), 1 if frac > 0
    float ew, invL;      // end weight frac/2, 1/(n + frac)
    int hl, hr;          // u halo before / after the tile along the axis
    int nu, nq;          // u positions (TA + hl + hr), q positions (TA + n - 1 + 2 fr)
    int pu, pq, pg;      // LDS pitches: of u, q/W and g lines (horizontal) or rows (vertical)
    int slide;           // 1: windows slide between re-basing points; 0: every window summed directly
};

// LDS pitch of an array whose lines are read by the threads (line c = t % TC,
// chunk t / TC): horizontal lines need pitch = 1 mod 8 (the 8 chunks of a
// wavefront start 8*k words apart); vertical rows need 8 * pitch = TC mod 64.
__host__ __device__ inline int box_pitch(int width, bool vert, int TC)
{
    const int want = vert ? (TC / 8) % 8 : 1;
    int p = width;
    while (p % 8 != want) ++p;
    return p;
}

template <bool VERT, int TA, int TC>
__host__ __device__ inline BoxGeom box_geom(int H, int W, int n, float frac)
{
    BoxGeom g;
    g.N = VERT ? H : W;
    g.M = VERT ? W : H;
    g.n = n;
    g.aL = (n - 1) / 2;
    g.bL = n / 2;
    g.fr = frac > 0.0f ? 1 : 0;
    g.ew = 0.5f * frac;
    g.invL = 1.0f / ((float)n + frac);
    const int h = n - 1 + 2 * g.fr;
    g.hl = h + BOX_SEG - 1 > 2 ? h + BOX_SEG - 1 : 2;
    g.hr = h > 2 ? h : 2;
    g.nu = TA + g.hl + g.hr;
    g.nq = TA + n - 1 + 2 * g.fr;
    g.slide = n > BOX_SEG && (long)H * W > 512L * 512L;
    if (VERT) {
        g.pu = box_pitch(TC + 4, true, TC);
        g.pq = box_pitch(TC, true, TC);
        g.pg = box_pitch(TC + 2, true, TC);
    } else {
        g.pu = box_pitch(g.nu, false, TC);
        g.pq = box_pitch(g.nq, false, TC);
        g.pg = box_pitch(TA + 2, false, TC);
    }
    return g;
}

// LDS words of a tile: u, f/q, W, g.
template <bool VERT, int TA, int TC>
__host__ __device__ inline int box_lds_words(const BoxGeom& g)
{
    if (VERT) return g.nu * g.pu + 2 * g.nq * g.pq + (TA + 2) * g.pg;
    return (TC + 4) * g.pu + 2 * TC * g.pq + (TC + 2) * g.pg;
}

// Element (line c, position j) of an LDS array with pitch p.
template <bool VERT>
DEBLUR_DEV int box_at(int c, int j, int p)
{
    return VERT ? j * p + c : c * p + j;
}

// Floor division by BOX_SEG for possibly negative x.
DEBLUR_DEV int seg_floor(int x) { return x >= 0 ? x / BOX_SEG : -((-x + BOX_SEG - 1) / BOX_SEG); }

// p[0] + p[s] + ... + p[(n-1) s], added in this order, with the loads issued
// eight at a time (positions past n add +0, which leaves a non-negative sum
// unchanged bit for bit).
DEBLUR_DEV float seq_sum(const float* __restrict__ p, int s, int n)
{
    float S = 0.0f;
    for (int d = 0; d < n; d += 8) {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = p[min(d + k, n - 1) * s];
#pragma unroll
        for (int k = 0; k < 8; ++k) S += d + k < n ? v[k] : 0.0f;
    }
    return S;
}

// The same for two arrays at once (the two channels of the correlation).
DEBLUR_DEV void seq_sum2(const float* __restrict__ p, const float* __restrict__ q, int s, int n, float& Sp, float& Sq)
{
    Sp = Sq = 0.0f;
    for (int d = 0; d < n; d += 8) {
        float v[8], w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v[k] = p[min(d + k, n - 1) * s];
            w[k] = q[min(d + k, n - 1) * s];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            Sp += d + k < n ? v[k] : 0.0f;
            Sq += d + k < n ? w[k] : 0.0f;
        }
    }
}

template <bool VERT, int TA, int TC>
struct BoxTileOps {
    static_assert(TA % BOX_SEG == 0 && (TC * TA) % BOX_NT == 0 && TC % 4 == 0, "whole outputs per thread");
    static constexpr int OPT = TC * TA / BOX_NT;   // outputs per thread in phase C

    // Largest u / q extents of a tile (box arrays have at most 65 entries:
    // n - 1 + 2 fr <= 63).
    static constexpr int NU_MAX = TA + 2 * 63 + BOX_SEG - 1;
    static constexpr int NQ_MAX = TA + 64;

    // Phase A: u tile and f at the q positions.  Every global load of a
    // thread is issued before its first LDS store (one memory latency per
    // tile); interior tiles index directly, border tiles through the
    // continuation of the image.
    static DEBLUR_DEV void load(int t, float* __restrict__ lds, const float* __restrict__ u,
                                const float* __restrict__ f, int pitch, const BoxGeom& g, int bc, int a0, int c0)
    {
        const int ulo = a0 - g.hl;
        if (ulo >= 0 && ulo + g.nu <= g.N)
            load_impl<true>(t, lds, u, f, pitch, g, bc, a0, c0);
        else
            load_impl<false>(t, lds, u, f, pitch, g, bc, a0, c0);
    }

    template <bool INNER>
    static DEBLUR_DEV void load_impl(int t, float* __restrict__ lds, const float* __restrict__ u,
                                     const float* __restrict__ f, int pitch, const BoxGeom& g, int bc, int a0, int c0)
    {
        float* U = lds;
        float* Q = U + (VERT ? g.nu * g.pu : (TC + 4) * g.pu);
        const int ulo = a0 - g.hl;                      // along index of u position 0
        const int qlo = a0 - g.aL - g.fr;               // along index of q position 0
        auto along = [&](int i) { return INNER ? i : ext_index(i, g.N, bc); };
        if (VERT) {
            // u: rows j (along = y), columns c; thread t: column t % CW, rows t / CW + k RPP
            constexpr int CW = TC + 4, RPP = BOX_NT / CW, KU = (NU_MAX + RPP - 1) / RPP;
            // f: column t % TC, rows t / TC + k QPP
            constexpr int QPP = BOX_NT / TC, KQ = (NQ_MAX + QPP - 1) / QPP;
            const int c = t % CW, r0 = t / CW;
            const int cq = t % TC, q0 = t / TC;
            const float* ucol = u + clampi(c0 - 2 + c, g.M) + (INNER ? (size_t)(ulo + r0) * pitch : 0);
            const float* fcol = f + clampi(c0 + cq, g.M) + (INNER ? (size_t)(qlo + q0) * pitch : 0);
            const size_t su = (size_t)RPP * pitch, sq = (size_t)QPP * pitch;
            float vu[KU], vq[KQ];
#pragma unroll
            for (int k = 0; k < KU; ++k) {
                const int j = r0 + k * RPP;
                if (r0 < RPP && j < g.nu) vu[k] = INNER ? ucol[k * su] : ucol[(size_t)along(ulo + j) * pitch];
            }
#pragma unroll
            for (int k = 0; k < KQ; ++k) {
                const int m = q0 + k * QPP;
                if (m < g.nq) vq[k] = INNER ? fcol[k * sq] : fcol[(size_t)along(qlo + m) * pitch];
            }
            float* Uc = U + r0 * g.pu + c;
            float* Qc = Q + q0 * g.pq + cq;
#pragma unroll
            for (int k = 0; k < KU; ++k) {
                const int j = r0 + k * RPP;
                if (r0 < RPP && j < g.nu) Uc[k * RPP * g.pu] = vu[k];
            }
#pragma unroll
            for (int k = 0; k < KQ; ++k) {
                const int m = q0 + k * QPP;
                if (m < g.nq) Qc[k * QPP * g.pq] = vq[k];
            }
        } else {
            // lines c (image rows): wavefront w takes lines w, w + 4, ...; lanes along x
            constexpr int LU = (TC + 4 + 3) / 4, LQ = TC / 4;
            constexpr int RU = (NU_MAX + 63) / 64, RQ = (NQ_MAX + 63) / 64;
            const int w = t >> 6, lane = t & 63;
            float vu[LU][RU], vq[LQ][RQ];
#pragma unroll
            for (int l = 0; l < LU; ++l) {
                const int c = w + 4 * l;
                const float* row = u + (size_t)clampi(c0 - 2 + c, g.M) * pitch + (INNER ? ulo + lane : 0);
#pragma unroll
                for (int r = 0; r < RU; ++r) {
                    const int j = lane + 64 * r;
                    if (c < TC + 4 && j < g.nu) vu[l][r] = INNER ? row[64 * r] : row[along(ulo + j)];
                }
            }
#pragma unroll
            for (int l = 0; l < LQ; ++l) {
                const int c = w + 4 * l;
                const float* row = f + (size_t)clampi(c0 + c, g.M) * pitch + (INNER ? qlo + lane : 0);
#pragma unroll
                for (int r = 0; r < RQ; ++r) {
                    const int m = lane + 64 * r;
                    if (m < g.nq) vq[l][r] = INNER ? row[64 * r] : row[along(qlo + m)];
                }
            }
#pragma unroll
            for (int l = 0; l < LU; ++l) {
                float* Ul = U + (w + 4 * l) * g.pu + lane;
#pragma unroll
                for (int r = 0; r < RU; ++r) {
                    const int c = w + 4 * l, j = lane + 64 * r;
                    if (c < TC + 4 && j < g.nu) Ul[64 * r] = vu[l][r];
                }
            }
#pragma unroll
            for (int l = 0; l < LQ; ++l) {
                float* Ql = Q + (w + 4 * l) * g.pq + lane;
#pragma unroll
                for (int r = 0; r < RQ; ++r) {
                    const int m = lane + 64 * r;
                    if (m < g.nq) Ql[64 * r] = vq[l][r];
                }
            }
        }
    }

    // Phase B1: s = A u at the q positions (into the W array); B2: g.
    static DEBLUR_DEV void sums(int t, float* __restrict__ lds, const BoxGeom& g, const IterParams& p, int a0, int c0)
    {
        // explicit fmaf only: no multiply-add fused by the compiler, so that every
        // tile shape (every instantiation) rounds the same operations
#pragma clang fp contract(off)
        float* U = lds;
        float* Q = U + (VERT ? g.nu * g.pu : (TC + 4) * g.pu);
        float* Wt = Q + (VERT ? g.nq * g.pq : TC * g.pq);
        float* G = Wt + (VERT ? g.nq * g.pq : TC * g.pq);
        const int qlo = a0 - g.aL - g.fr;
        const int ulo = a0 - g.hl;
        if (!g.slide) {
            // B1 without sliding: every window summed directly, one q position
            // per thread and step (the positions are spread over all threads,
            // as in the weights phase, so the tile has no long serial chain)
            auto direct = [&](int c, int m) {
                const int x = qlo + m;
                const int xc = ext_index(x, g.N, p.bc);
                const int js = (p.bc == BC_PERIODIC ? x : xc) - ulo;
                const int cu = c + 2;
                float sum = seq_sum(U + box_at<VERT>(cu, js - g.bL, g.pu), VERT ? g.pu : 1, g.n);
                if (g.fr)
                    sum = fmaf(g.ew,
                               U[box_at<VERT>(cu, js - g.bL - 1, g.pu)] + U[box_at<VERT>(cu, js + g.aL + 1, g.pu)],
                               sum);
                Wt[box_at<VERT>(c, m, g.pq)] = fmaxf(sum, 0.0f) * g.invL;
            };
            if (VERT) {
                constexpr int QPP = BOX_NT / TC;
                const int c = t % TC;
                if (c0 + c < g.M)
                    for (int m = t / TC; m < g.nq; m += QPP) direct(c, m);
            } else {
                const int w = t >> 6, lane = t & 63;
                for (int c = w; c < TC && c0 + c < g.M; c += 4)
                    for (int m = lane; m < g.nq; m += 64) direct(c, m);
            }
        } else {
            // B1 with sliding: thread t takes line t % TC and the aligned blocks
            // of BOX_SEG q positions t / TC + k NB
            constexpr int NB = BOX_NT / TC;
            const int c = t % TC;
            const int kfirst = seg_floor(qlo), klast = seg_floor(qlo + g.nq - 1);
            const int cu = c + 2;                         // u line of this q line
            float S = 0.0f;
            if (c0 + c < g.M) {
                const int su = VERT ? g.pu : 1, sq = VERT ? g.pq : 1;
                const float* Ul = U + (VERT ? cu : cu * g.pu);
                float* Wl = Wt + (VERT ? c : c * g.pq);
                for (int k = kfirst + t / TC; k <= klast; k += NB) {
                    const int xb = max(qlo, k * BOX_SEG), xe = min(qlo + g.nq - 1, k * BOX_SEG + BOX_SEG - 1);
                    if (xb == k * BOX_SEG && xe == xb + BOX_SEG - 1 && xb >= 0 && xe < g.N) {
                        // whole block inside the q range and the image: straight-line form
                        // of the loop below (re-base at xb, then slide)
                        const float* ub = Ul + (xb - ulo) * su;   // u at the block's first sample
                        float* wo = Wl + (xb - qlo) * sq;
                        auto emit = [&](int i) {
                            float sum = S;
                            if (g.fr) sum = fmaf(g.ew, ub[(i - g.bL - 1) * su] + ub[(i + g.aL + 1) * su], sum);
                            wo[i * sq] = fmaxf(sum, 0.0f) * g.invL;
                        };
                        S = seq_sum(ub - g.bL * su, su, g.n);
                        emit(0);
#pragma unroll
                        for (int i = 1; i < BOX_SEG; ++i) {
                            S = (S + ub[(i + g.aL) * su]) - ub[(i - g.bL - 1) * su];
                            emit(i);
                        }
                        continue;
                    }
                    S = 0.0f;
                    int jprev = -(1 << 30);
                    for (int x = xb; x <= xe; ++x) {               // along index of the q position
                        const int xc = ext_index(x, g.N, p.bc);     // its image position
                        // u position of the sample: the clamped position under constant
                        // continuation, x itself (the tile holds the wrapped u) if periodic
                        const int js = (p.bc == BC_PERIODIC ? x : xc) - ulo;
                        const int r = xc % BOX_SEG;
                        if (js == jprev) {
                            // same sample as the previous position (clamped border run)
                        } else if (js == jprev + 1 && r != 0) {
                            S = (S + U[box_at<VERT>(cu, js + g.aL, g.pu)]) - U[box_at<VERT>(cu, js - g.bL - 1, g.pu)];
                        } else {
                            // re-base at the last multiple of BOX_SEG, slide to xc
                            const int j0 = js - r;
                            S = seq_sum(Ul + (j0 - g.bL) * su, su, g.n);
                            for (int d = 1; d <= r; ++d)
                                S = (S + U[box_at<VERT>(cu, j0 + d + g.aL, g.pu)]) -
                                    U[box_at<VERT>(cu, j0 + d - g.bL - 1, g.pu)];
                        }
                        jprev = js;
                        float sum = S;
                        if (g.fr)
                            sum = fmaf(g.ew,
                                       U[box_at<VERT>(cu, js - g.bL - 1, g.pu)] + U[box_at<VERT>(cu, js + g.aL + 1, g.pu)],
                                       sum);
                        Wt[box_at<VERT>(c, x - qlo, g.pq)] = fmaxf(sum, 0.0f) * g.invL;
                    }
                }
            }
        }
        // B2: diffusivity at across c0 - 1 + cc, along a0 - 1 + k (u position j = hl - 1 + k)
        {
            const int jmin = max(0, -ulo), jmax = min(g.nu - 1, g.N - 1 - ulo);
            if (jmin <= g.hl - 2 && jmax >= g.hl + TA + 1)
                diffusivity<false>(t, U, G, g, p, jmin, jmax);
            else
                diffusivity<true>(t, U, G, g, p, jmin, jmax);
        }
    }

    // g at (cc, k), cc < TC + 2, k < TA + 2; EDGE: along neighbours clamped to
    // the image (u positions jmin .. jmax).
    template <bool EDGE>
    static DEBLUR_DEV void diffusivity(int t, const float* __restrict__ U, float* __restrict__ G, const BoxGeom& g,
                                       const IterParams& p, int jmin, int jmax)
    {
        // explicit fmaf only: no multiply-add fused by the compiler, so that every
        // tile shape (every instantiation) rounds the same operations
#pragma clang fp contract(off)
        constexpr int GW = TA + 2, GL = TC + 2;
        const int su = VERT ? g.pu : 1, lu = VERT ? 1 : g.pu;
        auto one = [&](int cc, int k) {
            const int j = g.hl - 1 + k;
            const int jm = EDGE ? max(j - 1, jmin) : j - 1, jp = EDGE ? min(j + 1, jmax) : j + 1;
            const int jc = EDGE ? min(max(j, jmin), jmax) : j;
            const float* U1 = U + (cc + 1) * lu;
            const float da = 0.5f * (U1[jp * su] - U1[jm * su]);
            const float dc = 0.5f * (U1[jc * su + lu] - U1[jc * su - lu]);
            G[VERT ? k * g.pg + cc : cc * g.pg + k] = tv_diffusivity(da * da + dc * dc, p);
        };
        if (VERT) {
            // column cc = t % GL, rows t / GL + r RPG
            constexpr int RPG = BOX_NT / GL, R = (GW + RPG - 1) / RPG;
            const int cc = t % GL, k0 = t / GL;
            if (k0 < RPG) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (k0 + r * RPG < GW) one(cc, k0 + r * RPG);
            }
        } else {
            // wavefront w: lines w, w + 4, ...; lanes along k
            constexpr int LG = (GL + 3) / 4, R = (GW + 63) / 64;
            const int w = t >> 6, lane = t & 63;
#pragma unroll
            for (int l = 0; l < LG; ++l)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (w + 4 * l < GL && lane + 64 * r < GW) one(w + 4 * l, lane + 64 * r);
        }
    }

    // Phase B3: robust weight W and quotient q from s (W array) and f (Q
    // array), in place, one position per thread and step.
    static DEBLUR_DEV void weights(int t, float* __restrict__ lds, const BoxGeom& g, const IterParams& p, int c0)
    {
        // explicit fmaf only: no multiply-add fused by the compiler, so that every
        // tile shape (every instantiation) rounds the same operations
#pragma clang fp contract(off)
        float* Q = lds + (VERT ? g.nu * g.pu : (TC + 4) * g.pu);
        float* Wt = Q + (VERT ? g.nq * g.pq : TC * g.pq);
        auto one = [&](int iq, float sv, float fv) {
            const float s = fmaxf(sv, p.s_min);
            const float wt = p.robust ? pen_deriv(fmaxf(rf_eval(fv, s, p), 0.0f), p.eps_d2) : 1.0f;
            Q[iq] = wt * fmaxf(fv, 0.0f) * rcp(s);
            Wt[iq] = wt;
        };
        // the positions of a thread, K at a time: all loads first
        constexpr int K = 4;
        if (VERT) {
            // column t % TC, rows t / TC + k QPP
            constexpr int QPP = BOX_NT / TC;
            const int c = t % TC;
            if (c0 + c < g.M)
                for (int m0 = t / TC; m0 < g.nq; m0 += K * QPP) {
                    float sv[K], fv[K];
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const int iq = min(m0 + k * QPP, g.nq - 1) * g.pq + c;
                        sv[k] = Wt[iq];
                        fv[k] = Q[iq];
                    }
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (m0 + k * QPP < g.nq) one((m0 + k * QPP) * g.pq + c, sv[k], fv[k]);
                }
        } else {
            const int w = t >> 6, lane = t & 63;
            for (int c = w; c < TC && c0 + c < g.M; c += 4)
                for (int m0 = lane; m0 < g.nq; m0 += K * 64) {
                    float sv[K], fv[K];
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const int iq = c * g.pq + min(m0 + 64 * k, g.nq - 1);
                        sv[k] = Wt[iq];
                        fv[k] = Q[iq];
                    }
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (m0 + 64 * k < g.nq) one(c * g.pq + m0 + 64 * k, sv[k], fv[k]);
                }
        }
    }

    // Phase C for a chunk of OPT outputs x0 .. x0 + OPT - 1 whose along
    // neighbours all lie inside the image (x0 >= 1, x0 + OPT < N): the same
    // arithmetic as the general loop below, in straight-line form.  x0 is a
    // multiple of OPT, and OPT divides BOX_SEG or is a multiple of it, so the
    // re-basing points inside a chunk are the multiples of BOX_SEG of i.
    static DEBLUR_DEV void update_inner(int c, int o0, const float* __restrict__ U, const float* __restrict__ Q,
                                        const float* __restrict__ Wt, const float* __restrict__ G,
                                        float* __restrict__ un, float* __restrict__ ckpt, int pitch,
                                        const BoxGeom& g, const IterParams& p, int x0, int gc)
    {
        // explicit fmaf only: no multiply-add fused by the compiler, so that every
        // tile shape (every instantiation) rounds the same operations
#pragma clang fp contract(off)
        static_assert(OPT % BOX_SEG == 0 || BOX_SEG % OPT == 0, "chunks aligned to the re-basing period");
        const int sq = VERT ? g.pq : 1, su = VERT ? g.pu : 1, sg = VERT ? g.pg : 1;
        const int lu = VERT ? 1 : g.pu, lg = VERT ? 1 : g.pg;   // next line
        const float* qb = Q + (VERT ? c : c * g.pq) + (o0 + g.fr) * sq;   // B window start of output o0
        const float* wb = Wt + (VERT ? c : c * g.pq) + (o0 + g.fr) * sq;
        const float* U2 = U + (c + 2) * lu + (g.hl + o0) * su;
        const float* G1 = G + (c + 1) * lg + (o0 + 1) * sg;
        const int n = g.n;
        auto finish = [&](int i, float N1, float N2) {
            float s1 = N1, s2 = N2;
            if (g.fr) {
                s1 = fmaf(g.ew, qb[(i - 1) * sq] + qb[(i + n) * sq], s1);
                s2 = fmaf(g.ew, wb[(i - 1) * sq] + wb[(i + n) * sq], s2);
            }
            const float n1 = fmaxf(s1, 0.0f) * g.invL, n2 = fmaxf(s2, 0.0f) * g.invL;
            const float up = U2[i * su];
            const float gp = G1[i * sg];
            const float D = 0.5f * (gp + G1[(i - 1) * sg]) * (U2[(i - 1) * su] - up)
                          + 0.5f * (gp + G1[(i + 1) * sg]) * (U2[(i + 1) * su] - up)
                          + 0.5f * (gp + G1[i * sg - lg]) * (U2[i * su - lu] - up)
                          + 0.5f * (gp + G1[i * sg + lg]) * (U2[i * su + lu] - up);
            const float num = n1 + p.alpha * fmaxf(D, 0.0f);
            const float den = n2 - p.alpha * fminf(D, 0.0f);
            const size_t off = VERT ? (size_t)(x0 + i) * pitch + gc : (size_t)gc * pitch + x0 + i;
            if (ckpt) ckpt[off] = up;
            un[off] = up * num * rcp(den);
        };
        float N1, N2;
        if (!g.slide) {
            // every window summed directly, in a rolled loop (one copy of the code)
#pragma unroll 1
            for (int i = 0; i < OPT; ++i) {
                seq_sum2(qb + i * sq, wb + i * sq, sq, n, N1, N2);
                finish(i, N1, N2);
            }
            return;
        }
        {
            // re-base at the last multiple of BOX_SEG (a chunk shorter than
            // BOX_SEG may start after it), then slide to output 0
            const int r = OPT % BOX_SEG != 0 ? x0 % BOX_SEG : 0;
            seq_sum2(qb - r * sq, wb - r * sq, sq, n, N1, N2);
            for (int d = 1; d <= r; ++d) {
                N1 = (N1 + qb[(d - r + n - 1) * sq]) - qb[(d - r - 1) * sq];
                N2 = (N2 + wb[(d - r + n - 1) * sq]) - wb[(d - r - 1) * sq];
            }
        }
        finish(0, N1, N2);
#pragma unroll
        for (int i = 1; i < OPT; ++i) {
            if (i % BOX_SEG == 0) {
                seq_sum2(qb + i * sq, wb + i * sq, sq, n, N1, N2);
            } else {
                N1 = (N1 + qb[(i + n - 1) * sq]) - qb[(i - 1) * sq];
                N2 = (N2 + wb[(i + n - 1) * sq]) - wb[(i - 1) * sq];
            }
            finish(i, N1, N2);
        }
    }

    // Phase C: correlation, diffusion term, update; thread t takes line t % TC
    // and OPT consecutive outputs.
    static DEBLUR_DEV void update(int t, const float* __restrict__ lds, float* __restrict__ un,
                                  float* __restrict__ ckpt, int pitch, const BoxGeom& g, const IterParams& p, int a0,
                                  int c0)
    {
        // explicit fmaf only: no multiply-add fused by the compiler, so that every
        // tile shape (every instantiation) rounds the same operations
#pragma clang fp contract(off)
        const float* U = lds;
        const float* Q = U + (VERT ? g.nu * g.pu : (TC + 4) * g.pu);
        const float* Wt = Q + (VERT ? g.nq * g.pq : TC * g.pq);
        const float* G = Wt + (VERT ? g.nq * g.pq : TC * g.pq);
        const int ulo = a0 - g.hl;
        const int jmin = max(0, -ulo), jmax = min(g.nu - 1, g.N - 1 - ulo);
        const int c = t % TC, o0 = (t / TC) * OPT;
        const int gc = c0 + c;
        if (gc >= g.M) return;
        if (a0 + o0 >= 1 && a0 + o0 + OPT < g.N) {
            update_inner(c, o0, U, Q, Wt, G, un, ckpt, pitch, g, p, a0 + o0, gc);
            return;
        }
        float N1 = 0.0f, N2 = 0.0f;
        for (int o = o0; o < o0 + OPT; ++o) {
            const int x = a0 + o;
            if (x >= g.N) break;
            // B window [x - aL, x + bL] at q positions [o + fr, o + fr + n - 1]
            const int w0 = o + g.fr;
            if (x % BOX_SEG == 0 || o == o0 || !g.slide) {
                // re-base at the last multiple of BOX_SEG (o0 is one); no sliding: direct sums
                const int r = g.slide ? x % BOX_SEG : 0;
                const int i0 = box_at<VERT>(c, w0 - r, g.pq);
                seq_sum2(Q + i0, Wt + i0, VERT ? g.pq : 1, g.n, N1, N2);
                for (int d = 1; d <= r; ++d) {
                    const int ih = box_at<VERT>(c, w0 - r + d + g.n - 1, g.pq), il = box_at<VERT>(c, w0 - r + d - 1, g.pq);
                    N1 = (N1 + Q[ih]) - Q[il];
                    N2 = (N2 + Wt[ih]) - Wt[il];
                }
            } else {
                const int ih = box_at<VERT>(c, w0 + g.n - 1, g.pq), il = box_at<VERT>(c, w0 - 1, g.pq);
                N1 = (N1 + Q[ih]) - Q[il];
                N2 = (N2 + Wt[ih]) - Wt[il];
            }
            float s1 = N1, s2 = N2;
            if (g.fr) {
                const int e0 = box_at<VERT>(c, o, g.pq), e1 = box_at<VERT>(c, o + g.n + 1, g.pq);
                s1 = fmaf(g.ew, Q[e0] + Q[e1], s1);
                s2 = fmaf(g.ew, Wt[e0] + Wt[e1], s2);
            }
            const float n1 = fmaxf(s1, 0.0f) * g.invL, n2 = fmaxf(s2, 0.0f) * g.invL;
            // diffusion term: neighbours along beyond the image read u_p (zero flux)
            const int j = g.hl + o;
            const int jm = max(j - 1, jmin), jp = min(j + 1, jmax);
            const int k = o + 1;
            const float up = U[box_at<VERT>(c + 2, j, g.pu)];
            const float gp = G[box_at<VERT>(c + 1, k, g.pg)];
            const float D = 0.5f * (gp + G[box_at<VERT>(c + 1, k - 1, g.pg)]) * (U[box_at<VERT>(c + 2, jm, g.pu)] - up)
                          + 0.5f * (gp + G[box_at<VERT>(c + 1, k + 1, g.pg)]) * (U[box_at<VERT>(c + 2, jp, g.pu)] - up)
                          + 0.5f * (gp + G[box_at<VERT>(c, k, g.pg)]) * (U[box_at<VERT>(c + 1, j, g.pu)] - up)
                          + 0.5f * (gp + G[box_at<VERT>(c + 2, k, g.pg)]) * (U[box_at<VERT>(c + 3, j, g.pu)] - up);
            const float num = n1 + p.alpha * fmaxf(D, 0.0f);
            const float den = n2 - p.alpha * fminf(D, 0.0f);
            const size_t off = VERT ? (size_t)x * pitch + gc : (size_t)gc * pitch + x;
            if (ckpt) ckpt[off] = up;
            un[off] = up * num * rcp(den);
        }
    }
};

// Tile shape (TA along, TC across) of box tile variant v = 1..5: calls
// f(TA, TC) with both as std::integral_constant.  Variants 1 and 2 swap
// between the orientations so that variant 1 is the wide-along shape for
// horizontal and the tall-across one for vertical motion.
template <bool VERT, typename F>
inline void with_box_shape(int v, F&& f)
{
    using std::integral_constant;
    switch (v) {
        case 1:
            if constexpr (VERT) f(integral_constant<int, 128>{}, integral_constant<int, 16>{});
            else f(integral_constant<int, 256>{}, integral_constant<int, 8>{});
            break;
        case 2:
            if constexpr (VERT) f(integral_constant<int, 256>{}, integral_constant<int, 8>{});
            else f(integral_constant<int, 128>{}, integral_constant<int, 16>{});
            break;
        case 3: f(integral_constant<int, 64>{}, integral_constant<int, 32>{}); break;
        case 4: f(integral_constant<int, 64>{}, integral_constant<int, 8>{}); break;
        default: f(integral_constant<int, 64>{}, integral_constant<int, 4>{}); break;
    }
}
constexpr int BOX_VARIANTS = 5;

template <bool VERT, int TA, int TC>
DEBLUR_DEV void box_seg_tile(float* __restrict__ lds, const float* __restrict__ u, const float* __restrict__ f,
                             float* __restrict__ un, float* __restrict__ ckpt, int pitch, const BoxGeom& g,
                             const IterParams& p, int a0, int c0)
{
    using Ops = BoxTileOps<VERT, TA, TC>;
    const int t = threadIdx.x;
    Ops::load(t, lds, u, f, pitch, g, p.bc, a0, c0);
    __syncthreads();
    Ops::sums(t, lds, g, p, a0, c0);
    __syncthreads();
    Ops::weights(t, lds, g, p, c0);
    __syncthreads();
    Ops::update(t, lds, un, ckpt, pitch, g, p, a0, c0);
}

}  // namespace deblur
