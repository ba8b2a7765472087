// Box tiles of the RRRL iteration (Sec. 2.3, eqs. (9)-(12)) for uniform linear motion blur
// along a coordinate axis (box PSF of length L = n + frac), one fused kernel per
// iteration.
//
// The paper's fast box filter (Sec. 4.3, uniform linear motion) updates a
// window sum by one addition and one subtraction per pixel.  Here every
// workgroup owns a tile and forms inclusive prefix sums of its tile rows
// along the blur axis in LDS, so a window sum is a difference of two prefix
// values.  The prefix restarts at every tile (a few hundred terms) and is
// accumulated in FP64, so a window sum is as accurate as a direct FP32 sum of
// its L terms even for short windows; window sums of non-negative data are
// clamped at zero.
//
// Per tile (TA outputs along the blur axis x TC across it):
//   1. u on the tile plus halo L-1 along (for A evaluated on the halo that B
//      needs) and 2 across (diffusion term); f is read where needed.
//   2. prefix of u along; diffusivity g on the tile + 1.
//   3. s = A u, W, q on the TA + L - 1 positions B reads.
//   4. prefix of (q, W) along.
//   5. N1 = B q, N2 = B W, D(u), u' = u (N1 + a[D]_+) / (N2 - a[D]_-).
// A: window [x - floor(n/2), x + floor((n-1)/2)]; B: [x - floor((n-1)/2), x + floor(n/2)],
// weight 1/L.  A non-integer length adds the two pixels just outside each
// window with weight (frac/2)/L (Sec. 4.3): the window sums gain two end
// terms, read from the u tile (A) or as differences of the (q, W) prefix (B);
// the halo along and the q/W span grow by one position on each side.
// Orientation: VERT = false for horizontal motion (along = x), true for
// vertical motion (along = y).  LDS rows are "lines" of the tile along the
// blur axis for horizontal motion and image rows for vertical motion, so that
// global accesses stay coalesced along x in both cases.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace deblur {


struct BoxTile {
    int along_n, across_n;  // image extent along / across the blur axis
    int L, aL, bL, hA;      // integer length n, floor((n-1)/2), floor(n/2), halo along
    int fr;                 // 1 for a non-integer length (end pixels), else 0
    float ew, invL;         // end weight frac/2 (relative to the inner weight), 1/(n + frac)
    int nu, nq;             // tile positions along: u (TA + 2hA), q/W (TA + n - 1 + 2fr)
};

DEBLUR_DEV double2 operator+(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
DEBLUR_DEV double2 operator-(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

template <bool VERT, int TA, int TC>
struct BoxLayout {
    // LDS element (c, j): across index c, along index j, line length n
    static DEBLUR_DEV int at(int c, int j, int n, int lines)
    {
        return VERT ? j * lines + c : c * (n + 1) + j;
    }
};

// Visits every (line c < LINES, position j < n) of a tile: value = load(c, j)
// then store(c, j, value), with the loads of up to U positions of every line
// a thread owns issued before the first store.  Horizontal tiles: wavefront
// w takes lines w, w + 4, ...; its lanes run along j (coalesced along x).
// Vertical tiles: flat index i = j LINES + c (coalesced along x = c).  No
// division by a run-time value.
template <bool VERT, int LINES, int U, typename L, typename S>
DEBLUR_DEV void tile_pass(int n, L load, S store)
{
    using T = decltype(load(0, 0));
    if constexpr (VERT) {
        const int total = n * LINES;
        for (int base = threadIdx.x; base < total; base += U * 256) {
            T v[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int i = base + k * 256, j = i / LINES, c = i - j * LINES;
                if (i < total) v[k] = load(c, j);
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int i = base + k * 256, j = i / LINES, c = i - j * LINES;
                if (i < total) store(c, j, v[k]);
            }
        }
    } else {
        constexpr int NC = (LINES + 3) / 4;
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int j0 = lane; j0 < n; j0 += U * 64) {
            T v[NC][U];
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const int c = w + 4 * q, j = j0 + 64 * k;
                    if (c < LINES && j < n) v[q][k] = load(c, j);
                }
#pragma unroll
            for (int q = 0; q < NC; ++q)
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const int c = w + 4 * q, j = j0 + 64 * k;
                    if (c < LINES && j < n) store(c, j, v[q][k]);
                }
        }
    }
}

// Inclusive prefix along each of `lines` LDS lines of length n (in place),
// block-wide.  The G = 256/TC threads of a line are consecutive lanes of one
// wavefront; each sums a contiguous chunk, the chunk offsets come from a
// shuffle scan over the G lanes.
template <typename T>
DEBLUR_DEV T shfl_up_T(T v, int d, int width);
template <>
DEBLUR_DEV double shfl_up_T<double>(double v, int d, int width) { return __shfl_up(v, d, width); }
template <>
DEBLUR_DEV double2 shfl_up_T<double2>(double2 v, int d, int width)
{
    return make_double2(__shfl_up(v.x, d, width), __shfl_up(v.y, d, width));
}

template <bool VERT, int TA, int TC, typename T>
DEBLUR_DEV void prefix_lines(T* buf, int n, int lines, T* /*sums*/)
{
    constexpr int G = 256 / TC;
    static_assert(G <= 64 && (G & (G - 1)) == 0, "line group within a wavefront");
    const int t = threadIdx.x;
    const int c = t / G, g = t % G;
    const int ch = (n + G - 1) / G;
    const int j0 = g * ch, j1 = min(n, j0 + ch);
    T acc = T{};
    if (c < lines)
        for (int j = j0; j < j1; ++j) acc = acc + buf[BoxLayout<VERT, TA, TC>::at(c, j, n, lines)];
    // inclusive scan of the chunk sums over the G lanes of this line
    T inc = acc;
    for (int d = 1; d < G; d <<= 1) {
        const T v = shfl_up_T(inc, d, G);
        if (g >= d) inc = inc + v;
    }
    T off = inc - acc;
    if (c < lines) {
        for (int j = j0; j < j1; ++j) {
            const int i = BoxLayout<VERT, TA, TC>::at(c, j, n, lines);
            off = off + buf[i];
            buf[i] = off;
        }
    }
    __syncthreads();
}



// One box-iteration tile: outputs along [a0, a0+TA), across [c0, c0+TC);
// smem_raw: dynamic LDS of box_lds_bytes() for this tile geometry.
template <bool VERT, int TA, int TC>
DEBLUR_DEV void box_iter_tile(unsigned char* __restrict__ smem_raw, const float* __restrict__ u,
                              const float* __restrict__ f, float* __restrict__ un, float* __restrict__ ckpt, int pitch,
                              const BoxTile& bt, const IterParams& p, int a0, int c0)
{
    using Lay = BoxLayout<VERT, TA, TC>;
    constexpr int CU = TC + 4;   // u lines (across halo 2)
    constexpr int G = 256 / TC;
    const int nu = bt.nu, nq = bt.nq;
    float* us = reinterpret_cast<float*>(smem_raw);                 // CU lines of nu (u tile)
    float* gs = us + CU * (nu + 1);                                  // (TC+2) x (TA+2) diffusivity
    const int doff = (CU * (nu + 1) + (TC + 2) * (TA + 3) + 3) & ~3;
    double* ps = reinterpret_cast<double*>(us + doff);               // TC lines of nu: prefix of u
    double2* qs = reinterpret_cast<double2*>(ps + TC * (nu + 1));    // TC lines of nq: prefix of (q, W)
    double2* sums2 = qs + TC * (nq + 1);
    double* sums = reinterpret_cast<double*>(sums2 + 256);

    const int lo = a0 - bt.hA;                               // along index of tile position 0
    const int t = threadIdx.x;
    const int H = VERT ? bt.along_n : bt.across_n;
    const int W = VERT ? bt.across_n : bt.along_n;

    // 1. u tile: along extended by the boundary mode, across clamped
    tile_pass<VERT, CU, 4>(
        nu,
        [&](int c, int j) {
            const int ga = ext_index(lo + j, bt.along_n, p.bc);
            const int gc = clampi(c0 - 2 + c, bt.across_n);
            const int y = VERT ? ga : gc, x = VERT ? gc : ga;
            return u[(size_t)y * pitch + x];
        },
        [&](int c, int j, float v) { us[Lay::at(c, j, nu, CU)] = v; });
    __syncthreads();
    // 2a. copy of the TC center lines for the prefix, 2b. diffusivity
    tile_pass<VERT, TC, 1>(
        nu, [&](int c, int j) { return us[Lay::at(c + 2, j, nu, CU)]; },
        [&](int c, int j, float v) { ps[Lay::at(c, j, nu, TC)] = (double)v; });
    // tile positions of the first/last image index along (clamping for TV)
    const int jmin = max(0, -lo), jmax = min(nu - 1, bt.along_n - 1 - lo);
    constexpr int GA = TA + 2;
    for (int i = t; i < (TC + 2) * GA; i += 256) {
        int c, k;
        if (VERT) { k = i / (TC + 2); c = i - k * (TC + 2); } else { c = i / GA; k = i - c * GA; }
        // g at across c0 - 1 + c, along a0 - 1 + k (tile j = hA - 1 + k)
        const int j = bt.hA - 1 + k;
        const int jm = max(j - 1, jmin), jp = min(j + 1, jmax), jc = min(max(j, jmin), jmax);
        const float da = 0.5f * (us[Lay::at(c + 1, jp, nu, CU)] - us[Lay::at(c + 1, jm, nu, CU)]);
        const float dc = 0.5f * (us[Lay::at(c + 2, jc, nu, CU)] - us[Lay::at(c, jc, nu, CU)]);
        gs[VERT ? k * (TC + 2) + c : c * (GA + 1) + k] = tv_diffusivity(da * da + dc * dc, p);
    }
    __syncthreads();
    prefix_lines<VERT, TA, TC, double>(ps, nu, TC, sums);
    // 3. s = A u, W, q on positions m = 0..nq-1 (along a0 - aL - fr + m)
    const float invL = bt.invL;
    // f is fetched for several positions before any is used
    tile_pass<VERT, TC, 4>(
        nq,
        [&](int c, int m) {
            const int gc = c0 + c;
            if (gc >= bt.across_n) return 0.0f;
            const int ga = ext_index(a0 - bt.aL - bt.fr + m, bt.along_n, p.bc);
            const int y = VERT ? ga : gc, x = VERT ? gc : ga;
            return f[(size_t)y * pitch + x];
        },
        [&](int c, int m, float fv) {
            const int gc = c0 + c;
            double2 qw = make_double2(0.0, 0.0);
            if (gc < bt.across_n) {
                // B reads E(q)(x'): q at the continued position.  Periodic: the
                // tile holds the wrapped u, so x' itself is used; constant
                // continuation: q(clamp(x')), i.e. A u at the clamped position.
                const int xa = a0 - bt.aL - bt.fr + m;
                const int ga = ext_index(xa, bt.along_n, p.bc);
                const int j = (p.bc == BC_PERIODIC ? xa : ga) - lo;  // tile position of the sample
                const int hi = j + bt.aL, lo2 = j - bt.bL - 1;          // A window [j - bL, j + aL]
                double sum = ps[Lay::at(c, hi, nu, TC)] - (lo2 >= 0 ? ps[Lay::at(c, lo2, nu, TC)] : 0.0);
                if (bt.fr)   // end pixels j - bL - 1 and j + aL + 1
                    sum += (double)bt.ew * ((double)us[Lay::at(c + 2, lo2, nu, CU)] +
                                            (double)us[Lay::at(c + 2, hi + 1, nu, CU)]);
                const float s = fmaxf((float)fmax(sum, 0.0) * invL, p.s_min);
                const float wt = p.robust ? pen_deriv(fmaxf(rf_eval(fv, s, p), 0.0f), p.eps_d2) : 1.0f;
                qw = make_double2((double)(wt * fmaxf(fv, 0.0f) * rcp(s)), (double)wt);
            }
            qs[Lay::at(c, m, nq, TC)] = qw;
        });
    __syncthreads();
    prefix_lines<VERT, TA, TC, double2>(qs, nq, TC, sums2);
    // 5. correlation, diffusion term, update
    for (int i = t; i < TC * TA; i += 256) {
        int c, o;
        if (VERT) { o = i / TC; c = i - o * TC; } else { c = i / TA; o = i - c * TA; }
        const int gc = c0 + c, ga = a0 + o;
        if (gc >= bt.across_n || ga >= bt.along_n) continue;
        // B window [o + fr, o + fr + n - 1] in q positions; end pixels o and
        // o + n + 1 (non-integer length) as differences of the prefix
        const int w0 = o + bt.fr;
        const double2 hi = qs[Lay::at(c, w0 + bt.L - 1, nq, TC)];
        const double2 lw = w0 > 0 ? qs[Lay::at(c, w0 - 1, nq, TC)] : make_double2(0.0, 0.0);
        double2 sum = hi - lw;
        if (bt.fr) {
            const double2 e0 = qs[Lay::at(c, o, nq, TC)] - (o > 0 ? qs[Lay::at(c, o - 1, nq, TC)] : make_double2(0.0, 0.0));
            const double2 e1 = qs[Lay::at(c, o + bt.L + 1, nq, TC)] - hi;
            const double ew = (double)bt.ew;
            sum = sum + make_double2(ew * (e0.x + e1.x), ew * (e0.y + e1.y));
        }
        const float n1 = (float)fmax(sum.x, 0.0) * invL, n2 = (float)fmax(sum.y, 0.0) * invL;
        const int j = bt.hA + o;
        const int jm = max(j - 1, jmin), jp = min(j + 1, jmax);
        const float up = us[Lay::at(c + 2, j, nu, CU)];
        const int k = o + 1;
        auto G_ = [&](int cc, int kk) { return gs[VERT ? kk * (TC + 2) + cc : cc * (GA + 1) + kk]; };
        const float gp = G_(c + 1, k);
        // along neighbours beyond the image border read u_p itself (zero flux)
        const float D = 0.5f * (gp + G_(c + 1, k - 1)) * (us[Lay::at(c + 2, jm, nu, CU)] - up)
                      + 0.5f * (gp + G_(c + 1, k + 1)) * (us[Lay::at(c + 2, jp, nu, CU)] - up)
                      + 0.5f * (gp + G_(c, k)) * (us[Lay::at(c + 1, j, nu, CU)] - up)
                      + 0.5f * (gp + G_(c + 2, k)) * (us[Lay::at(c + 3, j, nu, CU)] - up);
        const float num = n1 + p.alpha * fmaxf(D, 0.0f);
        const float den = n2 - p.alpha * fminf(D, 0.0f);
        const int y = VERT ? ga : gc, x = VERT ? gc : ga;
        const size_t off = (size_t)y * pitch + x;
        if (ckpt) ckpt[off] = up;
        un[off] = up * num * rcp(den);
    }
    (void)G;
    (void)H;
    (void)W;
}


template <bool VERT, int TA, int TC>
inline size_t box_lds_bytes(const BoxTile& bt)
{
    constexpr int CU = TC + 4;
    const size_t fl = ((size_t)CU * (bt.nu + 1) + (size_t)(TC + 2) * (TA + 3) + 3) & ~(size_t)3;
    return fl * 4 + (size_t)TC * (bt.nu + 1) * 8 + ((size_t)TC * (bt.nq + 1) + 256) * 16 + 256 * 8;
}

__host__ __device__ inline BoxTile make_tile(int H, int W, int L, float frac, bool vert, int TA)
{
    BoxTile bt;
    bt.along_n = vert ? H : W;
    bt.across_n = vert ? W : H;
    bt.L = L;
    bt.aL = (L - 1) / 2;
    bt.bL = L / 2;
    bt.fr = frac > 0.0f ? 1 : 0;
    bt.ew = 0.5f * frac;
    bt.invL = 1.0f / ((float)L + frac);
    const int h = L - 1 + 2 * bt.fr;
    bt.hA = h > 2 ? h : 2;
    bt.nu = TA + 2 * bt.hA;
    bt.nq = TA + L - 1 + 2 * bt.fr;
    return bt;
}

// Tile shapes (positions along the blur axis x lines across): the narrow
// shapes serve vertical blur, small images and the batched graph; the wide
// horizontal shape serves single images above 512^2, where it measured faster.
constexpr int BOXH_TA = 64, BOXH_TC = 4, BOXV_TA = 64, BOXV_TC = 8;
constexpr int BOXH_WIDE_TA = 128, BOXH_WIDE_TC = 8;

}  // namespace deblur
