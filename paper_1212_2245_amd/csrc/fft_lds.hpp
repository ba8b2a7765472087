// Mixed-radix (2, 3, 4, 8) Stockham FFT of a batch of rows held in LDS.
//
// The paper uses its own power-of-two FFT with twiddles precomputed once
// (Sec. 4.1).  Here the transform lengths are n = 2^a 3^b (image sides such as
// 192, 384, 768 occur in the batched workload), the butterflies run in FP32
// in LDS and the twiddles exp(-2 pi i m / n) are generated in FP64 per
// workgroup and rounded once to FP32.
//
// The same code runs in FP64 (complex type double2, FP64 twiddles) for the
// Wiener step's FP64 variant.
//
// Stockham autosort formulation: pass p with radix R and stride Ns (product of
// the radices already applied) maps butterfly j (0 <= j < n/R), k = j mod Ns,
//   inputs   x[j + r n/R],  r = 0..R-1
//   twiddle  x_r *= w_n^(k r n/(Ns R))
//   outputs  y[(j - k) R + k + r Ns] = DFT_R(x)_r
// and leaves the result in natural order after the last pass.  Forward
// transforms only (sign -1); inverses use conj(FFT(conj(X)))/n.
#pragma once

#include "common.hpp"

namespace deblur {

struct FftPlan {
    int n;
    int npass;
    int radix[16];
    unsigned mag[16];   // ceil(2^32 / Ns) of pass q (Ns = product of the earlier radices)
};

DEBLUR_DEV float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
DEBLUR_DEV float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
DEBLUR_DEV float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
DEBLUR_DEV float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i
DEBLUR_DEV float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }

DEBLUR_DEV double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
DEBLUR_DEV double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
DEBLUR_DEV double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
DEBLUR_DEV double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
DEBLUR_DEV double2 cmul_mi(double2 a) { return make_double2(a.y, -a.x); }

// Real type and constructor of a complex type.
template <typename C> struct Cplx;
template <> struct Cplx<float2> {
    using R = float;
    static DEBLUR_DEV float2 make(float x, float y) { return make_float2(x, y); }
};
template <> struct Cplx<double2> {
    using R = double;
    static DEBLUR_DEV double2 make(double x, double y) { return make_double2(x, y); }
};

// Twiddle table tw[m] = exp(-2 pi i m / n), m < n, from FP64 sincospi rounded
// once.  For n divisible by 8 only the first octant is evaluated and the rest
// follows exactly from the symmetries of sin and cos (swaps and sign changes).
template <typename C>
DEBLUR_DEV void twiddle_table(C* tw, int n)
{
    using R = decltype(tw[0].x);
    if (n % 8 == 0) {
        const int Q = n / 4;
        for (int m = threadIdx.x; m <= n / 8; m += blockDim.x) {
            double sd, cd;
            sincospi(2.0 * (double)m / (double)n, &sd, &cd);
            const R c = (R)cd, s = (R)sd;   // exact for R = double
            tw[m] = C{c, -s};
            tw[Q - m] = C{s, -c};
            tw[Q + m] = C{-s, -c};
            tw[2 * Q - m] = C{-c, -s};
            tw[2 * Q + m] = C{-c, s};
            tw[3 * Q - m] = C{-s, c};
            tw[3 * Q + m] = C{s, c};
            if (m > 0) tw[4 * Q - m] = C{c, s};
        }
    } else {
        for (int m = threadIdx.x; m < n; m += blockDim.x) {
            double sd, cd;
            sincospi(2.0 * (double)m / (double)n, &sd, &cd);
            tw[m] = C{(R)cd, (R)-sd};
        }
    }
}

DEBLUR_DEV void fft_twiddles(float2* tw, int n) { twiddle_table(tw, n); }
DEBLUR_DEV void fft_twiddles(double2* tw, int n) { twiddle_table(tw, n); }

template <int R, typename C>
DEBLUR_DEV void dft_small(C* v)
{
    using T = typename Cplx<C>::R;
    if constexpr (R == 2) {
        const C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 3) {
        const T c = (T)0.86602540378443864676;  // sqrt(3)/2
        const C t1 = cadd(v[1], v[2]);
        const C t2 = Cplx<C>::make(v[0].x - (T)0.5 * t1.x, v[0].y - (T)0.5 * t1.y);
        const C d = csub(v[1], v[2]);
        const C t3 = Cplx<C>::make(c * d.y, -c * d.x);  // -i * c * (v1 - v2)
        v[0] = cadd(v[0], t1);
        v[1] = cadd(t2, t3);
        v[2] = csub(t2, t3);
    } else if constexpr (R == 4) {
        const C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        const C s13 = cadd(v[1], v[3]), d13 = cmul_mi(csub(v[1], v[3]));
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    } else if constexpr (R == 8) {
        C e[4] = {v[0], v[2], v[4], v[6]};
        C o[4] = {v[1], v[3], v[5], v[7]};
        dft_small<4>(e);
        dft_small<4>(o);
        const T r = (T)0.70710678118654752440;
        const C w1 = Cplx<C>::make(r * (o[1].x + o[1].y), r * (o[1].y - o[1].x));   // (1-i)/sqrt2
        const C w2 = cmul_mi(o[2]);                                                 // -i
        const C w3 = Cplx<C>::make(r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y));  // (-1-i)/sqrt2
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], w1);
        v[5] = csub(e[1], w1);
        v[2] = cadd(e[2], w2);
        v[6] = csub(e[2], w2);
        v[3] = cadd(e[3], w3);
        v[7] = csub(e[3], w3);
    }
}

template <int R, typename C>
DEBLUR_DEV void fft_pass(const C* __restrict__ src, C* __restrict__ dst, int nb,
                         int n, int Ns, unsigned mag, const C* __restrict__ tw)
{
    const int m = n / R;
    const int tstride = n / (Ns * R);
    // butterflies of all nb rows in one index range, so that every thread has
    // work when n / R is smaller than the workgroup
    const int lm = 31 - __clz(m);
    const bool pow2 = (m & (m - 1)) == 0;
    for (int bj = threadIdx.x; bj < nb * m; bj += blockDim.x) {
        const int t = pow2 ? bj >> lm : bj / m, j = bj - t * m;
        const C* s = src + t * n;
        C* d = dst + t * n;
        // k = j mod Ns by a multiply-high (exact for j < 2^21, Ns < 2^11)
        const int k = Ns == 1 ? 0 : j - (int)__umulhi((unsigned)j, mag) * Ns;
        C v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = s[j + r * m];
        if (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[k * r * tstride]);
        }
        dft_small<R>(v);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) d[base + r * Ns] = v[r];
    }
}

// Forward FFT of nb rows of length p.n stored contiguously in `a`; `b` is a
// scratch buffer of the same size.  Returns the buffer holding the result.
// Must be called by all threads of the block; ends with a barrier.
template <typename C>
DEBLUR_DEV C* fft_rows(C* a, C* b, int nb, const FftPlan& p, const C* tw)
{
    int Ns = 1;
    for (int q = 0; q < p.npass; ++q) {
        const int R = p.radix[q];
        switch (R) {
            case 2: fft_pass<2>(a, b, nb, p.n, Ns, p.mag[q], tw); break;
            case 3: fft_pass<3>(a, b, nb, p.n, Ns, p.mag[q], tw); break;
            case 4: fft_pass<4>(a, b, nb, p.n, Ns, p.mag[q], tw); break;
            default: fft_pass<8>(a, b, nb, p.n, Ns, p.mag[q], tw); break;
        }
        __syncthreads();
        C* t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

// Radix sequence for n = 2^a 3^b: threes first, then eights, then 4 or 2.
inline FftPlan make_plan(int n)
{
    FftPlan p{};
    p.n = n;
    int m = n;
    while (m % 3 == 0) {
        p.radix[p.npass++] = 3;
        m /= 3;
    }
    while (m % 8 == 0) {
        p.radix[p.npass++] = 8;
        m /= 8;
    }
    if (m == 4) p.radix[p.npass++] = 4;
    if (m == 2) p.radix[p.npass++] = 2;
    unsigned long long ns = 1;
    for (int q = 0; q < p.npass; ++q) {
        p.mag[q] = ns > 1 ? (unsigned)(((1ull << 32) + ns - 1) / ns) : 0u;
        ns *= (unsigned long long)p.radix[q];
    }
    return p;
}

}  // namespace deblur
