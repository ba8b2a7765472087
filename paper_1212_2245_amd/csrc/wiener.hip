// Wiener filter initialisation of WR3L (Sec. 2.1 eq. (2), Sec. 3.2).
//
//   u^0 = max( Re IDFT( DFT(f) * M ), pos_floor ),  M = conj(h^) / (|h^|^2 + K)
//
// with periodic continuation (Fourier domain, Sec. 4.2).  M is formed in FP64
// (the division by |h^|^2 + K with small K).  Default: M stored as complex64,
// transforms in FP32 in LDS.  FP64 variant (complex type double2): M, the
// spectra and the transforms in FP64, the output rounded once to FP32.
//
// Two paths:
//  * PSF supported on one row (horizontal motion): the 2D filter reduces to a
//    1D filter along every row (Sec. 4.3, non-uniform linear motion).  One
//    fused kernel per pair of rows: pack z = f_a + i f_b, FFT, multiply by M
//    (Hermitian, so both real rows stay separated), inverse FFT, floor, store.
//  * general PSF: half-spectrum 2D real FFT.  Row pass (pairs of rows packed
//    as one complex row, unpacked to two half spectra), column pass (FFT,
//    multiply by M, inverse FFT), inverse row pass (Hermitian extension,
//    rows packed again, inverse FFT, floor).
#include <algorithm>
#include <mutex>

#include "fft_lds.hpp"
#include "launch.hpp"
#include "psf.hpp"

namespace deblur {

// exp(-2 pi i m / n) for an integer m reduced mod n (exact reduction, FP64).
DEBLUR_DEV double2 unit_root(int m, int n)
{
    m %= n;
    if (m < 0) m += n;
    double s, c;
    sincospi(2.0 * (double)m / (double)n, &s, &c);
    return make_double2(c, -s);
}

DEBLUR_DEV double2 zmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// The PSF array in LDS (ph*pw floats, at most 65 x 65), filled with batched
// loads so the DFT loops below read no global memory.
constexpr int MULT_MAXP = 65;
DEBLUR_DEV void psf_to_lds(const PsfDev& psf, float* hs)
{
    stage_to_lds_n<8>(hs, psf.ph * psf.pw, [&](int t) { return psf_weight(psf, t / psf.pw, t % psf.pw); });
}

// sum_i h(j, i) exp(-2 pi i k (i - c) / n) over one PSF row j (hrow = h(j, .)),
// given w = exp(-2 pi i k / n) and t0 = exp(2 pi i k c / n); the phase is
// advanced by the FP64 recurrence t <- t w (at most 65 steps: relative drift
// ~1e-14, far below the FP32 rounding of the result).
DEBLUR_DEV double2 psf_row_dft(const float* hrow, int pw, double2 w, double2 t)
{
    double re = 0.0, im = 0.0;
    for (int i = 0; i < pw; ++i) {
        const double h = (double)hrow[i];
        re = fma(h, t.x, re);
        im = fma(h, t.y, im);
        t = zmul(t, w);
    }
    return make_double2(re, im);
}

// M(k) = conj(h^(k)) / (|h^(k)|^2 + K) for a PSF on one row, k < n; one
// workgroup of 256 frequencies (block blk).
template <typename C>
DEBLUR_DEV void mult_1d_block(const PsfDev& psf, int n, double K, C* __restrict__ M, int blk, float* hs)
{
    psf_to_lds(psf, hs);
    __syncthreads();
    const int k = blk * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double2 hk = psf_row_dft(hs, psf.pw, unit_root(k, n), unit_root(-k * ((psf.pw - 1) / 2), n));
    const double den = hk.x * hk.x + hk.y * hk.y + K;
    using R = typename Cplx<C>::R;
    M[k] = Cplx<C>::make((R)(hk.x / den), (R)(-hk.y / den));
}

// Kernels of the one-image path also run over a batch of equally shaped
// images (blockIdx.z = image): image z's f and u at z img bytes, its PSF
// taps at z taps bytes, its workspace (M, S) at z ws bytes from image 0's.
struct WienerZ {
    size_t img, taps, ws;
};

template <typename C>
__global__ void __launch_bounds__(256) wiener_mult_1d(PsfDev psf, int n, double K, C* __restrict__ M, WienerZ z)
{
    __shared__ float hs[MULT_MAXP];
    if (psf.taps) psf.taps = zadv(psf.taps, z.taps);
    mult_1d_block<C>(psf, n, K, zadv(M, z.ws), blockIdx.x, hs);
}

// One workgroup per `nb` row pairs (block blk); LDS: two ping-pong buffers
// of nb*n complex plus the twiddle table.
template <typename C>
DEBLUR_DEV void rows_fused_block(const float* __restrict__ f, float* __restrict__ u, int H, int W, int pitch, int nb,
                                 const FftPlan& plan, const C* __restrict__ M, float pos_floor, int blk,
                                 unsigned char* smem_raw)
{
    using R = typename Cplx<C>::R;
    C* tw = reinterpret_cast<C*>(smem_raw);
    C* a = tw + W;
    C* b = a + nb * W;
    fft_twiddles(tw, W);

    const int pair0 = blk * nb;
    stage_to_lds_n<8>(a, nb * W, [&](int idx) {
        const int t = idx / W, x = idx - t * W;
        const int ya = 2 * (pair0 + t), yb = ya + 1;
        const float va = ya < H ? f[(size_t)ya * pitch + x] : 0.0f;
        const float vb = yb < H ? f[(size_t)yb * pitch + x] : 0.0f;
        return Cplx<C>::make((R)va, (R)vb);
    });
    __syncthreads();
    C* X = fft_rows(a, b, nb, plan, tw);
    C* Y = X == a ? b : a;
    // Y = conj(X * M): the inverse transform is conj(FFT(conj(.)))/n
    for (int idx = threadIdx.x; idx < nb * W; idx += blockDim.x) {
        const int x = idx % W;
        X[idx] = cconj(cmul(X[idx], M[x]));
    }
    __syncthreads();
    X = fft_rows(X, Y, nb, plan, tw);
    const R inv = (R)1 / (R)W;
    for (int idx = threadIdx.x; idx < nb * W; idx += blockDim.x) {
        const int t = idx / W, x = idx - t * W;
        const int ya = 2 * (pair0 + t), yb = ya + 1;
        const C z = X[idx];
        if (ya < H) u[(size_t)ya * pitch + x] = fmaxf((float)(z.x * inv), pos_floor);
        if (yb < H) u[(size_t)yb * pitch + x] = fmaxf((float)(-z.y * inv), pos_floor);
    }
}

template <typename C>
__global__ void __launch_bounds__(256) wiener_rows_fused(const float* __restrict__ f, float* __restrict__ u,
                                                         int H, int W, int pitch, int nb, FftPlan plan,
                                                         const C* __restrict__ M, float pos_floor, WienerZ z)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    rows_fused_block<C>(zadv(f, z.img), zadv(u, z.img), H, W, pitch, nb, plan, zadv(M, z.ws), pos_floor, blockIdx.x,
                        smem_raw);
}

// M(ky, kx) for kx <= W/2, stored row-major with row pitch W/2+1 (the
// layout of the half spectra).  Workgroup = 16 consecutive kx (one 128-byte
// row segment of M per ky) x MULT_KY rows ky.  The PSF sides are odd, so the
// taps at offsets +d and -d from the centre pair up under one cosine and one
// sine: with phi = 2 pi kx / W,
//   G(j, kx) = h(j, cx) + sum_{e>=1} [(h(j,cx+e) + h(j,cx-e)) cos(phi e)
//                                  - i (h(j,cx+e) - h(j,cx-e)) sin(phi e)]
// and with theta = 2 pi ky / H, P_d = G(cy+d) + G(cy-d), Q_d = G(cy+d) - G(cy-d),
//   h^(ky, kx) = G(cy, kx) + sum_{d>=1} [P_d cos(theta d) - i Q_d sin(theta d)],
// in FP64, the cosines and sines advanced by the rotation recurrence from
// the exact first root (at most 32 steps).  Optionally also h^ itself (hh).
constexpr int MULT_KX = 16, MULT_KY = 64;
constexpr int MULT_HALF = (MULT_MAXP - 1) / 2;
// LDS of one multiplier block: G, P/Q, the PSF, the roots (16-byte aligned parts)
constexpr size_t MULT_G_OFF = 0, MULT_PQ_OFF = MULT_G_OFF + sizeof(double2) * MULT_MAXP * MULT_KX,
                 MULT_HS_OFF = MULT_PQ_OFF + sizeof(double2) * 2 * MULT_HALF * MULT_KX,
                 MULT_ROT_OFF = (MULT_HS_OFF + sizeof(float) * MULT_MAXP * MULT_MAXP + 15) & ~(size_t)15,
                 MULT_SMEM = MULT_ROT_OFF + sizeof(double2) * (MULT_KX + MULT_KY);

// One block (bx, by) of M: kx in [16 bx, 16 bx + 16), ky in [64 by, 64 by + 64).
template <typename C>
DEBLUR_DEV void mult_2d_block(const PsfDev& psf, int H, int W, double K, C* __restrict__ M,
                              float2* __restrict__ hh, int bx, int by, unsigned char* smem)
{
    using R = typename Cplx<C>::R;
    double2* G = reinterpret_cast<double2*>(smem + MULT_G_OFF);
    double2* PQ = reinterpret_cast<double2*>(smem + MULT_PQ_OFF);
    float* hs = reinterpret_cast<float*>(smem + MULT_HS_OFF);
    double2* rot = reinterpret_cast<double2*>(smem + MULT_ROT_OFF);   // exp(-2 pi i k / n) per kx, then per ky
    psf_to_lds(psf, hs);
    const int Wh = W / 2 + 1;
    const int cy = (psf.ph - 1) / 2, cx = (psf.pw - 1) / 2;
    const int kx0 = bx * MULT_KX, ky0 = by * MULT_KY;
    for (int t = threadIdx.x; t < MULT_KX + MULT_KY; t += blockDim.x)
        rot[t] = t < MULT_KX ? unit_root(kx0 + t, W) : unit_root(ky0 + t - MULT_KX, H);
    __syncthreads();
    // G(j, kx): two PSF rows per thread, their sums interleaved
    for (int idx = threadIdx.x; idx < psf.ph * MULT_KX; idx += 2 * blockDim.x) {
        const int q = idx % MULT_KX, j0 = idx / MULT_KX, j1 = j0 + (int)blockDim.x / MULT_KX;
        const bool two = j1 < psf.ph;
        const float* h0 = hs + j0 * psf.pw + cx;
        const float* h1 = hs + (two ? j1 : j0) * psf.pw + cx;
        const double c1 = rot[q].x, s1 = -rot[q].y;
        double c = c1, s = s1;
        double r0 = (double)h0[0], i0 = 0.0, r1 = (double)h1[0], i1 = 0.0;
        for (int e = 1; e <= cx; ++e) {
            r0 = fma((double)h0[e] + (double)h0[-e], c, r0);
            i0 = fma((double)h0[-e] - (double)h0[e], s, i0);
            r1 = fma((double)h1[e] + (double)h1[-e], c, r1);
            i1 = fma((double)h1[-e] - (double)h1[e], s, i1);
            const double cn = fma(c, c1, -s * s1);
            s = fma(s, c1, c * s1);
            c = cn;
        }
        const bool on = kx0 + q < Wh;
        G[idx] = on ? make_double2(r0, i0) : make_double2(0.0, 0.0);
        if (two) G[j1 * MULT_KX + q] = on ? make_double2(r1, i1) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < cy * MULT_KX; idx += blockDim.x) {
        const int d = idx / MULT_KX + 1, q = idx % MULT_KX;
        const double2 gp = G[(cy + d) * MULT_KX + q], gm = G[(cy - d) * MULT_KX + q];
        PQ[2 * idx] = make_double2(gp.x + gm.x, gp.y + gm.y);
        PQ[2 * idx + 1] = make_double2(gp.x - gm.x, gp.y - gm.y);
    }
    __syncthreads();
    const int lx = threadIdx.x % MULT_KX, kx = kx0 + lx;
    if (kx >= Wh) return;
    // NQ rows ky per thread (ky0 + q0 + r * 16), their sums interleaved;
    // P_d, Q_d are read once for all NQ
    constexpr int NQ = MULT_KY / (256 / MULT_KX);
    const int q0 = threadIdx.x / MULT_KX;
    const double2 g0 = G[cy * MULT_KX + lx];
    double c1[NQ], s1[NQ], c[NQ], s[NQ], re[NQ], im[NQ];
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
        const double2 w = rot[MULT_KX + q0 + r * (256 / MULT_KX)];
        c1[r] = c[r] = w.x;
        s1[r] = s[r] = -w.y;
        re[r] = g0.x;
        im[r] = g0.y;
    }
    for (int d = 1; d <= cy; ++d) {
        const double2 P = PQ[2 * ((d - 1) * MULT_KX + lx)], Q = PQ[2 * ((d - 1) * MULT_KX + lx) + 1];
#pragma unroll
        for (int r = 0; r < NQ; ++r) {
            re[r] = fma(P.x, c[r], fma(Q.y, s[r], re[r]));
            im[r] = fma(P.y, c[r], fma(-Q.x, s[r], im[r]));
            const double cn = fma(c[r], c1[r], -s[r] * s1[r]);
            s[r] = fma(s[r], c1[r], c[r] * s1[r]);
            c[r] = cn;
        }
    }
#pragma unroll
    for (int r = 0; r < NQ; ++r) {
        const int ky = ky0 + q0 + r * (256 / MULT_KX);
        if (ky >= H) break;
        const double inv = 1.0 / (re[r] * re[r] + im[r] * im[r] + K);
        M[(size_t)ky * Wh + kx] = Cplx<C>::make((R)(re[r] * inv), (R)(-im[r] * inv));
        if (hh) hh[(size_t)ky * Wh + kx] = make_float2((float)re[r], (float)im[r]);
    }
}

// blockIdx.z = image of a batch (strides of the taps, M and h^ in bytes)
__global__ void __launch_bounds__(256) wiener_mult_2d(PsfDev psf, int H, int W, double K, float2* __restrict__ M,
                                                      float2* __restrict__ hh, size_t zt, size_t zm, size_t zh)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (psf.taps) psf.taps = zadv(psf.taps, zt);
    mult_2d_block<float2>(psf, H, W, K, zadv(M, zm), hh ? zadv(hh, zh) : nullptr, blockIdx.x, blockIdx.y, smem_raw);
}

static void mult_2d_launch(const PsfDev& psf, int H, int W, double K, float2* M, float2* hh, hipStream_t st,
                           ZBatch zb)
{
    const dim3 grid((W / 2 + 1 + MULT_KX - 1) / MULT_KX, (H + MULT_KY - 1) / MULT_KY, zb.n);
    hipLaunchKernelGGL(wiener_mult_2d, grid, dim3(256), MULT_SMEM, st, psf, H, W, K, M, hh, zb.s0, zb.s1, zb.s2);
}

// Row pass: rows (2p, 2p+1) packed as z = f_a + i f_b, FFT along x, unpacked
// into the half spectra F_a(k), F_b(k), k <= W/2, written to S (row pitch W/2+1).
template <typename C>
DEBLUR_DEV void rows_fwd_block(const float* __restrict__ f, C* __restrict__ S, int H, int W, int pitch, int nb,
                               const FftPlan& plan, int blk, unsigned char* smem_raw)
{
    using R = typename Cplx<C>::R;
    C* tw = reinterpret_cast<C*>(smem_raw);
    C* a = tw + W;
    C* b = a + nb * W;
    fft_twiddles(tw, W);
    const int pair0 = blk * nb;
    stage_to_lds_n<8>(a, nb * W, [&](int idx) {
        const int t = idx / W, x = idx - t * W;
        const int ya = 2 * (pair0 + t), yb = ya + 1;
        const float va = ya < H ? f[(size_t)ya * pitch + x] : 0.0f;
        const float vb = yb < H ? f[(size_t)yb * pitch + x] : 0.0f;
        return Cplx<C>::make((R)va, (R)vb);
    });
    __syncthreads();
    const C* Z = fft_rows(a, b, nb, plan, tw);
    const int Wh = W / 2 + 1;
    for (int idx = threadIdx.x; idx < nb * Wh; idx += blockDim.x) {
        const int t = idx / Wh, k = idx - t * Wh;
        const int ya = 2 * (pair0 + t), yb = ya + 1;
        const C zk = Z[t * W + k];
        const C zm = Z[t * W + (k == 0 ? 0 : W - k)];
        // F_a = (Z(k) + conj Z(-k))/2,  F_b = (Z(k) - conj Z(-k))/(2i)
        const R h = (R)0.5;
        if (ya < H) S[(size_t)ya * Wh + k] = Cplx<C>::make(h * (zk.x + zm.x), h * (zk.y - zm.y));
        if (yb < H) S[(size_t)yb * Wh + k] = Cplx<C>::make(h * (zk.y + zm.y), -h * (zk.x - zm.x));
    }
}

template <typename C>
__global__ void __launch_bounds__(256) wiener_rows_fwd(const float* __restrict__ f, C* __restrict__ S,
                                                       int H, int W, int pitch, int nb, FftPlan plan, size_t zf,
                                                       size_t zs)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    rows_fwd_block(zadv(f, zf), zadv(S, zs), H, W, pitch, nb, plan, blockIdx.x, smem_raw);
}

// The row pass of f and the multiplier M in one launch: they are independent,
// and as one grid (row blocks first, then the M blocks) they overlap without
// a second stream.  LDS: the larger of the two needs.
template <typename C>
__global__ void __launch_bounds__(256) wiener_rows_fwd_mult(const float* __restrict__ f, C* __restrict__ S,
                                                            int H, int W, int pitch, int nb, FftPlan plan, int nrow,
                                                            PsfDev psf, double K, C* __restrict__ M, int gxm,
                                                            WienerZ z)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    f = zadv(f, z.img);
    S = zadv(S, z.ws);
    M = zadv(M, z.ws);
    if (psf.taps) psf.taps = zadv(psf.taps, z.taps);
    if ((int)blockIdx.x < nrow) {
        rows_fwd_block(f, S, H, W, pitch, nb, plan, blockIdx.x, smem_raw);
    } else {
        const int b = blockIdx.x - nrow, by = b / gxm;
        mult_2d_block<C>(psf, H, W, K, M, nullptr, b - by * gxm, by, smem_raw);
    }
}

// Column pass over `cb` consecutive columns kx of the half spectrum S (in
// place): mode 0: FFT along y, multiply by M (or conj M), inverse FFT (1/H);
// mode 1: forward FFT only; mode 2: inverse FFT only (1/H).
template <typename C>
DEBLUR_DEV void cols_block(C* __restrict__ S, const C* __restrict__ M, int H, int W, int cb, const FftPlan& plan,
                           int mode, int conjM, int blk, unsigned char* smem_raw)
{
    using R = typename Cplx<C>::R;
    C* tw = reinterpret_cast<C*>(smem_raw);
    C* a = tw + H;
    C* b = a + cb * H;
    fft_twiddles(tw, H);
    const int Wh = W / 2 + 1;
    const int c0 = blk * cb;
    // With at most 8 elements per thread, the multiplier M of the thread's
    // elements is fetched together with S, so its latency is not paid after
    // the forward transform.
    const bool pre = mode == 0 && cb * H <= 8 * (int)blockDim.x;
    const C zero = Cplx<C>::make((R)0, (R)0);
    C mv[8];
    for (int base = threadIdx.x; base < cb * H; base += 8 * blockDim.x) {
        C v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int idx = base + k * blockDim.x, y = idx / cb, c = idx - y * cb;
            const bool ok = idx < cb * H && c0 + c < Wh;
            v[k] = ok ? S[(size_t)y * Wh + c0 + c] : zero;
            if (pre) mv[k] = ok ? M[(size_t)y * Wh + c0 + c] : zero;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int idx = base + k * blockDim.x, y = idx / cb, c = idx - y * cb;
            if (idx < cb * H) a[c * H + y] = mode == 2 ? cconj(v[k]) : v[k];
        }
    }
    __syncthreads();
    C* X = fft_rows(a, b, cb, plan, tw);
    if (mode == 0) {
        C* Y = X == a ? b : a;
        if (pre) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int idx = threadIdx.x + k * blockDim.x, y = idx / cb, c = idx - y * cb;
                if (idx < cb * H) X[c * H + y] = cconj(cmul(X[c * H + y], conjM ? cconj(mv[k]) : mv[k]));
            }
        } else {
            for (int idx = threadIdx.x; idx < cb * H; idx += blockDim.x) {
                const int c = idx / H, y = idx - c * H;
                C m = (c0 + c < Wh) ? M[(size_t)y * Wh + c0 + c] : zero;
                if (conjM) m = cconj(m);
                X[idx] = cconj(cmul(X[idx], m));
            }
        }
        __syncthreads();
        X = fft_rows(X, Y, cb, plan, tw);
    }
    const R inv = mode == 1 ? (R)1 : (R)1 / (R)H;
    for (int idx = threadIdx.x; idx < cb * H; idx += blockDim.x) {
        const int y = idx / cb, c = idx - y * cb;
        if (c0 + c < Wh) {
            const C z = X[c * H + y];
            S[(size_t)y * Wh + c0 + c] = mode == 1 ? z : Cplx<C>::make(z.x * inv, -z.y * inv);
        }
    }
}

// Column blocks in an XCD-aware order (the blocks of one XCD take adjacent
// columns, which share cache lines of S).
template <typename C>
__global__ void __launch_bounds__(256) wiener_cols(C* __restrict__ S, const C* __restrict__ M,
                                                   int H, int W, int cb, FftPlan plan, int mode, int conjM,
                                                   size_t zs, size_t zm)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cols_block<C>(zadv(S, zs), M ? zadv(M, zm) : nullptr, H, W, cb, plan, mode, conjM,
                  xcd_group(blockIdx.x, gridDim.x), smem_raw);
}

// S_out = S_in * M (or conj M), elementwise on the half spectrum (S_out may
// alias S_in).
__global__ void __launch_bounds__(256) spectral_mul(const float2* Sin, const float2* __restrict__ M, int conjM,
                                                    float2* Sout, size_t n, size_t z0, size_t z1, size_t z2)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Sin = zadv(Sin, z0);
    M = zadv(M, z1);
    Sout = zadv(Sout, z2);
    const float2 m = conjM ? cconj(M[i]) : M[i];
    Sout[i] = cmul(Sin[i], m);
}

// Inverse row pass: U_a, U_b extended to full length by Hermitian symmetry,
// packed as Z = U_a + i U_b, inverse FFT (scaled by 1/W): u_a = Re, u_b = Im;
// non-positive values replaced by pos_floor (Sec. 3.2).
template <typename C>
DEBLUR_DEV void rows_inv_block(const C* __restrict__ S, float* __restrict__ u, int H, int W, int pitch, int nb,
                               const FftPlan& plan, float pos_floor, int accumulate, int blk, unsigned char* smem_raw)
{
    using R = typename Cplx<C>::R;
    C* tw = reinterpret_cast<C*>(smem_raw);
    C* a = tw + W;
    C* b = a + nb * W;
    fft_twiddles(tw, W);
    const int Wh = W / 2 + 1;
    const int pair0 = blk * nb;
    stage_to_lds_n<8>(a, nb * W, [&](int idx) {
        const int t = idx / W, k = idx - t * W;
        const int ya = 2 * (pair0 + t), yb = ya + 1;
        const bool lo = k < Wh;
        const int kk = lo ? k : W - k;
        const C zero = Cplx<C>::make((R)0, (R)0);
        C ua = ya < H ? S[(size_t)ya * Wh + kk] : zero;
        C ub = yb < H ? S[(size_t)yb * Wh + kk] : zero;
        if (!lo) {
            ua = cconj(ua);
            ub = cconj(ub);
        }
        // conj(U_a + i U_b) for the inverse via the forward transform
        return Cplx<C>::make(ua.x - ub.y, -(ua.y + ub.x));
    });
    __syncthreads();
    const C* Z = fft_rows(a, b, nb, plan, tw);
    const R inv = (R)1 / (R)W;
    for (int idx = threadIdx.x; idx < nb * W; idx += blockDim.x) {
        const int t = idx / W, x = idx - t * W;
        const int ya = 2 * (pair0 + t), yb = ya + 1;
        const C z = Z[idx];
        if (accumulate) {
            if (ya < H) u[(size_t)ya * pitch + x] += (float)(z.x * inv);
            if (yb < H) u[(size_t)yb * pitch + x] += (float)(-z.y * inv);
        } else {
            if (ya < H) u[(size_t)ya * pitch + x] = fmaxf((float)(z.x * inv), pos_floor);
            if (yb < H) u[(size_t)yb * pitch + x] = fmaxf((float)(-z.y * inv), pos_floor);
        }
    }
}

template <typename C>
__global__ void __launch_bounds__(256) wiener_rows_inv(const C* __restrict__ S, float* __restrict__ u,
                                                       int H, int W, int pitch, int nb, FftPlan plan,
                                                       float pos_floor, int accumulate, size_t zs, size_t zu)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    rows_inv_block<C>(zadv(S, zs), zadv(u, zu), H, W, pitch, nb, plan, pos_floor, accumulate, blockIdx.x, smem_raw);
}

// ------------------------------------------------- batched form (FP32)
// Many images of one size and one path in one launch: blockIdx.y selects the
// image's job, blockIdx.x the block within the image, as in the one-image
// kernels (the same block bodies, so the results are the same bit for bit).
template <typename C>
__global__ void __launch_bounds__(256) wiener_mult_1d_b(const WienerJob* __restrict__ jobs, int n)
{
    __shared__ float hs[MULT_MAXP];
    const WienerJob& j = jobs[blockIdx.y];
    mult_1d_block<C>(j.psf, n, j.K, reinterpret_cast<C*>(j.ws), blockIdx.x, hs);
}

template <typename C>
__global__ void __launch_bounds__(256) wiener_rows_fused_b(const WienerJob* __restrict__ jobs, int H, int W, int nb,
                                                           FftPlan plan)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const WienerJob& j = jobs[blockIdx.y];
    rows_fused_block<C>(j.f, j.u, H, W, j.pitch, nb, plan, reinterpret_cast<const C*>(j.ws), j.pos_floor, blockIdx.x,
                        smem_raw);
}

template <typename C>
__global__ void __launch_bounds__(256) wiener_rows_fwd_mult_b(const WienerJob* __restrict__ jobs, int H, int W,
                                                              int nb, FftPlan plan, int nrow, int gxm)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const WienerJob& j = jobs[blockIdx.y];
    C* M = reinterpret_cast<C*>(j.ws);
    C* S = M + (size_t)H * (W / 2 + 1);
    if ((int)blockIdx.x < nrow) {
        rows_fwd_block(j.f, S, H, W, j.pitch, nb, plan, blockIdx.x, smem_raw);
    } else {
        const int b = blockIdx.x - nrow, by = b / gxm;
        mult_2d_block<C>(j.psf, H, W, j.K, M, nullptr, b - by * gxm, by, smem_raw);
    }
}

template <typename C>
__global__ void __launch_bounds__(256) wiener_cols_b(const WienerJob* __restrict__ jobs, int H, int W, int cb,
                                                     FftPlan plan)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const WienerJob& j = jobs[blockIdx.y];
    C* M = reinterpret_cast<C*>(j.ws);
    C* S = M + (size_t)H * (W / 2 + 1);
    cols_block<C>(S, M, H, W, cb, plan, 0, 0, xcd_group(blockIdx.x, gridDim.x), smem_raw);
}

template <typename C>
__global__ void __launch_bounds__(256) wiener_rows_inv_b(const WienerJob* __restrict__ jobs, int H, int W, int nb,
                                                         FftPlan plan)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const WienerJob& j = jobs[blockIdx.y];
    const C* S = reinterpret_cast<const C*>(j.ws) + (size_t)H * (W / 2 + 1);
    rows_inv_block<C>(S, j.u, H, W, j.pitch, nb, plan, j.pos_floor, 0, blockIdx.x, smem_raw);
}

// ------------------------------------------------------------ host launchers
// Rows (pairs) and columns per workgroup of the transform passes: as few as
// keep a workgroup's threads busy, so that small images still spread over
// many workgroups (the passes are latency bound at these sizes).
static int row_batch(int W) { return W >= 256 ? 1 : 256 / W; }
static int col_batch(int H) { return H >= 512 ? 1 : (512 / H > 8 ? 8 : 512 / H); }
size_t wiener_ws_bytes(int H, int W, bool rowwise, bool fp64)
{
    const size_t cs = fp64 ? sizeof(double2) : sizeof(float2);
    if (rowwise) return (size_t)W * cs;
    const size_t Wh = (size_t)W / 2 + 1;
    return 2 * (size_t)H * Wh * cs;  // M and S
}

// FP64 transforms of 2048 points need more than 64 KB of LDS per workgroup;
// the limit is raised once per kernel.
template <typename K>
static void allow_lds(K* kernel)
{
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
}

template <typename C>
static void allow_wiener_lds()
{
    static std::once_flag once;
    std::call_once(once, [] {
        allow_lds(&wiener_rows_fused<C>);
        allow_lds(&wiener_rows_fwd_mult<C>);
        allow_lds(&wiener_cols<C>);
        allow_lds(&wiener_rows_inv<C>);
        allow_lds(&wiener_rows_fused_b<C>);
        allow_lds(&wiener_rows_fwd_mult_b<C>);
        allow_lds(&wiener_cols_b<C>);
        allow_lds(&wiener_rows_inv_b<C>);
    });
}

void prepare_wiener_kernels()
{
    allow_wiener_lds<float2>();
    allow_wiener_lds<double2>();
}

template <typename C>
static int launch_wiener_t(int B, const float* f, float* u, int H, int W, int pitch, const PsfDev& psf, double K,
                           float pos_floor, void* ws, bool rowwise, const WienerZ& z, hipStream_t st)
{
    allow_wiener_lds<C>();
    if (rowwise) {
        C* M = reinterpret_cast<C*>(ws);
        hipLaunchKernelGGL(wiener_mult_1d<C>, dim3((W + 255) / 256, 1, B), dim3(256), 0, st, psf, W, K, M, z);
        const int pairs = (H + 1) / 2;
        const int nb = row_batch(W);
        const size_t lds = (size_t)(W + 2 * nb * W) * sizeof(C);
        hipLaunchKernelGGL(wiener_rows_fused<C>, dim3((pairs + nb - 1) / nb, 1, B), dim3(256), lds, st, f, u, H, W,
                           pitch, nb, make_plan(W), (const C*)M, pos_floor, z);
    } else {
        const int Wh = W / 2 + 1;
        C* M = reinterpret_cast<C*>(ws);
        C* S = M + (size_t)H * Wh;
        const int pairs = (H + 1) / 2;
        const int nb = row_batch(W);
        const size_t lds_r = (size_t)(W + 2 * nb * W) * sizeof(C);
        const int nrow = (pairs + nb - 1) / nb;
        const int gxm = (Wh + MULT_KX - 1) / MULT_KX, gym = (H + MULT_KY - 1) / MULT_KY;
        hipLaunchKernelGGL(wiener_rows_fwd_mult<C>, dim3(nrow + gxm * gym, 1, B), dim3(256), std::max(lds_r, MULT_SMEM),
                           st, f, S, H, W, pitch, nb, make_plan(W), nrow, psf, K, M, gxm, z);
        const int cb = col_batch(H);
        const size_t lds_c = (size_t)(H + 2 * cb * H) * sizeof(C);
        hipLaunchKernelGGL(wiener_cols<C>, dim3((Wh + cb - 1) / cb, 1, B), dim3(256), lds_c, st, S, (const C*)M,
                           H, W, cb, make_plan(H), 0, 0, z.ws, z.ws);
        hipLaunchKernelGGL(wiener_rows_inv<C>, dim3((pairs + nb - 1) / nb, 1, B), dim3(256), lds_r, st,
                           (const C*)S, u, H, W, pitch, nb, make_plan(W), pos_floor, 0, z.ws, z.img);
    }
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

// The Wiener steps of n images of one size H x W and one path (jobs: device
// array of n descriptors, each with its own workspace of wiener_ws_bytes),
// FP32 transforms: one launch per kernel of the one-image form.
int launch_wiener_batch(const WienerJob* jobs, int n, int H, int W, bool rowwise, hipStream_t st)
{
    using C = float2;
    allow_wiener_lds<C>();
    const int pairs = (H + 1) / 2, nb = row_batch(W);
    const size_t lds_r = (size_t)(W + 2 * nb * W) * sizeof(C);
    if (rowwise) {
        hipLaunchKernelGGL(wiener_mult_1d_b<C>, dim3((W + 255) / 256, n), dim3(256), 0, st, jobs, W);
        hipLaunchKernelGGL(wiener_rows_fused_b<C>, dim3((pairs + nb - 1) / nb, n), dim3(256), lds_r, st, jobs, H, W,
                           nb, make_plan(W));
    } else {
        const int Wh = W / 2 + 1;
        const int nrow = (pairs + nb - 1) / nb;
        const int gxm = (Wh + MULT_KX - 1) / MULT_KX, gym = (H + MULT_KY - 1) / MULT_KY;
        hipLaunchKernelGGL(wiener_rows_fwd_mult_b<C>, dim3(nrow + gxm * gym, n), dim3(256), std::max(lds_r, MULT_SMEM),
                           st, jobs, H, W, nb, make_plan(W), nrow, gxm);
        const int cb = col_batch(H);
        hipLaunchKernelGGL(wiener_cols_b<C>, dim3((Wh + cb - 1) / cb, n), dim3(256), (size_t)(H + 2 * cb * H) * sizeof(C),
                           st, jobs, H, W, cb, make_plan(H));
        hipLaunchKernelGGL(wiener_rows_inv_b<C>, dim3((pairs + nb - 1) / nb, n), dim3(256), lds_r, st, jobs, H, W, nb,
                           make_plan(W));
    }
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_wiener(const float* f, float* u, int H, int W, int pitch, const PsfDev& psf, double K,
                  float pos_floor, void* ws, bool rowwise, bool fp64, hipStream_t st)
{
    return launch_wiener_z(1, f, u, H, W, pitch, 0, psf, 0, K, pos_floor, ws, 0, rowwise, fp64, st);
}

int launch_wiener_z(int B, const float* f, float* u, int H, int W, int pitch, size_t img_stride, const PsfDev& psf,
                    size_t taps_stride, double K, float pos_floor, void* ws, size_t ws_stride, bool rowwise, bool fp64,
                    hipStream_t st)
{
    const WienerZ z{img_stride, taps_stride, ws_stride};
    return fp64 ? launch_wiener_t<double2>(B, f, u, H, W, pitch, psf, K, pos_floor, ws, rowwise, z, st)
                : launch_wiener_t<float2>(B, f, u, H, W, pitch, psf, K, pos_floor, ws, rowwise, z, st);
}

int fft_row_batch(int W) { return row_batch(W); }

void launch_wiener_mult(const PsfDev& psf, int H, int W, double K, float2* M, float2* hh, hipStream_t st,
                        ZBatch zb)
{
    mult_2d_launch(psf, H, W, K, M, hh, st, zb);
}

void launch_fft2_forward(const float* x, int pitch, int H, int W, float2* S, hipStream_t st, ZBatch zb)
{
    const int nb = row_batch(W), cb = col_batch(H), Wh = W / 2 + 1, pairs = (H + 1) / 2;
    hipLaunchKernelGGL(wiener_rows_fwd<float2>, dim3((pairs + nb - 1) / nb, 1, zb.n), dim3(256),
                       (size_t)(W + 2 * nb * W) * 8, st, x, S, H, W, pitch, nb, make_plan(W), zb.s0, zb.s1);
    hipLaunchKernelGGL(wiener_cols<float2>, dim3((Wh + cb - 1) / cb, 1, zb.n), dim3(256), (size_t)(H + 2 * cb * H) * 8,
                       st, S, (const float2*)nullptr, H, W, cb, make_plan(H), 1, 0, zb.s1, (size_t)0);
}

void launch_fft2_inverse(float2* S, int H, int W, float* out, int pitch, float floor_, bool accumulate,
                         hipStream_t st, ZBatch zb)
{
    const int nb = row_batch(W), cb = col_batch(H), Wh = W / 2 + 1, pairs = (H + 1) / 2;
    hipLaunchKernelGGL(wiener_cols<float2>, dim3((Wh + cb - 1) / cb, 1, zb.n), dim3(256), (size_t)(H + 2 * cb * H) * 8,
                       st, S, (const float2*)nullptr, H, W, cb, make_plan(H), 2, 0, zb.s0, (size_t)0);
    hipLaunchKernelGGL(wiener_rows_inv<float2>, dim3((pairs + nb - 1) / nb, 1, zb.n), dim3(256),
                       (size_t)(W + 2 * nb * W) * 8, st, (const float2*)S, out, H, W, pitch, nb, make_plan(W), floor_,
                       accumulate ? 1 : 0, zb.s0, zb.s1);
}

void launch_rows_fwd(const float* x, int pitch, int H, int W, float2* S, hipStream_t st)
{
    const int nb = row_batch(W), pairs = (H + 1) / 2;
    hipLaunchKernelGGL(wiener_rows_fwd<float2>, dim3((pairs + nb - 1) / nb), dim3(256), (size_t)(W + 2 * nb * W) * 8, st, x,
                       S, H, W, pitch, nb, make_plan(W), (size_t)0, (size_t)0);
}

void launch_cols(float2* S, const float2* mult, bool conj_mult, int mode, int H, int W, hipStream_t st)
{
    const int cb = col_batch(H), Wh = W / 2 + 1;
    hipLaunchKernelGGL(wiener_cols<float2>, dim3((Wh + cb - 1) / cb), dim3(256), (size_t)(H + 2 * cb * H) * 8, st, S, mult, H,
                       W, cb, make_plan(H), mode, conj_mult ? 1 : 0, (size_t)0, (size_t)0);
}

void launch_spectral_mul(const float2* Sin, const float2* M, bool conjM, float2* Sout, size_t n, hipStream_t st,
                         ZBatch zb)
{
    hipLaunchKernelGGL(spectral_mul, dim3((unsigned)((n + 255) / 256), 1, zb.n), dim3(256), 0, st, Sin, M,
                       conjM ? 1 : 0, Sout, n, zb.s0, zb.s1, zb.s2);
}

}  // namespace deblur
