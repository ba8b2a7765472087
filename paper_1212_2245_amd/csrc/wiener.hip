// Wiener filter initialisation of WR3L (Sec. 2.1 eq. (2), Sec. 3.2).
//
//   u^0 = max( Re IDFT( DFT(f) * M ), pos_floor ),  M = conj(h^) / (|h^|^2 + K)
//
// with periodic continuation (Fourier domain, Sec. 4.2).  M is formed in FP64
// (the division by |h^|^2 + K with small K) and stored as complex64; the
// transforms run in FP32 in LDS.
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

// M(k) = conj(h^(k)) / (|h^(k)|^2 + K) for a PSF on one row, k < n.
__global__ void __launch_bounds__(256) wiener_mult_1d(PsfDev psf, int n, double K, float2* __restrict__ M)
{
    __shared__ float hs[MULT_MAXP];
    psf_to_lds(psf, hs);
    __syncthreads();
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double2 hk = psf_row_dft(hs, psf.pw, unit_root(k, n), unit_root(-k * ((psf.pw - 1) / 2), n));
    const double den = hk.x * hk.x + hk.y * hk.y + K;
    M[k] = make_float2((float)(hk.x / den), (float)(-hk.y / den));
}

// One workgroup per `nb` row pairs; LDS: two ping-pong buffers of nb*n
// complex plus the twiddle table.
__global__ void __launch_bounds__(256) wiener_rows_fused(const float* __restrict__ f, float* __restrict__ u,
                                                         int H, int W, int pitch, int nb, FftPlan plan,
                                                         const float2* __restrict__ M, float pos_floor)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* tw = reinterpret_cast<float2*>(smem_raw);
    float2* a = tw + W;
    float2* b = a + nb * W;
    fft_twiddles(tw, W);

    const int pair0 = blockIdx.x * nb;
    stage_to_lds_n<8>(a, nb * W, [&](int idx) {
        const int t = idx / W, x = idx - t * W;
        const int ya = 2 * (pair0 + t), yb = ya + 1;
        const float va = ya < H ? f[(size_t)ya * pitch + x] : 0.0f;
        const float vb = yb < H ? f[(size_t)yb * pitch + x] : 0.0f;
        return make_float2(va, vb);
    });
    __syncthreads();
    float2* X = fft_rows(a, b, nb, plan, tw);
    float2* Y = X == a ? b : a;
    // Y = conj(X * M): the inverse transform is conj(FFT(conj(.)))/n
    for (int idx = threadIdx.x; idx < nb * W; idx += blockDim.x) {
        const int x = idx % W;
        X[idx] = cconj(cmul(X[idx], M[x]));
    }
    __syncthreads();
    X = fft_rows(X, Y, nb, plan, tw);
    const float inv = 1.0f / (float)W;
    for (int idx = threadIdx.x; idx < nb * W; idx += blockDim.x) {
        const int t = idx / W, x = idx - t * W;
        const int ya = 2 * (pair0 + t), yb = ya + 1;
        const float2 z = X[idx];
        if (ya < H) u[(size_t)ya * pitch + x] = fmaxf(z.x * inv, pos_floor);
        if (yb < H) u[(size_t)yb * pitch + x] = fmaxf(-z.y * inv, pos_floor);
    }
}

// M(ky, kx) for kx <= W/2, stored row-major with row pitch W/2+1 (the
// layout of the half spectra).  Workgroup = 16 consecutive kx (one 128-byte
// row segment of M per ky) x MULT_KY rows ky.  The PSF rows are first
// transformed along x, G(j, kx) = sum_i h(j, i) e^{-2 pi i kx (i - cx)/W}
// (LDS, FP64), then h^(ky, kx) = sum_j G(j, kx) e^{-2 pi i ky (j - cy)/H}.
// Optionally also h^ itself (hh, complex64).
constexpr int MULT_KX = 16, MULT_KY = 64;
__global__ void __launch_bounds__(256) wiener_mult_2d(PsfDev psf, int H, int W, double K, float2* __restrict__ M,
                                                      float2* __restrict__ hh)
{
    __shared__ double2 G[MULT_MAXP * MULT_KX];
    __shared__ float hs[MULT_MAXP * MULT_MAXP];
    __shared__ double2 rot[2 * (MULT_KX + MULT_KY)];   // per kx, ky: exp(-2 pi i k/n), exp(2 pi i k c/n)
    psf_to_lds(psf, hs);
    const int Wh = W / 2 + 1;
    const int cy = (psf.ph - 1) / 2, cx = (psf.pw - 1) / 2;
    const int kx0 = blockIdx.x * MULT_KX, ky0 = blockIdx.y * MULT_KY;
    for (int t = threadIdx.x; t < 2 * (MULT_KX + MULT_KY); t += blockDim.x) {
        const int q = t % (MULT_KX + MULT_KY), start = t >= MULT_KX + MULT_KY;
        const bool isx = q < MULT_KX;
        const int k = isx ? kx0 + q : ky0 + q - MULT_KX, n = isx ? W : H, c = isx ? cx : cy;
        rot[t] = unit_root(start ? -k * c : k, n);
    }
    __syncthreads();
    const double2* wx = rot;
    const double2* wy = rot + MULT_KX;
    const double2* tx0 = rot + MULT_KX + MULT_KY;
    const double2* ty0 = tx0 + MULT_KX;
    for (int idx = threadIdx.x; idx < psf.ph * MULT_KX; idx += blockDim.x) {
        const int j = idx / MULT_KX, q = idx % MULT_KX;
        G[idx] = kx0 + q < Wh ? psf_row_dft(hs + j * psf.pw, psf.pw, wx[q], tx0[q]) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int lx = threadIdx.x % MULT_KX, kx = kx0 + lx;
    if (kx >= Wh) return;
    for (int q = threadIdx.x / MULT_KX; q < MULT_KY && ky0 + q < H; q += 256 / MULT_KX) {
        const int ky = ky0 + q;
        const double2 w = wy[q];
        double2 t = ty0[q];
        double re = 0.0, im = 0.0;
        for (int j = 0; j < psf.ph; ++j) {
            const double2 g = G[j * MULT_KX + lx];
            re = fma(g.x, t.x, fma(-g.y, t.y, re));
            im = fma(g.x, t.y, fma(g.y, t.x, im));
            t = zmul(t, w);
        }
        const double den = re * re + im * im + K;
        M[(size_t)ky * Wh + kx] = make_float2((float)(re / den), (float)(-im / den));
        if (hh) hh[(size_t)ky * Wh + kx] = make_float2((float)re, (float)im);
    }
}

static void mult_2d_launch(const PsfDev& psf, int H, int W, double K, float2* M, float2* hh, hipStream_t st)
{
    const dim3 grid((W / 2 + 1 + MULT_KX - 1) / MULT_KX, (H + MULT_KY - 1) / MULT_KY);
    hipLaunchKernelGGL(wiener_mult_2d, grid, dim3(256), 0, st, psf, H, W, K, M, hh);
}

// Row pass: rows (2p, 2p+1) packed as z = f_a + i f_b, FFT along x, unpacked
// into the half spectra F_a(k), F_b(k), k <= W/2, written to S (row pitch W/2+1).
__global__ void __launch_bounds__(256) wiener_rows_fwd(const float* __restrict__ f, float2* __restrict__ S,
                                                       int H, int W, int pitch, int nb, FftPlan plan)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* tw = reinterpret_cast<float2*>(smem_raw);
    float2* a = tw + W;
    float2* b = a + nb * W;
    fft_twiddles(tw, W);
    const int pair0 = blockIdx.x * nb;
    stage_to_lds_n<8>(a, nb * W, [&](int idx) {
        const int t = idx / W, x = idx - t * W;
        const int ya = 2 * (pair0 + t), yb = ya + 1;
        const float va = ya < H ? f[(size_t)ya * pitch + x] : 0.0f;
        const float vb = yb < H ? f[(size_t)yb * pitch + x] : 0.0f;
        return make_float2(va, vb);
    });
    __syncthreads();
    const float2* Z = fft_rows(a, b, nb, plan, tw);
    const int Wh = W / 2 + 1;
    for (int idx = threadIdx.x; idx < nb * Wh; idx += blockDim.x) {
        const int t = idx / Wh, k = idx - t * Wh;
        const int ya = 2 * (pair0 + t), yb = ya + 1;
        const float2 zk = Z[t * W + k];
        const float2 zm = Z[t * W + (k == 0 ? 0 : W - k)];
        // F_a = (Z(k) + conj Z(-k))/2,  F_b = (Z(k) - conj Z(-k))/(2i)
        if (ya < H) S[(size_t)ya * Wh + k] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
        if (yb < H) S[(size_t)yb * Wh + k] = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
    }
}

// Column pass over `cb` consecutive columns kx of the half spectrum S (in
// place): mode 0: FFT along y, multiply by M (or conj M), inverse FFT (1/H);
// mode 1: forward FFT only; mode 2: inverse FFT only (1/H).
__global__ void __launch_bounds__(256) wiener_cols(float2* __restrict__ S, const float2* __restrict__ M,
                                                   int H, int W, int cb, FftPlan plan, int mode, int conjM)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* tw = reinterpret_cast<float2*>(smem_raw);
    float2* a = tw + H;
    float2* b = a + cb * H;
    fft_twiddles(tw, H);
    const int Wh = W / 2 + 1;
    const int c0 = xcd_group(blockIdx.x, gridDim.x) * cb;
    for (int base = threadIdx.x; base < cb * H; base += 8 * blockDim.x) {
        float2 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int idx = base + k * blockDim.x, y = idx / cb, c = idx - y * cb;
            v[k] = (idx < cb * H && c0 + c < Wh) ? S[(size_t)y * Wh + c0 + c] : make_float2(0.0f, 0.0f);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int idx = base + k * blockDim.x, y = idx / cb, c = idx - y * cb;
            if (idx < cb * H) a[c * H + y] = mode == 2 ? cconj(v[k]) : v[k];
        }
    }
    __syncthreads();
    float2* X = fft_rows(a, b, cb, plan, tw);
    if (mode == 0) {
        float2* Y = X == a ? b : a;
        for (int idx = threadIdx.x; idx < cb * H; idx += blockDim.x) {
            const int c = idx / H, y = idx - c * H;
            float2 m = (c0 + c < Wh) ? M[(size_t)y * Wh + c0 + c] : make_float2(0.0f, 0.0f);
            if (conjM) m = cconj(m);
            X[idx] = cconj(cmul(X[idx], m));
        }
        __syncthreads();
        X = fft_rows(X, Y, cb, plan, tw);
    }
    const float inv = mode == 1 ? 1.0f : 1.0f / (float)H;
    for (int idx = threadIdx.x; idx < cb * H; idx += blockDim.x) {
        const int y = idx / cb, c = idx - y * cb;
        if (c0 + c < Wh) {
            const float2 z = X[c * H + y];
            S[(size_t)y * Wh + c0 + c] = mode == 1 ? z : make_float2(z.x * inv, -z.y * inv);
        }
    }
}

// S_out = S_in * M (or conj M), elementwise on the half spectrum (S_out may
// alias S_in).
__global__ void __launch_bounds__(256) spectral_mul(const float2* Sin, const float2* __restrict__ M, int conjM,
                                                    float2* Sout, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 m = conjM ? cconj(M[i]) : M[i];
    Sout[i] = cmul(Sin[i], m);
}

// Inverse row pass: U_a, U_b extended to full length by Hermitian symmetry,
// packed as Z = U_a + i U_b, inverse FFT (scaled by 1/W): u_a = Re, u_b = Im;
// non-positive values replaced by pos_floor (Sec. 3.2).
__global__ void __launch_bounds__(256) wiener_rows_inv(const float2* __restrict__ S, float* __restrict__ u,
                                                       int H, int W, int pitch, int nb, FftPlan plan,
                                                       float pos_floor, int accumulate)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* tw = reinterpret_cast<float2*>(smem_raw);
    float2* a = tw + W;
    float2* b = a + nb * W;
    fft_twiddles(tw, W);
    const int Wh = W / 2 + 1;
    const int pair0 = blockIdx.x * nb;
    stage_to_lds_n<8>(a, nb * W, [&](int idx) {
        const int t = idx / W, k = idx - t * W;
        const int ya = 2 * (pair0 + t), yb = ya + 1;
        const bool lo = k < Wh;
        const int kk = lo ? k : W - k;
        float2 ua = ya < H ? S[(size_t)ya * Wh + kk] : make_float2(0.0f, 0.0f);
        float2 ub = yb < H ? S[(size_t)yb * Wh + kk] : make_float2(0.0f, 0.0f);
        if (!lo) {
            ua = cconj(ua);
            ub = cconj(ub);
        }
        // conj(U_a + i U_b) for the inverse via the forward transform
        return make_float2(ua.x - ub.y, -(ua.y + ub.x));
    });
    __syncthreads();
    const float2* Z = fft_rows(a, b, nb, plan, tw);
    const float inv = 1.0f / (float)W;
    for (int idx = threadIdx.x; idx < nb * W; idx += blockDim.x) {
        const int t = idx / W, x = idx - t * W;
        const int ya = 2 * (pair0 + t), yb = ya + 1;
        const float2 z = Z[idx];
        if (accumulate) {
            if (ya < H) u[(size_t)ya * pitch + x] += z.x * inv;
            if (yb < H) u[(size_t)yb * pitch + x] += -z.y * inv;
        } else {
            if (ya < H) u[(size_t)ya * pitch + x] = fmaxf(z.x * inv, pos_floor);
            if (yb < H) u[(size_t)yb * pitch + x] = fmaxf(-z.y * inv, pos_floor);
        }
    }
}

// ------------------------------------------------------------ host launchers
size_t wiener_ws_bytes(int H, int W, bool rowwise)
{
    if (rowwise) return (size_t)W * sizeof(float2);
    const size_t Wh = (size_t)W / 2 + 1;
    return 2 * (size_t)H * Wh * sizeof(float2);  // M and S
}

int launch_wiener(const float* f, float* u, int H, int W, int pitch, const PsfDev& psf, double K,
                  float pos_floor, void* ws, bool rowwise, hipStream_t st)
{
    if (rowwise) {
        float2* M = reinterpret_cast<float2*>(ws);
        hipLaunchKernelGGL(wiener_mult_1d, dim3((W + 255) / 256), dim3(256), 0, st, psf, W, K, M);
        const int pairs = (H + 1) / 2;
        const int nb = W >= 1024 ? 1 : 1024 / W;
        const size_t lds = (size_t)(W + 2 * nb * W) * sizeof(float2);
        hipLaunchKernelGGL(wiener_rows_fused, dim3((pairs + nb - 1) / nb), dim3(256), lds, st, f, u, H, W,
                           pitch, nb, make_plan(W), (const float2*)M, pos_floor);
    } else {
        const int Wh = W / 2 + 1;
        float2* M = reinterpret_cast<float2*>(ws);
        float2* S = M + (size_t)H * Wh;
        mult_2d_launch(psf, H, W, K, M, nullptr, st);
        const int pairs = (H + 1) / 2;
        const int nb = W >= 1024 ? 1 : 1024 / W;
        const size_t lds_r = (size_t)(W + 2 * nb * W) * sizeof(float2);
        hipLaunchKernelGGL(wiener_rows_fwd, dim3((pairs + nb - 1) / nb), dim3(256), lds_r, st, f, S, H, W,
                           pitch, nb, make_plan(W));
        const int cb = H >= 2048 ? 1 : (2048 / H > 8 ? 8 : 2048 / H);
        const size_t lds_c = (size_t)(H + 2 * cb * H) * sizeof(float2);
        hipLaunchKernelGGL(wiener_cols, dim3((Wh + cb - 1) / cb), dim3(256), lds_c, st, S, (const float2*)M,
                           H, W, cb, make_plan(H), 0, 0);
        hipLaunchKernelGGL(wiener_rows_inv, dim3((pairs + nb - 1) / nb), dim3(256), lds_r, st,
                           (const float2*)S, u, H, W, pitch, nb, make_plan(W), pos_floor, 0);
    }
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

static int row_batch(int W) { return W >= 1024 ? 1 : 1024 / W; }
int fft_row_batch(int W) { return row_batch(W); }
static int col_batch(int H) { return H >= 2048 ? 1 : (2048 / H > 8 ? 8 : 2048 / H); }

void launch_wiener_mult(const PsfDev& psf, int H, int W, double K, float2* M, float2* hh, hipStream_t st)
{
    mult_2d_launch(psf, H, W, K, M, hh, st);
}

void launch_fft2_forward(const float* x, int pitch, int H, int W, float2* S, hipStream_t st)
{
    const int nb = row_batch(W), cb = col_batch(H), Wh = W / 2 + 1, pairs = (H + 1) / 2;
    hipLaunchKernelGGL(wiener_rows_fwd, dim3((pairs + nb - 1) / nb), dim3(256), (size_t)(W + 2 * nb * W) * 8, st, x,
                       S, H, W, pitch, nb, make_plan(W));
    hipLaunchKernelGGL(wiener_cols, dim3((Wh + cb - 1) / cb), dim3(256), (size_t)(H + 2 * cb * H) * 8, st, S,
                       (const float2*)nullptr, H, W, cb, make_plan(H), 1, 0);
}

void launch_fft2_inverse(float2* S, int H, int W, float* out, int pitch, float floor_, bool accumulate,
                         hipStream_t st)
{
    const int nb = row_batch(W), cb = col_batch(H), Wh = W / 2 + 1, pairs = (H + 1) / 2;
    hipLaunchKernelGGL(wiener_cols, dim3((Wh + cb - 1) / cb), dim3(256), (size_t)(H + 2 * cb * H) * 8, st, S,
                       (const float2*)nullptr, H, W, cb, make_plan(H), 2, 0);
    hipLaunchKernelGGL(wiener_rows_inv, dim3((pairs + nb - 1) / nb), dim3(256), (size_t)(W + 2 * nb * W) * 8, st,
                       (const float2*)S, out, H, W, pitch, nb, make_plan(W), floor_, accumulate ? 1 : 0);
}

void launch_rows_fwd(const float* x, int pitch, int H, int W, float2* S, hipStream_t st)
{
    const int nb = row_batch(W), pairs = (H + 1) / 2;
    hipLaunchKernelGGL(wiener_rows_fwd, dim3((pairs + nb - 1) / nb), dim3(256), (size_t)(W + 2 * nb * W) * 8, st, x,
                       S, H, W, pitch, nb, make_plan(W));
}

void launch_cols(float2* S, const float2* mult, bool conj_mult, int mode, int H, int W, hipStream_t st)
{
    const int cb = col_batch(H), Wh = W / 2 + 1;
    hipLaunchKernelGGL(wiener_cols, dim3((Wh + cb - 1) / cb), dim3(256), (size_t)(H + 2 * cb * H) * 8, st, S, mult, H,
                       W, cb, make_plan(H), mode, conj_mult ? 1 : 0);
}

void launch_spectral_mul(const float2* Sin, const float2* M, bool conjM, float2* Sout, size_t n, hipStream_t st)
{
    hipLaunchKernelGGL(spectral_mul, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Sin, M, conjM ? 1 : 0,
                       Sout, n);
}

}  // namespace deblur
