// RRRL iteration (Sec. 2.3, eqs. (9)-(12)) with the convolutions evaluated in
// the Fourier domain (Sec. 4.3, general 2D setting), which implies periodic
// continuation (Sec. 4.2).  Cost per iteration is independent of the PSF size:
//   s = IDFT(DFT(u) h^)                    rows_fwd, cols (x h^), rows_inv + weights
//   W = Phi'(r_f(s)), q = W f / s           (fused into the inverse row pass)
//   (Bq, BW) = IDFT(DFT(q, W) conj(h^))     q and W packed as one complex row
//   D(u), u' = u (N1 + a[D]_+)/(N2 - a[D]_-) tile kernel (zero-flux diffusion)
// h^ (the DFT of the centred PSF) is formed once per call in FP64.
#include "common.hpp"
#include "fft_lds.hpp"
#include "launch.hpp"
#include "psf.hpp"

namespace deblur {

// Inverse row pass of the blurred image s (pairs of rows, Hermitian
// extension as in the Wiener inverse pass), followed by the robust weight and
// quotient: q, W planes (dense H x W).
__global__ void __launch_bounds__(256) fftp_rows_inv_weights(const float2* __restrict__ S, const float* __restrict__ f,
                                                             float* __restrict__ qo, float* __restrict__ wo, int H,
                                                             int W, int pitch, int nb, FftPlan plan, IterParams p)
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
        return make_float2(ua.x - ub.y, -(ua.y + ub.x));
    });
    __syncthreads();
    const float2* Z = fft_rows(a, b, nb, plan, tw);
    const float inv = 1.0f / (float)W;
    for (int idx = threadIdx.x; idx < nb * W; idx += blockDim.x) {
        const int t = idx / W, x = idx - t * W;
        const int ya = 2 * (pair0 + t);
        const float2 z = Z[idx];
        for (int h = 0; h < 2; ++h) {
            const int y = ya + h;
            if (y >= H) break;
            const float s = fmaxf(h == 0 ? z.x * inv : -z.y * inv, p.s_min);
            const float fv = f[(size_t)y * pitch + x];
            const float wt = p.robust ? pen_deriv(fmaxf(rf_eval(fv, s, p), 0.0f), p.eps_d2) : 1.0f;
            qo[(size_t)y * W + x] = wt * fmaxf(fv, 0.0f) * rcp(s);
            wo[(size_t)y * W + x] = wt;
        }
    }
}

// Forward row pass of the pair (q, W) of one row: z = q + i W, FFT, unpack
// into the half spectra of q and of W.
__global__ void __launch_bounds__(256) fftp_rows_fwd_pair(const float* __restrict__ qi, const float* __restrict__ wi,
                                                          float2* __restrict__ Sq, float2* __restrict__ Sw, int H,
                                                          int W, int nb, FftPlan plan)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* tw = reinterpret_cast<float2*>(smem_raw);
    float2* a = tw + W;
    float2* b = a + nb * W;
    fft_twiddles(tw, W);
    const int y0 = blockIdx.x * nb;
    stage_to_lds_n<8>(a, nb * W, [&](int idx) {
        const int t = idx / W, x = idx - t * W;
        const int y = y0 + t;
        return y < H ? make_float2(qi[(size_t)y * W + x], wi[(size_t)y * W + x]) : make_float2(0.0f, 0.0f);
    });
    __syncthreads();
    const float2* Z = fft_rows(a, b, nb, plan, tw);
    const int Wh = W / 2 + 1;
    for (int idx = threadIdx.x; idx < nb * Wh; idx += blockDim.x) {
        const int t = idx / Wh, k = idx - t * Wh;
        const int y = y0 + t;
        if (y >= H) continue;
        const float2 zk = Z[t * W + k];
        const float2 zm = Z[t * W + (k == 0 ? 0 : W - k)];
        Sq[(size_t)y * Wh + k] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
        Sw[(size_t)y * Wh + k] = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
    }
}

// Inverse row pass of the pair: Z = Sq + i Sw (Hermitian extension), inverse
// FFT: N1 = Re, N2 = Im (both sums of non-negative terms: clamped at 0).
__global__ void __launch_bounds__(256) fftp_rows_inv_pair(const float2* __restrict__ Sq, const float2* __restrict__ Sw,
                                                          float* __restrict__ n1, float* __restrict__ n2, int H, int W,
                                                          int nb, FftPlan plan)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2* tw = reinterpret_cast<float2*>(smem_raw);
    float2* a = tw + W;
    float2* b = a + nb * W;
    fft_twiddles(tw, W);
    const int Wh = W / 2 + 1;
    const int y0 = blockIdx.x * nb;
    stage_to_lds_n<8>(a, nb * W, [&](int idx) {
        const int t = idx / W, k = idx - t * W;
        const int y = y0 + t;
        const bool lo = k < Wh;
        const int kk = lo ? k : W - k;
        float2 ua = y < H ? Sq[(size_t)y * Wh + kk] : make_float2(0.0f, 0.0f);
        float2 ub = y < H ? Sw[(size_t)y * Wh + kk] : make_float2(0.0f, 0.0f);
        if (!lo) {
            ua = cconj(ua);
            ub = cconj(ub);
        }
        return make_float2(ua.x - ub.y, -(ua.y + ub.x));
    });
    __syncthreads();
    const float2* Z = fft_rows(a, b, nb, plan, tw);
    const float inv = 1.0f / (float)W;
    for (int idx = threadIdx.x; idx < nb * W; idx += blockDim.x) {
        const int t = idx / W, x = idx - t * W;
        const int y = y0 + t;
        if (y >= H) continue;
        const float2 z = Z[idx];
        n1[(size_t)y * W + x] = fmaxf(z.x * inv, 0.0f);
        n2[(size_t)y * W + x] = fmaxf(-z.y * inv, 0.0f);
    }
}

// Diffusion term and multiplicative update on 64 x TH tiles.
template <int TH>
__global__ void __launch_bounds__(256) fftp_update(const float* __restrict__ u, const float* __restrict__ n1,
                                                   const float* __restrict__ n2, float* __restrict__ u_next,
                                                   float* __restrict__ ckpt, int H, int W, int pitch, IterParams p)
{
    constexpr int TW = 64, UW = TW + 4, UH = TH + 4, GW = TW + 2, GH = TH + 2, R = TH / 4;
    __shared__ float ut[UH * UW];
    __shared__ float gt[GH * GW];
    const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < UH * UW; idx += 256) {
        const int ly = idx / UW, lx = idx - ly * UW;
        ut[idx] = u[(size_t)clampi(y0 - 2 + ly, H) * pitch + clampi(x0 - 2 + lx, W)];
    }
    __syncthreads();
    for (int idx = tid; idx < GH * GW; idx += 256) {
        const int a = idx / GW, b = idx - a * GW;
        const float gx = 0.5f * (ut[(a + 1) * UW + b + 2] - ut[(a + 1) * UW + b]);
        const float gy = 0.5f * (ut[(a + 2) * UW + b + 1] - ut[a * UW + b + 1]);
        gt[idx] = tv_diffusivity(gx * gx + gy * gy, p);
    }
    __syncthreads();
    const int tx = tid & 63, ty = tid >> 6;
    const int x = x0 + tx;
    if (x >= W) return;
    for (int i = 0; i < R; ++i) {
        const int ry = ty * R + i, y = y0 + ry;
        if (y >= H) break;
        const int c = (ry + 2) * UW + tx + 2, cg = (ry + 1) * GW + tx + 1;
        const float up = ut[c], gp = gt[cg];
        const float D = 0.5f * (gp + gt[cg - GW]) * (ut[c - UW] - up) + 0.5f * (gp + gt[cg + GW]) * (ut[c + UW] - up)
                      + 0.5f * (gp + gt[cg - 1]) * (ut[c - 1] - up) + 0.5f * (gp + gt[cg + 1]) * (ut[c + 1] - up);
        const size_t o = (size_t)y * W + x;
        const float num = n1[o] + p.alpha * fmaxf(D, 0.0f);
        const float den = n2[o] - p.alpha * fminf(D, 0.0f);
        const size_t op = (size_t)y * pitch + x;
        if (ckpt) ckpt[op] = up;
        u_next[op] = up * num * rcp(den);
    }
}

static size_t r256(size_t n) { return (n + 255) & ~(size_t)255; }

size_t fft_iter_ws_bytes(int H, int W, int pitch)
{
    const size_t half = r256((size_t)H * (W / 2 + 1) * 8), pl = r256((size_t)H * W * 4);
    const size_t img = r256((size_t)H * pitch * 4);
    return 5 * half + 4 * pl + 2 * img;
}

int launch_rrrl_fft(const float* f, const float* u_in, float* u_out, int H, int W, int pitch, const PsfDev& psf,
                    const IterParams& p, int iters, float* ckpt, void* ws, hipStream_t st)
{
    const size_t half = r256((size_t)H * (W / 2 + 1) * 8), pl = r256((size_t)H * W * 4);
    const size_t img = r256((size_t)H * pitch * 4);
    unsigned char* w8 = reinterpret_cast<unsigned char*>(ws);
    float2* hh = reinterpret_cast<float2*>(w8);
    float2* Mtmp = reinterpret_cast<float2*>(w8 + half);
    float2* Su = reinterpret_cast<float2*>(w8 + 2 * half);
    float2* Sq = reinterpret_cast<float2*>(w8 + 3 * half);
    float2* Sw = reinterpret_cast<float2*>(w8 + 4 * half);
    float* q = reinterpret_cast<float*>(w8 + 5 * half);
    float* wpl = reinterpret_cast<float*>(w8 + 5 * half + pl);
    float* n1 = reinterpret_cast<float*>(w8 + 5 * half + 2 * pl);
    float* n2 = reinterpret_cast<float*>(w8 + 5 * half + 3 * pl);
    float* t0 = reinterpret_cast<float*>(w8 + 5 * half + 4 * pl);
    float* t1 = reinterpret_cast<float*>(w8 + 5 * half + 4 * pl + img);
    const size_t rowb = (size_t)pitch * sizeof(float);
    launch_wiener_mult(psf, H, W, 1.0, Mtmp, hh, st);  // h^ (the multiplier itself is not used)
    if (iters == 0) {
        if (u_out != u_in)
            (void)hipMemcpy2DAsync(u_out, rowb, u_in, rowb, W * sizeof(float), H, hipMemcpyDeviceToDevice, st);
        return hipGetLastError() == hipSuccess ? 0 : -4;
    }
    const float* src = u_in;
    if (u_in == u_out && (iters - 1) % 2 == 0) {
        (void)hipMemcpy2DAsync(t1, rowb, u_in, rowb, W * sizeof(float), H, hipMemcpyDeviceToDevice, st);
        src = t1;
    }
    const int nb = fft_row_batch(W);
    const FftPlan pw = make_plan(W);
    const size_t lds = (size_t)(W + 2 * nb * W) * 8;
    for (int k = 0; k < iters; ++k) {
        float* dst = ((iters - 1 - k) % 2 == 0) ? u_out : t0;
        float* ck = ckpt ? ckpt + (size_t)k * H * pitch : nullptr;
        launch_rows_fwd(src, pitch, H, W, Su, st);
        launch_cols(Su, hh, false, 0, H, W, st);
        hipLaunchKernelGGL(fftp_rows_inv_weights, dim3(((H + 1) / 2 + nb - 1) / nb), dim3(256), lds, st,
                           (const float2*)Su, f, q, wpl, H, W, pitch, nb, pw, p);
        hipLaunchKernelGGL(fftp_rows_fwd_pair, dim3((H + nb - 1) / nb), dim3(256), lds, st, (const float*)q,
                           (const float*)wpl, Sq, Sw, H, W, nb, pw);
        launch_cols(Sq, hh, true, 0, H, W, st);
        launch_cols(Sw, hh, true, 0, H, W, st);
        hipLaunchKernelGGL(fftp_rows_inv_pair, dim3((H + nb - 1) / nb), dim3(256), lds, st, (const float2*)Sq,
                           (const float2*)Sw, n1, n2, H, W, nb, pw);
        hipLaunchKernelGGL(fftp_update<32>, dim3((W + 63) / 64, (H + 31) / 32), dim3(256), 0, st, src,
                           (const float*)n1, (const float*)n2, dst, ck, H, W, pitch, p);
        src = dst;
    }
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace deblur
