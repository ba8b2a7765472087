// Backward (reverse-mode) pass through WR3L: the unrolled RRRL iterations
// (Sec. 2.3, eqs. (9)-(12)) and the Wiener initialisation with its positivity
// floor (Sec. 2.1 eq. (2), Sec. 3.2), for gradients of a loss L(u^K) with
// respect to the observed image f, the PSF taps h and the weight alpha.
//
// Per reversed iteration k (lam = dL/du^{k+1}), from the checkpoint u^k:
//   recompute  s = A u (raw), W, e = W (f - s)/s = q - W   (stage-1 kernel)
//   adj_update N2 = B W, N3 = B e = N1 - N2, D, g; rho = Num/Den;
//              a = lam u/Den (= dL/dN1), b = -a rho (= dL/dN2),
//              c = alpha (a 1[D>0] - b 1[D<0]), du = lam rho, alpha part;
//              stored: a and bb = b + a = -a (N3 + alpha D)/Den
//   dq, dBb = B^T (a, bb)        B^T = zero-extended convolution + border fold
//   adj_point  dW = B^T b + dq f/s = dq (f - s)/s + dBb; r_f, s chain -> ds
// Near convergence b ~ -a and f ~ s: the rearranged forms avoid the FP32
// cancellation of B^T b + (B^T a) f/s.
//   A^T ds                       zero-extended correlation + border fold
//   adj_tv     lam' = du + A^T ds + diffusion adjoint (frozen g and through g)
//   adj_dh     per-workgroup partial sums of dL/dh(d) for every PSF entry
// Under periodic continuation B^T = A and A^T = B (wrapped, no fold).
// The transpose of a gather from the constant continuation E(v)(x) =
// v(clamp(x)) is a scatter onto clamp(x): outputs are formed on a grid
// extended by the PSF radius and the extension is summed onto the border
// pixels (fold).  Partial sums are reduced in a fixed order (deterministic).
//
// Every kernel runs over a batch of equally shaped images at once: blockIdx.z
// is the image, whose planes sit at fixed strides from the first image's.  A
// single image is the batch of one.
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"
#include "psf.hpp"
#include "stencil_tiles.hpp"

namespace deblur {

constexpr int BW_TW = 64, BW_NT = 256;

// Byte strides from one image of a batch to the next: workspace, image planes
// (f, dL/du^K, dL/df, dL/du^0), checkpoints.  alpha: the images' regulariser
// weights (device array; nullptr: the IterParams value).
struct BwdZ {
    size_t ws, img, ck;
    const float* alpha;
};

// Stage 1 recomputed from a checkpoint: s (raw), (e, W) = (q - W, W).
template <int RAD, int TH, int NT>
__global__ void __launch_bounds__(NT) bwd_stage1(const float* __restrict__ u, const float* __restrict__ f,
                                                 float2* __restrict__ qw, float* __restrict__ s_out, int H, int W,
                                                 int pitch, const float* __restrict__ pkg, const int* __restrict__ hdr,
                                                 IterParams p, BwdZ z)
{
    __shared__ float tile[stage1_lds_floats<RAD, TH>()];
    __shared__ float pk[packed_words_max<RAD>()];
    const int2 t = xcd_tile();
    stage1_tile<RAD, TH, NT>(tile, pk, zadv(u, z.ck), zadv(f, z.img), zadv(qw, z.ws), zadv(s_out, z.ws), H, W, pitch,
                             t.x * 64, t.y * TH, zadv(pkg, z.ws), zadv(hdr, z.ws), p);
}

// ------------------------------------------------ adjoint of the update step
template <int RAD, int TH>
__global__ void __launch_bounds__(BW_NT) adj_update(const float2* __restrict__ qw, const float* __restrict__ u,
                                                    const float* __restrict__ lam, int lam_pitch,
                                                    float2* __restrict__ ab, float* __restrict__ cpl,
                                                    float* __restrict__ du, double* __restrict__ alpha_part,
                                                    int H, int W, int pitch, const float* __restrict__ pkg,
                                                    const int* __restrict__ hdr, IterParams p, BwdZ z, size_t lam_z)
{
    constexpr int TW = BW_TW, LW = TW + 2 * RAD, LH = TH + 2 * RAD, R = TH / (BW_NT / 64);
    constexpr int UW = TW + 4, UH = TH + 4, GW = TW + 2, GH = TH + 2;
    qw = zadv(qw, z.ws);
    u = zadv(u, z.ck);
    lam = zadv(lam, lam_z);
    ab = zadv(ab, z.ws);
    cpl = zadv(cpl, z.ws);
    du = zadv(du, z.ws);
    alpha_part = zadv(alpha_part, z.ws);
    pkg = zadv(pkg, z.ws);
    hdr = zadv(hdr, z.ws);
    const float alpha = z.alpha ? z.alpha[blockIdx.z] : p.alpha;
    __shared__ float2 qt[LH * LW];
    __shared__ float ut[UH * UW];
    __shared__ float gt[GH * GW];
    const int2 tile_xy = xcd_tile();   // XCD-aware tile order (halo rows share an L2)
    const int x0 = tile_xy.x * TW, y0 = tile_xy.y * TH;
    const int tid = threadIdx.x;
    // the packed taps are read in place (wave-uniform addresses: scalar
    // loads), which leaves LDS for three workgroups per CU at 16 rows
    int cnt[TAP_GROUP_MAX];
    group_counts(hdr, cnt);
    // tiles whose halo lies inside the image need no continuation: plain row
    // copies (16-byte loads of two (e, W) pairs from an even column)
    const bool inner = x0 >= RAD && y0 >= RAD && x0 + TW + RAD <= W && y0 + TH + RAD <= H;
    if (inner && W % 2 == 0 && ((uintptr_t)qw & 15) == 0) {
        copy_rows_f4<BW_NT, LH, 2 * LW>(reinterpret_cast<float*>(qt),
                                        reinterpret_cast<const float*>(qw + (size_t)(y0 - RAD) * W + (x0 - RAD)),
                                        2 * (size_t)W);
    } else if (inner) {
        const float2* src = qw + (size_t)(y0 - RAD) * W + (x0 - RAD);
        stage_to_lds<BW_NT, LH * LW>(qt, [&](int idx) {
            const int ly = idx / LW;
            return src[(size_t)ly * W + (idx - ly * LW)];
        });
    } else {
        stage_to_lds<BW_NT, LH * LW>(qt, [&](int idx) {
            const int ly = idx / LW, lx = idx - ly * LW;
            const int gy = ext_index(y0 - RAD + ly, H, p.bc), gx = ext_index(x0 - RAD + lx, W, p.bc);
            return qw[(size_t)gy * W + gx];
        });
    }
    if (inner) {
        const float* src = u + (size_t)(y0 - 2) * pitch + (x0 - 2);
        stage_to_lds<BW_NT, UH * UW>(ut, [&](int idx) {
            const int ly = idx / UW;
            return src[(size_t)ly * pitch + (idx - ly * UW)];
        });
    } else {
        stage_to_lds<BW_NT, UH * UW>(ut, [&](int idx) {
            const int ly = idx / UW, lx = idx - ly * UW;
            return u[(size_t)clampi(y0 - 2 + ly, H) * pitch + clampi(x0 - 2 + lx, W)];
        });
    }
    __syncthreads();
    for (int idx = tid; idx < GH * GW; idx += BW_NT) {
        const int a = idx / GW, b = idx - a * GW;
        const float gx = 0.5f * (ut[(a + 1) * UW + b + 2] - ut[(a + 1) * UW + b]);
        const float gy = 0.5f * (ut[(a + 2) * UW + b + 1] - ut[a * UW + b + 1]);
        gt[idx] = tv_diffusivity(gx * gx + gy * gy, p);
    }
    const int tx = tid & 63, ty = tid >> 6;
    float2 nn[R];   // (N3, N2) = B (e, W)
#pragma unroll
    for (int i = 0; i < R; ++i) nn[i] = make_float2(0.0f, 0.0f);
    stencil_groups<1, R, LW>(qt + (ty * R + RAD) * LW + tx + RAD, pkg, cnt, nn);
    __syncthreads();
    const int x = x0 + tx;
    const int ntx = (W + TW - 1) / TW;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int ry = ty * R + i;
        const int y = y0 + ry;
        // dL/dalpha of this image row's 64 columns: one wave holds the row,
        // summed by a fixed shuffle tree into the row's own slot (the same
        // grouping whatever the tile height)
        double apart = 0.0;
        if (x < W && y < H) {
        const int c = (ry + 2) * UW + tx + 2;
        const int cg = (ry + 1) * GW + tx + 1;
        const float up = ut[c], gp = gt[cg];
        const float D = 0.5f * (gp + gt[cg - GW]) * (ut[c - UW] - up) + 0.5f * (gp + gt[cg + GW]) * (ut[c + UW] - up)
                      + 0.5f * (gp + gt[cg - 1]) * (ut[c - 1] - up) + 0.5f * (gp + gt[cg + 1]) * (ut[c + 1] - up);
        // nn.x = N3 = B e (e = q - W), nn.y = N2 = B W
        const float n1 = nn[i].x, n2 = nn[i].y;
        const float dp = fmaxf(D, 0.0f), dm = fminf(D, 0.0f);
        const float num = n2 + n1 + alpha * dp, den = n2 - alpha * dm;
        const float rho = num / den;
        const float l = lam[(size_t)y * lam_pitch + x];
        const float a = l * up / den;
        const float b = -a * rho;
        const float bb = -a * ((n1 + alpha * D) / den);
        const size_t o = (size_t)y * W + x;
        ab[o] = make_float2(a, bb);
        cpl[o] = alpha * ((D > 0.0f ? a : 0.0f) - (D < 0.0f ? b : 0.0f));
        du[o] = l * rho;
        apart = (double)a * dp - (double)b * dm;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) apart += __shfl_xor(apart, off, 64);
        if (tx == 0 && y < H) alpha_part[(size_t)y * ntx + tile_xy.x] += apart;
    }
}

// ----------------------------------- transposed blur: stencil on a grid
// out(z) = sum_t h(d_t) V(z + SIGN d_t) for z on the grid with origin
// (oy, ox) and size OH x OW; V is the input extended by zero (constant-
// continuation transposes, before the fold) or wrapped (periodic).
template <int RAD, int TH, int SIGN, typename T>
__global__ void __launch_bounds__(BW_NT) adj_stencil(const T* __restrict__ v, int vpitch, int H, int W, int wrap,
                                                     T* __restrict__ out, int opitch, int oy, int ox, int OH, int OW,
                                                     const float* __restrict__ pkg, const int* __restrict__ hdr,
                                                     size_t zws)
{
    constexpr int TW = BW_TW, LW = TW + 2 * RAD, LH = TH + 2 * RAD, R = TH / (BW_NT / 64);
    v = zadv(v, zws);
    out = zadv(out, zws);
    pkg = zadv(pkg, zws);
    hdr = zadv(hdr, zws);
    __shared__ T vt[LH * LW];
    const int2 tile_xy = xcd_tile();   // XCD-aware tile order (halo rows share an L2)
    const int zx0 = ox + tile_xy.x * TW, zy0 = oy + tile_xy.y * TH;
    const int tid = threadIdx.x;
    // the packed taps are read in place (wave-uniform addresses: scalar loads)
    int cnt[TAP_GROUP_MAX];
    group_counts(hdr, cnt);
    const bool inner = zy0 >= RAD && zx0 >= RAD && zy0 + TH + RAD <= H && zx0 + TW + RAD <= W;
    if (inner) {   // the window lies inside the input: plain row copies
        const T* src = v + (size_t)(zy0 - RAD) * vpitch + (zx0 - RAD);
        stage_to_lds<BW_NT, LH * LW>(vt, [&](int idx) {
            const int ly = idx / LW;
            return src[(size_t)ly * vpitch + (idx - ly * LW)];
        });
    } else stage_to_lds<BW_NT, LH * LW>(vt, [&](int idx) {
        const int ly = idx / LW, lx = idx - ly * LW;
        int gy = zy0 - RAD + ly, gx = zx0 - RAD + lx;
        T val{};
        if (wrap) {
            gy = ext_index(gy, H, BC_PERIODIC);
            gx = ext_index(gx, W, BC_PERIODIC);
            val = v[(size_t)gy * vpitch + gx];
        } else if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            val = v[(size_t)gy * vpitch + gx];
        }
        return val;
    });
    __syncthreads();
    const int tx = tid & 63, ty = tid >> 6;
    T acc[R];
#pragma unroll
    for (int i = 0; i < R; ++i) acc[i] = T{};
    stencil_groups<SIGN, R, LW>(vt + (ty * R + RAD) * LW + tx + RAD, pkg, cnt, acc);
    const int zx = zx0 + tx;
    if (zx >= ox + OW) return;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int zy = zy0 + ty * R + i;
        if (zy >= oy + OH) break;
        out[(size_t)(zy - oy) * opitch + (zx - ox)] = acc[i];
    }
}

// Fold of an output extended by (ry, rx): every image pixel sums the grid
// points whose clamped position it is.  Only border pixels have more than one
// (their own point plus the extension beyond them); an interior pixel's value
// is its own grid point, read in place by the consumers (ext_or_border).  The
// border pixels' sums go to a buffer of 2W + 2H entries (border_index): first
// along x for every extended row (the columns that clamp to x), then along y
// (the rows that clamp to y), each in order, with the loads eight at a time.
DEBLUR_DEV void add_to(float& a, float b) { a += b; }
DEBLUR_DEV void add_to(float2& a, float2 b)
{
    a.x += b.x;
    a.y += b.y;
}

// Slot of border pixel (y, x) in the fold buffer, -1 for interior pixels:
// row 0, row H-1, then column 0 and column W-1 without their end rows.
DEBLUR_DEV int border_index(int y, int x, int H, int W)
{
    if (y == 0) return x;
    if (y == H - 1) return W + x;
    if (x == 0) return 2 * W + (y - 1);
    if (x == W - 1) return 2 * W + (H - 2) + (y - 1);
    return -1;
}

template <typename T>
__global__ void __launch_bounds__(256) adj_fold_border(const T* __restrict__ ext, int epitch, int ry, int rx, int H,
                                                       int W, T* __restrict__ bd, size_t zws)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int y, x;
    if (t < W) {
        y = 0, x = t;
    } else if (t < 2 * W) {
        y = H - 1, x = t - W;
        if (H == 1) return;
    } else if (t < 2 * W + max(H - 2, 0)) {
        y = t - 2 * W + 1, x = 0;
    } else if (t < 2 * W + 2 * max(H - 2, 0)) {
        y = t - 2 * W - (H - 2) + 1, x = W - 1;
        if (W == 1) return;
    } else {
        return;
    }
    ext = zadv(ext, zws);
    bd = zadv(bd, zws);
    const int lox = x == 0 ? 0 : x + rx, hix = x == W - 1 ? W - 1 + 2 * rx : x + rx;   // extended columns
    const int loy = y == 0 ? 0 : y + ry, hiy = y == H - 1 ? H - 1 + 2 * ry : y + ry;   // extended rows
    T acc{};
    for (int b0 = loy; b0 <= hiy; b0 += 8) {
        T v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v[k] = T{};
            if (b0 + k <= hiy) {
                const T* row = ext + (size_t)(b0 + k) * epitch;
                for (int c0 = lox; c0 <= hix; c0 += 8) {
                    T w[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) w[q] = c0 + q <= hix ? row[c0 + q] : T{};
#pragma unroll
                    for (int q = 0; q < 8; ++q) add_to(v[k], w[q]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) add_to(acc, v[k]);
    }
    bd[border_index(y, x, H, W)] = acc;
}

// A transposed-blur output at image pixel (y, x): the folded value of a border
// pixel, else the pixel's own point of the extended grid (origin (oy, ox)).
// Periodic continuation: bd = nullptr, oy = ox = 0 (the plain image grid).
template <typename T>
DEBLUR_DEV T ext_or_border(const T* __restrict__ ext, int epitch, int oy, int ox, const T* __restrict__ bd, int y,
                           int x, int H, int W)
{
    if (bd) {
        const int b = border_index(y, x, H, W);
        if (b >= 0) return bd[b];
    }
    return ext[(size_t)(y + oy) * epitch + x + ox];
}

// ------------------------------- adjoint of W, q = W f / s, r_f and the guard
// (dq, dW) = B^T (a, bb): on the extended grid (pitch epitch, origin (oy, ox))
// with the folded border values in bd (nullptr: periodic, no fold).
__global__ void __launch_bounds__(256) adj_point(const float2* __restrict__ dqw, int epitch, int oy, int ox,
                                                 const float2* __restrict__ dbd, const float2* __restrict__ qw,
                                                 const float* __restrict__ s_raw, const float* __restrict__ f,
                                                 float* __restrict__ grad_f, float* __restrict__ ds, int H, int W,
                                                 int pitch, IterParams p, BwdZ z)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= W) return;
    dqw = zadv(dqw, z.ws);
    if (dbd) dbd = zadv(dbd, z.ws);
    qw = zadv(qw, z.ws);
    s_raw = zadv(s_raw, z.ws);
    f = zadv(f, z.img);
    grad_f = zadv(grad_f, z.img);
    ds = zadv(ds, z.ws);
    const size_t o = (size_t)y * W + x, of = (size_t)y * pitch + x;
    const float2 d = ext_or_border(dqw, epitch, oy, ox, dbd, y, x, H, W);   // (B^T a, B^T bb)
    const float2 v = qw[o];                                                   // (e, W)
    const float sr = s_raw[o];
    const float st = fmaxf(sr, p.s_min);
    const float fv = f[of];
    const float fp = fmaxf(fv, 0.0f);
    const float wt = v.y;
    const float dW = d.x * ((fp - st) / st) + d.y;
    float dst = -d.x * wt * fp / (st * st);
    float df = fv > 0.0f ? d.x * wt / st : 0.0f;
    if (p.robust) {
        const float r = info_div(fv, st);
        const float dr = r > 0.0f ? dW * (-0.5f) * wt * wt * wt : 0.0f;
        if (fv > 0.0f) {
            dst += dr * (1.0f - fv / st);
            df += dr * (-logf(st / fv));
        } else {
            dst += dr;
        }
    }
    ds[o] = sr > p.s_min ? dst : 0.0f;
    grad_f[of] += df;
}

// ------------------------------------------ adjoint of the diffusion term
// lam_out = du + aT + (L_g c) + (through g), c = dL/dD, frozen-g operator L_g
// symmetric; g = Psi'(gx^2 + gy^2) with central differences of clamped u.
// aT = A^T ds on the extended grid (pitch epitch, origin (oy, ox)) with the
// folded border values in abd (nullptr: periodic, no fold).
template <int TH>
__global__ void __launch_bounds__(BW_NT) adj_tv(const float* __restrict__ u, int pitch, const float* __restrict__ cpl,
                                                const float* __restrict__ du, const float* __restrict__ aT, int epitch,
                                                int oy, int ox, const float* __restrict__ abd,
                                                float* __restrict__ lam_out, int H, int W, IterParams p, BwdZ z)
{
    constexpr int TW = BW_TW, UW = TW + 4, UH = TH + 4, GW = TW + 2, GH = TH + 2;
    u = zadv(u, z.ck);
    cpl = zadv(cpl, z.ws);
    du = zadv(du, z.ws);
    aT = zadv(aT, z.ws);
    if (abd) abd = zadv(abd, z.ws);
    lam_out = zadv(lam_out, z.ws);
    __shared__ float ut[UH * UW], ct[UH * UW];
    __shared__ float gt[GH * GW], dgx[GH * GW], dgy[GH * GW];
    const int2 tile_xy = xcd_tile();   // XCD-aware tile order (halo rows share an L2)
    const int x0 = tile_xy.x * TW, y0 = tile_xy.y * TH;
    const int tid = threadIdx.x;
    if (x0 >= 2 && y0 >= 2 && x0 + TW + 2 <= W && y0 + TH + 2 <= H) {   // no clamping needed
        const float* su = u + (size_t)(y0 - 2) * pitch + (x0 - 2);
        const float* sc = cpl + (size_t)(y0 - 2) * W + (x0 - 2);
        stage_to_lds<BW_NT, UH * UW>(ut, [&](int idx) {
            const int ly = idx / UW;
            return su[(size_t)ly * pitch + (idx - ly * UW)];
        });
        stage_to_lds<BW_NT, UH * UW>(ct, [&](int idx) {
            const int ly = idx / UW;
            return sc[(size_t)ly * W + (idx - ly * UW)];
        });
    } else {
        stage_to_lds<BW_NT, UH * UW>(ut, [&](int idx) {
            const int ly = idx / UW, lx = idx - ly * UW;
            return u[(size_t)clampi(y0 - 2 + ly, H) * pitch + clampi(x0 - 2 + lx, W)];
        });
        stage_to_lds<BW_NT, UH * UW>(ct, [&](int idx) {
            const int ly = idx / UW, lx = idx - ly * UW;
            return cpl[(size_t)clampi(y0 - 2 + ly, H) * W + clampi(x0 - 2 + lx, W)];
        });
    }
    __syncthreads();
    // at grid points (y0-1+a, x0-1+b): g, and dL/dgx, dL/dgy through g
    for (int idx = tid; idx < GH * GW; idx += BW_NT) {
        const int a = idx / GW, b = idx - a * GW;
        const int c = (a + 1) * UW + b + 1;
        const float up = ut[c], cp = ct[c];
        const float gx = 0.5f * (ut[c + 1] - ut[c - 1]);
        const float gy = 0.5f * (ut[c + UW] - ut[c - UW]);
        const float g = tv_diffusivity(gx * gx + gy * gy, p);
        // dL/dg(p) = sum_n (u_n - u_p)(c_p - c_n)/2 (neighbours outside read u_p: 0)
        const float dg = 0.5f * ((ut[c - UW] - up) * (cp - ct[c - UW]) + (ut[c + UW] - up) * (cp - ct[c + UW])
                                 + (ut[c - 1] - up) * (cp - ct[c - 1]) + (ut[c + 1] - up) * (cp - ct[c + 1]));
        const float g3 = -tv_slope(g, p) * dg;
        gt[idx] = g;
        dgx[idx] = g3 * gx;
        dgy[idx] = g3 * gy;
    }
    __syncthreads();
    constexpr int R = TH / (BW_NT / 64);
    const int tx = tid & 63, ty = tid >> 6;
    const int x = x0 + tx;
    if (x >= W) return;
    for (int i = 0; i < R; ++i) {
        const int ry = ty * R + i, y = y0 + ry;
        if (y >= H) break;
        const int c = (ry + 2) * UW + tx + 2, k = (ry + 1) * GW + tx + 1;
        const float gm = gt[k], cm = ct[c];
        float acc = 0.5f * (gm + gt[k - GW]) * (ct[c - UW] - cm) + 0.5f * (gm + gt[k + GW]) * (ct[c + UW] - cm)
                  + 0.5f * (gm + gt[k - 1]) * (ct[c - 1] - cm) + 0.5f * (gm + gt[k + 1]) * (ct[c + 1] - cm);
        // gx(p) = (u(p_x+1 clamped) - u(p_x-1 clamped))/2: gather the scatter
        if (x > 0) acc += 0.5f * dgx[k - 1];
        if (x == W - 1) acc += 0.5f * dgx[k];
        if (x < W - 1) acc -= 0.5f * dgx[k + 1];
        if (x == 0) acc -= 0.5f * dgx[k];
        if (y > 0) acc += 0.5f * dgy[k - GW];
        if (y == H - 1) acc += 0.5f * dgy[k];
        if (y < H - 1) acc -= 0.5f * dgy[k + GW];
        if (y == 0) acc -= 0.5f * dgy[k];
        const size_t o = (size_t)y * W + x;
        lam_out[o] = du[o] + ext_or_border(aT, epitch, oy, ox, abd, y, x, H, W) + acc;
    }
}

// ------------------------------------------------------ dL/dh partial sums
// For every entry (j, i) of the PSF array, d = (j - cy, i - cx):
//   sum over the tile of a(x) q(E(x + d)) + b(x) W(E(x + d)) + ds(x) u(E(x - d))
// where the first two terms are formed as a e(E(x+d)) + bb W(E(x+d))
// (q = e + W, bb = a + b); the result is added to this workgroup's slot of
// `part` (FP64).
//
// Work unit = one lag block (a PSF row dy and 8 adjacent columns dx0..dx0+7)
// over a share of the tile rows.  Along a tile row the unit takes 8 pixels at
// a time: their 8 factors and the 15 values at x + dx0 .. x + 7 + dx0 + 7 give
// 64 products per channel from registers (no per-product LDS read).  The
// extended tile covers columns x0 - RAD - 8 .. x0 + 64 + RAD + 8 so that the
// padded lags of the last block stay inside it.
constexpr int DH_TH = 8;
template <int RAD>
__global__ void __launch_bounds__(BW_NT) adj_dh(const float2* __restrict__ ab, const float2* __restrict__ qw,
                                                const float* __restrict__ ds, const float* __restrict__ u,
                                                int pitch, int H, int W, int ph, int pw, int bc,
                                                double* __restrict__ part, BwdZ z)
{
    ab = zadv(ab, z.ws);
    qw = zadv(qw, z.ws);
    ds = zadv(ds, z.ws);
    u = zadv(u, z.ck);
    part = zadv(part, z.ws);
    // LW odd: rows of the extended tile start in different LDS banks
    constexpr int TH = DH_TH, TW = 64, XO = RAD + 8, LW = TW + 2 * XO + 1, LH = TH + 2 * RAD;
    constexpr int MAXB = (2 * RAD + 1) * ((2 * RAD + 1 + 7) / 8);   // lag blocks of the largest PSF
    constexpr int MAXU = (MAXB + BW_NT - 1) / BW_NT;
    __shared__ float2 ct[TH * TW];
    __shared__ float2 ht[LH * LW];
    __shared__ float red[BW_NT * 8];
    const int2 tile_xy = xcd_tile();   // XCD-aware tile order (halo rows share an L2)
    const int x0 = tile_xy.x * TW, y0 = tile_xy.y * TH;
    const int tid = threadIdx.x;
    const int PP = ph * pw, cy = (ph - 1) / 2, cx = (pw - 1) / 2;
    const int nxb = (pw + 7) / 8, nb = ph * nxb;
    const int rp = max(1, min(TH, BW_NT / nb));        // row parts per lag block
    const int rows = (TH + rp - 1) / rp;
    float acc[MAXU][8];
#pragma unroll
    for (int k = 0; k < MAXU; ++k)
#pragma unroll
        for (int l = 0; l < 8; ++l) acc[k][l] = 0.0f;

    // a, bb on the tile; (e, W) on the extended tile
    stage_to_lds<BW_NT, TH * TW>(ct, [&](int idx) {
        const int ly = idx / TW, lx = idx - ly * TW;
        const int y = y0 + ly, x = x0 + lx;
        return (y < H && x < W) ? ab[(size_t)y * W + x] : make_float2(0.0f, 0.0f);
    });
    stage_to_lds<BW_NT, LH * LW>(ht, [&](int idx) {
        const int ly = idx / LW, lx = idx - ly * LW;
        const int gy = ext_index(y0 - RAD + ly, H, bc), gx = ext_index(x0 - XO + lx, W, bc);
        return qw[(size_t)gy * W + gx];
    });
    __syncthreads();
#pragma unroll
    for (int k = 0; k < MAXU; ++k) {
        const int unit = tid + k * BW_NT;
        if (unit >= nb * rp) break;
        const int blk = unit % nb, r = unit / nb;
        const int dy = blk / nxb - cy, dx0 = (blk % nxb) * 8 - cx;
        const int ya = r * rows, yb = min(TH, ya + rows);
        for (int y = ya; y < yb; ++y) {
            const float2* hrow = ht + (y + RAD + dy) * LW + XO + dx0;
            for (int xc = 0; xc < TW; xc += 8) {
                float2 c[8], h[15];
#pragma unroll
                for (int q = 0; q < 8; ++q) c[q] = ct[y * TW + xc + q];
#pragma unroll
                for (int q = 0; q < 15; ++q) h[q] = hrow[xc + q];
#pragma unroll
                for (int q = 0; q < 8; ++q)
#pragma unroll
                    for (int l = 0; l < 8; ++l) acc[k][l] = fmaf(c[q].x, h[q + l].x, fmaf(c[q].y, h[q + l].y, acc[k][l]));
            }
        }
    }
    __syncthreads();
    // ds on the tile; u on the extended tile (x - d)
    float* cs = reinterpret_cast<float*>(ct);
    float* hs = reinterpret_cast<float*>(ht);
    stage_to_lds<BW_NT, TH * TW>(cs, [&](int idx) {
        const int ly = idx / TW, lx = idx - ly * TW;
        const int y = y0 + ly, x = x0 + lx;
        return (y < H && x < W) ? ds[(size_t)y * W + x] : 0.0f;
    });
    stage_to_lds<BW_NT, LH * LW>(hs, [&](int idx) {
        const int ly = idx / LW, lx = idx - ly * LW;
        const int gy = ext_index(y0 - RAD + ly, H, bc), gx = ext_index(x0 - XO + lx, W, bc);
        return u[(size_t)gy * pitch + gx];
    });
    __syncthreads();
#pragma unroll
    for (int k = 0; k < MAXU; ++k) {
        const int unit = tid + k * BW_NT;
        if (unit >= nb * rp) break;
        const int blk = unit % nb, r = unit / nb;
        const int dy = blk / nxb - cy, dx0 = (blk % nxb) * 8 - cx;
        const int ya = r * rows, yb = min(TH, ya + rows);
        for (int y = ya; y < yb; ++y) {
            // u(x - dx0 - l) for pixel x = xc + q: column xc + XO - dx0 - 7 + (q - l + 7)
            const float* urow = hs + (y + RAD - dy) * LW + XO - dx0 - 7;
            for (int xc = 0; xc < TW; xc += 8) {
                float c[8], h[15];
#pragma unroll
                for (int q = 0; q < 8; ++q) c[q] = cs[y * TW + xc + q];
#pragma unroll
                for (int q = 0; q < 15; ++q) h[q] = urow[xc + q];
#pragma unroll
                for (int q = 0; q < 8; ++q)
#pragma unroll
                    for (int l = 0; l < 8; ++l) acc[k][l] = fmaf(c[q], h[q - l + 7], acc[k][l]);
            }
        }
    }
    // combine the row parts of each lag block in a fixed order
    const size_t base = (size_t)(blockIdx.y * gridDim.x + blockIdx.x) * PP;
#pragma unroll
    for (int k = 0; k < MAXU; ++k) {
        __syncthreads();
        const int unit = tid + k * BW_NT;
        const bool live = unit < nb * rp;
        if (live)
#pragma unroll
            for (int l = 0; l < 8; ++l) red[tid * 8 + l] = acc[k][l];
        __syncthreads();
        if (live && unit / nb == 0) {
            const int blk = unit % nb;
            const int j = blk / nxb, i0 = (blk % nxb) * 8;
#pragma unroll
            for (int l = 0; l < 8; ++l) {
                if (i0 + l >= pw) break;
                double sum = 0.0;
                for (int r = 0; r < rp; ++r) sum += (double)red[(tid + r * nb) * 8 + l];
                part[base + j * pw + i0 + l] += sum;
            }
        }
    }
}

// The same partial sums on the matrix cores, for PSF arrays of at most 32 x 32
// entries (radius class 16): one 32 x 32 block of lags covers the whole
// array.  Written as products of matrices, for an image row y of the tile and
// a column x' of the extended grid:
//   a e   and  bb W :  D[dy][dx] += E(y + dy, x') * A(y, x' - dx)
//   ds u           :  D[dy][dx] += U(y - dy, x') * S(y, x' + dx)
// with A, S zero outside the tile.  Each operand value v is staged as two
// bfloat16 numbers, hi = v rounded to nearest even and lo = (v - hi) rounded
// likewise (|v - hi - lo| <= 2^-16 |v|), and a product is taken as
// lo hi' + hi lo' + hi hi' (the dropped lo lo' and the two remainders bound
// its relative error by about 3 * 2^-16; the products are exact and summed in
// FP32).  K runs along x' sixteen columns per v_mfma_f32_32x32x16_bf16,
// three per step (lane l: block row / column l mod 32, columns 8 (l/32) ..
// 8 (l/32) + 7 of the step in both operands, so the order in which the
// instruction pairs them does not matter; accumulator r holds row
// 8 (r/4) + 4 (l/32) + r mod 4, column l mod 32).  Rows and columns of the
// block beyond the PSF read clamped (in-range) operands and are discarded.
// A workgroup marches down a segment of DHM_SEG rows of a 256-column strip,
// DHM_TB (= RAD) rows per step, for each of the three products in turn: the
// extended rows of e, W or u are a ring of three blocks of DHM_TB rows, and a
// step stages only the block that enters its halo (plus the tile plane of a,
// bb or ds with zero margins of twice the radius), so two workgroups fit a
// CU.  A wave takes every eighth row of a step; the eight waves' blocks are
// summed in a fixed order (FP64) into this workgroup's slot of `part`.
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned uintx4 __attribute__((ext_vector_type(4)));

// v = hi + lo as bfloat16 bit patterns, packed hi << 16 | lo (finite v).
DEBLUR_DEV unsigned bf16_split(float v)
{
    auto rne = [](float x) {
        const unsigned b = __float_as_uint(x);
        return (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
    };
    const unsigned hi = rne(v);
    return hi << 16 | rne(v - __uint_as_float(hi << 16));
}

// One half (selector 0x07060302: the hi parts, 0x05040100: the lo parts) of
// eight packed words as an MFMA operand.
DEBLUR_DEV bf16x8 bf16_halves(const unsigned (&w)[8], unsigned sel)
{
    uintx4 o;
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = __builtin_amdgcn_perm(w[2 * i + 1], w[2 * i], sel);
    return __builtin_bit_cast(bf16x8, o);
}

constexpr int DHM_TB = 16, DHM_TW = 256, DHM_NT = 512, DHM_WAVES = DHM_NT / 64, DHM_SEG = 128;

template <int RAD>
__global__ void __launch_bounds__(DHM_NT) adj_dh_mfma(const float2* __restrict__ ab, const float2* __restrict__ qw,
                                                   const float* __restrict__ ds, const float* __restrict__ u,
                                                   int pitch, int H, int W, int ph, int pw, int bc,
                                                   double* __restrict__ part, BwdZ z)
{
    constexpr int TB = DHM_TB, TW = DHM_TW;
    static_assert(TB == RAD, "the halo of a step is one block of rows above and one below");
    // extended rows: a pitch of whole 16-byte units, so that the eight words a
    // lane reads per step are two aligned 16-byte reads (the lanes of a half
    // read rows 292 words apart: disjoint banks); the tile plane keeps an odd
    // pitch (its lanes start at different columns)
    constexpr int QP = (TW + 2 * RAD + 1 + 3) & ~3, AP = TW + 4 * RAD + 1;
    // K steps of sixteen columns (rounded up) with the next step read ahead:
    // reads pass the end of a row by at most 29 columns, into the next row or
    // a zeroed tail.  A step past the useful columns multiplies by the zero
    // margin of the tile plane (2 RAD >= 32 zero columns on each side).
    constexpr int TAIL = 64;
    static_assert(2 * RAD >= 30 && DHM_WAVES * 1024 <= 3 * TB * QP, "margins and reduction space");
    // extended rows as a ring of three blocks of TB rows (block b: rows
    // ys - TB + TB b .., slot b mod 3); the tile plane of the current step
    __shared__ __align__(16) unsigned qe[3 * TB * QP + TAIL];   // columns x0 - RAD .. (split words)
    __shared__ unsigned at[TB * AP + TAIL];       // columns x0 - 2 RAD ..
    ab = zadv(ab, z.ws);
    qw = zadv(qw, z.ws);
    ds = zadv(ds, z.ws);
    u = zadv(u, z.ck);
    part = zadv(part, z.ws);
    const int2 txy = xcd_tile();
    const int x0 = txy.x * TW, ys = txy.y * DHM_SEG;
    const int nsteps = (min(DHM_SEG, H - ys) + TB - 1) / TB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int bi = lane & 31, k = lane >> 5;
    const int cy = (ph - 1) / 2, cx = (pw - 1) / 2;
    const int dy = min(bi - cy, cy), dx = min(bi - cx, cx);   // this lane's lags (clamped beyond the PSF)
    const int c_lo = (RAD - cx) & ~3, c_hi = RAD + TW + cx;   // columns x' with a non-zero product
    const int nk = (c_hi - c_lo + 16) / 16;   // K steps
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    if (tid < TAIL) {
        qe[3 * TB * QP + tid] = 0u;
        at[TB * AP + tid] = 0u;
    }
    // block b of the extended rows of product `phase` into its ring slot
    auto stage_block = [&](int phase, int b) {
        unsigned* dst = qe + (b % 3) * TB * QP;
        const int r0 = ys - TB + TB * b;
        stage_to_lds_n<8>(dst, TB * QP, [&](int idx) {
            const int r = idx / QP, c = idx - r * QP;
            const int gy = ext_index(r0 + r, H, bc), gx = ext_index(x0 - RAD + min(c, TW + 2 * RAD - 1), W, bc);
            return bf16_split(phase == 2 ? u[(size_t)gy * pitch + gx]
                                         : (phase == 0 ? qw[(size_t)gy * W + gx].x : qw[(size_t)gy * W + gx].y));
        });
    };

    for (int phase = 0; phase < 3; ++phase) {
        const int sy = phase == 2 ? -dy : dy, sx = phase == 2 ? dx : -dx;
        for (int s = 0; s < nsteps; ++s) {
            const int y0 = ys + TB * s;
            __syncthreads();   // the previous step's reads of the slot and of the tile plane are done
            if (s == 0) {
                stage_block(phase, 0);
                stage_block(phase, 1);
            }
            stage_block(phase, s + 2);
            stage_to_lds_n<8>(at, TB * AP, [&](int idx) {
                const int t = idx / AP, x = x0 - 2 * RAD + (idx - t * AP), y = y0 + t;
                if (y >= H || x < x0 || x >= x0 + TW || x >= W) return 0u;
                const size_t o = (size_t)y * W + x;
                return bf16_split(phase == 2 ? ds[o] : (phase == 0 ? ab[o].x : ab[o].y));
            });
            __syncthreads();
            for (int t = wave; t < TB; t += DHM_WAVES) {
                if (y0 + t >= H) break;
                // ring row of extended row y0 + t + sy (block-relative q)
                const int q = TB + TB * s + t + sy;
                const unsigned* ar = qe + ((q / TB) % 3 * TB + q % TB) * QP + 8 * k + c_lo;
                const unsigned* br = at + t * AP + RAD + sx + 8 * k + c_lo;
                // the words of the next K step are read from LDS while the
                // current step's three products run on the matrix core; two
                // register sets take turns (steps read: 0 .. nk)
                unsigned a[8], b[8], a2[8], b2[8];
                auto words = [&](unsigned (&x)[8], unsigned (&y)[8], int n) {
#pragma unroll
                    for (int m = 0; m < 8; ++m) y[m] = br[16 * n + m];
                    const uintx4* a4 = reinterpret_cast<const uintx4*>(ar + 16 * n);
                    const uintx4 lo4 = a4[0], hi4 = a4[1];
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        x[m] = lo4[m];
                        x[4 + m] = hi4[m];
                    }
                };
                auto products = [&](const unsigned (&x)[8], const unsigned (&y)[8]) {
                    const bf16x8 xh = bf16_halves(x, 0x07060302u), xl = bf16_halves(x, 0x05040100u);
                    const bf16x8 yh = bf16_halves(y, 0x07060302u), yl = bf16_halves(y, 0x05040100u);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl, yh, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh, yl, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh, yh, acc, 0, 0, 0);
                };
                words(a, b, 0);
                for (int n = 0; n < nk; n += 2) {
                    words(a2, b2, n + 1);
                    products(a, b);
                    if (n + 1 < nk) {
                        words(a, b, n + 2);
                        products(a2, b2);
                    }
                }
            }
        }
    }
    __syncthreads();
    float* red = reinterpret_cast<float*>(qe);
#pragma unroll
    for (int r = 0; r < 16; ++r) red[wave * 1024 + (8 * (r >> 2) + 4 * k + (r & 3)) * 32 + bi] = acc[r];
    __syncthreads();
    const size_t base = (size_t)(blockIdx.y * gridDim.x + blockIdx.x) * ph * pw;
    for (int o = tid; o < 1024; o += DHM_NT) {
        const int j = o >> 5, i = o & 31;
        if (j < ph && i < pw) {
            double sum = 0.0;
            for (int w = 0; w < DHM_WAVES; ++w) sum += (double)red[w * 1024 + o];
            part[base + j * pw + i] += sum;
        }
    }
}

// The dL/dh kernel for a PSF: the matrix-core one for arrays of at most
// 32 x 32 entries in radius class 16, else the vector one; and its number of
// workgroups (partial-sum slots) per image.
static bool dh_on_mfma(const PsfDev& psf, int rad) { return rad == 16 && psf.ph <= 32 && psf.pw <= 32; }
static size_t dh_blocks(int H, int W, const PsfDev& psf, int rad)
{
    if (dh_on_mfma(psf, rad)) return (size_t)((W + DHM_TW - 1) / DHM_TW) * ((H + DHM_SEG - 1) / DHM_SEG);
    return (size_t)((W + 63) / 64) * ((H + DH_TH - 1) / DH_TH);
}

// Fixed-order reduction of the per-workgroup partial sums.
__global__ void __launch_bounds__(256) adj_reduce(const double* __restrict__ part, int nblocks, int PP,
                                                  const double* __restrict__ alpha_part, int nalpha,
                                                  double* __restrict__ dh, double* __restrict__ dalpha, size_t zws)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    part = zadv(part, zws);
    alpha_part = zadv(alpha_part, zws);
    dh = zadv(dh, zws);
    dalpha = zadv(dalpha, zws);
    if (t < PP) {
        // fixed order b = 0, 1, ...; eight loads in flight
        double s = 0.0;
        for (int b0 = 0; b0 < nblocks; b0 += 8) {
            double v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = b0 + k < nblocks ? part[(size_t)(b0 + k) * PP + t] : 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) s += v[k];
        }
        dh[t] = s;
    }
    if (blockIdx.x == 0) {
        // dL/dalpha: thread k sums the contiguous chunk k of the row slots in
        // order, then a fixed tree over the 256 chunk sums
        __shared__ double red[256];
        const int k = threadIdx.x, chunk = (nalpha + 255) / 256;
        double s = 0.0;
        for (int b = k * chunk; b < min(nalpha, (k + 1) * chunk); ++b) s += alpha_part[b];
        red[k] = s;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (k < off) red[k] += red[k + off];
            __syncthreads();
        }
        if (k == 0) dalpha[0] = red[0];
    }
}

__global__ void __launch_bounds__(256) fill_zero_f64(double* __restrict__ p, size_t n, size_t zs)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) zadv(p, zs)[i] = 0.0;
}

__global__ void __launch_bounds__(256) fill_zero_f32(float* __restrict__ p, int W, int H, int pitch, size_t zs)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x < W) zadv(p, zs)[(size_t)y * pitch + x] = 0.0f;
}

__global__ void __launch_bounds__(256) copy_plane(const float* __restrict__ src, int spitch, float* __restrict__ dst,
                                                  int dpitch, int W, size_t zsrc, size_t zdst)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x < W) zadv(dst, zdst)[(size_t)y * dpitch + x] = zadv(src, zsrc)[(size_t)y * spitch + x];
}

// -------------------------------------------------------- Wiener adjoint
// G = lam0 1[u_pre > floor]
__global__ void __launch_bounds__(256) wiener_mask(const float* __restrict__ lam0, const float* __restrict__ upre,
                                                   float* __restrict__ G, int W, float floor_, size_t zws)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x < W) {
        const size_t o = (size_t)y * W + x;
        zadv(G, zws)[o] = zadv(upre, zws)[o] > floor_ ? zadv(lam0, zws)[o] : 0.0f;
    }
}

// Y = Z c1 + conj(Z c2), Z = F conj(G), c1 = K / (|h^|^2+K)^2,
// c2 = -conj(h^)^2 / (|h^|^2+K)^2, on the half spectrum (FP64 arithmetic).
// (Y may alias Fh: each element is read before it is written by the same thread.)
__global__ void __launch_bounds__(256) wiener_dh_spectrum(const float2* Fh, const float2* __restrict__ Gh,
                                                          const float2* __restrict__ hh, float2* Y, size_t n, double K,
                                                          size_t zs)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Fh = zadv(Fh, zs);
    Gh = zadv(Gh, zs);
    hh = zadv(hh, zs);
    Y = zadv(Y, zs);
    const double fr = Fh[i].x, fi = Fh[i].y, gr = Gh[i].x, gi = Gh[i].y;
    const double zr = fr * gr + fi * gi, zi = fi * gr - fr * gi;   // F conj(G)
    const double hr = hh[i].x, hi = hh[i].y;
    const double m2 = hr * hr + hi * hi + K;
    const double den = m2 * m2;
    const double c1 = K / den;
    const double c2r = -(hr * hr - hi * hi) / den, c2i = (2.0 * hr * hi) / den;  // -conj(h)^2/den
    const double pr = zr * c2r - zi * c2i, pi = zr * c2i + zi * c2r;              // Z c2
    Y[i] = make_float2((float)(zr * c1 + pr), (float)(zi * c1 - pi));
}

// dh(j, i) += R((j - cy) mod H, (i - cx) mod W)
__global__ void __launch_bounds__(256) wiener_dh_gather(const float* __restrict__ R, int H, int W, int ph, int pw,
                                                        double* __restrict__ dh, size_t zws)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ph * pw) return;
    R = zadv(R, zws);
    dh = zadv(dh, zws);
    const int j = t / pw, i = t - j * pw;
    const int y = ext_index(j - (ph - 1) / 2, H, BC_PERIODIC), x = ext_index(i - (pw - 1) / 2, W, BC_PERIODIC);
    dh[t] += (double)R[(size_t)y * W + x];
}

// Image z's dL/dh at grad_taps + z PP, its dL/dalpha at grad_alpha + z.
__global__ void __launch_bounds__(256) write_grads(const double* __restrict__ dh, int PP, const double* __restrict__ da,
                                                   float* __restrict__ grad_taps, float* __restrict__ grad_alpha,
                                                   size_t zws)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    dh = zadv(dh, zws);
    da = zadv(da, zws);
    if (grad_taps) grad_taps += (size_t)blockIdx.z * PP;
    if (grad_alpha) grad_alpha += blockIdx.z;
    if (grad_taps && t < PP) grad_taps[t] = (float)dh[t];
    if (grad_alpha && t == 0) grad_alpha[0] = (float)da[0];
}

// ------------------------------------------------------------ host driver
static size_t r256(size_t n) { return (n + 255) & ~(size_t)255; }

struct BwdLayout {
    size_t list, qw, s, ab, c, du, ds, lamA, lamB, ext, bd2, bd1, part, apart, dh, da, total;
};

static int bwd_rad(const PsfDev& psf) { return tap_radius_class(max((psf.ph - 1) / 2, (psf.pw - 1) / 2)); }

// Rows per tile of the backward iteration kernels, by bwd_tile variant:
// 1: 8, 2: 4, 3: 16, 4: 32.  The default (0) goes by the workgroups of one
// launch over the batch: 8 rows while 16-row tiles would leave fewer than
// 8192 (a single 512^2 image: 512 workgroups of 8 rows, two per CU), else 16
// (a batch of 512^2 images: the halo rows of the radius are re-read less
// often).  The results do not depend on it (per-pixel sums in tap order; the
// dL/dalpha partial sums are per image row).
constexpr int BWD_VARIANTS = 4;
static int bwd_th(const IterParams& p, int B, int H, int W)
{
    switch (p.bwd_tile) {
        case 1: return 8;
        case 2: return 4;
        case 3: return 16;
        case 4: return 32;
        default: break;
    }
    const long tiles16 = (long)B * ((H + 15) / 16) * ((W + 63) / 64);
    return tiles16 >= 8192 ? 16 : 8;
}
int backward_tile_variants() { return BWD_VARIANTS; }

static BwdLayout bwd_layout(int H, int W, const PsfDev& psf)
{
    BwdLayout L{};
    const int cy = (psf.ph - 1) / 2, cx = (psf.pw - 1) / 2;
    const size_t pl = r256((size_t)H * W * 4), pl2 = r256((size_t)H * W * 8);
    const size_t ext2 = r256((size_t)(H + 2 * cy) * (W + 2 * cx) * 8);
    const size_t nb_it = (size_t)((W + 63) / 64) * H;      // dL/dalpha slots: per image row and 64 columns
    const size_t nb_dh = dh_blocks(H, W, psf, bwd_rad(psf));
    size_t o = 0;
    L.list = o; o += r256(tap_list_bytes(psf));
    L.qw = o; o += pl2;
    L.s = o; o += pl;
    L.ab = o; o += pl2;
    L.c = o; o += pl;
    L.du = o; o += pl;
    L.ds = o; o += pl;
    L.lamA = o; o += pl;
    L.lamB = o; o += pl;
    L.ext = o; o += ext2;   // B^T (a, bb), then A^T ds: the extended grid (periodic: the image grid)
    L.bd2 = o; o += r256((size_t)(2 * W + 2 * H) * 8);   // folded border values of B^T (a, bb)
    L.bd1 = o; o += r256((size_t)(2 * W + 2 * H) * 4);   // and of A^T ds
    L.part = o; o += r256(nb_dh * psf.ph * psf.pw * 8);
    L.apart = o; o += r256(nb_it * 8);
    L.dh = o; o += r256((size_t)psf.ph * psf.pw * 8);
    L.da = o; o += 256;
    L.total = o;
    return L;
}

size_t backward_ws_bytes(int H, int W, const PsfDev& psf, bool through_wiener)
{
    BwdLayout L = bwd_layout(H, W, psf);
    size_t need = L.total;
    if (through_wiener) {
        // after the iteration planes (lam0 lives in lamA/lamB, dh/da are kept):
        // M, S1, S2, h^ (half planes, complex64) + u_pre, G, R (real planes)
        const size_t half = r256((size_t)H * (W / 2 + 1) * 8), pl = r256((size_t)H * W * 4);
        need += 4 * half + 3 * pl;
    }
    return need;
}

// Stage-1 tile shape of the recomputation: by the tiles of the whole batch
// (every shape gives the same bits), as the forward picks its default (a
// large batch of several images: 32 x 512).
template <int RAD>
static void launch_bwd_stage1(int B, const float* f, const float* u, float2* qw, float* s, int H, int W, int pitch,
                              const float* taps, const int* nt, const IterParams& p, const BwdZ& z, hipStream_t st)
{
    const long tiles64 = (long)B * ((W + 63) / 64) * ((H + 63) / 64);
    auto go = [&](auto th, auto ntr) {
        constexpr int TH = decltype(th)::value, NT = decltype(ntr)::value;
        const dim3 g((W + 63) / 64, (H + TH - 1) / TH, B);
        hipLaunchKernelGGL((bwd_stage1<RAD, TH, NT>), g, dim3(NT), 0, st, u, f, qw, s, H, W, pitch, taps, nt, p, z);
    };
    if (tiles64 >= 1024 && B > 1)
        go(std::integral_constant<int, 32>{}, std::integral_constant<int, 512>{});
    else if (tiles64 >= 1024)
        go(std::integral_constant<int, 32>{}, std::integral_constant<int, 256>{});
    else if (tiles64 >= 256)
        go(std::integral_constant<int, 32>{}, std::integral_constant<int, 512>{});
    else
        go(std::integral_constant<int, 16>{}, std::integral_constant<int, 512>{});
}

// One reversed iteration for the B images of a batch (lam: dL/du^{k+1} with
// its pitch and image stride; u: the checkpoints u^k).
template <int RAD, int TH>
static void launch_bwd_iter(int B, const float* f, const float* u, const float* lam, int lam_pitch, size_t lam_z,
                            float* lam_out, float* grad_f, int H, int W, int pitch, const PsfDev& psf,
                            const IterParams& p, unsigned char* w8, const BwdLayout& L, const BwdZ& z, hipStream_t st)
{
    const float* taps = reinterpret_cast<const float*>(w8 + L.list + tap_packed_offset(psf.ph, psf.pw));
    const int* nt = reinterpret_cast<const int*>(w8 + L.list);
    float2* qw = reinterpret_cast<float2*>(w8 + L.qw);
    float* s = reinterpret_cast<float*>(w8 + L.s);
    float2* ab = reinterpret_cast<float2*>(w8 + L.ab);
    float* c = reinterpret_cast<float*>(w8 + L.c);
    float* du = reinterpret_cast<float*>(w8 + L.du);
    float* ds = reinterpret_cast<float*>(w8 + L.ds);
    double* part = reinterpret_cast<double*>(w8 + L.part);
    double* apart = reinterpret_cast<double*>(w8 + L.apart);
    const int cy = (psf.ph - 1) / 2, cx = (psf.pw - 1) / 2;
    const bool per = p.bc == BC_PERIODIC;
    const size_t zw = z.ws;
    // the transposed blurs' outputs: the extended grid (EH x EW, origin
    // (-cy, -cx)) with the border folded into bd; periodic: the image grid
    const int EH = per ? H : H + 2 * cy, EW = per ? W : W + 2 * cx;
    const int oy = per ? 0 : cy, ox = per ? 0 : cx;
    const dim3 ge((EW + 63) / 64, (EH + TH - 1) / TH, B);
    const unsigned nbd = (unsigned)((2 * W + 2 * H + 255) / 256);

    launch_bwd_stage1<RAD>(B, f, u, qw, s, H, W, pitch, taps, nt, p, z, st);
    const dim3 gi((W + 63) / 64, (H + TH - 1) / TH, B);
    hipLaunchKernelGGL((adj_update<RAD, TH>), gi, dim3(BW_NT), 0, st, (const float2*)qw, u, lam, lam_pitch, ab, c,
                       du, apart, H, W, pitch, taps, nt, p, z, lam_z);
    // dq, dW = B^T (a, b)
    float2* ext2 = reinterpret_cast<float2*>(w8 + L.ext);
    float2* bd2 = per ? nullptr : reinterpret_cast<float2*>(w8 + L.bd2);
    hipLaunchKernelGGL((adj_stencil<RAD, TH, -1, float2>), ge, dim3(BW_NT), 0, st, (const float2*)ab, W, H, W,
                       per ? 1 : 0, ext2, EW, -oy, -ox, EH, EW, taps, nt, zw);
    if (!per)
        hipLaunchKernelGGL(adj_fold_border<float2>, dim3(nbd, 1, B), dim3(256), 0, st, (const float2*)ext2, EW, cy, cx,
                           H, W, bd2, zw);
    hipLaunchKernelGGL(adj_point, dim3((W + 255) / 256, H, B), dim3(256), 0, st, (const float2*)ext2, EW, oy, ox,
                       (const float2*)bd2, (const float2*)qw, (const float*)s, f, grad_f, ds, H, W, pitch, p, z);
    // A^T ds
    float* ext1 = reinterpret_cast<float*>(w8 + L.ext);
    float* bd1 = per ? nullptr : reinterpret_cast<float*>(w8 + L.bd1);
    hipLaunchKernelGGL((adj_stencil<RAD, TH, 1, float>), ge, dim3(BW_NT), 0, st, (const float*)ds, W, H, W,
                       per ? 1 : 0, ext1, EW, -oy, -ox, EH, EW, taps, nt, zw);
    if (!per)
        hipLaunchKernelGGL(adj_fold_border<float>, dim3(nbd, 1, B), dim3(256), 0, st, (const float*)ext1, EW, cy, cx, H,
                           W, bd1, zw);
    hipLaunchKernelGGL((adj_tv<TH>), dim3((W + 63) / 64, (H + TH - 1) / TH, B), dim3(BW_NT), 0, st, u, pitch,
                       (const float*)c, (const float*)du, (const float*)ext1, EW, oy, ox, (const float*)bd1, lam_out,
                       H, W, p, z);
    if constexpr (RAD == 16) {
        if (dh_on_mfma(psf, RAD)) {
            hipLaunchKernelGGL((adj_dh_mfma<RAD>), dim3((W + DHM_TW - 1) / DHM_TW, (H + DHM_SEG - 1) / DHM_SEG, B),
                               dim3(DHM_NT), 0, st, (const float2*)ab, (const float2*)qw, (const float*)ds, u, pitch, H, W,
                               psf.ph, psf.pw, p.bc, part, z);
            return;
        }
    }
    hipLaunchKernelGGL((adj_dh<RAD>), dim3((W + 63) / 64, (H + DH_TH - 1) / DH_TH, B), dim3(BW_NT), 0, st,
                       (const float2*)ab, (const float2*)qw, (const float*)ds, u, pitch, H, W, psf.ph, psf.pw, p.bc,
                       part, z);
}

template <int RAD>
static void launch_bwd_iter_th(int th, int B, const float* f, const float* u, const float* lam, int lam_pitch,
                               size_t lam_z, float* lam_out, float* grad_f, int H, int W, int pitch,
                               const PsfDev& psf, const IterParams& p, unsigned char* w8, const BwdLayout& L,
                               const BwdZ& z, hipStream_t st)
{
    switch (th) {
        case 4:
            launch_bwd_iter<RAD, 4>(B, f, u, lam, lam_pitch, lam_z, lam_out, grad_f, H, W, pitch, psf, p, w8, L, z, st);
            break;
        case 16:
            launch_bwd_iter<RAD, 16>(B, f, u, lam, lam_pitch, lam_z, lam_out, grad_f, H, W, pitch, psf, p, w8, L, z, st);
            break;
        case 32:
            launch_bwd_iter<RAD, 32>(B, f, u, lam, lam_pitch, lam_z, lam_out, grad_f, H, W, pitch, psf, p, w8, L, z, st);
            break;
        default:
            launch_bwd_iter<RAD, 8>(B, f, u, lam, lam_pitch, lam_z, lam_out, grad_f, H, W, pitch, psf, p, w8, L, z, st);
            break;
    }
}

size_t backward_batch_stride(int H, int W, const PsfDev& psf, bool through_wiener)
{
    return r256(backward_ws_bytes(H, W, psf, through_wiener));
}

int launch_rrrl_backward_batch(int B, const float* f, const float* ckpt, const float* grad_uK, int H, int W,
                               int pitch, size_t img_stride, size_t ck_stride, const PsfDev& psf, size_t taps_stride,
                               const float* alpha, const IterParams& p, int iters, bool through_wiener, double K,
                               float pos_floor, float* grad_f, float* grad_taps, float* grad_alpha, float* grad_u0,
                               void* ws, size_t ws_stride, hipStream_t st)
{
    const int rad = bwd_rad(psf);
    if (rad < 0) return -2;
    unsigned char* w8 = reinterpret_cast<unsigned char*>(ws);
    const BwdLayout L = bwd_layout(H, W, psf);
    const int PP = psf.ph * psf.pw;
    const int th = bwd_th(p, B, H, W);
    const BwdZ z{ws_stride, img_stride, ck_stride, alpha};
    const size_t zw = ws_stride;
    const size_t nb_it = (size_t)((W + 63) / 64) * H;
    const size_t nb_dh = dh_blocks(H, W, psf, rad);
    double* part = reinterpret_cast<double*>(w8 + L.part);
    double* apart = reinterpret_cast<double*>(w8 + L.apart);
    double* dh = reinterpret_cast<double*>(w8 + L.dh);
    double* da = reinterpret_cast<double*>(w8 + L.da);
    float* lamA = reinterpret_cast<float*>(w8 + L.lamA);
    float* lamB = reinterpret_cast<float*>(w8 + L.lamB);

    launch_compile_taps(psf, w8 + L.list, st, ZBatch{B, taps_stride, zw});
    hipLaunchKernelGGL(fill_zero_f64, dim3((unsigned)((nb_dh * PP + 255) / 256), 1, B), dim3(256), 0, st, part,
                       nb_dh * PP, zw);
    hipLaunchKernelGGL(fill_zero_f64, dim3((unsigned)((nb_it + 255) / 256), 1, B), dim3(256), 0, st, apart, nb_it, zw);
    hipLaunchKernelGGL(fill_zero_f32, dim3((W + 255) / 256, H, B), dim3(256), 0, st, grad_f, W, H, pitch, img_stride);

    const float* lam = grad_uK;
    int lam_pitch = pitch;
    size_t lam_z = img_stride;
    for (int k = iters - 1; k >= 0; --k) {
        float* lam_out = (k % 2 == 0) ? lamA : lamB;
        const float* u = ckpt + (size_t)k * H * pitch;
        switch (rad) {
            case 4:
                launch_bwd_iter_th<4>(th, B, f, u, lam, lam_pitch, lam_z, lam_out, grad_f, H, W, pitch, psf, p, w8, L, z, st);
                break;
            case 8:
                launch_bwd_iter_th<8>(th, B, f, u, lam, lam_pitch, lam_z, lam_out, grad_f, H, W, pitch, psf, p, w8, L, z, st);
                break;
            case 16:
                launch_bwd_iter_th<16>(th, B, f, u, lam, lam_pitch, lam_z, lam_out, grad_f, H, W, pitch, psf, p, w8, L, z, st);
                break;
            default:
                launch_bwd_iter_th<32>(th, B, f, u, lam, lam_pitch, lam_z, lam_out, grad_f, H, W, pitch, psf, p, w8, L, z, st);
                break;
        }
        lam = lam_out;
        lam_pitch = W;
        lam_z = zw;
    }
    hipLaunchKernelGGL(adj_reduce, dim3((PP + 255) / 256, 1, B), dim3(256), 0, st, (const double*)part, (int)nb_dh, PP,
                       (const double*)apart, (int)nb_it, dh, da, zw);
    if (iters == 0) {
        // no iteration: lam0 = grad_uK, dalpha = 0 (apart zeroed)
        hipLaunchKernelGGL(copy_plane, dim3((W + 255) / 256, H, B), dim3(256), 0, st, grad_uK, pitch, lamA, W, W,
                           img_stride, zw);
        lam = lamA;
    }
    // lam now holds dL/du^0 (dense, pitch W, in each image's workspace)
    if (grad_u0)
        hipLaunchKernelGGL(copy_plane, dim3((W + 255) / 256, H, B), dim3(256), 0, st, lam, W, grad_u0, pitch, W, zw,
                           img_stride);
    if (through_wiener) {
        const size_t half = r256((size_t)H * (W / 2 + 1) * 8), pl = r256((size_t)H * W * 4);
        unsigned char* wb = w8 + L.total;
        float2* Sa = reinterpret_cast<float2*>(wb);
        float2* Sb = reinterpret_cast<float2*>(wb + half);
        float2* M = reinterpret_cast<float2*>(wb + 2 * half);
        float2* hh = reinterpret_cast<float2*>(wb + 3 * half);
        float* upre = reinterpret_cast<float*>(wb + 4 * half);
        float* G = reinterpret_cast<float*>(wb + 4 * half + pl);
        float* R = reinterpret_cast<float*>(wb + 4 * half + 2 * pl);
        const size_t nh = (size_t)H * (W / 2 + 1);
        // M, h^; F^ = DFT(f); u_pre = IDFT(F^ M) (no floor); G = lam0 1[u_pre > floor]
        launch_wiener_mult(psf, H, W, K, M, hh, st, ZBatch{B, taps_stride, zw, zw});
        launch_fft2_forward(f, pitch, H, W, Sa, st, ZBatch{B, img_stride, zw});
        launch_spectral_mul(Sa, M, false, Sb, nh, st, ZBatch{B, zw, zw, zw});
        launch_fft2_inverse(Sb, H, W, upre, W, -INFINITY, false, st, ZBatch{B, zw, zw});
        hipLaunchKernelGGL(wiener_mask, dim3((W + 255) / 256, H, B), dim3(256), 0, st, lam, (const float*)upre, G, W,
                           pos_floor, zw);
        launch_fft2_forward(G, W, H, W, Sb, st, ZBatch{B, zw, zw});                   // Sb = G^
        launch_wiener_dh_prep(Sa, Sb, hh, Sa, nh, K, st, ZBatch{B, zw});              // Sa <- Y
        launch_spectral_mul(Sb, M, true, Sb, nh, st, ZBatch{B, zw, zw, zw});          // dL/df += IDFT(G^ conj M)
        launch_fft2_inverse(Sb, H, W, grad_f, pitch, 0.0f, true, st, ZBatch{B, zw, img_stride});
        launch_fft2_inverse(Sa, H, W, R, W, -INFINITY, false, st, ZBatch{B, zw, zw});  // R = IDFT(Y)
        hipLaunchKernelGGL(wiener_dh_gather, dim3((PP + 255) / 256, 1, B), dim3(256), 0, st, (const float*)R, H, W,
                           psf.ph, psf.pw, dh, zw);
    }
    hipLaunchKernelGGL(write_grads, dim3((PP + 255) / 256, 1, B), dim3(256), 0, st, (const double*)dh, PP,
                       (const double*)da, grad_taps, grad_alpha, zw);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int launch_rrrl_backward(const float* f, const float* ckpt, const float* grad_uK, int H, int W, int pitch,
                         const PsfDev& psf, const IterParams& p, int iters, bool through_wiener, double K,
                         float pos_floor, float* grad_f, float* grad_taps, float* grad_alpha, float* grad_u0,
                         void* ws, hipStream_t st)
{
    return launch_rrrl_backward_batch(1, f, ckpt, grad_uK, H, W, pitch, 0, 0, psf, 0, nullptr, p, iters,
                                      through_wiener, K, pos_floor, grad_f, grad_taps, grad_alpha, grad_u0, ws, 0, st);
}

void launch_wiener_dh_prep(const float2* Fh, const float2* Gh, const float2* hh, float2* Y, size_t n, double K,
                           hipStream_t st, ZBatch zb)
{
    hipLaunchKernelGGL(wiener_dh_spectrum, dim3((unsigned)((n + 255) / 256), 1, zb.n), dim3(256), 0, st, Fh, Gh, hh, Y,
                       n, K, zb.s0);
}

}  // namespace deblur
