// RRRL iteration (Sec. 2.3, eqs. (9)-(12)) for a general PSF given as taps,
// by direct summation in the spatial domain (Sec. 4.1, 4.3) on LDS tiles.
//
// One iteration = two kernels:
//   stage 1: s = A u (blur), W = Phi'(r_f(s)), q = W f / s   -> plane (q, W)
//   stage 2: N1 = B q, N2 = B W (correlation with h, i.e. convolution with
//            h*), TV term D(u), update u' = u (N1 + a[D]_+) / (N2 - a[D]_-)
// A and B use constant or periodic continuation at the border (Sec. 4.2);
// the diffusion term always has zero flux across the border.
//
// Tiles are 64 columns wide (one wavefront: lane = column, so LDS reads are
// consecutive and conflict-free) and TH rows tall; each of the 4 wavefronts
// of a workgroup owns TH/4 consecutive rows, so one LDS address computation
// per tap serves TH/4 reads with immediate offsets.  Only non-zero taps are
// visited (a compacted tap list built on the device from the PSF).
#include "common.hpp"
#include "launch.hpp"
#include "psf.hpp"
#include "stencil_tiles.hpp"

namespace deblur {

// Inclusive prefix sums over the 256 threads of a workgroup of N values per
// thread (wavefront shuffles, one barrier round through `tot`).
template <int N>
DEBLUR_DEV void block_scan256(int (&v)[N], int (*tot)[N])
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const int o = __shfl_up(v[q], d, 64);
            if (lane >= d) v[q] += o;
        }
    }
    __syncthreads();
    if (lane == 63) {
#pragma unroll
        for (int q = 0; q < N; ++q) tot[wv][q] = v[q];
    }
    __syncthreads();
    for (int w = 0; w < wv; ++w) {
#pragma unroll
        for (int q = 0; q < N; ++q) v[q] += tot[w][q];
    }
}

// Compacted list of the non-zero taps, row-major order: {dy, dx, w bits, 0},
// count in hdr[0].  Then the column groups: runs of vertically adjacent
// non-zero taps of one PSF column, split every TAP_GROUP_MAX rows, ordered by
// run length S (longest first) and within one length by column and row;
// hdr[1] = number of groups, hdr[1 + S] = number of groups of length S;
// the packed copy (one header word and S weights per group) has hdr[10]
// words.
// Single workgroup of 256 threads (pw <= 256).
__global__ void __launch_bounds__(256) build_tap_list(PsfDev psf, int4* __restrict__ list,
                                                      TapGroup* __restrict__ groups, float* __restrict__ packed,
                                                      int* __restrict__ hdr, size_t zt, size_t zl)
{
    // blockIdx.z = PSF of a batch (byte strides of the taps and of the lists)
    if (psf.taps) psf.taps = global_ptr(zadv(psf.taps, zt));
    list = zadv(list, zl);
    groups = zadv(groups, zl);
    packed = zadv(packed, zl);
    hdr = zadv(hdr, zl);
    __shared__ int tot1[4][1], tot8[4][TAP_GROUP_MAX];
    __shared__ int cls_base[TAP_GROUP_MAX], word_base[TAP_GROUP_MAX];
    __shared__ float hs[65 * 65];             // the PSF array (ph, pw <= 65)
    __shared__ unsigned long long mask0[65];  // per column: non-zero rows 0..63
    __shared__ int mask1[65];                 // per column: row 64 non-zero
    const int n = psf.ph * psf.pw;
    stage_to_lds_n<8>(hs, n, [&](int t) { return psf_weight(psf, t / psf.pw, t % psf.pw); });
    __syncthreads();
    auto wgt = [&](int j, int i) { return hs[j * psf.pw + i]; };
    const int per = (n + 255) / 256;
    const int b = threadIdx.x * per, e = min(n, b + per);
    int c[1] = {0};
    for (int k = b; k < e; ++k) c[0] += hs[k] != 0.0f;
    const int mine = c[0];
    block_scan256<1>(c, tot1);
    int o = c[0] - mine;
    const int cy = (psf.ph - 1) / 2, cx = (psf.pw - 1) / 2;
    for (int k = b; k < e; ++k) {
        const int j = k / psf.pw, i = k % psf.pw;
        const float w = hs[k];
        if (w != 0.0f) list[o++] = make_int4(j - cy, i - cx, __float_as_int(w), 0);
    }
    if (threadIdx.x == 255) hdr[0] = c[0];

    // column groups.  The non-zero pattern of each PSF column as a 65-bit mask
    // (rows 0..63 by one wavefront ballot, row 64 separately); thread `col`
    // (< pw) then visits the runs of its column: a run of r adjacent non-zero
    // taps gives floor(r/8) groups of 8 and one of r mod 8.
    const int col = threadIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = wv; i < psf.pw; i += 4) {
        const unsigned long long m = __ballot(lane < psf.ph && wgt(lane, i) != 0.0f);
        if (lane == 0) {
            mask0[i] = m;
            mask1[i] = psf.ph > 64 && wgt(64, i) != 0.0f;
        }
    }
    __syncthreads();
    const unsigned long long m0 = col < psf.pw ? mask0[col] : 0ull;
    const bool b64 = col < psf.pw && mask1[col] != 0;
    // calls fn(start, length) for every maximal run of set bits of (m0, b64)
    auto for_runs = [&](auto fn) {
        int j = 0;
        while (j <= 64) {
            if (j == 64) {
                if (b64) fn(64, 1);
                break;
            }
            const unsigned long long rest = m0 >> j;
            if (rest == 0ull) {
                j = 64;
                continue;
            }
            const int start = j + __builtin_ctzll(rest);
            const unsigned long long inv = ~(m0 >> start);
            int len = inv == 0ull ? 64 - start : __builtin_ctzll(inv);
            if (len > 64 - start) len = 64 - start;
            if (start + len == 64 && b64) ++len;
            fn(start, len);
            j = start + len + 1;
        }
    };
    int my[TAP_GROUP_MAX];
#pragma unroll
    for (int q = 0; q < TAP_GROUP_MAX; ++q) my[q] = 0;
    for_runs([&](int, int len) {
        my[TAP_GROUP_MAX - 1] += len / TAP_GROUP_MAX;
        const int r = len % TAP_GROUP_MAX;
#pragma unroll
        for (int q = 0; q < TAP_GROUP_MAX - 1; ++q) my[q] += r == q + 1;
    });
    // inclusive scan over the columns of the eight per-length counts
    int sc[TAP_GROUP_MAX];
#pragma unroll
    for (int q = 0; q < TAP_GROUP_MAX; ++q) sc[q] = my[q];
    block_scan256<TAP_GROUP_MAX>(sc, tot8);
    if (threadIdx.x == 255) {
        int base = 0, words = 0;
        for (int q = TAP_GROUP_MAX - 1; q >= 0; --q) {
            cls_base[q] = base;
            word_base[q] = words;
            base += sc[q];
            words += sc[q] * (q + 2);
            hdr[2 + q] = sc[q];
        }
        hdr[1] = base;
        hdr[10] = words;
    }
    __syncthreads();
    int next[TAP_GROUP_MAX];
#pragma unroll
    for (int q = 0; q < TAP_GROUP_MAX; ++q) next[q] = cls_base[q] + sc[q] - my[q];
    auto emit = [&](int j0, int run) {
        int slot = 0;
#pragma unroll
        for (int q = 0; q < TAP_GROUP_MAX; ++q)
            if (run == q + 1) slot = next[q]++;
        float w[TAP_GROUP_MAX];
#pragma unroll
        for (int t = 0; t < TAP_GROUP_MAX; ++t) w[t] = t < run ? wgt(j0 + t, col) : 0.0f;
        int4* g4 = reinterpret_cast<int4*>(groups + slot);
        g4[0] = make_int4(col - cx, j0 - cy, run, 0);
        g4[1] = make_int4(__float_as_int(w[0]), __float_as_int(w[1]), __float_as_int(w[2]), __float_as_int(w[3]));
        g4[2] = make_int4(__float_as_int(w[4]), __float_as_int(w[5]), __float_as_int(w[6]), __float_as_int(w[7]));
        // packed copy: word offset from the group's rank within its length
        const int q = run - 1;
        float* pw_ = packed + word_base[q] + (slot - cls_base[q]) * (run + 1);
        pw_[0] = __int_as_float((int)(((unsigned)(col - cx) & 0xffffu) | ((unsigned)(j0 - cy) << 16)));
        for (int t = 0; t < run; ++t) pw_[1 + t] = w[t];
    };
    for_runs([&](int start, int len) {
        for (int k = 0; k < len; k += TAP_GROUP_MAX) emit(start + k, min(TAP_GROUP_MAX, len - k));
    });
}

// ------------------------------------------------------------ host launchers
int tap_radius_class(int rad)
{
    if (rad <= 4) return 4;
    if (rad <= 8) return 8;
    if (rad <= 16) return 16;
    if (rad <= 32) return 32;
    return -1;
}

// Tile variants (rows per tile TH, threads per workgroup NT); every variant
// visits the taps of a pixel in the same order, so results are bitwise equal.
struct TileVariant {
    int th, nt;
};
static constexpr TileVariant kVariants[] = {{64, 1024}, {64, 256}, {32, 256}, {32, 512}, {16, 256},
                                            {16, 512}, {32, 1024}, {16, 1024}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int taps_num_variants() { return kNumVariants; }

template <int RAD, int TH, int NT>
static void stage1_inst(const float* f, const float* u, float2* qw, float* s_out, int H, int W, int pitch,
                        const float* taps, const int* nt, const IterParams& p, hipStream_t st, int B, const IterZ& z)
{
    const dim3 g((W + 63) / 64, (H + TH - 1) / TH, B);
    hipLaunchKernelGGL((rrrl_taps_stage1<RAD, TH, NT>), g, dim3(NT), 0, st, u, f, qw, s_out, H, W, pitch, taps, nt,
                       p, z);
}

template <int RAD, int TH, int NT>
static void stage2_inst(const float2* qw, const float* u, float* un, float* ckpt, int H, int W, int pitch,
                        const float* taps, const int* nt, const IterParams& p, hipStream_t st, int B, const IterZ& z)
{
    const dim3 g((W + 63) / 64, (H + TH - 1) / TH, B);
    hipLaunchKernelGGL((rrrl_taps_stage2<RAD, TH, NT>), g, dim3(NT), 0, st, qw, u, un, ckpt, H, W, pitch, taps, nt,
                       p, z);
}

template <int RAD>
static void launch_stage1_t(int v, const float* f, const float* u, float2* qw, float* s_out, int H, int W,
                            int pitch, const float* taps, const int* nt, const IterParams& p, hipStream_t st, int B,
                            const IterZ& z)
{
    switch (v) {
        case 0: stage1_inst<RAD, 64, 1024>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st, B, z); break;
        case 1: stage1_inst<RAD, 64, 256>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st, B, z); break;
        case 2: stage1_inst<RAD, 32, 256>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st, B, z); break;
        case 3: stage1_inst<RAD, 32, 512>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st, B, z); break;
        case 4: stage1_inst<RAD, 16, 256>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st, B, z); break;
        case 5: stage1_inst<RAD, 16, 512>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st, B, z); break;
        case 6: stage1_inst<RAD, 32, 1024>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st, B, z); break;
        default: stage1_inst<RAD, 16, 1024>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st, B, z); break;
    }
}

template <int RAD>
static void launch_stage2_t(int v, const float2* qw, const float* u, float* un, float* ckpt, int H, int W,
                            int pitch, const float* taps, const int* nt, const IterParams& p, hipStream_t st, int B,
                            const IterZ& z)
{
    // 64-row tiles of the two-channel plane exceed LDS for the largest radius
    if (RAD >= 32 && (v == 0 || v == 1)) v = 3;
    switch (v) {
        case 0: stage2_inst<RAD, (RAD >= 32 ? 32 : 64), 1024>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st, B, z); break;
        case 1: stage2_inst<RAD, (RAD >= 32 ? 32 : 64), 256>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st, B, z); break;
        case 2: stage2_inst<RAD, 32, 256>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st, B, z); break;
        case 3: stage2_inst<RAD, 32, 512>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st, B, z); break;
        case 4: stage2_inst<RAD, 16, 256>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st, B, z); break;
        case 5: stage2_inst<RAD, 16, 512>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st, B, z); break;
        case 6: stage2_inst<RAD, 32, 1024>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st, B, z); break;
        default: stage2_inst<RAD, 16, 1024>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st, B, z); break;
    }
}

// Default tile shape (index into kVariants) by image size, from a sweep of
// every shape with a sparse (31-px line) and a dense (31x31) PSF at 256^2 ..
// 2048^2: small images want many workgroups (16 rows x 512 threads, 2 rows
// per thread), large ones more rows per thread for reuse of the loaded
// column values (32 x 512, then 32 x 256).  Both stages use the same shape.
// A launch over a batch of B images counts the tiles of all of them; a batch
// that large takes 32 x 512 (64 images of 512^2 with 31x31 line PSFs: 3.29
// ms per 10-iteration forward against 3.56 ms with 32 x 256).
static int default_variant(int H, int W, int B)
{
    const long tiles64 = (long)B * ((W + 63) / 64) * ((H + 63) / 64);
    if (tiles64 >= 1024) return B > 1 ? 3 : 2;
    if (tiles64 >= 256) return 3;
    return 5;
}

size_t tap_list_bytes(const PsfDev& psf)
{
    const size_t P = (size_t)psf.ph * psf.pw;
    return tap_packed_offset(psf.ph, psf.pw) + 4 * 2 * P;
}

void launch_compile_taps(const PsfDev& psf, void* list, hipStream_t st, ZBatch zb)
{
    unsigned char* w8 = reinterpret_cast<unsigned char*>(list);
    hipLaunchKernelGGL(build_tap_list, dim3(1, 1, zb.n), dim3(256), 0, st, psf, reinterpret_cast<int4*>(w8 + 256),
                       reinterpret_cast<TapGroup*>(w8 + tap_groups_offset(psf.ph, psf.pw)),
                       reinterpret_cast<float*>(w8 + tap_packed_offset(psf.ph, psf.pw)), reinterpret_cast<int*>(w8),
                       zb.s0, zb.s1);
}

static int psf_radius_class(const PsfDev& psf)
{
    return tap_radius_class(max((psf.ph - 1) / 2, (psf.pw - 1) / 2));
}

int launch_taps_stage1(const float* f, const float* u, float* qw, int H, int W, int pitch, const PsfDev& psf,
                       const void* list, const IterParams& p, int variant, hipStream_t st, float* s_out, int B,
                       const IterZ& z)
{
    const int v = variant > 0 ? variant - 1 : default_variant(H, W, B);
    const unsigned char* w8 = reinterpret_cast<const unsigned char*>(list);
    const int* nt = reinterpret_cast<const int*>(w8);
    const float* taps = reinterpret_cast<const float*>(w8 + tap_packed_offset(psf.ph, psf.pw));
    float2* q2 = reinterpret_cast<float2*>(qw);
    switch (psf_radius_class(psf)) {
        case 4: launch_stage1_t<4>(v, f, u, q2, s_out, H, W, pitch, taps, nt, p, st, B, z); break;
        case 8: launch_stage1_t<8>(v, f, u, q2, s_out, H, W, pitch, taps, nt, p, st, B, z); break;
        case 16: launch_stage1_t<16>(v, f, u, q2, s_out, H, W, pitch, taps, nt, p, st, B, z); break;
        case 32: launch_stage1_t<32>(v, f, u, q2, s_out, H, W, pitch, taps, nt, p, st, B, z); break;
        default: return -2;
    }
    return 0;
}

int launch_taps_stage2(const float* qw, const float* u, float* un, float* ckpt, int H, int W, int pitch,
                       const PsfDev& psf, const void* list, const IterParams& p, int variant, hipStream_t st, int B,
                       const IterZ& z)
{
    const int v = variant > 0 ? variant - 1 : default_variant(H, W, B);
    const unsigned char* w8 = reinterpret_cast<const unsigned char*>(list);
    const int* nt = reinterpret_cast<const int*>(w8);
    const float* taps = reinterpret_cast<const float*>(w8 + tap_packed_offset(psf.ph, psf.pw));
    const float2* q2 = reinterpret_cast<const float2*>(qw);
    switch (psf_radius_class(psf)) {
        case 4: launch_stage2_t<4>(v, q2, u, un, ckpt, H, W, pitch, taps, nt, p, st, B, z); break;
        case 8: launch_stage2_t<8>(v, q2, u, un, ckpt, H, W, pitch, taps, nt, p, st, B, z); break;
        case 16: launch_stage2_t<16>(v, q2, u, un, ckpt, H, W, pitch, taps, nt, p, st, B, z); break;
        case 32: launch_stage2_t<32>(v, q2, u, un, ckpt, H, W, pitch, taps, nt, p, st, B, z); break;
        default: return -2;
    }
    return 0;
}

}  // namespace deblur
