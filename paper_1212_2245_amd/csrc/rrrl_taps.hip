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

// Compacted list of the non-zero taps, row-major order: {dy, dx, w bits, 0},
// count in hdr[0].  Then the column groups: runs of vertically adjacent
// non-zero taps of one PSF column, split every TAP_GROUP_MAX rows, ordered by
// run length S (longest first) and within one length by column and row;
// hdr[1] = number of groups, hdr[1 + S] = number of groups of length S.
// Single workgroup of 256 threads (pw <= 256).
__global__ void __launch_bounds__(256) build_tap_list(PsfDev psf, int4* __restrict__ list,
                                                      TapGroup* __restrict__ groups, int* __restrict__ hdr)
{
    __shared__ int counts[256];
    __shared__ int cls[TAP_GROUP_MAX][256];   // groups of length S+1 in column i, then their offsets
    __shared__ int cls_base[TAP_GROUP_MAX];
    const int n = psf.ph * psf.pw;
    const int per = (n + 255) / 256;
    const int b = threadIdx.x * per, e = min(n, b + per);
    int c = 0;
    for (int k = b; k < e; ++k) c += psf_weight(psf, k / psf.pw, k % psf.pw) != 0.0f;
    counts[threadIdx.x] = c;
    __syncthreads();
    // inclusive Hillis-Steele scan
    for (int off = 1; off < 256; off <<= 1) {
        const int v = threadIdx.x >= off ? counts[threadIdx.x - off] : 0;
        __syncthreads();
        counts[threadIdx.x] += v;
        __syncthreads();
    }
    int o = counts[threadIdx.x] - c;
    const int cy = (psf.ph - 1) / 2, cx = (psf.pw - 1) / 2;
    for (int k = b; k < e; ++k) {
        const int j = k / psf.pw, i = k % psf.pw;
        const float w = psf_weight(psf, j, i);
        if (w != 0.0f) list[o++] = make_int4(j - cy, i - cx, __float_as_int(w), 0);
    }
    if (threadIdx.x == 255) hdr[0] = counts[255];

    // column groups: thread `col` walks PSF column col; a run of r adjacent
    // non-zero taps gives floor(r/8) groups of 8 and one of r mod 8
    const int col = threadIdx.x;
    for (int q = 0; q < TAP_GROUP_MAX; ++q) cls[q][col] = 0;
    if (col < psf.pw) {
        int run = 0;
        for (int j = 0; j <= psf.ph; ++j) {
            const bool nz = j < psf.ph && psf_weight(psf, j, col) != 0.0f;
            if (nz && run < TAP_GROUP_MAX) {
                ++run;
                continue;
            }
            if (run > 0) ++cls[run - 1][col];
            run = nz ? 1 : 0;
        }
    }
    __syncthreads();
    // exclusive prefix over the columns, one length class per thread
    if (threadIdx.x < TAP_GROUP_MAX) {
        int acc = 0;
        for (int i = 0; i < psf.pw; ++i) {
            const int v = cls[threadIdx.x][i];
            cls[threadIdx.x][i] = acc;
            acc += v;
        }
        counts[threadIdx.x] = acc;   // total of the class
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int base = 0;
        for (int q = TAP_GROUP_MAX - 1; q >= 0; --q) {
            cls_base[q] = base;
            base += counts[q];
            hdr[2 + q] = counts[q];
        }
        hdr[1] = base;
    }
    __syncthreads();
    if (col < psf.pw) {
        int next[TAP_GROUP_MAX];
        for (int q = 0; q < TAP_GROUP_MAX; ++q) next[q] = cls_base[q] + cls[q][col];
        int run = 0, j0 = 0;
        for (int j = 0; j <= psf.ph; ++j) {
            const bool nz = j < psf.ph && psf_weight(psf, j, col) != 0.0f;
            if (nz && run < TAP_GROUP_MAX) {
                if (run == 0) j0 = j;
                ++run;
                continue;
            }
            if (run > 0) {
                TapGroup& g = groups[next[run - 1]++];
                g.dx = col - cx;
                g.dy0 = j0 - cy;
                g.S = run;
                g.pad = 0;
                for (int s = 0; s < TAP_GROUP_MAX; ++s) g.w[s] = s < run ? psf_weight(psf, j0 + s, col) : 0.0f;
            }
            run = nz ? 1 : 0;
            j0 = j;
        }
    }
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
                        const TapGroup* taps, const int* nt, const IterParams& p, hipStream_t st)
{
    const dim3 g((W + 63) / 64, (H + TH - 1) / TH);
    hipLaunchKernelGGL((rrrl_taps_stage1<RAD, TH, NT>), g, dim3(NT), 0, st, u, f, qw, s_out, H, W, pitch, taps, nt,
                       p);
}

template <int RAD, int TH, int NT>
static void stage2_inst(const float2* qw, const float* u, float* un, float* ckpt, int H, int W, int pitch,
                        const TapGroup* taps, const int* nt, const IterParams& p, hipStream_t st)
{
    const dim3 g((W + 63) / 64, (H + TH - 1) / TH);
    hipLaunchKernelGGL((rrrl_taps_stage2<RAD, TH, NT>), g, dim3(NT), 0, st, qw, u, un, ckpt, H, W, pitch, taps, nt,
                       p);
}

template <int RAD>
static void launch_stage1_t(int v, const float* f, const float* u, float2* qw, float* s_out, int H, int W,
                            int pitch, const TapGroup* taps, const int* nt, const IterParams& p, hipStream_t st)
{
    switch (v) {
        case 0: stage1_inst<RAD, 64, 1024>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st); break;
        case 1: stage1_inst<RAD, 64, 256>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st); break;
        case 2: stage1_inst<RAD, 32, 256>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st); break;
        case 3: stage1_inst<RAD, 32, 512>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st); break;
        case 4: stage1_inst<RAD, 16, 256>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st); break;
        case 5: stage1_inst<RAD, 16, 512>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st); break;
        case 6: stage1_inst<RAD, 32, 1024>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st); break;
        default: stage1_inst<RAD, 16, 1024>(f, u, qw, s_out, H, W, pitch, taps, nt, p, st); break;
    }
}

template <int RAD>
static void launch_stage2_t(int v, const float2* qw, const float* u, float* un, float* ckpt, int H, int W,
                            int pitch, const TapGroup* taps, const int* nt, const IterParams& p, hipStream_t st)
{
    // 64-row tiles of the two-channel plane exceed LDS for the largest radius
    if (RAD >= 32 && (v == 0 || v == 1)) v = 3;
    switch (v) {
        case 0: stage2_inst<RAD, (RAD >= 32 ? 32 : 64), 1024>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st); break;
        case 1: stage2_inst<RAD, (RAD >= 32 ? 32 : 64), 256>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st); break;
        case 2: stage2_inst<RAD, 32, 256>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st); break;
        case 3: stage2_inst<RAD, 32, 512>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st); break;
        case 4: stage2_inst<RAD, 16, 256>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st); break;
        case 5: stage2_inst<RAD, 16, 512>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st); break;
        case 6: stage2_inst<RAD, 32, 1024>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st); break;
        default: stage2_inst<RAD, 16, 1024>(qw, u, un, ckpt, H, W, pitch, taps, nt, p, st); break;
    }
}

// Default variant when the caller does not choose one: enough tiles to give
// every CU several workgroups, else the smallest tiles.
static int default_variant(int H, int W, int stage)
{
    const long tiles64 = (long)((W + 63) / 64) * ((H + 63) / 64);
    if (tiles64 >= 1024) return stage == 1 ? 1 : 2;
    if (tiles64 >= 256) return stage == 1 ? 0 : 3;
    return 4;
}

size_t tap_list_bytes(const PsfDev& psf)
{
    const size_t P = (size_t)psf.ph * psf.pw;
    return tap_groups_offset(psf.ph, psf.pw) + sizeof(TapGroup) * P;
}

void launch_compile_taps(const PsfDev& psf, void* list, hipStream_t st)
{
    unsigned char* w8 = reinterpret_cast<unsigned char*>(list);
    hipLaunchKernelGGL(build_tap_list, dim3(1), dim3(256), 0, st, psf, reinterpret_cast<int4*>(w8 + 256),
                       reinterpret_cast<TapGroup*>(w8 + tap_groups_offset(psf.ph, psf.pw)),
                       reinterpret_cast<int*>(w8));
}

static int psf_radius_class(const PsfDev& psf)
{
    return tap_radius_class(max((psf.ph - 1) / 2, (psf.pw - 1) / 2));
}

int launch_taps_stage1(const float* f, const float* u, float* qw, int H, int W, int pitch, const PsfDev& psf,
                       const void* list, const IterParams& p, int variant, hipStream_t st, float* s_out)
{
    const int v = variant > 0 ? variant - 1 : default_variant(H, W, 1);
    const unsigned char* w8 = reinterpret_cast<const unsigned char*>(list);
    const int* nt = reinterpret_cast<const int*>(w8);
    const TapGroup* taps = reinterpret_cast<const TapGroup*>(w8 + tap_groups_offset(psf.ph, psf.pw));
    float2* q2 = reinterpret_cast<float2*>(qw);
    switch (psf_radius_class(psf)) {
        case 4: launch_stage1_t<4>(v, f, u, q2, s_out, H, W, pitch, taps, nt, p, st); break;
        case 8: launch_stage1_t<8>(v, f, u, q2, s_out, H, W, pitch, taps, nt, p, st); break;
        case 16: launch_stage1_t<16>(v, f, u, q2, s_out, H, W, pitch, taps, nt, p, st); break;
        case 32: launch_stage1_t<32>(v, f, u, q2, s_out, H, W, pitch, taps, nt, p, st); break;
        default: return -2;
    }
    return 0;
}

int launch_taps_stage2(const float* qw, const float* u, float* un, float* ckpt, int H, int W, int pitch,
                       const PsfDev& psf, const void* list, const IterParams& p, int variant, hipStream_t st)
{
    const int v = variant > 0 ? variant - 1 : default_variant(H, W, 2);
    const unsigned char* w8 = reinterpret_cast<const unsigned char*>(list);
    const int* nt = reinterpret_cast<const int*>(w8);
    const TapGroup* taps = reinterpret_cast<const TapGroup*>(w8 + tap_groups_offset(psf.ph, psf.pw));
    const float2* q2 = reinterpret_cast<const float2*>(qw);
    switch (psf_radius_class(psf)) {
        case 4: launch_stage2_t<4>(v, q2, u, un, ckpt, H, W, pitch, taps, nt, p, st); break;
        case 8: launch_stage2_t<8>(v, q2, u, un, ckpt, H, W, pitch, taps, nt, p, st); break;
        case 16: launch_stage2_t<16>(v, q2, u, un, ckpt, H, W, pitch, taps, nt, p, st); break;
        case 32: launch_stage2_t<32>(v, q2, u, un, ckpt, H, W, pitch, taps, nt, p, st); break;
        default: return -2;
    }
    return 0;
}

}  // namespace deblur
