// Single-image launcher of the fused box-iteration kernel (tile body in
// box_seg.hpp).  Five tile shapes per orientation; every shape gives
// bitwise-identical results (re-basing points are image coordinates and the
// tile arithmetic is compiled without multiply-add contraction).
#include <mutex>

#include "box_seg.hpp"

namespace deblur {

// Tiles in raster order (along the blur axis fastest), remapped so that the
// workgroups of one XCD take a contiguous range: tiles that share halos then
// mostly share an L2.
// blockIdx.z = image of a batch of equally shaped images (strides in z).
template <bool VERT, int TA, int TC>
__global__ void __launch_bounds__(BOX_NT) rrrl_box_iter(const float* __restrict__ u, const float* __restrict__ f,
                                                        float* __restrict__ un, float* __restrict__ ckpt, int pitch,
                                                        BoxGeom g, IterParams p, int tiles_along, IterZ z)
{
    extern __shared__ __align__(16) float box_lds[];
    const int w = xcd_group(blockIdx.x, gridDim.x);
    const int tc = w / tiles_along, ta = w - tc * tiles_along;
    if (z.alpha) p.alpha = z.alpha[blockIdx.z];
    box_seg_tile<VERT, TA, TC>(box_lds, zadv(u, z.u), zadv(f, z.f), zadv(un, z.un), ckpt ? zadv(ckpt, z.ck) : nullptr,
                               pitch, g, p, ta * TA, tc * TC);
}

template <bool VERT, int TA, int TC>
static void launch_box(const float* f, const float* u, float* un, float* ckpt, int H, int W, int pitch, int L,
                       float frac, const IterParams& p, hipStream_t st, int B, const IterZ& z)
{
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rrrl_box_iter<VERT, TA, TC>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    });
    const BoxGeom g = box_geom<VERT, TA, TC>(H, W, L, frac);
    const int ta = (g.N + TA - 1) / TA, tc = (g.M + TC - 1) / TC;
    const size_t lds = (size_t)box_lds_words<VERT, TA, TC>(g) * sizeof(float);
    hipLaunchKernelGGL((rrrl_box_iter<VERT, TA, TC>), dim3(ta * tc, 1, B), dim3(BOX_NT), lds, st, u, f, un, ckpt, pitch,
                       g, p, ta, z);
}

int box_num_variants() { return BOX_VARIANTS; }

// Default shape per orientation and size (variant 0); 1..5 explicit.  Images
// up to 512^2 take the 64x4 tiles (one output per thread), which spread them
// over more compute units.
int box_default_variant(int H, int W, bool vert)
{
    (void)vert;
    if ((long)H * W <= 512L * 512L) return 5;
    return 1;
}

int launch_rrrl_box_iter(const float* f, const float* u, float* un, float* ckpt, int H, int W, int pitch, int L,
                         float frac, bool vert, const IterParams& p, hipStream_t st, int B, const IterZ& z)
{
    const int v = p.tile > 0 ? p.tile : box_default_variant(H, W, vert);
    if (v > box_num_variants()) return -2;
    if (vert)
        with_box_shape<true>(v, [&](auto ta, auto tc) {
            launch_box<true, decltype(ta)::value, decltype(tc)::value>(f, u, un, ckpt, H, W, pitch, L, frac, p, st, B, z);
        });
    else
        with_box_shape<false>(v, [&](auto ta, auto tc) {
            launch_box<false, decltype(ta)::value, decltype(tc)::value>(f, u, un, ckpt, H, W, pitch, L, frac, p, st, B, z);
        });
    return 0;
}

}  // namespace deblur
