// Single-image launcher of the fused box-iteration kernel (tiles in
// box_tiles.hpp).
#include <mutex>

#include "box_tiles.hpp"

namespace deblur {

template <bool VERT, int TA, int TC>
__global__ void __launch_bounds__(256) rrrl_box_iter(const float* __restrict__ u, const float* __restrict__ f,
                                                     float* __restrict__ un, float* __restrict__ ckpt, int pitch,
                                                     BoxTile bt, IterParams p)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // vertical blur: tiles in raster order, a contiguous range per XCD, so the
    // tiles above and below (which share halo rows) mostly share an L2 (for
    // horizontal blur the neighbours along the axis are adjacent blocks and
    // the default order measured as fast)
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    const int w = VERT ? xcd_group(b, gridDim.x * gridDim.y) : b;
    const int by = w / gridDim.x, bx = w - by * gridDim.x;
    box_iter_tile<VERT, TA, TC>(smem_raw, u, f, un, ckpt, pitch, bt, p, (VERT ? by : bx) * TA, (VERT ? bx : by) * TC);
}

// ------------------------------------------------------------ host launchers
// Tiles for long boxes need more than 64 KB of dynamic LDS (gfx950 has
// 160 KB per workgroup); the limit is raised once per process.
static void allow_large_lds()
{
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rrrl_box_iter<false, BOXH_WIDE_TA, BOXH_WIDE_TC>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rrrl_box_iter<false, BOXH_TA, BOXH_TC>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&rrrl_box_iter<true, BOXV_TA, BOXV_TC>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    });
}

int launch_rrrl_box_iter(const float* f, const float* u, float* un, float* ckpt, int H, int W, int pitch, int L,
                         float frac, bool vert, const IterParams& p, hipStream_t st)
{
    allow_large_lds();
    // tile shapes: vertical blur BOXV at every size measured (256^2 ..
    // 2048^2); horizontal blur BOXH up to 512^2 (a 256^2 image gives only 64
    // workgroups with wide tiles), BOXH_WIDE above
    if (vert) {
        const BoxTile bt = make_tile(H, W, L, frac, true, BOXV_TA);
        const dim3 g((W + BOXV_TC - 1) / BOXV_TC, (H + BOXV_TA - 1) / BOXV_TA);
        const size_t lds = box_lds_bytes<true, BOXV_TA, BOXV_TC>(bt);
        hipLaunchKernelGGL((rrrl_box_iter<true, BOXV_TA, BOXV_TC>), g, dim3(256), lds, st, u, f, un, ckpt, pitch,
                           bt, p);
    } else if ((long)H * W <= 512L * 512L) {
        const BoxTile bt = make_tile(H, W, L, frac, false, BOXH_TA);
        const dim3 g((W + BOXH_TA - 1) / BOXH_TA, (H + BOXH_TC - 1) / BOXH_TC);
        const size_t lds = box_lds_bytes<false, BOXH_TA, BOXH_TC>(bt);
        hipLaunchKernelGGL((rrrl_box_iter<false, BOXH_TA, BOXH_TC>), g, dim3(256), lds, st, u, f, un, ckpt, pitch,
                           bt, p);
    } else {
        const BoxTile bt = make_tile(H, W, L, frac, false, BOXH_WIDE_TA);
        const dim3 g((W + BOXH_WIDE_TA - 1) / BOXH_WIDE_TA, (H + BOXH_WIDE_TC - 1) / BOXH_WIDE_TC);
        const size_t lds = box_lds_bytes<false, BOXH_WIDE_TA, BOXH_WIDE_TC>(bt);
        hipLaunchKernelGGL((rrrl_box_iter<false, BOXH_WIDE_TA, BOXH_WIDE_TC>), g, dim3(256), lds, st, u, f, un,
                           ckpt, pitch, bt, p);
    }
    return 0;
}


}  // namespace deblur
