// Starting images for RRRL without the Wiener step (Sec. 2.3: the RRRL
// columns of Table 1 iterate from an initial image the paper does not
// state).  Two starts:
//   flat:     u0 = max(mean(f), pos_floor) everywhere;
//   observed: u0 = max(f, pos_floor).
// Both are positive, as the multiplicative update requires (Sec. 3.2).
#include "common.hpp"
#include "launch.hpp"

namespace deblur {

constexpr int START_NT = 1024;

// One workgroup: the FP64 sum of f in a fixed order (wavefront w takes rows
// w, w + 16, ...; its lanes run along x), a fixed reduction tree, then the
// fill.  A one-time step of about the cost of one pass over the image.
__global__ void __launch_bounds__(START_NT) start_flat(const float* __restrict__ f, float* __restrict__ u0, int H,
                                                      int W, int pitch, float pos_floor)
{
    __shared__ double part[START_NT];
    constexpr int NW = START_NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double acc = 0.0;
    for (int y = w; y < H; y += NW)
        for (int x = lane; x < W; x += 64) acc += (double)f[(size_t)y * pitch + x];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = START_NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    const float v = fmaxf((float)(part[0] / ((double)H * (double)W)), pos_floor);
    for (int y = w; y < H; y += NW)
        for (int x = lane; x < W; x += 64) u0[(size_t)y * pitch + x] = v;
}

__global__ void __launch_bounds__(256) start_observed(const float* __restrict__ f, float* __restrict__ u0, int H,
                                                     int W, int pitch, float pos_floor)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x < W && y < H) u0[(size_t)y * pitch + x] = fmaxf(f[(size_t)y * pitch + x], pos_floor);
}

int launch_rrrl_start(const float* f, float* u0, int H, int W, int pitch, int mode, float pos_floor, hipStream_t st)
{
    if (mode == 0)
        hipLaunchKernelGGL(start_flat, dim3(1), dim3(START_NT), 0, st, f, u0, H, W, pitch, pos_floor);
    else
        hipLaunchKernelGGL(start_observed, dim3((W + 63) / 64, (H + 3) / 4), dim3(256), 0, st, f, u0, H, W, pitch,
                           pos_floor);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace deblur
