// Device helpers shared by the WR3L kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DEBLUR_DEV __device__ __forceinline__

namespace deblur {

enum { BC_REPLICATE = 0, BC_PERIODIC = 1 };

// Index of the continued image (Sec. 4.2): constant continuation clamps,
// periodic continuation wraps.
DEBLUR_DEV int ext_index(int i, int n, int bc)
{
    if (bc == BC_PERIODIC) {
        const int m = i % n;
        return m < 0 ? m + n : m;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b mod 8, each XCD with its own L2).  xcd_group maps block b of n to a work
// index so that the blocks of one XCD take consecutive indices: neighbours
// that share cache lines then share an L2.  A bijection on [0, n).
DEBLUR_DEV int xcd_group(int b, int n)
{
    const int x = b & 7, slot = b >> 3, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + slot;
}

DEBLUR_DEV int clampi(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

// Information divergence r_f(s) = s - f - f ln(s/f) (eq. (7)) in FP32,
// written as f * (x - ln(1+x)) with x = (s-f)/f to avoid the cancellation of
// the literal form near s = f.  |x| < 1/16: Taylor series of x - ln(1+x)
// through x^8 (truncation < 1e-9 relative); x < -1/2: ln(s/f) directly
// (x may round to -1 when s << f).  f <= 0: the limit r_0(s) = s.
DEBLUR_DEV float info_div(float f, float s)
{
    if (!(f > 0.0f)) return s;
    const float x = (s - f) / f;
    float t;
    if (fabsf(x) < 0.0625f) {
        const float p = 0.5f + x * (-1.0f / 3.0f + x * (0.25f + x * (-0.2f + x * (1.0f / 6.0f
                        + x * (-1.0f / 7.0f + x * 0.125f)))));
        t = x * x * p;
    } else if (x < -0.5f) {
        t = x - logf(s / f);
    } else {
        t = x - log1pf(x);
    }
    return f * t;
}

// Penaliser derivative of the regularised L1 / TV type (Sec. 2.3), up to the
// common factor 1/2 that cancels in the RRRL quotient: (z + eps^2)^(-1/2).
DEBLUR_DEV float pen_deriv(float z, float eps2) { return 1.0f / sqrtf(z + eps2); }

}  // namespace deblur
