// PSF descriptor as seen by the kernels.
#pragma once

#include "common.hpp"

namespace deblur {

enum { PSF_BOX_H = 0, PSF_BOX_V = 1, PSF_TAPS = 2 };

struct PsfDev {
    int kind;          // PSF_*
    int length;        // box kinds: integer part n of the length L = n + frac
    int ph, pw;        // odd array dims (box: 1 x P or P x 1, P = n + (n even) + 2 (frac > 0))
    const float* taps; // PSF_TAPS: ph*pw row-major device array
    float frac;        // box kinds: fractional part of the length, [0, 1)
};

// Weight of array entry (j, i).  Box taps around the centre (P - 1)/2: 1/L on
// offsets d in [-floor((n-1)/2), floor(n/2)] and, for a non-integer length,
// (frac/2)/L on the two offsets just outside (Sec. 4.3, uniform linear motion).
DEBLUR_DEV float psf_weight(const PsfDev& p, int j, int i)
{
    if (p.kind == PSF_TAPS) return p.taps[j * p.pw + i];
    const int P = p.kind == PSF_BOX_H ? p.pw : p.ph;
    const int k = p.kind == PSF_BOX_H ? i : j;
    const int d = k - (P - 1) / 2;
    const int a = (p.length - 1) / 2, b = p.length / 2;
    const float L = (float)p.length + p.frac;
    if (d >= -a && d <= b) return 1.0f / L;
    if (p.frac > 0.0f && (d == -a - 1 || d == b + 1)) return 0.5f * p.frac / L;
    return 0.0f;
}

}  // namespace deblur
