// PSF descriptor as seen by the kernels.
#pragma once

#include "common.hpp"

namespace deblur {

enum { PSF_BOX_H = 0, PSF_BOX_V = 1, PSF_TAPS = 2 };

struct PsfDev {
    int kind;          // PSF_*
    int length;        // box length L (box kinds)
    int ph, pw;        // odd array dims (box: 1 x P or P x 1, P = L + (L even))
    const float* taps; // PSF_TAPS: ph*pw row-major device array
};

// Weight of array entry (j, i); box taps are 1/L on offsets
// d in [-floor((L-1)/2), floor(L/2)] around the centre (P - 1)/2.
DEBLUR_DEV float psf_weight(const PsfDev& p, int j, int i)
{
    if (p.kind == PSF_TAPS) return p.taps[j * p.pw + i];
    const int P = p.kind == PSF_BOX_H ? p.pw : p.ph;
    const int k = p.kind == PSF_BOX_H ? i : j;
    const int d = k - (P - 1) / 2;
    return (d >= -((p.length - 1) / 2) && d <= p.length / 2) ? 1.0f / (float)p.length : 0.0f;
}

}  // namespace deblur
