// Device helpers shared by the WR3L kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define DEBLUR_DEV __device__ __forceinline__

namespace deblur {

enum { BC_REPLICATE = 0, BC_PERIODIC = 1 };

// Index of the continued image (Sec. 4.2): constant continuation clamps,
// periodic continuation wraps.
DEBLUR_DEV int ext_index(int i, int n, int bc)
{
    if (bc == BC_PERIODIC) {
        if (i >= 0 && i < n) return i;
        if (i < 0 && i >= -n) return i + n;   // halos shorter than the image: no division
        if (i >= n && i < 2 * n) return i - n;
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

// Launches over a batch of equally shaped images take the image index from
// blockIdx.z: image z's plane is the first image's advanced by z times a
// byte stride (stride 0: one plane shared by the batch).
// A pointer read from device memory (a descriptor of a batched launch) is
// generic to the compiler, which then emits flat accesses (slower, and
// counted with the LDS operations, so an LDS wait also waits for them).
// Every such pointer here addresses global memory: the cast lets the
// compiler emit global accesses.
template <typename T>
DEBLUR_DEV T* global_ptr(T* p)
{
    using G = __attribute__((address_space(1))) T;
    G* g = (G*)(uintptr_t)p;   // the same address, as a global-space pointer
    return (T*)g;
}

// (Byte-pointer arithmetic, not an integer round trip: the compiler keeps
// the pointer's global address space and emits global, not flat, accesses.)
template <typename T>
DEBLUR_DEV T* zadv(T* p, size_t stride)
{
    using B = typename std::conditional<std::is_const<T>::value, const unsigned char, unsigned char>::type;
    return reinterpret_cast<T*>(reinterpret_cast<B*>(p) + (size_t)blockIdx.z * stride);
}

// Cooperative copy of N elements into LDS: lds[idx] = fetch(idx), idx < N,
// by NT threads.  All global loads of a thread are issued before the first
// LDS store, so their latencies overlap (a plain strided loop would wait for
// each load before issuing the next).
template <int NT, int N, typename T, typename F>
DEBLUR_DEV void stage_to_lds(T* __restrict__ lds, F fetch)
{
    constexpr int NL = (N + NT - 1) / NT;
    T v[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        if (N % NT == 0 || idx < N) v[k] = fetch(idx);
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int idx = (int)threadIdx.x + k * NT;
        if (N % NT == 0 || idx < N) lds[idx] = v[k];
    }
}

// ROWS x COLS floats (COLS a multiple of 4) from src (row pitch sp floats,
// every row 16-byte aligned) into dense LDS rows, as 16-byte loads.
template <int NT, int ROWS, int COLS>
DEBLUR_DEV void copy_rows_f4(float* __restrict__ lds, const float* __restrict__ src, size_t sp)
{
    static_assert(COLS % 4 == 0, "16-byte rows");
    constexpr int C4 = COLS / 4;
    stage_to_lds<NT, ROWS * C4>(reinterpret_cast<float4*>(lds), [&](int i) {
        const int r = i / C4;
        return reinterpret_cast<const float4*>(src + (size_t)r * sp)[i - r * C4];
    });
}

// Same for a run-time count n, U loads in flight per thread.
template <int U, typename T, typename F>
DEBLUR_DEV void stage_to_lds_n(T* __restrict__ lds, int n, F fetch)
{
    const int nt = blockDim.x;
    for (int base = threadIdx.x; base < n; base += U * nt) {
        T v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int idx = base + k * nt;
            if (idx < n) v[k] = fetch(idx);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int idx = base + k * nt;
            if (idx < n) lds[idx] = v[k];
        }
    }
}

// Generalisation: for every idx < n, value = load(idx) then store(idx,
// value); the loads of U consecutive strides are issued before any store.
template <int U, typename L, typename S>
DEBLUR_DEV void batched_n(int n, L load, S store)
{
    using T = decltype(load(0));
    const int nt = blockDim.x;
    for (int base = threadIdx.x; base < n; base += U * nt) {
        T v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int idx = base + k * nt;
            if (idx < n) v[k] = load(idx);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int idx = base + k * nt;
            if (idx < n) store(idx, v[k]);
        }
    }
}

// Reciprocal and reciprocal square root by the hardware approximations
// (v_rcp_f32, v_rsq_f32: about 1 ulp).  Callers pass normal positive numbers.
DEBLUR_DEV float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Natural logarithm of a normal positive number through v_log_f32 (log2).
DEBLUR_DEV float ln_approx(float y) { return __builtin_amdgcn_logf(y) * 0.693147180559945309f; }

// Information divergence r_f(s) = s - f - f ln(s/f) (eq. (7)) in FP32,
// written as f * t(x), t(x) = x - ln(1+x), x = (s-f)/f, to avoid the
// cancellation of the literal form near s = f.  |x| < 1/4: Taylor series of
// t through x^13 (truncation below 1e-8 relative); elsewhere t = x - ln(s/f),
// where the cancellation costs at most a factor ~10.  Both branches are
// evaluated and one is selected (no divergence).  f <= 0: the limit
// r_0(s) = s.
DEBLUR_DEV float info_div(float f, float s)
{
    const bool pos = f > 0.0f;
    const float fr = pos ? f : 1.0f;
    const float rf = rcp(fr);
    const float x = (s - fr) * rf;
    // t = x^2 (1/2 - x/3 + x^2/4 - ... - x^11/13)
    float pz = -1.0f / 13.0f;
    pz = fmaf(pz, x, 1.0f / 12.0f);
    pz = fmaf(pz, x, -1.0f / 11.0f);
    pz = fmaf(pz, x, 1.0f / 10.0f);
    pz = fmaf(pz, x, -1.0f / 9.0f);
    pz = fmaf(pz, x, 1.0f / 8.0f);
    pz = fmaf(pz, x, -1.0f / 7.0f);
    pz = fmaf(pz, x, 1.0f / 6.0f);
    pz = fmaf(pz, x, -1.0f / 5.0f);
    pz = fmaf(pz, x, 1.0f / 4.0f);
    pz = fmaf(pz, x, -1.0f / 3.0f);
    pz = fmaf(pz, x, 0.5f);
    const float ts = x * x * pz;
    const float tl = x - ln_approx(s * rf);
    const float t = fabsf(x) < 0.25f ? ts : tl;
    return pos ? fr * t : s;
}

// Penaliser derivative of the regularised L1 / TV type (Sec. 2.3), up to the
// common factor 1/2 that cancels in the RRRL quotient: (z + eps^2)^(-1/2).
DEBLUR_DEV float pen_deriv(float z, float eps2) { return __builtin_amdgcn_rsqf(z + eps2); }

}  // namespace deblur
