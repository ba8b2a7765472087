// Batched WR3L: many images of different sizes, each with its own PSF and
// parameters, run by one hipGraph launch.
//
// A plan compiles every image's tap list, lays out per-image ping-pong and
// (q, W) planes, and builds flat tile lists per kernel class (stencil radius
// classes 4/8/16/32; horizontal and vertical box, each split at 512 x 512
// pixels) spanning all images of a group.  The captured graph runs, per
// group, one independent chain per class: the Wiener steps of the class's
// images (one batched launch per kernel for each image size), then for each
// iteration one launch per stage, whose workgroups each take one tile of one
// image from the list; a timestamp kernel follows the chains' join.  Groups
// run one after another.  In the
// launches of the last iteration every tile counts itself done for its image
// (an atomic counter) and the image's last tile writes the image's
// completion time: per-image latencies, no waiting inside any kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "box_seg.hpp"
#include "launch.hpp"
#include "psf.hpp"
#include "stencil_tiles.hpp"

namespace deblur {

struct BatchImg {
    const float* f;
    float* buf[2];          // ping-pong; buf[0] is the caller's output
    float2* qw;             // (q, W) plane of stencil images
    const float* taps;      // packed column groups of the compiled PSF
    const int* hdr;         // compiled PSF header (group counts per run length)
    int H, W, pitch, L;     // L: integer part of the box length (box classes)
    float frac;             // fractional part of the box length
    int ntiles;             // tiles of one launch of the image's class
    IterParams p;
};

// Completion of the image of tile t in a launch of the last iteration: the
// launch's last tile of the image stamps the time (all threads call).
DEBLUR_DEV void count_tile(const BatchImg& im, int img, unsigned* cnt, unsigned long long* ts)
{
    if (!cnt) return;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned old = atomicAdd(&cnt[img], 1u);
        if (old + 1 == (unsigned)im.ntiles) ts[img] = wall_clock64();
    }
}

struct BatchTile {
    int img, x0, y0, pad;   // x0/y0: along/across origin for box tiles
};

// Stencil tile shapes of the batch (rows TH of a 64-column tile, NT threads),
// variant 1..3 (0: variant 1).  Every shape sums a pixel's taps in the same
// order: the results do not depend on the choice.
constexpr int BATCH_STENCIL_VARIANTS = 3;

template <typename F>
inline void with_batch_stencil_shape(int v, F&& f)
{
    using std::integral_constant;
    switch (v) {
        case 2: f(integral_constant<int, 16>{}, integral_constant<int, 256>{}); break;
        case 3: f(integral_constant<int, 32>{}, integral_constant<int, 256>{}); break;
        default: f(integral_constant<int, 32>{}, integral_constant<int, 512>{}); break;
    }
}

template <int RAD, int TH, int NT>
__global__ void __launch_bounds__(NT) batch_stage1(const BatchTile* __restrict__ tiles,
                                                   const BatchImg* __restrict__ imgs, int src)
{
    __shared__ float tile[stage1_lds_floats<RAD, TH>()];
    __shared__ float pk[packed_words_max<RAD>()];
    const BatchTile t = tiles[blockIdx.x];
    const BatchImg& im = imgs[t.img];
    stage1_tile<RAD, TH, NT>(tile, pk, global_ptr(im.buf[src]), global_ptr(im.f), global_ptr(im.qw), nullptr, im.H,
                             im.W, im.pitch, t.x0, t.y0, global_ptr(im.taps), global_ptr(im.hdr), im.p);
}

template <int RAD, int TH, int NT>
__global__ void __launch_bounds__(NT) batch_stage2(const BatchTile* __restrict__ tiles,
                                                   const BatchImg* __restrict__ imgs, int src, unsigned* cnt,
                                                   unsigned long long* ts)
{
    __shared__ Stage2Smem<RAD, TH> sm;
    const BatchTile t = tiles[blockIdx.x];
    const BatchImg& im = imgs[t.img];
    stage2_tile<RAD, TH, NT>(sm, global_ptr(im.qw), global_ptr(im.buf[src]), global_ptr(im.buf[1 - src]), nullptr,
                             im.H, im.W, im.pitch, t.x0, t.y0, global_ptr(im.taps), global_ptr(im.hdr), im.p);
    count_tile(im, t.img, cnt, ts);
}

// Box tiles of the batch: one tile shape per class (a box variant of the
// single-image kernel).  LARGE (the class of images above 512 x 512 pixels)
// does not change the code; it gives the two size classes' launches their
// own kernel names even when they take the same tile shape, so that a
// profile attributes each launch to its class.
template <bool VERT, int TA, int TC, bool LARGE>
__global__ void __launch_bounds__(BOX_NT) batch_box(const BatchTile* __restrict__ tiles,
                                                    const BatchImg* __restrict__ imgs, int src, unsigned* cnt,
                                                    unsigned long long* ts)
{
    extern __shared__ __align__(16) float box_lds[];
    const BatchTile t = tiles[blockIdx.x];
    const BatchImg& im = imgs[t.img];
    const BoxGeom g = box_geom<VERT, TA, TC>(im.H, im.W, im.L, im.frac);
    box_seg_tile<VERT, TA, TC>(box_lds, global_ptr(im.buf[src]), global_ptr(im.f), global_ptr(im.buf[1 - src]),
                               nullptr, im.pitch, g, im.p, t.x0, t.y0);
    count_tile(im, t.img, cnt, ts);
}

// The batch's default box shapes per (orientation, size class): 64 x 4
// tiles (variant 5) for images up to 512 x 512, variant 1 above.
constexpr int BATCH_BOX_DEFAULT_SMALL = 5, BATCH_BOX_DEFAULT_LARGE = 1;

__global__ void batch_timestamp(unsigned long long* ts, int slot)
{
    if (threadIdx.x == 0) ts[slot] = wall_clock64();
}

// Clears the per-image tile counters (a fill kernel inside the graph).
__global__ void batch_clear(unsigned* cnt, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) cnt[i] = 0u;
}

// ---------------------------------------------------------------- host side
// Tile classes: stencil radius classes, then box classes by orientation and
// image size (up to 512 x 512 / above: different tile shapes suit them).
enum { CL_R4 = 0, CL_R8, CL_R16, CL_R32, CL_BOXH, CL_BOXV, CL_BOXH_L, CL_BOXV_L, NCLASS };
constexpr bool is_box(int cls) { return cls >= CL_BOXH; }
constexpr bool box_vert(int cls) { return cls == CL_BOXV || cls == CL_BOXV_L; }


struct ClassList {
    BatchTile* d = nullptr;   // device tile list
    int count = 0;
    size_t lds = 0;           // dynamic LDS bytes (box classes)
};

struct BatchPlan {
    int n = 0, groups = 0, iters = 0, start = 0;
    int st_var = 1;     // tile shapes: stencil; box per class (CL_BOXH + b)
    int box_var[4] = {BATCH_BOX_DEFAULT_SMALL, BATCH_BOX_DEFAULT_SMALL, BATCH_BOX_DEFAULT_LARGE,
                      BATCH_BOX_DEFAULT_LARGE};
    std::vector<int> class_of_img;      // image -> tile class
    std::vector<std::vector<ClassList>> lists;   // [group][class]
    BatchImg* dimgs = nullptr;
    std::vector<int> group_of;          // image -> group
    std::vector<void*> allocs;          // device allocations owned by the plan
    unsigned long long* ts = nullptr;   // groups + 1 timestamps
    unsigned* img_cnt = nullptr;        // per image: tiles of the last iteration done
    unsigned long long* img_ts = nullptr;   // per image: completion time
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> chains;
    std::vector<hipEvent_t> events;
    int clock_khz = 0;
};

static int class_of(const PsfDev& d, bool stencil, int H, int W)
{
    const bool large = (long)H * W > 512L * 512L;
    if (!stencil && d.kind == PSF_BOX_H) return large ? CL_BOXH_L : CL_BOXH;
    if (!stencil && d.kind == PSF_BOX_V) return large ? CL_BOXV_L : CL_BOXV;
    switch (tap_radius_class(max((d.ph - 1) / 2, (d.pw - 1) / 2))) {
        case 4: return CL_R4;
        case 8: return CL_R8;
        case 16: return CL_R16;
        default: return CL_R32;
    }
}

static void* dalloc(BatchPlan* P, size_t bytes)
{
    void* p = nullptr;
    if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) return nullptr;
    P->allocs.push_back(p);
    return p;
}

void batch_plan_destroy(BatchPlan* P)
{
    if (!P) return;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    for (hipEvent_t e : P->events) (void)hipEventDestroy(e);
    for (hipStream_t s : P->chains)
        if (s) (void)hipStreamDestroy(s);
    if (P->cap) (void)hipStreamDestroy(P->cap);
    for (void* p : P->allocs) (void)hipFree(p);
    delete P;
}

template <bool VERT, bool LARGE>
static void set_box_attr(int v)
{
    with_box_shape<VERT>(v, [](auto ta, auto tc) {
        (void)hipFuncSetAttribute(
            reinterpret_cast<const void*>(&batch_box<VERT, decltype(ta)::value, decltype(tc)::value, LARGE>),
            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    });
}

// One launch of one class over the tiles of list L: stage 1 and/or 2 of a
// stencil class (stages & 1, & 2), the box kernel of a box class.  The
// launches of an image's last iteration count tiles into cnt (else null).
static void launch_class(const BatchPlan* P, const ClassList& L, int cls, int stages, int src, unsigned* cnt,
                         hipStream_t cs)
{
    const BatchTile* d = L.d;
    const dim3 grid(L.count);
    unsigned long long* its = P->img_ts;
    const BatchImg* dimgs = P->dimgs;
    if (is_box(cls)) {
        auto box = [&](auto vert, auto large) {
            constexpr bool V = decltype(vert)::value, BIG = decltype(large)::value;
            with_box_shape<V>(P->box_var[cls - CL_BOXH], [&](auto ta, auto tc) {
                hipLaunchKernelGGL((batch_box<V, decltype(ta)::value, decltype(tc)::value, BIG>), grid, dim3(BOX_NT),
                                   L.lds, cs, d, dimgs, src, cnt, its);
            });
        };
        switch (cls) {
            case CL_BOXH: box(std::false_type{}, std::false_type{}); break;
            case CL_BOXV: box(std::true_type{}, std::false_type{}); break;
            case CL_BOXH_L: box(std::false_type{}, std::true_type{}); break;
            default: box(std::true_type{}, std::true_type{}); break;
        }
        return;
    }
    with_batch_stencil_shape(P->st_var, [&](auto th, auto nt) {
        constexpr int TH = decltype(th)::value, NT = decltype(nt)::value;
        auto both = [&](auto rad) {
            constexpr int R = decltype(rad)::value;
            if (stages & 1) hipLaunchKernelGGL((batch_stage1<R, TH, NT>), grid, dim3(NT), 0, cs, d, dimgs, src);
            if (stages & 2)
                hipLaunchKernelGGL((batch_stage2<R, TH, NT>), grid, dim3(NT), 0, cs, d, dimgs, src, cnt, its);
        };
        switch (cls) {
            case CL_R4: both(std::integral_constant<int, 4>{}); break;
            case CL_R8: both(std::integral_constant<int, 8>{}); break;
            case CL_R16: both(std::integral_constant<int, 16>{}); break;
            default: both(std::integral_constant<int, 32>{}); break;
        }
    });
}

// Builds the plan; items already validated, tiles (5 entries or null: stencil
// variant; box variants of horizontal and vertical images up to 512^2, then
// of larger ones; 0 = default) in range.
// Returns 0, -3 (allocation) or -4.
int batch_plan_create(const BatchItemDev* items, int n, int group_size, const int* tiles, BatchPlan** out)
{
    BatchPlan* P = new BatchPlan();
    P->n = n;
    P->iters = items[0].iters;
    if (tiles) {
        if (tiles[0] > 0) P->st_var = tiles[0];
        for (int b = 0; b < 4; ++b)
            if (tiles[1 + b] > 0) P->box_var[b] = tiles[1 + b];
    }
    int st_th = 32;
    with_batch_stencil_shape(P->st_var, [&](auto th, auto) { st_th = decltype(th)::value; });
    int box_ta[4], box_tc[4];   // per box class CL_BOXH + b
    for (int b = 0; b < 4; ++b) {
        auto get = [&](int& ta_out, int& tc_out) {
            if (box_vert(CL_BOXH + b))
                with_box_shape<true>(P->box_var[b], [&](auto ta, auto tc) { ta_out = ta; tc_out = tc; });
            else
                with_box_shape<false>(P->box_var[b], [&](auto ta, auto tc) { ta_out = ta; tc_out = tc; });
        };
        get(box_ta[b], box_tc[b]);
    }
    const int gs = group_size > 0 ? group_size : n;
    P->groups = (n + gs - 1) / gs;
    P->group_of.resize(n);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&P->clock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) {
        batch_plan_destroy(P);
        return -4;
    }
    const int start = P->iters % 2;  // Wiener writes buf[start]; the last iteration writes buf[0]
    P->start = start;
    P->class_of_img.resize(n);
    std::vector<BatchImg> imgs(n);
    for (int i = 0; i < n; ++i) {
        const BatchItemDev& it = items[i];
        BatchImg& b = imgs[i];
        b.f = it.f;
        b.buf[0] = it.u;
        b.buf[1] = static_cast<float*>(dalloc(P, (size_t)it.H * it.pitch * 4));
        const int cls = class_of(it.psf, it.stencil, it.H, it.W);
        P->class_of_img[i] = cls;
        b.qw = cls < CL_BOXH ? static_cast<float2*>(dalloc(P, (size_t)it.H * it.W * 8)) : nullptr;
        void* list = dalloc(P, tap_list_bytes(it.psf));
        if (!b.buf[1] || (cls < CL_BOXH && !b.qw) || !list) {
            batch_plan_destroy(P);
            return -3;
        }
        launch_compile_taps(it.psf, list, nullptr);
        b.hdr = reinterpret_cast<const int*>(list);
        b.taps = reinterpret_cast<const float*>(static_cast<unsigned char*>(list) +
                                                tap_packed_offset(it.psf.ph, it.psf.pw));
        b.H = it.H;
        b.W = it.W;
        b.pitch = it.pitch;
        b.L = it.psf.length;
        b.frac = it.psf.frac;
        if (cls < CL_BOXH) {
            b.ntiles = ((it.W + 63) / 64) * ((it.H + st_th - 1) / st_th);
        } else {
            const bool vert = box_vert(cls);
            const int TA = box_ta[cls - CL_BOXH], TC = box_tc[cls - CL_BOXH];
            const int along = vert ? it.H : it.W, across = vert ? it.W : it.H;
            b.ntiles = ((along + TA - 1) / TA) * ((across + TC - 1) / TC);
        }
        b.p = it.p;
        P->group_of[i] = i / gs;
    }
    BatchImg* dimgs = static_cast<BatchImg*>(dalloc(P, sizeof(BatchImg) * n));
    P->dimgs = dimgs;
    P->ts = static_cast<unsigned long long*>(dalloc(P, sizeof(unsigned long long) * (P->groups + 1)));
    P->img_cnt = static_cast<unsigned*>(dalloc(P, sizeof(unsigned) * n));
    P->img_ts = static_cast<unsigned long long*>(dalloc(P, sizeof(unsigned long long) * n));
    if (!dimgs || !P->ts || !P->img_cnt || !P->img_ts ||
        hipMemcpy(dimgs, imgs.data(), sizeof(BatchImg) * n, hipMemcpyHostToDevice) != hipSuccess) {
        batch_plan_destroy(P);
        return -3;
    }
    // tile lists per (group, class)
    P->lists.assign(P->groups, std::vector<ClassList>(NCLASS));
    auto& lists = P->lists;
    for (int g = 0; g < P->groups; ++g) {
        std::vector<std::vector<BatchTile>> host(NCLASS);
        for (int i = g * gs; i < std::min(n, (g + 1) * gs); ++i) {
            const BatchItemDev& it = items[i];
            const int cls = P->class_of_img[i];
            if (cls < CL_BOXH) {
                for (int y0 = 0; y0 < it.H; y0 += st_th)
                    for (int x0 = 0; x0 < it.W; x0 += 64) host[cls].push_back({i, x0, y0, 0});
            } else {
                const bool vert = box_vert(cls);
                const int TA = box_ta[cls - CL_BOXH], TC = box_tc[cls - CL_BOXH];
                const int along = vert ? it.H : it.W, across = vert ? it.W : it.H;
                for (int c0 = 0; c0 < across; c0 += TC)
                    for (int a0 = 0; a0 < along; a0 += TA) host[cls].push_back({i, a0, c0, 0});
                size_t lds = 0;
                auto words = [&](auto v) {
                    constexpr bool V = decltype(v)::value;
                    with_box_shape<V>(P->box_var[cls - CL_BOXH], [&](auto ta, auto tc) {
                        constexpr int A = decltype(ta)::value, C = decltype(tc)::value;
                        lds = 4 * (size_t)box_lds_words<V, A, C>(box_geom<V, A, C>(it.H, it.W, it.psf.length,
                                                                                    it.psf.frac));
                    });
                };
                if (vert) words(std::true_type{});
                else words(std::false_type{});
                lists[g][cls].lds = std::max(lists[g][cls].lds, lds);
            }
        }
        for (int c = 0; c < NCLASS; ++c) {
            if (host[c].empty()) continue;
            lists[g][c].count = (int)host[c].size();
            lists[g][c].d = static_cast<BatchTile*>(dalloc(P, sizeof(BatchTile) * host[c].size()));
            if (!lists[g][c].d || hipMemcpy(lists[g][c].d, host[c].data(), sizeof(BatchTile) * host[c].size(),
                                            hipMemcpyHostToDevice) != hipSuccess) {
                batch_plan_destroy(P);
                return -3;
            }
        }
    }
    set_box_attr<false, false>(P->box_var[CL_BOXH - CL_BOXH]);
    set_box_attr<true, false>(P->box_var[CL_BOXV - CL_BOXH]);
    set_box_attr<false, true>(P->box_var[CL_BOXH_L - CL_BOXH]);
    set_box_attr<true, true>(P->box_var[CL_BOXV_L - CL_BOXH]);
    // Wiener steps: per group and tile class, the images of one size and one
    // path (one-row PSF or general) form one job list, run by one batched
    // launch per kernel at the head of the class's chain; every image has its
    // own workspace.
    struct JobSet {
        WienerJob* d = nullptr;
        int count = 0, H = 0, W = 0, cls = 0;
        bool rowwise = false;
    };
    std::vector<std::vector<JobSet>> jobsets(P->groups);
    for (int g = 0; g < P->groups; ++g) {
        std::vector<std::pair<long, std::vector<WienerJob>>> sets;   // key: (class, H, W, rowwise)
        for (int i = g * gs; i < std::min(n, (g + 1) * gs); ++i) {
            const BatchItemDev& it = items[i];
            const bool rowwise = it.psf.ph == 1;
            const long key = ((long)P->class_of_img[i] << 56) | ((long)it.H << 28) | ((long)it.W << 1) |
                             (rowwise ? 1 : 0);
            void* w = dalloc(P, wiener_ws_bytes(it.H, it.W, rowwise));
            if (!w) {
                batch_plan_destroy(P);
                return -3;
            }
            WienerJob j;
            j.f = it.f;
            j.u = imgs[i].buf[start];
            j.pitch = it.pitch;
            j.pos_floor = it.pos_floor;
            j.K = it.K;
            j.psf = it.psf;
            j.ws = w;
            auto e = std::find_if(sets.begin(), sets.end(), [&](const auto& x) { return x.first == key; });
            if (e == sets.end()) sets.push_back({key, {j}});
            else e->second.push_back(j);
        }
        for (auto& kv : sets) {
            JobSet js;
            js.count = (int)kv.second.size();
            js.cls = (int)(kv.first >> 56);
            js.H = (int)((kv.first >> 28) & 0xfffffffL);
            js.W = (int)((kv.first >> 1) & 0x7ffffffL);
            js.rowwise = kv.first & 1;
            js.d = static_cast<WienerJob*>(dalloc(P, sizeof(WienerJob) * kv.second.size()));
            if (!js.d || hipMemcpy(js.d, kv.second.data(), sizeof(WienerJob) * kv.second.size(),
                                   hipMemcpyHostToDevice) != hipSuccess) {
                batch_plan_destroy(P);
                return -3;
            }
            jobsets[g].push_back(js);
        }
    }
    prepare_wiener_kernels();   // runtime attribute calls stay out of the capture
    if (hipDeviceSynchronize() != hipSuccess) {  // tap lists and copies complete
        batch_plan_destroy(P);
        return -4;
    }
    // ---- capture
    bool ok = hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking) == hipSuccess;
    // one chain per tile class
    P->chains.resize(NCLASS, nullptr);
    for (int c = 0; c < NCLASS && ok; ++c)
        ok = hipStreamCreateWithFlags(&P->chains[c], hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        batch_plan_destroy(P);
        return -4;
    }
    auto event = [&]() {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return (hipEvent_t) nullptr;
        P->events.push_back(e);
        return e;
    };
    hipStream_t s = P->cap;
    ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(batch_clear, dim3((n + 255) / 256), dim3(256), 0, s, P->img_cnt, n);
        hipLaunchKernelGGL(batch_timestamp, dim3(1), dim3(64), 0, s, P->ts, 0);
    }
    for (int g = 0; g < P->groups && ok; ++g) {
        // every tile class (stencil radius, box axis and size) covers its own
        // images, which depend only on themselves, so each class is an
        // independent chain, forked once per group and joined at its end:
        // the batched Wiener steps of its images, then all iterations
        const auto& L = lists[g];
        hipEvent_t fork = event();
        ok = fork && hipEventRecord(fork, s) == hipSuccess;
        for (int cls = 0; cls < NCLASS && ok; ++cls) {
            if (!L[cls].count) continue;
            hipStream_t cs = P->chains[cls];
            ok = hipStreamWaitEvent(cs, fork, 0) == hipSuccess;
            for (size_t k = 0; ok && k < jobsets[g].size(); ++k) {
                const JobSet& js = jobsets[g][k];
                if (js.cls == cls) ok = launch_wiener_batch(js.d, js.count, js.H, js.W, js.rowwise, cs) == 0;
            }
            for (int k = 0; k < P->iters && ok; ++k)
                launch_class(P, L[cls], cls, 3, (start + k) % 2, k == P->iters - 1 ? P->img_cnt : nullptr, cs);
            hipEvent_t join = ok ? event() : nullptr;
            ok = ok && join && hipEventRecord(join, cs) == hipSuccess && hipStreamWaitEvent(s, join, 0) == hipSuccess;
        }
        if (ok) hipLaunchKernelGGL(batch_timestamp, dim3(1), dim3(64), 0, s, P->ts, g + 1);
    }
    hipGraph_t graph = nullptr;
    const hipError_t end = hipStreamEndCapture(s, &graph);
    ok = ok && end == hipSuccess && graph;
    P->graph = graph;
    if (!ok || hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0) != hipSuccess) {
        batch_plan_destroy(P);
        return -4;
    }
    *out = P;
    return 0;
}

int batch_run(BatchPlan* P, hipStream_t st) { return hipGraphLaunch(P->exec, st) == hipSuccess ? 0 : -4; }

// Per-image latency: from the start of the graph to the completion of the
// image's last tile (written by that tile; 0 iterations: its group's end).
int batch_latencies(BatchPlan* P, double* us)
{
    std::vector<unsigned long long> t(P->groups + 1), ti(P->n);
    if (hipMemcpy(t.data(), P->ts, sizeof(unsigned long long) * t.size(), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(ti.data(), P->img_ts, sizeof(unsigned long long) * ti.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return -4;
    const double per_us = (double)P->clock_khz / 1000.0;  // ticks per microsecond
    for (int i = 0; i < P->n; ++i) {
        const unsigned long long end = P->iters > 0 ? ti[i] : t[P->group_of[i] + 1];
        us[i] = (double)(end - t[0]) / per_us;
    }
    return 0;
}

int batch_size(const BatchPlan* P) { return P->n; }

int batch_class_of(const BatchPlan* P, int img) { return P->class_of_img[img]; }

int batch_class_tiles(const BatchPlan* P, int cls) { return P->lists[0][cls].count; }

// One launch of one class's kernel over the first group's tiles, outside the
// graph, on st: reads buffer 0 (the outputs), writes buffer 1 and the (q, W)
// planes.  -2: no tiles of that class in the first group, or a stage the
// class does not have.
int batch_launch_class(const BatchPlan* P, int cls, int stage, hipStream_t st)
{
    const ClassList& L = P->lists[0][cls];
    if (!L.count) return -2;
    const bool box = is_box(cls);
    if ((box && stage != 1) || (!box && stage != 1 && stage != 2)) return -2;
    launch_class(P, L, cls, box ? 1 : stage, 0, nullptr, st);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int batch_num_variants(int family) { return family == 0 ? BATCH_STENCIL_VARIANTS : BOX_VARIANTS; }

}  // namespace deblur
