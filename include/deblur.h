/*
 * deblur.h - C ABI of the MI355X (gfx950) WR3L deblurring library.
 *
 * Method: Welk, Raudaschl, Schwarzbauer, Erler, Lauter, "Fast and Robust
 * Linear Motion Deblurring".  WR3L (Sec. 3.2) is a Wiener filter (Sec. 2.1,
 * eq. (2)) whose non-positive outputs are replaced by a small positive value,
 * followed by a few iterations of robust and regularised Richardson-Lucy
 * deconvolution, RRRL (Sec. 2.3, eqs. (6)-(12)), for a known space-invariant
 * point-spread function (PSF, blur model eq. (1)).
 *
 * Conventions for every entry point:
 *  - Images are row-major float32 arrays of H rows and W columns with a row
 *    pitch of `pitch` elements (pitch >= W).  Image, PSF-tap, checkpoint,
 *    gradient and workspace pointers are DEVICE pointers; descriptor structs
 *    (deblur_psf, deblur_params) are HOST pointers read during the call.
 *  - The caller owns all memory.  The library allocates nothing on these
 *    calls; scratch space is the caller's workspace of at least
 *    deblur_workspace_bytes(...) bytes, 256-byte aligned.  One exception:
 *    the first call with deblur_params.rf_lut = 1 on a device uploads a
 *    16 KB table that the library keeps until the process ends.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *    null stream) and the call returns without synchronising.  Inputs must
 *    stay valid until the stream reaches the work.  Calls on distinct streams
 *    with distinct workspaces may run concurrently.
 *  - Every argument is validated on the host before anything is enqueued; on
 *    an error nothing is written.  Return value: DEBLUR_OK or a negative
 *    deblur_status (deblur_status_string gives the text).  Launch failures
 *    are reported as DEBLUR_EDEVICE.
 *  - Preconditions that are not checked: PSF taps non-negative with sum 1
 *    (normalised PSF, eq. (1)); observed image values >= 0 (values <= 0 are
 *    treated as 0 in the data term, where r_f(s) = s); buffers not
 *    overlapping except where an entry point says so.
 */
#ifndef DEBLUR_H
#define DEBLUR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DEBLUR_OK = 0,
    DEBLUR_EINVAL = -1,       /* invalid argument (null pointer, bad size, bad enum, ...) */
    DEBLUR_EUNSUPPORTED = -2, /* valid but not implemented (FFT length, PSF radius, ...) */
    DEBLUR_EWORKSPACE = -3,   /* workspace missing or smaller than required */
    DEBLUR_EDEVICE = -4,      /* HIP launch or runtime failure */
    DEBLUR_ESCRATCH = -5      /* the problem needs more than the static scratch of
                                 deblur_rrrl_iterate_noalloc (DEBLUR_NOALLOC_SCRATCH_BYTES) */
} deblur_status;

/* Boundary continuation of the blur A and adjoint blur B (Sec. 4.2): the
 * paper uses constant continuation for spatial-domain convolutions and
 * periodic continuation for Fourier-domain ones.  The Wiener step is always
 * periodic; the diffusion term always has zero flux across the border. */
typedef enum { DEBLUR_BC_REPLICATE = 0, DEBLUR_BC_PERIODIC = 1 } deblur_boundary;

/* PSF kinds (Sec. 4.3).  Offsets d = (dy, dx) are relative to the centre of
 * an odd-sized array.  BOX_H / BOX_V: uniform linear motion of length
 * L = n + frac along x / y (n = length >= 1, 0 <= frac < 1).  Integer L: taps
 * 1/L at d in [-floor((n-1)/2), floor(n/2)], array length n + (n even).  A
 * non-integer length adds one pixel of smaller weight at each end (Sec. 4.3,
 * uniform linear motion): taps (frac/2)/L at d = -floor((n-1)/2) - 1 and
 * d = floor(n/2) + 1, the n inner taps 1/L; array length n + (n even) + 2.
 * TAPS: a general ph x pw array (ph, pw odd). */
typedef enum { DEBLUR_PSF_BOX_H = 0, DEBLUR_PSF_BOX_V = 1, DEBLUR_PSF_TAPS = 2 } deblur_psf_kind;

/* How the RRRL iteration evaluates A and B: AUTO picks the fastest exact
 * spatial method for the PSF kind (running sums for boxes, LDS stencil for
 * taps); FFT evaluates both convolutions in the Fourier domain (Sec. 4.3),
 * which implies periodic continuation (boundary must be PERIODIC; H, W must
 * be 2^a 3^b <= 2048) and costs the same for any PSF size.  The stage-level
 * entry points and the backward pass use the stencil. */
typedef enum {
    DEBLUR_CONV_AUTO = 0,
    DEBLUR_CONV_RUNSUM = 1,
    DEBLUR_CONV_STENCIL = 2,
    DEBLUR_CONV_FFT = 3
} deblur_conv;

typedef struct {
    int32_t kind;       /* deblur_psf_kind */
    int32_t length;     /* box length L (BOX_H, BOX_V); ignored for TAPS */
    int32_t ph, pw;     /* TAPS: odd array dims, 1..65 each; ignored for boxes */
    const float* taps;  /* TAPS: device array ph*pw, row-major; may be NULL for boxes */
    float frac;         /* boxes: fractional part of the length, 0 <= frac < 1 (else
                           DEBLUR_EINVAL); ignored for TAPS */
} deblur_psf;

typedef struct {
    float alpha;     /* regulariser weight alpha >= 0 (eq. (9)) */
    float eps_data;  /* epsilon > 0 of the data penaliser Phi(z) = sqrt(z + eps^2) (Sec. 2.3) */
    float eps_tv;    /* > 0: epsilon of the TV penaliser Psi (Sec. 2.3), or the contrast
                        parameter lambda of the Perona-Malik penaliser (psi = 1) */
    float s_min;     /* > 0: the blurred iterate is bounded below by s_min before dividing */
    int32_t iters;   /* number of RRRL iterations, >= 0 */
    int32_t robust;  /* 1: W = Phi'(r_f(u*h)) (eq. (10)); 0: W = 1 (plain RL data term) */
    int32_t boundary;/* deblur_boundary */
    int32_t conv;    /* deblur_conv */
    int32_t tile;    /* tile shape: 0 = library default for the image size, else an explicit
                        shape (an autotuner's choice), 1..deblur_tile_variants() for the stencil
                        kernels, 1..deblur_box_tile_variants() for the running-sum kernel (boxes
                        with conv AUTO or RUNSUM); all shapes give bitwise-identical results */
    int32_t psi;     /* regulariser Psi (Sec. 2.3): 0 = regularised TV, Psi(z) = sqrt(z + eps^2);
                        1 = Perona-Malik, Psi(z) = (lambda^2/2) ln(1 + z/lambda^2), non-convex in
                        |grad u| (diffusivity lambda^2 / (lambda^2 + z)); else DEBLUR_EINVAL */
    int32_t rf_lut;  /* 0: exact r_f (eq. (7)); 1: the lookup mode of Sec. 4.1, r_f(s) = f r_1(s/f)
                        with r_1(x) = x - 1 - ln x tabulated at x = k/64 up to 65, linear
                        interpolation, the tangent at 65 beyond.  The first call with rf_lut = 1 on a
                        device allocates and uploads the 16 KB table (keep that call out of graph
                        capture); the backward pass rejects it (DEBLUR_EUNSUPPORTED). */
    int32_t bwd_tile;/* tile rows of the backward's iteration kernels: 0 = default (8 rows, 16
                        when a launch over the batch holds at least 8192 tiles of 16 rows),
                        1 = 8, 2 = 4, 3 = 16, 4 = 32 rows of 64 columns (an autotuner's choice; all
                        give bitwise-identical gradients); ignored by the forward entry points; else
                        DEBLUR_EINVAL */
} deblur_params;

/* Text for a status code (static storage). */
const char* deblur_status_string(int status);

/* Library ABI version (major*10000 + minor*100 + patch). */
int deblur_version(void);

/* Number of explicit tile shapes selectable through deblur_params.tile:
 * of the stencil kernels (TAPS PSFs, or boxes with conv = STENCIL) and of the
 * running-sum kernel (boxes otherwise). */
int deblur_tile_variants(void);
int deblur_box_tile_variants(void);
/* Number of explicit tile-row shapes of the backward (deblur_params.bwd_tile,
 * 1..n; 0 = default). */
int deblur_backward_tile_variants(void);

/* Workspace bytes needed by an entry point: op 0 = deblur_wiener,
 * 1 = deblur_rrrl_iterate, 2 = deblur_rrrl_backward without the Wiener step,
 * 3 = deblur_rrrl_backward through the Wiener step, 4 = deblur_wiener_fp64.  Returns 0 for invalid
 * arguments (the matching call then returns DEBLUR_EINVAL or
 * DEBLUR_EUNSUPPORTED). */
size_t deblur_workspace_bytes(int32_t op, int32_t H, int32_t W, int32_t pitch, const deblur_psf* psf,
                              const deblur_params* p);

/* Workspace bytes of the batched entry points (deblur_wiener_batch,
 * deblur_rrrl_iterate_batch, deblur_rrrl_backward_batch) for B images: op as
 * deblur_workspace_bytes; B per-image workspaces, each rounded up to 256
 * bytes.  0 for invalid arguments, B outside 1..65535, or op 1 with the
 * Fourier-domain iteration (which has no batched form). */
size_t deblur_workspace_bytes_batch(int32_t op, int32_t B, int32_t H, int32_t W, int32_t pitch,
                                    const deblur_psf* psf, const deblur_params* p);

/* Wiener initialisation of WR3L (Sec. 2.1 eq. (2); Sec. 3.2):
 *   u0 = max( Re IDFT( DFT(f) conj(h^) / (|h^|^2 + K) ), pos_floor )
 * with h^ the DFT of the PSF centred at index (0,0), periodic continuation.
 * f, u0: device H x W, pitch `pitch` (must not overlap).  K > 0,
 * pos_floor > 0.  H and W must factor as 2^a 3^b with H, W <= 2048 (only W
 * for a PSF on one row, where the filter runs along rows).  The spectral
 * division is done in FP64, the transforms in FP32. */
int deblur_wiener(const float* f, float* u0, int32_t H, int32_t W, int32_t pitch, const deblur_psf* psf,
                  double K, float pos_floor, void* ws, size_t ws_bytes, void* stream);

/* The Wiener initialisation of deblur_wiener (same formula, arguments,
 * layouts and errors) with the multiplier M, the spectra and the transforms
 * in FP64; only the output is rounded, once, to FP32.  The FP32 transforms of
 * deblur_wiener leave u0 a few units of FP32 roundoff away from the exact
 * result; this variant rounds it correctly, which matters where the output
 * feeds a gradient of an ill-conditioned iteration (the periodic Wiener step
 * rings at image borders, Sec. 4.2).  Workspace: deblur_workspace_bytes(4,
 * ...), twice that of deblur_wiener. */
int deblur_wiener_fp64(const float* f, float* u0, int32_t H, int32_t W, int32_t pitch, const deblur_psf* psf,
                       double K, float pos_floor, void* ws, size_t ws_bytes, void* stream);

/* deblur_wiener (fp64 = 0) or deblur_wiener_fp64 (fp64 = 1) for B images of
 * one size at once, one launch per kernel over all of them: image b's f and
 * u0 at f + b img_stride and u0 + b img_stride (floats, >= H pitch), its PSF
 * at psf->taps + b taps_stride for DEBLUR_PSF_TAPS (>= ph pw; 0: one PSF for
 * the batch; box kinds: shared, taps_stride 0).  K and pos_floor are shared.
 * Each image's u0 equals the one-image call's bit for bit.  ws: at least
 * deblur_workspace_bytes_batch(0 or 4, B, ...) bytes.  1 <= B <= 65535;
 * other errors as deblur_wiener. */
int deblur_wiener_batch(int32_t B, const float* f, float* u0, int32_t H, int32_t W, int32_t pitch, int64_t img_stride,
                        const deblur_psf* psf, int64_t taps_stride, double K, float pos_floor, int32_t fp64,
                        void* ws, size_t ws_bytes, void* stream);

/* Starting image for RRRL without the Wiener step (Sec. 2.3; the RRRL columns
 * of Table 1 start from an image the paper does not state):
 *   DEBLUR_START_FLAT:     u0 = max(mean(f), pos_floor) at every pixel (the mean
 *                          summed in FP64 in a fixed order: deterministic);
 *   DEBLUR_START_OBSERVED: u0 = max(f, pos_floor).
 * f, u0: device H x W, pitch `pitch`, must not overlap; pos_floor > 0 (the
 * multiplicative update needs a positive start, Sec. 3.2).  No workspace. */
typedef enum { DEBLUR_START_FLAT = 0, DEBLUR_START_OBSERVED = 1 } deblur_start;
int deblur_rrrl_start(const float* f, float* u0, int32_t H, int32_t W, int32_t pitch, int32_t mode,
                      float pos_floor, void* stream);

/* p->iters RRRL iterations (Sec. 2.3 eq. (9)-(12)) from u_in:
 *   s = max(A u, s_min),  W = Phi'(r_f(s)) (or 1),  q = W max(f,0) / s,
 *   u <- u (B q + alpha [D(u)]_+) / (B W - alpha [D(u)]_-),
 * A = blur with h, B = blur with h*(x) = h(-x), D = div(Psi'(|grad u|^2) grad u)
 * by central differences (Sec. 4.1).  f, u_in, u_out: device H x W, pitch
 * `pitch`; u_in == u_out is allowed, other overlaps are not.  ckpt
 * (nullable): device array of p->iters * H * pitch floats receiving the
 * iterates u^0 .. u^{iters-1} (for the backward pass).  PSF radius <= 32 in
 * each direction and <= min(H, W). */
int deblur_rrrl_iterate(const float* f, const float* u_in, float* u_out, int32_t H, int32_t W, int32_t pitch,
                        const deblur_psf* psf, const deblur_params* p, float* ckpt, void* ws, size_t ws_bytes,
                        void* stream);

/* deblur_rrrl_iterate for B images of one size at once, one launch per
 * kernel and iteration over all of them (the stencil and running-sum paths;
 * p->conv = DEBLUR_CONV_FFT returns DEBLUR_EUNSUPPORTED).  Image b's f, u_in
 * and u_out at + b img_stride (floats, >= H pitch), its checkpoints (if ckpt)
 * at ckpt + b ckpt_stride (>= p->iters H pitch), its PSF at psf->taps +
 * b taps_stride for DEBLUR_PSF_TAPS (>= ph pw; 0: shared; box kinds: shared,
 * taps_stride 0), its alpha at alpha[b] (device array of B floats, not
 * validated; NULL: p->alpha for every image); the other parameters are
 * shared.  Each image's results equal the one-image call's bit for bit.  ws:
 * at least deblur_workspace_bytes_batch(1, B, ...) bytes.  1 <= B <= 65535;
 * other errors as deblur_rrrl_iterate. */
int deblur_rrrl_iterate_batch(int32_t B, const float* f, const float* u_in, float* u_out, int32_t H, int32_t W,
                              int32_t pitch, int64_t img_stride, const deblur_psf* psf, int64_t taps_stride,
                              const float* alpha, const deblur_params* p, float* ckpt, int64_t ckpt_stride, void* ws,
                              size_t ws_bytes, void* stream);

/* Variant of deblur_rrrl_iterate for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, hosts that forbid
 * hipMalloc): the same arguments without the workspace, the same kernels and
 * results bit for bit.  Its scratch is a static device array of
 * DEBLUR_NOALLOC_SCRATCH_BYTES (64 MiB) that each GPU the library runs on
 * holds from library load until the process ends; the call allocates nothing
 * (no hipMalloc, no library allocation).
 *  - A problem whose workspace, deblur_workspace_bytes(1, ...), exceeds the
 *    scratch returns DEBLUR_ESCRATCH before anything is enqueued (e.g. the
 *    stencil path holds 16 bytes per pixel: up to about 4 Mpx).
 *  - rf_lut = 1 returns DEBLUR_EUNSUPPORTED (that mode allocates its table on
 *    first use).
 *  - Every call on a GPU shares that GPU's one scratch array, which keeps the
 *    last call's contents: calls that overlap in time on one GPU (different
 *    streams, or host threads) race and give undefined results.  Serialise
 *    them, e.g. by issuing them on one stream.
 * Other arguments, layouts, ownership and errors: as deblur_rrrl_iterate. */
#define DEBLUR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int deblur_rrrl_iterate_noalloc(const float* f, const float* u_in, float* u_out, int32_t H, int32_t W,
                                int32_t pitch, const deblur_psf* psf, const deblur_params* p, float* ckpt,
                                void* stream);

/* Reverse-mode derivative of a loss L(u^K) through p->iters unrolled RRRL
 * iterations (eqs. (9)-(12)) and, if through_wiener, through the Wiener
 * initialisation with its positivity floor (eq. (2), Sec. 3.2), for the
 * observed image f, the PSF entries and alpha.
 *   ckpt:     device, p->iters * H * pitch floats: u^0 .. u^{K-1} as written by
 *             deblur_rrrl_iterate (may be NULL when p->iters == 0);
 *   grad_uK:  device H x pitch, dL/du^K;
 *   grad_f:   device H x pitch, receives dL/df (overwritten);
 *   grad_taps (nullable): device array of the PSF's ph*pw entries (boxes: the
 *             1 x P or P x 1 array of the box), receives dL/dh for every entry,
 *             zero or not (overwritten);
 *   grad_alpha (nullable): device scalar, receives dL/dalpha;
 *   grad_u0 (nullable): device H x pitch, receives dL/du^0 (the derivative at
 *             the Wiener output, before the Wiener adjoint).
 * K, pos_floor: the Wiener parameters of the forward call (used when
 * through_wiener; then H and W must be 2^a 3^b <= 2048).  Derivatives of
 * max/min take the branch taken (0 at ties); d r_f/df is taken as 0 where
 * f <= 0.  For PSF arrays of at most 32 x 32 entries whose longer side has
 * more than 16, dL/dh runs on the matrix cores with each factor split into
 * two bfloat16 parts: a product's relative error is about 3 * 2^-16, and
 * the sums are FP32.
 * Partial sums are reduced in a fixed order: results are deterministic.
 * Output buffers must not overlap the inputs. */
int deblur_rrrl_backward(const float* f, const float* ckpt, const float* grad_uK, int32_t H, int32_t W,
                         int32_t pitch, const deblur_psf* psf, const deblur_params* p, int32_t through_wiener,
                         double K, float pos_floor, float* grad_f, float* grad_taps, float* grad_alpha,
                         float* grad_u0, void* ws, size_t ws_bytes, void* stream);

/* deblur_rrrl_backward for B images at once (the same derivatives, eqs.
 * (9)-(12), eq. (2)): one launch per kernel covers every image, so a batch of
 * small images fills the GPU.  All images share H, W, pitch, the PSF array
 * dimensions, *p except alpha, through_wiener, K and pos_floor; each has its
 * own f, checkpoints, dL/du^K, PSF taps and alpha.  Image b (0 <= b < B):
 *   f + b img_stride, grad_uK + b img_stride, grad_f + b img_stride,
 *   grad_u0 + b img_stride (each H x pitch floats);
 *   ckpt + b ckpt_stride (p->iters * H * pitch floats);
 *   PSF: psf->taps + b taps_stride for DEBLUR_PSF_TAPS (taps_stride 0: one
 *   PSF shared by the batch); box kinds are shared and need taps_stride 0;
 *   grad_taps + b ph pw (nullable; B ph pw floats), grad_alpha + b
 *   (nullable; B floats);
 *   alpha: device array of B floats, image b's regulariser weight; NULL uses
 *   p->alpha for every image.  Its values are read by the kernels and are not
 *   validated (they must be finite and >= 0).
 * Strides are in floats: img_stride >= H pitch, ckpt_stride >= p->iters H
 * pitch, taps_stride >= ph pw (or 0).  1 <= B <= 65535.  Each image's results
 * equal deblur_rrrl_backward's for that image bit for bit.  ws: at least
 * deblur_workspace_bytes_batch(2 or 3, B, ...) bytes.  Output ranges (over
 * the whole batch) must not overlap the inputs'.  Errors as
 * deblur_rrrl_backward; DEBLUR_EINVAL for B or a stride out of range. */
int deblur_rrrl_backward_batch(int32_t B, const float* f, const float* ckpt, const float* grad_uK, int32_t H,
                               int32_t W, int32_t pitch, int64_t img_stride, int64_t ckpt_stride,
                               const deblur_psf* psf, int64_t taps_stride, const float* alpha,
                               const deblur_params* p, int32_t through_wiener, double K, float pos_floor,
                               float* grad_f, float* grad_taps, float* grad_alpha, float* grad_u0, void* ws,
                               size_t ws_bytes, void* stream);

/* ---- Batched form: many images of different sizes, each with its own PSF
 * and parameters, in one hipGraph launch.
 * An item binds the device pointers f (input) and u (output, H x pitch), the
 * PSF, the parameters (all items must have the same p.iters) and the Wiener
 * K and pos_floor; the computation per item is deblur_wiener followed by
 * deblur_rrrl_iterate.  deblur_batch_plan_create validates every item (the
 * status of the first invalid one is returned), then allocates the plan's
 * device memory (per-image scratch planes and Wiener workspaces, compiled
 * tap lists, tile lists, the Wiener job lists),
 * compiles the PSFs (their taps are read here: a changed PSF needs a new
 * plan) and captures the graph; it synchronises the device.  group_size > 0
 * runs the images in consecutive groups of that many (a group starts when
 * the previous one has ended), 0 = one group. */
typedef struct deblur_batch_plan deblur_batch_plan;
typedef struct {
    const float* f;
    float* u;
    int32_t H, W, pitch;
    deblur_psf psf;
    deblur_params p;
    double K;
    float pos_floor;
} deblur_batch_item;

int deblur_batch_plan_create(const deblur_batch_item* items, int32_t n, int32_t group_size,
                             deblur_batch_plan** plan);

/* Tile shapes of a plan.  Family DEBLUR_BATCH_STENCIL: the 64-column tiles
 * of the stencil classes (1: 32 rows / 512 threads, 2: 16 / 256, 3: 32 /
 * 256); DEBLUR_BATCH_BOX: the box tile variants of deblur_box_tile_variants,
 * per orientation.  Every shape gives bitwise-identical results. */
#define DEBLUR_BATCH_STENCIL 0
#define DEBLUR_BATCH_BOX 1
#define DEBLUR_BATCH_NTILES 5
/* Number of shapes of a family (0 for an unknown family). */
int32_t deblur_batch_tile_variants(int32_t family);
/* deblur_batch_plan_create with chosen tile shapes: tiles (host,
 * DEBLUR_BATCH_NTILES entries, or NULL for the defaults) = {stencil variant,
 * box variant of horizontal images up to 512 x 512 pixels, of vertical ones
 * up to 512 x 512, of larger horizontal ones, of larger vertical ones}, each
 * 0 (default: 1, 5, 5, 1, 1) .. the family's count, else DEBLUR_EINVAL.
 * Items with p.conv == DEBLUR_CONV_FFT are rejected with
 * DEBLUR_EUNSUPPORTED by both create calls: a plan runs the direct paths
 * (stencil, running sums) only. */
int deblur_batch_plan_create_tiled(const deblur_batch_item* items, int32_t n, int32_t group_size,
                                   const int32_t* tiles, deblur_batch_plan** plan);

/* Tile classes of a plan: 0..3 stencil radius classes 4, 8, 16, 32; 4
 * horizontal and 5 vertical box images up to 512 x 512 pixels; 6 horizontal
 * and 7 vertical box images above. */
#define DEBLUR_BATCH_NCLASS 8
/* Class of an item (>= 0), or DEBLUR_EINVAL. */
int32_t deblur_batch_class_of(const deblur_batch_plan* plan, int32_t image);
/* Tiles of one launch of a class in the plan's first group (0 if none), or
 * DEBLUR_EINVAL. */
int32_t deblur_batch_class_tiles(const deblur_batch_plan* plan, int32_t cls);
/* For per-kernel timing: enqueues on `stream`, outside the graph, one launch
 * of one kernel of a class over the first group's tiles (stage 1 or 2 of a
 * stencil class; stage 1 = the box kernel of a box class), reading the
 * items' outputs and writing the plan's own scratch planes.  The outputs are
 * left unchanged and the next deblur_batch_run recomputes everything.  It
 * must not overlap a run of the same plan.  DEBLUR_EINVAL: no such class
 * tiles or stage. */
int deblur_batch_launch_class(deblur_batch_plan* plan, int32_t cls, int32_t stage, void* stream);
/* Enqueues the whole batch (one graph launch) on `stream`. */
int deblur_batch_run(deblur_batch_plan* plan, void* stream);
/* Number of items of the plan. */
int32_t deblur_batch_size(const deblur_batch_plan* plan);
/* After a run has completed: per-item latency in microseconds from the start
 * of the graph to the completion of the item's last tile in its last
 * iteration (device clock; items with 0 iterations: their group's end).  Host
 * array of deblur_batch_size(plan) doubles.  Synchronous. */
int deblur_batch_latencies(deblur_batch_plan* plan, double* us_out);
/* Frees the plan (NULL is allowed). */
void deblur_batch_plan_destroy(deblur_batch_plan* plan);

/* ---- Stage-level entry points of one RRRL iteration (spatial stencil path).
 * deblur_rrrl_iterate chains them; they are exported for callers that
 * schedule the iteration themselves, and for per-stage verification and
 * profiling.  Each is one kernel launch. */

/* Bytes of the compiled tap list of a PSF (0 for an invalid descriptor). */
size_t deblur_taps_bytes(const deblur_psf* psf);

/* Compiles the PSF (eq. (1)) in the device buffer `taps_out` of at least
 * deblur_taps_bytes(psf) bytes, 256-byte aligned.  The result is read by the
 * two stage entry points below and stays valid while the PSF is unchanged.
 * Layout (little-endian, P = ph*pw of the PSF array, cy = (ph-1)/2,
 * cx = (pw-1)/2):
 *   int32 [0]        number of non-zero taps T
 *   int32 [1]        number of column groups G
 *   int32 [1 + S]    number of column groups of length S, S = 1..8
 *   int32 [10]       number of packed words (G + T)
 *   bytes 256 ..     T records {int32 dy, int32 dx, float32 h, int32 0},
 *                    the non-zero taps in row-major order
 *   bytes 256+16P .. G records of 48 bytes {int32 dx, int32 dy0, int32 S,
 *                    int32 0, float32 w[8]}: taps (dy0 + s, dx) with weights
 *                    w[s], s < S, a run of vertically adjacent non-zero taps
 *                    of one PSF column (runs longer than 8 are split);
 *                    ordered by S descending, then dx, then dy0.
 *   bytes 256+64P .. the groups again, packed: per group one int32
 *                    (dx & 0xffff) | (dy0 << 16) followed by its S weights.
 * The stencil kernels sum the taps of a pixel in the group order. */
int deblur_compile_taps(const deblur_psf* psf, void* taps_out, size_t taps_bytes, void* stream);

/* Stage 1 of eq. (9): s = max(A u, s_min) (blur with h, eq. (1)), robust
 * weight W = Phi'(r_f(s)) (eq. (10), or 1 if p->robust == 0) and quotient
 * q = W max(f,0) / s.  f, u: device H x W, pitch `pitch`; qw: device output
 * of H*W interleaved pairs (q, W), row pitch 2*W floats.  p->iters is
 * ignored.  PSF radius <= 32. */
int deblur_rrrl_weights(const float* f, const float* u, float* qw, int32_t H, int32_t W, int32_t pitch,
                        const deblur_psf* psf, const void* taps, const deblur_params* p, void* stream);

/* Stage 2 of eq. (9): N1 = B q, N2 = B W (blur with h*), diffusion term
 * D(u) (eq. (11)) and the update u_out = u (N1 + alpha [D]_+) / (N2 - alpha [D]_-).
 * qw as written by deblur_rrrl_weights; u, u_out: device H x W, pitch
 * `pitch`, must not overlap; u_copy (nullable) receives a copy of u (the
 * checkpoint of this iteration).  p->iters is ignored. */
int deblur_rrrl_update(const float* qw, const float* u, float* u_out, float* u_copy, int32_t H, int32_t W,
                       int32_t pitch, const deblur_psf* psf, const void* taps, const deblur_params* p,
                       void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DEBLUR_H */
