/*
 * FP64 CPU oracle of the robust and regularised Richardson-Lucy (RRRL)
 * iteration of Welk et al., "Fast and Robust Linear Motion Deblurring".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition the GPU kernels are checked against.  Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may build, load or call
 * it; the product path never does.  It shares no code with the GPU path.
 *
 * Everything is FP64, straightforward loops, no blocking or reordering;
 * compiled without fast-math and with -ffp-contract=off.  OpenMP only splits
 * the outer row loop (each output is still one sequential sum).
 *
 * Notation (Sec. 2): image u on the grid {0..H-1}x{0..W-1}, row-major.
 * PSF array h[Py][Px] with odd sizes, centre (cy,cx) = ((Py-1)/2,(Px-1)/2),
 * tap offset d = (j-cy, i-cx).  E(v) is the continued image: constant
 * continuation (replicate) for spatial convolutions, or periodic
 * continuation (Sec. 4.2).
 *
 *   A v (x) = sum_d h(d) E(v)(x - d)     blur with h, eq. (1)
 *   B v (x) = sum_d h(d) E(v)(x + d)     convolution with h*(x) = h(-x)
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int ext(int i, int n, int bc)
{
    if (bc == ORC_BC_PERIODIC) {
        int m = i % n;
        return m < 0 ? m + n : m;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* A v: convolution with the PSF under boundary continuation `bc` (eq. (1)). */
void orc_blur(const double* v, int H, int W, const double* h, int Py, int Px,
              int bc, double* out, int nthreads)
{
    const int cy = (Py - 1) / 2, cx = (Px - 1) / 2;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int j = 0; j < Py; ++j)
                for (int i = 0; i < Px; ++i) {
                    const double w = h[j * Px + i];
                    if (w == 0.0) continue;
                    const int dy = j - cy, dx = i - cx;
                    acc += w * v[(size_t)ext(y - dy, H, bc) * W + ext(x - dx, W, bc)];
                }
            out[(size_t)y * W + x] = acc;
        }
}

/* B v: convolution with the adjoint PSF h*(x) = h(-x), i.e. correlation
 * with h, under boundary continuation `bc` (Sec. 2, definition of h*). */
void orc_corr(const double* v, int H, int W, const double* h, int Py, int Px,
              int bc, double* out, int nthreads)
{
    const int cy = (Py - 1) / 2, cx = (Px - 1) / 2;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int j = 0; j < Py; ++j)
                for (int i = 0; i < Px; ++i) {
                    const double w = h[j * Px + i];
                    if (w == 0.0) continue;
                    const int dy = j - cy, dx = i - cx;
                    acc += w * v[(size_t)ext(y + dy, H, bc) * W + ext(x + dx, W, bc)];
                }
            out[(size_t)y * W + x] = acc;
        }
}

/* Information divergence r_f(s) = s - f - f ln(s/f), eq. (7).
 * For f <= 0 the limit f ln(s/f) -> 0 gives r_0(s) = s. */
double orc_rf(double f, double s)
{
    if (f <= 0.0) return s;
    return s - f - f * log(s / f);
}

/* The lookup mode of Sec. 4.1: r_1(x) = x - 1 - ln x known at the samples
 * x_k = k/64, k = 1..65*64, linearly interpolated between them; below the
 * first sample the first sample; beyond 65 the tangent of r_1 at 65; and
 * r_f(s) = f r_1(s/f) (r_0(s) = s). */
static double r1_exact(double x) { return x - 1.0 - log(x); }

double orc_rf_lut(double f, double s)
{
    if (f <= 0.0) return s;
    const double x = s / f;
    if (x > 65.0) return f * (r1_exact(65.0) + (1.0 - 1.0 / 65.0) * (x - 65.0));
    double t = x * 64.0;
    if (t < 1.0) t = 1.0;
    int k = (int)t;
    if (k > 65 * 64 - 1) k = 65 * 64 - 1;
    const double a = r1_exact(k / 64.0), b = r1_exact((k + 1) / 64.0);
    return f * (a + (t - k) * (b - a));
}

/* Diffusivity of the regularised L1 / TV penaliser, up to the constant
 * factor 1/2 that cancels in the quotient of eq. (9):
 *   phi(z) = (z + eps^2)^(-1/2). */
static double pen_deriv(double z, double eps)
{
    return 1.0 / sqrt(z + eps * eps);
}

/* Diffusivity g = 2 Psi'(z) of the regulariser (same scaling as pen_deriv):
 *   psi = 0: regularised TV, Psi(z) = sqrt(z + eps^2)      -> (z + eps^2)^(-1/2)
 *   psi = 1: a penaliser non-convex in |grad u| (Sec. 2.3, "non-convex
 *            w.r.t. s"), Perona-Malik Psi(z) = (lam^2/2) ln(1 + z/lam^2)
 *            -> lam^2 / (lam^2 + z), lam = eps. */
static double diffusivity(double z, double eps, int psi)
{
    return psi ? eps * eps / (eps * eps + z) : pen_deriv(z, eps);
}

/* -2 dg/dz expressed through g: g^3 (TV) or 2 g^2 / lam^2 (Perona-Malik). */
static double diffusivity_slope(double g, double eps, int psi)
{
    return psi ? 2.0 * g * g / (eps * eps) : g * g * g;
}

/* Nonlinear diffusion term D(u) = div(Psi'(|grad u|^2) grad u), eq. (11),
 * by central differences (Sec. 4.1):
 *   g(p)  = psi(gx^2 + gy^2), gx = (u(y,x+1) - u(y,x-1))/2,
 *           gy = (u(y+1,x) - u(y-1,x))/2, neighbours clamped into the image;
 *   D(p)  = sum over the 4-neighbours n of p inside the image of
 *           (g(p) + g(n))/2 * (u(n) - u(p))
 * (fluxes between pixel centres with averaged diffusivity, zero flux across
 * the image border). */
void orc_tv(const double* u, int H, int W, double eps_t, int psi, double* D, int nthreads)
{
    double* g = (double*)malloc(sizeof(double) * (size_t)H * W);
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int xm = ext(x - 1, W, ORC_BC_REPLICATE), xp = ext(x + 1, W, ORC_BC_REPLICATE);
            const int ym = ext(y - 1, H, ORC_BC_REPLICATE), yp = ext(y + 1, H, ORC_BC_REPLICATE);
            const double gx = (u[(size_t)y * W + xp] - u[(size_t)y * W + xm]) / 2.0;
            const double gy = (u[(size_t)yp * W + x] - u[(size_t)ym * W + x]) / 2.0;
            g[(size_t)y * W + x] = diffusivity(gx * gx + gy * gy, eps_t, psi);
        }
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const size_t p = (size_t)y * W + x;
            const int ny[4] = {y - 1, y + 1, y, y};
            const int nx[4] = {x, x, x - 1, x + 1};
            double acc = 0.0;
            for (int k = 0; k < 4; ++k) {
                if (ny[k] < 0 || ny[k] >= H || nx[k] < 0 || nx[k] >= W) continue;
                const size_t n = (size_t)ny[k] * W + nx[k];
                acc += 0.5 * (g[p] + g[n]) * (u[n] - u[p]);
            }
            D[p] = acc;
        }
    free(g);
}

/* One RRRL step, eqs. (9)-(12), with the multiplicative factor u^k of the
 * Richardson-Lucy form:
 *   s   = max(A u, s_min)
 *   W   = phi(r_f(s))  (robust)   or 1 (non-robust)
 *   q   = W * max(f,0) / s
 *   u'  = u * (B q + alpha [D(u)]_+) / (B W - alpha [D(u)]_-)
 * with [z]_+ = max(z,0), [z]_- = min(z,0) (eq. (12)).
 * If `parts` is non-NULL it receives s, W, q, N1 = Bq, N2 = BW, D (6 planes). */
void orc_rrrl_step(const double* f, const double* u, double* u_next, int H, int W,
                   const double* h, int Py, int Px, const orc_params* p,
                   double* parts, int nthreads)
{
    const size_t n = (size_t)H * W;
    double* buf = (double*)malloc(sizeof(double) * n * 6);
    double *s = buf, *Wt = buf + n, *q = buf + 2 * n, *N1 = buf + 3 * n, *N2 = buf + 4 * n,
           *D = buf + 5 * n;

    orc_blur(u, H, W, h, Py, Px, p->bc, s, nthreads);
    for (size_t i = 0; i < n; ++i) {
        const double si = s[i] > p->s_min ? s[i] : p->s_min;
        s[i] = si;
        if (p->robust) {
            const double r = p->rf_lut ? orc_rf_lut(f[i], si) : orc_rf(f[i], si);
            Wt[i] = pen_deriv(r > 0.0 ? r : 0.0, p->eps_data);
        } else {
            Wt[i] = 1.0;
        }
        q[i] = Wt[i] * (f[i] > 0.0 ? f[i] : 0.0) / si;
    }
    orc_corr(q, H, W, h, Py, Px, p->bc, N1, nthreads);
    orc_corr(Wt, H, W, h, Py, Px, p->bc, N2, nthreads);
    orc_tv(u, H, W, p->eps_tv, p->psi, D, nthreads);
    for (size_t i = 0; i < n; ++i) {
        const double dp = D[i] > 0.0 ? D[i] : 0.0;
        const double dm = D[i] < 0.0 ? D[i] : 0.0;
        u_next[i] = u[i] * (N1[i] + p->alpha * dp) / (N2[i] - p->alpha * dm);
    }
    if (parts) memcpy(parts, buf, sizeof(double) * n * 6);
    free(buf);
}

/* `iters` RRRL steps from u0.  ckpt (nullable) receives u^0..u^{iters-1}. */
void orc_rrrl(const double* f, const double* u0, double* uK, int H, int W,
              const double* h, int Py, int Px, const orc_params* p, int iters,
              double* ckpt, int nthreads)
{
    const size_t n = (size_t)H * W;
    double* a = (double*)malloc(sizeof(double) * n);
    double* b = (double*)malloc(sizeof(double) * n);
    memcpy(a, u0, sizeof(double) * n);
    for (int k = 0; k < iters; ++k) {
        if (ckpt) memcpy(ckpt + (size_t)k * n, a, sizeof(double) * n);
        orc_rrrl_step(f, a, b, H, W, h, Py, Px, p, NULL, nthreads);
        double* t = a; a = b; b = t;
    }
    memcpy(uK, a, sizeof(double) * n);
    free(a);
    free(b);
}

/* ------------------------------------------------------------------ adjoint
 * Reverse-mode derivative of one RRRL step u -> u' = step(u; f, h, alpha),
 * written out term by term from the forward definition above.  Given
 * lam = dL/du', writes du = dL/du and ACCUMULATES dL/df into df, dL/dh into
 * dh (Py*Px, every array entry, zero or not) and dL/dalpha into *dalpha.
 * Derivatives of max/min/clamp are taken as the indicator of the branch
 * taken (0 at ties); r_f(s) := s for f <= 0 has df = 0 there. */

/* transpose of A: scatter v(x) h(d) onto the continued index of x - d */
static void blur_T(const double* v, int H, int W, const double* h, int Py, int Px, int bc, double* out)
{
    const int cy = (Py - 1) / 2, cx = (Px - 1) / 2;
    memset(out, 0, sizeof(double) * (size_t)H * W);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int j = 0; j < Py; ++j)
                for (int i = 0; i < Px; ++i) {
                    const double w = h[j * Px + i];
                    if (w == 0.0) continue;
                    const int dy = j - cy, dx = i - cx;
                    out[(size_t)ext(y - dy, H, bc) * W + ext(x - dx, W, bc)] += w * v[(size_t)y * W + x];
                }
}

/* transpose of B: scatter v(x) h(d) onto the continued index of x + d */
static void corr_T(const double* v, int H, int W, const double* h, int Py, int Px, int bc, double* out)
{
    const int cy = (Py - 1) / 2, cx = (Px - 1) / 2;
    memset(out, 0, sizeof(double) * (size_t)H * W);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int j = 0; j < Py; ++j)
                for (int i = 0; i < Px; ++i) {
                    const double w = h[j * Px + i];
                    if (w == 0.0) continue;
                    const int dy = j - cy, dx = i - cx;
                    out[(size_t)ext(y + dy, H, bc) * W + ext(x + dx, W, bc)] += w * v[(size_t)y * W + x];
                }
}

void orc_rrrl_step_adjoint(const double* f, const double* u, int H, int W, const double* h, int Py, int Px,
                           const orc_params* p, const double* lam, double* du, double* df, double* dh,
                           double* dalpha, int nthreads)
{
    const size_t n = (size_t)H * W;
    const int cy = (Py - 1) / 2, cx = (Px - 1) / 2;
    double* buf = (double*)malloc(sizeof(double) * n * 16);
    double *s = buf, *st = buf + n, *r = buf + 2 * n, *Wt = buf + 3 * n, *q = buf + 4 * n, *N1 = buf + 5 * n,
           *N2 = buf + 6 * n, *g = buf + 7 * n, *D = buf + 8 * n, *a = buf + 9 * n, *b = buf + 10 * n,
           *c = buf + 11 * n, *dq = buf + 12 * n, *dW = buf + 13 * n, *ds = buf + 14 * n, *tmp = buf + 15 * n;

    /* forward intermediates */
    orc_blur(u, H, W, h, Py, Px, p->bc, s, nthreads);
    for (size_t i = 0; i < n; ++i) {
        st[i] = s[i] > p->s_min ? s[i] : p->s_min;
        r[i] = orc_rf(f[i], st[i]);
        Wt[i] = p->robust ? pen_deriv(r[i] > 0.0 ? r[i] : 0.0, p->eps_data) : 1.0;
        q[i] = Wt[i] * (f[i] > 0.0 ? f[i] : 0.0) / st[i];
    }
    orc_corr(q, H, W, h, Py, Px, p->bc, N1, nthreads);
    orc_corr(Wt, H, W, h, Py, Px, p->bc, N2, nthreads);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const int xm = ext(x - 1, W, ORC_BC_REPLICATE), xp = ext(x + 1, W, ORC_BC_REPLICATE);
            const int ym = ext(y - 1, H, ORC_BC_REPLICATE), yp = ext(y + 1, H, ORC_BC_REPLICATE);
            const double gx = (u[(size_t)y * W + xp] - u[(size_t)y * W + xm]) / 2.0;
            const double gy = (u[(size_t)yp * W + x] - u[(size_t)ym * W + x]) / 2.0;
            g[(size_t)y * W + x] = diffusivity(gx * gx + gy * gy, p->eps_tv, p->psi);
        }
    orc_tv(u, H, W, p->eps_tv, p->psi, D, nthreads);

    /* update u' = u * Num / Den */
    for (size_t i = 0; i < n; ++i) {
        const double dp = D[i] > 0.0 ? D[i] : 0.0, dm = D[i] < 0.0 ? D[i] : 0.0;
        const double num = N1[i] + p->alpha * dp, den = N2[i] - p->alpha * dm;
        du[i] = lam[i] * num / den;
        a[i] = lam[i] * u[i] / den;                 /* dL/dNum = dL/dN1 */
        b[i] = -lam[i] * u[i] * num / (den * den);  /* dL/dDen = dL/dN2 */
        *dalpha += a[i] * dp - b[i] * dm;
        c[i] = p->alpha * (a[i] * (D[i] > 0.0 ? 1.0 : 0.0) - b[i] * (D[i] < 0.0 ? 1.0 : 0.0)); /* dL/dD */
    }
    /* N1 = B q, N2 = B W */
    corr_T(a, H, W, h, Py, Px, p->bc, dq);
    corr_T(b, H, W, h, Py, Px, p->bc, dW);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int j = 0; j < Py; ++j)
                for (int i = 0; i < Px; ++i) {
                    const size_t src = (size_t)ext(y + j - cy, H, p->bc) * W + ext(x + i - cx, W, p->bc);
                    const size_t o = (size_t)y * W + x;
                    dh[j * Px + i] += a[o] * q[src] + b[o] * Wt[src];
                }
    /* q = W f+ / s~,  W = phi(r),  r = r_f(s~),  s~ = max(s, s_min) */
    for (size_t i = 0; i < n; ++i) {
        const double fp = f[i] > 0.0 ? f[i] : 0.0;
        double dWi = dW[i] + dq[i] * fp / st[i];
        double dst = -dq[i] * Wt[i] * fp / (st[i] * st[i]);
        if (f[i] > 0.0) df[i] += dq[i] * Wt[i] / st[i];
        if (p->robust) {
            const double dr = r[i] > 0.0 ? dWi * (-0.5) * Wt[i] * Wt[i] * Wt[i] : 0.0;
            if (f[i] > 0.0) {
                dst += dr * (1.0 - f[i] / st[i]);
                df[i] += dr * (-log(st[i] / f[i]));
            } else {
                dst += dr;
            }
        }
        ds[i] = s[i] > p->s_min ? dst : 0.0;
    }
    /* s = A u */
    blur_T(ds, H, W, h, Py, Px, p->bc, tmp);
    for (size_t i = 0; i < n; ++i) du[i] += tmp[i];
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int j = 0; j < Py; ++j)
                for (int i = 0; i < Px; ++i) {
                    const size_t src = (size_t)ext(y - (j - cy), H, p->bc) * W + ext(x - (i - cx), W, p->bc);
                    dh[j * Px + i] += ds[(size_t)y * W + x] * u[src];
                }
    /* D = sum_n (g_p + g_n)/2 (u_n - u_p): with g frozen, and through g */
    double* dg = dq;  /* reuse */
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const size_t pp = (size_t)y * W + x;
            const int ny[4] = {y - 1, y + 1, y, y};
            const int nx[4] = {x, x, x - 1, x + 1};
            double acc = 0.0, accg = 0.0;
            for (int k = 0; k < 4; ++k) {
                if (ny[k] < 0 || ny[k] >= H || nx[k] < 0 || nx[k] >= W) continue;
                const size_t nn = (size_t)ny[k] * W + nx[k];
                acc += 0.5 * (g[pp] + g[nn]) * (c[nn] - c[pp]);
                accg += 0.5 * (u[nn] - u[pp]) * (c[pp] - c[nn]);
            }
            du[pp] += acc;
            dg[pp] = accg;
        }
    /* g = psi(gx^2 + gy^2), central differences with clamped neighbours */
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const size_t pp = (size_t)y * W + x;
            const int xm = ext(x - 1, W, ORC_BC_REPLICATE), xp = ext(x + 1, W, ORC_BC_REPLICATE);
            const int ym = ext(y - 1, H, ORC_BC_REPLICATE), yp = ext(y + 1, H, ORC_BC_REPLICATE);
            const double gx = (u[(size_t)y * W + xp] - u[(size_t)y * W + xm]) / 2.0;
            const double gy = (u[(size_t)yp * W + x] - u[(size_t)ym * W + x]) / 2.0;
            const double g3 = diffusivity_slope(g[pp], p->eps_tv, p->psi);
            const double dgx = dg[pp] * (-g3 * gx), dgy = dg[pp] * (-g3 * gy);
            du[(size_t)y * W + xp] += 0.5 * dgx;
            du[(size_t)y * W + xm] -= 0.5 * dgx;
            du[(size_t)yp * W + x] += 0.5 * dgy;
            du[(size_t)ym * W + x] -= 0.5 * dgy;
        }
    free(buf);
}
