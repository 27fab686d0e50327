/*
 * rl_oracle.c -- plain, slow, obviously correct FP64 CPU oracle for Richardson-Lucy
 * deconvolution and its thinned (selective) variant.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load this library.  The product path (the HIP library and its Python
 * binding) never includes, links or calls anything in this directory, and this file
 * includes nothing of the product path.
 *
 * What it computes (notation of the paper):
 *   - blur model and problem statement f ~ u*h              (Section 1, eq. 1-2)
 *   - RL: u^0 = f, u^{k+1} = (h^* * (f / (u^k*h))) . u^k      (Section 2, eq. 3)
 *     where h^* is h reflected about the origin, so h^* * r is the correlation of r
 *     with h                                                  (Section 2, text after eq. 3)
 *   - boundary: every missing pixel is replaced by an image pixel (Section 2, "Boundary
 *     treatment").  Two readings are offered:
 *       BC_REFLECT   half-sample symmetric continuation (c b a | a b c), period 2N;
 *       BC_REPLICATE the closest image pixel (constant continuation), the paper's rule.
 *   - robustified data term (Section 2 names such variants): weights 1/sqrt(d + eps^2) of
 *     the I-divergence d of u^k*h from f, see oracle_rl_robust
 *   - thinned RL: active pixels get fresh v^k and u^{k+1}; inactive pixels keep v^{k-1}
 *     (here: keep their ratio r) and u^k; every R-th iteration all pixels are active
 *     (Section 4, eq. 4-5 and the reset rule after them).
 *
 * Conventions: images are row-major H x W; the PSF is kh x kw with origin
 * (oy, ox) = (kh/2, kw/2), so tap h[i][j] sits at offset (i-oy, j-ox).
 *   conv(u)(y,x) = sum_{i,j} h[i][j] * u[fold(y-(i-oy))][fold(x-(j-ox))]
 *   corr(r)(y,x) = sum_{i,j} h[i][j] * r[fold(y+(i-oy))][fold(x+(j-ox))]
 * Sums run over i ascending, then j ascending; zero taps are skipped (exact).
 * r = f / v where v > 0, else 0 (the paper does not say what happens at v = 0).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (build() in __init__.py).
 * -ffp-contract=off keeps every product and sum a separately rounded FP64 operation.
 * OpenMP only splits the image rows among threads; every pixel's sum is computed by one
 * thread in the order above, so the result does not depend on the thread count.
 *
 * ORACLE_MUTANT (compile-time, default 0) plants one deliberate mistake.  It exists only
 * so the test suite can show that its pins catch each kind of mistake.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

enum { BC_REFLECT = 0, BC_REPLICATE = 1 };
enum { THIN_OFF = 0, THIN_ABS = 1, THIN_REL = 2 };

/* ---- boundary fold (Section 2, "Boundary treatment") -------------------------------- */
long oracle_fold(long i, long n, int bc)
{
    if (bc == BC_REPLICATE) {
        if (i < 0) return 0;
        if (i >= n) return n - 1;
        return i;
    }
    long p = i % (2 * n);
    if (p < 0) p += 2 * n;
#if ORACLE_MUTANT == 1
    /* planted: whole-sample mirror (c b | a b c) instead of half-sample */
    if (n > 1) { p = i % (2 * n - 2); if (p < 0) p += 2 * n - 2; return p < n ? p : 2 * n - 2 - p; }
    return 0;
#else
    return p < n ? p : 2 * n - 1 - p;
#endif
}

/* ---- one output of the forward convolution u*h at (y,x) (Section 1, eq. 2) ----------- */
static double conv_at(const double *u, long H, long W, const double *h, int kh, int kw,
                      int bc, long y, long x)
{
    const int oy = kh / 2, ox = kw / 2;
    double s = 0.0;
    for (int i = 0; i < kh; ++i) {
        for (int j = 0; j < kw; ++j) {
#if ORACLE_MUTANT == 2
            double w = h[j * kh + i]; /* planted: transposed PSF (only differs if kh==kw) */
            if (kh != kw) w = h[i * kw + j];
#else
            double w = h[i * kw + j];
#endif
#if ORACLE_MUTANT == 3
            if (i == kh - 1 && j == kw - 1) continue; /* planted: last tap dropped */
#endif
            if (w == 0.0) continue;
            long sy = oracle_fold(y - (i - oy), H, bc);
            long sx = oracle_fold(x - (j - ox), W, bc);
            s += w * u[sy * W + sx];
        }
    }
    return s;
}

/* ---- one output of the adjoint h^* * r at (y,x) (Section 2, eq. 3) -------------------- */
static double corr_at(const double *r, long H, long W, const double *h, int kh, int kw,
                      int bc, long y, long x)
{
    const int oy = kh / 2, ox = kw / 2;
    double s = 0.0;
    for (int i = 0; i < kh; ++i) {
        for (int j = 0; j < kw; ++j) {
            double w = h[i * kw + j];
            if (w == 0.0) continue;
#if ORACLE_MUTANT == 4
            long sy = oracle_fold(y - (i - oy), H, bc); /* planted: h instead of h^* */
            long sx = oracle_fold(x - (j - ox), W, bc);
#else
            long sy = oracle_fold(y + (i - oy), H, bc);
            long sx = oracle_fold(x + (j - ox), W, bc);
#endif
            s += w * r[sy * W + sx];
        }
    }
    return s;
}

void oracle_conv(const double *u, int H, int W, const double *h, int kh, int kw, int bc,
                 double *out)
{
#pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x)
            out[y * W + x] = conv_at(u, H, W, h, kh, kw, bc, y, x);
}

void oracle_corr(const double *r, int H, int W, const double *h, int kh, int kw, int bc,
                 double *out)
{
#pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x)
            out[y * W + x] = corr_at(r, H, W, h, kh, kw, bc, y, x);
}

/* ratio f / (u*h), guarded: a non-positive denominator gives 0 */
static double ratio(double f, double v)
{
#if ORACLE_MUTANT == 5
    return f > 0.0 ? v / f : 0.0; /* planted: inverted ratio */
#else
    return v > 0.0 ? f / v : 0.0;
#endif
}

static double update(double u, double c)
{
#if ORACLE_MUTANT == 6
    (void)u;
    return c; /* planted: the multiplicative factor u^k is dropped */
#else
    return u * c;
#endif
}

/*
 * Plain RL (Section 2, eq. 3): K iterations from u (in/out; the caller sets u^0, usually f).
 * Work arrays v and r of H*W doubles are supplied by the caller.
 */
void oracle_rl(const double *f, double *u, int H, int W, const double *h, int kh, int kw,
               int bc, int K, double *r)
{
    const long N = (long)H * W;
    for (int k = 0; k < K; ++k) {
#pragma omp parallel for schedule(static)
        for (long y = 0; y < H; ++y)
            for (long x = 0; x < W; ++x)
                r[y * W + x] = ratio(f[y * W + x], conv_at(u, H, W, h, kh, kw, bc, y, x));
#pragma omp parallel for schedule(static)
        for (long y = 0; y < H; ++y)
            for (long x = 0; x < W; ++x)
                u[y * W + x] = update(u[y * W + x], corr_at(r, H, W, h, kh, kw, bc, y, x));
        (void)N;
    }
}

/*
 * Regularised RL with a total-variation term (the variant of Dey et al., 2006; the paper
 * names regularised RL among the methods its optimisations carry over to, Section 2):
 *   u^{k+1} = u^k . c / (1 - lambda * div(grad u^k / |grad u^k|_eps)),  c as in eq. 3.
 * Discretisation (a reading; the paper gives none): forward differences for the gradient,
 *   gx(y,x) = u(y,x+1) - u(y,x),  gy(y,x) = u(y+1,x) - u(y,x),
 * which are 0 across the last column / row (both boundary rules continue the image with
 * its edge pixel there); n = (gx, gy) / sqrt(gx^2 + gy^2 + eps^2); backward differences for
 * the divergence, div(y,x) = nx(y,x) - nx(y,x-1) + ny(y,x) - ny(y-1,x), with n = 0 before
 * the first column / row.  Forward gradient and backward divergence are negative adjoints
 * of each other, which the tests check.
 */
static double tv_n(const double *u, long H, long W, long y, long x, int axis)
{
    const double c = u[y * W + x];
    const double gx = x + 1 < W ? u[y * W + x + 1] - c : 0.0;
    const double gy = y + 1 < H ? u[(y + 1) * W + x] - c : 0.0;
    return (axis == 0 ? gx : gy);
}

void oracle_tv_div(const double *u, int H, int W, double eps, double *div)
{
#pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            double d = 0.0;
            /* n at (y, x), (y, x-1) and (y-1, x) */
            const long py[3] = {y, y, y - 1}, px[3] = {x, x - 1, x};
            for (int q = 0; q < 3; ++q) {
                if (py[q] < 0 || px[q] < 0) continue;
                const double gx = tv_n(u, H, W, py[q], px[q], 0);
                const double gy = tv_n(u, H, W, py[q], px[q], 1);
                const double m = sqrt(gx * gx + gy * gy + eps * eps);
                if (q == 0) d += gx / m + gy / m;
                else if (q == 1) d -= gx / m;
                else d -= gy / m;
            }
            div[y * W + x] = d;
        }
}

/* K iterations of TV-regularised RL from u (in/out); r and div are work arrays. */
void oracle_rl_tv(const double *f, double *u, int H, int W, const double *h, int kh, int kw,
                  int bc, int K, double lambda, double eps, double *r, double *div)
{
    for (int k = 0; k < K; ++k) {
        oracle_tv_div(u, H, W, eps, div);
#pragma omp parallel for schedule(static)
        for (long y = 0; y < H; ++y)
            for (long x = 0; x < W; ++x)
                r[y * W + x] = ratio(f[y * W + x], conv_at(u, H, W, h, kh, kw, bc, y, x));
#pragma omp parallel for schedule(static)
        for (long y = 0; y < H; ++y)
            for (long x = 0; x < W; ++x) {
                const double c = corr_at(r, H, W, h, kh, kw, bc, y, x);
                u[y * W + x] = update(u[y * W + x], c) / (1.0 - lambda * div[y * W + x]);
            }
    }
}

/*
 * Robustified data term (Section 2 names robust variants among the methods the
 * optimisations carry over to).  Reading: the multiplicative iteration of a robust
 * penaliser Phi applied to the pointwise I-divergence of the blurred estimate v = u*h
 * from f,
 *   d(v, f) = v - f - f ln(v / f)   (d = v where f = 0),
 * with Phi(d) = 2 sqrt(d + eps^2), i.e. weights w = Phi'(d) = 1 / sqrt(d + eps^2):
 *   u^{k+1} = u^k . (h^* * (w f / v)) / (h^* * w).
 * Where v <= 0 the ratio is 0 (as in plain RL) and d is taken as 0.  A constant w (eps
 * large) gives plain RL.
 */
double oracle_idiv(double v, double f)
{
    if (!(v > 0.0)) return 0.0;
    if (f == 0.0) return v;
#if ORACLE_MUTANT == 9
    return v - f + f * log(v / f); /* planted: sign of the log term */
#else
    return v - f - f * log(v / f);
#endif
}

static double robust_weight(double d, double eps)
{
#if ORACLE_MUTANT == 8
    return 1.0 / (d + eps * eps); /* planted: weight without the square root */
#else
    return 1.0 / sqrt(d + eps * eps);
#endif
}

/* The two correlations of one robust iteration at u: num = h^* * (w f / v), den = h^* * w;
 * r and w are work arrays (they receive w f / v and w). */
void oracle_robust_terms(const double *f, const double *u, int H, int W, const double *h,
                         int kh, int kw, int bc, double eps, double *r, double *w, double *num,
                         double *den)
{
#pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            const double v = conv_at(u, H, W, h, kh, kw, bc, y, x);
            const double fw = f[y * W + x];
            const double wt = robust_weight(oracle_idiv(v, fw), eps);
            w[y * W + x] = wt;
            r[y * W + x] = wt * ratio(fw, v);
        }
#pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            num[y * W + x] = corr_at(r, H, W, h, kh, kw, bc, y, x);
            den[y * W + x] = corr_at(w, H, W, h, kh, kw, bc, y, x);
        }
}

/* K robust iterations from u (in/out); r, w, num, den are work arrays. */
void oracle_rl_robust(const double *f, double *u, int H, int W, const double *h, int kh, int kw,
                      int bc, int K, double eps, double *r, double *w, double *num, double *den)
{
    for (int k = 0; k < K; ++k) {
        oracle_robust_terms(f, u, H, W, h, kh, kw, bc, eps, r, w, num, den);
        /* every term of den is positive: den > 0 wherever the PSF is non-empty */
        for (long q = 0; q < (long)H * W; ++q) u[q] = update(u[q], num[q]) / den[q];
    }
}

/*
 * The convergence test of thinned RL, taken in single precision on the float32 values of
 * u^{k+1} (a) and u^k (b) (Section 4: "absolute changes ... below a given threshold").
 * ABS: |a-b| < tau;  REL: |a-b| < tau*b.  tau <= 0 never freezes; a pixel that stays 0
 * counts as converged.  Every operation is one correctly rounded float32 operation.
 */
int oracle_below(float a, float b, int mode, float tau)
{
    if (!(tau > 0.0f)) return 0;
    if (b == 0.0f && a == 0.0f) return 1;
    volatile float d = a - b; /* volatile: keep the float32 rounding of each step */
    float ad = fabsf(d);
    volatile float t = (mode == THIN_REL) ? tau * b : tau;
#if ORACLE_MUTANT == 7
    return ad <= t * 2.0f; /* planted: threshold doubled */
#else
    return ad < t;
#endif
}

/*
 * One thinned RL iteration k (Section 4, eq. 4-5, reset rule after them).
 *   full  = (k == 0) or (R > 0 and k mod R == 0): every pixel is active;
 *   else  pixel p is active iff cnt[p] < hyst.
 * Active pixels: r = f / (u^k*h) (guarded); then u^{k+1} = u^k . (h^* * r), where inactive
 * neighbours contribute their stale r; then the float32 convergence test updates cnt
 * (below: cnt = min(cnt+1, 255), else cnt = 0).  Inactive pixels keep u, r and cnt.
 * u, r, cnt are in/out.  u_prev is a caller-supplied H*W work array.
 * Returns the number of active pixels |A_k|.
 */
long oracle_thin_step(const double *f, double *u, double *r, uint8_t *cnt, int H, int W,
                      const double *h, int kh, int kw, int bc, long k, int mode, float tau,
                      int hyst, int reset_period, double *u_prev)
{
    const long N = (long)H * W;
    const int full = (k == 0) || (reset_period > 0 && k % reset_period == 0);
    long n_active = 0;
    for (long p = 0; p < N; ++p) {
        u_prev[p] = u[p];
        if (full || cnt[p] < hyst) ++n_active;
    }
#pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            long p = y * W + x;
#if ORACLE_MUTANT == 11
            /* planted: the ratio of inactive pixels is recomputed instead of kept stale */
            r[p] = ratio(f[p], conv_at(u_prev, H, W, h, kh, kw, bc, y, x));
#else
            if (full || cnt[p] < hyst)
                r[p] = ratio(f[p], conv_at(u_prev, H, W, h, kh, kw, bc, y, x));
#endif
        }
#pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            long p = y * W + x;
#if ORACLE_MUTANT == 10
            /* planted: frozen pixels are still updated (only their counter is kept) */
            if (!(full || cnt[p] < hyst)) {
                u[p] = update(u_prev[p], corr_at(r, H, W, h, kh, kw, bc, y, x));
                continue;
            }
#else
            if (!(full || cnt[p] < hyst)) continue;
#endif
            double un = update(u_prev[p], corr_at(r, H, W, h, kh, kw, bc, y, x));
            u[p] = un;
            if (mode != THIN_OFF) {
                int below = oracle_below((float)un, (float)u_prev[p], mode, tau);
                cnt[p] = below ? (uint8_t)(cnt[p] < 255 ? cnt[p] + 1 : 255) : 0;
            }
        }
    return n_active;
}

/*
 * One thinned RL iteration k under the block rule (a refinement of the adaptive update rule
 * of Section 4, which leaves such rules open): the image is cut into B x B blocks aligned
 * at (0, 0) (the last ones cut by the image edge), and the decision to freeze is taken per
 * block.  Block t's counter is the counter of its top-left pixel.
 *   full  = (k == 0) or (R > 0 and k mod R == 0): every block is active;
 *   else  block t is active iff its counter < hyst.
 * Every pixel of an active block is active: r = f / (u^k*h) (guarded), then
 * u^{k+1} = u^k . (h^* * r), where pixels of frozen blocks contribute their stale r.  Then
 * the block's counter becomes min(c+1, 255) if the float32 convergence test holds for
 * every one of its pixels, else 0.  Frozen blocks keep u and r.  On return every pixel of
 * every block carries its block's counter.  B = 1 is the per-pixel rule above.
 * Returns the number of active pixels.
 */
long oracle_thin_step_blocks(const double *f, double *u, double *r, uint8_t *cnt, int H,
                             int W, const double *h, int kh, int kw, int bc, long k, int mode,
                             float tau, int hyst, int reset_period, int B, double *u_prev)
{
    const long N = (long)H * W;
    const int full = (k == 0) || (reset_period > 0 && k % reset_period == 0);
    const int TY = (H + B - 1) / B, TX = (W + B - 1) / B;
    const long NT = (long)TY * TX;
    uint8_t *tc = (uint8_t *)malloc((size_t)NT);
    uint8_t *act = (uint8_t *)malloc((size_t)NT);
    uint8_t *all = (uint8_t *)malloc((size_t)NT);
    for (int ty = 0; ty < TY; ++ty)
        for (int tx = 0; tx < TX; ++tx) {
            long t = (long)ty * TX + tx;
            tc[t] = cnt[(long)ty * B * W + (long)tx * B];
            act[t] = (uint8_t)(full || tc[t] < hyst);
            all[t] = 1;
        }
    long n_active = 0;
    for (long p = 0; p < N; ++p) {
        u_prev[p] = u[p];
        if (act[(p / W / B) * TX + (p % W) / B]) ++n_active;
    }
#pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x)
            if (act[(y / B) * TX + x / B])
                r[y * W + x] = ratio(f[y * W + x], conv_at(u_prev, H, W, h, kh, kw, bc, y, x));
#pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x)
            if (act[(y / B) * TX + x / B])
                u[y * W + x] = update(u_prev[y * W + x], corr_at(r, H, W, h, kh, kw, bc, y, x));
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            long t = (y / B) * TX + x / B, p = y * W + x;
            if (!act[t]) continue;
#if ORACLE_MUTANT == 12
            /* planted: a block freezes when any one of its pixels passes the test */
            if (all[t] == 1) all[t] = 0;
            if (oracle_below((float)u[p], (float)u_prev[p], mode, tau)) all[t] = 2;
#else
            if (!(mode != THIN_OFF && oracle_below((float)u[p], (float)u_prev[p], mode, tau)))
                all[t] = 0;
#endif
        }
    for (long t = 0; t < NT; ++t)
        if (act[t]) {
#if ORACLE_MUTANT == 12
            const int pass = all[t] == 2;
#else
            const int pass = all[t] != 0 && mode != THIN_OFF;
#endif
            tc[t] = pass ? (uint8_t)(tc[t] < 255 ? tc[t] + 1 : 255) : 0;
        }
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) cnt[y * W + x] = tc[(y / B) * TX + x / B];
    free(tc);
    free(act);
    free(all);
    return n_active;
}

/* The convergence test above applied to n pairs (a[i], b[i]); out[i] = 0 or 1. */
void oracle_below_many(const float *a, const float *b, long n, int mode, float tau,
                       uint8_t *out)
{
    for (long i = 0; i < n; ++i) out[i] = (uint8_t)oracle_below(a[i], b[i], mode, tau);
}

/* Sum in row-major order (used for the flux sum(u)). */
double oracle_sum(const double *a, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i];
    return s;
}

int oracle_mutant(void) { return ORACLE_MUTANT; }

/* Thread count of the row loops (timing only: results do not depend on it). */
#ifdef _OPENMP
#include <omp.h>
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_threads(void) { return omp_get_max_threads(); }
#else
void oracle_set_threads(int n) { (void)n; }
int oracle_threads(void) { return 1; }
#endif
