/*
 * Test driver: runs every function of the FP64 oracle on one small problem read from
 * stdin and prints the results as hexadecimal floats, so that a build of the oracle with
 * AddressSanitizer and UndefinedBehaviorSanitizer can be exercised and its results
 * compared with the regular build's.  Test infrastructure only.
 *
 * stdin: H W kh kw bc K mode tau hyst R, then H*W values of f and kh*kw values of h.
 * stdout: "<name> <count>" then one value per line, for each output.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_conv(const double *u, int H, int W, const double *h, int kh, int kw, int bc,
                 double *out);
void oracle_corr(const double *r, int H, int W, const double *h, int kh, int kw, int bc,
                 double *out);
void oracle_rl(const double *f, double *u, int H, int W, const double *h, int kh, int kw,
               int bc, int K, double *r);
void oracle_rl_tv(const double *f, double *u, int H, int W, const double *h, int kh, int kw,
                  int bc, int K, double lambda, double eps, double *r, double *div);
void oracle_rl_robust(const double *f, double *u, int H, int W, const double *h, int kh,
                      int kw, int bc, int K, double eps, double *r, double *w, double *num,
                      double *den);
long oracle_thin_step(const double *f, double *u, double *r, uint8_t *cnt, int H, int W,
                      const double *h, int kh, int kw, int bc, long k, int mode, float tau,
                      int hyst, int reset_period, double *u_prev);
long oracle_thin_step_blocks(const double *f, double *u, double *r, uint8_t *cnt, int H,
                             int W, const double *h, int kh, int kw, int bc, long k, int mode,
                             float tau, int hyst, int reset_period, int B, double *u_prev);
double oracle_sum(const double *a, long n);

static void put(const char *name, const double *a, long n)
{
    printf("%s %ld\n", name, n);
    for (long i = 0; i < n; ++i) printf("%a\n", a[i]);
}

int main(void)
{
    int H, W, kh, kw, bc, K, mode, hyst, R;
    float tau;
    if (scanf("%d %d %d %d %d %d %d %f %d %d", &H, &W, &kh, &kw, &bc, &K, &mode, &tau, &hyst,
              &R) != 10)
        return 2;
    const long n = (long)H * W, m = (long)kh * kw;
    double *f = malloc(sizeof(double) * n), *h = malloc(sizeof(double) * m);
    double *u = malloc(sizeof(double) * n), *r = malloc(sizeof(double) * n);
    double *a = malloc(sizeof(double) * n), *b = malloc(sizeof(double) * n);
    double *c = malloc(sizeof(double) * n), *d = malloc(sizeof(double) * n);
    uint8_t *cnt = malloc((size_t)n);
    for (long i = 0; i < n; ++i)
        if (scanf("%lf", &f[i]) != 1) return 2;
    for (long i = 0; i < m; ++i)
        if (scanf("%lf", &h[i]) != 1) return 2;

    oracle_conv(f, H, W, h, kh, kw, bc, a);
    put("conv", a, n);
    oracle_corr(f, H, W, h, kh, kw, bc, a);
    put("corr", a, n);

    memcpy(u, f, sizeof(double) * n);
    oracle_rl(f, u, H, W, h, kh, kw, bc, K, r);
    put("rl", u, n);

    memcpy(u, f, sizeof(double) * n);
    memset(r, 0, sizeof(double) * n);
    memset(cnt, 0, (size_t)n);
    double act[64];
    int ks = K < 64 ? K : 64;
    for (int k = 0; k < ks; ++k)
        act[k] = (double)oracle_thin_step(f, u, r, cnt, H, W, h, kh, kw, bc, k, mode, tau,
                                          hyst, R, a);
    put("thin_u", u, n);
    put("thin_r", r, n);
    for (long i = 0; i < n; ++i) a[i] = cnt[i];
    put("thin_cnt", a, n);
    put("thin_active", act, ks);

    memcpy(u, f, sizeof(double) * n);
    memset(r, 0, sizeof(double) * n);
    memset(cnt, 0, (size_t)n);
    for (int k = 0; k < ks; ++k)
        act[k] = (double)oracle_thin_step_blocks(f, u, r, cnt, H, W, h, kh, kw, bc, k, mode,
                                                 tau, hyst, R, 3, a);
    put("block_u", u, n);
    for (long i = 0; i < n; ++i) a[i] = cnt[i];
    put("block_cnt", a, n);
    put("block_active", act, ks);

    memcpy(u, f, sizeof(double) * n);
    oracle_rl_tv(f, u, H, W, h, kh, kw, bc, K, 0.1, 1e-3, r, a);
    put("tv", u, n);

    memcpy(u, f, sizeof(double) * n);
    oracle_rl_robust(f, u, H, W, h, kh, kw, bc, K, 0.05, r, a, b, c);
    put("robust", u, n);

    double s = oracle_sum(f, n);
    put("sum", &s, 1);
    free(f); free(h); free(u); free(r); free(a); free(b); free(c); free(d); free(cnt);
    return 0;
}
