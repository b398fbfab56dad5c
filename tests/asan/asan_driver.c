/* Host AddressSanitizer / UndefinedBehaviorSanitizer run of the C oracle and
 * of the library's host-only tuning-cache code (test infrastructure).  Every
 * oracle entry point is called on small seeded inputs, with the adjoint
 * identity A^H A x = (2^(m+1) - 2) x as a sanity check, and the cache is
 * stored to, read, corrupted and rewritten.  Exit status 0 = clean. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int mro_forward_level(int m, int i, const double *x, double *y, int method);
int mro_forward(int m, const double *x, double *y, int method);
int mro_forward_bin(int m, int i, int64_t w, int64_t k, const double *x, double *out);
int mro_adjoint(int m, const double *gy, double *gx, int method);
int mro_adjoint_point(int m, int64_t p, const double *gy, double *out);
int mro_spectral_loss(int m, const double *x, const double *z, double *num_den, double *L);
int mro_spectral_loss_grad(int m, const double *x, const double *z, const double *num_den, double gL, double *gx);
int mro_max_order(void);
int mrdft_tune_cache_lookup(const char *path, const char *key, int *t, int *g, int *o, int *s);
int mrdft_tune_cache_store(const char *path, const char *key, int t, int g, int o, int s);

static uint64_t state = 1507;
static double uni(void) {
    state = state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(state >> 11) / 9007199254740992.0 - 0.5;
}

static int check(int ok, const char *what) {
    if (!ok) fprintf(stderr, "FAILED: %s\n", what);
    return ok ? 0 : 1;
}

int main(int argc, char **argv) {
    const char *dir = argc > 1 ? argv[1] : ".";
    int bad = 0;
    for (int m = 1; m <= 13; ++m) {
        const int64_t n = (int64_t)1 << m;
        double *x = malloc(sizeof(double) * 2 * n), *z = malloc(sizeof(double) * n);
        double *xr = malloc(sizeof(double) * n);
        double *y = malloc(sizeof(double) * 2 * n * m), *y2 = malloc(sizeof(double) * 2 * n * m);
        double *g = malloc(sizeof(double) * 2 * n), *nd = malloc(sizeof(double) * 2 * m);
        for (int64_t q = 0; q < 2 * n; ++q) x[q] = uni();
        for (int64_t q = 0; q < n; ++q) { z[q] = uni(); xr[q] = uni(); }
        bad += check(mro_forward(m, x, y, 0) == 0, "forward direct");
        bad += check(mro_forward(m, x, y2, 1) == 0, "forward fft");
        double e = 0, r = 0;
        for (int64_t q = 0; q < 2 * n * m; ++q) { e += (y[q] - y2[q]) * (y[q] - y2[q]); r += y[q] * y[q]; }
        bad += check(sqrt(e / r) < 1e-12, "direct vs fft");
        bad += check(mro_forward_level(m, m, x, y2, -1) == 0, "forward level");
        double b[2];
        bad += check(mro_forward_bin(m, m, 0, n - 1, x, b) == 0, "forward bin");
        bad += check(mro_adjoint(m, y, g, 0) == 0 && mro_adjoint(m, y, g, 1) == 0, "adjoint");
        double ee = 0, rr = 0;
        for (int64_t q = 0; q < 2 * n; ++q) {
            const double want = (double)(((int64_t)2 << m) - 2) * x[q];
            ee += (g[q] - want) * (g[q] - want);
            rr += want * want;
        }
        bad += check(sqrt(ee / rr) < 1e-12, "A^H A x");
        bad += check(mro_adjoint_point(m, n - 1, y, b) == 0, "adjoint point");
        double L = 0;
        bad += check(mro_spectral_loss(m, xr, z, nd, &L) == 0, "loss");
        bad += check(mro_spectral_loss_grad(m, xr, z, nd, 0.5, g) == 0, "loss grad");
        free(x); free(z); free(xr); free(y); free(y2); free(g); free(nd);
    }
    bad += check(mro_forward(0, NULL, NULL, 0) != 0, "order 0 rejected");
    bad += check(mro_max_order() > 0, "max order");
    char path[4096];
    snprintf(path, sizeof(path), "%s/asan_tune.json", dir);
    int t = 0, gr = 0, o = 0, s = 0;
    bad += check(mrdft_tune_cache_store(path, "gfx950|c64|1x2^18", 11, 0, 3, 1) == 0, "store");
    bad += check(mrdft_tune_cache_store(path, "gfx950|r32|64x2^16", 12, 0, 3, 0) == 0, "store 2");
    bad += check(mrdft_tune_cache_lookup(path, "gfx950|c64|1x2^18", &t, &gr, &o, &s) == 1 && t == 11 && o == 3 && s == 1,
                 "lookup");
    FILE *f = fopen(path, "wb");
    if (f) { fputs("{\"format\": \"mrdft-tune\", \"version\": 1, \"entries\": {\"k\": {\"tile_log\": ", f); fclose(f); }
    bad += check(mrdft_tune_cache_lookup(path, "k", &t, &gr, &o, &s) == 0, "corrupt ignored");
    bad += check(mrdft_tune_cache_store(path, "k", 11, 512, 0, 0) == 0, "rewrite");
    bad += check(mrdft_tune_cache_lookup(path, "k", &t, &gr, &o, &s) == 1 && gr == 512, "lookup after rewrite");
    bad += check(mrdft_tune_cache_lookup(path, "a\"b", &t, &gr, &o, &s) == -1, "bad key");
    remove(path);
    if (bad) return 1;
    printf("asan driver clean\n");
    return 0;
}
