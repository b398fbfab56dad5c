/*
 * FP64 reference implementation of the multiresolution DFT (MrDFT).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link or call
 * this file: it exists so that tests, the smoke check and the benchmark's
 * CPU baseline can compare the GPU path against a plain, obviously correct
 * implementation.  It shares no code, header, table or constant with the GPU
 * library.
 *
 * What is computed (Section 2, eq. (1)).  For a signal x of N = 2^m complex
 * samples, level i (i = 1..m) is the 2^i-point DFT of every non-overlapping
 * length-2^i rectangular window:
 *
 *     Y^(i)[w*2^i + k] = sum_{n < 2^i} x[w*2^i + n] * exp(-j*2*pi*n*k / 2^i)
 *
 * for window w = 0 .. N/2^i - 1 and bin k = 0 .. 2^i - 1.  Levels are stacked
 * i = 1 first, each N values long, bins in natural order inside a window and
 * windows in time order.  No normalisation is applied.
 *
 * Reading taken: eq. (1) prints the level block as I_{2^{m-1}} (x) E_{2^i},
 * which is not N x N; the block used here is I_{2^{m-i}} (x) E_{2^i}, the only
 * one that gives N outputs per level and matches the text below eq. (1)
 * (level i is a short-time DFT with a rectangular window of length 2^i).
 *
 * Two evaluation routes for the same definition:
 *   - direct sums: the exponent n*k is reduced modulo 2^i exactly in 64-bit
 *     integers, then looked up in a table of exp(-j*2*pi*e/2^i) computed with
 *     the C library cos/sin in double;
 *   - a plain recursive radix-2 decimation-in-time FFT of every window (a
 *     library-style primitive standing in for the per-window DFT).
 * The direct route is the definition written out; tests cross-check the two.
 *
 * Adjoint.  The conjugate transpose of eq. (1) maps per-level gradients gY to
 *     gx[w*2^i + n] += sum_k gY^(i)[w*2^i + k] * exp(+j*2*pi*n*k / 2^i),
 * summed over all levels i = 1..m.
 *
 * Spectral loss.  For real signals x, z of length N:
 *     num_i = || Y^(i)(x) - Y^(i)(z) ||^2,  den_i = || Y^(i)(z) ||^2,
 *     L = (1/m) * sum_i num_i / den_i,
 * and dL/dx = Re( A^H g ) with g^(i) = gL * 2 * (Y^(i)(x) - Y^(i)(z)) / (m*den_i),
 * where A^H is the adjoint above (gradient convention: for a real loss the
 * gradient of a complex value is dL/dRe + j*dL/dIm).
 *
 * All buffers are interleaved (re, im) doubles.  Every entry point returns 0
 * on success and a negative value for invalid arguments; nothing aborts.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MRO_MAX_M 30

typedef struct {
    double re, im;
} cplx;

static cplx c_add(cplx a, cplx b) { cplx r = {a.re + b.re, a.im + b.im}; return r; }
static cplx c_sub(cplx a, cplx b) { cplx r = {a.re - b.re, a.im - b.im}; return r; }
static cplx c_mul(cplx a, cplx b)
{
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}
static cplx c_conj(cplx a) { cplx r = {a.re, -a.im}; return r; }

/* Table of exp(-j*2*pi*e/len) for e = 0..len-1, cos/sin evaluated in double. */
static cplx *twiddle_table(int64_t len)
{
    cplx *t = (cplx *)malloc((size_t)len * sizeof(cplx));
    if (!t)
        return NULL;
    for (int64_t e = 0; e < len; ++e) {
        double a = 2.0 * M_PI * (double)e / (double)len;
        t[e].re = cos(a);
        t[e].im = -sin(a);
    }
    return t;
}

static int bad_order(int m) { return m < 1 || m > MRO_MAX_M; }

/* ---------------------------------------------------------------------------
 * Direct sums, one level.  y receives the N values of level i.
 * ------------------------------------------------------------------------ */
static int level_direct(int m, int i, const cplx *x, cplx *y)
{
    const int64_t n_all = (int64_t)1 << m;
    const int64_t len = (int64_t)1 << i;
    const int64_t mask = len - 1;
    cplx *tw = twiddle_table(len);
    if (!tw)
        return -2;
    for (int64_t base = 0; base < n_all; base += len) {
        for (int64_t k = 0; k < len; ++k) {
            cplx acc = {0.0, 0.0};
            for (int64_t n = 0; n < len; ++n)
                acc = c_add(acc, c_mul(x[base + n], tw[(n * k) & mask]));
            y[base + k] = acc;
        }
    }
    free(tw);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Recursive radix-2 DIT FFT:  out[k] = sum_q in[q*stride] * exp(-j 2 pi q k / n)
 * tw holds exp(-j*2*pi*e/top) for the top size; tws = top / n.
 * ------------------------------------------------------------------------ */
static void fft_rec(const cplx *in, int64_t stride, cplx *out, int64_t n,
                    const cplx *tw, int64_t tws)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    const int64_t h = n / 2;
    fft_rec(in, 2 * stride, out, h, tw, 2 * tws);          /* even samples */
    fft_rec(in + stride, 2 * stride, out + h, h, tw, 2 * tws); /* odd samples */
    for (int64_t k = 0; k < h; ++k) {
        cplx e = out[k];
        cplx o = c_mul(out[k + h], tw[k * tws]);
        out[k] = c_add(e, o);
        out[k + h] = c_sub(e, o);
    }
}

static int level_fft(int m, int i, const cplx *x, cplx *y)
{
    const int64_t n_all = (int64_t)1 << m;
    const int64_t len = (int64_t)1 << i;
    cplx *tw = twiddle_table(len);
    if (!tw)
        return -2;
    for (int64_t base = 0; base < n_all; base += len)
        fft_rec(x + base, 1, y + base, len, tw, 1);
    free(tw);
    return 0;
}

/* Inverse (conjugate) per-window transform of one level, added into gx. */
static int level_adjoint_direct(int m, int i, const cplx *gy, cplx *gx)
{
    const int64_t n_all = (int64_t)1 << m;
    const int64_t len = (int64_t)1 << i;
    const int64_t mask = len - 1;
    cplx *tw = twiddle_table(len);
    if (!tw)
        return -2;
    for (int64_t base = 0; base < n_all; base += len) {
        for (int64_t n = 0; n < len; ++n) {
            cplx acc = {0.0, 0.0};
            for (int64_t k = 0; k < len; ++k)
                acc = c_add(acc, c_mul(gy[base + k], c_conj(tw[(n * k) & mask])));
            gx[base + n] = c_add(gx[base + n], acc);
        }
    }
    free(tw);
    return 0;
}

/* conj(FFT(conj(v))) is the unnormalised inverse DFT. */
static int level_adjoint_fft(int m, int i, const cplx *gy, cplx *gx)
{
    const int64_t n_all = (int64_t)1 << m;
    const int64_t len = (int64_t)1 << i;
    cplx *tw = twiddle_table(len);
    cplx *a = (cplx *)malloc((size_t)len * sizeof(cplx));
    cplx *b = (cplx *)malloc((size_t)len * sizeof(cplx));
    if (!tw || !a || !b) {
        free(tw);
        free(a);
        free(b);
        return -2;
    }
    for (int64_t base = 0; base < n_all; base += len) {
        for (int64_t k = 0; k < len; ++k)
            a[k] = c_conj(gy[base + k]);
        fft_rec(a, 1, b, len, tw, 1);
        for (int64_t n = 0; n < len; ++n)
            gx[base + n] = c_add(gx[base + n], c_conj(b[n]));
    }
    free(tw);
    free(a);
    free(b);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Public entry points
 * ------------------------------------------------------------------------ */

/* method: 0 = direct sums, 1 = recursive FFT, -1 = direct for N <= 2^12 else FFT. */
static int pick(int m, int method) { return method >= 0 ? method : (m <= 12 ? 0 : 1); }

/* One level i of one signal: x has N = 2^m complex values, y receives N. */
int mro_forward_level(int m, int i, const double *x, double *y, int method)
{
    if (bad_order(m) || i < 1 || i > m || !x || !y)
        return -1;
    return pick(m, method) == 0 ? level_direct(m, i, (const cplx *)x, (cplx *)y)
                                : level_fft(m, i, (const cplx *)x, (cplx *)y);
}

/* All m levels of one signal: y receives m*N values, level 1 first. */
int mro_forward(int m, const double *x, double *y, int method)
{
    if (bad_order(m) || !x || !y)
        return -1;
    const int64_t n_all = (int64_t)1 << m;
    for (int i = 1; i <= m; ++i) {
        int rc = mro_forward_level(m, i, x, y + 2 * (size_t)(i - 1) * (size_t)n_all, method);
        if (rc)
            return rc;
    }
    return 0;
}

/* A single output Y^(i)[w*2^i + k], by its direct sum. */
int mro_forward_bin(int m, int i, int64_t w, int64_t k, const double *x, double *out)
{
    if (bad_order(m) || i < 1 || i > m || !x || !out)
        return -1;
    const int64_t len = (int64_t)1 << i;
    if (w < 0 || w >= ((int64_t)1 << (m - i)) || k < 0 || k >= len)
        return -1;
    const cplx *xs = (const cplx *)x + w * len;
    const int64_t mask = len - 1;
    cplx acc = {0.0, 0.0};
    for (int64_t n = 0; n < len; ++n) {
        double a = 2.0 * M_PI * (double)((n * k) & mask) / (double)len;
        cplx t = {cos(a), -sin(a)};
        acc = c_add(acc, c_mul(xs[n], t));
    }
    out[0] = acc.re;
    out[1] = acc.im;
    return 0;
}

/* gx (N values) = sum over levels of the per-window conjugate transforms of gy (m*N). */
int mro_adjoint(int m, const double *gy, double *gx, int method)
{
    if (bad_order(m) || !gy || !gx)
        return -1;
    const int64_t n_all = (int64_t)1 << m;
    memset(gx, 0, (size_t)n_all * sizeof(cplx));
    for (int i = 1; i <= m; ++i) {
        const cplx *g = (const cplx *)gy + (size_t)(i - 1) * (size_t)n_all;
        int rc = pick(m, method) == 0 ? level_adjoint_direct(m, i, g, (cplx *)gx)
                                      : level_adjoint_fft(m, i, g, (cplx *)gx);
        if (rc)
            return rc;
    }
    return 0;
}

/* A single adjoint output gx[p], by its direct double sum over levels and bins. */
int mro_adjoint_point(int m, int64_t p, const double *gy, double *out)
{
    if (bad_order(m) || !gy || !out)
        return -1;
    const int64_t n_all = (int64_t)1 << m;
    if (p < 0 || p >= n_all)
        return -1;
    cplx acc = {0.0, 0.0};
    for (int i = 1; i <= m; ++i) {
        const int64_t len = (int64_t)1 << i;
        const int64_t base = (p / len) * len;
        const int64_t n = p - base;
        const cplx *g = (const cplx *)gy + (size_t)(i - 1) * (size_t)n_all + base;
        for (int64_t k = 0; k < len; ++k) {
            double a = 2.0 * M_PI * (double)((n * k) & (len - 1)) / (double)len;
            cplx t = {cos(a), sin(a)};
            acc = c_add(acc, c_mul(g[k], t));
        }
    }
    out[0] = acc.re;
    out[1] = acc.im;
    return 0;
}

/* Spectral loss of one real pair (x, z), both N doubles.  num_den receives
 * [m][2] = (num_i, den_i); *loss receives L. */
int mro_spectral_loss(int m, const double *x, const double *z, double *num_den,
                      double *loss, int method)
{
    if (bad_order(m) || !x || !z || !num_den || !loss)
        return -1;
    const int64_t n_all = (int64_t)1 << m;
    cplx *cx = (cplx *)calloc((size_t)n_all, sizeof(cplx));
    cplx *cz = (cplx *)calloc((size_t)n_all, sizeof(cplx));
    cplx *yx = (cplx *)malloc((size_t)n_all * sizeof(cplx));
    cplx *yz = (cplx *)malloc((size_t)n_all * sizeof(cplx));
    int rc = 0;
    if (!cx || !cz || !yx || !yz) {
        rc = -2;
        goto done;
    }
    for (int64_t n = 0; n < n_all; ++n) {
        cx[n].re = x[n];
        cz[n].re = z[n];
    }
    double total = 0.0;
    for (int i = 1; i <= m; ++i) {
        rc = mro_forward_level(m, i, (const double *)cx, (double *)yx, method);
        if (!rc)
            rc = mro_forward_level(m, i, (const double *)cz, (double *)yz, method);
        if (rc)
            goto done;
        double num = 0.0, den = 0.0;
        for (int64_t n = 0; n < n_all; ++n) {
            cplx d = c_sub(yx[n], yz[n]);
            num += d.re * d.re + d.im * d.im;
            den += yz[n].re * yz[n].re + yz[n].im * yz[n].im;
        }
        num_den[2 * (i - 1)] = num;
        num_den[2 * (i - 1) + 1] = den;
        total += num / den;
    }
    *loss = total / (double)m;
done:
    free(cx);
    free(cz);
    free(yx);
    free(yz);
    return rc;
}

/* Gradient of the spectral loss w.r.t. real x, scaled by gL; gx receives N doubles.
 * num_den must hold the den_i values from mro_spectral_loss. */
int mro_spectral_loss_grad(int m, const double *x, const double *z, const double *num_den,
                           double gL, double *gx, int method)
{
    if (bad_order(m) || !x || !z || !num_den || !gx)
        return -1;
    const int64_t n_all = (int64_t)1 << m;
    cplx *cx = (cplx *)calloc((size_t)n_all, sizeof(cplx));
    cplx *cz = (cplx *)calloc((size_t)n_all, sizeof(cplx));
    cplx *yx = (cplx *)malloc((size_t)n_all * sizeof(cplx));
    cplx *yz = (cplx *)malloc((size_t)n_all * sizeof(cplx));
    cplx *acc = (cplx *)calloc((size_t)n_all, sizeof(cplx));
    int rc = 0;
    if (!cx || !cz || !yx || !yz || !acc) {
        rc = -2;
        goto done;
    }
    for (int64_t n = 0; n < n_all; ++n) {
        cx[n].re = x[n];
        cz[n].re = z[n];
    }
    for (int i = 1; i <= m; ++i) {
        rc = mro_forward_level(m, i, (const double *)cx, (double *)yx, method);
        if (!rc)
            rc = mro_forward_level(m, i, (const double *)cz, (double *)yz, method);
        if (rc)
            goto done;
        const double s = gL * 2.0 / ((double)m * num_den[2 * (i - 1) + 1]);
        for (int64_t n = 0; n < n_all; ++n) {
            cplx d = c_sub(yx[n], yz[n]);
            yx[n].re = s * d.re;
            yx[n].im = s * d.im;
        }
        rc = pick(m, method) == 0 ? level_adjoint_direct(m, i, yx, acc)
                                  : level_adjoint_fft(m, i, yx, acc);
        if (rc)
            goto done;
    }
    for (int64_t n = 0; n < n_all; ++n)
        gx[n] = acc[n].re;
done:
    free(cx);
    free(cz);
    free(yx);
    free(yz);
    free(acc);
    return rc;
}

int mro_max_order(void) { return MRO_MAX_M; }
