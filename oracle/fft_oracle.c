/*
 * FP64 CPU oracle for batched 1D complex-to-complex DFTs.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; it is the independent
 * definition the GPU results are compared against.
 *
 * What it computes (paper section "Fast Fourier Transform"):
 *   forward, Eq. (dft):   X_k = sum_n x_n w_N^{kn},  w_N = exp(-2 pi i / N)
 *   inverse, Eq. (idft):  x_k = (1/N) sum_n X_n w_N^{-kn}
 * evaluated with the recursive radix-2 decimation-in-time split of
 * Eq. (radix2): X_k = E_k + w_N^k O_k and X_{k+N/2} = E_k - w_N^k O_k for
 * k in [0, N/2), where E and O are the half-length DFTs of the even- and
 * odd-indexed samples.  Twiddles come straight from libm cos/sin in double
 * precision.  No blocking, no tables, no reordering beyond the recursion.
 *
 * Generalised entry point: fft(sign s, scale c) maps x to
 *   y_k = c * sum_n x_n exp(s * 2 pi i k n / N).
 * forward = (s=-1, c=1), inverse = (s=+1, c=1/N), and the adjoint of the
 * map (s, c) is (-s, c) for real c.
 *
 * Layout: interleaved (re, im) doubles, transform b at element offset b*n
 * (batched) or offsets[b] (ragged).  Work is split over POSIX threads by
 * transform, which changes nothing in the arithmetic of any one transform.
 *
 * Build with -DORACLE_MUTANT=k (k >= 1) to plant one deliberate mistake;
 * the test-suite does that to show its pins catch each of them.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

static const double TWO_PI = 6.283185307179586476925286766559;

/* Radix-2 DIT of Eq. (radix2): DFT of the n samples x[0], x[xs], x[2xs], ...
 * (x interleaved re/im, xs in complex elements) written to X[0..n).  E goes
 * to the first half of X, O to the second half, then the butterflies
 * combine them in place. */
static void rec(const double *x, int64_t xs, double *X, int64_t n, int sign)
{
    if (n == 1) {
        X[0] = x[0];
        X[1] = x[1];
        return;
    }
    const int64_t h = n / 2;
#if ORACLE_MUTANT == 4
    /* mutant: even and odd halves swapped */
    rec(x + 2 * xs, 2 * xs, X, h, sign);
    rec(x, 2 * xs, X + 2 * h, h, sign);
#else
    rec(x, 2 * xs, X, h, sign);              /* E_k: even-indexed samples */
    rec(x + 2 * xs, 2 * xs, X + 2 * h, h, sign); /* O_k: odd-indexed samples */
#endif
    for (int64_t k = 0; k < h; k++) {
#if ORACLE_MUTANT == 1
        const double ang = TWO_PI * (double)k / (double)n * (double)(-sign); /* wrong sign */
#elif ORACLE_MUTANT == 2
        const double ang = TWO_PI * (double)k / (double)h * (double)sign; /* wrong period */
#elif ORACLE_MUTANT == 5
        const double ang = TWO_PI * (double)(k + 1) / (double)n * (double)sign; /* index off by one */
#else
        const double ang = TWO_PI * (double)k / (double)n * (double)sign;
#endif
        const double wr = cos(ang), wi = sin(ang);
        double *e = X + 2 * k;
        double *o = X + 2 * (k + h);
        const double er = e[0], ei = e[1];
        const double tr = wr * o[0] - wi * o[1];
#if ORACLE_MUTANT == 7
        const double ti = wr * o[1] - wi * o[0]; /* conjugated product */
#else
        const double ti = wr * o[1] + wi * o[0];
#endif
        e[0] = er + tr;
        e[1] = ei + ti;
#if ORACLE_MUTANT == 3
        o[0] = er + tr; /* dropped minus in the lower butterfly output */
        o[1] = ei + ti;
#else
        o[0] = er - tr;
        o[1] = ei - ti;
#endif
    }
}

static int is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }

/* One transform: y = scale * DFT_sign(x), n complex elements. */
static void one(const double *x, double *y, int64_t n, int sign, double scale)
{
    rec(x, 1, y, n, sign);
#if ORACLE_MUTANT == 6
    (void)scale; /* mutant: normalisation dropped */
#else
    if (scale != 1.0)
        for (int64_t i = 0; i < 2 * n; i++)
            y[i] *= scale;
#endif
}

typedef struct {
    const double *in;
    double *out;
    const int64_t *offsets; /* NULL: uniform batch with stride n */
    int64_t n;              /* uniform length (batched form) */
    int64_t lo, hi;         /* transform range for this worker */
    int sign;
    int scale_mode;         /* 0: scale by `scale`; 1: scale by 1/len */
    double scale;
} job_t;

static void *worker(void *arg)
{
    const job_t *j = (const job_t *)arg;
    for (int64_t b = j->lo; b < j->hi; b++) {
        int64_t off, len;
        if (j->offsets) {
            off = j->offsets[b];
            len = j->offsets[b + 1] - off;
        } else {
            off = b * j->n;
            len = j->n;
        }
        const double c = j->scale_mode ? 1.0 / (double)len : j->scale;
        one(j->in + 2 * off, j->out + 2 * off, len, j->sign, c);
    }
    return NULL;
}

static int run(const double *in, double *out, const int64_t *offsets, int64_t n,
               int64_t count, int sign, int scale_mode, double scale, int nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    if ((int64_t)nthreads > count)
        nthreads = count > 0 ? (int)count : 1;
    pthread_t th[256];
    job_t jobs[256];
    for (int t = 0; t < nthreads; t++) {
        jobs[t].in = in;
        jobs[t].out = out;
        jobs[t].offsets = offsets;
        jobs[t].n = n;
        jobs[t].lo = count * t / nthreads;
        jobs[t].hi = count * (t + 1) / nthreads;
        jobs[t].sign = sign;
        jobs[t].scale_mode = scale_mode;
        jobs[t].scale = scale;
    }
    int started = 0;
    for (int t = 1; t < nthreads; t++) {
        if (pthread_create(&th[t], NULL, worker, &jobs[t]) != 0)
            break;
        started = t;
    }
    worker(&jobs[0]);
    for (int t = 1; t <= started; t++)
        pthread_join(th[t], NULL);
    /* any worker that failed to start runs here */
    for (int t = started + 1; t < nthreads; t++)
        worker(&jobs[t]);
    return 0;
}

/* y[b] = scale * DFT_sign(x[b]) for b < batch; n a power of two >= 1.
 * Returns 0, or -1 for an invalid argument. */
int oracle_fft(const double *in, double *out, int64_t n, int64_t batch, int sign,
               double scale, int nthreads)
{
    if (!in || !out || !is_pow2(n) || batch < 0 || (sign != 1 && sign != -1))
        return -1;
    return run(in, out, NULL, n, batch, sign, 0, scale, nthreads);
}

/* Ragged form: transform b occupies elements [offsets[b], offsets[b+1]) of
 * both in and out.  scale_mode 0 multiplies by `scale`; scale_mode 1 by
 * 1/length of each transform (the inverse of Eq. (idft) per segment). */
int oracle_fft_ragged(const double *in, double *out, const int64_t *offsets,
                      int64_t count, int sign, int scale_mode, double scale,
                      int nthreads)
{
    if (!in || !out || !offsets || count < 0 || (sign != 1 && sign != -1))
        return -1;
    for (int64_t b = 0; b < count; b++)
        if (!is_pow2(offsets[b + 1] - offsets[b]))
            return -1;
    return run(in, out, offsets, 0, count, sign, scale_mode, scale, nthreads);
}

int oracle_mutant_id(void) { return ORACLE_MUTANT; }
