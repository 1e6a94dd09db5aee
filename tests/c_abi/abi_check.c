/*
 * Standalone use of the C ABI: no Python, no torch.  Device memory from
 * hipMalloc, a non-default stream, a batched forward and inverse FFT, a
 * real-input plan and the error paths; results against direct DFT sums in
 * double precision.  Prints "abi_check ok" and exits 0 on success.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mifft.h"

#define CHECK(cond, ...)                     \
    do {                                     \
        if (!(cond)) {                       \
            fprintf(stderr, __VA_ARGS__);    \
            fprintf(stderr, "\n");           \
            return 1;                        \
        }                                    \
    } while (0)

/* deterministic input in [-1, 1) */
static float val(long i) { return (float)((i * 2654435761UL) % 2001) / 1000.0f - 1.0f; }

/* relative L2 error of one transform's bins against the direct sum of
 * Eq. (dft) with sign s and scale c, in double precision */
static double dft_err(const float* x, const float* y, int n, int s, double c, int nbins, int real_in)
{
    double num = 0, den = 0;
    for (int k = 0; k < nbins; k++) {
        double re = 0, im = 0;
        for (int j = 0; j < n; j++) {
            const double a = 2.0 * 3.14159265358979323846 * (double)(((long)k * j) % n) / n * s;
            const double xr = real_in ? x[j] : x[2 * j], xi = real_in ? 0.0 : x[2 * j + 1];
            re += xr * cos(a) - xi * sin(a);
            im += xr * sin(a) + xi * cos(a);
        }
        re *= c;
        im *= c;
        num += (y[2 * k] - re) * (y[2 * k] - re) + (y[2 * k + 1] - im) * (y[2 * k + 1] - im);
        den += re * re + im * im;
    }
    return sqrt(num / den);
}

int main(void)
{
    const int n = 2048, batch = 37;
    const size_t bytes = sizeof(float) * 2 * (size_t)n * batch;
    float* hx = (float*)malloc(bytes);
    float* hy = (float*)malloc(bytes);
    for (long i = 0; i < 2L * n * batch; i++)
        hx[i] = val(i);
    void *dx, *dy;
    hipStream_t st;
    CHECK(hipMalloc(&dx, bytes) == hipSuccess && hipMalloc(&dy, bytes) == hipSuccess, "hipMalloc failed");
    CHECK(hipStreamCreate(&st) == hipSuccess, "hipStreamCreate failed");
    CHECK(hipMemcpy(dx, hx, bytes, hipMemcpyHostToDevice) == hipSuccess, "copy in failed");

    /* argument errors are reported before any device work */
    CHECK(fft_plan_create(12, 1, -1, FFT_C32) == NULL && fft_last_error() == FFT_EINVAL_N, "bad n accepted");
    CHECK(fft_plan_create(256, 0, -1, FFT_C32) == NULL && fft_last_error() == FFT_EINVAL_BATCH, "bad batch");

    /* forward */
    fft_plan p = fft_plan_create(n, batch, -1, FFT_C32);
    CHECK(p != NULL, "fft_plan_create: %s", fft_last_error_string());
    CHECK(fft_execute(p, dx, dx, st) == FFT_EOVERLAP, "in-place call not rejected");
    CHECK(fft_execute(p, dx, dy, st) == FFT_OK, "fft_execute: %s", fft_last_error_string());
    CHECK(hipStreamSynchronize(st) == hipSuccess, "sync failed");
    CHECK(hipMemcpy(hy, dy, bytes, hipMemcpyDeviceToHost) == hipSuccess, "copy out failed");
    for (int b = 0; b < batch; b += 12) {
        const double e = dft_err(hx + 2L * n * b, hy + 2L * n * b, n, -1, 1.0, 64, 0);
        CHECK(e <= 1e-5, "forward transform %d: rel L2 %.3e", b, e);
    }
    fft_plan_desc d;
    CHECK(fft_plan_describe(p, &d) == FFT_OK && d.n == n && d.batch == batch, "describe failed");

    /* inverse of the spectrum gives the input back */
    fft_plan q = fft_plan_create(n, batch, +1, FFT_C32);
    CHECK(q != NULL, "inverse plan: %s", fft_last_error_string());
    CHECK(fft_execute(q, dy, dx, st) == FFT_OK, "inverse execute: %s", fft_last_error_string());
    CHECK(hipStreamSynchronize(st) == hipSuccess, "sync failed");
    float* hz = (float*)malloc(bytes);
    CHECK(hipMemcpy(hz, dx, bytes, hipMemcpyDeviceToHost) == hipSuccess, "copy out failed");
    double num = 0, den = 0;
    for (long i = 0; i < 2L * n * batch; i++) {
        num += (hz[i] - hx[i]) * (double)(hz[i] - hx[i]);
        den += (double)hx[i] * hx[i];
    }
    CHECK(sqrt(num / den) <= 2e-5, "round trip: rel L2 %.3e", sqrt(num / den));

    /* real input: n reals -> n/2 + 1 bins */
    const int nr = 1024, br = 5;
    float* hr = (float*)malloc(sizeof(float) * nr * br);
    float* hb = (float*)malloc(sizeof(float) * 2 * (nr / 2 + 1) * br);
    for (long i = 0; i < (long)nr * br; i++)
        hr[i] = val(7 * i + 3);
    CHECK(hipMemcpy(dx, hr, sizeof(float) * nr * br, hipMemcpyHostToDevice) == hipSuccess, "copy in failed");
    fft_plan r = fft_plan_create(nr, br, -1, FFT_R32);
    CHECK(r != NULL, "real plan: %s", fft_last_error_string());
    CHECK(fft_execute(r, dx, dy, st) == FFT_OK, "real execute: %s", fft_last_error_string());
    CHECK(hipStreamSynchronize(st) == hipSuccess, "sync failed");
    CHECK(hipMemcpy(hb, dy, sizeof(float) * 2 * (nr / 2 + 1) * br, hipMemcpyDeviceToHost) == hipSuccess,
          "copy out failed");
    for (int b = 0; b < br; b++) {
        const double e = dft_err(hr + (long)nr * b, hb + 2L * (nr / 2 + 1) * b, nr, -1, 1.0, nr / 2 + 1, 1);
        CHECK(e <= 1e-5, "real transform %d: rel L2 %.3e", b, e);
    }

    fft_plan_destroy(p);
    fft_plan_destroy(q);
    fft_plan_destroy(r);
    fft_plan_destroy(NULL);
    hipStreamDestroy(st);
    hipFree(dx);
    hipFree(dy);
    printf("abi_check ok (%s)\n", fft_version());
    free(hx);
    free(hy);
    free(hz);
    free(hr);
    free(hb);
    return 0;
}
