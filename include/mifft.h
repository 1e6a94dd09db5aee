/*
 * mifft -- batched 1D complex-to-complex FFTs of power-of-two length on
 * AMD Instinct MI355X (gfx950).  C ABI.
 *
 * What is computed (paper section "Fast Fourier Transform"):
 *   forward, Eq. (dft):   X_k = sum_{n<N} x_n w_N^{kn},        w_N = exp(-2 pi i / N)
 *   inverse, Eq. (idft):  x_k = (1/N) sum_{n<N} X_n w_N^{-kn}
 * for every transform of a batch, by Cooley-Tukey / Stockham passes of
 * radix 2..16 (section "Implementation": radix-2/4/8 stages selected on
 * the host from N; single precision, complex-to-complex, out of place,
 * N up to 2^11), extended here to 2^14 in one pass and to 2^20 by the
 * four-step split.  Both input and output are in natural order.
 *
 * Real input (FFT_R32; the paper's inputs may be real- or complex-valued,
 * section "Fast Fourier Transform"): a real sequence has a Hermitian
 * spectrum, X_{n-k} = conj(X_k), so bins 0..n/2 determine it.
 *   forward (sign -1):  X_k = sum_{j<n} x_j w_n^{jk},  k = 0..n/2
 *   inverse (sign +1):  x_j = (1/n) sum_{k<n} X~_k w_n^{-jk},  X~ the
 *                       Hermitian extension of X_0..X_{n/2}, with the
 *                       imaginary parts of X_0 and X_{n/2} ignored
 * computed as one length-n/2 complex transform of z_j = x_{2j} + i x_{2j+1}
 * plus the even/odd split of Eq. (radix2), fused into one kernel.
 *
 * Conventions shared by every entry point
 *   - Data are interleaved (re, im) pairs.  FFT_C32: two float32 per element
 *     (8 bytes, the layout of std::complex<float> / torch.complex64).
 *     FFT_C16 / FFT_CBF16: two float16 / bfloat16 per element (4 bytes).
 *   - Transform b of a batched plan occupies elements [b*n, (b+1)*n).
 *     FFT_R32: the real side holds n float32 values per transform
 *     (floats [b*n, (b+1)*n)), the spectrum side n/2 + 1 complex float32
 *     bins per transform (bins [b*(n/2+1), (b+1)*(n/2+1))).
 *   - `in` and `out` are device pointers owned by the caller, aligned to
 *     their element (FFT_C32 and complex bins: 8 bytes; FFT_C16 / FFT_CBF16
 *     pairs and FFT_R32 reals: 4 bytes; any offset view of a tensor of that
 *     element type qualifies), and must not overlap (out of place only).
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Every
 *     execute call only enqueues work: it allocates nothing, synchronises
 *     nothing and copies nothing, so it may be captured into a hipGraph.
 *   - Status codes below; 0 is success.  The last status and a message
 *     (including the HIP error string where HIP failed) are kept per host
 *     thread: fft_last_error / fft_last_error_string.  Arguments are
 *     checked before any HIP call is made.  Faults inside a kernel are
 *     asynchronous and surface at the caller's next synchronisation.
 *   - A plan is bound to the HIP device that was current when it was
 *     created and is immutable afterwards, so executes of one plan on
 *     several streams may run concurrently (plan-owned workspaces are the
 *     exception; see the plans that have one).
 */
#ifndef MIFFT_H
#define MIFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mifft_plan_s *fft_plan;

/* element types (interleaved complex) */
enum {
    FFT_C32 = 0,   /* float32 re, im  */
    FFT_C16 = 1,   /* float16 re, im  */
    FFT_CBF16 = 2, /* bfloat16 re, im */
    FFT_R32 = 3    /* real input: float32 reals <-> float32 (re, im) bins   */
};

/* status codes */
enum {
    FFT_OK = 0,
    FFT_EINVAL_N = 1,       /* n not a supported power of two (see create)     */
    FFT_EINVAL_BATCH = 2,   /* batch < 1, or the batch does not fit one launch  */
    FFT_EINVAL_SIGN = 3,    /* sign not -1 or +1                               */
    FFT_EINVAL_DTYPE = 4,   /* unknown dtype, or dtype not valid for the call   */
    FFT_ENULL = 5,          /* a required pointer or plan is NULL               */
    FFT_EOVERLAP = 6,       /* input and output byte ranges overlap             */
    FFT_EINVAL_OFFSETS = 7, /* ragged offsets malformed                         */
    FFT_EHIP = 8,           /* a HIP call failed (message has the HIP string)   */
    FFT_ENOMEM = 9,         /* host or device allocation failed                 */
    FFT_EINVAL_CONFIG = 10, /* requested kernel variant does not exist          */
    FFT_EALIGN = 11,        /* a buffer not aligned to its element (complex64:
                               8 bytes; 16-bit pairs, float32: 4 bytes)         */
    FFT_EDEVICE = 12,       /* current device is not a gfx950 GPU, or plan used
                               while another device is current                  */
    FFT_ECAPTURE = 13       /* plan creation while a stream capture is active   */
};

/* Description of what a plan launches (fft_plan_describe / fft_plan_query). */
typedef struct {
    int64_t n;          /* transform length (batched plans), 0 for ragged     */
    int64_t batch;      /* transforms per execute                             */
    int sign;           /* -1 forward (Eq. (dft)), +1 inverse (Eq. (idft))    */
    int dtype;          /* FFT_C32 / FFT_C16 / FFT_CBF16 / FFT_R32             */
    float scale;        /* output scale: 1 (forward) or 1/n (inverse)         */
    int ept;            /* complex elements held per thread (FFT_R32: of the
                           half-length transform, as npasses and radices)  */
    int wg;             /* threads per workgroup                              */
    int transforms_per_wg;
    int64_t grid;       /* workgroups per execute (persistent kernels: those
                           resident at once, each walking the batch)     */
    int npasses;        /* Stockham passes                                    */
    int radices[8];     /* radix of each pass, first to last                  */
    int lds_bytes;      /* LDS per workgroup                                  */
    int kind;           /* 0 batched, 1 ragged, 2 multidimensional            */
    int64_t tiles;      /* ragged: work tiles                                 */
    int variant;        /* kernel family: 0 one transform group per
                           workgroup; 1..4 twiddle-row kernels (1, 2: one
                           group per workgroup, twiddles kept / re-read;
                           3, 4: persistent with next-group prefetch);
                           5..8 as 1..4 with wavefront-local exchanges
                           (transforms of at most 64 threads); 9 the
                           four-step split (n > 2048); 10 the single-pass
                           2D kernel (multidimensional plans); 11 one
                           transform per thread (n <= 16) with the block
                           staged through LDS in 16-byte vectors; 12 the
                           same staging for n = 32, 64 (several threads
                           per transform, wavefront-local exchanges);
                           13 the single-pass 3D kernel (multidimensional
                           plans)                                      */
    int ept_by_log2n[12]; /* ragged: elements per thread used for length 2^L */
    int rank;           /* multidimensional plans: number of axes (else 0)   */
    int64_t dims[3];    /* multidimensional plans: axis lengths, first to last */
} fft_plan_desc;

/*
 * Create a plan for `batch` transforms of length n.
 *   n      power of two.  FFT_C32: [2, 2^20].  Lengths up to 2^14 run one
 *          single-pass kernel (up to 2^11, the paper's range, section
 *          "Implementation", several transforms per workgroup; above, one
 *          transform per workgroup of up to 1024 threads and 160 KiB of
 *          LDS); 2^15 .. 2^20 (the paper's future work, section
 *          "Conclusions") use the four-step split N = N1 N2: a column pass
 *          with the w_N^{n2 k1} twiddles, then an in-place row pass in
 *          `out` (two kernels on the stream).  FFT_C16 / FFT_CBF16: [2, 2048]
 *          (2048: radix-16 passes on MFMA; below: the FP32 passes with
 *          16-bit storage).
 *          FFT_R32: [2, 2^21]; up to 2^15 one fused kernel per
 *          execute, above it the half-length four-step transform plus a
 *          split pass through a plan-owned workspace of n/2 complex values
 *          per transform (allocated here; executes of one such plan must
 *          not overlap in time).
 *   batch  >= 1.
 *   sign   -1: forward transform Eq. (dft), scale 1.
 *          +1: inverse transform Eq. (idft), scale 1/n.
 *          FFT_R32: -1 maps n reals to n/2 + 1 bins (R2C), +1 maps
 *          n/2 + 1 bins to n reals with the 1/n (C2R).
 *   dtype  FFT_C32, FFT_C16, FFT_CBF16 or FFT_R32.
 * Binds to the current HIP device, allocates and fills the plan's twiddle
 * table (blocking, on the legacy default stream).  Returns NULL on error;
 * see fft_last_error().  The kernel variant (elements per thread and
 * workgroup size) comes from the built-in tuned table, or from the file
 * named by the environment variable MIFFT_TUNE_TABLE if set.
 * Plan creation (this and every other fft_plan_create_* call) allocates and
 * synchronises, so it must not run while a stream capture is active: it
 * returns NULL with FFT_ECAPTURE when HIP reports one.  Create plans before
 * capturing; the executes are what a graph holds.
 * Accuracy (per-transform relative L2 against the exact DFT of the stored
 * input): FP32 about 1e-7 (bar 1e-5).  FP16 / BF16 at N = 2048: about
 * 4e-4 (FP16) and 1.8e-3 (BF16), bar 3e-3.  Below 2048 the FP16/BF16 error is
 * the rounding of the stored output itself, bounded by 2^-11 (FP16) and
 * 2^-8 = 3.9e-3 (BF16, 8 significant bits): a BF16 transform of few points
 * can exceed 3e-3 (3.8e-3 measured at N = 2).
 */
fft_plan fft_plan_create(int64_t n, int64_t batch, int sign, int dtype);

/*
 * As fft_plan_create, forcing the kernel variant: `ept` complex elements
 * per thread (2, 4, 8 or 16), `wg` threads per workgroup (64 .. 1024) and
 * the kernel family `variant` (0..8, 11 or 12, see fft_plan_desc.variant; 9 = the
 * four-step split, n > 2048).  FFT_C32 and FFT_R32 only; for FFT_R32 ept
 * and wg describe the half-length transform (ept 1..16) and variant is 0
 * (a whole half-length transform per thread), 2, 3, 6 or 7.  Used by the
 * autotuner.  FFT_EINVAL_CONFIG if that variant is not compiled in.
 */
fft_plan fft_plan_create_config(int64_t n, int64_t batch, int sign, int dtype, int ept, int wg, int variant);

/*
 * Ragged batch: `count` transforms of mixed power-of-two lengths packed
 * back to back.  `offsets` is a HOST array of count+1 int64 values, copied
 * into the plan: offsets[0] = 0, and each length offsets[b+1]-offsets[b]
 * is a power of two in [2, 2048]; transform b occupies elements
 * [offsets[b], offsets[b+1]) of both input and output.  Every execute is
 * one kernel launch over length-grouped work tiles (largest transforms
 * first), dealt to its workgroups in a fixed order; the launch keeps no
 * device state between executes, so it can be captured into a hipGraph
 * and executes of one plan on several streams may overlap.
 * Only FFT_C32.  sign as for fft_plan_create; the inverse scales each
 * transform by 1/its length.
 */
fft_plan fft_plan_create_ragged(int64_t count, const int64_t *offsets, int sign, int dtype);

/*
 * As fft_plan_create_ragged with the per-length kernel variant forced:
 * ept_by_log2n[L] (L = 1..11; entries 0 ignored) gives the elements per
 * thread used for length 2^L, `wg` the workgroup size of the launch and
 * `ctas_per_cu` how many workgroups per compute unit the launch holds
 * (0: as many as fit; the grid is never larger than the tile count, and
 * workgroups loop over the tiles when it is smaller).  wg must be 64, 128
 * or 256 (0: the built-in choice).  Used by the autotuner.
 */
fft_plan fft_plan_create_ragged_config(int64_t count, const int64_t *offsets, int sign, int dtype,
                                       const int *ept_by_log2n, int wg, int ctas_per_cu);

/*
 * Multidimensional transforms (the paper's future work, section
 * "Conclusions"): `batch` arrays of shape dims[0] x ... x dims[rank-1],
 * row-major (the last axis contiguous), each transformed by
 *   X[k] = s * sum_n x[n] prod_a exp(sign 2 pi i k_a n_a / dims[a]),
 * s = 1 (sign -1) or 1/prod(dims) (sign +1).  The kernel factors over the
 * axes, so the plan runs the 1D batched kernels over the last axis
 * (in -> out) and then one in-place pass per remaining axis over `out`,
 * each over tiles of transforms adjacent in memory.  A 2D array that fits
 * one workgroup's LDS (at most 16384 points, both axes >= 16 points per
 * thread group, e.g. 128 x 128) instead runs one kernel: rows, a
 * transpose through LDS and columns, one pass over HBM
 * (fft_plan_desc.variant 10).  A 3D array that fits one workgroup's LDS
 * (at most 16384 points, every axis at least 4) runs one kernel as well:
 * the three axes with two transposes through LDS, one pass over HBM
 * (variant 13).  Otherwise a 3D plan whose last two axes form a single-pass
 * 2D array runs that kernel over them, then one pass for its first axis.
 *   rank   1, 2 or 3 (rank 1 is fft_plan_create).
 *   dims   host array of `rank` powers of two: the last in [2, 2^20], the
 *          others in [2, 2048].  Copied into the plan.
 *   dtype  FFT_C32 only.
 * fft_execute / fft_execute_adjoint apply the transform / its adjoint
 * (opposite sign, same scale) with n = prod(dims) elements per array.
 * FFT_EINVAL_N for a bad rank or dims, FFT_ENULL for NULL dims.
 */
fft_plan fft_plan_create_nd(int rank, const int64_t *dims, int64_t batch, int sign, int dtype);

/*
 * Apply the plan's transform: out = plan(in).  Asynchronous on `stream`.
 * Byte ranges: n*batch*elem_size (batched) or offsets[count]*elem_size
 * (ragged) for both in and out; FFT_R32: 4*n*batch on the real side and
 * 8*(n/2+1)*batch on the spectrum side.  FP16/BF16 plans behave as
 * fft_execute_scaled with NULL exponent arrays.
 */
int fft_execute(fft_plan p, const void *in, void *out, void *stream);

/* Bytes of the library's static scratch array on each GPU (64 MiB). */
#define MIFFT_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * For callers that cannot allocate device memory or call hipMalloc/hipFree
 * while they execute (code under stream capture, tight serving loops,
 * harnesses that forbid allocation): fft_execute with every intermediate in
 * memory the library already holds.  Allocates nothing and frees nothing.
 *   FFT_R32 plans above 2^15 (the half-length four-step transform plus the
 *   split pass): the intermediate spectrum of n/2 complex values per
 *   transform goes to a static scratch array of MIFFT_STATIC_SCRATCH_BYTES
 *   per GPU instead of the plan's workspace, so (n/2) * batch * 8 bytes must
 *   fit: FFT_EINVAL_BATCH otherwise, with the largest batch for that length
 *   in the message (e.g. 256 transforms of 2^16 reals, 8 of 2^21).
 *   Every other plan: exactly fft_execute (those executes use no workspace).
 * Arguments, layouts, sizes and error codes otherwise as fft_execute.
 * The scratch array's device address is looked up on the first call on each
 * device.  All calls on one GPU share that GPU's array, and it keeps the
 * last call's contents (nothing in it needs to start at zero): two calls
 * that overlap in time on one GPU (on different streams, or from different
 * threads without ordering) race on it and give wrong results.  Calls on
 * one stream are ordered and safe.  Plans must still be created beforehand
 * (plan creation allocates).
 */
int fft_execute_static_scratch(fft_plan p, const void *in, void *out, void *stream);

/*
 * Apply the adjoint (conjugate transpose) of the plan's transform: the
 * opposite sign at the SAME scale.  For a forward plan that is the
 * unnormalised inverse sum (no 1/n); for an inverse plan it is the forward
 * sum times 1/n.  Used as the backward pass of the differentiable FFT.
 * FFT_C16 / FFT_CBF16 plans write the adjoint at unit scale (no exponent
 * array), as fft_execute does for them.
 * FFT_R32 plans map the other way round (spectrum side -> real side for a
 * sign -1 plan) and apply the adjoint under the real inner product
 * Re<a, b>, which is the gradient PyTorch takes through the transform:
 *   adjoint of R2C:  x_j = Re sum_{k<=n/2} g_k w_n^{-jk}
 *   adjoint of C2R:  X_k = (c_k/n) sum_j v_j w_n^{jk},  c_k = 1 at k = 0
 *                    and n/2, 2 in between.
 */
int fft_execute_adjoint(fft_plan p, const void *in, void *out, void *stream);

/*
 * Block-floating-point execute for FFT_C16 / FFT_CBF16 plans: the logical
 * value of transform b is stored * 2^exp[b].  `in_exp` (device int32[batch])
 * may be NULL for all-zero input exponents.  `out_exp` (device int32[batch])
 * receives the output exponents, chosen per transform so the stored
 * half-precision output neither overflows nor loses range; if NULL the
 * output is written at unit scale (values beyond the format's range become
 * +-inf).  FFT_EINVAL_DTYPE on an FFT_C32 plan.
 */
int fft_execute_scaled(fft_plan p, const void *in, const int32_t *in_exp, void *out,
                       int32_t *out_exp, void *stream);

/*
 * Fused weighted spectral power loss and its gradient, for batched FFT_C32
 * plans.  With A the plan's transform (sign and scale as created) and w a
 * device float32 array laid out like the transforms (n*batch values, w >= 0
 * in the intended use):
 *   loss[b] = sum_k w[b,k] |(A x_b)_k|^2          (device float32[batch])
 *   grad_b  = A^H (2 w_b (A x_b))                  (device, like x)
 * grad is the gradient of sum_b loss[b] with respect to x in PyTorch's
 * complex convention (dL/dRe x + i dL/dIm x).  One pass: x and w are read
 * once and grad written once.  x and grad must not overlap, nor w/loss
 * overlap grad.  Used by the differentiable loss of the Python binding.
 * The kernel's shape (elements per thread, workgroup size) comes from its
 * own tuned table ("loss" lines of MIFFT_TUNE_TABLE), or from the plan's
 * forced variant for a plan made by fft_plan_create_config.
 */
int fft_execute_loss_grad(fft_plan p, const void *x, const float *w, void *grad, float *loss, void *stream);

/* Free the plan and its device memory.  NULL is a no-op.  The caller must
 * make sure no execute of this plan is still in flight. */
void fft_plan_destroy(fft_plan p);

/* Fill *d with what the plan launches.  FFT_ENULL for NULL arguments. */
int fft_plan_describe(fft_plan p, fft_plan_desc *d);

/* Host-only planning: what fft_plan_create(n, batch, sign, dtype) would
 * launch, without touching any device.  Same argument checks and codes. */
int fft_plan_query(int64_t n, int64_t batch, int sign, int dtype, fft_plan_desc *d);

/* Host-only: the FP32 kernel variants compiled in for length n (a power of
 * two in [2, 2048]) that fft_plan_create_config accepts for both signs.
 * Writes up to `cap` triples (ept, wg, variant) to out[3*i .. 3*i+2] and
 * returns how many variants exist (which may exceed cap; out may be NULL
 * when cap is 0).  Returns -1 with FFT_EINVAL_N / FFT_ENULL set on error.
 * Touches no device.  Used by the autotuner and the tests. */
int fft_c32_variants(int64_t n, int *out, int cap);

/* Device address of the plan's FP32 twiddle table tw[m] = exp(-2 pi i m/2048),
 * m < 2048 (16 KiB), or NULL.  Read-only; owned by the plan. */
const void *fft_plan_twiddles(fft_plan p);

/* Last status / message of the calling host thread (FFT_OK / "" if none). */
int fft_last_error(void);
const char *fft_last_error_string(void);

/* Library version string. */
const char *fft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MIFFT_H */
