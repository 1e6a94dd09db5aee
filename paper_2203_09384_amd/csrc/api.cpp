// C ABI of mifft: argument checks, planning, plan ownership and dispatch.
// Kernels live in the *.hip translation units; this file only decides
// which variant to launch and with what arguments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/mifft.h"
#include "fourstep.hpp"
#include "fused_loss.hpp"
#include "half.hpp"
#include "index_maps.hpp"
#include "nd.hpp"
#include "nd2.hpp"
#include "nd3.hpp"
#include "ragged.hpp"
#include "real.hpp"
#include "registry.hpp"

namespace mifft {
hipError_t launch_twiddle_2048(void* tw, hipStream_t stream);
hipError_t launch_twiddle_rows(const void* tw, void* rows, int L, int E, int total, hipStream_t stream);
}

using namespace mifft;

// ------------------------------------------------------------------ errors
namespace {
thread_local int g_err = FFT_OK;
thread_local char g_msg[512] = "";

int set_err(int code, const char* fmt, ...)
{
    g_err = code;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof g_msg, fmt, ap);
    va_end(ap);
    return code;
}

int ok()
{
    g_err = FFT_OK;
    g_msg[0] = '\0';
    return FFT_OK;
}

int hip_err(hipError_t e, const char* what)
{
    if (e == hipErrorStreamCaptureUnsupported || e == hipErrorStreamCaptureImplicit ||
        e == hipErrorStreamCaptureInvalidated)
        return set_err(FFT_ECAPTURE, "%s: %s (%d): plans must be created outside stream capture", what,
                       hipGetErrorString(e), (int)e);
    return set_err(FFT_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v)
{
    int l = 0;
    while ((int64_t(1) << l) < v)
        l++;
    return l;
}
size_t elem_bytes(int dtype) { return (dtype == FFT_C32 || dtype == FFT_R32) ? 8 : 4; }
}  // namespace

// Status reporting for the entry points defined in other translation units.
namespace mifft {
int record_error(int code, const char* msg) { return set_err(code, "%s", msg); }
int record_hip_error(hipError_t e, const char* what) { return hip_err(e, what); }
int record_ok() { return ok(); }
}  // namespace mifft

// ------------------------------------------------------------------ registry
namespace mifft {
static std::vector<KernelC32>& c32_reg()
{
    static std::vector<KernelC32> r;
    return r;
}
void register_c32(const KernelC32& k) { c32_reg().push_back(k); }
const KernelC32* find_c32(int log2n, int log2ept, int wg, int sign, int kind)
{
    for (const auto& k : c32_reg())
        if (k.log2n == log2n && k.log2ept == log2ept && k.wg == wg && k.sign == sign && k.kind == kind)
            return &k;
    return nullptr;
}
int count_c32() { return (int)c32_reg().size(); }
static std::vector<FourStep>& fs_reg()
{
    static std::vector<FourStep> r;
    return r;
}
void register_fourstep(const FourStep& f) { fs_reg().push_back(f); }
const FourStep* find_fourstep(int log2n)
{
    for (const auto& f : fs_reg())
        if (f.log2n == log2n)
            return &f;
    return nullptr;
}
static std::vector<KernelLossGrad>& lg_reg()
{
    static std::vector<KernelLossGrad> r;
    return r;
}
void register_loss_grad(const KernelLossGrad& k) { lg_reg().push_back(k); }
const KernelLossGrad* find_loss_grad(int log2n, int log2ept, int wg, int sign)
{
    for (const auto& k : lg_reg())
        if (k.log2n == log2n && k.log2ept == log2ept && k.wg == wg && k.sign == sign)
            return &k;
    return nullptr;
}
static std::vector<KernelReal>& real_reg()
{
    static std::vector<KernelReal> r;
    return r;
}
void register_real(const KernelReal& k) { real_reg().push_back(k); }
const KernelReal* find_real(int log2m, int log2ept, int wg, int dir, int kind)
{
    for (const auto& k : real_reg())
        if (k.log2m == log2m && k.log2ept == log2ept && k.wg == wg && k.dir == dir && k.kind == kind)
            return &k;
    return nullptr;
}
static std::vector<KernelAxis>& axis_reg()
{
    static std::vector<KernelAxis> r;
    return r;
}
void register_axis(const KernelAxis& k) { axis_reg().push_back(k); }
const KernelAxis* find_axis(int log2n, int sign)
{
    for (const auto& k : axis_reg())
        if (k.log2n == log2n && k.sign == sign)
            return &k;
    return nullptr;
}
static std::vector<KernelNd2>& nd2_reg()
{
    static std::vector<KernelNd2> r;
    return r;
}
void register_nd2(const KernelNd2& k) { nd2_reg().push_back(k); }
static std::vector<KernelNd3>& nd3_reg()
{
    static std::vector<KernelNd3> r;
    return r;
}
void register_nd3(const KernelNd3& k) { nd3_reg().push_back(k); }
const KernelNd3* find_nd3(int log2n0, int log2n1, int log2n2, int sign)
{
    for (const auto& k : nd3_reg())
        if (k.log2n[0] == log2n0 && k.log2n[1] == log2n1 && k.log2n[2] == log2n2 && k.sign == sign)
            return &k;
    return nullptr;
}
const KernelNd2* find_nd2(int log2n0, int log2n1, int sign)
{
    for (const auto& k : nd2_reg())
        if (k.log2n0 == log2n0 && k.log2n1 == log2n1 && k.sign == sign)
            return &k;
    return nullptr;
}
const KernelC32* c32_at(int i) { return (i >= 0 && i < count_c32()) ? &c32_reg()[i] : nullptr; }
}  // namespace mifft

// ------------------------------------------------------------------ tuning
namespace {
struct Variant {
    int log2ept, wg, kind;
};

// Built-in choice per log2 N (index 1..11) for FP32: the autotuner's pick on
// MI355X at 2^26 elements per launch (log2 EPT, workgroup size, variant).
const Variant kDefaultC32[21] = {
    {0, 0, 0},     // unused
    {1, 64, 11},   // N=2     one thread per transform, block staged through LDS
    {2, 128, 11},  // N=4
    {3, 64, 11},   // N=8
    {4, 128, 11},  // N=16
    {3, 64, 12},   // N=32    several threads per transform, block staged through LDS
    {3, 256, 12},  // N=64
    {3, 64, 12},   // N=128
    {4, 128, 12},  // N=256
    {3, 64, 12},   // N=512
    {4, 64, 3},    // N=1024  persistent, next-group prefetch
    {4, 128, 3},   // N=2048  persistent, next-group prefetch
    {3, 512, 3},   // N=2^12  one transform per workgroup
    {4, 512, 3},   // N=2^13
    {4, 1024, 2},  // N=2^14  135 KiB LDS
    {0, 0, 9},     // N=2^15 .. 2^20: four-step (column + row pass)
    {0, 0, 9}, {0, 0, 9}, {0, 0, 9}, {0, 0, 9}, {0, 0, 9},
};

// Real-input transforms (FFT_R32), per log2 of the half length M = n/2
// (index 0..14): the half-length transform's configuration, the
// autotuner's pick on MI355X (R2C + C2R over 2^27 reals).
const Variant kDefaultR32[15] = {
    {0, 256, 0},   // n=2     one thread per transform, no passes
    {1, 64, 0},    // n=4     the half-length transform inside one thread
    {2, 256, 0},   // n=8
    {2, 256, 2},   // n=16
    {2, 256, 2},   // n=32
    {3, 256, 3},   // n=64    persistent, next-group prefetch
    {2, 256, 2},   // n=128
    {3, 256, 6},   // n=256   wavefront-local exchanges
    {4, 256, 3},   // n=512   persistent, next-group prefetch
    {4, 256, 3},   // n=1024
    {4, 64, 3},    // n=2048
    {4, 128, 3},   // n=4096
    {4, 256, 3},   // n=2^13  one transform per workgroup
    {4, 512, 3},   // n=2^14
    {4, 1024, 2},  // n=2^15
};

// Fused loss-gradient kernel (two transforms per group, so its own best
// shape differs from the plain transform's), per log2 N (index 1..11):
// the autotuner's pick on MI355X at 2^25 elements (log2 EPT, workgroup
// size; the kind field is unused).
const Variant kDefaultLoss[12] = {
    {0, 0, 0},     // unused
    {1, 128, 0},   // N=2
    {2, 64, 0},    // N=4
    {3, 256, 0},   // N=8
    {2, 64, 0},    // N=16
    {2, 256, 0},   // N=32
    {2, 256, 0},   // N=64
    {3, 256, 0},   // N=128
    {4, 64, 0},    // N=256
    {3, 256, 0},   // N=512
    {4, 256, 0},   // N=1024
    {4, 128, 0},   // N=2048
};

std::once_flag g_tune_once;
Variant g_tuned_c32[21];
bool g_have_tuned_c32[21];
Variant g_tuned_r32[15];
bool g_have_tuned_r32[15];
Variant g_tuned_loss[12];
bool g_have_tuned_loss[12];

// MIFFT_TUNE_TABLE: text lines "c32 <log2n> <ept> <wg> <kind>",
// "r32 <log2(n/2)> <ept> <wg> <kind>" and "loss <log2n> <ept> <wg>"; '#'
// starts a comment.
void load_tune_table()
{
    const char* path = getenv("MIFFT_TUNE_TABLE");
    if (!path || !*path)
        return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t h = line.find('#');
        if (h != std::string::npos)
            line.resize(h);
        std::istringstream ss(line);
        std::string dt;
        int l = 0, ept = 0, wg = 0, kind = 0;
        if (!(ss >> dt >> l >> ept >> wg))
            continue;
        if (!(ss >> kind))
            kind = 0;
        if (dt == "c32" && l >= 1 && l <= 20 && ((is_pow2(ept) && ept >= 2 && ept <= 16) || kind == 9)) {
            g_tuned_c32[l] = Variant{kind == 9 ? 0 : ilog2(ept), wg, kind};
            g_have_tuned_c32[l] = true;
        }
        if (dt == "r32" && l >= 1 && l <= 14 && is_pow2(ept) && ept >= 2 && ept <= 16) {
            g_tuned_r32[l] = Variant{ilog2(ept), wg, kind};
            g_have_tuned_r32[l] = true;
        }
        if (dt == "loss" && l >= 1 && l <= 11 && is_pow2(ept) && ept >= 2 && ept <= 16) {
            g_tuned_loss[l] = Variant{ilog2(ept), wg, 0};
            g_have_tuned_loss[l] = true;
        }
    }
}

Variant choose_c32(int log2n)
{
    std::call_once(g_tune_once, load_tune_table);
    if (g_have_tuned_c32[log2n]) {
        const Variant v = g_tuned_c32[log2n];
        if ((v.kind == 9 && log2n > 11) || find_c32(log2n, v.log2ept, v.wg, -1, v.kind))
            return v;
    }
    return kDefaultC32[log2n];
}

Variant choose_loss(int log2n)
{
    std::call_once(g_tune_once, load_tune_table);
    return g_have_tuned_loss[log2n] ? g_tuned_loss[log2n] : kDefaultLoss[log2n];
}

Variant choose_r32(int log2m)
{
    std::call_once(g_tune_once, load_tune_table);
    if (g_have_tuned_r32[log2m]) {
        const Variant v = g_tuned_r32[log2m];
        if (find_real(log2m, v.log2ept, v.wg, 0, v.kind) && find_real(log2m, v.log2ept, v.wg, 1, v.kind))
            return v;
    }
    return kDefaultR32[log2m];
}

// Stockham schedule of (log2 N, log2 EPT): a remainder pass first, then
// passes of radix EPT (the schedule functions the kernels use).
int schedule(int log2n, int log2ept, int* radices)
{
    const int np = idx::sched_np(log2n, log2ept);
    for (int p = 0; p < np; p++)
        radices[p] = 1 << idx::sched_log2r(log2n, log2ept, p);
    return np;
}
}  // namespace

// ------------------------------------------------------------------ plan
struct mifft_plan_s {
    int kind = 0;  // 0 batched, 1 ragged
    int64_t n = 0, batch = 0;
    int sign = -1, dtype = FFT_C32;
    float scale = 1.f;
    int device = -1;
    int log2n = 0;
    Variant var{};
    const KernelC32* fwd = nullptr;  // sign -1 kernel
    const KernelC32* bwd = nullptr;  // sign +1 kernel
    void* tw = nullptr;              // device FP32 twiddle table (2048 entries)
    void* rows = nullptr;            // per-pass twiddle rows (kind >= 1)
    int64_t grid_limit = 0;          // persistent kinds: CUs x workgroups per CU
    const FourStep* fs = nullptr;    // lengths above 2048: two-pass four-step
    void* fs_rows1 = nullptr;
    void* fs_rows2 = nullptr;
    void* fs_tw = nullptr;           // two-level w_N table: 1024 + N/1024 entries
    const KernelLossGrad* lossgrad = nullptr;  // fused loss + gradient kernel (FP32)
    void* lg_rows = nullptr;         // its twiddle rows when they differ from `rows`
    int64_t lg_grid_limit = 0;
    int64_t total = 0;               // elements per execute (either kind)
    RaggedPlan* ragged = nullptr;
    HalfPlan* half = nullptr;
    const KernelReal* r2c = nullptr;  // FFT_R32: real -> bins kernel
    const KernelReal* c2r = nullptr;  // FFT_R32: bins -> real kernel
    void* wn = nullptr;               // FFT_R32: w_n^k, k < n/2
    // FFT_R32 above 2^15: four-step half-length sub-plan, its workspace
    // (n/2 complex per transform) and the two-level w_n table of the split
    mifft_plan_s* real_sub = nullptr;
    void* real_ws = nullptr;
    void* real_tw = nullptr;
    // multidimensional plans (kind 2): the last axis as a batched sub-plan,
    // then in-place axis passes from the second-to-last axis to the first
    int rank = 1;
    int64_t dims[3] = {0, 0, 0};
    mifft_plan_s* last = nullptr;
    const KernelAxis* ax_same[2] = {nullptr, nullptr};  // the plan's sign
    const KernelAxis* ax_opp[2] = {nullptr, nullptr};   // the adjoint's sign
    void* ax_rows[2] = {nullptr, nullptr};
    int ax_log2s[2] = {0, 0};
    int64_t ax_count[2] = {0, 0};
    float ax_scale[2] = {1.f, 1.f};
    int ax_first = -1;  // the axis passes run for axes ax_first .. 0
    // single-pass 2D (the array fits one workgroup's LDS): no sub-plan
    const KernelNd2* nd2_same = nullptr;
    const KernelNd2* nd2_opp = nullptr;
    void* nd2_rows[2] = {nullptr, nullptr};  // column, row transforms
    int64_t nd2_grid_cap = 0;                // persistent single-pass 2D kernel: its resident workgroups
    const KernelNd3* nd3_same = nullptr;     // single-pass 3D kernel (this sign / the opposite one)
    const KernelNd3* nd3_opp = nullptr;
    void* nd3_rows = nullptr;                // its twiddle rows, axes 0, 1, 2 back to back
};

namespace {
constexpr int64_t kMaxN = int64_t(1) << 20;
constexpr int64_t kMaxRealN = int64_t(1) << 21;
constexpr int64_t kMaxFusedRealN = int64_t(1) << 15;  // above: four-step half length + split pass

int check_common(int64_t n, int64_t batch, int sign, int dtype)
{
    if (dtype != FFT_C32 && dtype != FFT_C16 && dtype != FFT_CBF16 && dtype != FFT_R32)
        return set_err(FFT_EINVAL_DTYPE, "dtype %d is not FFT_C32, FFT_C16, FFT_CBF16 or FFT_R32", dtype);
    if (dtype == FFT_R32 && (!is_pow2(n) || n < 2 || n > kMaxRealN))
        return set_err(FFT_EINVAL_N, "n=%lld: real-input (FFT_R32) lengths are powers of two in [2, 2^21]",
                       (long long)n);
    if (dtype != FFT_R32 && (!is_pow2(n) || n < 2 || n > kMaxN))
        return set_err(FFT_EINVAL_N, "n=%lld is not a power of two in [2, 2^20]", (long long)n);
    if (n > 2048 && dtype != FFT_C32 && dtype != FFT_R32)
        return set_err(FFT_EINVAL_N, "n=%lld: lengths above 2048 are FFT_C32 / FFT_R32 only", (long long)n);
    if (batch < 1)
        return set_err(FFT_EINVAL_BATCH, "batch=%lld must be >= 1", (long long)batch);
    if (batch > (int64_t(1) << 40) / n)
        return set_err(FFT_EINVAL_BATCH, "n*batch=%lld*%lld exceeds 2^40 elements", (long long)n,
                       (long long)batch);
    if (sign != -1 && sign != 1)
        return set_err(FFT_EINVAL_SIGN, "sign=%d must be -1 (forward) or +1 (inverse)", sign);
    return FFT_OK;
}

int fill_desc_fourstep(int64_t n, int64_t batch, int sign, int dtype, fft_plan_desc* d)
{
    memset(d, 0, sizeof *d);
    const FourStep* f = find_fourstep(ilog2(n));
    d->n = n;
    d->batch = batch;
    d->sign = sign;
    d->dtype = dtype;
    d->scale = sign > 0 ? 1.0f / (float)n : 1.0f;
    d->kind = 0;
    d->variant = 9;
    if (!f)
        return FFT_OK;
    d->ept = 1 << f->log2e1;
    d->wg = f->tile1 * (int)((1 << f->log2n1) >> f->log2e1);
    d->transforms_per_wg = f->tile1;
    d->grid = batch * ((int64_t(1) << f->log2n2) / f->tile1);
    int r1[8], r2[8];
    const int n1 = schedule(f->log2n1, f->log2e1, r1), n2 = schedule(f->log2n2, f->log2e2, r2);
    d->npasses = std::min(8, n1 + n2);
    for (int i = 0; i < d->npasses; i++)
        d->radices[i] = i < n1 ? r1[i] : r2[i - n1];
    d->lds_bytes = std::max(f->lds1, f->lds2);
    return FFT_OK;
}

int fill_desc_c32(int64_t n, int64_t batch, int sign, int dtype, Variant v, int64_t grid_limit, fft_plan_desc* d)
{
    if (v.kind == 9)
        return fill_desc_fourstep(n, batch, sign, dtype, d);
    memset(d, 0, sizeof *d);
    const int log2n = ilog2(n);
    d->n = n;
    d->batch = batch;
    d->sign = sign;
    d->dtype = dtype;
    d->scale = sign > 0 ? 1.0f / (float)n : 1.0f;
    d->ept = 1 << v.log2ept;
    d->wg = v.wg;
    const int tpt = (int)(n >> v.log2ept);
    d->transforms_per_wg = v.wg / tpt;
    d->grid = (batch + d->transforms_per_wg - 1) / d->transforms_per_wg;
    d->npasses = schedule(log2n, v.log2ept, d->radices);
    if (grid_limit > 0 && d->grid > grid_limit)
        d->grid = grid_limit;
    const KernelC32* k = find_c32(log2n, v.log2ept, v.wg, sign, v.kind);
    d->lds_bytes = k ? k->lds_bytes : 0;
    d->kind = 0;
    d->variant = v.kind;
    return FFT_OK;
}

// FFT_R32: the half-length (n/2) complex transform's shape; ept, radices
// and lds describe it.
int fill_desc_r32(int64_t n, int64_t batch, int sign, Variant v, int64_t grid_limit, fft_plan_desc* d)
{
    if (n > kMaxFusedRealN) {
        // the half-length four-step transform (plus the split pass)
        fill_desc_fourstep(n / 2, batch, sign, FFT_C32, d);
        d->n = n;
        d->dtype = FFT_R32;
        d->scale = sign > 0 ? 1.0f / (float)n : 1.0f;
        return FFT_OK;
    }
    memset(d, 0, sizeof *d);
    const int log2m = ilog2(n) - 1;
    d->n = n;
    d->batch = batch;
    d->sign = sign;
    d->dtype = FFT_R32;
    d->scale = sign > 0 ? 1.0f / (float)n : 1.0f;
    d->ept = 1 << v.log2ept;
    d->wg = v.wg;
    const int tpt = (int)((n / 2) >> v.log2ept);
    d->transforms_per_wg = v.wg / std::max(tpt, 1);
    d->grid = (batch + d->transforms_per_wg - 1) / d->transforms_per_wg;
    if (grid_limit > 0 && d->grid > grid_limit)
        d->grid = grid_limit;
    d->npasses = log2m > 0 ? schedule(log2m, v.log2ept, d->radices) : 0;
    const KernelReal* k = find_real(log2m, v.log2ept, v.wg, sign < 0 ? 0 : 1, v.kind);
    d->lds_bytes = k ? k->lds_bytes : 0;
    d->kind = 0;
    d->variant = v.kind;
    return FFT_OK;
}

// Plan creation allocates device memory and fills tables on the legacy
// default stream, then waits for them: none of that may happen while a
// stream capture is active (it would end or invalidate the capture).  A
// query of the legacy stream reports a capture in progress on any stream of
// the process (global capture mode) or of this thread.
int check_not_capturing()
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    const hipError_t e = hipStreamIsCapturing(nullptr, &st);
    if (e == hipErrorStreamCaptureImplicit || (e == hipSuccess && st != hipStreamCaptureStatusNone))
        return set_err(FFT_ECAPTURE, "plan creation during stream capture (it allocates and synchronises); "
                                     "create plans before capturing");
    if (e != hipSuccess)
        return hip_err(e, "hipStreamIsCapturing");
    return FFT_OK;
}

// Device checks of plan creation: not capturing, and a gfx950 device current.
int current_gfx950(int* dev)
{
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess)
        return hip_err(e, "hipGetDevice");
    if (check_not_capturing() != FFT_OK)
        return g_err;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, *dev);
    if (e != hipSuccess)
        return hip_err(e, "hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_err(FFT_EDEVICE, "device %d is %s; this library is built for gfx950", *dev,
                       prop.gcnArchName);
    return FFT_OK;
}

int make_twiddles(mifft_plan_s* p)
{
    hipError_t e = hipMalloc(&p->tw, 2048 * sizeof(float2));
    if (e != hipSuccess) {
        p->tw = nullptr;
        return e == hipErrorOutOfMemory ? set_err(FFT_ENOMEM, "hipMalloc(twiddles) failed")
                                        : hip_err(e, "hipMalloc(twiddles)");
    }
    e = launch_twiddle_2048(p->tw, nullptr);
    if (e != hipSuccess)
        return hip_err(e, "twiddle kernel launch");
    e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess)
        return hip_err(e, "twiddle kernel");
    return FFT_OK;
}

// Tables of a four-step plan: rows of both inner transforms and the two-level
// w_N table.
int make_fourstep(mifft_plan_s* p)
{
    const FourStep* f = find_fourstep(p->log2n);
    p->fs = f;
    const size_t nt = 1024 + ((size_t)1 << (p->log2n - 10));
    hipError_t e = hipMalloc(&p->fs_rows1, std::max(f->rows1, 1) * sizeof(float2));
    if (e == hipSuccess)
        e = hipMalloc(&p->fs_rows2, std::max(f->rows2, 1) * sizeof(float2));
    if (e == hipSuccess)
        e = hipMalloc(&p->fs_tw, nt * sizeof(float2));
    if (e != hipSuccess)
        return e == hipErrorOutOfMemory ? set_err(FFT_ENOMEM, "hipMalloc(four-step tables) failed")
                                        : hip_err(e, "hipMalloc(four-step tables)");
    e = launch_twiddle_rows(p->tw, p->fs_rows1, f->log2n1, f->log2e1, f->rows1, nullptr);
    if (e == hipSuccess)
        e = launch_twiddle_rows(p->tw, p->fs_rows2, f->log2n2, f->log2e2, f->rows2, nullptr);
    if (e == hipSuccess)
        e = launch_twiddle_big(p->fs_tw, static_cast<float2*>(p->fs_tw) + 1024, p->log2n, nullptr);
    if (e == hipSuccess)
        e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess)
        return hip_err(e, "four-step tables");
    return FFT_OK;
}

// Twiddle rows and the persistent grid size of a kind >= 1 variant.
int make_rows(mifft_plan_s* p)
{
    const KernelC32* k = p->fwd;
    if (k->rows > 0) {
        hipError_t e = hipMalloc(&p->rows, (size_t)k->rows * sizeof(float2));
        if (e != hipSuccess) {
            p->rows = nullptr;
            return e == hipErrorOutOfMemory ? set_err(FFT_ENOMEM, "hipMalloc(twiddle rows) failed")
                                            : hip_err(e, "hipMalloc(twiddle rows)");
        }
        e = launch_twiddle_rows(p->tw, p->rows, k->log2n, k->log2ept, k->rows, nullptr);
        if (e != hipSuccess)
            return hip_err(e, "twiddle rows launch");
        e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess)
            return hip_err(e, "twiddle rows kernel");
    }
    p->grid_limit = 0;
    if ((k->kind == 3 || k->kind == 4 || k->kind == 7 || k->kind == 8) && k->occupancy) {
        int cus = 0;
        hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
        if (e != hipSuccess)
            return hip_err(e, "hipDeviceGetAttribute(CU count)");
        const int occ = std::max(k->occupancy(), std::max(p->bwd->occupancy ? p->bwd->occupancy() : 1, 1));
        p->grid_limit = (int64_t)cus * occ;
    }
    return FFT_OK;
}

// The fused loss-gradient kernel of a batched FP32 plan: the tuned shape
// for its length (a plan created with a forced variant: that variant's
// EPT and WG) when compiled, else the first compiled one; its twiddle rows
// are shared with the plan's when the schedules agree.
int make_loss_grad(mifft_plan_s* p, bool forced)
{
    const Variant want = forced ? p->var : choose_loss(p->log2n);
    const KernelLossGrad* k = find_loss_grad(p->log2n, want.log2ept, want.wg, p->sign);
    for (int e = 4; e >= 1 && !k; e--)
        for (int wg : {256, 128, 64})
            if (!k)
                k = find_loss_grad(p->log2n, e, wg, p->sign);
    if (!k)
        return set_err(FFT_EINVAL_CONFIG, "no fused loss kernel for n=%lld", (long long)p->n);
    p->lossgrad = k;
    if (k->rows > 0 && !(p->rows && p->fwd->log2ept == k->log2ept)) {
        hipError_t e = hipMalloc(&p->lg_rows, (size_t)k->rows * sizeof(float2));
        if (e != hipSuccess) {
            p->lg_rows = nullptr;
            return e == hipErrorOutOfMemory ? set_err(FFT_ENOMEM, "hipMalloc(loss rows) failed")
                                            : hip_err(e, "hipMalloc(loss rows)");
        }
        e = launch_twiddle_rows(p->tw, p->lg_rows, k->log2n, k->log2ept, k->rows, nullptr);
        if (e == hipSuccess)
            e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess)
            return hip_err(e, "loss twiddle rows");
    }
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess)
        return hip_err(e, "hipDeviceGetAttribute(CU count)");
    p->lg_grid_limit = (int64_t)cus * std::max(k->occupancy(), 1);
    return FFT_OK;
}

// Tables of an FFT_R32 plan: the half-length transform's twiddle rows, the
// w_n^k of the even/odd split, and the persistent grid size.
int make_real(mifft_plan_s* p)
{
    const KernelReal* k = p->r2c;
    hipError_t e = hipSuccess;
    if (k->rows > 0) {
        e = hipMalloc(&p->rows, (size_t)k->rows * sizeof(float2));
        if (e != hipSuccess)
            p->rows = nullptr;
    }
    if (e == hipSuccess) {
        e = hipMalloc(&p->wn, (size_t)(p->n / 2) * sizeof(float2));
        if (e != hipSuccess)
            p->wn = nullptr;
    }
    if (e != hipSuccess)
        return e == hipErrorOutOfMemory ? set_err(FFT_ENOMEM, "hipMalloc(real-input tables) failed")
                                        : hip_err(e, "hipMalloc(real-input tables)");
    if (k->rows > 0)
        e = launch_twiddle_rows(p->tw, p->rows, k->log2m, k->log2ept, k->rows, nullptr);
    if (e == hipSuccess)
        e = launch_twiddle_real(p->tw, p->wn, p->log2n, nullptr);
    if (e == hipSuccess)
        e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess)
        return hip_err(e, "real-input tables");
    p->grid_limit = 0;
    if ((k->kind == 3 || k->kind == 7) && k->occupancy) {
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
        if (e != hipSuccess)
            return hip_err(e, "hipDeviceGetAttribute(CU count)");
        const int occ = std::max(std::max(k->occupancy(), p->c2r->occupancy ? p->c2r->occupancy() : 1), 1);
        p->grid_limit = (int64_t)cus * occ;
    }
    return FFT_OK;
}

void free_plan(mifft_plan_s* p)
{
    if (!p)
        return;
    if (p->last)
        free_plan(p->last);
    if (p->real_sub)
        free_plan(p->real_sub);
    for (void* q : {p->real_ws, p->real_tw})
        if (q)
            (void)hipFree(q);
    for (void* q : {p->ax_rows[0], p->ax_rows[1], p->nd2_rows[0], p->nd2_rows[1], p->nd3_rows})
        if (q)
            (void)hipFree(q);
    if (p->ragged)
        ragged_destroy(p->ragged);
    if (p->half)
        half_destroy(p->half);
    if (p->tw)
        (void)hipFree(p->tw);
    if (p->rows)
        (void)hipFree(p->rows);
    if (p->lg_rows)
        (void)hipFree(p->lg_rows);
    for (void* q : {p->fs_rows1, p->fs_rows2, p->fs_tw, p->wn})
        if (q)
            (void)hipFree(q);
    delete p;
}

fft_plan create_batched(int64_t n, int64_t batch, int sign, int dtype, const Variant* force);

// Real input above 2^15: the half-length complex transform as a four-step
// sub-plan into a workspace, and the even/odd split as a pass of its own.
fft_plan create_real_large(int64_t n, int64_t batch, int sign)
{
    const int64_t m = n / 2;
    const int64_t kblocks = ((m / 2 + 1) + 255) / 256;
    if (batch > 0x7fffffffLL / kblocks) {
        set_err(FFT_EINVAL_BATCH, "batch=%lld needs more than 2^31-1 workgroups", (long long)batch);
        return nullptr;
    }
    mifft_plan_s* sub = create_batched(m, batch, sign, FFT_C32, nullptr);
    if (!sub)
        return nullptr;
    auto* p = new (std::nothrow) mifft_plan_s();
    if (!p) {
        free_plan(sub);
        set_err(FFT_ENOMEM, "out of host memory");
        return nullptr;
    }
    p->kind = 0;
    p->n = n;
    p->batch = batch;
    p->sign = sign;
    p->dtype = FFT_R32;
    p->scale = sign > 0 ? 1.0f / (float)n : 1.0f;
    p->device = sub->device;
    p->log2n = ilog2(n);
    p->total = n * batch;
    p->real_sub = sub;
    p->var = Variant{0, 0, 9};
    hipError_t e = hipMalloc(&p->real_ws, (size_t)m * (size_t)batch * sizeof(float2));
    if (e != hipSuccess) {
        p->real_ws = nullptr;
    } else {
        e = hipMalloc(&p->real_tw, (size_t)(1024 + n / 1024) * sizeof(float2));
        if (e != hipSuccess)
            p->real_tw = nullptr;
    }
    if (e != hipSuccess) {
        e == hipErrorOutOfMemory ? set_err(FFT_ENOMEM, "hipMalloc(real-input workspace) failed")
                                 : hip_err(e, "hipMalloc(real-input workspace)");
        free_plan(p);
        return nullptr;
    }
    e = launch_twiddle_big(p->real_tw, static_cast<float2*>(p->real_tw) + 1024, p->log2n, nullptr);
    if (e == hipSuccess)
        e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        hip_err(e, "real-input split table");
        free_plan(p);
        return nullptr;
    }
    ok();
    return p;
}

fft_plan create_real(int64_t n, int64_t batch, int sign, const Variant* force)
{
    if (n > kMaxFusedRealN) {
        if (force && force->kind != 9) {
            set_err(FFT_EINVAL_CONFIG, "real-input lengths above 2^15 use the four-step split (variant 9)");
            return nullptr;
        }
        return create_real_large(n, batch, sign);
    }
    const int log2m = ilog2(n) - 1;
    const Variant v = force ? *force : choose_r32(log2m);
    const KernelReal* r2c = find_real(log2m, v.log2ept, v.wg, 0, v.kind);
    const KernelReal* c2r = find_real(log2m, v.log2ept, v.wg, 1, v.kind);
    if (!r2c || !c2r) {
        set_err(FFT_EINVAL_CONFIG, "no real-input kernel for n=%lld ept=%d wg=%d kind=%d", (long long)n,
                1 << v.log2ept, v.wg, v.kind);
        return nullptr;
    }
    const int tpb = v.wg / (int)std::max<int64_t>((n / 2) >> v.log2ept, 1);
    if ((batch + tpb - 1) / tpb > 0x7fffffffLL) {
        set_err(FFT_EINVAL_BATCH, "batch=%lld needs more than 2^31-1 workgroups", (long long)batch);
        return nullptr;
    }
    int dev = -1;
    if (current_gfx950(&dev) != FFT_OK)
        return nullptr;
    auto* p = new (std::nothrow) mifft_plan_s();
    if (!p) {
        set_err(FFT_ENOMEM, "out of host memory");
        return nullptr;
    }
    p->kind = 0;
    p->n = n;
    p->batch = batch;
    p->sign = sign;
    p->dtype = FFT_R32;
    p->scale = sign > 0 ? 1.0f / (float)n : 1.0f;
    p->device = dev;
    p->log2n = ilog2(n);
    p->var = v;
    p->total = n * batch;
    p->r2c = r2c;
    p->c2r = c2r;
    if (make_twiddles(p) != FFT_OK || make_real(p) != FFT_OK) {
        free_plan(p);
        return nullptr;
    }
    ok();
    return p;
}

fft_plan create_batched(int64_t n, int64_t batch, int sign, int dtype, const Variant* force)
{
    if (check_common(n, batch, sign, dtype) != FFT_OK)
        return nullptr;
    if (dtype == FFT_R32)
        return create_real(n, batch, sign, force);
    const int log2n = ilog2(n);
    Variant v{};
    const bool four_step = dtype == FFT_C32 && n > 2048 &&
                           (force ? force->kind == 9 : choose_c32(log2n).kind == 9);
    if (four_step) {
        const FourStep* f = find_fourstep(log2n);
        if (!f) {
            set_err(FFT_EINVAL_N, "no four-step kernels for n=%lld", (long long)n);
            return nullptr;
        }
        if (batch > (0x7fffffffLL - 16) / ((int64_t(1) << f->log2n2) / 8)) {
            set_err(FFT_EINVAL_BATCH, "batch=%lld needs more than 2^31-1 workgroups", (long long)batch);
            return nullptr;
        }
        v = Variant{f->log2e1, 0, 9};
    } else if (dtype == FFT_C32) {
        if (force) {
            v = *force;
            if (!find_c32(log2n, v.log2ept, v.wg, -1, v.kind) || !find_c32(log2n, v.log2ept, v.wg, +1, v.kind)) {
                set_err(FFT_EINVAL_CONFIG, "no FP32 kernel for n=%lld ept=%d wg=%d kind=%d", (long long)n,
                        1 << v.log2ept, v.wg, v.kind);
                return nullptr;
            }
        } else {
            v = choose_c32(log2n);
        }
        const int tpb = v.wg / (int)(n >> v.log2ept);
        if ((batch + tpb - 1) / tpb > 0x7fffffffLL) {
            set_err(FFT_EINVAL_BATCH, "batch=%lld needs more than 2^31-1 workgroups", (long long)batch);
            return nullptr;
        }
    } else if (!half_supported(n)) {
        set_err(FFT_EINVAL_DTYPE, "FP16/BF16 plans support n in {%s}", half_supported_lengths());
        return nullptr;
    }
    int dev = -1;
    if (current_gfx950(&dev) != FFT_OK)
        return nullptr;
    auto* p = new (std::nothrow) mifft_plan_s();
    if (!p) {
        set_err(FFT_ENOMEM, "out of host memory");
        return nullptr;
    }
    p->kind = 0;
    p->n = n;
    p->batch = batch;
    p->sign = sign;
    p->dtype = dtype;
    p->scale = sign > 0 ? 1.0f / (float)n : 1.0f;
    p->device = dev;
    p->log2n = log2n;
    p->var = v;
    p->total = n * batch;
    if (dtype == FFT_C32 && !four_step) {
        p->fwd = find_c32(log2n, v.log2ept, v.wg, -1, v.kind);
        p->bwd = find_c32(log2n, v.log2ept, v.wg, +1, v.kind);
    }
    if (make_twiddles(p) != FFT_OK) {
        free_plan(p);
        return nullptr;
    }
    if (four_step) {
        if (make_fourstep(p) != FFT_OK) {
            free_plan(p);
            return nullptr;
        }
        ok();
        return p;
    }
    if (dtype == FFT_C32 && p->fwd->kind >= 1 && make_rows(p) != FFT_OK) {
        free_plan(p);
        return nullptr;
    }
    if (dtype == FFT_C32 && n <= 2048 && make_loss_grad(p, force != nullptr) != FFT_OK) {
        free_plan(p);
        return nullptr;
    }
    if (dtype != FFT_C32) {
        int rc = half_create(&p->half, n, batch, dtype, p->tw);
        if (rc != FFT_OK) {
            set_err(rc, "%s", half_last_message());
            free_plan(p);
            return nullptr;
        }
    }
    ok();
    return p;
}

constexpr int64_t kMaxAxisN = 2048;

// A 2D plan whose arrays fit one workgroup's LDS: one kernel, one HBM pass.
fft_plan create_nd2(const int64_t* dims, int64_t batch, int sign)
{
    const int L0 = ilog2(dims[0]), L1 = ilog2(dims[1]);
    const KernelNd2* k = find_nd2(L0, L1, sign);
    if ((batch + k->arrays_per_wg - 1) / k->arrays_per_wg > 0x7fffffffLL) {
        set_err(FFT_EINVAL_BATCH, "batch=%lld needs more than 2^31-1 workgroups", (long long)batch);
        return nullptr;
    }
    int dev = -1;
    if (current_gfx950(&dev) != FFT_OK)
        return nullptr;
    auto* p = new (std::nothrow) mifft_plan_s();
    if (!p) {
        set_err(FFT_ENOMEM, "out of host memory");
        return nullptr;
    }
    p->kind = 2;
    p->n = dims[0] * dims[1];
    p->batch = batch;
    p->sign = sign;
    p->dtype = FFT_C32;
    p->scale = sign > 0 ? 1.0f / (float)p->n : 1.0f;
    p->device = dev;
    p->log2n = L0 + L1;
    p->total = p->n * batch;
    p->rank = 2;
    p->dims[0] = dims[0];
    p->dims[1] = dims[1];
    p->nd2_same = k;
    p->nd2_opp = find_nd2(L0, L1, -sign);
    if (k->slots)
        p->nd2_grid_cap = k->slots();
    if (make_twiddles(p) != FFT_OK) {
        free_plan(p);
        return nullptr;
    }
    const int Ls[2] = {L0, L1}, counts[2] = {k->rows0, k->rows1};
    for (int i = 0; i < 2; i++) {
        if (counts[i] <= 0)
            continue;
        hipError_t e = hipMalloc(&p->nd2_rows[i], (size_t)counts[i] * sizeof(float2));
        if (e != hipSuccess) {
            p->nd2_rows[i] = nullptr;
            e == hipErrorOutOfMemory ? set_err(FFT_ENOMEM, "hipMalloc(2D twiddle rows) failed")
                                     : hip_err(e, "hipMalloc(2D twiddle rows)");
            free_plan(p);
            return nullptr;
        }
        e = launch_twiddle_rows(p->tw, p->nd2_rows[i], Ls[i], k->log2ept, counts[i], nullptr);
        if (e == hipSuccess)
            e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) {
            hip_err(e, "2D twiddle rows");
            free_plan(p);
            return nullptr;
        }
    }
    ok();
    return p;
}

// A 3D plan whose arrays fit one workgroup's LDS: one kernel, one HBM pass.
fft_plan create_nd3(const int64_t* dims, int64_t batch, int sign)
{
    const int L[3] = {ilog2(dims[0]), ilog2(dims[1]), ilog2(dims[2])};
    const KernelNd3* k = find_nd3(L[0], L[1], L[2], sign);
    if ((batch + k->arrays_per_wg - 1) / k->arrays_per_wg > 0x7fffffffLL) {
        set_err(FFT_EINVAL_BATCH, "batch=%lld needs more than 2^31-1 workgroups", (long long)batch);
        return nullptr;
    }
    int dev = -1;
    if (current_gfx950(&dev) != FFT_OK)
        return nullptr;
    auto* p = new (std::nothrow) mifft_plan_s();
    if (!p) {
        set_err(FFT_ENOMEM, "out of host memory");
        return nullptr;
    }
    p->kind = 2;
    p->n = dims[0] * dims[1] * dims[2];
    p->batch = batch;
    p->sign = sign;
    p->dtype = FFT_C32;
    p->scale = sign > 0 ? 1.0f / (float)p->n : 1.0f;
    p->device = dev;
    p->log2n = L[0] + L[1] + L[2];
    p->total = p->n * batch;
    p->rank = 3;
    for (int a = 0; a < 3; a++)
        p->dims[a] = dims[a];
    p->nd3_same = k;
    p->nd3_opp = find_nd3(L[0], L[1], L[2], -sign);
    if (make_twiddles(p) != FFT_OK) {
        free_plan(p);
        return nullptr;
    }
    const int total = k->rows[0] + k->rows[1] + k->rows[2];
    if (total > 0) {
        hipError_t e = hipMalloc(&p->nd3_rows, (size_t)total * sizeof(float2));
        if (e != hipSuccess) {
            p->nd3_rows = nullptr;
            e == hipErrorOutOfMemory ? set_err(FFT_ENOMEM, "hipMalloc(3D twiddle rows) failed")
                                     : hip_err(e, "hipMalloc(3D twiddle rows)");
            free_plan(p);
            return nullptr;
        }
        int off = 0;
        for (int a = 0; a < 3 && e == hipSuccess; a++) {
            if (k->rows[a] > 0)
                e = launch_twiddle_rows(p->tw, static_cast<float2*>(p->nd3_rows) + off, L[a], k->log2ept, k->rows[a],
                                        nullptr);
            off += k->rows[a];
        }
        if (e == hipSuccess)
            e = hipStreamSynchronize(nullptr);
        if (e != hipSuccess) {
            hip_err(e, "3D twiddle rows");
            free_plan(p);
            return nullptr;
        }
    }
    ok();
    return p;
}

fft_plan create_nd(int rank, const int64_t* dims, int64_t batch, int sign, int dtype)
{
    if (!dims) {
        set_err(FFT_ENULL, "dims is NULL");
        return nullptr;
    }
    if (rank < 1 || rank > 3) {
        set_err(FFT_EINVAL_N, "rank=%d must be 1, 2 or 3", rank);
        return nullptr;
    }
    if (dtype != FFT_C32) {
        set_err(FFT_EINVAL_DTYPE, "multidimensional plans are FFT_C32 only");
        return nullptr;
    }
    int64_t n = 1;
    for (int a = 0; a < rank; a++) {
        const int64_t d = dims[a];
        const int64_t hi = a == rank - 1 ? kMaxN : kMaxAxisN;
        if (!is_pow2(d) || d < 2 || d > hi) {
            set_err(FFT_EINVAL_N, "dims[%d]=%lld must be a power of two in [2, %lld]", a, (long long)d,
                    (long long)hi);
            return nullptr;
        }
        if (n > (int64_t(1) << 40) / d) {
            set_err(FFT_EINVAL_N, "the transform has more than 2^40 elements");
            return nullptr;
        }
        n *= d;
    }
    if (batch < 1) {
        set_err(FFT_EINVAL_BATCH, "batch=%lld must be >= 1", (long long)batch);
        return nullptr;
    }
    if (batch > (int64_t(1) << 40) / n) {
        set_err(FFT_EINVAL_BATCH, "n*batch=%lld*%lld exceeds 2^40 elements", (long long)n, (long long)batch);
        return nullptr;
    }
    if (sign != -1 && sign != 1) {
        set_err(FFT_EINVAL_SIGN, "sign=%d must be -1 (forward) or +1 (inverse)", sign);
        return nullptr;
    }
    if (rank == 1)
        return create_batched(dims[0], batch, sign, dtype, nullptr);
    for (int a = 0; a + 1 < rank; a++) {
        const KernelAxis* k = find_axis(ilog2(dims[a]), sign);
        if (!k) {
            set_err(FFT_EINVAL_CONFIG, "no axis kernel compiled for length %lld", (long long)dims[a]);
            return nullptr;
        }
        if ((batch * (n / dims[a]) + k->tile - 1) / k->tile > 0x7fffffffLL - 16) {
            set_err(FFT_EINVAL_BATCH, "axis %d: batch=%lld needs more than 2^31-1 workgroups", a,
                    (long long)batch);
            return nullptr;
        }
    }
    if (rank == 2 && find_nd2(ilog2(dims[0]), ilog2(dims[1]), sign) &&
        find_nd2(ilog2(dims[0]), ilog2(dims[1]), -sign))
        return create_nd2(dims, batch, sign);
    if (rank == 3 && find_nd3(ilog2(dims[0]), ilog2(dims[1]), ilog2(dims[2]), sign) &&
        find_nd3(ilog2(dims[0]), ilog2(dims[1]), ilog2(dims[2]), -sign))
        return create_nd3(dims, batch, sign);
    // The trailing axes handled by the sub-plan: the last one (batched 1D),
    // or for 3D the last two when they fit the single-pass 2D kernel.
    const bool tail2 = rank == 3 && find_nd2(ilog2(dims[1]), ilog2(dims[2]), sign) &&
                       find_nd2(ilog2(dims[1]), ilog2(dims[2]), -sign);
    mifft_plan_s* last = tail2 ? create_nd2(dims + 1, batch * dims[0], sign)
                               : create_batched(dims[rank - 1], batch * (n / dims[rank - 1]), sign, dtype, nullptr);
    if (!last)
        return nullptr;
    auto* p = new (std::nothrow) mifft_plan_s();
    if (!p) {
        free_plan(last);
        set_err(FFT_ENOMEM, "out of host memory");
        return nullptr;
    }
    p->kind = 2;
    p->n = n;
    p->batch = batch;
    p->sign = sign;
    p->dtype = dtype;
    p->scale = sign > 0 ? 1.0f / (float)n : 1.0f;
    p->device = last->device;
    p->log2n = ilog2(n);
    p->total = n * batch;
    p->rank = rank;
    p->last = last;
    for (int a = 0; a < rank; a++)
        p->dims[a] = dims[a];
    if (make_twiddles(p) != FFT_OK) {
        free_plan(p);
        return nullptr;
    }
    int log2s = ilog2(dims[rank - 1]) + (tail2 ? ilog2(dims[1]) : 0);
    p->ax_first = tail2 ? 0 : rank - 2;
    for (int a = p->ax_first; a >= 0; a--) {
        const int L = ilog2(dims[a]);
        p->ax_same[a] = find_axis(L, sign);
        p->ax_opp[a] = find_axis(L, -sign);
        p->ax_log2s[a] = log2s;
        p->ax_count[a] = batch * (n / dims[a]);
        p->ax_scale[a] = sign > 0 ? 1.0f / (float)dims[a] : 1.0f;
        log2s += L;
        const KernelAxis* k = p->ax_same[a];
        if (k->rows > 0) {
            hipError_t e = hipMalloc(&p->ax_rows[a], (size_t)k->rows * sizeof(float2));
            if (e != hipSuccess) {
                p->ax_rows[a] = nullptr;
                e == hipErrorOutOfMemory ? set_err(FFT_ENOMEM, "hipMalloc(axis twiddle rows) failed")
                                         : hip_err(e, "hipMalloc(axis twiddle rows)");
                free_plan(p);
                return nullptr;
            }
            e = launch_twiddle_rows(p->tw, p->ax_rows[a], L, k->log2ept, k->rows, nullptr);
            if (e == hipSuccess)
                e = hipStreamSynchronize(nullptr);
            if (e != hipSuccess) {
                hip_err(e, "axis twiddle rows");
                free_plan(p);
                return nullptr;
            }
        }
    }
    ok();
    return p;
}

// Byte sizes of an FFT_R32 plan's two sides: n float32 reals and n/2 + 1
// complex bins per transform.
uintptr_t real_side_bytes(fft_plan p) { return (uintptr_t)p->batch * (uintptr_t)p->n * 4; }
uintptr_t bins_side_bytes(fft_plan p) { return (uintptr_t)p->batch * (uintptr_t)(p->n / 2 + 1) * 8; }

// to_bins: for FFT_R32 plans, whether `in` holds reals and `out` bins.
int check_exec(fft_plan p, const void* in, const void* out, bool to_bins = false)
{
    if (!p)
        return set_err(FFT_ENULL, "plan is NULL");
    if (!in || !out)
        return set_err(FFT_ENULL, "in/out pointer is NULL");
    uintptr_t in_bytes = (uintptr_t)p->total * elem_bytes(p->dtype), out_bytes = in_bytes;
    // element alignment: complex64 8 bytes; 16-bit (re, im) pairs and
    // float32 reals 4 bytes
    uintptr_t in_align = elem_bytes(p->dtype), out_align = in_align;
    if (p->dtype == FFT_R32) {
        in_bytes = to_bins ? real_side_bytes(p) : bins_side_bytes(p);
        out_bytes = to_bins ? bins_side_bytes(p) : real_side_bytes(p);
        in_align = to_bins ? 4 : 8;
        out_align = to_bins ? 8 : 4;
    }
    if ((reinterpret_cast<uintptr_t>(in) & (in_align - 1)) || (reinterpret_cast<uintptr_t>(out) & (out_align - 1)))
        return set_err(FFT_EALIGN, "in (%p) must be %d-byte and out (%p) %d-byte aligned (element alignment)", in,
                       (int)in_align, out, (int)out_align);
    const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
    if (a < b + out_bytes && b < a + in_bytes)
        return set_err(FFT_EOVERLAP, "in [%p, +%zu) and out [%p, +%zu) overlap (out of place only)", in,
                       (size_t)in_bytes, out, (size_t)out_bytes);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_err(e, "hipGetDevice");
    if (dev != p->device)
        return set_err(FFT_EDEVICE, "plan was created on device %d, current device is %d", p->device, dev);
    return FFT_OK;
}

int exec_c32(fft_plan p, const void* in, void* out, int sign, float scale, hipStream_t st);

// FFT_R32: to_bins selects the real -> bins kernel; we / wi weight the
// edge and interior bins (see real.hip).  ws: the workspace of a plan above
// 2^15 (n/2 complex values per transform), NULL for the plan's own.
int exec_real(fft_plan p, const void* in, void* out, bool to_bins, float we, float wi, hipStream_t st,
              void* ws = nullptr)
{
    if (p->real_sub) {
        // Z = DFT_{n/2}(z) into the workspace, then the split (or the
        // reverse); the complex transform runs unscaled, the weights carry
        // the plan's scale
        const float2* tw = static_cast<const float2*>(p->real_tw);
        if (!ws)
            ws = p->real_ws;
        if (to_bins) {
            int rc = exec_c32(p->real_sub, in, ws, -1, 1.0f, st);
            if (rc != FFT_OK)
                return rc;
            hipError_t e = launch_real_split(0, ws, out, tw, tw + 1024, p->log2n, p->batch, we, wi, st);
            return e == hipSuccess ? ok() : hip_err(e, "real-input split launch");
        }
        hipError_t e = launch_real_split(1, in, ws, tw, tw + 1024, p->log2n, p->batch, we, wi, st);
        if (e != hipSuccess)
            return hip_err(e, "real-input split launch");
        return exec_c32(p->real_sub, ws, out, +1, 1.0f, st);
    }
    const KernelReal* k = to_bins ? p->r2c : p->c2r;
    hipError_t e = k->fn(in, out, p->rows, p->wn, p->batch, we, wi, p->grid_limit, st);
    if (e != hipSuccess)
        return hip_err(e, "real-input FFT kernel launch");
    return ok();
}

// direction: the sign of the exponent actually applied; scale as given.
int exec_c32(fft_plan p, const void* in, void* out, int sign, float scale, hipStream_t st)
{
    if (p->kind == 2 && p->nd3_same) {
        const KernelNd3* k = sign == p->sign ? p->nd3_same : p->nd3_opp;
        hipError_t e = k->fn(in, out, p->nd3_rows, p->batch, p->scale, st);
        if (e != hipSuccess)
            return hip_err(e, "3D kernel launch");
        return ok();
    }
    if (p->kind == 2 && p->nd2_same) {
        const KernelNd2* k = sign == p->sign ? p->nd2_same : p->nd2_opp;
        hipError_t e = k->fn(in, out, p->nd2_rows[0], p->nd2_rows[1], p->batch, p->scale, st);
        if (e != hipSuccess)
            return hip_err(e, "2D kernel launch");
        return ok();
    }
    if (p->kind == 2) {
        // last axis (batched 1D), then the other axes in place in `out`
        int rc = exec_c32(p->last, in, out, sign, p->last->scale, st);
        if (rc != FFT_OK)
            return rc;
        for (int a = p->ax_first; a >= 0; a--) {
            const KernelAxis* k = sign == p->sign ? p->ax_same[a] : p->ax_opp[a];
            hipError_t e = k->fn(out, p->ax_rows[a], p->ax_count[a], p->ax_log2s[a], p->ax_scale[a], st);
            if (e != hipSuccess)
                return hip_err(e, "axis kernel launch");
        }
        return ok();
    }
    if (p->kind == 1) {
        int rc = ragged_execute(p->ragged, in, out, p->tw, sign, p->sign > 0, st);
        if (rc != FFT_OK)
            return set_err(rc, "%s", ragged_last_message());
        return ok();
    }
    if (p->fs) {
        const LaunchFourStep fn = sign < 0 ? p->fs->fwd : p->fs->bwd;
        hipError_t e = fn(in, out, p->fs_rows1, p->fs_rows2, p->fs_tw, static_cast<const float2*>(p->fs_tw) + 1024,
                          p->batch, scale, st);
        if (e != hipSuccess)
            return hip_err(e, "four-step kernel launch");
        return ok();
    }
    const KernelC32* k = sign < 0 ? p->fwd : p->bwd;
    hipError_t e = k->fn(in, out, p->tw, p->rows, p->batch, scale, p->grid_limit, st);
    if (e != hipSuccess)
        return hip_err(e, "FFT kernel launch");
    return ok();
}
}  // namespace

// ------------------------------------------------------------------ C ABI
// ------------------------------------------------------------------ static scratch
// Device memory for fft_execute_static_scratch: the intermediate half-length
// spectrum of real-input plans above 2^15, for callers that cannot allocate.
// Every GPU the library runs on holds its own copy until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// it is only a stand-in for the symbol): it uses the device address that
// hipGetSymbolAddress returns, looked up once per device with that device
// current, and kept below.
namespace {
constexpr size_t kScratchBytes = MIFFT_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) float2 scratch[kScratchBytes / sizeof(float2)];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on device `dev` (the current device).
int scratch_address(int dev, void** ptr)
{
    if (dev < 0 || dev >= kMaxScratchDevices)
        return set_err(FFT_EDEVICE, "device %d: the static scratch is tracked for devices 0..%d", dev,
                       kMaxScratchDevices - 1);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* a = nullptr;
        const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_err(e, "hipGetSymbolAddress(scratch)");
        if (!a)
            return set_err(FFT_EHIP, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch_ptr[dev] = a;
    }
    *ptr = g_scratch_ptr[dev];
    return FFT_OK;
}
}  // namespace

extern "C" {

fft_plan fft_plan_create(int64_t n, int64_t batch, int sign, int dtype)
{
    return create_batched(n, batch, sign, dtype, nullptr);
}

fft_plan fft_plan_create_nd(int rank, const int64_t* dims, int64_t batch, int sign, int dtype)
{
    return create_nd(rank, dims, batch, sign, dtype);
}

fft_plan fft_plan_create_config(int64_t n, int64_t batch, int sign, int dtype, int ept, int wg, int variant)
{
    if (check_common(n, batch, sign, dtype) != FFT_OK)
        return nullptr;
    if (dtype == FFT_R32) {
        if (!is_pow2(ept) || ept < 1 || ept > 16 || !is_pow2(wg) || wg < 64 || wg > 1024 ||
            !(variant == 0 || variant == 2 || variant == 3 || variant == 6 || variant == 7)) {
            set_err(FFT_EINVAL_CONFIG, "real-input configs: ept 1..16, wg 64..1024 (powers of two), variant 0, 2, 3, 6 or 7");
            return nullptr;
        }
        Variant v{ilog2(ept), wg, variant};
        return create_batched(n, batch, sign, dtype, &v);
    }
    if (dtype != FFT_C32) {
        set_err(FFT_EINVAL_DTYPE, "fft_plan_create_config selects FP32 variants only");
        return nullptr;
    }
    if (variant != 9 && (!is_pow2(ept) || ept < 2 || ept > 16 || !is_pow2(wg) || wg < 64 || wg > 1024 ||
                         variant < 0 || (variant > 8 && variant != 11 && variant != 12))) {
        set_err(FFT_EINVAL_CONFIG, "ept=%d must be 2..16, wg=%d 64..1024 (powers of two), variant=%d 0..9, 11 or 12",
                ept, wg, variant);
        return nullptr;
    }
    if (variant == 9 && n <= 2048) {
        set_err(FFT_EINVAL_CONFIG, "the four-step variant is for n > 2048");
        return nullptr;
    }
    Variant v{variant == 9 ? 0 : ilog2(ept), variant == 9 ? 0 : wg, variant};
    return create_batched(n, batch, sign, dtype, &v);
}

fft_plan fft_plan_create_ragged_config(int64_t count, const int64_t* offsets, int sign, int dtype,
                                       const int* ept_by_log2n, int wg, int ctas_per_cu)
{
    if (dtype != FFT_C32 && dtype != FFT_C16 && dtype != FFT_CBF16) {
        set_err(FFT_EINVAL_DTYPE, "dtype %d is not FFT_C32, FFT_C16 or FFT_CBF16", dtype);
        return nullptr;
    }
    if (dtype != FFT_C32) {
        set_err(FFT_EINVAL_DTYPE, "ragged plans are FFT_C32 only");
        return nullptr;
    }
    if (sign != -1 && sign != 1) {
        set_err(FFT_EINVAL_SIGN, "sign=%d must be -1 (forward) or +1 (inverse)", sign);
        return nullptr;
    }
    if (!offsets) {
        set_err(FFT_ENULL, "offsets is NULL");
        return nullptr;
    }
    if (count < 1) {
        set_err(FFT_EINVAL_BATCH, "count=%lld must be >= 1", (long long)count);
        return nullptr;
    }
    if (offsets[0] != 0) {
        set_err(FFT_EINVAL_OFFSETS, "offsets[0]=%lld must be 0", (long long)offsets[0]);
        return nullptr;
    }
    for (int64_t b = 0; b < count; b++) {
        const int64_t len = offsets[b + 1] - offsets[b];
        if (!is_pow2(len) || len < 2 || len > 2048) {
            set_err(FFT_EINVAL_OFFSETS, "transform %lld has length %lld; lengths must be powers of two in [2, 2048]",
                    (long long)b, (long long)len);
            return nullptr;
        }
    }
    if (offsets[count] > (int64_t(1) << 40)) {
        set_err(FFT_EINVAL_OFFSETS, "total length %lld exceeds 2^40 elements", (long long)offsets[count]);
        return nullptr;
    }
    int rc = ragged_check_config(ept_by_log2n, wg, ctas_per_cu);
    if (rc != FFT_OK) {
        set_err(rc, "%s", ragged_last_message());
        return nullptr;
    }
    int dev = -1;
    if (current_gfx950(&dev) != FFT_OK)
        return nullptr;
    auto* p = new (std::nothrow) mifft_plan_s();
    if (!p) {
        set_err(FFT_ENOMEM, "out of host memory");
        return nullptr;
    }
    p->kind = 1;
    p->n = 0;
    p->batch = count;
    p->sign = sign;
    p->dtype = dtype;
    p->scale = 1.0f;
    p->device = dev;
    p->total = offsets[count];
    if (make_twiddles(p) != FFT_OK) {
        free_plan(p);
        return nullptr;
    }
    rc = ragged_create(&p->ragged, count, offsets, ept_by_log2n, wg, ctas_per_cu, dev, p->tw);
    if (rc != FFT_OK) {
        set_err(rc, "%s", ragged_last_message());
        free_plan(p);
        return nullptr;
    }
    ok();
    return p;
}

fft_plan fft_plan_create_ragged(int64_t count, const int64_t* offsets, int sign, int dtype)
{
    return fft_plan_create_ragged_config(count, offsets, sign, dtype, nullptr, 0, 0);
}

int fft_execute(fft_plan p, const void* in, void* out, void* stream)
{
    int rc = check_exec(p, in, out, p && p->sign < 0);
    if (rc != FFT_OK)
        return rc;
    if (p->dtype == FFT_R32) {
        const float s = p->scale;
        return exec_real(p, in, out, p->sign < 0, s, s, static_cast<hipStream_t>(stream));
    }
    if (p->dtype != FFT_C32)
        return fft_execute_scaled(p, in, nullptr, out, nullptr, stream);
    return exec_c32(p, in, out, p->sign, p->scale, static_cast<hipStream_t>(stream));
}

int fft_execute_static_scratch(fft_plan p, const void* in, void* out, void* stream)
{
    int rc = check_exec(p, in, out, p && p->sign < 0);
    if (rc != FFT_OK)
        return rc;
    if (!(p->dtype == FFT_R32 && p->real_sub))
        return fft_execute(p, in, out, stream);  // no workspace: the plain execute allocates nothing either
    const size_t need = (size_t)(p->n / 2) * (size_t)p->batch * sizeof(float2);
    if (need > kScratchBytes)
        return set_err(FFT_EINVAL_BATCH,
                       "n=%lld batch=%lld needs %zu bytes of scratch; the static scratch holds %zu "
                       "(at most %lld transforms of this length)",
                       (long long)p->n, (long long)p->batch, need, kScratchBytes,
                       (long long)(kScratchBytes / ((size_t)(p->n / 2) * sizeof(float2))));
    void* ws = nullptr;
    rc = scratch_address(p->device, &ws);
    if (rc != FFT_OK)
        return rc;
    const float s = p->scale;
    return exec_real(p, in, out, p->sign < 0, s, s, static_cast<hipStream_t>(stream), ws);
}

int fft_execute_adjoint(fft_plan p, const void* in, void* out, void* stream)
{
    int rc = check_exec(p, in, out, p && p->sign > 0);
    if (rc != FFT_OK)
        return rc;
    if (p->dtype == FFT_R32) {
        // adjoint of real -> bins: bins -> real with interior bins halved;
        // adjoint of bins -> real (scale 1/n): real -> bins, interior doubled
        if (p->sign < 0)
            return exec_real(p, in, out, false, 1.0f, 0.5f, static_cast<hipStream_t>(stream));
        const float s = p->scale;
        return exec_real(p, in, out, true, s, 2.0f * s, static_cast<hipStream_t>(stream));
    }
    if (p->dtype != FFT_C32) {
        // FP16/BF16: the opposite sign at the plan's scale, unit-scale output
        // (as fft_execute on these plans)
        rc = half_execute(p->half, in, nullptr, out, nullptr, p->tw, -p->sign, p->sign > 0,
                          static_cast<hipStream_t>(stream));
        if (rc != FFT_OK)
            return set_err(rc, "%s", half_last_message());
        return ok();
    }
    return exec_c32(p, in, out, -p->sign, p->scale, static_cast<hipStream_t>(stream));
}

int fft_execute_scaled(fft_plan p, const void* in, const int32_t* in_exp, void* out, int32_t* out_exp,
                       void* stream)
{
    int rc = check_exec(p, in, out);
    if (rc != FFT_OK)
        return rc;
    if (p->dtype == FFT_C32 || p->dtype == FFT_R32 || !p->half)
        return set_err(FFT_EINVAL_DTYPE, "fft_execute_scaled needs an FFT_C16 or FFT_CBF16 plan");
    if ((reinterpret_cast<uintptr_t>(in_exp) | reinterpret_cast<uintptr_t>(out_exp)) & 3)
        return set_err(FFT_EALIGN, "exponent arrays must be 4-byte aligned");
    rc = half_execute(p->half, in, in_exp, out, out_exp, p->tw, p->sign, p->sign > 0, static_cast<hipStream_t>(stream));
    if (rc != FFT_OK)
        return set_err(rc, "%s", half_last_message());
    return ok();
}

int fft_execute_loss_grad(fft_plan p, const void* x, const float* w, void* grad, float* loss, void* stream)
{
    int rc = check_exec(p, x, grad);
    if (rc != FFT_OK)
        return rc;
    if (!w || !loss)
        return set_err(FFT_ENULL, "w/loss pointer is NULL");
    if (p->kind != 0 || p->dtype != FFT_C32 || !p->lossgrad)
        return set_err(FFT_EINVAL_DTYPE, "the fused loss is provided for batched FFT_C32 plans of n <= 2048");
    if ((reinterpret_cast<uintptr_t>(w) | reinterpret_cast<uintptr_t>(loss)) & 3)
        return set_err(FFT_EALIGN, "w/loss must be 4-byte aligned");
    const uintptr_t wb = reinterpret_cast<uintptr_t>(w), gb = reinterpret_cast<uintptr_t>(grad);
    const uintptr_t wbytes = (uintptr_t)p->total * 4, gbytes = (uintptr_t)p->total * 8;
    if (wb < gb + gbytes && gb < wb + wbytes)
        return set_err(FFT_EOVERLAP, "w and grad overlap");
    const uintptr_t lb = reinterpret_cast<uintptr_t>(loss), lbytes = (uintptr_t)p->batch * 4;
    if (lb < gb + gbytes && gb < lb + lbytes)
        return set_err(FFT_EOVERLAP, "loss and grad overlap");
    const void* rows = p->lg_rows ? p->lg_rows : p->rows;
    hipError_t e = p->lossgrad->fn(x, w, grad, loss, rows, p->batch, p->scale, p->lg_grid_limit,
                                   static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return hip_err(e, "fused loss kernel launch");
    return ok();
}

void fft_plan_destroy(fft_plan p) { free_plan(p); }

int fft_plan_describe(fft_plan p, fft_plan_desc* d)
{
    if (!p || !d)
        return set_err(FFT_ENULL, "plan or desc is NULL");
    if (p->kind == 2 && p->nd3_same) {
        const KernelNd3* k = p->nd3_same;
        memset(d, 0, sizeof *d);
        d->n = p->n;
        d->batch = p->batch;
        d->sign = p->sign;
        d->dtype = FFT_C32;
        d->scale = p->scale;
        d->ept = 1 << k->log2ept;
        d->wg = k->wg;
        d->transforms_per_wg = k->arrays_per_wg;
        d->grid = (p->batch + k->arrays_per_wg - 1) / k->arrays_per_wg;
        if (k->slots) {
            const int64_t s = k->slots();
            if (s > 0 && d->grid > s)
                d->grid = s;  // workgroups walk the batch
        }
        int np = 0;
        for (int a = 2; a >= 0; a--) {  // passes in execution order: axis 2, 1, 0
            int r[8];
            const int na = schedule(k->log2n[a], k->log2ept, r);
            for (int i = 0; i < na && np < 8; i++)
                d->radices[np++] = r[i];
        }
        d->npasses = np;
        d->lds_bytes = k->lds_bytes;
        d->kind = 2;
        d->variant = 13;
        d->rank = 3;
        for (int a = 0; a < 3; a++)
            d->dims[a] = p->dims[a];
        return ok();
    }
    if (p->kind == 2 && p->nd2_same) {
        const KernelNd2* k = p->nd2_same;
        memset(d, 0, sizeof *d);
        d->n = p->n;
        d->batch = p->batch;
        d->sign = p->sign;
        d->dtype = FFT_C32;
        d->scale = p->scale;
        d->ept = 1 << k->log2ept;
        d->wg = k->wg;
        d->transforms_per_wg = k->arrays_per_wg;
        d->grid = (p->batch + k->arrays_per_wg - 1) / k->arrays_per_wg;
        if (p->nd2_grid_cap > 0 && d->grid > p->nd2_grid_cap)
            d->grid = p->nd2_grid_cap;  // workgroups walk the batch
        int r0[8], r1[8];
        const int n0 = schedule(k->log2n0, k->log2ept, r0), n1 = schedule(k->log2n1, k->log2ept, r1);
        d->npasses = std::min(8, n0 + n1);
        for (int i = 0; i < d->npasses; i++)
            d->radices[i] = i < n1 ? r1[i] : r0[i - n1];
        d->lds_bytes = k->lds_bytes;
        d->kind = 2;
        d->variant = 10;
        d->rank = 2;
        d->dims[0] = p->dims[0];
        d->dims[1] = p->dims[1];
        return ok();
    }
    if (p->kind == 2) {
        // the sub-plan's kernel shape (the last axis; for 3D with variant 10
        // the last two axes in one pass), with the whole plan's sizes
        fft_plan_describe(p->last, d);
        d->n = p->n;
        d->batch = p->batch;
        d->scale = p->scale;
        d->kind = 2;
        d->rank = p->rank;
        for (int a = 0; a < 3; a++)
            d->dims[a] = a < p->rank ? p->dims[a] : 0;
        return ok();
    }
    if (p->kind == 1) {
        memset(d, 0, sizeof *d);
        d->n = 0;
        d->batch = p->batch;
        d->sign = p->sign;
        d->dtype = p->dtype;
        d->scale = 1.0f;
        d->kind = 1;
        ragged_describe(p->ragged, &d->wg, &d->grid, &d->tiles, &d->lds_bytes, d->ept_by_log2n);
        return ok();
    }
    if (p->dtype == FFT_R32) {
        fill_desc_r32(p->n, p->batch, p->sign, p->var, p->grid_limit, d);
    } else if (p->dtype == FFT_C32) {
        fill_desc_c32(p->n, p->batch, p->sign, p->dtype, p->var, p->grid_limit, d);
    } else {
        memset(d, 0, sizeof *d);
        d->n = p->n;
        d->batch = p->batch;
        d->sign = p->sign;
        d->dtype = p->dtype;
        d->scale = p->scale;
        half_describe(p->half, d);
    }
    return ok();
}

int fft_plan_query(int64_t n, int64_t batch, int sign, int dtype, fft_plan_desc* d)
{
    if (!d)
        return set_err(FFT_ENULL, "desc is NULL");
    int rc = check_common(n, batch, sign, dtype);
    if (rc != FFT_OK)
        return rc;
    if (dtype == FFT_R32 && n > kMaxFusedRealN) {
        if (!find_fourstep(ilog2(n) - 1))
            return set_err(FFT_EINVAL_CONFIG, "no four-step kernels for the half length of n=%lld", (long long)n);
        fill_desc_r32(n, batch, sign, Variant{0, 0, 9}, 0, d);
        return ok();
    }
    if (dtype == FFT_R32) {
        const Variant v = choose_r32(ilog2(n) - 1);
        if (!find_real(ilog2(n) - 1, v.log2ept, v.wg, sign < 0 ? 0 : 1, v.kind))
            return set_err(FFT_EINVAL_CONFIG, "no real-input kernel compiled for n=%lld", (long long)n);
        fill_desc_r32(n, batch, sign, v, 0, d);
        return ok();
    }
    if (dtype != FFT_C32) {
        if (!half_supported(n))
            return set_err(FFT_EINVAL_DTYPE, "FP16/BF16 plans support n in {%s}", half_supported_lengths());
        memset(d, 0, sizeof *d);
        d->n = n;
        d->batch = batch;
        d->sign = sign;
        d->dtype = dtype;
        d->scale = sign > 0 ? 1.0f / (float)n : 1.0f;
        half_query(n, batch, d);
        return ok();
    }
    const Variant v = choose_c32(ilog2(n));
    if (v.kind == 9 ? !find_fourstep(ilog2(n)) : !find_c32(ilog2(n), v.log2ept, v.wg, sign, v.kind))
        return set_err(FFT_EINVAL_CONFIG, "no FP32 kernel compiled for n=%lld", (long long)n);
    fill_desc_c32(n, batch, sign, dtype, v, 0, d);
    return ok();
}

int fft_c32_variants(int64_t n, int* out, int cap)
{
    if (!is_pow2(n) || n < 2 || n > 2048)
        return set_err(FFT_EINVAL_N, "n=%lld: variants are listed for powers of two in [2, 2048]", (long long)n), -1;
    if (cap > 0 && !out)
        return set_err(FFT_ENULL, "out is NULL"), -1;
    const int log2n = ilog2(n);
    int count = 0;
    for (int i = 0; i < mifft::count_c32(); i++) {
        const mifft::KernelC32* k = mifft::c32_at(i);
        if (k->log2n != log2n || k->sign != -1 || !mifft::find_c32(log2n, k->log2ept, k->wg, +1, k->kind))
            continue;
        if (count < cap) {
            out[3 * count + 0] = 1 << k->log2ept;
            out[3 * count + 1] = k->wg;
            out[3 * count + 2] = k->kind;
        }
        count++;
    }
    ok();
    return count;
}

const void* fft_plan_twiddles(fft_plan p) { return p ? p->tw : nullptr; }

int fft_last_error(void) { return g_err; }
const char* fft_last_error_string(void) { return g_msg; }
const char* fft_version(void) { return "mifft 0.1 (gfx950)"; }

}  // extern "C"
