// Planner of ragged batches: buckets transforms by length, cuts each bucket
// into workgroup-sized tiles, orders tiles largest length first (longest
// processing time first), builds the per-length twiddle rows and uploads
// everything once.  Executes are a single launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/mifft.h"
#include "index_maps.hpp"
#include "ragged.hpp"
#include "ragged_kernel.hpp"

namespace mifft {
hipError_t launch_twiddle_rows(const void* tw, void* rows, int L, int E, int total, hipStream_t stream);

namespace {
thread_local char g_rmsg[512] = "";

int rerr(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_rmsg, sizeof g_rmsg, fmt, ap);
    va_end(ap);
    return code;
}

std::vector<KernelRagged>& reg()
{
    static std::vector<KernelRagged> r;
    return r;
}

// Rows of the twiddle table for a (log2 N, log2 EPT) schedule (none when
// one thread holds the whole transform).
int rows_total(int L, int E) { return ((1 << L) >> E) < 2 ? 0 : idx::rows_total(L, E); }

// Built-in per-length log2 EPT (index = log2 N) and launch shape.  EPT 8
// up to N = 2048 keeps the kernel at 62 VGPRs and 24 KiB of LDS, so every
// tile of a 4096-transform batch (922 tiles) is resident at once (MI355X:
// 8.2 us against 9.6-10 us with EPT 16 for N = 1024 and 2048).
const int kDefaultE[12] = {0, 1, 2, 3, 2, 2, 2, 3, 3, 3, 3, 3};
const int kDefaultWG = 256;

std::once_flag g_once;
int g_tuned_e[12];
int g_tuned_wg = 0, g_tuned_ctas = 0;

// MIFFT_TUNE_TABLE lines: "ragged <log2n> <ept>" and "ragged_wg <wg> <ctas_per_cu>".
void load_table()
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
        std::string key;
        int a = 0, b = 0;
        if (!(ss >> key >> a >> b))
            continue;
        if (key == "ragged" && a >= 1 && a <= 11 && b >= 2 && b <= 16 && (b & (b - 1)) == 0) {
            int e = 0;
            while ((1 << e) < b)
                e++;
            g_tuned_e[a] = e;
        } else if (key == "ragged_wg") {
            g_tuned_wg = a;
            g_tuned_ctas = b;
        }
    }
}
}  // namespace

void register_ragged(const KernelRagged& k) { reg().push_back(k); }
const KernelRagged* find_ragged(int wg, int maxe, int sign)
{
    for (const auto& k : reg())
        if (k.wg == wg && k.maxe == maxe && k.sign == sign)
            return &k;
    return nullptr;
}

struct RaggedPlan {
    int64_t count = 0;
    int ntiles = 0;
    int wg = 0, maxe = 0, grid = 0;
    int e_by_l[12] = {0};
    int rows_off[12] = {0};
    const KernelRagged* fwd = nullptr;
    const KernelRagged* bwd = nullptr;
    void* toff = nullptr;
    void* tiles = nullptr;
    void* rows = nullptr;
};

const char* ragged_last_message() { return g_rmsg; }

int ragged_check_config(const int* ept_by_log2n, int wg, int ctas_per_cu)
{
    if (wg != 0 && wg != 64 && wg != 128 && wg != 256)
        return rerr(FFT_EINVAL_CONFIG, "ragged workgroup size %d must be 64, 128 or 256", wg);
    if (ctas_per_cu < 0)
        return rerr(FFT_EINVAL_CONFIG, "ctas_per_cu=%d must be >= 0", ctas_per_cu);
    if (ept_by_log2n) {
        for (int L = 1; L <= 11; L++) {
            const int ept = ept_by_log2n[L];
            if (ept == 0)
                continue;
            if (ept < 2 || ept > 16 || (ept & (ept - 1)) != 0 || ept > (1 << L))
                return rerr(FFT_EINVAL_CONFIG, "ragged ept %d for n=%d must be a power of two in [2, min(16, n)]",
                            ept, 1 << L);
        }
    }
    return FFT_OK;
}

static void free_dev(RaggedPlan* rp)
{
    if (rp->toff)
        (void)hipFree(rp->toff);
    if (rp->tiles)
        (void)hipFree(rp->tiles);
    if (rp->rows)
        (void)hipFree(rp->rows);
}

void ragged_destroy(RaggedPlan* rp)
{
    if (!rp)
        return;
    free_dev(rp);
    delete rp;
}

int ragged_create(RaggedPlan** out, int64_t count, const int64_t* offsets, const int* ept_by_log2n, int wg,
                  int ctas_per_cu, int device, const void* tw)
{
    *out = nullptr;
    std::call_once(g_once, load_table);
    auto* rp = new (std::nothrow) RaggedPlan();
    if (!rp)
        return rerr(FFT_ENOMEM, "out of host memory");
    rp->count = count;
    rp->wg = wg ? wg : (g_tuned_wg ? g_tuned_wg : kDefaultWG);
    if (!ctas_per_cu && !wg)
        ctas_per_cu = g_tuned_ctas;
    // per-length elements per thread
    int64_t per_len[12] = {0};
    for (int64_t b = 0; b < count; b++) {
        const int64_t len = offsets[b + 1] - offsets[b];
        int L = 0;
        while ((int64_t(1) << L) < len)
            L++;
        per_len[L]++;
    }
    rp->maxe = 1;
    for (int L = 1; L <= 11; L++) {
        int e = kDefaultE[L];
        if (g_tuned_e[L])
            e = g_tuned_e[L];
        if (ept_by_log2n && ept_by_log2n[L]) {
            e = 0;
            while ((1 << e) < ept_by_log2n[L])
                e++;
        }
        if (e > L)
            e = L;
        // at most wg threads per transform
        while (((1 << L) >> e) > rp->wg)
            e++;
        if (e == 1 && L > 2)
            e = 2;
        rp->e_by_l[L] = e;
        if (per_len[L] && !ragged_pair_ok(L, e, rp->wg, 4)) {
            ragged_destroy(rp);
            return rerr(FFT_EINVAL_CONFIG, "no ragged kernel case for n=%d ept=%d wg=%d", 1 << L, 1 << e, rp->wg);
        }
        if (per_len[L] && e > rp->maxe)
            rp->maxe = e;
    }
    rp->maxe = rp->maxe <= 3 ? 3 : 4;
    rp->fwd = find_ragged(rp->wg, rp->maxe, -1);
    rp->bwd = find_ragged(rp->wg, rp->maxe, +1);
    if (!rp->fwd || !rp->bwd) {
        ragged_destroy(rp);
        return rerr(FFT_EINVAL_CONFIG, "no ragged kernel for wg=%d maxe=%d", rp->wg, rp->maxe);
    }

    // tiles: lengths in decreasing order, transforms in input order within a length
    std::vector<int64_t> toff;
    toff.reserve(count);
    std::vector<RaggedTile> tiles;
    for (int L = 11; L >= 1; L--) {
        if (!per_len[L])
            continue;
        const int e = rp->e_by_l[L];
        const int tpb = rp->wg / ((1 << L) >> e);
        int in_tile = 0;
        for (int64_t b = 0; b < count; b++) {
            if (offsets[b + 1] - offsets[b] != (int64_t(1) << L))
                continue;
            if (in_tile == 0)
                tiles.push_back(RaggedTile{L, e, 0, (int)toff.size()});
            toff.push_back(offsets[b]);
            tiles.back().count++;
            if (++in_tile == tpb)
                in_tile = 0;
        }
    }
    if (toff.size() > 0x7fffffff || tiles.size() > 0x7fffffff) {
        ragged_destroy(rp);
        return rerr(FFT_EINVAL_BATCH, "too many transforms for one ragged plan");
    }
    rp->ntiles = (int)tiles.size();

    // twiddle rows per length used
    int rows_total_all = 0;
    for (int L = 1; L <= 11; L++) {
        rp->rows_off[L] = rows_total_all;
        if (per_len[L])
            rows_total_all += rows_total(L, rp->e_by_l[L]);
    }

    hipError_t e = hipMalloc(&rp->toff, toff.size() * sizeof(int64_t));
    if (e == hipSuccess)
        e = hipMalloc(&rp->tiles, tiles.size() * sizeof(RaggedTile));
    if (e == hipSuccess)
        e = hipMalloc(&rp->rows, std::max(rows_total_all, 1) * 2 * sizeof(float));
    if (e != hipSuccess) {
        ragged_destroy(rp);
        return rerr(e == hipErrorOutOfMemory ? FFT_ENOMEM : FFT_EHIP, "ragged plan allocation: %s",
                    hipGetErrorString(e));
    }
    e = hipMemcpy(rp->toff, toff.data(), toff.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(rp->tiles, tiles.data(), tiles.size() * sizeof(RaggedTile), hipMemcpyHostToDevice);
    for (int L = 1; L <= 11 && e == hipSuccess; L++)
        if (per_len[L])
            e = launch_twiddle_rows(tw, static_cast<float2*>(rp->rows) + rp->rows_off[L], L, rp->e_by_l[L],
                                    rows_total(L, rp->e_by_l[L]), nullptr);
    if (e == hipSuccess)
        e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        ragged_destroy(rp);
        return rerr(FFT_EHIP, "ragged plan upload: %s", hipGetErrorString(e));
    }

    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) {
        ragged_destroy(rp);
        return rerr(FFT_EHIP, "hipDeviceGetAttribute: %s", hipGetErrorString(e));
    }
    int occ = std::min(rp->fwd->occupancy(), rp->bwd->occupancy());
    if (occ < 1)
        occ = 1;
    if (ctas_per_cu > 0 && ctas_per_cu < occ)
        occ = ctas_per_cu;
    rp->grid = (int)std::min<int64_t>((int64_t)cus * occ, std::max(rp->ntiles, 1));
    *out = rp;
    return FFT_OK;
}

int ragged_execute(RaggedPlan* rp, const void* in, void* out, const void* /*tw*/, int sign, bool inverse_scale,
                   hipStream_t stream)
{
    RaggedArgs a{};
    a.in = in;
    a.out = out;
    a.rows = rp->rows;
    a.toff = static_cast<const int64_t*>(rp->toff);
    a.tiles = static_cast<const RaggedTile*>(rp->tiles);
    a.ntiles = rp->ntiles;
    a.inv = inverse_scale ? 1 : 0;
    for (int L = 0; L < 12; L++)
        a.rows_off[L] = rp->rows_off[L];
    const KernelRagged* k = sign < 0 ? rp->fwd : rp->bwd;
    hipError_t e = k->fn(a, rp->grid, stream);
    if (e != hipSuccess)
        return rerr(FFT_EHIP, "ragged kernel launch: %s", hipGetErrorString(e));
    return FFT_OK;
}

void ragged_describe(const RaggedPlan* rp, int* wg, int64_t* grid, int64_t* tiles, int* lds_bytes, int* ept_by_log2n)
{
    *wg = rp->wg;
    *grid = rp->grid;
    *tiles = rp->ntiles;
    *lds_bytes = rp->fwd ? rp->fwd->lds_bytes : 0;
    if (ept_by_log2n)
        for (int L = 0; L < 12; L++)
            ept_by_log2n[L] = rp->e_by_l[L] ? 1 << rp->e_by_l[L] : 0;
}

}  // namespace mifft
