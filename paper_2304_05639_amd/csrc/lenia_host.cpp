// Host side of liblenia.so: descriptor validation, plan construction (kernel
// tables in FP64, rounded to FP32), workspace management, step scheduling and
// the C ABI of include/lenia.h.  No C++ exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lenia.h"
#include "lenia_internal.h"
#include "lenia_plan.h"

using namespace lenia;

namespace {

thread_local std::string g_last_error;

// Allocation-failure test hook (lenia_debug_fail_alloc): the number of device
// allocations still let through before the failing ones, and how many fail.
std::mutex g_fail_mu;
int g_fail_skip = 0, g_fail_count = 0;

lenia_status fail(lenia_status s, const std::string& msg)
{
    g_last_error = msg;
    return s;
}

}  // namespace

namespace lenia {

lenia_status set_error(lenia_status s, const std::string& msg) { return fail(s, msg); }

lenia_status hip_fail(hipError_t e, const char* what)
{
    return fail(LENIA_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

hipError_t device_alloc(void** ptr, size_t bytes)
{
    *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_fail_mu);
        if (g_fail_count > 0) {
            if (g_fail_skip > 0) {
                --g_fail_skip;
            } else {
                --g_fail_count;
                return hipErrorOutOfMemory;
            }
        }
    }
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *ptr = nullptr;
    }
    return e;
}

// ---------------------------------------------------------------------------
// Kernel construction (Section 2.1 normalization; ring-shell reading of the
// kernel core).  FP64 on the host.
// ---------------------------------------------------------------------------
static double shell_core(double r)
{
    if (!(r > 0.0 && r < 1.0)) return 0.0;
    return std::exp(4.0 - 1.0 / (r * (1.0 - r)));
}

// Shell index of offset (dy, dx) and the core value there; -1 outside |d| < R.
static int shell_at(int R, int B, int dy, int dx, double* core)
{
    const long d2 = (long)dy * dy + (long)dx * dx;
    if (d2 >= (long)R * R) return -1;
    const double rho = (double)B * std::sqrt((double)d2) / (double)R;
    const int i = (int)std::floor(rho);
    if (i >= B) return -1;
    *core = shell_core(rho - (double)i);
    return i;
}

double raw_kernel_tap(int R, int B, const double* beta, int dy, int dx)
{
    double c = 0.0;
    const int i = shell_at(R, B, dy, dx, &c);
    return (i < 0) ? 0.0 : beta[i] * c;
}

double raw_kernel_sum(int R, int B, const double* beta)
{
    double z = 0.0;
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) z += raw_kernel_tap(R, B, beta, dy, dx);
    return z;
}

// Orbit representatives in the order of Orbits<R>::tab.
void orbit_list(int R, std::vector<int>& a, std::vector<int>& b)
{
    a.clear();
    b.clear();
    for (int x = 0; x < R; ++x)
        for (int y = 0; y <= x; ++y)
            if (x * x + y * y > 0 && x * x + y * y < R * R) {
                a.push_back(x);
                b.push_back(y);
            }
}

int orbit_size(int a, int b) { return (b == 0 || a == b) ? 4 : 8; }

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
static bool finite(double x) { return std::isfinite(x); }

int table_of(const lenia_desc* d)
{
    if (d->n_channels == 1 && d->n_kernels == 1) {
        if (d->src[0] == Table1x1::src[0] && d->dst[0] == Table1x1::dst[0]) return TABLE_1x1;
        return -1;
    }
    if (d->n_channels == 3 && d->n_kernels == 15) {
        for (int k = 0; k < 15; ++k)
            if (d->src[k] != Table3x15::src[k] || d->dst[k] != Table3x15::dst[k]) return -1;
        return TABLE_3x15;
    }
    return -1;
}

int mode_of(const lenia_desc* d)
{
    if (!d->localized) return MODE_GLOBAL;
    return d->genotype_update ? MODE_LOCAL_UPDATE : MODE_LOCAL_READONLY;
}

lenia_status validate(const lenia_desc* d)
{
    if (!d) return fail(LENIA_ERR_INVALID_ARG, "descriptor is NULL");
    if (d->H < 1 || d->W < 1 || d->H > 65536 || d->W > 65536)
        return fail(LENIA_ERR_INVALID_ARG, "H and W must be in [1, 65536]");
    if ((int64_t)d->H * d->W >= ((int64_t)1 << 30))
        return fail(LENIA_ERR_INVALID_ARG, "H * W must be below 2^30 (a plane below 4 GiB)");
    if (d->n_channels < 1 || d->n_channels > LENIA_MAX_CHANNELS)
        return fail(LENIA_ERR_INVALID_ARG, "n_channels must be in [1, 3]");
    if (d->n_kernels < 1 || d->n_kernels > LENIA_MAX_KERNELS)
        return fail(LENIA_ERR_INVALID_ARG, "n_kernels must be in [1, 15]");
    if (d->n_ring < 0) return fail(LENIA_ERR_INVALID_ARG, "n_ring must be >= 0");
    const bool rings = (d->n_ring > 0);
    if (!d->src || !d->dst || (!rings && (!d->n_shells || !d->beta)))
        return fail(LENIA_ERR_INVALID_ARG, "src, dst, n_shells and beta must be non-NULL");
    for (int k = 0; k < d->n_kernels; ++k) {
        if (d->src[k] < 0 || d->src[k] >= d->n_channels || d->dst[k] < 0 ||
            d->dst[k] >= d->n_channels)
            return fail(LENIA_ERR_INVALID_ARG, "kernel " + std::to_string(k) +
                                                   ": src/dst channel out of range");
        if (rings) continue;   // kernels come from the genes
        if (d->n_shells[k] < 1 || d->n_shells[k] > LENIA_MAX_SHELLS)
            return fail(LENIA_ERR_INVALID_ARG, "kernel " + std::to_string(k) +
                                                   ": n_shells must be in [1, 3]");
        for (int i = 0; i < d->n_shells[k]; ++i)
            if (!finite(d->beta[3 * k + i]) || d->beta[3 * k + i] < 0.0)
                return fail(LENIA_ERR_INVALID_ARG, "kernel " + std::to_string(k) +
                                                       ": shell heights must be finite and >= 0");
    }
    if (d->R < 1) return fail(LENIA_ERR_INVALID_ARG, "R must be >= 1");
    for (int k = 0; k < d->n_kernels && !rings; ++k)
        if (!(raw_kernel_sum(d->R, d->n_shells[k], d->beta + 3 * k) > 0.0))
            return fail(LENIA_ERR_INVALID_ARG,
                        "kernel " + std::to_string(k) + " is identically zero (cannot normalize)");
    if (!finite(d->dt) || !(d->dt > 0.0)) return fail(LENIA_ERR_INVALID_ARG, "dt must be > 0");
    if (d->localized != 0 && d->localized != 1)
        return fail(LENIA_ERR_INVALID_ARG, "localized must be 0 or 1");
    if (d->genotype_update != 0 && d->genotype_update != 1)
        return fail(LENIA_ERR_INVALID_ARG, "genotype_update must be 0 or 1");
    if (d->genotype_update && !d->localized)
        return fail(LENIA_ERR_INVALID_ARG, "genotype_update needs localized genes");
    if (!d->localized) {
        if (!d->m || !d->s || !d->h)
            return fail(LENIA_ERR_INVALID_ARG, "global mode needs m, s, h");
        for (int k = 0; k < d->n_kernels; ++k)
            if (!finite(d->m[k]) || !finite(d->s[k]) || !finite(d->h[k]) || !(d->s[k] > 0.0))
                return fail(LENIA_ERR_INVALID_ARG, "global genes must be finite with s > 0");
    }
    if (!finite(d->eps) || d->eps < 0.0 || d->eps >= 1.0)
        return fail(LENIA_ERR_INVALID_ARG, "eps must be in [0, 1)");
    if (d->genotype_update && d->eps < 0x1p-64)
        return fail(LENIA_ERR_INVALID_ARG, "eps must be >= 2^-64 with genotype_update");
    if (d->genotype_update && d->r_diff < 0)
        return fail(LENIA_ERR_INVALID_ARG, "r_diff must be >= 0");
    if (d->conv < LENIA_CONV_AUTO || d->conv > LENIA_CONV_DFT_SPLIT_F16)
        return fail(LENIA_ERR_INVALID_ARG, "unknown conv form");
    if ((d->tile_y == 0) != (d->tile_x == 0) || d->tile_y < 0 || d->tile_x < 0)
        return fail(LENIA_ERR_INVALID_ARG, "tile_y and tile_x must both be 0 or both > 0");
    if (d->flags & ~(LENIA_FLAG_AUTOTUNE | LENIA_FLAG_CHECK_FINITE | LENIA_FLAG_DFT_FUSED))
        return fail(LENIA_ERR_INVALID_ARG, "unknown flags");
    if (rings && !(d->localized && d->genotype_update))
        return fail(LENIA_ERR_INVALID_ARG, "ring-decomposed kernels need localized genes with "
                                           "genotype_update");

    // what the compiled kernels cover
    const int table = table_of(d);
    if (table < 0)
        return fail(LENIA_ERR_UNSUPPORTED,
                    "kernel table not compiled in: supported are 1 channel / 1 kernel and the "
                    "3-channel / 15-kernel table (self k=0..8 src=dst=k/3; cross 0->1, 0->2, "
                    "1->0, 1->2, 2->0, 2->1)");
    if (d->genotype_update && d->r_diff != 1)
        return fail(LENIA_ERR_UNSUPPORTED, "only r_diff = 1 is compiled in");
    if (rings) {
        if (table != TABLE_3x15 || d->R != 12 || d->n_ring != 24)
            return fail(LENIA_ERR_UNSUPPORTED, "ring-decomposed kernels are compiled for 3 channels "
                                               "/ 15 kernels, R = 12 and n_ring = 24");
        if (d->conv != LENIA_CONV_AUTO && d->conv != LENIA_CONV_DIRECT_F32)
            return fail(LENIA_ERR_UNSUPPORTED, "ring-decomposed kernels use the direct form");
        if (d->flags & LENIA_FLAG_AUTOTUNE)
            return fail(LENIA_ERR_UNSUPPORTED, "no autotuning for ring-decomposed kernels");
        if (d->tile_y && !(d->tile_y == 8 && d->tile_x == 32))
            return fail(LENIA_ERR_UNSUPPORTED, "ring-decomposed kernels run 8 x 32 tiles");
        return LENIA_OK;
    }
    if (d->conv != LENIA_CONV_AUTO && d->conv != LENIA_CONV_DIRECT_F32 &&
        !conv_form_supported(d->conv, table, d->R))
        return fail(LENIA_ERR_UNSUPPORTED, "conv form not available for this table / R");
    int tys[16], txs[16];
    const int nc = step_tile_candidates(table, d->R, tys, txs, 16);
    if (nc == 0)
        return fail(LENIA_ERR_UNSUPPORTED, "no kernel compiled for R = " + std::to_string(d->R) +
                                               " with this table");
    if (d->tile_y) {
        bool ok = false;
        for (int i = 0; i < nc && i < 16; ++i) ok |= (tys[i] == d->tile_y && txs[i] == d->tile_x);
        if (!ok) return fail(LENIA_ERR_UNSUPPORTED, "requested tile not compiled in");
    }
    return LENIA_OK;
}

float eps_below(double eps)
{
    float f = (float)eps;
    if ((double)f > eps) f = std::nextafter(f, -1.0f);
    return f;
}

}  // namespace lenia

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* lenia_status_str(lenia_status s)
{
    switch (s) {
    case LENIA_OK: return "LENIA_OK";
    case LENIA_ERR_INVALID_ARG: return "LENIA_ERR_INVALID_ARG";
    case LENIA_ERR_UNSUPPORTED: return "LENIA_ERR_UNSUPPORTED";
    case LENIA_ERR_OUT_OF_MEMORY: return "LENIA_ERR_OUT_OF_MEMORY";
    case LENIA_ERR_HIP: return "LENIA_ERR_HIP";
    case LENIA_ERR_STATE: return "LENIA_ERR_STATE";
    case LENIA_ERR_NONFINITE: return "LENIA_ERR_NONFINITE";
    }
    return "LENIA_ERR_UNKNOWN";
}

const char* lenia_last_error(void) { return g_last_error.c_str(); }

void lenia_debug_fail_alloc(int32_t after, int32_t count)
{
    std::lock_guard<std::mutex> lock(g_fail_mu);
    g_fail_skip = after > 0 ? after : 0;
    g_fail_count = count > 0 ? count : 0;
}

lenia_status lenia_desc_validate(const lenia_desc* d)
{
    try {
        g_last_error.clear();
        return validate(d);
    } catch (...) {
        return fail(LENIA_ERR_INVALID_ARG, "exception during validation");
    }
}

lenia_status lenia_kernel_taps(const lenia_desc* d, int32_t k, double* out)
{
    try {
        lenia_status st = validate(d);
        if (st != LENIA_OK && st != LENIA_ERR_UNSUPPORTED) return st;
        if (k < 0 || k >= d->n_kernels || !out)
            return fail(LENIA_ERR_INVALID_ARG, "kernel index out of range or out is NULL");
        const int R = d->R, S = 2 * R + 1, B = d->n_shells[k];
        const double* beta = d->beta + 3 * k;
        const double z = raw_kernel_sum(R, B, beta);
        for (int dy = -R; dy <= R; ++dy)
            for (int dx = -R; dx <= R; ++dx)
                out[(dy + R) * S + (dx + R)] = raw_kernel_tap(R, B, beta, dy, dx) / z;
        return LENIA_OK;
    } catch (...) {
        return fail(LENIA_ERR_INVALID_ARG, "exception in lenia_kernel_taps");
    }
}

}  // extern "C"
