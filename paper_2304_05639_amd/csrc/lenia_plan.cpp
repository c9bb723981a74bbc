// Plans, step scheduling (ping-pong buffers, batched work list, HIP graph) and
// the tile autotuner of liblenia.so.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "lenia.h"
#include "lenia_internal.h"
#include "lenia_plan.h"

using namespace lenia;

namespace lenia {


WorldArgs WorldPlan::args_template() const
{
    WorldArgs a;
    std::memset(&a, 0, sizeof(a));
    a.w = d_w;
    a.wt = d_wtp;
    a.shc = d_shc;
    a.H = H;
    a.W = W;
    a.dt = (float)dt;
    a.eps = eps_below(eps);
    a.cnt_scale = std::ldexp(1.0f, 100);
    a.cnt_bias = -a.cnt_scale * a.eps;
    {
        const double t = (double)a.eps * (1.0 - 1.0 / 1024.0);
        float f = (float)t;
        if ((double)f > t) f = std::nextafter(f, -1.0f);
        a.skip_thr = f;
        const double to = (double)f / (double)(NK > 0 ? NK : 1);
        float g = (float)to;
        if ((double)g > to) g = std::nextafter(g, -1.0f);
        a.org_thr = g;
    }
    for (int k = 0; k < NK && k < kMaxK; ++k) {
        if (!gm.empty()) {
            a.gm[k] = (float)gm[k];
            a.gs[k] = (float)gs[k];
            a.gh[k] = (float)gh[k];
        }
    }
    return a;
}

static lenia_status dmalloc(lenia_plan_t p, void** ptr, size_t bytes)
{
    *ptr = nullptr;
    if (bytes == 0) return LENIA_OK;
    hipError_t e = device_alloc(ptr, bytes);
    if (e != hipSuccess) {
        return set_error(LENIA_ERR_OUT_OF_MEMORY,
                         "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                             hipGetErrorString(e));
    }
    p->allocations.push_back(*ptr);
    p->ws_bytes += bytes;
    return LENIA_OK;
}

lenia_status debug_checks(lenia_plan_t p, const DebugBuf* bufs, int n, hipStream_t s)
{
    if (!p->check_finite) return LENIA_OK;
    for (int i = 0; i < n; ++i) {
        if (!bufs[i].ptr || !bufs[i].bytes) continue;
        hipDeviceptr_t base = nullptr;
        size_t size = 0;
        hipError_t e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)bufs[i].ptr);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(LENIA_ERR_INVALID_ARG,
                             std::string(bufs[i].name) + " is not in a device allocation");
        }
        const size_t left = (size_t)((const char*)base + size - (const char*)bufs[i].ptr);
        if (bufs[i].bytes > left)
            return set_error(LENIA_ERR_INVALID_ARG,
                             std::string(bufs[i].name) + " needs " + std::to_string(bufs[i].bytes) +
                                 " bytes, its allocation holds " + std::to_string(left) +
                                 " from there");
    }
    hipError_t e = launch_clear_bytes((uint8_t*)p->d_nonfinite, sizeof(uint32_t), s);
    for (int i = 0; i < n && e == hipSuccess; ++i)
        if (bufs[i].ptr && bufs[i].scan)
            e = launch_find_nonfinite((const float*)bufs[i].ptr, bufs[i].bytes / sizeof(float),
                                      p->d_nonfinite, 1u << i, s);
    uint32_t found = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&found, p->d_nonfinite, sizeof(found), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "finite check");
    for (int i = 0; i < n; ++i)
        if (found & (1u << i))
            return set_error(LENIA_ERR_NONFINITE,
                             std::string("non-finite value in ") + bufs[i].name);
    return LENIA_OK;
}

static void free_all(lenia_plan_t p)
{
    if (p->graph) (void)hipGraphExecDestroy(p->graph);
    p->graph = nullptr;
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    p->capture_stream = nullptr;
    for (void* q : p->allocations) (void)hipFree(q);
    p->allocations.clear();
}

// The step kernel's compile-time kernel cores (ShellBasis<R>) against the FP64
// kernel of the plan: for every orbit and B = 1, 2, 3, the unit-height tap of
// the orbit's shell must round to the compiled value (within one float ulp,
// for a libm exp that differs in the last bits) and every other shell's must
// be 0.
template <int R>
static bool shell_basis_matches()
{
    constexpr auto& t = ShellBasis<R>::tab;
    for (int o = 0; o < ShellBasis<R>::NO; ++o)
        for (int B = 1; B <= 3; ++B)
            for (int i = 0; i < B; ++i) {
                double unit[3] = {0, 0, 0};
                unit[i] = 1.0;
                const double v = raw_kernel_tap(R, B, unit, t.a[o], t.b[o]);
                const float c = t.core[o][B - 1];
                if (shell_pair(B, i) != t.pair[o][B - 1]) {
                    if (v != 0.0) return false;
                } else if (std::fabs((double)c - v) > std::ldexp(std::fabs(v), -23)) {
                    return false;
                }
            }
    return true;
}

// Kernel tables of one world: orbit weights (K~_k at each orbit representative)
// and the shell-height gradient coefficients
//   bcoef[k][i][t] = (S_i(t) - |S_i| K~_k(t)) / Z_k,  Z_k = sum_i beta_i |S_i|,
// so that dL/dbeta_{k,i} = sum_t G_k(t) bcoef[k][i][t] with G_k(t) the orbit
// sum of dL/dK~_k.
static lenia_status build_world(lenia_plan_t p, const lenia_desc* d, WorldPlan& w,
                                hipStream_t s, std::vector<void*>& host_keep)
{
    w.H = d->H;
    w.W = d->W;
    w.C = d->n_channels;
    w.NK = d->n_kernels;
    w.R = d->R;
    w.mode = mode_of(d);
    w.dt = d->dt;
    w.eps = d->eps;
    w.table = p->table;
    lenia_status st;
    if (d->n_ring > 0) {
        // ring-decomposed kernels: the weights come from the genes in the
        // kernel, no tables; 9 gene types per kernel
        w.gene_types = 9;
        if ((st = dmalloc(p, (void**)&w.ws_A, w.a_elems() * sizeof(float))) != LENIA_OK) return st;
        return dmalloc(p, (void**)&w.ws_P, w.p_elems() * sizeof(float));
    }
    w.n_shells.assign(d->n_shells, d->n_shells + w.NK);
    w.beta.assign(d->beta, d->beta + 3 * w.NK);
    if (!d->localized) {
        w.gm.assign(d->m, d->m + w.NK);
        w.gs.assign(d->s, d->s + w.NK);
        w.gh.assign(d->h, d->h + w.NK);
    }
    std::vector<int> oa, ob;
    orbit_list(w.R, oa, ob);
    w.n_orbits = (int)oa.size();
    const int NO = w.n_orbits;
    std::vector<float> hw((size_t)w.NK * NO), hb((size_t)w.NK * 3 * NO, 0.f);
    for (int k = 0; k < w.NK; ++k) {
        const int B = w.n_shells[k];
        const double* beta = &w.beta[3 * k];
        const double z = raw_kernel_sum(w.R, B, beta);
        // |S_i|: sum over all taps of shell i's basis
        double size[3] = {0, 0, 0};
        for (int dy = -w.R; dy <= w.R; ++dy)
            for (int dx = -w.R; dx <= w.R; ++dx)
                for (int i = 0; i < B; ++i) {
                    double unit[3] = {0, 0, 0};
                    unit[i] = 1.0;
                    size[i] += raw_kernel_tap(w.R, B, unit, dy, dx);
                }
        for (int t = 0; t < NO; ++t) {
            const double kt = raw_kernel_tap(w.R, B, beta, oa[t], ob[t]) / z;
            hw[(size_t)k * NO + t] = (float)kt;
            for (int i = 0; i < B; ++i) {
                double unit[3] = {0, 0, 0};
                unit[i] = 1.0;
                const double si = raw_kernel_tap(w.R, B, unit, oa[t], ob[t]);
                hb[((size_t)k * 3 + i) * NO + t] = (float)((si - size[i] * kt) / z);
            }
        }
    }
    // the same weights ordered (orbit, source channel, slot of the kernel among
    // the kernels reading that channel), 8 slots per source
    const int kps = (p->table == TABLE_3x15) ? Table3x15::KPS : Table1x1::KPS;
    // orbit order of the step kernel's loops: axis (a,0), diagonal (a,a),
    // then general (a,b) with 0 < b < a, each by increasing a (then b)
    std::vector<int> korder;
    {
        auto index_of = [&](int a, int b) {
            for (int t = 0; t < NO; ++t)
                if (oa[t] == a && ob[t] == b) return t;
            return -1;
        };
        for (int a = 1; a < w.R; ++a) korder.push_back(index_of(a, 0));
        for (int a = 1; 2 * a * a < w.R * w.R; ++a) korder.push_back(index_of(a, a));
        for (int a = 2; a < w.R; ++a)
            for (int b = 1; b < a && a * a + b * b < w.R * w.R; ++b) korder.push_back(index_of(a, b));
    }
    if ((int)korder.size() != NO) return set_error(LENIA_ERR_STATE, "orbit enumeration mismatch");
    std::vector<float> hwt((size_t)NO * w.C * 8, 0.f);
    for (int i = 0; i < NO; ++i)
        for (int sc = 0; sc < w.C; ++sc)
            for (int j = 0; j < kps; ++j) {
                const int k = (p->table == TABLE_3x15) ? Table3x15::kidx[sc][j] : Table1x1::kidx[sc][j];
                hwt[((size_t)i * w.C + sc) * 8 + j] = hw[(size_t)k * NO + korder[i]];
            }
    if ((st = dmalloc(p, (void**)&w.d_wt, hwt.size() * sizeof(float))) != LENIA_OK) return st;
    {
        float* keep_t = new float[hwt.size()];
        std::memcpy(keep_t, hwt.data(), hwt.size() * sizeof(float));
        host_keep.push_back(keep_t);
        hipError_t e0 = hipMemcpyAsync(w.d_wt, keep_t, hwt.size() * sizeof(float),
                                       hipMemcpyHostToDevice, s);
        if (e0 != hipSuccess) return hip_fail(e0, "uploading kernel tables");
    }
    // the same weights packed per orbit (source * KPS + slot, stride
    // wt_stride), so that the step reads an orbit's weights in one scalar load
    {
        const int C = w.C, ws = (C * kps == 1) ? 1 : 16;
        if (C * kps > ws) return set_error(LENIA_ERR_STATE, "packed weight table too small");
        std::vector<float> hwp((size_t)NO * ws, 0.f);
        for (int i = 0; i < NO; ++i)
            for (int sc = 0; sc < C; ++sc)
                for (int j = 0; j < kps; ++j) hwp[(size_t)i * ws + sc * kps + j] = hwt[((size_t)i * C + sc) * 8 + j];
        if ((st = dmalloc(p, (void**)&w.d_wtp, hwp.size() * sizeof(float))) != LENIA_OK) return st;
        float* keep_p = new float[hwp.size()];
        std::memcpy(keep_p, hwp.data(), hwp.size() * sizeof(float));
        host_keep.push_back(keep_p);
        hipError_t e0 = hipMemcpyAsync(w.d_wtp, keep_p, hwp.size() * sizeof(float), hipMemcpyHostToDevice, s);
        if (e0 != hipSuccess) return hip_fail(e0, "uploading kernel tables");
    }
    // the 15-kernel step's shell coefficients: slot (source s, j) of kernel k
    // with B shells combines the shell sums of B with beta_{k,i} / z_k
    if (p->table == TABLE_3x15 && (w.R == 12 || w.R == 13)) {
        if (!(w.R == 12 ? shell_basis_matches<12>() : shell_basis_matches<13>()))
            return set_error(LENIA_ERR_STATE, "compiled kernel cores differ from the FP64 kernel");
        std::vector<float> hsc((size_t)Table3x15::C * Table3x15::KPS * 8, 0.f);
        for (int sc = 0; sc < Table3x15::C; ++sc)
            for (int j = 0; j < Table3x15::KPS; ++j) {
                const int k = Table3x15::kidx[sc][j];
                const int B = w.n_shells[k];
                const double z = raw_kernel_sum(w.R, B, &w.beta[3 * k]);
                for (int i = 0; i < B; ++i)
                    hsc[(size_t)(sc * Table3x15::KPS + j) * 8 + shell_pair(B, i)] = (float)(w.beta[3 * k + i] / z);
            }
        if ((st = dmalloc(p, (void**)&w.d_shc, hsc.size() * sizeof(float))) != LENIA_OK) return st;
        float* keep_c = new float[hsc.size()];
        std::memcpy(keep_c, hsc.data(), hsc.size() * sizeof(float));
        host_keep.push_back(keep_c);
        hipError_t e0 = hipMemcpyAsync(w.d_shc, keep_c, hsc.size() * sizeof(float), hipMemcpyHostToDevice, s);
        if (e0 != hipSuccess) return hip_fail(e0, "uploading kernel tables");
    }
    // shell-height coefficients in the same orbit order: [orbit][source][16],
    // slot j and shell i at j * 3 + i
    std::vector<float> hbt((size_t)NO * w.C * 16, 0.f);
    for (int tt = 0; tt < NO; ++tt)
        for (int sc = 0; sc < w.C; ++sc)
            for (int j = 0; j < kps; ++j) {
                const int k = (p->table == TABLE_3x15) ? Table3x15::kidx[sc][j] : Table1x1::kidx[sc][j];
                for (int i = 0; i < 3; ++i)
                    hbt[((size_t)tt * w.C + sc) * 16 + j * 3 + i] =
                        hb[((size_t)k * 3 + i) * NO + korder[tt]];
            }
    if ((st = dmalloc(p, (void**)&w.d_bt, hbt.size() * sizeof(float))) != LENIA_OK) return st;
    if ((st = dmalloc(p, (void**)&w.d_nshells, w.NK * sizeof(int))) != LENIA_OK) return st;
    {
        float* keep_bt = new float[hbt.size()];
        std::memcpy(keep_bt, hbt.data(), hbt.size() * sizeof(float));
        host_keep.push_back(keep_bt);
        float* keep_ns = new float[w.NK];
        std::memcpy(keep_ns, w.n_shells.data(), w.NK * sizeof(int));
        host_keep.push_back(keep_ns);
        hipError_t e1 = hipMemcpyAsync(w.d_bt, keep_bt, hbt.size() * sizeof(float),
                                       hipMemcpyHostToDevice, s);
        if (e1 == hipSuccess)
            e1 = hipMemcpyAsync(w.d_nshells, keep_ns, w.NK * sizeof(int), hipMemcpyHostToDevice, s);
        if (e1 != hipSuccess) return hip_fail(e1, "uploading kernel tables");
    }
    if ((st = dmalloc(p, (void**)&w.d_w, hw.size() * sizeof(float))) != LENIA_OK) return st;
    if ((st = dmalloc(p, (void**)&w.d_bcoef, hb.size() * sizeof(float))) != LENIA_OK) return st;
    // host copies stay alive until the stream has consumed them
    float* keep_w = new float[hw.size()];
    float* keep_b = new float[hb.size()];
    std::memcpy(keep_w, hw.data(), hw.size() * sizeof(float));
    std::memcpy(keep_b, hb.data(), hb.size() * sizeof(float));
    host_keep.push_back(keep_w);
    host_keep.push_back(keep_b);
    hipError_t e = hipMemcpyAsync(w.d_w, keep_w, hw.size() * sizeof(float), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w.d_bcoef, keep_b, hb.size() * sizeof(float), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "uploading kernel tables");
    if ((st = dmalloc(p, (void**)&w.ws_A, w.a_elems() * sizeof(float))) != LENIA_OK) return st;
    if (w.mode == MODE_LOCAL_UPDATE &&
        (st = dmalloc(p, (void**)&w.ws_P, w.p_elems() * sizeof(float))) != LENIA_OK)
        return st;
    return LENIA_OK;
}

static int tiles_of(int n, int t) { return (n + t - 1) / t; }

// ---------------------------------------------------------------------------
// Autotuner: times every compiled tile on synthetic content and keeps the
// fastest; results are cached in a text file keyed by the problem.
// ---------------------------------------------------------------------------
static std::string tune_cache_path()
{
    const char* e = std::getenv("LENIA_TUNE_CACHE");
    if (e && *e) return e;
    const char* home = std::getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/lenia_mi355x_tune.txt";
}

static std::string tune_key(lenia_plan_t p)
{
    hipDeviceProp_t prop;
    std::string arch = "gfx?";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
    std::ostringstream k;
    k << arch << ":t" << p->table << ":R" << p->R << ":m" << p->mode << ":"
      << (p->batched ? "batch" : "single");
    for (size_t i = 0; i < p->worlds.size() && i < 4; ++i)
        k << ":" << p->worlds[i].H << "x" << p->worlds[i].W;
    k << ":n" << p->worlds.size();
    return k.str();
}

static bool tune_lookup(const std::string& key, int* ty, int* tx)
{
    std::ifstream f(tune_cache_path());
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        int a, b;
        if (is >> k >> a >> b && k == key) {
            *ty = a;
            *tx = b;
            found = true;
        }
    }
    return found;
}

static void tune_store(const std::string& key, int ty, int tx, double ms)
{
    const std::string path = tune_cache_path();
    const size_t slash = path.find_last_of('/');
    if (slash != std::string::npos) {
        // create missing parent directories
        const std::string dir = path.substr(0, slash);
        for (size_t pos = 1; pos <= dir.size(); ++pos)
            if (pos == dir.size() || dir[pos] == '/') (void)mkdir(dir.substr(0, pos).c_str(), 0755);
    }
    std::ofstream f(path, std::ios::app);
    if (f) f << key << " " << ty << " " << tx << " " << ms << "\n";
}

lenia_status fill_batch_tables(lenia_plan_t p, float* const* A, float* const* P, hipStream_t s);

static lenia_status autotune(lenia_plan_t p, hipStream_t s)
{
    int tys[16], txs[16];
    const int nc = std::min(16, step_tile_candidates(p->table, p->R, tys, txs, 16));
    const std::string key = tune_key(p);
    int bty = 0, btx = 0;
    if (tune_lookup(key, &bty, &btx)) {
        for (int i = 0; i < nc; ++i)
            if (tys[i] == bty && txs[i] == btx) {
                p->tile_y = bty;
                p->tile_x = btx;
                return LENIA_OK;
            }
    }
    // scratch outputs; inputs are the (synthetic-filled) workspaces
    std::vector<float*> outA(p->worlds.size(), nullptr), outP(p->worlds.size(), nullptr);
    lenia_status st = LENIA_OK;
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < p->worlds.size() && st == LENIA_OK; ++i) {
        WorldPlan& w = p->worlds[i];
        if ((e = device_alloc((void**)&outA[i], w.a_elems() * sizeof(float))) != hipSuccess) break;
        if (w.mode == MODE_LOCAL_UPDATE &&
            (e = device_alloc((void**)&outP[i], w.p_elems() * sizeof(float))) != hipSuccess)
            break;
        if ((e = launch_fill_synthetic(w.ws_A, w.a_elems(), w.mode == MODE_GLOBAL ? nullptr : w.ws_P,
                                       w.cells(), w.NK, s)) != hipSuccess)
            break;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double best = 1e30;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int c = 0; c < nc && e == hipSuccess; ++c) {
        const int ty = tys[c], tx = txs[c];
        // the launch arguments of this tile (for a batch, its work list in
        // device memory), built before the timed region, which holds the
        // kernel launches alone
        WorldArgs single{};
        WorldArgs* dtab = nullptr;
        int2* ditems = nullptr;
        int n_items = 0;
        if (!p->batched) {
            WorldPlan& w = p->worlds[0];
            single = w.args_template();
            single.A = w.ws_A;
            single.P = (w.mode == MODE_GLOBAL) ? nullptr : w.ws_P;
            single.A_out = outA[0];
            single.P_out = outP[0];
            single.tiles_x = tiles_of(w.W, tx);
            single.n_tiles = tiles_of(w.H, ty) * single.tiles_x;
        } else {
            std::vector<WorldArgs> tab(p->worlds.size());
            std::vector<int2> items;
            for (size_t i = 0; i < p->worlds.size(); ++i) {
                WorldPlan& w = p->worlds[i];
                WorldArgs a = w.args_template();
                a.A = w.ws_A;
                a.P = (w.mode == MODE_GLOBAL) ? nullptr : w.ws_P;
                a.A_out = outA[i];
                a.P_out = outP[i];
                a.tiles_x = tiles_of(w.W, tx);
                a.n_tiles = tiles_of(w.H, ty) * a.tiles_x;
                tab[i] = a;
                for (int t = 0; t < a.n_tiles; ++t) items.push_back(make_int2((int)i, t));
            }
            n_items = (int)items.size();
            e = device_alloc((void**)&dtab, tab.size() * sizeof(WorldArgs));
            if (e == hipSuccess) e = device_alloc((void**)&ditems, items.size() * sizeof(int2));
            if (e == hipSuccess)
                e = hipMemcpy(dtab, tab.data(), tab.size() * sizeof(WorldArgs), hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(ditems, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice);
        }
        float ms = 0.f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {   // rep 0 = warm-up
            e = hipEventRecord(e0, s);
            for (int it = 0; it < 3 && e == hipSuccess; ++it) {
                if (!p->batched) {
                    e = find_step_launcher(p->table, p->R, ty, tx)(single, p->mode, s);
                } else {
                    BatchList bl{dtab, ditems, n_items};
                    e = find_batch_launcher(p->table, p->R, ty, tx)(bl, p->mode, s);
                }
            }
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        }
        if (dtab) (void)hipFree(dtab);
        if (ditems) (void)hipFree(ditems);
        if (e == hipSuccess && ms < best) {
            best = ms;
            bty = ty;
            btx = tx;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (size_t i = 0; i < outA.size(); ++i) {
        if (outA[i]) (void)hipFree(outA[i]);
        if (outP[i]) (void)hipFree(outP[i]);
    }
    if (e != hipSuccess) return hip_fail(e, "autotune");
    p->tile_y = bty;
    p->tile_x = btx;
    tune_store(key, bty, btx, best / 3.0);
    return LENIA_OK;
}

// 8 x 32 cells with one cell per thread (the fastest measured tile at 4096^2
// and the one with the most parallelism for small worlds).
static void default_tile(lenia_plan_t p)
{
    int tys[16], txs[16];
    const int nc = std::min(16, step_tile_candidates(p->table, p->R, tys, txs, 16));
    p->tile_y = tys[0];
    p->tile_x = txs[0];
    for (int i = 0; i < nc; ++i)
        if (tys[i] == 8 && txs[i] == 32) {
            p->tile_y = 8;
            p->tile_x = 32;
        }
}

static lenia_status finish_tile_choice(lenia_plan_t p, const lenia_desc* d, hipStream_t s)
{
    lenia_status st = LENIA_OK;
    if (p->rings) {
        p->tile_y = 8;
        p->tile_x = 32;
        p->step_fn = find_ring_step_launcher(p->table, p->R, p->tile_y, p->tile_x);
        if (!p->step_fn) return set_error(LENIA_ERR_UNSUPPORTED, "ring form not compiled in");
        return LENIA_OK;
    }
    if (d->tile_y) {
        p->tile_y = d->tile_y;
        p->tile_x = d->tile_x;
    } else if (d->flags & LENIA_FLAG_AUTOTUNE) {
        st = autotune(p, s);
    } else {
        default_tile(p);
    }
    if (st != LENIA_OK) return st;
    p->step_fn = find_step_launcher(p->table, p->R, p->tile_y, p->tile_x);
    p->batch_fn = find_batch_launcher(p->table, p->R, p->tile_y, p->tile_x);
    if (!p->step_fn) return set_error(LENIA_ERR_UNSUPPORTED, "tile not compiled in");
    return LENIA_OK;
}

}  // namespace lenia

// ---------------------------------------------------------------------------
// C ABI: plans
// ---------------------------------------------------------------------------
static lenia_status make_plan(const lenia_desc* ds, int n, void* stream, lenia_plan_t* out,
                              bool batched)
{
    if (!out) return set_error(LENIA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ds || n < 1) return set_error(LENIA_ERR_INVALID_ARG, "no descriptors");
    for (int i = 0; i < n; ++i) {
        lenia_status st = validate(&ds[i]);
        if (st != LENIA_OK) return st;
    }
    const int table = table_of(&ds[0]), mode = mode_of(&ds[0]);
    for (int i = 1; i < n; ++i)
        if (table_of(&ds[i]) != table || mode_of(&ds[i]) != mode || ds[i].R != ds[0].R)
            return set_error(LENIA_ERR_UNSUPPORTED,
                             "worlds of a batched plan must share kernel table, gene mode and R");
    if (ds[0].conv != LENIA_CONV_AUTO && ds[0].conv != LENIA_CONV_DIRECT_F32 && batched)
        return set_error(LENIA_ERR_UNSUPPORTED, "batched plans use the direct FP32 form");
    for (int i = 0; i < n; ++i)
        if (ds[i].n_ring > 0 && batched)
            return set_error(LENIA_ERR_UNSUPPORTED, "ring-decomposed kernels run single-world plans");
    hipStream_t s = (hipStream_t)stream;
    lenia_plan_t p = new (std::nothrow) lenia_plan_;
    if (!p) return set_error(LENIA_ERR_OUT_OF_MEMORY, "host allocation failed");
    (void)hipGetDevice(&p->device);
    p->batched = batched;
    p->table = table;
    p->mode = mode;
    p->R = ds[0].R;
    p->rings = (ds[0].n_ring > 0);
    p->conv = (ds[0].conv == LENIA_CONV_AUTO) ? LENIA_CONV_DIRECT_F32 : ds[0].conv;
    p->worlds.resize(n);
    std::vector<void*> keep;
    lenia_status st = LENIA_OK;
    for (int i = 0; i < n && st == LENIA_OK; ++i) st = build_world(p, &ds[i], p->worlds[i], s, keep);
    if (st == LENIA_OK && conv_is_dft(p->conv)) {
        st = build_dft_tables(p, p->worlds[0], s, keep);
        // one kernel per step once the world fills the GPU several times over
        // (LENIA_FLAG_DFT_FUSED: always)
        WorldPlan& w0 = p->worlds[0];
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess)
            cus = 0;
        const int v = dft_valid_side(w0.R);
        const long tiles = (long)((w0.H + v - 1) / v) * (long)((w0.W + v - 1) / v);
        w0.dft_fused = (ds[0].flags & LENIA_FLAG_DFT_FUSED) || (cus > 0 && tiles >= 4L * cus);
    }
    for (int i = 0; i < n; ++i)
        if (ds[i].flags & LENIA_FLAG_CHECK_FINITE) p->check_finite = true;
    if (st == LENIA_OK && p->check_finite)
        st = dmalloc(p, (void**)&p->d_nonfinite, sizeof(uint32_t));
    if (st == LENIA_OK && batched) {
        for (int ph = 0; ph < 2 && st == LENIA_OK; ++ph) {
            void* q = nullptr;
            st = [&] {
                hipError_t e = device_alloc(&q, n * sizeof(WorldArgs));
                if (e != hipSuccess) return set_error(LENIA_ERR_OUT_OF_MEMORY, "world table");
                p->allocations.push_back(q);
                p->d_tables[ph] = (WorldArgs*)q;
                return LENIA_OK;
            }();
        }
    }
    if (st == LENIA_OK) st = finish_tile_choice(p, &ds[0], s);
    if (st == LENIA_OK && batched) {
        std::vector<int2> items;
        for (int i = 0; i < n; ++i) {
            const WorldPlan& w = p->worlds[i];
            const int nt = tiles_of(w.H, p->tile_y) * tiles_of(w.W, p->tile_x);
            for (int t = 0; t < nt; ++t) items.push_back(make_int2(i, t));
        }
        p->n_items = (int)items.size();
        void* q = nullptr;
        hipError_t e = device_alloc(&q, items.size() * sizeof(int2));
        if (e != hipSuccess) {
            st = set_error(LENIA_ERR_OUT_OF_MEMORY, "work list");
        } else {
            p->allocations.push_back(q);
            p->d_items = (int2*)q;
            e = hipMemcpyAsync(p->d_items, items.data(), items.size() * sizeof(int2),
                               hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = hip_fail(e, "uploading work list");
        }
    }
    if (st == LENIA_OK) {
        hipError_t e = hipStreamSynchronize(s);   // host table copies must outlive the upload
        if (e != hipSuccess) st = hip_fail(e, "plan upload");
    }
    for (void* q : keep) delete[] (char*)q;
    if (st != LENIA_OK) {
        free_all(p);
        delete p;
        return st;
    }
    *out = p;
    return LENIA_OK;
}

extern "C" {

lenia_status lenia_plan(const lenia_desc* d, void* stream, lenia_plan_t* out)
{
    try {
        return make_plan(d, 1, stream, out, false);
    } catch (...) {
        return set_error(LENIA_ERR_OUT_OF_MEMORY, "exception in lenia_plan");
    }
}

lenia_status lenia_plan_batched(const lenia_desc* descs, int32_t n_worlds, void* stream,
                                lenia_plan_t* out)
{
    try {
        return make_plan(descs, n_worlds, stream, out, true);
    } catch (...) {
        return set_error(LENIA_ERR_OUT_OF_MEMORY, "exception in lenia_plan_batched");
    }
}

lenia_status lenia_plan_destroy(lenia_plan_t p)
{
    if (!p) return LENIA_OK;
    try {
        (void)hipDeviceSynchronize();
        free_all(p);
        delete p;
        return LENIA_OK;
    } catch (...) {
        return set_error(LENIA_ERR_STATE, "exception in lenia_plan_destroy");
    }
}

size_t lenia_saved_bytes(lenia_plan_t p)
{
    if (!p || p->batched || p->rings) return 0;
    const WorldPlan& w = p->worlds[0];
    const size_t u = (size_t)w.NK * w.cells() * sizeof(float);
    return u + ((w.cells() + 255) / 256) * 256;
}

lenia_status lenia_plan_get_info(lenia_plan_t p, lenia_plan_info* info)
{
    if (!p || !info) return set_error(LENIA_ERR_INVALID_ARG, "NULL plan or info");
    info->conv = p->conv;
    info->tile_y = p->tile_y;
    info->tile_x = p->tile_x;
    if (conv_is_dft(p->conv))
        info->tile_y = info->tile_x = dft_valid_side(p->R);
    info->n_worlds = (int32_t)p->worlds.size();
    int64_t cells = 0;
    for (const WorldPlan& w : p->worlds) cells += (int64_t)w.cells();
    info->cells = cells;
    info->workspace_bytes = p->ws_bytes;
    info->saved_bytes = lenia_saved_bytes(p);
    return LENIA_OK;
}

// ---------------------------------------------------------------------------
// Single-world steps.  Buffers b_0 = in, b_n = out; intermediate buffers
// alternate between `out` and the plan workspace so that no launch reads and
// writes the same buffer.  In place with n odd ends in the workspace and is
// copied back.
// ---------------------------------------------------------------------------
lenia_status lenia_step(lenia_plan_t p, const float* A_in, const float* P_in, float* A_out,
                        float* P_out, int32_t n_steps, void* saved, void* stream)
{
    try {
        if (!p) return set_error(LENIA_ERR_INVALID_ARG, "plan is NULL");
        if (p->batched) return set_error(LENIA_ERR_STATE, "batched plan: use lenia_step_batched");
        if (n_steps < 0) return set_error(LENIA_ERR_INVALID_ARG, "n_steps < 0");
        if (saved && n_steps != 1) return set_error(LENIA_ERR_INVALID_ARG, "saved needs n_steps == 1");
        if (saved && p->rings)
            return set_error(LENIA_ERR_UNSUPPORTED, "no saved buffer for ring-decomposed kernels");
        WorldPlan& w = p->worlds[0];
        if (!A_in || !A_out) return set_error(LENIA_ERR_INVALID_ARG, "A_in / A_out is NULL");
        if (((uintptr_t)A_in | (uintptr_t)A_out) & 3)
            return set_error(LENIA_ERR_INVALID_ARG, "A buffers must be 4-byte aligned");
        if (w.mode != MODE_GLOBAL && !P_in) return set_error(LENIA_ERR_INVALID_ARG, "P_in is NULL");
        if (w.mode == MODE_LOCAL_UPDATE && !P_out)
            return set_error(LENIA_ERR_INVALID_ARG, "P_out is NULL");
        if (w.mode != MODE_GLOBAL && ((uintptr_t)P_in & 3))
            return set_error(LENIA_ERR_INVALID_ARG, "P buffers must be 4-byte aligned");
        if (w.mode == MODE_LOCAL_UPDATE && ((uintptr_t)P_out & 3))
            return set_error(LENIA_ERR_INVALID_ARG, "P buffers must be 4-byte aligned");
        const bool upd = (w.mode == MODE_LOCAL_UPDATE);
        if (upd && ((A_in == A_out) != (P_in == P_out)))
            return set_error(LENIA_ERR_INVALID_ARG,
                             "A and P must both be in place or both out of place");
        hipStream_t s = (hipStream_t)stream;
        const size_t abytes = w.a_elems() * sizeof(float), pbytes = w.p_elems() * sizeof(float);
        {
            const bool loc = (w.mode != MODE_GLOBAL);
            const DebugBuf db[] = {{A_in, abytes, "A_in", true},
                                   {loc ? P_in : nullptr, pbytes, "P_in", true},
                                   {A_out, abytes, "A_out", false},
                                   {upd ? P_out : nullptr, pbytes, "P_out", false},
                                   {saved, saved ? lenia_saved_bytes(p) : 0, "saved", false}};
            lenia_status dst = debug_checks(p, db, 5, s);
            if (dst != LENIA_OK) return dst;
        }
        if (n_steps == 0) {
            hipError_t e = hipSuccess;
            if (A_out != A_in) e = hipMemcpyAsync(A_out, A_in, abytes, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess && upd && P_out != P_in)
                e = hipMemcpyAsync(P_out, P_in, pbytes, hipMemcpyDeviceToDevice, s);
            return e == hipSuccess ? LENIA_OK : hip_fail(e, "copy");
        }
        const bool inplace = (A_in == A_out);
        WorldArgs a = w.args_template();
        a.tiles_x = tiles_of(w.W, p->tile_x);
        a.n_tiles = tiles_of(w.H, p->tile_y) * a.tiles_x;
        // zero-gene tile flags of the two output buffers: known only for what
        // this call has written, so cleared at its start
        const bool zero_flags = upd && !saved && !conv_is_dft(p->conv) && n_steps > 2;
        if (zero_flags) {
            if (!w.p_zero) {
                lenia_status zs = dmalloc(p, (void**)&w.p_zero, 2 * (size_t)a.n_tiles);
                if (zs != LENIA_OK) return zs;
            }
            hipError_t ze = launch_clear_bytes(w.p_zero, 2u * (uint32_t)a.n_tiles, s);
            if (ze != hipSuccess) return hip_fail(ze, "clearing tile flags");
        }
        if (saved) {
            a.U_save = (float*)saved;
            a.alpha_save = (uint8_t*)saved + (size_t)w.NK * w.cells() * sizeof(float);
        }
        const float* curA = A_in;
        const float* curP = P_in;
        for (int i = 1; i <= n_steps; ++i) {
            float *nA, *nP;
            if (i == n_steps && !inplace) {
                nA = A_out;
                nP = P_out;
            } else if (inplace) {
                // X -> ws -> X -> ws ...; odd n ends in ws
                const bool to_ws = (i % 2 == 1);
                nA = to_ws ? w.ws_A : A_out;
                nP = to_ws ? w.ws_P : P_out;
            } else {
                const bool to_ws = ((n_steps - i) % 2 == 1);
                nA = to_ws ? w.ws_A : A_out;
                nP = to_ws ? w.ws_P : P_out;
            }
            a.A = curA;
            a.P = upd ? curP : P_in;
            a.A_out = nA;
            a.P_out = upd ? nP : nullptr;
            a.p_zero = zero_flags ? w.p_zero + (nP == w.ws_P ? a.n_tiles : 0) : nullptr;
            hipError_t e;
            if (conv_is_dft(p->conv) && !saved && w.mode == MODE_LOCAL_UPDATE && w.dft_fused) {
                // the whole step in one kernel: potentials stay on chip
                e = launch_dft_step(p, w, a, s);
            } else if (conv_is_dft(p->conv)) {
                // potentials on the MFMA units into the saved buffer (or the
                // plan's workspace), then the per-cell epilogue reads them
                float* U = saved ? (float*)saved : w.dft_u;
                e = launch_dft_potentials(p, w, curA, U, s);
                if (e == hipSuccess) {
                    WorldArgs ea = a;
                    ea.U_save = nullptr;
                    e = find_epilogue_launcher(p->table)(ea, U, w.mode, s);
                }
            } else {
                e = p->step_fn(a, w.mode, s);
            }
            if (e != hipSuccess) return hip_fail(e, "step launch");
            curA = nA;
            curP = nP;
        }
        if (inplace && (n_steps % 2 == 1)) {
            hipError_t e = hipMemcpyAsync(A_out, w.ws_A, abytes, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess && upd)
                e = hipMemcpyAsync(P_out, w.ws_P, pbytes, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_fail(e, "copy back");
        }
        return LENIA_OK;
    } catch (...) {
        return set_error(LENIA_ERR_STATE, "exception in lenia_step");
    }
}

lenia_status lenia_potentials(lenia_plan_t p, const float* A, float* U, void* stream)
{
    try {
        if (!p) return set_error(LENIA_ERR_INVALID_ARG, "plan is NULL");
        if (p->batched) return set_error(LENIA_ERR_STATE, "batched plan");
        if (p->rings)
            return set_error(LENIA_ERR_UNSUPPORTED,
                             "ring-decomposed potentials depend on the genes: not available");
        if (!A || !U) return set_error(LENIA_ERR_INVALID_ARG, "A / U is NULL");
        if (((uintptr_t)A | (uintptr_t)U) & 3)
            return set_error(LENIA_ERR_INVALID_ARG, "buffers must be 4-byte aligned");
        if ((const void*)A == (const void*)U)
            return set_error(LENIA_ERR_INVALID_ARG, "U must not alias A");
        WorldPlan& w = p->worlds[0];
        hipStream_t s = (hipStream_t)stream;
        {
            const DebugBuf db[] = {{A, w.a_elems() * sizeof(float), "A", true},
                                   {U, (size_t)w.NK * w.cells() * sizeof(float), "U", false}};
            lenia_status dst = debug_checks(p, db, 2, s);
            if (dst != LENIA_OK) return dst;
        }
        hipError_t e;
        if (conv_is_dft(p->conv)) {
            e = launch_dft_potentials(p, w, A, U, s);
        } else {
            WorldArgs a = w.args_template();
            a.tiles_x = tiles_of(w.W, p->tile_x);
            a.n_tiles = tiles_of(w.H, p->tile_y) * a.tiles_x;
            a.A = A;
            a.U_save = U;
            e = p->step_fn(a, MODE_POTENTIALS, s);
        }
        return e == hipSuccess ? LENIA_OK : hip_fail(e, "potentials launch");
    } catch (...) {
        return set_error(LENIA_ERR_STATE, "exception in lenia_potentials");
    }
}

}  // extern "C"

namespace lenia {

// Phase 0 reads the caller's buffers and writes the workspaces, phase 1 the
// reverse.
lenia_status fill_batch_tables(lenia_plan_t p, float* const* A, float* const* P, hipStream_t s)
{
    const int n = (int)p->worlds.size();
    std::vector<WorldArgs> t0(n), t1(n);
    // zero-gene tile flags (as in lenia_step), two arrays per world, cleared by
    // lenia_step_batched at the start of every call
    size_t zbytes = 0;
    for (int i = 0; i < n; ++i) {
        const WorldPlan& w = p->worlds[i];
        if (w.mode == MODE_LOCAL_UPDATE)
            zbytes += 2 * (size_t)tiles_of(w.W, p->tile_x) * tiles_of(w.H, p->tile_y);
    }
    if (zbytes && !p->batch_zero) {
        lenia_status zs = dmalloc(p, (void**)&p->batch_zero, zbytes);
        if (zs != LENIA_OK) return zs;
        p->batch_zero_bytes = zbytes;
    }
    size_t zoff = 0;
    for (int i = 0; i < n; ++i) {
        WorldPlan& w = p->worlds[i];
        WorldArgs a = w.args_template();
        a.tiles_x = tiles_of(w.W, p->tile_x);
        a.n_tiles = tiles_of(w.H, p->tile_y) * a.tiles_x;
        const bool upd = (w.mode == MODE_LOCAL_UPDATE);
        if (upd && p->batch_zero) {
            a.p_zero = p->batch_zero + zoff;
            zoff += 2 * (size_t)a.n_tiles;
        }
        WorldArgs b = a;
        if (a.p_zero) b.p_zero = a.p_zero + a.n_tiles;
        a.A = A[i];
        a.P = (w.mode == MODE_GLOBAL) ? nullptr : P[i];
        a.A_out = w.ws_A;
        a.P_out = upd ? w.ws_P : nullptr;
        b.A = w.ws_A;
        b.P = (w.mode == MODE_GLOBAL) ? nullptr : (upd ? w.ws_P : P[i]);
        b.A_out = A[i];
        b.P_out = upd ? P[i] : nullptr;
        t0[i] = a;
        t1[i] = b;
    }
    hipError_t e = hipMemcpyAsync(p->d_tables[0], t0.data(), n * sizeof(WorldArgs),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->d_tables[1], t1.data(), n * sizeof(WorldArgs), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "uploading world tables");
    return LENIA_OK;
}

}  // namespace lenia

extern "C" {

// Batched steps: one launch per step over the work list; a pair of steps (phase 0 then
// phase 1) is captured into a HIP graph once per pointer set and replayed.
lenia_status lenia_step_batched(lenia_plan_t p, float* const* A, float* const* P, int32_t n_steps,
                                void* stream)
{
    try {
        if (!p) return set_error(LENIA_ERR_INVALID_ARG, "plan is NULL");
        if (!p->batched) return set_error(LENIA_ERR_STATE, "not a batched plan");
        if (n_steps < 0) return set_error(LENIA_ERR_INVALID_ARG, "n_steps < 0");
        if (!A) return set_error(LENIA_ERR_INVALID_ARG, "A is NULL");
        const int n = (int)p->worlds.size();
        if (p->mode != MODE_GLOBAL && !P) return set_error(LENIA_ERR_INVALID_ARG, "P is NULL");
        for (int i = 0; i < n; ++i) {
            if (!A[i] || ((uintptr_t)A[i] & 3))
                return set_error(LENIA_ERR_INVALID_ARG, "A[" + std::to_string(i) + "] NULL or misaligned");
            if (p->mode != MODE_GLOBAL && (!P[i] || ((uintptr_t)P[i] & 3)))
                return set_error(LENIA_ERR_INVALID_ARG, "P[" + std::to_string(i) + "] NULL or misaligned");
        }
        hipStream_t s = (hipStream_t)stream;
        for (int i = 0; i < n && p->check_finite; ++i) {
            const WorldPlan& w = p->worlds[i];
            const std::string na = "A[" + std::to_string(i) + "]", np = "P[" + std::to_string(i) + "]";
            const DebugBuf db[] = {{A[i], w.a_elems() * sizeof(float), na.c_str(), true},
                                   {P ? P[i] : nullptr, w.p_elems() * sizeof(float), np.c_str(), true}};
            lenia_status dst = debug_checks(p, db, 2, s);
            if (dst != LENIA_OK) return dst;
        }
        if (n_steps == 0) return LENIA_OK;
        std::vector<float*> va(A, A + n), vp(n, nullptr);
        if (P) vp.assign(P, P + n);
        hipError_t e = hipSuccess;
        const bool same = (va == p->graph_A && vp == p->graph_P && p->graph);
        if (!same) {
            lenia_status st = fill_batch_tables(p, A, P ? P : vp.data(), s);
            if (st != LENIA_OK) return st;
            if (p->graph) {
                (void)hipGraphExecDestroy(p->graph);
                p->graph = nullptr;
            }
            // capture the two-phase pair on the plan's private stream (the
            // caller's stream may be the legacy null stream, which cannot be
            // captured); the graph is then launched into the caller's stream
            if (!p->capture_stream) {
                e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
                if (e != hipSuccess) return hip_fail(e, "creating the capture stream");
            }
            hipStream_t cs = p->capture_stream;
            hipGraph_t g = nullptr;
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                BatchList b0{p->d_tables[0], p->d_items, p->n_items};
                BatchList b1{p->d_tables[1], p->d_items, p->n_items};
                hipError_t le = p->batch_fn(b0, p->mode, cs);
                if (le == hipSuccess) le = p->batch_fn(b1, p->mode, cs);
                e = hipStreamEndCapture(cs, &g);
                if (e == hipSuccess) e = le;
            }
            if (e == hipSuccess) e = hipGraphInstantiate(&p->graph, g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                p->graph = nullptr;
                return hip_fail(e, "graph capture");
            }
            p->graph_A = va;
            p->graph_P = vp;
        }
        // the tile flags only describe what this call writes
        if (p->batch_zero) {
            e = launch_clear_bytes(p->batch_zero, (uint32_t)p->batch_zero_bytes, s);
            if (e != hipSuccess) return hip_fail(e, "clearing tile flags");
        }
        for (int i = 0; i + 1 < n_steps && e == hipSuccess; i += 2) e = hipGraphLaunch(p->graph, s);
        if (e == hipSuccess && (n_steps % 2 == 1)) {
            // last step: caller -> workspace, then copy back
            BatchList b0{p->d_tables[0], p->d_items, p->n_items};
            e = p->batch_fn(b0, p->mode, s);
            for (int i = 0; i < n && e == hipSuccess; ++i) {
                WorldPlan& w = p->worlds[i];
                e = hipMemcpyAsync(A[i], w.ws_A, w.a_elems() * sizeof(float), hipMemcpyDeviceToDevice, s);
                if (e == hipSuccess && w.mode == MODE_LOCAL_UPDATE)
                    e = hipMemcpyAsync(P[i], w.ws_P, w.p_elems() * sizeof(float),
                                       hipMemcpyDeviceToDevice, s);
            }
        }
        if (e != hipSuccess) return hip_fail(e, "batched step");
        return LENIA_OK;
    } catch (...) {
        return set_error(LENIA_ERR_STATE, "exception in lenia_step_batched");
    }
}

}  // extern "C"
