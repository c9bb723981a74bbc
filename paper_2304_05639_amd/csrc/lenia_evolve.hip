// The environmental and random operators of Algorithm 2 around a step on
// gfx950: walls (Section 2.7), the penalizing area of exploding patterns
// (Section 2.6) and the gene updates of mutation (Section 2.5) and
// penalization (Section 2.6).  The step itself is the fused step kernel,
// asked for a per-cell flags byte (bit 0 alpha, bit 1 organic matter
// sum_k u_k > eps).
#include <cmath>
#include <cstdlib>

#include "lenia.h"
#include "lenia_device.h"
#include "lenia_internal.h"
#include "lenia_plan.h"

namespace lenia {

constexpr int kMaxOxy = 16;

// Wall cells of the state: A and all gene planes set to 0.  Each lane takes
// kWallCells cells a grid apart, so that consecutive lanes read consecutive
// mask bytes and write consecutive cells of every plane; all of a lane's mask
// bytes are read before any store, so their latencies overlap.
constexpr int kWallCells = 8;

__global__ __launch_bounds__(256) void walls_kernel(float* A, float* P, const uint8_t* walls,
                                                    uint32_t HW, int C, int NPG)
{
    const uint32_t stride = gridDim.x * 256u;
    const uint32_t i0 = blockIdx.x * 256u + threadIdx.x;
    uint8_t m[kWallCells];
#pragma unroll
    for (int k = 0; k < kWallCells; ++k) {
        const uint32_t idx = i0 + (uint32_t)k * stride;
        m[k] = (idx < HW) ? walls[idx] : 0;
    }
#pragma unroll
    for (int k = 0; k < kWallCells; ++k) {
        if (!m[k]) continue;
        const uint32_t idx = i0 + (uint32_t)k * stride;
        for (int c = 0; c < C; ++c) A[(size_t)c * HW + idx] = 0.f;
        if (P)
            for (int q = 0; q < NPG; ++q) P[(size_t)q * HW + idx] = 0.f;
    }
}

// out(x) = 1 if some cell d of the disk |d| <= r around x (on the torus) has
// bit `bit` of src clear.  A tile of TY x TX cells stages, for each of its
// TY + 2r rows, the prefix counts of clear cells over its TX + 2r columns, so
// that each disk row is one difference of two counts.  Each wave stages whole
// rows (lanes are columns): the row's clear cells become two ballots over
// columns [0, 64) and [64, TX + 2r) (TX = 64, 2r <= 32), and the prefix count
// at column j is the number of set bits below j, the lane-masked bit count.
constexpr int OXY_TY = 16, OXY_TX = 64;

__global__ __launch_bounds__(256) void disk_clear_kernel(const uint8_t* src, int bit, uint8_t* out,
                                                         int H, int W, int r)
{
    constexpr int MR = kMaxOxy;
    constexpr int RY = OXY_TY + 2 * MR, RX = OXY_TX + 2 * MR + 1;
    __shared__ uint16_t zc[RY][RX];     // zc[row][j] = clear cells among columns [0, j)
    const int tiles_x = (W + OXY_TX - 1) / OXY_TX;
    const int ty0 = (blockIdx.x / tiles_x) * OXY_TY, tx0 = (blockIdx.x % tiles_x) * OXY_TX;
    const int ny = OXY_TY + 2 * r, nx = OXY_TX + 2 * r;
    // stage the tile and its r-cell halo (wrapped): wave v takes rows v, v + 4,
    // ..., all of its loads issued before the first ballot; a single wrap
    // suffices unless the torus is smaller than tile + halo
    {
        constexpr int ROWS = (RY + 3) / 4;   // rows per wave at most
        const bool single_wrap = (H >= ny) && (W >= nx);
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const auto wrap = [&](int g, int n) {
            return single_wrap ? g + ((g < 0) ? n : 0) - ((g >= n) ? n : 0) : ((g % n) + n) % n;
        };
        const bool in0 = lane < nx, in1 = 64 + lane < nx;
        const int gx0 = wrap(tx0 + lane - r, W), gx1 = wrap(tx0 + 64 + lane - r, W);
        uint8_t v0[ROWS], v1[ROWS];
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const int row = wave + 4 * k;
            v0[k] = v1[k] = 1u << bit;        // "set" (not clear) off the staged area
            if (row < ny) {
                const size_t base = (size_t)wrap(ty0 + row - r, H) * W;
                if (in0) v0[k] = src[base + gx0];
                if (in1) v1[k] = src[base + gx1];
            }
        }
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const int row = wave + 4 * k;
            if (row < ny) {
                const uint64_t m0 = __ballot(((v0[k] >> bit) & 1) == 0);
                const uint64_t m1 = __ballot(((v1[k] >> bit) & 1) == 0);
                const unsigned below0 = __builtin_amdgcn_mbcnt_hi(
                    (unsigned)(m0 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m0, 0u));
                const unsigned below1 = __builtin_amdgcn_mbcnt_hi(
                    (unsigned)(m1 >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m1, 0u));
                zc[row][lane] = (uint16_t)below0;
                if (64 + lane <= nx) zc[row][64 + lane] = (uint16_t)(__popcll(m0) + below1);
            }
        }
    }
    __syncthreads();
    // the thread's cells: column lx, rows ly0, ly0 + 4, ..., all tested together
    // so that the counts of one disk row are read in one round trip; the disk
    // row dy spans columns [lx - w, lx + w], w the largest with w^2 + dy^2 <= r^2
    // (uniform, updated as dy runs from -r to r)
    constexpr int NQ = OXY_TY / 4;
    const int lx = threadIdx.x & 63, ly0 = threadIdx.x >> 6;
    bool hit[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) hit[q] = false;
    int w = 0;
    for (int dy = -r; dy <= r; ++dy) {
        while ((w + 1) * (w + 1) + dy * dy <= r * r) ++w;
        while (w * w + dy * dy > r * r) --w;
        const int c0 = lx + r - w, c1 = lx + r + w + 1;
        uint16_t z0[NQ], z1[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int row = ly0 + 4 * q + r + dy;
            z0[q] = zc[row][c0];
            z1[q] = zc[row][c1];
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) hit[q] = hit[q] || (z1[q] != z0[q]);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int gy = ty0 + ly0 + 4 * q, gx = tx0 + lx;
        if (gy < H && gx < W) out[(size_t)gy * W + gx] = (uint8_t)hit[q];
    }
}

// Mutation, then penalization, of one iteration, on the new gene state, one
// thread per cell.  The square's first row and column (sy0, sx0) come reduced
// to [0, H) x [0, W), so a cell's offsets from them need one conditional add.
__global__ __launch_bounds__(256) void events_kernel(float* P, const uint8_t* flags,
                                                     const uint8_t* epen, int H, int W,
                                                     int mut_plane, int sy0, int sx0, int side,
                                                     float mut_add, int pen_plane, float pen_add)
{
    const uint32_t HW = (uint32_t)H * (uint32_t)W;
    const uint32_t idx = blockIdx.x * 256u + threadIdx.x;
    if (idx >= HW || !(flags[idx] & 1)) return;       // both act only where alpha = 1
    if (mut_add != 0.f) {
        const int y = (int)(idx / (uint32_t)W), x = (int)(idx - (uint32_t)y * W);
        int oy = y - sy0, ox = x - sx0;
        oy += (oy < 0) ? H : 0;
        ox += (ox < 0) ? W : 0;
        if (oy < side && ox < side) P[(size_t)mut_plane * HW + idx] += mut_add;
    }
    if (pen_add != 0.f && epen[idx]) P[(size_t)pen_plane * HW + idx] += pen_add;
}

}  // namespace lenia

using namespace lenia;

extern "C" lenia_status lenia_step_evolve(lenia_plan_t p, float* A_in, float* P_in, float* A_out,
                                          float* P_out, int32_t n_steps, const lenia_evolution* evo,
                                          const lenia_event* events, void* stream)
{
    try {
        if (!p) return set_error(LENIA_ERR_INVALID_ARG, "plan is NULL");
        if (p->batched) return set_error(LENIA_ERR_UNSUPPORTED, "operators run single-world plans");
        if (p->rings) return set_error(LENIA_ERR_UNSUPPORTED, "operators run the shell form");
        WorldPlan& w = p->worlds[0];
        if (w.mode != MODE_LOCAL_UPDATE)
            return set_error(LENIA_ERR_UNSUPPORTED, "operators need localized, updated genes");
        if (!evo) return set_error(LENIA_ERR_INVALID_ARG, "evo is NULL");
        if (n_steps < 0) return set_error(LENIA_ERR_INVALID_ARG, "n_steps < 0");
        if (!A_in || !A_out || !P_in || !P_out)
            return set_error(LENIA_ERR_INVALID_ARG, "NULL state buffer");
        if (((uintptr_t)A_in | (uintptr_t)A_out | (uintptr_t)P_in | (uintptr_t)P_out) & 3)
            return set_error(LENIA_ERR_INVALID_ARG, "state buffers must be 4-byte aligned");
        if ((A_in == A_out) != (P_in == P_out))
            return set_error(LENIA_ERR_INVALID_ARG, "A and P must both be in place or both out of place");
        if (!std::isfinite(evo->gamma_mut) || !std::isfinite(evo->gamma_pen))
            return set_error(LENIA_ERR_INVALID_ARG, "rates must be finite");
        if (evo->mut_half < 0 || 2 * evo->mut_half > w.H || 2 * evo->mut_half > w.W)
            return set_error(LENIA_ERR_INVALID_ARG, "the mutated square must fit in the torus");
        if (evo->r_oxy < 0 || evo->r_oxy > kMaxOxy)
            return set_error(LENIA_ERR_INVALID_ARG, "r_oxy must be in [0, 16]");
        const bool mut = (evo->gamma_mut != 0.0), pen = (evo->gamma_pen != 0.0);
        if ((mut || pen) && n_steps > 0 && !events)
            return set_error(LENIA_ERR_INVALID_ARG, "events are needed when a rate is nonzero");
        for (int i = 0; i < n_steps && (mut || pen); ++i) {
            const lenia_event& e = events[i];
            if (mut && (e.mut_p < 0 || e.mut_p > 2 || e.mut_k < 0 || e.mut_k >= w.NK))
                return set_error(LENIA_ERR_INVALID_ARG, "event " + std::to_string(i) + ": mutated gene out of range");
            if (mut && (std::abs((long long)e.mut_y0) > (1ll << 30) || std::abs((long long)e.mut_x0) > (1ll << 30)))
                return set_error(LENIA_ERR_INVALID_ARG, "event " + std::to_string(i) + ": square centre beyond +-2^30");
            if (mut && !std::isfinite(e.mut_delta))
                return set_error(LENIA_ERR_INVALID_ARG, "event " + std::to_string(i) + ": delta must be finite");
            if (pen && !std::isfinite(e.pen_delta))
                return set_error(LENIA_ERR_INVALID_ARG, "event " + std::to_string(i) + ": delta must be finite");
            if (pen && (e.pen_p < 0 || e.pen_p > 1 || e.pen_k < 0 || e.pen_k >= w.NK))
                return set_error(LENIA_ERR_INVALID_ARG, "event " + std::to_string(i) + ": penalized gene must be m or s");
        }
        hipStream_t s = (hipStream_t)stream;
        const size_t cells = w.cells();
        {
            const size_t ab = w.a_elems() * sizeof(float), pb = w.p_elems() * sizeof(float);
            const DebugBuf db[] = {{A_in, ab, "A_in", true}, {P_in, pb, "P_in", true},
                                   {A_out, ab, "A_out", false}, {P_out, pb, "P_out", false},
                                   {evo->walls, cells, "walls", false}};
            lenia_status dst = debug_checks(p, db, 5, s);
            if (dst != LENIA_OK) return dst;
        }
        if (!p->evo_flags) {
            void* q = nullptr;
            if (device_alloc(&q, 3 * cells) != hipSuccess)
                return set_error(LENIA_ERR_OUT_OF_MEMORY, "operator workspace");
            p->allocations.push_back(q);
            p->ws_bytes += 3 * cells;
            p->evo_flags = (uint8_t*)q;
            p->evo_eoxy = p->evo_flags + cells;
            p->evo_epen = p->evo_eoxy + cells;
        }
        const size_t abytes = w.a_elems() * sizeof(float), pbytes = w.p_elems() * sizeof(float);
        const unsigned cell_blocks = (unsigned)((cells + 255) / 256);
        const unsigned wall_blocks = (unsigned)((cells + kWallCells * 256 - 1) / (kWallCells * 256));
        const int NPG = w.gene_types * w.NK;
        hipError_t e = hipSuccess;
        if (n_steps == 0) {
            if (evo->walls)
                hipLaunchKernelGGL(walls_kernel, dim3(wall_blocks), dim3(256), 0, s, A_in, P_in, evo->walls,
                                   (uint32_t)cells, w.C, NPG);
            if (A_out != A_in) e = hipMemcpyAsync(A_out, A_in, abytes, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess && P_out != P_in) e = hipMemcpyAsync(P_out, P_in, pbytes, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = hipGetLastError();
            return e == hipSuccess ? LENIA_OK : hip_fail(e, "operators");
        }
        const bool inplace = (A_in == A_out);
        WorldArgs a = w.args_template();
        a.tiles_x = (w.W + p->tile_x - 1) / p->tile_x;
        a.n_tiles = ((w.H + p->tile_y - 1) / p->tile_y) * a.tiles_x;
        a.flags_out = p->evo_flags;
        // zero-gene tile flags of the two output buffers, as in lenia_step (the
        // walls only write zeros and the events only touch cells where alpha
        // holds, which lie in tiles that write their genes, so neither breaks
        // them)
        const bool zero_flags = !conv_is_dft(p->conv) && n_steps > 2;
        if (zero_flags) {
            if (!w.p_zero) {
                void* q = nullptr;
                if (device_alloc(&q, 2 * (size_t)a.n_tiles) != hipSuccess)
                    return set_error(LENIA_ERR_OUT_OF_MEMORY, "tile flags");
                p->allocations.push_back(q);
                p->ws_bytes += 2 * (size_t)a.n_tiles;
                w.p_zero = (uint8_t*)q;
            }
            e = launch_clear_bytes(w.p_zero, 2u * (uint32_t)a.n_tiles, s);
            if (e != hipSuccess) return hip_fail(e, "clearing tile flags");
        }
        const int oxy_tiles = ((w.H + OXY_TY - 1) / OXY_TY) * ((w.W + OXY_TX - 1) / OXY_TX);
        float* curA = A_in;
        float* curP = P_in;
        for (int i = 1; i <= n_steps; ++i) {
            float *nA, *nP;
            if (i == n_steps && !inplace) {
                nA = A_out;
                nP = P_out;
            } else if (inplace) {
                const bool to_ws = (i % 2 == 1);
                nA = to_ws ? w.ws_A : A_out;
                nP = to_ws ? w.ws_P : P_out;
            } else {
                const bool to_ws = ((n_steps - i) % 2 == 1);
                nA = to_ws ? w.ws_A : A_out;
                nP = to_ws ? w.ws_P : P_out;
            }
            // 1. walls on the state the step starts from
            if (evo->walls)
                hipLaunchKernelGGL(walls_kernel, dim3(wall_blocks), dim3(256), 0, s, curA, curP, evo->walls,
                                   (uint32_t)cells, w.C, NPG);
            // 2. the step, with the flags
            a.A = curA;
            a.P = curP;
            a.A_out = nA;
            a.P_out = nP;
            a.p_zero = zero_flags ? w.p_zero + (nP == w.ws_P ? a.n_tiles : 0) : nullptr;
            if (conv_is_dft(p->conv)) {
                e = launch_dft_potentials(p, w, curA, w.dft_u, s);
                if (e == hipSuccess) e = find_epilogue_launcher(p->table)(a, w.dft_u, w.mode, s);
            } else {
                e = p->step_fn(a, w.mode, s);
            }
            if (e != hipSuccess) return hip_fail(e, "step launch");
            // 3. penalizing area, 4-5. gene updates
            if (pen) {
                hipLaunchKernelGGL(disk_clear_kernel, dim3(oxy_tiles), dim3(256), 0, s, p->evo_flags, 1,
                                   p->evo_eoxy, w.H, w.W, evo->r_oxy);
                hipLaunchKernelGGL(disk_clear_kernel, dim3(oxy_tiles), dim3(256), 0, s, p->evo_eoxy, 0,
                                   p->evo_epen, w.H, w.W, evo->r_oxy);
            }
            if (mut || pen) {
                const lenia_event& ev = events[i - 1];
                const float mut_add = mut ? (float)(evo->gamma_mut * (double)ev.mut_delta) : 0.f;
                const float pen_add = pen ? (float)(evo->gamma_pen * (double)ev.pen_delta) : 0.f;
                // the square's first row and column on the torus
                const int64_t y0 = ((int64_t)ev.mut_y0 - evo->mut_half) % w.H;
                const int64_t x0 = ((int64_t)ev.mut_x0 - evo->mut_half) % w.W;
                // an operator that is off leaves its (unchecked) fields unused
                const int mut_plane = mut ? ev.mut_p * w.NK + ev.mut_k : 0;
                const int pen_plane = pen ? ev.pen_p * w.NK + ev.pen_k : 0;
                hipLaunchKernelGGL(events_kernel, dim3(cell_blocks), dim3(256), 0, s, nP,
                                   p->evo_flags, p->evo_epen, w.H, w.W, mut_plane,
                                   (int)(y0 < 0 ? y0 + w.H : y0), (int)(x0 < 0 ? x0 + w.W : x0),
                                   2 * evo->mut_half, mut_add, pen_plane, pen_add);
            }
            e = hipGetLastError();
            if (e != hipSuccess) return hip_fail(e, "operator launch");
            curA = nA;
            curP = nP;
        }
        if (inplace && (n_steps % 2 == 1)) {
            e = hipMemcpyAsync(A_out, w.ws_A, abytes, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(P_out, w.ws_P, pbytes, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_fail(e, "copy back");
        }
        return LENIA_OK;
    } catch (...) {
        return set_error(LENIA_ERR_STATE, "exception in lenia_step_evolve");
    }
}
