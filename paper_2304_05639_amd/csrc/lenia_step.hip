// Fused Lenia step for gfx950: direct torus convolution + gene diffusion +
// alpha mask + growth + clipped update in one pass over a tile.
//
// Per output tile (TY x TX cells) a 256-thread workgroup
//   1. stages the tile plus an R-cell halo of every channel of A into LDS
//      (wrapped on the torus, so tiny tori accumulate multiply-wrapped taps);
//   2. per cell, forms the potentials u_k = K~_k * A_src(k) (Section 2.1) by
//      summing each lattice-symmetry orbit of taps once per source channel and
//      multiplying by the orbit weight of each kernel reading that channel;
//   3. diffuses the 3*NK gene planes with the r_diff = 1 disk (Section 2.3),
//      forms alpha from the potentials and diffused genes (Section 2.2),
//      applies the localized growth (Section 2.4) and the clipped dt update,
//      and writes A', P' (and, on request, u_k and alpha for the adjoint).
// Output goes to buffers distinct from the inputs (the host ping-pongs).
#include <utility>

#include "lenia_internal.h"

namespace lenia {

#ifndef LENIA_MIN_WAVES
#define LENIA_MIN_WAVES 2   // minimum waves per SIMD the register budget must allow
#endif

// Block id -> tile id such that consecutive tiles land on the same XCD (the
// dispatcher deals workgroups round-robin over the 8 XCDs, each with its own
// L2): XCD x receives a contiguous band of tile rows, so halo re-reads of
// neighbouring tiles hit that XCD's L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int xcd = bid & 7, slot = bid >> 3;
    return (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// Kernel weights, per orbit t and source channel s: wt[(t * C + s) * 8 + j] is
// the weight of the j-th kernel reading channel s (slot order of the table),
// read through the constant address space: the index is uniform, so these
// are scalar loads feeding the FMAs as SGPR operands.
typedef const __attribute__((address_space(4))) float cfloat;

// Potentials of one cell: u_k = sum over offsets d of K~_k(d) A_src(k)(x + d).
// The offsets are walked orbit by orbit (a, b), 1 <= a < R, 0 <= b <= a,
// a^2 + b^2 < R^2, in the same order as Orbits<R>; each orbit's cells are
// summed once per source channel and multiplied once per kernel.  `c` points
// at the cell in the LDS tile of channel 0; channel s is CHS floats further.
template <class T, int R, int PITCH, int CHS>
__device__ __forceinline__ void conv_cell(const float* c, cfloat* __restrict__ wt,
                                          float (&u)[T::NK])
{
    float acc[T::C][T::KPS];
#pragma unroll
    for (int s = 0; s < T::C; ++s)
#pragma unroll
        for (int j = 0; j < T::KPS; ++j) acc[s][j] = 0.f;
    int t = 0;
#pragma unroll 1
    for (int a = 1; a < R; ++a) {
#pragma unroll 1
        for (int b = 0; b <= a && a * a + b * b < R * R; ++b, ++t) {
            float sum[T::C];
            if (b == 0) {
                const float* p0 = c + a * PITCH;
                const float* p1 = c - a * PITCH;
                const float* p2 = c + a;
                const float* p3 = c - a;
#pragma unroll
                for (int s = 0; s < T::C; ++s)
                    sum[s] = (p0[s * CHS] + p1[s * CHS]) + (p2[s * CHS] + p3[s * CHS]);
            } else if (b == a) {
                const float* p0 = c + a * PITCH + a;
                const float* p1 = c + a * PITCH - a;
                const float* p2 = c - a * PITCH + a;
                const float* p3 = c - a * PITCH - a;
#pragma unroll
                for (int s = 0; s < T::C; ++s)
                    sum[s] = (p0[s * CHS] + p1[s * CHS]) + (p2[s * CHS] + p3[s * CHS]);
            } else {
                const float* p0 = c + a * PITCH + b;
                const float* p1 = c + a * PITCH - b;
                const float* p2 = c - a * PITCH + b;
                const float* p3 = c - a * PITCH - b;
                const float* p4 = c + b * PITCH + a;
                const float* p5 = c + b * PITCH - a;
                const float* p6 = c - b * PITCH + a;
                const float* p7 = c - b * PITCH - a;
#pragma unroll
                for (int s = 0; s < T::C; ++s)
                    sum[s] = ((p0[s * CHS] + p1[s * CHS]) + (p2[s * CHS] + p3[s * CHS])) +
                             ((p4[s * CHS] + p5[s * CHS]) + (p6[s * CHS] + p7[s * CHS]));
            }
            cfloat* w = wt + t * (T::C * 8);
#pragma unroll
            for (int s = 0; s < T::C; ++s)
#pragma unroll
                for (int j = 0; j < T::KPS; ++j) acc[s][j] = fmaf(w[s * 8 + j], sum[s], acc[s][j]);
        }
    }
#pragma unroll
    for (int s = 0; s < T::C; ++s)
#pragma unroll
        for (int j = 0; j < T::KPS; ++j) u[T::kidx[s][j]] = acc[s][j];
}

__device__ __forceinline__ float growth(float u, float m, float s, float h)
{
    const float d = u - m;
    return h * (2.f * expf(-(d * d) / (2.f * s * s)) - 1.f);
}

__device__ __forceinline__ float clip01(float x) { return fminf(fmaxf(x, 0.f), 1.f); }

// One tile of one world.
template <class T, int R, int TY, int TX>
__device__ __forceinline__ void process_tile(const WorldArgs& wd, int tile, int mode, float* sA)
{
    constexpr int PY = TY + 2 * R, PX = TX + 2 * R;
    constexpr int PITCH = PX;
    constexpr int CHS = PY * PITCH;
    constexpr int NK = T::NK;
    constexpr int NP = 3 * NK;

    const int H = wd.H, W = wd.W;
    const size_t HW = (size_t)H * W;
    const int tyi = tile / wd.tiles_x;
    const int txi = tile - tyi * wd.tiles_x;
    const int y0 = tyi * TY, x0 = txi * TX;

    // 1. stage A (+halo, wrapped) with all of a thread's loads in flight at once
    {
        constexpr int NT = TY * TX;
        constexpr int NS = T::C * PY * PX;
        constexpr int IT = (NS + NT - 1) / NT;
        // a single wrap suffices unless the torus is smaller than tile + halo
        const bool single_wrap = (H >= TY + R) && (W >= TX + R);
        float v[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int i = threadIdx.x + it * NT;
            if (i < NS) {
                const int c = i / (PY * PX);
                const int r = i - c * (PY * PX);
                const int yy = r / PX;
                const int xx = r - yy * PX;
                int gy = y0 + yy - R, gx = x0 + xx - R;
                if (single_wrap) {
                    gy += (gy < 0) ? H : 0;
                    gy -= (gy >= H) ? H : 0;
                    gx += (gx < 0) ? W : 0;
                    gx -= (gx >= W) ? W : 0;
                } else {
                    gy = ((gy % H) + H) % H;
                    gx = ((gx % W) + W) % W;
                }
                v[it] = wd.A[(size_t)c * HW + (size_t)gy * W + gx];
            }
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int i = threadIdx.x + it * NT;
            if (i < NS) sA[i] = v[it];
        }
    }
    __syncthreads();

    // one output cell per thread (no cell loop: nothing for the compiler to
    // hoist across cells)
    {
        const int cell = threadIdx.x;
        const int ly = cell / TX;
        const int lx = cell - ly * TX;
        const int gy = y0 + ly, gx = x0 + lx;
        if (gy >= H || gx >= W) return;

        // 2. potentials
        float u[NK];
        conv_cell<T, R, PITCH, CHS>(sA + (ly + R) * PITCH + (lx + R), (cfloat*)wd.wt, u);

        const size_t oc = (size_t)gy * W + gx;
        const float eps = wd.eps;
        float sum[T::C];
#pragma unroll
        for (int c = 0; c < T::C; ++c) sum[c] = 0.f;

        if (mode == MODE_LOCAL_UPDATE) {
            // 3a. diffusion of every gene plane, alpha
            const int ym = (gy == 0) ? H - 1 : gy - 1;
            const int yp = (gy == H - 1) ? 0 : gy + 1;
            const int xm = (gx == 0) ? W - 1 : gx - 1;
            const int xp = (gx == W - 1) ? 0 : gx + 1;
            const size_t ou = (size_t)ym * W + gx, od = (size_t)yp * W + gx;
            const size_t ol = (size_t)gy * W + xm, orr = (size_t)gy * W + xp;
            // alpha needs every potential above the cutoff; where one is not,
            // the genes are masked to 0 and need not be read at all
            bool alpha = true;
#pragma unroll
            for (int k = 0; k < NK; ++k) alpha = alpha && (u[k] > eps);
            float pd[NP];
            if (alpha) {
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    const float* pl = wd.P + (size_t)q * HW;
                    const float vu = pl[ou], vl = pl[ol], vc = pl[oc], vr = pl[orr], vd = pl[od];
                    const float num = (((vu + vl) + vc) + vr) + vd;
                    const int n = (vu > eps) + (vl > eps) + (vc > eps) + (vr > eps) + (vd > eps);
                    const float v = (n > 0) ? clip01(num / (float)n) : 0.f;
                    pd[q] = v;
                    alpha = alpha && (v > eps);
                }
            }
            // 3b. localized growth and update
            if (alpha) {
#pragma unroll
                for (int k = 0; k < NK; ++k)
                    sum[T::dst[k]] += growth(u[k], pd[k], pd[NK + k], pd[2 * NK + k]);
            }
#pragma unroll
            for (int q = 0; q < NP; ++q) wd.P_out[(size_t)q * HW + oc] = alpha ? pd[q] : 0.f;
            if (wd.alpha_save) wd.alpha_save[oc] = alpha ? 1 : 0;
        } else if (mode == MODE_LOCAL_READONLY) {
#pragma unroll
            for (int k = 0; k < NK; ++k)
                sum[T::dst[k]] += growth(u[k], wd.P[(size_t)k * HW + oc],
                                         wd.P[(size_t)(NK + k) * HW + oc],
                                         wd.P[(size_t)(2 * NK + k) * HW + oc]);
            if (wd.alpha_save) wd.alpha_save[oc] = 1;
        } else {
#pragma unroll
            for (int k = 0; k < NK; ++k) sum[T::dst[k]] += growth(u[k], wd.gm[k], wd.gs[k], wd.gh[k]);
            if (wd.alpha_save) wd.alpha_save[oc] = 1;
        }
#pragma unroll
        for (int c = 0; c < T::C; ++c) {
            const float a = sA[c * CHS + (ly + R) * PITCH + (lx + R)];
            wd.A_out[(size_t)c * HW + oc] = clip01(a + wd.dt * sum[c]);
        }
        if (wd.U_save) {
#pragma unroll
            for (int k = 0; k < NK; ++k) wd.U_save[(size_t)k * HW + oc] = u[k];
        }
    }
}

template <class T, int R, int TY, int TX>
__global__ __launch_bounds__(TY * TX, LENIA_MIN_WAVES) void step_kernel(WorldArgs wd, int mode)
{
    __shared__ float sA[T::C * (TY + 2 * R) * (TX + 2 * R)];
    process_tile<T, R, TY, TX>(wd, xcd_tile(blockIdx.x, gridDim.x), mode, sA);
}

// Persistent form: a fixed grid walks the (world, tile) work list.
template <class T, int R, int TY, int TX>
__global__ __launch_bounds__(TY * TX, LENIA_MIN_WAVES) void step_batch_kernel(BatchList bl, int mode)
{
    __shared__ float sA[T::C * (TY + 2 * R) * (TX + 2 * R)];
    for (int i = blockIdx.x; i < bl.n_items; i += gridDim.x) {
        const int2 it = bl.items[i];
        process_tile<T, R, TY, TX>(bl.worlds[it.x], it.y, mode, sA);
        __syncthreads();   // LDS reuse by the next item
    }
}

template <class T, int R, int TY, int TX>
hipError_t launch_step(const WorldArgs& w, int mode, hipStream_t s)
{
    hipLaunchKernelGGL((step_kernel<T, R, TY, TX>), dim3(w.n_tiles), dim3(TY * TX), 0, s, w,
                       mode);
    return hipGetLastError();
}

template <class T, int R, int TY, int TX>
hipError_t launch_batch(const BatchList& b, int mode, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((step_batch_kernel<T, R, TY, TX>), dim3(grid), dim3(TY * TX), 0, s, b,
                       mode);
    return hipGetLastError();
}

struct Entry {
    int table, R, ty, tx;
    step_launch_fn step;
    batch_launch_fn batch;
};

#define LENIA_ENTRY(TB, TID, RR, TYY, TXX) \
    {TID, RR, TYY, TXX, &launch_step<TB, RR, TYY, TXX>, &launch_batch<TB, RR, TYY, TXX>}

static const Entry kEntries[] = {
    LENIA_ENTRY(Table3x15, TABLE_3x15, 12, 8, 64),
    LENIA_ENTRY(Table3x15, TABLE_3x15, 12, 4, 64),
    LENIA_ENTRY(Table3x15, TABLE_3x15, 12, 16, 32),
    LENIA_ENTRY(Table3x15, TABLE_3x15, 12, 16, 64),
    LENIA_ENTRY(Table3x15, TABLE_3x15, 13, 8, 64),
    LENIA_ENTRY(Table1x1, TABLE_1x1, 13, 8, 64),
    LENIA_ENTRY(Table1x1, TABLE_1x1, 13, 16, 64),
    LENIA_ENTRY(Table1x1, TABLE_1x1, 12, 8, 64),
};

step_launch_fn find_step_launcher(int table, int R, int ty, int tx)
{
    for (const Entry& e : kEntries)
        if (e.table == table && e.R == R && e.ty == ty && e.tx == tx) return e.step;
    return nullptr;
}

batch_launch_fn find_batch_launcher(int table, int R, int ty, int tx)
{
    for (const Entry& e : kEntries)
        if (e.table == table && e.R == R && e.ty == ty && e.tx == tx) return e.batch;
    return nullptr;
}

int step_tile_candidates(int table, int R, int* ty, int* tx, int max)
{
    int n = 0;
    for (const Entry& e : kEntries)
        if (e.table == table && e.R == R) {
            if (n < max) {
                ty[n] = e.ty;
                tx[n] = e.tx;
            }
            ++n;
        }
    return n;
}

}  // namespace lenia

namespace lenia {

// Synthetic content for timing tile candidates: A uniform in [0,1), genes in
// the ranges that keep the alpha mask on (the most expensive path).
__device__ __forceinline__ float hash01(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return (float)(x >> 8) * (1.0f / 16777216.0f);
}

__global__ void fill_synthetic_kernel(float* A, size_t nA, float* P, size_t plane, int nk)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nA; i += stride)
        A[i] = hash01((uint32_t)i * 2654435761u + 12345u);
    if (!P) return;
    const size_t nP = 3 * (size_t)nk * plane;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nP; i += stride) {
        const int p = (int)(i / ((size_t)nk * plane));
        const float r = hash01((uint32_t)i * 2246822519u + 777u);
        P[i] = (p == 0) ? 0.1f + 0.3f * r : (p == 1) ? 0.02f + 0.08f * r : 0.05f + 0.95f * r;
    }
}

hipError_t launch_fill_synthetic(float* A, size_t nA, float* P, size_t plane, int nk, hipStream_t s)
{
    hipLaunchKernelGGL(fill_synthetic_kernel, dim3(1024), dim3(256), 0, s, A, nA, P, plane, nk);
    return hipGetLastError();
}

}  // namespace lenia
