// Fused Lenia step for gfx950: direct torus convolution + gene diffusion +
// alpha mask + growth + clipped update in one pass over a tile.
//
// Per output tile (TY x TX cells) a workgroup (one thread per cell, or per
// vertical pair of cells in tiles of more than 256 cells)
//   1. stages the tile plus an (R-1)-cell halo of every channel of A into LDS
//      (every tap has |d| < R, so no offset exceeds R - 1 along either axis)
//      (wrapped on the torus, so tiny tori accumulate multiply-wrapped taps),
//      and, where alpha is provably 0 on the whole tile (an empty channel or
//      a dead gene plane), writes A' = clip01(A), P' = 0 and stops;
//   2. per cell, forms the potentials u_k = K~_k * A_src(k) (Section 2.1) by
//      summing each lattice-symmetry orbit of taps once per source channel,
//      then either weighting the orbit sum once per kernel reading the channel
//      (one kernel per channel), or adding it into the channel's six shell
//      sums (B = 1, 2, 3 shells, compile-time kernel cores) that each kernel
//      combines with its shell heights (the 15-kernel table);
//   3. diffuses the 3*NK gene planes with the r_diff = 1 disk (Section 2.3),
//      forms alpha from the potentials and diffused genes (Section 2.2),
//      applies the localized growth (Section 2.4) and the clipped dt update,
//      and writes A', P' (and, on request, u_k and alpha for the adjoint).
// Output goes to buffers distinct from the inputs (the host ping-pongs).
#include <algorithm>
#include <utility>

#include "lenia_device.h"
#include "lenia_internal.h"
#include "lenia_plan.h"

namespace lenia {

#ifndef LENIA_MIN_WAVES
#define LENIA_MIN_WAVES 2   // minimum waves per SIMD the register budget must allow
#endif
#ifndef LENIA_GENE_GROUP
#define LENIA_GENE_GROUP 3  // gene planes per group of disk reads in the epilogue
#endif

// Layout of the staged tile (TY + 2 HALO rows of TX + 2 HALO positions, with
// HALO = R - 1: the kernels' support is the open disk |d| < R) in LDS.  A
// position (y, x) starts at float (y * PITCH + x) * ES; its channel s is CHS
// floats further.  With three channels they are interleaved, one 16-byte
// vector per position (4th lane zero), so that a tap of every channel is one
// 128-bit LDS read at an immediate offset from the cell; a single channel is
// stored as a plane with rows padded to a multiple of 64 floats.
template <class T, int R, int TY, int TX>
struct TileLayout {
    static constexpr bool interleaved = (T::C == 3);
    static constexpr int HALO = R - 1;
    static constexpr int ES = interleaved ? 4 : 1;
    static constexpr int PITCH = interleaved ? (TX + 2 * HALO) : tile_pitch<HALO, TX>();
    static constexpr int RS = ES * PITCH;   // floats per row
    static constexpr int CHS = interleaved ? 1 : (TY + 2 * HALO) * PITCH;
    static constexpr int floats = (interleaved ? 4 : T::C) * (TY + 2 * HALO) * PITCH;
};

// Kernel weights, per orbit t and source channel s: wt[t * WS + s * KPS + j]
// is the weight of the j-th kernel reading channel s (slot order of the
// table).  The index is uniform: an orbit's weights are one scalar load (16
// floats with three channels), so the walk waits once per orbit for them.
template <class T>
constexpr int wt_stride() { return (T::C * T::KPS == 1) ? 1 : 16; }

// acc[q][s][j] += w[s][j] * sum[q][s]: one orbit's contribution to the
// potentials of the Q cells, the orbit sum of each source channel times the
// weight of each kernel reading it.
template <class T, int Q>
__device__ __forceinline__ void orbit_fma(float (&acc)[Q][T::C][T::KPS], const float (&sum)[Q][T::C],
                                          cfloat* w)
{
    typedef float wvec __attribute__((ext_vector_type(wt_stride<T>())));
    typedef const __attribute__((address_space(4))) wvec cwvec;
    const wvec wv = *(cwvec*)w;
#pragma unroll
    for (int s = 0; s < T::C; ++s)
#pragma unroll
        for (int j = 0; j < T::KPS; ++j) {
            const float wj = wv[s * T::KPS + j];
#pragma unroll
            for (int q = 0; q < Q; ++q) acc[q][s][j] = fmaf(wj, sum[q][s], acc[q][s][j]);
        }
}

// Values of one tap for the thread's Q cells (one row apart) and every
// channel: p points at the tap of the first cell.
template <class T, int Q, class L>
__device__ __forceinline__ void tap_load(float (&v)[Q][T::C], const float* p)
{
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if constexpr (L::interleaved) {
            const float4 x = *reinterpret_cast<const float4*>(p + q * L::RS);
            v[q][0] = x.x;
            v[q][1] = x.y;
            v[q][2] = x.z;
        } else {
#pragma unroll
            for (int s = 0; s < T::C; ++s) v[q][s] = p[s * L::CHS + q * L::RS];
        }
    }
}

// sum = (t0 + t1) + (t2 + t3) for each (cell, channel)
template <class T, int Q, class L>
__device__ __forceinline__ void quad_sum(float (&sum)[Q][T::C], const float* p0, const float* p1,
                                         const float* p2, const float* p3)
{
    float v0[Q][T::C], v1[Q][T::C], v2[Q][T::C], v3[Q][T::C];
    tap_load<T, Q, L>(v0, p0);
    tap_load<T, Q, L>(v1, p1);
    tap_load<T, Q, L>(v2, p2);
    tap_load<T, Q, L>(v3, p3);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int s = 0; s < T::C; ++s) sum[q][s] = (v0[q][s] + v1[q][s]) + (v2[q][s] + v3[q][s]);
}

// Potentials of Q vertically adjacent cells (c, c + RS, ...):
//   u_k = sum over offsets d of K~_k(d) A_src(k)(x + d).
// The offsets are walked orbit by orbit in three branch-free loops, in the
// order of the weight table: axis orbits (a, 0), diagonal orbits (a, a), then
// general orbits (a, b), 0 < b < a (all with a^2 + b^2 < R^2).  Each orbit's
// cells are summed once per source channel and multiplied once per kernel.
template <class T, int Q, int R, class L>
__device__ __forceinline__ void conv_cells(const float* c, cfloat* __restrict__ wt,
                                           float (&u)[Q][T::NK])
{
    constexpr int WS = wt_stride<T>();   // weights per orbit
    float acc[Q][T::C][T::KPS];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int s = 0; s < T::C; ++s)
#pragma unroll
            for (int j = 0; j < T::KPS; ++j) acc[q][s][j] = 0.f;
    constexpr int RS = L::RS, ES = L::ES;
    cfloat* w = wt;
    // axis orbits: (+-a, 0), (0, +-a)
#pragma unroll 1
    for (int a = 1; a < R; ++a, w += WS) {
        float sum[Q][T::C];
        quad_sum<T, Q, L>(sum, c + a * RS, c - a * RS, c + a * ES, c - a * ES);
        orbit_fma<T, Q>(acc, sum, w);
    }
    // diagonal orbits: (+-a, +-a)
#pragma unroll 1
    for (int a = 1; 2 * a * a < R * R; ++a, w += WS) {
        float sum[Q][T::C];
        quad_sum<T, Q, L>(sum, c + a * (RS + ES), c + a * (RS - ES), c - a * (RS - ES),
                                   c - a * (RS + ES));
        orbit_fma<T, Q>(acc, sum, w);
    }
    // general orbits: (+-a, +-b), (+-b, +-a), 0 < b < a.  For each a the four
    // base pointers (rows c +- a, columns c +- a) are formed once; the b loop is
    // unrolled so that every tap is an immediate offset from one of them.
#pragma unroll 1
    for (int a = 2; a < R; ++a) {
        const float* rp = c + a * RS;
        const float* rm = c - a * RS;
        const float* cp = c + a * ES;
        const float* cm = c - a * ES;
#pragma unroll
        for (int b = 1; b < R - 1; ++b) {
            if (b < a && a * a + b * b < R * R) {
                float s0[Q][T::C], s1[Q][T::C];
                quad_sum<T, Q, L>(s0, rp + b * ES, rp - b * ES, rm + b * ES, rm - b * ES);
                quad_sum<T, Q, L>(s1, cp + b * RS, cm + b * RS, cp - b * RS,
                                           cm - b * RS);
                float sum[Q][T::C];
#pragma unroll
                for (int q = 0; q < Q; ++q)
#pragma unroll
                    for (int s = 0; s < T::C; ++s) sum[q][s] = s0[q][s] + s1[q][s];
                orbit_fma<T, Q>(acc, sum, w);
                w += WS;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int s = 0; s < T::C; ++s)
#pragma unroll
            for (int j = 0; j < T::KPS; ++j) u[q][T::kidx[s][j]] = acc[q][s][j];
}

// The same potentials through the shell sums (ShellBasis): the orbit walk is
// unrolled at compile time, each orbit's sum (same taps, same pairwise order
// as conv_cells) enters the (B, shell) sums of B = 1, 2, 3 with the kernel
// core as an instruction constant, and each kernel then combines six of them
// with its coefficients (wd.shc).  3 multiply-adds per orbit and channel
// instead of KPS = 5, and no weight loads in the walk.
// acc[.][P][.] += k * sum (k = 0 on a shell boundary: nothing to add)
template <class T, int Q, int P>
__device__ __forceinline__ void shell_fma(float (&acc)[Q][6][T::C], const float (&sum)[Q][T::C], float k)
{
    if (k == 0.f) return;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int s = 0; s < T::C; ++s) acc[q][P][s] = fmaf(k, sum[q][s], acc[q][P][s]);
}

template <class T, int Q, class L, int R, int I>
__device__ __forceinline__ void shell_walk(float (&acc)[Q][6][T::C], const float* c)
{
    if constexpr (I < ShellBasis<R>::NO) {
        constexpr auto& t = ShellBasis<R>::tab;
        constexpr int a = t.a[I], b = t.b[I];
        constexpr int RS = L::RS, ES = L::ES;
        float sum[Q][T::C];
        if constexpr (b == 0) {
            quad_sum<T, Q, L>(sum, c + a * RS, c - a * RS, c + a * ES, c - a * ES);
        } else if constexpr (a == b) {
            quad_sum<T, Q, L>(sum, c + a * (RS + ES), c + a * (RS - ES), c - a * (RS - ES), c - a * (RS + ES));
        } else {
            const float* rp = c + a * RS;
            const float* rm = c - a * RS;
            const float* cp = c + a * ES;
            const float* cm = c - a * ES;
            float s0[Q][T::C], s1[Q][T::C];
            quad_sum<T, Q, L>(s0, rp + b * ES, rp - b * ES, rm + b * ES, rm - b * ES);
            quad_sum<T, Q, L>(s1, cp + b * RS, cm + b * RS, cp - b * RS, cm - b * RS);
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int s = 0; s < T::C; ++s) sum[q][s] = s0[q][s] + s1[q][s];
        }
        // constexpr locals: the values become instruction constants (the
        // table itself is a device global the compiler may not fold)
        constexpr float k1 = t.core[I][0], k2 = t.core[I][1], k3 = t.core[I][2];
        shell_fma<T, Q, t.pair[I][0]>(acc, sum, k1);
        shell_fma<T, Q, t.pair[I][1]>(acc, sum, k2);
        shell_fma<T, Q, t.pair[I][2]>(acc, sum, k3);
        shell_walk<T, Q, L, R, I + 1>(acc, c);
    }
}

template <class T, int Q, int R, class L>
__device__ __forceinline__ void conv_cells_shells(const float* c, cfloat* __restrict__ shc,
                                                  float (&u)[Q][T::NK])
{
    float acc[Q][6][T::C];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int p = 0; p < 6; ++p)
#pragma unroll
            for (int s = 0; s < T::C; ++s) acc[q][p][s] = 0.f;
    shell_walk<T, Q, L, R, 0>(acc, c);
    typedef float f8v __attribute__((ext_vector_type(8)));
    typedef const __attribute__((address_space(4))) f8v cf8v;
#pragma unroll
    for (int s = 0; s < T::C; ++s)
#pragma unroll
        for (int j = 0; j < T::KPS; ++j) {
            const f8v cv = *(cf8v*)(shc + (s * T::KPS + j) * 8);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                float v = cv[0] * acc[q][0][s];
#pragma unroll
                for (int p = 1; p < 6; ++p) v = fmaf(cv[p], acc[q][p][s], v);
                u[q][T::kidx[s][j]] = v;
            }
        }
}

// Gene diffusion, alpha mask, growth and update of one cell (gy, gx) given its
// potentials u and its current state a[c]; writes A' and P' (and the saved
// potentials / alpha when requested).
template <class T, bool KMAJOR = true>
__device__ __forceinline__ void epilogue_cell(const WorldArgs& wd, int mode, const float (&u)[T::NK],
                                              const float (&a)[T::C], int gy, int gx)
{
    constexpr int NK = T::NK;
    constexpr int NP = 3 * NK;
    const int H = wd.H, W = wd.W;
    const size_t HW = (size_t)H * W;
    // byte offsets within a plane fit 32 bits (a plane is below 4 GiB); every
    // plane is accessed through a scalar buffer descriptor
    const uint32_t ob = 4u * ((uint32_t)gy * (uint32_t)W + (uint32_t)gx);
    const uint32_t pb = 4u * (uint32_t)HW;
    const float eps = wd.eps;
    float sum[T::C];
#pragma unroll
    for (int c = 0; c < T::C; ++c) sum[c] = 0.f;

    if (mode == MODE_LOCAL_UPDATE) {
        // alpha needs every potential above the cutoff; where one is not, the
        // genes are masked to 0 and need not be read at all
        bool alpha = true;
#pragma unroll
        for (int k = 0; k < NK; ++k) alpha = alpha && (u[k] > eps);
        if constexpr (KMAJOR) {
            if (alpha) {
                // diffuse every gene plane (Section 2.3), kernel by kernel in table
                // order: kernel k's m, s and h disks (planes k, NK + k, 2 NK + k)
                // are read together, two kernels' reads in flight ahead of the
                // one being reduced (the scheduling barriers keep the compiler
                // from serialising them).  Each kernel's diffused genes are tested
                // against the cutoff, written out while alpha holds, and enter
                // its growth at once, so no diffused plane stays live; a cell
                // whose alpha fails gets all its genes written as 0 below.
                const NbrB nb = neighbour_bytes(gy, gx, H, W);
                const float cs = wd.cnt_scale, ncs = wd.cnt_bias;
                auto load_kernel = [&](float (&vv)[3][5], int pos) {
                    const int kk = T::kidx[pos / T::KPS][pos % T::KPS];
#pragma unroll
                    for (int p = 0; p < 3; ++p) load_disk(vv[p], plane(wd.P + (size_t)(p * NK + kk) * HW, pb), nb);
                };
                float v[3][3][5];
                load_kernel(v[0], 0);
                if (NK > 1) load_kernel(v[1], 1);
#pragma unroll
                for (int pos = 0; pos < NK; ++pos) {
                    const int k = T::kidx[pos / T::KPS][pos % T::KPS];
                    if (pos + 2 < NK) load_kernel(v[(pos + 2) % 3], pos + 2);
                    __builtin_amdgcn_sched_barrier(0);
                    const float m = diffuse_disk(v[pos % 3][0], cs, ncs);
                    const float sg = diffuse_disk(v[pos % 3][1], cs, ncs);
                    const float h = diffuse_disk(v[pos % 3][2], cs, ncs);
                    alpha = alpha && (m > eps) && (sg > eps) && (h > eps);
                    // once alpha has failed the stores go past the plane (dropped)
                    const uint32_t oa = alpha ? ob : 0xFFFFFFF0u;
                    pst_stream(plane(wd.P_out + (size_t)k * HW, pb), oa, m);
                    pst_stream(plane(wd.P_out + (size_t)(NK + k) * HW, pb), oa, sg);
                    pst_stream(plane(wd.P_out + (size_t)(2 * NK + k) * HW, pb), oa, h);
                    // growth summed per source channel, each channel's kernels in
                    // table order (the order the DFT form's fused step follows)
                    sum[T::dst[k]] = growth_acc(sum[T::dst[k]], u[k], m, sg, h);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            if (!alpha) {
#pragma unroll
                for (int c = 0; c < T::C; ++c) sum[c] = 0.f;
#pragma unroll
                for (int q = 0; q < NP; ++q) pst_stream(plane(wd.P_out + (size_t)q * HW, pb), ob, 0.f);
            }
        } else {
            float pd[NP];
            if (alpha) {
                // diffuse every gene plane (Section 2.3) and test it against the
                // cutoff.  The disks are read in groups of G planes, the next
                // group's reads issued before the current group is reduced, so a
                // wave has one round trip in flight rather than one per plane (the
                // scheduling barriers keep the compiler from serialising them again).
                constexpr int G = (NP % LENIA_GENE_GROUP == 0) ? LENIA_GENE_GROUP : 3, NG = NP / G;
                static_assert(NP % G == 0, "gene planes come in threes");
                const NbrB nb = neighbour_bytes(gy, gx, H, W);
                const float cs = wd.cnt_scale, ncs = wd.cnt_bias;
                float v[2][G][5];
#pragma unroll
                for (int i = 0; i < G; ++i) load_disk(v[0][i], plane(wd.P + (size_t)i * HW, pb), nb);
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    if (g + 1 < NG) {
#pragma unroll
                        for (int i = 0; i < G; ++i)
                            load_disk(v[(g + 1) & 1][i], plane(wd.P + (size_t)((g + 1) * G + i) * HW, pb), nb);
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int i = 0; i < G; ++i) {
                        pd[g * G + i] = diffuse_disk(v[g & 1][i], cs, ncs);
                        alpha = alpha && (pd[g * G + i] > eps);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // growth summed per source channel, each channel's kernels in table
            // order (the order the DFT form's fused step follows)
            if (alpha) {
#pragma unroll
                for (int s = 0; s < T::C; ++s)
#pragma unroll
                    for (int j = 0; j < T::KPS; ++j) {
                        const int k = T::kidx[s][j];
                        sum[T::dst[k]] = growth_acc(sum[T::dst[k]], u[k], pd[k], pd[NK + k], pd[2 * NK + k]);
                    }
            }
#pragma unroll
            for (int q = 0; q < NP; ++q) pst_stream(plane(wd.P_out + (size_t)q * HW, pb), ob, alpha ? pd[q] : 0.f);
        }
        if (wd.alpha_save) wd.alpha_save[ob >> 2] = alpha ? 1 : 0;
        if (wd.flags_out) {
            float su = 0.f;
#pragma unroll
            for (int k = 0; k < NK; ++k) su += u[k];
            wd.flags_out[ob >> 2] = (uint8_t)((alpha ? 1 : 0) | ((su > eps) ? 2 : 0));
        }
    } else if (mode == MODE_LOCAL_READONLY) {
#pragma unroll
        for (int k = 0; k < NK; ++k)
            sum[T::dst[k]] = growth_acc(sum[T::dst[k]], u[k], pld(plane(wd.P + (size_t)k * HW, pb), ob),
                                     pld(plane(wd.P + (size_t)(NK + k) * HW, pb), ob),
                                     pld(plane(wd.P + (size_t)(2 * NK + k) * HW, pb), ob));
        if (wd.alpha_save) wd.alpha_save[ob >> 2] = 1;
    } else {
#pragma unroll
        for (int k = 0; k < NK; ++k) sum[T::dst[k]] = growth_acc(sum[T::dst[k]], u[k], wd.gm[k], wd.gs[k], wd.gh[k]);
        if (wd.alpha_save) wd.alpha_save[ob >> 2] = 1;
    }
#pragma unroll
    for (int c = 0; c < T::C; ++c)
        pst(plane(wd.A_out + (size_t)c * HW, pb), ob, clip01(fmaf(wd.dt, sum[c], a[c])));
    if (wd.U_save) {
#pragma unroll
        for (int k = 0; k < NK; ++k) pst(plane(wd.U_save + (size_t)k * HW, pb), ob, u[k]);
    }
}

// Outputs of the thread's Q vertically adjacent cells (gy + q, gx) whose alpha
// is 0 (no growth, genes masked to 0): A' = clip01(A), P' = 0, and flags 0
// when requested (only tiles whose potentials all stay below eps / NK skip
// then).  c points at the
// first cell in the staged tile (channel 0); cells past the torus edge are
// skipped.  Planes are the outer loop, so each plane's descriptor is used for
// all the cells and then dropped.  With genes = false the gene planes, known
// to hold 0 on the tile already, are left alone.
template <class T, int Q, class L, int NPG>
__device__ __forceinline__ void write_dead_cells(const WorldArgs& wd, const float* c, int gy, int gx,
                                                 bool genes = true)
{
    const size_t HW = (size_t)wd.H * wd.W;
    const uint32_t pb = 4u * (uint32_t)HW;
    uint32_t ob[Q];
    bool in[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        in[q] = (gy + q < wd.H) && (gx < wd.W);
        ob[q] = 4u * ((uint32_t)(gy + q) * (uint32_t)wd.W + (uint32_t)gx);
    }
#pragma unroll
    for (int ch = 0; ch < T::C; ++ch) {
        const plane_t pl = plane(wd.A_out + (size_t)ch * HW, pb);
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (in[q]) pst(pl, ob[q], clip01(c[ch * L::CHS + q * L::RS]));
    }
    if (genes) {
#pragma unroll
        for (int p = 0; p < NPG; ++p) {
            const plane_t pl = plane(wd.P_out + (size_t)p * HW, pb);
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (in[q]) pst_stream(pl, ob[q], 0.f);
        }
    }
    if (wd.alpha_save) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (in[q]) wd.alpha_save[ob[q] >> 2] = 0;
    }
    if (wd.flags_out) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (in[q]) wd.flags_out[ob[q] >> 2] = 0;
    }
}

// ---------------------------------------------------------------------------
// Ring-decomposed localized kernels (Section 2.4).  The disk |d| < R is split
// into NR = 2R rings, ring j holding the offsets with floor(NR |d| / R) = j.
// Each kernel's two bumps (r_i, w_i, b_i) are genes of the cell, and
//   u_k = sum_j kw_j S_j / sum_j kw_j n_j,
//   kw_j = sum_i b_i exp(-(j/NR - r_i)^2 / (2 w_i^2)),
// with S_j the sum of the source channel over ring j and n_j its offset count.
// Every orbit of the lattice symmetries lies in one ring, so the ring sums come
// from the same orbit walk as the cast kernels' potentials.  Genes P[9][NK]
// in the order r1, w1, b1, r2, w2, b2, m, s, h.
// ---------------------------------------------------------------------------
struct RingOrbit {
    int a, b, ring;   // representative offset (a, b), 0 <= b <= a
};

// floor(NR sqrt(d2) / R) in integers
constexpr int ring_of_d2(int R, int NR, int d2)
{
    int j = 0;
    while ((j + 1) * (j + 1) * R * R <= NR * NR * d2) ++j;
    return j;
}

template <int R>
struct RingTables {
    static constexpr int NR = 2 * R;
    static constexpr int NO = [] {
        int n = 0;
        for (int a = 0; a < R; ++a)
            for (int b = 0; b <= a; ++b)
                if (a * a + b * b < R * R) ++n;
        return n;
    }();
    RingOrbit orb[NO];    // in ring order (centre first)
    int slot[NR];         // ring -> index among the non-empty rings, or -1
    int ring_of_slot[NR];
    int size_of_slot[NR];
    int nre;              // number of non-empty rings
};

template <int R>
constexpr RingTables<R> make_ring_tables()
{
    RingTables<R> t{};
    constexpr int NR = RingTables<R>::NR;
    int size[NR] = {};
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx)
            if (dy * dy + dx * dx < R * R) ++size[ring_of_d2(R, NR, dy * dy + dx * dx)];
    t.nre = 0;
    for (int j = 0; j < NR; ++j) {
        t.slot[j] = -1;
        if (size[j] > 0) {
            t.slot[j] = t.nre;
            t.ring_of_slot[t.nre] = j;
            t.size_of_slot[t.nre] = size[j];
            ++t.nre;
        }
    }
    int n = 0;
    for (int j = 0; j < NR; ++j)
        for (int a = 0; a < R; ++a)
            for (int b = 0; b <= a; ++b)
                if (a * a + b * b < R * R && ring_of_d2(R, NR, a * a + b * b) == j) t.orb[n++] = {a, b, j};
    return t;
}

template <int R>
inline constexpr RingTables<R> kRings = make_ring_tables<R>();

// Adds orbit I (and, recursively, the following ones) of the ring walk into
// the ring sums S[slot][channel] of the cell at c.
template <class T, class L, int R, int I>
__device__ __forceinline__ void ring_walk(float (&S)[kRings<R>.nre][T::C], const float* c)
{
    if constexpr (I < RingTables<R>::NO) {
        constexpr RingOrbit o = kRings<R>.orb[I];
        constexpr int sl = kRings<R>.slot[o.ring];
        constexpr int RS = L::RS, ES = L::ES;
        float sum[1][T::C];
        if constexpr (o.a == 0) {
            tap_load<T, 1, L>(sum, c);
        } else if constexpr (o.b == 0) {
            quad_sum<T, 1, L>(sum, c + o.a * RS, c - o.a * RS, c + o.a * ES, c - o.a * ES);
        } else if constexpr (o.b == o.a) {
            quad_sum<T, 1, L>(sum, c + o.a * (RS + ES), c + o.a * (RS - ES), c - o.a * (RS - ES),
                              c - o.a * (RS + ES));
        } else {
            float s0[1][T::C], s1[1][T::C];
            quad_sum<T, 1, L>(s0, c + o.a * RS + o.b * ES, c + o.a * RS - o.b * ES,
                              c - o.a * RS + o.b * ES, c - o.a * RS - o.b * ES);
            quad_sum<T, 1, L>(s1, c + o.b * RS + o.a * ES, c + o.b * RS - o.a * ES,
                              c - o.b * RS + o.a * ES, c - o.b * RS - o.a * ES);
#pragma unroll
            for (int ch = 0; ch < T::C; ++ch) sum[0][ch] = s0[0][ch] + s1[0][ch];
        }
#pragma unroll
        for (int ch = 0; ch < T::C; ++ch) S[sl][ch] += sum[0][ch];
        ring_walk<T, L, R, I + 1>(S, c);
    }
}

// Gene diffusion, ring weights, potentials, alpha, growth and update of one
// cell in the ring form.  The kernels are taken source channel by source
// channel (the ring sums of channel c serve its kernels); each kernel's 9 gene
// planes are diffused and stored, and a lane stops working on further kernels
// once its alpha has failed.  Where alpha = 0 at the end, A' = clip01(A) and
// every gene plane is overwritten with 0.
template <class T, int R>
__device__ __forceinline__ void ring_epilogue_cell(const WorldArgs& wd, const float (&S)[kRings<R>.nre][T::C],
                                                   const float (&a)[T::C], int gy, int gx)
{
    constexpr int NK = T::NK, NPG = 9 * NK, NRE = kRings<R>.nre, NR = RingTables<R>::NR;
    const int H = wd.H, W = wd.W;
    const size_t HW = (size_t)H * W;
    const uint32_t ob = 4u * ((uint32_t)gy * (uint32_t)W + (uint32_t)gx);
    const uint32_t pb = 4u * (uint32_t)HW;
    const float eps = wd.eps, cs = wd.cnt_scale, ncs = wd.cnt_bias;
    const NbrB nb = neighbour_bytes(gy, gx, H, W);
    bool alpha = true;
    float sum[T::C];
#pragma unroll
    for (int ch = 0; ch < T::C; ++ch) sum[ch] = 0.f;
    // The 9 genes of each kernel are read as 3 groups of 3 planes (their r = 1
    // disks), 45 groups in all, kernels in table order.  Two groups are kept
    // in flight ahead of the one being reduced, across kernel boundaries too,
    // so that the loads of the next kernel's genes run under this kernel's
    // ring weights (48 exponentials).  Group 3 j + i lives in buffer i.
    auto kernel_at = [](int pos) { return T::kidx[pos / T::KPS][pos % T::KPS]; };
    auto load_group = [&](float (&v)[3][5], int pos, int grp) {
        const int kk = kernel_at(pos);
#pragma unroll
        for (int i = 0; i < 3; ++i) load_disk(v[i], plane(wd.P + (size_t)((grp * 3 + i) * NK + kk) * HW, pb), nb);
    };
    float v[3][3][5];
    load_group(v[0], 0, 0);
    load_group(v[1], 0, 1);
#pragma unroll
    for (int c = 0; c < T::C; ++c) {
#pragma unroll 1
      for (int j = 0; j < T::KPS; ++j) {
        // a wave whose cells have all lost alpha stops reading
        if (!__any(alpha)) continue;
        const int pos = c * T::KPS + j;
        const int k = T::kidx[c][j];
        // stores of a cell whose alpha has failed go past the plane (dropped)
        float g[9];
#pragma unroll
        for (int grp = 0; grp < 3; ++grp) {
            // issue the group two ahead: this kernel's third, or the next
            // kernel's first or second
            if (grp == 0) load_group(v[2], pos, 2);
            else if (pos + 1 < NK) load_group(v[grp - 1], pos + 1, grp - 1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int q = grp * 3 + i;
                g[q] = diffuse_disk(v[grp][i], cs, ncs);
                alpha = alpha && (g[q] > eps);
                pst_stream(plane(wd.P_out + (size_t)(q * NK + k) * HW, pb), alpha ? ob : 0xFFFFFFF0u, g[q]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // ring weights of the two bumps: b exp2(c (x - r)^2), c = -log2(e) / (2 w^2)
        const float c1 = -0.72134752044448170f * __builtin_amdgcn_rcpf(g[1] * g[1]);
        const float c2 = -0.72134752044448170f * __builtin_amdgcn_rcpf(g[4] * g[4]);
        float num = 0.f, den = 0.f;
#pragma unroll
        for (int sl = 0; sl < NRE; ++sl) {
            constexpr float inv_nr = 1.0f / (float)NR;
            const float x = (float)kRings<R>.ring_of_slot[sl] * inv_nr;
            const float d1 = x - g[0], d2 = x - g[3];
            const float kw = g[2] * __builtin_amdgcn_exp2f(c1 * (d1 * d1)) +
                             g[5] * __builtin_amdgcn_exp2f(c2 * (d2 * d2));
            num = fmaf(kw, S[sl][c], num);
            den = fmaf(kw, (float)kRings<R>.size_of_slot[sl], den);
        }
        const float u = (den > 0.f) ? num / den : 0.f;
        alpha = alpha && (u > eps);
        const float gk = growth(u, g[6], g[7], g[8]);
        const int dk = T::dst[k];
#pragma unroll
        for (int ch = 0; ch < T::C; ++ch) sum[ch] += (alpha && dk == ch) ? gk : 0.f;
      }
    }
#pragma unroll
    for (int ch = 0; ch < T::C; ++ch)
        pst(plane(wd.A_out + (size_t)ch * HW, pb), ob, clip01(alpha ? fmaf(wd.dt, sum[ch], a[ch]) : a[ch]));
    if (!alpha) {
#pragma unroll
        for (int q = 0; q < NPG; ++q) pst_stream(plane(wd.P_out + (size_t)q * HW, pb), ob, 0.f);
    }
}

// Cells per thread: tiles of at most 256 cells give each thread one cell (for
// small worlds, where parallelism is short), larger tiles a vertical pair.
template <int TY, int TX>
constexpr int step_cells_per_thread() { return (TY * TX <= 256) ? 1 : 2; }

template <int TY, int TX>
constexpr int step_threads() { return TY * TX / step_cells_per_thread<TY, TX>(); }


template <class T, int R, int TY, int TX>
constexpr int tile_lds_floats() { return TileLayout<T, R, TY, TX>::floats; }

// One tile of one world.  Each thread owns Q vertically adjacent cells.
template <class T, int R, int TY, int TX, bool RINGS = false, bool KMAJOR = true>
__device__ __forceinline__ void process_tile(const WorldArgs& wd, int tile, int mode, float* sA,
                                             int* tile_flag)
{
    using L = TileLayout<T, R, TY, TX>;
    constexpr int NPG = (RINGS ? 9 : 3) * T::NK;   // gene planes
    constexpr int HALO = L::HALO;
    constexpr int PY = TY + 2 * HALO, PX = TX + 2 * HALO;
    constexpr int NK = T::NK;
    constexpr int NT = step_threads<TY, TX>();
    constexpr int Q = step_cells_per_thread<TY, TX>();

    const int H = wd.H, W = wd.W;
    const size_t HW = (size_t)H * W;
    const int tyi = tile / wd.tiles_x;
    const int txi = tile - tyi * wd.tiles_x;
    const int y0 = tyi * TY, x0 = txi * TX;

    // Tiles where alpha = 0 everywhere (Section 2.2), found before the
    // convolution, so that A' = clip01(A) and P' = 0 are written exactly
    // without it.  Two sufficient conditions:
    //  * an empty channel: the potentials u_k are averages (non-negative
    //    weights summing to 1) of their source channel over the window, so if
    //    some channel's window stays <= skip_thr < eps, every u_k reading it is
    //    below the cutoff;
    //  * a dead gene plane: if every value of gene plane 0 on the tile and its
    //    1-cell ring is <= eps, no disk of the diffusion counts a value above
    //    eps, so the diffused gene is 0 on the tile (P' = 0 where alpha was 0
    //    leaves such regions behind).
    // Decided only where the potentials are not requested.  Where the flags
    // (alpha, organic sum_k u_k > eps) are, only a tile whose window stays at
    // or below org_thr = skip_thr / NK in every channel is skipped: there every
    // u_k is at most org_thr, so the sum is below eps and both flags are 0.
    const bool may_skip = (mode == MODE_LOCAL_UPDATE) && (wd.U_save == nullptr);
    const bool want_flags = (wd.flags_out != nullptr);
    // bit 30 of the tile flag: the output's gene planes already hold 0 on this
    // tile (thread 0 reads the flag here and updates it after the last barrier)
    constexpr int kGenesZero = 1 << 30;
    if (may_skip && threadIdx.x == 0)
        *tile_flag = (wd.p_zero != nullptr && wd.p_zero[tile] != 0) ? kGenesZero : 0;
    int wave_bits = 0;   // bit c < C: some window value of channel c above skip_thr
                         // (above org_thr with flags); bit C: some value of gene
                         // plane 0 above eps (without flags)

    // a single wrap suffices unless the torus is smaller than tile + halo
    const bool single_wrap = (H >= TY + R) && (W >= TX + R);
    // 1. stage A (+halo, wrapped) with all of a thread's loads in flight at once;
    // the index arithmetic of a halo position is shared by the channels
    {
        constexpr int NG = PY * PX;
        constexpr int IT = (NG + NT - 1) / NT;
        float v[IT][T::C];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int i = threadIdx.x + it * NT;
            if (i < NG) {
                const int yy = i / PX;
                const int xx = i - yy * PX;
                int gy = y0 + yy - HALO, gx = x0 + xx - HALO;
                if (single_wrap) {
                    gy += (gy < 0) ? H : 0;
                    gy -= (gy >= H) ? H : 0;
                    gx += (gx < 0) ? W : 0;
                    gx -= (gx >= W) ? W : 0;
                } else {
                    gy = ((gy % H) + H) % H;
                    gx = ((gx % W) + W) % W;
                }
                const uint32_t o = (uint32_t)gy * (uint32_t)W + (uint32_t)gx;
#pragma unroll
                for (int ch = 0; ch < T::C; ++ch) v[it][ch] = (wd.A + (size_t)ch * HW)[o];
            }
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int i = threadIdx.x + it * NT;
            if (i < NG) {
                const int yy = i / PX;
                const int xx = i - yy * PX;
                float* d = sA + (yy * L::PITCH + xx) * L::ES;
                if constexpr (L::interleaved) {
                    *reinterpret_cast<float4*>(d) = make_float4(v[it][0], v[it][1], v[it][2], 0.f);
                } else {
#pragma unroll
                    for (int ch = 0; ch < T::C; ++ch) d[ch * L::CHS] = v[it][ch];
                }
            }
        }
        if (may_skip) {
            const float thr = want_flags ? wd.org_thr : wd.skip_thr;
#pragma unroll
            for (int ch = 0; ch < T::C; ++ch) {
                bool above = false;
#pragma unroll
                for (int it = 0; it < IT; ++it)
                    above = above || ((threadIdx.x + it * NT < NG) && (v[it][ch] > thr));
                wave_bits |= (__ballot(above) != 0ull) ? (1 << ch) : 0;
            }
        }
        if (may_skip && !want_flags) {
            // gene plane 0 on the tile plus a 1-cell ring
            constexpr int G1X = TX + 2, NG1 = (TY + 2) * G1X;
            const plane_t p0 = plane(wd.P, 4u * (uint32_t)HW);
            bool live = false;
#pragma unroll
            for (int i0 = 0; i0 < NG1; i0 += NT) {
                const int i = i0 + (int)threadIdx.x;
                if (i < NG1) {
                    const int yy = i / G1X;
                    int gy = y0 + yy - 1, gx = x0 + (i - yy * G1X) - 1;
                    wrap2(gy, gx, H, W, single_wrap);
                    live = live || (pld(p0, 4u * ((uint32_t)gy * (uint32_t)W + (uint32_t)gx)) > wd.eps);
                }
            }
            wave_bits |= (__ballot(live) != 0ull) ? (1 << T::C) : 0;
        }
    }
    __syncthreads();
    if (may_skip) {
        if ((threadIdx.x & 63) == 0 && wave_bits != 0) atomicOr(tile_flag, wave_bits);
        __syncthreads();
        const int bits = *tile_flag & ((2 << T::C) - 1);
        if (want_flags ? (bits == 0) : (bits != (2 << T::C) - 1)) {
            // an empty channel or a dead gene plane (with flags: every channel
            // empty): alpha = 0 on the tile
            const int ly = Q * (threadIdx.x / TX);
            const int lx = threadIdx.x % TX;
            write_dead_cells<T, Q, L, NPG>(wd, sA + ((ly + HALO) * L::PITCH + (lx + HALO)) * L::ES, y0 + ly,
                                           x0 + lx, (*tile_flag & kGenesZero) == 0);
            if (wd.p_zero != nullptr && threadIdx.x == 0) wd.p_zero[tile] = 1;
            return;
        }
        if (wd.p_zero != nullptr && threadIdx.x == 0) wd.p_zero[tile] = 0;
    }

    // 2. potentials of the thread's cells, 3. their epilogues
    const int ly = Q * (threadIdx.x / TX);
    const int lx = threadIdx.x % TX;
    const int gy = y0 + ly, gx = x0 + lx;
    if (gy >= H || gx >= W) return;
    const float* c = sA + ((ly + HALO) * L::PITCH + (lx + HALO)) * L::ES;
    if constexpr (RINGS) {
        static_assert(Q == 1 && L::interleaved, "the ring form runs one cell per thread, 3 channels");
        float S[kRings<R>.nre][T::C];
#pragma unroll
        for (int sl = 0; sl < kRings<R>.nre; ++sl)
#pragma unroll
            for (int ch = 0; ch < T::C; ++ch) S[sl][ch] = 0.f;
        ring_walk<T, L, R, 0>(S, c);
        // materialize every ring sum here: otherwise the compiler sinks the sums
        // of channels 1 and 2 to their first use after channel 0's kernels and
        // keeps all their tap values live (and spilled) until then
#pragma unroll
        for (int sl = 0; sl < kRings<R>.nre; ++sl)
#pragma unroll
            for (int ch = 0; ch < T::C; ++ch) asm volatile("" : "+v"(S[sl][ch]));
        float a[T::C];
#pragma unroll
        for (int ch = 0; ch < T::C; ++ch) a[ch] = c[ch * L::CHS];
        ring_epilogue_cell<T, R>(wd, S, a, gy, gx);
        return;
    }
    float u[Q][NK];
    if constexpr (T::KPS > 3)
        conv_cells_shells<T, Q, R, L>(c, (cfloat*)wd.shc, u);
    else
        conv_cells<T, Q, R, L>(c, (cfloat*)wd.wt, u);
    if (mode == MODE_POTENTIALS) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (gy + q < H) {
                const uint32_t o = (uint32_t)(gy + q) * (uint32_t)W + (uint32_t)gx;
#pragma unroll
                for (int k = 0; k < NK; ++k) (wd.U_save + (size_t)k * HW)[o] = u[q][k];
            }
        return;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (gy + q < H) {
            float a[T::C];
#pragma unroll
            for (int ch = 0; ch < T::C; ++ch) a[ch] = c[ch * L::CHS + q * L::RS];
            epilogue_cell<T, KMAJOR>(wd, mode, u[q], a, gy + q, gx);
        }
    }
}

template <class T, int R, int TY, int TX>
__global__ __launch_bounds__((step_threads<TY, TX>()), LENIA_MIN_WAVES) void step_kernel(WorldArgs wd, int mode)
{
    __shared__ __attribute__((aligned(16))) float sA[tile_lds_floats<T, R, TY, TX>()];
    __shared__ int tile_flag;
    process_tile<T, R, TY, TX>(wd, xcd_tile(blockIdx.x, gridDim.x), mode, sA, &tile_flag);
}

// Step with ring-decomposed localized kernels (genes P[9][NK][H][W]).
template <class T, int R, int TY, int TX>
__global__ __launch_bounds__((step_threads<TY, TX>()), LENIA_MIN_WAVES) void ring_step_kernel(WorldArgs wd, int mode)
{
    __shared__ __attribute__((aligned(16))) float sA[tile_lds_floats<T, R, TY, TX>()];
    __shared__ int tile_flag;
    process_tile<T, R, TY, TX, true>(wd, xcd_tile(blockIdx.x, gridDim.x), mode, sA, &tile_flag);
}

template <class T, int R, int TY, int TX>
hipError_t launch_ring_step(const WorldArgs& w, int mode, hipStream_t s)
{
    hipLaunchKernelGGL((ring_step_kernel<T, R, TY, TX>), dim3(w.n_tiles), dim3(step_threads<TY, TX>()), 0, s,
                       w, mode);
    return hipGetLastError();
}

step_launch_fn find_ring_step_launcher(int table, int R, int ty, int tx)
{
    if (table == TABLE_3x15 && R == 12 && ty == 8 && tx == 32) return &launch_ring_step<Table3x15, 12, 8, 32>;
    return nullptr;
}

// Epilogue of a step whose potentials were computed elsewhere (the MFMA DFT
// form): one thread per cell reads u_k from U.
template <class T>
__global__ __launch_bounds__(256) void epilogue_kernel(WorldArgs wd, const float* __restrict__ U,
                                                       int mode)
{
    const uint32_t HW = (uint32_t)wd.H * (uint32_t)wd.W;
    const uint32_t idx = blockIdx.x * 256u + threadIdx.x;
    if (idx >= HW) return;
    const int gy = (int)(idx / (uint32_t)wd.W), gx = (int)(idx - (uint32_t)gy * wd.W);
    float u[T::NK], a[T::C];
#pragma unroll
    for (int k = 0; k < T::NK; ++k) u[k] = (U + (size_t)k * HW)[idx];
#pragma unroll
    for (int c = 0; c < T::C; ++c) a[c] = (wd.A + (size_t)c * HW)[idx];
    epilogue_cell<T>(wd, mode, u, a, gy, gx);
}

template <class T>
hipError_t launch_epilogue(const WorldArgs& w, const float* U, int mode, hipStream_t s)
{
    const unsigned cells = (unsigned)w.H * (unsigned)w.W;
    hipLaunchKernelGGL((epilogue_kernel<T>), dim3((cells + 255) / 256), dim3(256), 0, s, w, U, mode);
    return hipGetLastError();
}

epilogue_launch_fn find_epilogue_launcher(int table)
{
    return (table == TABLE_3x15) ? &launch_epilogue<Table3x15> : &launch_epilogue<Table1x1>;
}

// Batched form: one workgroup per (world, tile) item of the work list, so
// that the hardware dispatcher balances tiles of uneven cost.
template <class T, int R, int TY, int TX>
__global__ __launch_bounds__((step_threads<TY, TX>()), LENIA_MIN_WAVES) void step_batch_kernel(BatchList bl, int mode)
{
    __shared__ __attribute__((aligned(16))) float sA[tile_lds_floats<T, R, TY, TX>()];
    __shared__ int tile_flag;
    // blocks map to items through the same XCD-aware permutation as tiles of
    // a single world (the list holds the tiles of a world in row order); the
    // world table is read-only for the launch, so it is read through the
    // constant address space, where its fields are scalar loads no store aliases
    typedef const __attribute__((address_space(4))) int cint;
    if ((int)blockIdx.x >= bl.n_items) return;
    const cint* item = (const cint*)(bl.items + xcd_tile(blockIdx.x, bl.n_items));
    const int world = item[0], tile = item[1];
    constexpr int NW = sizeof(WorldArgs) / sizeof(int);
    static_assert(NW * sizeof(int) == sizeof(WorldArgs), "WorldArgs is a whole number of words");
    const cint* src = (const cint*)(bl.worlds + world);
    int words[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) words[i] = src[i];
    const WorldArgs wd = __builtin_bit_cast(WorldArgs, words);
    process_tile<T, R, TY, TX, false, false>(wd, tile, mode, sA, &tile_flag);
}

template <class T, int R, int TY, int TX>
hipError_t launch_step(const WorldArgs& w, int mode, hipStream_t s)
{
    hipLaunchKernelGGL((step_kernel<T, R, TY, TX>), dim3(w.n_tiles), dim3(step_threads<TY, TX>()), 0, s, w,
                       mode);
    return hipGetLastError();
}

template <class T, int R, int TY, int TX>
hipError_t launch_batch(const BatchList& b, int mode, hipStream_t s)
{
    if (b.n_items <= 0) return hipSuccess;
    hipLaunchKernelGGL((step_batch_kernel<T, R, TY, TX>), dim3(b.n_items), dim3(step_threads<TY, TX>()), 0, s,
                       b, mode);
    return hipGetLastError();
}

struct Entry {
    int table, R, ty, tx;
    step_launch_fn step;
    batch_launch_fn batch;
};

#define LENIA_ENTRY(TB, TID, RR, TYY, TXX)                                                   \
    {TID, RR, TYY, TXX, &launch_step<TB, RR, TYY, TXX>, &launch_batch<TB, RR, TYY, TXX>}

static const Entry kEntries[] = {
    LENIA_ENTRY(Table3x15, TABLE_3x15, 12, 16, 32),
    LENIA_ENTRY(Table3x15, TABLE_3x15, 12, 32, 32),
    LENIA_ENTRY(Table3x15, TABLE_3x15, 12, 16, 64),
    LENIA_ENTRY(Table3x15, TABLE_3x15, 12, 8, 64),
    LENIA_ENTRY(Table3x15, TABLE_3x15, 12, 8, 32),
    LENIA_ENTRY(Table3x15, TABLE_3x15, 12, 4, 64),
    LENIA_ENTRY(Table3x15, TABLE_3x15, 13, 16, 32),
    LENIA_ENTRY(Table3x15, TABLE_3x15, 13, 8, 32),
    LENIA_ENTRY(Table1x1, TABLE_1x1, 13, 16, 32),
    LENIA_ENTRY(Table1x1, TABLE_1x1, 13, 8, 32),
    LENIA_ENTRY(Table1x1, TABLE_1x1, 12, 16, 32),
    LENIA_ENTRY(Table1x1, TABLE_1x1, 12, 8, 32),
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

__global__ __launch_bounds__(256) void fill_bytes_kernel(uint8_t* p, uint32_t n)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_clear_bytes(uint8_t* p, uint32_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_bytes_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void find_nonfinite_kernel(const float* __restrict__ x, size_t n,
                                                            uint32_t* flag, uint32_t bit)
{
    const size_t stride = (size_t)gridDim.x * 256;
    bool bad = false;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
        bad |= !isfinite(x[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, bit);
}

hipError_t launch_find_nonfinite(const float* x, size_t n, uint32_t* flag, uint32_t bit,
                                 hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(find_nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, n, flag, bit);
    return hipGetLastError();
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
