// Adjoint (vector-Jacobian product) of one Lenia step on gfx950.
//
// Forward at a cell (see lenia_step.hip):  P_d = diffusion of P (Section 2.3),
// u_k = K~_k * A_src(k) (Section 2.1), alpha = all u_k > eps and all P_d > eps
// (Section 2.2), g_k = alpha h_k (2 e_k - 1), e_k = exp(-(u_k - m_k)^2/(2 s_k^2))
// with (m, s, h) = alpha P_d (Section 2.4), z_c = A_c + dt sum_{dst(k)=c} g_k,
// A'_c = clip01(z_c), P' = alpha P_d.  Given cotangents (gA', gP') the adjoint
// is, with alpha and the diffusion counts n held fixed (piecewise constant) and
// the clips' inclusive subgradients:
//   zbar_c   = gA'_c [0 <= z_c <= 1]                     -> gA_c (direct term)
//   ubar_k   = dt zbar_dst(k) (-2 h e (u-m)/s^2)
//   Pbar_d   = alpha (gP' + dt zbar_dst(k) (dg/dm, dg/ds, dg/dh))
//   numbar   = Pbar_d [n > 0 and 0 <= num/n <= 1] / n
//   gA_c    += sum_{src(k)=c} K~_k (x) ubar_k  (K~ even: correlation again)
//   gP(y)    = sum over the r = 1 disk of numbar(y + d)
//   dL/dbeta_{k,i} = < ubar_k, sum_t bcoef_{k,i}(t) orbit-sum_t A_src >
// Three kernels: a per-cell pass, a tiled gather pass (convolution transpose,
// diffusion transpose, shell-height partials per tile), and a fixed-order
// reduction of the partials.  No float atomics: results are deterministic.
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "lenia.h"
#include "lenia_device.h"
#include "lenia_internal.h"
#include "lenia_plan.h"

namespace lenia {

struct BwdArgs {
    const float* A;          // A_t    [C][H][W]
    const float* P;          // P_t    [3NK][H][W]
    const float* U;          // saved potentials [NK][H][W]
    const uint8_t* alpha;    // saved alpha [H][W]
    const float* gA1;        // gA_next [C][H][W]
    const float* gP1;        // gP_next [3NK][H][W] or null (zero)
    float* gA;               // gA_t (written by the cell pass, completed by the gather pass)
    float* gP;               // gP_t
    float* ubar;             // workspace [NK][H][W]
    float* numbar;           // workspace [3NK][H][W] (gene update only)
    float* part;             // workspace [n_tiles][NK][3]
    const float* wt;         // orbit weights [NO][C][8] in the step kernel's orbit order
    const float* bt;         // shell-height coefficients [NO][C][16] (slot j, shell i at
                             // j * 3 + i) in the same orbit order
    int H, W, tiles_x, n_tiles;
    float dt, eps;
    int mode;
};

// ---------------------------------------------------------------------------
// 1. per-cell pass
// ---------------------------------------------------------------------------
// One thread per (cell, target channel c): the 5 kernels updating channel c,
// their 15 gene planes, the clip of z_c.  alpha comes from the saved mask.
template <class T>
__global__ __launch_bounds__(256) void bwd_cell_kernel(BwdArgs b)
{
    constexpr int NK = T::NK, KPD = T::KPD;
    const int H = b.H, W = b.W;
    const uint32_t HW = (uint32_t)H * (uint32_t)W;
    const uint32_t idx = blockIdx.x * 256u + threadIdx.x;
    if (idx >= HW) return;
    const int c = blockIdx.y;
    const int gy = (int)(idx / (uint32_t)W), gx = (int)(idx - (uint32_t)gy * W);
    const float eps = b.eps, dt = b.dt;
    const bool update = (b.mode == MODE_LOCAL_UPDATE);
    const bool alpha = update ? (b.alpha[idx] != 0) : true;
    const float a = (b.A + (size_t)c * HW)[idx];
    const float g1 = (b.gA1 + (size_t)c * HW)[idx];

    if (!alpha) {
        // no growth: z = A, P' = 0.  ubar and numbar vanish here; the gather
        // pass masks them by alpha instead of reading stored zeros.
        (b.gA + (size_t)c * HW)[idx] = (a >= 0.f && a <= 1.f) ? g1 : 0.f;
        return;
    }
    int kk[KPD];
#pragma unroll
    for (int j = 0; j < KPD; ++j) kk[j] = T::kdst[c][j];

    // Every read of the thread is issued before the arithmetic that needs it
    // (one round trip rather than one per gene plane): the genes of the
    // channel's kernels (their r = 1 disks when they are diffused), the
    // potentials and the incoming gene cotangents.
    const Nbr nb = neighbours(gy, gx, H, W);
    float pv[3][KPD][5];
    if (update) {
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int j = 0; j < KPD; ++j) {
                const float* pl = b.P + (size_t)(p * NK + kk[j]) * HW;
                pv[p][j][0] = pl[nb.ou];
                pv[p][j][1] = pl[nb.ol];
                pv[p][j][2] = pl[nb.oc];
                pv[p][j][3] = pl[nb.orr];
                pv[p][j][4] = pl[nb.od];
            }
    } else {
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int j = 0; j < KPD; ++j) pv[p][j][2] = (b.P + (size_t)(p * NK + kk[j]) * HW)[idx];
    }
    float u[KPD];
#pragma unroll
    for (int j = 0; j < KPD; ++j) u[j] = (b.U + (size_t)kk[j] * HW)[idx];
    float gp1[3][KPD];
    if (b.gP1) {
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int j = 0; j < KPD; ++j) gp1[p][j] = (b.gP1 + (size_t)(p * NK + kk[j]) * HW)[idx];
    } else {
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int j = 0; j < KPD; ++j) gp1[p][j] = 0.f;
    }

    // genes: diffused (update) or as stored (read-only)
    float pd[3][KPD], rn[3][KPD];
    bool clip_ok[3][KPD];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int j = 0; j < KPD; ++j) {
            if (update) {
                const Diffused df = diffuse_vals(pv[p][j], eps);
                pd[p][j] = df.v;
                const float inv = (df.n > 0) ? __builtin_amdgcn_rcpf((float)df.n) : 0.f;
                const float qq = df.num * inv;
                clip_ok[p][j] = (df.n > 0) && (qq >= 0.f) && (qq <= 1.f);
                rn[p][j] = inv;
            } else {
                pd[p][j] = pv[p][j][2];
                clip_ok[p][j] = true;
                rn[p][j] = 1.f;
            }
        }
    // forward growth and pre-clip update (same arithmetic and order as the step
    // kernel: kdst lists the channel's kernels in its summation order)
    float sum = 0.f;
#pragma unroll
    for (int j = 0; j < KPD; ++j) sum = growth_acc(sum, u[j], pd[0][j], pd[1][j], pd[2][j]);
    const float z = fmaf(dt, sum, a);   // as the forward step forms it
    const float zb = (z >= 0.f && z <= 1.f) ? g1 : 0.f;
    (b.gA + (size_t)c * HW)[idx] = zb;
    const float gb = dt * zb;
    // growth derivatives
#pragma unroll
    for (int j = 0; j < KPD; ++j) {
        const float m = pd[0][j], s = pd[1][j], h = pd[2][j];
        const float d = u[j] - m;
        const float e = growth_bell(d, s);
        const float is2 = __builtin_amdgcn_rcpf(s * s);
        const float common = 2.f * h * e * d * is2;           // dg/dm
        (b.ubar + (size_t)kk[j] * HW)[idx] = -gb * common;    // dg/du = -dg/dm
        const float dd[3] = {gb * common, gb * common * d * __builtin_amdgcn_rcpf(s),
                             gb * (2.f * e - 1.f)};
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const size_t q = (size_t)(p * NK + kk[j]) * HW;
            const float pb = gp1[p][j] + dd[p];
            if (update)
                b.numbar[q + idx] = clip_ok[p][j] ? pb * rn[p][j] : 0.f;
            else
                b.gP[q + idx] = pb;
        }
    }
}

// ---------------------------------------------------------------------------
// 2. tiled gather pass
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// LDS layout of the gather's NPL staged planes over NPOS positions (row pitch
// PX positions): planes in groups of four interleaved per position, one
// 16-byte vector each, and the remaining one to three planes interleaved in a
// last group of width RW (with six planes: one group of four and a pair), so a
// tap of every plane is one 128-bit and one 64-bit LDS read.
template <int NPL, int NPOS, int PX>
struct GatherLayout {
    static constexpr int N4 = NPL / 4;
    static constexpr int REM = NPL - 4 * N4;
    static constexpr int RW = (REM == 0) ? 0 : (REM == 1) ? 1 : (REM == 2) ? 2 : 4;
    static constexpr int RB = 4 * N4 * NPOS;   // first float of the last group
    static constexpr int floats = RB + RW * NPOS;

    __device__ static __forceinline__ void store(float* d, int pos, const float (&v)[NPL])
    {
#pragma unroll
        for (int g = 0; g < N4; ++g)
            *reinterpret_cast<float4*>(d + g * 4 * NPOS + 4 * pos) =
                make_float4(v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3]);
        if constexpr (RW == 1) d[RB + pos] = v[4 * N4];
        if constexpr (RW == 2)
            *reinterpret_cast<float2*>(d + RB + 2 * pos) = make_float2(v[4 * N4], v[4 * N4 + 1]);
        if constexpr (RW == 4)
            *reinterpret_cast<float4*>(d + RB + 4 * pos) =
                make_float4(v[4 * N4], REM > 1 ? v[4 * N4 + 1] : 0.f, REM > 2 ? v[4 * N4 + 2] : 0.f, 0.f);
    }

    // A position of the staged tile as pointers to its first float in the
    // groups of four and in the last group; offsets move both, so that taps at
    // constant offsets from a base are immediate offsets of LDS reads.
    struct Pos {
        const float* a;
        const float* b;
        __device__ __forceinline__ Pos operator+(int dpos) const { return {a + 4 * dpos, b + RW * dpos}; }
        __device__ __forceinline__ Pos operator-(int dpos) const { return {a - 4 * dpos, b - RW * dpos}; }
    };
    __device__ static __forceinline__ Pos at(const float* d, int pos) { return {d + 4 * pos, d + RB + RW * pos}; }

    // v[plane][q] = staged value of the plane at position p + q * PX
    template <int Q>
    __device__ static __forceinline__ void load(float (&v)[NPL][Q], Pos p)
    {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int o = q * PX;
#pragma unroll
            for (int g = 0; g < N4; ++g) {
                const float4 x = *reinterpret_cast<const float4*>(p.a + g * 4 * NPOS + 4 * o);
                v[4 * g][q] = x.x;
                v[4 * g + 1][q] = x.y;
                v[4 * g + 2][q] = x.z;
                v[4 * g + 3][q] = x.w;
            }
            if constexpr (RW == 1) v[4 * N4][q] = p.b[o];
            if constexpr (RW == 2) {
                const float2 x = *reinterpret_cast<const float2*>(p.b + 2 * o);
                v[4 * N4][q] = x.x;
                v[4 * N4 + 1][q] = x.y;
            }
            if constexpr (RW == 4) {
                const float4 x = *reinterpret_cast<const float4*>(p.b + 4 * o);
                v[4 * N4][q] = x.x;
                if constexpr (REM > 1) v[4 * N4 + 1][q] = x.y;
                if constexpr (REM > 2) v[4 * N4 + 2][q] = x.z;
            }
        }
    }
};

// sum = (t0 + t1) + (t2 + t3) for each (plane, cell)
template <class L, int NPL, int Q, class P>
__device__ __forceinline__ void quad_planes(float (&sum)[NPL][Q], P p0, P p1, P p2, P p3)
{
    float v0[NPL][Q], v1[NPL][Q], v2[NPL][Q], v3[NPL][Q];
    L::template load<Q>(v0, p0);
    L::template load<Q>(v1, p1);
    L::template load<Q>(v2, p2);
    L::template load<Q>(v3, p3);
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
        for (int q = 0; q < Q; ++q) sum[pl][q] = (v0[pl][q] + v1[pl][q]) + (v2[pl][q] + v3[pl][q]);
}

// One orbit: transpose-convolution FMAs for the KPS ubar planes (weights w),
// and the shell-height coefficient FMAs on the A plane (index KPS):
// v[q][j][i] += bcoef_{k_j, i}(t) * (orbit sum of A at cell q).
template <class T, int NPL, int Q>
__device__ __forceinline__ void orbit_bwd(float (&g)[Q], float (&v)[Q][T::KPS][3],
                                          const float (&sum)[NPL][Q], cfloat* w, cfloat* bc)
{
    // the orbit's 8 weight slots and 16 coefficient slots, each one scalar load
    typedef float f8v __attribute__((ext_vector_type(8)));
    typedef float f16v __attribute__((ext_vector_type(16)));
    const f8v wv = *(const __attribute__((address_space(4))) f8v*)w;
    const f16v bv = *(const __attribute__((address_space(4))) f16v*)bc;
#pragma unroll
    for (int j = 0; j < T::KPS; ++j) {
        const float wj = wv[j];
#pragma unroll
        for (int q = 0; q < Q; ++q) g[q] = fmaf(wj, sum[j][q], g[q]);
    }
#pragma unroll
    for (int j = 0; j < T::KPS; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float c = bv[j * 3 + i];
#pragma unroll
            for (int q = 0; q < Q; ++q) v[q][j][i] = fmaf(c, sum[NPL - 1][q], v[q][j][i]);
        }
}

template <int TY, int TX>
constexpr int bwd_cells_per_thread() { return (TY * TX <= 256) ? 1 : 2; }

template <int TY, int TX>
constexpr int bwd_threads() { return TY * TX / bwd_cells_per_thread<TY, TX>(); }

// Orbit counts of the walk (axis, diagonal, general with a below a_end), in
// the order of the weight table.
template <int R>
constexpr int n_axis_orbits() { return R - 1; }

template <int R>
constexpr int n_diag_orbits()
{
    int n = 0;
    for (int a = 1; 2 * a * a < R * R; ++a) ++n;
    return n;
}

template <int R>
constexpr int n_general_orbits_below(int a_end)
{
    int n = 0;
    for (int a = 2; a < a_end; ++a)
        for (int bb = 1; bb < a; ++bb)
            if (a * a + bb * bb < R * R) ++n;
    return n;
}

// Where the walk is split between two threads of a cell: the first takes the
// axis and diagonal orbits and the general orbits with a below the returned
// value, the second the rest.  Costs per orbit in the ratio of their
// instruction counts (4 taps: 3, 8 taps: 4).
template <int R>
constexpr int gather_split_a()
{
    const int ad = 3 * (n_axis_orbits<R>() + n_diag_orbits<R>());
    const int total = ad + 4 * n_general_orbits_below<R>(R);
    int best = 2, best_cost = total;
    for (int a = 2; a <= R; ++a) {
        const int c0 = ad + 4 * n_general_orbits_below<R>(a);
        const int m = (c0 > total - c0) ? c0 : total - c0;
        if (m < best_cost) {
            best_cost = m;
            best = a;
        }
    }
    return best;
}

// One workgroup per (tile, source channel s): the transposed convolution into
// gA_s, the shell-height partials of the kernels reading s, and the diffusion
// transpose of the gene planes q with q % C == s.  S threads share each cell
// (or vertical pair of cells): with S = 2 (for worlds of few tiles, to double
// the waves in flight) they walk disjoint parts of the orbits and the second
// hands its sums to the first through LDS, which adds them in a fixed order.
template <class T, int R, int TY, int TX, int S>
__global__ __launch_bounds__((S * bwd_threads<TY, TX>())) void bwd_gather_kernel(BwdArgs b)
{
    static_assert(S == 1 || S == 2, "one or two threads per cell");
    constexpr int Q = bwd_cells_per_thread<TY, TX>();
    constexpr int NTC = bwd_threads<TY, TX>();   // threads per part of the walk
    constexpr int NT = S * NTC;
    constexpr int NWV = NTC / 64;
    constexpr int KPS = T::KPS;
    constexpr int NPL = KPS + 1;
    // the kernels' support is |d| < R: an (R - 1)-cell halo covers every tap
    constexpr int HALO = R - 1;
    constexpr int PY = TY + 2 * HALO, PX = TX + 2 * HALO;
    using L = GatherLayout<NPL, PY * PX, PX>;
    constexpr int WS = T::C * 8;     // weights per orbit
    constexpr int BS = T::C * 16;    // shell-height coefficients per orbit
    constexpr int NV = Q * (1 + KPS * 3);   // sums a thread hands over
    constexpr int SPLIT = gather_split_a<R>();
    static_assert(S == 1 || L::floats >= NTC * NV, "hand-over fits the staging buffer");
    __shared__ __attribute__((aligned(16))) float sm[L::floats];
    __shared__ float red[NWV][KPS * 3];

    const int H = b.H, W = b.W;
    const size_t HW = (size_t)H * W;
    const int s = blockIdx.y;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tyi = tile / b.tiles_x, txi = tile - tyi * b.tiles_x;
    const int y0 = tyi * TY, x0 = txi * TX;
    const int tc = (S == 1) ? (int)threadIdx.x : (int)threadIdx.x % NTC;
    // wave-uniform; read from the first lane so that the compiler knows it, and
    // the weight addresses that depend on it stay scalar
    const int part = (S == 1) ? 0 : __builtin_amdgcn_readfirstlane((int)threadIdx.x / NTC);
    const int ly = Q * (tc / TX), lx = tc % TX;
    const int gy = y0 + ly, gx = x0 + lx;
    bool valid[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) valid[q] = (gy + q < H) && (gx < W);
    const int wave = tc / 64, lane = tc % 64;
    const typename L::Pos c = L::at(sm, (ly + HALO) * PX + (lx + HALO));   // the thread's first cell

    const float* src[NPL];
#pragma unroll
    for (int j = 0; j < KPS; ++j) src[j] = b.ubar + (size_t)T::kidx[s][j] * HW;
    src[KPS] = b.A + (size_t)s * HW;
    // ubar is staged masked by alpha (only alpha cells hold it); A unmasked.
    // Where no cell of the window has alpha, every staged ubar is 0, so the
    // transposed convolution and the shell-height sums of the tile are exactly
    // 0 and the orbit walk is skipped (the tile's outputs are still written).
    bool kept = true;
    if (b.mode == MODE_LOCAL_UPDATE)
        kept = stage_planes<L, NPL, HALO, TY, TX, NT, KPS>(sm, src, H, W, y0, x0, b.alpha);
    else
        stage_planes<L, NPL, HALO, TY, TX, NT>(sm, src, H, W, y0, x0);
    const bool active = __syncthreads_or(kept) != 0;
    float uc[KPS][Q];
    {
        float cv[NPL][Q];
        L::template load<Q>(cv, c);
#pragma unroll
        for (int j = 0; j < KPS; ++j)
#pragma unroll
            for (int q = 0; q < Q; ++q) uc[j][q] = valid[q] ? cv[j][q] : 0.f;
    }
    float g[Q];
    float v[Q][KPS][3];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        g[q] = 0.f;
#pragma unroll
        for (int j = 0; j < KPS; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) v[q][j][i] = 0.f;
    }
    cfloat* w = (cfloat*)b.wt + s * 8;
    cfloat* bc = (cfloat*)b.bt + s * 16;
    // this part's range of general orbits
    const int ga0 = (S == 2 && part == 1) ? SPLIT : 2;
    const int ga1 = (S == 2 && part == 0) ? SPLIT : R;
    if (active) {
        if (part == 0) {
#pragma unroll 1
            for (int a = 1; a < R; ++a, w += WS, bc += BS) {
                float sum[NPL][Q];
                quad_planes<L, NPL, Q>(sum, c + a * PX, c - a * PX, c + a, c - a);
                orbit_bwd<T, NPL, Q>(g, v, sum, w, bc);
            }
#pragma unroll 1
            for (int a = 1; 2 * a * a < R * R; ++a, w += WS, bc += BS) {
                float sum[NPL][Q];
                quad_planes<L, NPL, Q>(sum, c + a * PX + a, c + a * PX - a, c - a * PX + a,
                                       c - a * PX - a);
                orbit_bwd<T, NPL, Q>(g, v, sum, w, bc);
            }
        } else {
            constexpr int skip = n_axis_orbits<R>() + n_diag_orbits<R>() + n_general_orbits_below<R>(SPLIT);
            w += skip * WS;
            bc += skip * BS;
        }
        // general orbits: the four base positions (rows c +- a, columns c +- a)
        // are formed once per a; the b loop is unrolled so that every tap is an
        // immediate offset from one of them
#pragma unroll 1
        for (int a = ga0; a < ga1; ++a) {
            const typename L::Pos rp = c + a * PX, rm = c - a * PX, cp = c + a, cm = c - a;
#pragma unroll
            for (int bb = 1; bb < R - 1; ++bb) {
                if (bb < a && a * a + bb * bb < R * R) {
                    float s0[NPL][Q], s1[NPL][Q], sum[NPL][Q];
                    quad_planes<L, NPL, Q>(s0, rp + bb, rp - bb, rm + bb, rm - bb);
                    quad_planes<L, NPL, Q>(s1, cp + bb * PX, cm + bb * PX, cp - bb * PX,
                                           cm - bb * PX);
#pragma unroll
                    for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
                        for (int q = 0; q < Q; ++q) sum[pl][q] = s0[pl][q] + s1[pl][q];
                    orbit_bwd<T, NPL, Q>(g, v, sum, w, bc);
                    w += WS;
                    bc += BS;
                }
            }
        }
    }
    if constexpr (S == 2) {
        // the second part's sums go through the (no longer needed) staging buffer
        __syncthreads();
        float* ho = sm + tc;   // element e of the thread at ho[e * NTC]
        if (part == 1) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                ho[(q * (1 + KPS * 3)) * NTC] = g[q];
#pragma unroll
                for (int j = 0; j < KPS; ++j)
#pragma unroll
                    for (int i = 0; i < 3; ++i) ho[(q * (1 + KPS * 3) + 1 + j * 3 + i) * NTC] = v[q][j][i];
            }
        }
        __syncthreads();
        if (part == 0) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                g[q] += ho[(q * (1 + KPS * 3)) * NTC];
#pragma unroll
                for (int j = 0; j < KPS; ++j)
#pragma unroll
                    for (int i = 0; i < 3; ++i) v[q][j][i] += ho[(q * (1 + KPS * 3) + 1 + j * 3 + i) * NTC];
            }
        }
    }
    // shell-height partials of this tile: ubar at the cell times its
    // coefficient-weighted orbit sums, reduced over the block in a fixed order
    if (part == 0) {
#pragma unroll
        for (int j = 0; j < KPS; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                float pr = 0.f;
#pragma unroll
                for (int q = 0; q < Q; ++q) pr = fmaf(uc[j][q], v[q][j][i], pr);
                pr = wave_sum(pr);
                if (lane == 0) red[wave][j * 3 + i] = pr;
            }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < KPS * 3; e += NT) {
        float acc = 0.f;
#pragma unroll
        for (int wv = 0; wv < NWV; ++wv) acc += red[wv][e];
        const int k = T::kidx[s][e / 3];
        b.part[((size_t)tile * T::NK + k) * 3 + (e % 3)] = acc;
    }

    // direct term from the cell pass + convolution transpose into channel s
    if (part == 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (!valid[q]) continue;
            const uint32_t o = (uint32_t)(gy + q) * (uint32_t)W + (uint32_t)gx;
            float* ga = b.gA + (size_t)s * HW;
            ga[o] = ga[o] + g[q];
        }
    }
    // transpose of the gene diffusion: gP(y) = sum over the disk of numbar(y + d)
    // for the planes pq = s + C i, i = part, part + S, ...  numbar holds values
    // only where alpha does: the disk values are read unconditionally (always
    // in bounds) and those of cells without alpha are dropped by a select, and
    // cells whose 5-neighbourhood has no alpha skip the reads.  All of a cell's
    // reads are issued before the sums.
    if (b.mode == MODE_LOCAL_UPDATE) {
        constexpr int NPQ = 3 * T::NK / T::C;       // gene planes per source channel
        constexpr int NPS = (NPQ + S - 1) / S;      // of them per part
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (!valid[q]) continue;
            const Nbr nb = neighbours(gy + q, gx, H, W);
            const bool au = b.alpha[nb.ou], al = b.alpha[nb.ol], ac = b.alpha[nb.oc],
                       ar = b.alpha[nb.orr], ad = b.alpha[nb.od];
            const bool any = au | al | ac | ar | ad;
            float val[NPS];
#pragma unroll
            for (int ii = 0; ii < NPS; ++ii) val[ii] = 0.f;
            if (any) {
                float dv[NPS][5];
#pragma unroll
                for (int ii = 0; ii < NPS; ++ii) {
                    const int i = part + S * ii;
                    if (i < NPQ) {
                        const float* nbp = b.numbar + (size_t)(s + T::C * i) * HW;
                        dv[ii][0] = nbp[nb.ou];
                        dv[ii][1] = nbp[nb.ol];
                        dv[ii][2] = nbp[nb.oc];
                        dv[ii][3] = nbp[nb.orr];
                        dv[ii][4] = nbp[nb.od];
                    }
                }
#pragma unroll
                for (int ii = 0; ii < NPS; ++ii) {
                    if (part + S * ii < NPQ) {
                        const float vu = au ? dv[ii][0] : 0.f, vl = al ? dv[ii][1] : 0.f;
                        const float vc = ac ? dv[ii][2] : 0.f, vr = ar ? dv[ii][3] : 0.f;
                        const float vd = ad ? dv[ii][4] : 0.f;
                        val[ii] = (((vu + vl) + vc) + vr) + vd;
                    }
                }
            }
#pragma unroll
            for (int ii = 0; ii < NPS; ++ii) {
                const int i = part + S * ii;
                if (i < NPQ) (b.gP + (size_t)(s + T::C * i) * HW)[nb.oc] = val[ii];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 3. fixed-order reduction of the per-tile shell-height partials into gbeta
// ---------------------------------------------------------------------------
// One wave per (k, i): lane l sums tiles l, l + 64, ... in order, then a
// fixed butterfly across the lanes (no LDS, no block barrier).
__global__ __launch_bounds__(64) void bwd_beta_reduce_kernel(const float* part, int n_tiles, int nk,
                                                            const int* n_shells, float* gbeta)
{
    const int e = blockIdx.x;           // (k, i)
    const int k = e / 3, i = e - 3 * (e / 3);
    float acc = 0.f;
    for (int t = threadIdx.x; t < n_tiles; t += 64) acc += part[((size_t)t * nk + k) * 3 + i];
    acc = wave_sum(acc);
    if (threadIdx.x == 0 && i < n_shells[k]) gbeta[k * 3 + i] += acc;
}

template <class T, int R, int TY, int TX, int S>
hipError_t launch_bwd(const BwdArgs& a, const int* d_nshells, float* gbeta, hipStream_t s)
{
    const unsigned cells = (unsigned)a.H * (unsigned)a.W;
    hipLaunchKernelGGL((bwd_cell_kernel<T>), dim3((cells + 255) / 256, T::C), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((bwd_gather_kernel<T, R, TY, TX, S>), dim3(a.n_tiles, T::C),
                       dim3(S * bwd_threads<TY, TX>()), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bwd_beta_reduce_kernel, dim3(T::NK * 3), dim3(64), 0, s, a.part, a.n_tiles,
                       T::NK, d_nshells, gbeta);
    return hipGetLastError();
}

typedef hipError_t (*bwd_launch_fn)(const BwdArgs&, const int*, float*, hipStream_t);

// Gather-pass tile: 16 x 32 cells, or, when that leaves too few tiles to fill
// the device, 8 x 32 cells with two threads per cell.
static bwd_launch_fn find_bwd(int table, int R, bool small)
{
    if (!small) {
        if (table == TABLE_3x15 && R == 12) return &launch_bwd<Table3x15, 12, 16, 32, 1>;
        if (table == TABLE_3x15 && R == 13) return &launch_bwd<Table3x15, 13, 16, 32, 1>;
        if (table == TABLE_1x1 && R == 12) return &launch_bwd<Table1x1, 12, 16, 32, 1>;
        if (table == TABLE_1x1 && R == 13) return &launch_bwd<Table1x1, 13, 16, 32, 1>;
    } else {
        if (table == TABLE_3x15 && R == 12) return &launch_bwd<Table3x15, 12, 8, 32, 2>;
        if (table == TABLE_3x15 && R == 13) return &launch_bwd<Table3x15, 13, 8, 32, 2>;
        if (table == TABLE_1x1 && R == 12) return &launch_bwd<Table1x1, 12, 8, 32, 2>;
        if (table == TABLE_1x1 && R == 13) return &launch_bwd<Table1x1, 13, 8, 32, 2>;
    }
    return nullptr;
}

// ---------------------------------------------------------------------------
// Workspace of lenia_backward_noalloc: a static device array, one copy per
// GPU, held until the process ends.  Its address is looked up once per device
// (hipGetSymbolAddress, with that device current) and passed to the kernels
// like the plan-owned workspaces of lenia_backward.  No element of it is read
// before the call that reads it has written it (the gather and diffusion
// transposes drop the values of cells without alpha through selects), so
// nothing is cleared between calls.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;        // by device ordinal

static lenia_status scratch_address(int dev, void** out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "looking up the static adjoint workspace");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LENIA_OK;
}

static size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Adjoint workspace sizes of a world: ubar [NK][H][W], numbar [3NK][H][W]
// (gene update only) and the per-tile shell-height partials, sized for the
// larger tile count of the two gather tiles.
static size_t bwd_part_tiles(const WorldPlan& w) { return (size_t)((w.W + 31) / 32) * ((w.H + 7) / 8); }

static void bwd_ws_sizes(const WorldPlan& w, size_t sizes[3])
{
    sizes[0] = (size_t)w.NK * w.cells() * sizeof(float);
    sizes[1] = (w.mode == MODE_LOCAL_UPDATE) ? 3 * (size_t)w.NK * w.cells() * sizeof(float) : 0;
    sizes[2] = bwd_part_tiles(w) * w.NK * 3 * sizeof(float);
}

// The plan's adjoint workspaces, allocated on first use: all three or none, so
// a failed allocation leaves the plan as it was and the next call tries again.
static lenia_status ensure_bwd_ws(lenia_plan_t p, const WorldPlan& w)
{
    if (p->bw.ubar) return LENIA_OK;
    size_t sizes[3];
    bwd_ws_sizes(w, sizes);
    void* q[3] = {nullptr, nullptr, nullptr};
    for (int i = 0; i < 3; ++i) {
        if (sizes[i] && device_alloc(&q[i], sizes[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j)
                if (q[j]) (void)hipFree(q[j]);
            return set_error(LENIA_ERR_OUT_OF_MEMORY, "adjoint workspace");
        }
    }
    for (int i = 0; i < 3; ++i)
        if (q[i]) {
            p->allocations.push_back(q[i]);
            p->ws_bytes += sizes[i];
        }
    p->bw.ubar = (float*)q[0];
    p->bw.numbar = (float*)q[1];
    p->bw.part = (float*)q[2];
    p->bw.n_part = (int)bwd_part_tiles(w);
    return LENIA_OK;
}

// Checks the plan and call arguments (nothing enqueued on error).
static lenia_status bwd_validate(lenia_plan_t p, const float* A_t, const float* P_t,
                                 const void* saved, const float* gA_next, const float* gP_next,
                                 float* gA_t, float* gP_t, float* gbeta)
{
    if (!p) return set_error(LENIA_ERR_INVALID_ARG, "plan is NULL");
    if (p->batched) return set_error(LENIA_ERR_STATE, "adjoint needs a single-world plan");
    if (p->rings) return set_error(LENIA_ERR_UNSUPPORTED, "no adjoint for ring-decomposed kernels");
    const WorldPlan& w = p->worlds[0];
    if (w.mode == MODE_GLOBAL) return set_error(LENIA_ERR_UNSUPPORTED, "adjoint needs localized genes");
    const bool small = ((size_t)((w.H + 15) / 16) * ((w.W + 31) / 32) < 1024);
    if (!find_bwd(p->table, p->R, small))
        return set_error(LENIA_ERR_UNSUPPORTED, "no adjoint kernel for this table / R");
    if (!A_t || !P_t || !saved || !gA_next || !gA_t || !gP_t || !gbeta)
        return set_error(LENIA_ERR_INVALID_ARG, "NULL argument (only gP_next may be NULL)");
    const uintptr_t al = (uintptr_t)A_t | (uintptr_t)P_t | (uintptr_t)saved | (uintptr_t)gA_next |
                         (uintptr_t)gA_t | (uintptr_t)gP_t | (uintptr_t)gbeta | (uintptr_t)gP_next;
    if (al & 3) return set_error(LENIA_ERR_INVALID_ARG, "buffers must be 4-byte aligned");
    const void* ins[] = {A_t, P_t, saved, gA_next, gP_next};
    for (const void* q : ins)
        if (q && (q == (const void*)gA_t || q == (const void*)gP_t))
            return set_error(LENIA_ERR_INVALID_ARG, "gA_t / gP_t must not alias an input");
    if ((const void*)gA_t == (const void*)gP_t)
        return set_error(LENIA_ERR_INVALID_ARG, "gA_t and gP_t must differ");
    return LENIA_OK;
}

// LENIA_FLAG_CHECK_FINITE on the adjoint's buffers.
static lenia_status bwd_debug_checks(lenia_plan_t p, const float* A_t, const float* P_t,
                                     const void* saved, const float* gA_next, const float* gP_next,
                                     float* gA_t, float* gP_t, float* gbeta, hipStream_t s)
{
    const WorldPlan& w = p->worlds[0];
    const size_t ab = w.a_elems() * sizeof(float), pb = w.p_elems() * sizeof(float);
    const DebugBuf db[] = {{A_t, ab, "A_t", true},
                           {P_t, pb, "P_t", true},
                           {saved, (size_t)w.NK * w.cells() * sizeof(float), "saved", true},
                           {(const char*)saved + (size_t)w.NK * w.cells() * sizeof(float), w.cells(),
                            "saved alpha", false},
                           {gA_next, ab, "gA_next", true},
                           {gP_next, pb, "gP_next", true},
                           {gA_t, ab, "gA_t", false},
                           {gP_t, pb, "gP_t", false},
                           {gbeta, (size_t)w.NK * 3 * sizeof(float), "gbeta", true}};
    return debug_checks(p, db, 9, s);
}

// Enqueues the three adjoint kernels with the given workspaces (every element
// of them that a kernel reads is written earlier in the same call).
static lenia_status bwd_enqueue(lenia_plan_t p, const float* A_t, const float* P_t,
                                const void* saved, const float* gA_next, const float* gP_next,
                                float* gA_t, float* gP_t, float* gbeta, float* ubar, float* numbar,
                                float* part, hipStream_t s)
{
    const WorldPlan& w = p->worlds[0];
    const bool small = ((size_t)((w.H + 15) / 16) * ((w.W + 31) / 32) < 1024);
    const int kBwdTY = small ? 8 : 16, kBwdTX = 32;
    bwd_launch_fn fn = find_bwd(p->table, p->R, small);
    const int tiles_x = (w.W + kBwdTX - 1) / kBwdTX;
    BwdArgs a{};
    a.A = A_t;
    a.P = P_t;
    a.U = (const float*)saved;
    a.alpha = (const uint8_t*)saved + (size_t)w.NK * w.cells() * sizeof(float);
    a.gA1 = gA_next;
    a.gP1 = gP_next;
    a.gA = gA_t;
    a.gP = gP_t;
    a.ubar = ubar;
    a.numbar = numbar;
    a.part = part;
    a.wt = w.d_wt;
    a.bt = w.d_bt;
    a.H = w.H;
    a.W = w.W;
    a.tiles_x = tiles_x;
    a.n_tiles = tiles_x * ((w.H + kBwdTY - 1) / kBwdTY);
    a.dt = (float)w.dt;
    a.eps = eps_below(w.eps);
    a.mode = w.mode;
    hipError_t e = fn(a, w.d_nshells, gbeta, s);
    if (e != hipSuccess) return hip_fail(e, "adjoint launch");
    return LENIA_OK;
}

}  // namespace lenia

using namespace lenia;

extern "C" lenia_status lenia_backward(lenia_plan_t p, const float* A_t, const float* P_t,
                                       const void* saved, const float* gA_next,
                                       const float* gP_next, float* gA_t, float* gP_t,
                                       float* gbeta, void* stream)
{
    try {
        lenia_status st = bwd_validate(p, A_t, P_t, saved, gA_next, gP_next, gA_t, gP_t, gbeta);
        if (st != LENIA_OK) return st;
        const WorldPlan& w = p->worlds[0];
        if ((st = bwd_debug_checks(p, A_t, P_t, saved, gA_next, gP_next, gA_t, gP_t, gbeta,
                                   (hipStream_t)stream)) != LENIA_OK)
            return st;
        if ((st = ensure_bwd_ws(p, w)) != LENIA_OK) return st;
        return bwd_enqueue(p, A_t, P_t, saved, gA_next, gP_next, gA_t, gP_t, gbeta, p->bw.ubar,
                           p->bw.numbar, p->bw.part, (hipStream_t)stream);
    } catch (...) {
        return set_error(LENIA_ERR_STATE, "exception in lenia_backward");
    }
}

extern "C" lenia_status lenia_backward_noalloc(lenia_plan_t p, const float* A_t, const float* P_t,
                                               const void* saved, const float* gA_next,
                                               const float* gP_next, float* gA_t, float* gP_t,
                                               float* gbeta, void* stream)
{
    try {
        lenia_status st = bwd_validate(p, A_t, P_t, saved, gA_next, gP_next, gA_t, gP_t, gbeta);
        if (st != LENIA_OK) return st;
        const WorldPlan& w = p->worlds[0];
        size_t sizes[3];
        bwd_ws_sizes(w, sizes);
        const size_t need = align256(sizes[0]) + align256(sizes[1]) + sizes[2];
        if (need > kScratchBytes)
            return set_error(LENIA_ERR_UNSUPPORTED,
                             "lenia_backward_noalloc: this world needs " + std::to_string(need) +
                                 " workspace bytes, the static workspace holds " +
                                 std::to_string(kScratchBytes) +
                                 " (about 2.7e5 cells with 15 kernels); use lenia_backward");
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
        if (dev != p->device)
            return set_error(LENIA_ERR_STATE, "the plan's device is not the current device");
        if ((st = bwd_debug_checks(p, A_t, P_t, saved, gA_next, gP_next, gA_t, gP_t, gbeta,
                                   (hipStream_t)stream)) != LENIA_OK)
            return st;
        void* base = nullptr;
        if ((st = scratch_address(dev, &base)) != LENIA_OK) return st;
        char* b = (char*)base;
        float* ubar = (float*)b;
        float* numbar = sizes[1] ? (float*)(b + align256(sizes[0])) : nullptr;
        float* part = (float*)(b + align256(sizes[0]) + align256(sizes[1]));
        return bwd_enqueue(p, A_t, P_t, saved, gA_next, gP_next, gA_t, gP_t, gbeta, ubar, numbar,
                           part, (hipStream_t)stream);
    } catch (...) {
        return set_error(LENIA_ERR_STATE, "exception in lenia_backward_noalloc");
    }
}
