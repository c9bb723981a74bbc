// Potentials by tile-local DFT as matrix products on the MFMA units (gfx950).
//
// u_k = K~_k * A_src(k) is a circular convolution; on a 64 x 64 window of A
// (the 40 x 40 output tile plus an R-cell halo, R = 12) it equals the inverse
// DFT of DFT(window) times the kernel's DFT (Section 2.1 computes the
// convolution through the convolution theorem).  The kernel is even, so its
// DFT is real, and the window is real, so its DFT is Hermitian: only the
// column frequencies b = 0..32 are formed.  Columns 0 and 32 of the row
// transform are real (sin(0) = sin(pi j) = 0); they share one complex column,
// Y0 + i Y32, which keeps every half spectrum at exactly 32 columns.  With
// C[f][i] = cos(2 pi f i / 64), S[f][i] = sin(2 pi f i / 64) and
// real-embedded complex matrices, per tile:
//   GEMM1  [Y_re | Y_im]     (64 x 64)  = X (64 x 64) F1                  per channel
//          F1 = [C_0 .. C_31 | (-1)^j, -S_1 .. -S_31] (column b of each half)
//   GEMM2  [T_re; T_im]      (128 x 32) = [[C, S], [-S, C]] [Y_re; Y_im]  per channel
//          T[a][b] = Xh[a][b] for b >= 1, and T[a][0] = Xh[a][0] + i Xh[a][32]
//   U[a][b] = Xh[a][b] Khat_k[a][b] for b >= 1; the packed column holds
//   U[a][0] + i U[a][32] = T[a] (K0 + K32) / 2 + conj(T[-a]) (K0 - K32) / 2
//   with K0 = Khat_k[a][0], K32 = Khat_k[a][32]                           per kernel
//   GEMM3  [Z_re; Z_im]^T    (32 x 2V)  = [U_re; U_im]^T [[C_V, -S_V], [S_V, C_V]]^T
//   GEMM4  u_k               (V x V)    = [Z_re | Z_im] F4
//          F4 row b (real part) = 2 cos(2 pi b (q + R) / 64), row 0 = 1;
//          row 32 + b (imaginary part) = -2 sin(...), row 32 = (-1)^(q + R)
// where C_V / S_V keep the V output rows of the inverse transform.  GEMM3's
// column 0 is the inverse of two Hermitian columns, so its real and imaginary
// parts are the real inverses of columns 0 and 32, and GEMM4 is the
// half-spectrum inverse along b (each column b = 1..31 stands for itself and
// its conjugate 64 - b).
// Every GEMM runs on v_mfma_f32_16x16x32_bf16 (or _f16) with FP32
// accumulation; each operand x is split as hi = e(x), lo = e(x - hi) in the
// operand type e and a product is hi*hi + hi*lo + lo*hi: about 16 significant
// bits with bf16 and 22 with fp16.  fp16 keeps those 22 bits only while lo
// stays a normal number, |x| >= 2^-3, so every operand is scaled by a power
// of two that puts its largest possible magnitude just below 2^14 (far from
// fp16's largest value, 65504): the DFT matrices (|x| <= 1) by 2^14 on the
// host (F4, |x| <= 2, by 2^13), the window by 2^a from its largest magnitude,
// and each intermediate by the bound its GEMM implies (a K-term sum of
// products below 2^28).  An element then loses precision only below 2^-17 of
// that bound, where its absolute error (half of fp16's subnormal step) is
// 2^-39 of it.  The scales are exact, so they cancel in the result and leave
// the bf16 form's rounding unchanged.  The DFT matrices are built in FP64 on
// the host and split there; data operands are split here.
//
// MFMA operand layouts (16x16x32): lane l holds A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16] for j < 8; the 16 x 16 FP32 result has
// D[4 (l / 16) + j][l % 16] in lane l, j < 4.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "lenia.h"
#include "lenia_device.h"
#include "lenia_internal.h"
#include "lenia_plan.h"

// A split must take hi and lo from one rounded FP32 value.  Left alone, the
// compiler converts a product x = a * b to fp16 for the stored hi from the
// rounded product, but rematerializes hi for lo = e(x - hi) as one fused
// v_fma_mix (the exact product rounded once to fp16); at an fp16 rounding tie
// the two differ and that element loses one hi-ulp (2^-11 relative).  Every
// split therefore reads its value through an empty register-constraint asm
// statement, which the compiler cannot look through, and floating-point
// contraction is off in this file.
#pragma clang fp contract(off)

namespace lenia {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Operand types of the split products: bf16 (8 significant bits per part)
// or fp16 (11 bits per part, a narrower exponent range).
template <class E>
struct Op;
template <>
struct Op<__bf16> {
    typedef __bf16 v8 __attribute__((ext_vector_type(8)));
    typedef __bf16 v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ f32x4 mma(const v8& a, const v8& b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct Op<_Float16> {
    typedef _Float16 v8 __attribute__((ext_vector_type(8)));
    typedef _Float16 v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ f32x4 mma(const v8& a, const v8& b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// Power-of-two scales of the operands (see the header): F1..F3 carry 2^14 and
// F4 2^13; GEMM1's output (64 terms below 2^28) is split at 2^-20, the
// spectral product (the transformed channel, 128 terms below 2^28, times a
// spectrum of magnitude <= 2^-12) at 2^-9, folded into the spectra, and
// GEMM3's output (128 terms) at 2^-21.  With the window scaled by 2^a the
// potentials come out scaled by 2^(a + 5).
constexpr int kMatExp = 14;
constexpr int kF4Exp = 13;
constexpr int kYExp = -20;
constexpr int kUExp = -9;
constexpr int kZExp = -21;
constexpr int kOutExp = 5;

constexpr int DT = 64;                   // DFT tile
constexpr int DT2 = 128;                 // real-embedded complex dimension of a full axis
constexpr int NB = 32;                   // half-spectrum columns (0 and 32 packed in column 0)
constexpr int XS_P = DT + 8;             // LDS row pitches (operand-type / fp32 elements)
constexpr int YT_P = DT2 + 16;
constexpr int TH_P = DT2 + 4;
constexpr int UST_P = DT2 + 16;
constexpr int ZC_P = DT + 8;
constexpr int ZC_ROWS = 48;              // GEMM4 rows (V <= 48)
constexpr int F3_ROWS = 80;              // GEMM3 columns (2V <= 80)

struct DftTables {
    const void* f1t;      // [2][64 c][64 j]  hi, lo of F1^T
    const void* f2;       // [2][128][128]    hi, lo of [[C, S], [-S, C]]
    const void* f3;       // [2][80][128]     hi, lo of [[C_V, -S_V], [S_V, C_V]] (rows >= 2V zero)
    const void* f4t;      // [2][48 q][64 k]  hi, lo of F4^T (rows >= V zero)
    const float* khat;    // [NK][33 b][64 a] real kernel spectra / 64^2, times 2^kUExp
};

struct DftArgs {
    const float* A;       // [C][H][W]
    float* U;             // [NK][H][W] potentials (output of the potentials-only kernel)
    DftTables t;
    int H, W, tiles_x, n_tiles;
    WorldArgs wd;         // the fused step: genes in, A' and P' out (MODE_LOCAL_UPDATE)
};

template <class E>
__device__ __forceinline__ f32x4 mma3(const typename Op<E>::v8& ah, const typename Op<E>::v8& al,
                                      const typename Op<E>::v8& bh, const typename Op<E>::v8& bl, f32x4 c)
{
    c = Op<E>::mma(al, bh, c);
    c = Op<E>::mma(ah, bl, c);
    c = Op<E>::mma(ah, bh, c);
    return c;
}

// The value as an opaque FP32 register (see the split note above).
__device__ __forceinline__ float opaque(float v)
{
    asm volatile("" : "+v"(v));
    return v;
}

template <class E>
__device__ __forceinline__ void split8(const float (&x)[8], typename Op<E>::v8& hi, typename Op<E>::v8& lo)
{
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float v = opaque(x[j]);
        const E h = (E)v;
        hi[j] = h;
        lo[j] = (E)(v - (float)h);
    }
}

template <class E>
__device__ __forceinline__ typename Op<E>::v8 ld8(const E* p) { return *(const typename Op<E>::v8*)p; }

// A buffer descriptor over a table of `bytes` bytes.
__device__ __forceinline__ plane_t make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// 8 operand-type elements (16 bytes) at byte offset off + soff of a table.
template <class E>
__device__ __forceinline__ typename Op<E>::v8 bld8(plane_t r, uint32_t off, int soff)
{
    return __builtin_bit_cast(typename Op<E>::v8, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, soff, 0));
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Writes 4 consecutive values (split) as hi / lo.
template <class E>
__device__ __forceinline__ void st4_split(E* hi, E* lo, const f32x4& v)
{
    typename Op<E>::v4 h, l;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float x = opaque(v[j]);
        const E b = (E)x;
        h[j] = b;
        l[j] = (E)(x - (float)b);
    }
    *(typename Op<E>::v4*)hi = h;
    *(typename Op<E>::v4*)lo = l;
}

// A workgroup barrier for LDS traffic only: this wave's LDS accesses complete,
// then s_barrier.  Vector-memory operations stay in flight (the gene planes'
// DMA into LDS, global stores); the memory clobber keeps the compiler from
// moving memory accesses across it.  Waves of a workgroup exchange data only
// through LDS here.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// The same after this wave's vector-memory operations (its DMA into LDS) have
// completed too.
__device__ __forceinline__ void dma_barrier()
{
    asm volatile("s_waitcnt vmcnt(0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// The same, leaving this wave's N newest vector-memory operations (the next
// kernel's gene DMA) in flight.
template <int N>
__device__ __forceinline__ void dma_barrier_keep()
{
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_waitcnt lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

// Gene diffusion of one cell from a staged plane (side hs, the cell at c):
// the disk values in the epilogue's order up, left, centre, right, down.
__device__ __forceinline__ float diffuse_staged(const float* g, int c, int hs, float cs, float ncs)
{
    const float v[5] = {g[c - hs], g[c - 1], g[c], g[c + 1], g[c + hs]};
    return diffuse_disk(v, cs, ncs);
}

// Height of the cell strips of the fused step: the least h for which a column
// of ceil(V / h) strips per tile column fits 256 threads.
constexpr int strip_height(int v)
{
    int h = 1;
    while (((v + h - 1) / h) * v > 256) ++h;
    return h;
}

// Torus coordinate of any integer position.
__device__ __forceinline__ int wrap_any(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// The fused step (FUSED = true) replaces the potentials' trip through HBM:
// each u_k goes from GEMM4 to LDS, and every thread carries the growth sums
// and the alpha test of its cells from one kernel to the next.  The three
// gene planes a kernel's growth reads (m, s, h) are staged into LDS with the
// tile's 1-cell ring by direct-to-LDS buffer loads issued when the kernel's
// turn begins, so their latency runs under its transform.  The result is the
// epilogue's, bitwise: the same diffusion, test and growth arithmetic, the
// growth summed in the same kernel order.
template <class T, int R, class E, bool FUSED>
__global__ __launch_bounds__(256, 2) void dft_conv_kernel(DftArgs g)
{
    typedef typename Op<E>::v8 ev8;
    const plane_t f1r = make_rsrc(g.t.f1t, 2 * DT * DT * sizeof(E));
    const plane_t f2r = make_rsrc(g.t.f2, 2 * DT2 * DT2 * sizeof(E));
    const E* f3m = (const E*)g.t.f3;
    const E* f4t = (const E*)g.t.f4t;
    constexpr int V = DT - 2 * R;
    static_assert(V <= ZC_ROWS && 2 * V <= F3_ROWS, "output tile exceeds the GEMM layout");
    // LDS (53 KB, three workgroups per CU): the half spectrum T of the channel
    // being processed (fp32), plus a scratch region shared by the forward
    // stages (Xs, Yt) and the inverse stages (the split spectral product Ust
    // and Zc, which do not overlap each other)
    //
    // The fused step also stages gene planes (below) in two buffers, so that
    // the next kernel's planes load while this one's are used; to fit two
    // workgroups per CU it overlays more of the scratch: Yt on Xs (GEMM1 keeps
    // its results in registers across a barrier), and Zc on Ust (likewise
    // GEMM3), with u_k of the current kernel after Zc.
    constexpr int HS = V + 2;
    constexpr int NGI = (HS * HS + 255) / 256;      // DMA instructions per wave and plane
    constexpr int GSLOT = 256 * NGI;
    // the fused step gives each thread a vertical strip of SH cells of the
    // V x V tile: column sq, rows p0 .. p0 + SH - 1 (strips of SH rows, the
    // last one moved up to end at row V - 1, its rows shared with the strip
    // above left to that one)
    constexpr int SH = strip_height(V);
    constexpr int NSG = (V + SH - 1) / SH;          // strips per column
    static_assert(NSG * V <= 256, "a strip per thread");
    constexpr int XS_E = 2 * DT * XS_P, YT_E = 2 * NB * YT_P, UST_E = 2 * NB * UST_P;
    constexpr int ZC_E = 2 * ZC_ROWS * ZC_P, UT_E = V * V * 4 / (int)sizeof(E);
    constexpr int FWD_E = FUSED ? (XS_E > YT_E ? XS_E : YT_E) : XS_E + YT_E;
    constexpr int INV_E = FUSED ? ((ZC_E + UT_E > UST_E) ? ZC_E + UT_E : UST_E) : UST_E + ZC_E;
    constexpr int SCRATCH_E = (FWD_E > INV_E) ? FWD_E : INV_E;
    static_assert(FUSED || V * V * 4 <= UST_E * (int)sizeof(E), "u_k must fit in Ust");
    __shared__ __attribute__((aligned(16))) float th[NB * TH_P];
    __shared__ __attribute__((aligned(16))) E scr[SCRATCH_E];
    __shared__ float wmax[4];
    __shared__ __attribute__((aligned(16))) float gstA[FUSED ? 3 * GSLOT : 1];
    __shared__ __attribute__((aligned(16))) float gstB[FUSED ? 3 * GSLOT : 1];
    E* xs_hi = scr;
    E* xs_lo = scr + DT * XS_P;
    E* yt_hi = FUSED ? scr : scr + XS_E;
    E* yt_lo = yt_hi + NB * YT_P;
    E* ust_hi = scr;
    E* ust_lo = scr + NB * UST_P;
    E* zc_hi = FUSED ? scr : scr + UST_E;
    E* zc_lo = zc_hi + ZC_ROWS * ZC_P;
    float* ut = FUSED ? (float*)(scr + ZC_E) : (float*)scr;

    const int H = g.H, W = g.W;
    const size_t HW = (size_t)H * W;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tyi = tile / g.tiles_x, txi = tile - tyi * g.tiles_x;
    const int y0 = tyi * V, x0 = txi * V;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = (lane >> 4) * 8, ld = (lane >> 4) * 4;
    const bool single_wrap = (H >= DT) && (W >= DT);

    // GEMM3 (Z^T, 32 x 80) has 2 row blocks x 5 column blocks: wave w takes
    // column block w of both row blocks, and waves 0 and 1 also row block w of
    // column block 4; the B fragments of a wave's column blocks stay in
    // registers.  GEMM4 (u, 48 x 48, K = 64): wave w < 3 takes column block w.
    ev8 b3h[2][4], b3l[2][4];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int nt = (q == 0) ? wave : 4;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int row = 16 * nt + lr, k0 = 32 * ks + lk;
            b3h[q][ks] = ld8(f3m + row * DT2 + k0);
            b3l[q][ks] = ld8(f3m + F3_ROWS * DT2 + row * DT2 + k0);
        }
    }
    ev8 b4h[2], b4l[2];
    {
        const int row = 16 * (wave < 3 ? wave : 0) + lr;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            b4h[ks] = ld8(f4t + row * DT + 32 * ks + lk);
            b4l[ks] = ld8(f4t + ZC_ROWS * DT + row * DT + 32 * ks + lk);
        }
    }
    // spectral-product work of this thread: column b, frequencies a8 .. a8 + 7.
    // Column 0 (the packed one, extra work) falls to wave 3, which has the
    // fewest GEMM3 tiles and no GEMM4 tile.
    const int sp_b = ((threadIdx.x >> 3) + 8) & (NB - 1), sp_a8 = (threadIdx.x & 7) * 8;
    // this thread's 16 window elements: rows r = threadIdx.x / 16 + 16 it,
    // columns c4 .. c4 + 3 (the same for every it), wrapped on the torus; the
    // byte offset in a plane is wrow[it] + wcol[j]
    const uint32_t pb = 4u * (uint32_t)HW;
    constexpr int NWIN = DT * DT / 4 / 256;
    uint32_t wrow[NWIN], wcol[4];
#pragma unroll
    for (int it = 0; it < NWIN; ++it) {
        const int r = (threadIdx.x + 256 * it) / (DT / 4);
        int gy = y0 - R + r, gx = 0;
        wrap2(gy, gx, H, W, single_wrap);
        wrow[it] = 4u * (uint32_t)gy * (uint32_t)W;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        int gy = 0, gx = x0 - R + (threadIdx.x % (DT / 4)) * 4 + j;
        wrap2(gy, gx, H, W, single_wrap);
        wcol[j] = 4u * (uint32_t)gx;
    }

    // fused step: the per-lane offsets of the staged gene window (DMA
    // instruction i of wave w loads window elements 256 i + 64 w + lane, row
    // by row from (y0 - 1, x0 - 1) on the torus), and the state of the SH
    // cells of this thread's strip: growth sums per target channel and the
    // position (in the kernel order the tile follows) where alpha failed,
    // kAlive while it holds, -1 off the world or left to another strip
    const WorldArgs& wd = g.wd;
    constexpr int kAlive = T::NK;
    uint32_t goff[FUSED ? NGI : 1];
    float gsum[FUSED ? SH : 1][T::C];
    int dead_at[FUSED ? SH : 1];
    if constexpr (FUSED) {
#pragma unroll
        for (int i = 0; i < NGI; ++i) {
            const int e = 256 * i + 64 * wave + lane;
            uint32_t o = 0;
            if (e < HS * HS) {
                const int row = e / HS, col = e - row * HS;
                const int gy = wrap_any(y0 - 1 + row, H), gx = wrap_any(x0 - 1 + col, W);
                o = 4u * ((uint32_t)gy * (uint32_t)W + (uint32_t)gx);
            }
            goff[i] = o;
        }
        const int sgr = threadIdx.x / V, sq = threadIdx.x - sgr * V;
        const int p0 = min(SH * sgr, V - SH);
#pragma unroll
        for (int r = 0; r < SH; ++r) {
            const int p = p0 + r;
            const bool own = sgr < NSG && p >= SH * sgr;
            dead_at[r] = (own && y0 + p < H && x0 + sq < W) ? kAlive : -1;
#pragma unroll
            for (int c = 0; c < T::C; ++c) gsum[r][c] = 0.f;
        }
    }

    // gene planes kk, NK + kk, 2 NK + kk (m, s, h of kernel kk) into a staging
    // buffer by direct-to-LDS loads; the buffers are distinct arrays, so that
    // the compiler's own waits before reading one do not wait for the other's
    auto stage_genes = [&](int kk, float* gb) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const plane_t pl = plane(wd.P + (size_t)(q * T::NK + kk) * HW, pb);
#pragma unroll
            for (int i = 0; i < NGI; ++i)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    pl, (__attribute__((address_space(3))) void*)(gb + q * GSLOT + 256 * i + 64 * wave), 4,
                    (int)goff[i], 0, 0, 0);
        }
    };
    if constexpr (FUSED) stage_genes(T::kidx[0][0], gstA);
    // this thread's spectrum values (row sp_b, and row 32 for the packed
    // column).  The potentials-only kernel loads them one kernel ahead, so
    // that their latency runs under the transforms of the kernel before (1.34
    // -> 1.30 ms at 4096^2); the fused step, whose registers are all taken,
    // loads them when the kernel's turn begins.
    f32x4 ks0, ks1, ks2, ks3;
    auto load_spectrum = [&](int kk) {
        const float* kh = g.t.khat + (size_t)kk * (NB + 1) * DT;
        ks0 = *(const f32x4*)(kh + sp_b * DT + sp_a8);
        ks1 = *(const f32x4*)(kh + sp_b * DT + sp_a8 + 4);
        if (sp_b == 0) {
            ks2 = *(const f32x4*)(kh + NB * DT + sp_a8);
            ks3 = *(const f32x4*)(kh + NB * DT + sp_a8 + 4);
        }
    };
    if constexpr (!FUSED) load_spectrum(T::kidx[0][0]);

    // ---- per source channel: forward transform, then its kernels ------------
#pragma unroll 1
    for (int s = 0; s < T::C; ++s) {
        // the forward transforms' tables are read again for each channel:
        // an opaque zero offset keeps the compiler from hoisting these
        // loop-invariant loads out of the channel loop, where they would hold
        // 128 registers for the whole tile
        int zoff;
        asm volatile("s_mov_b32 %0, 0" : "=s"(zoff));
        lds_barrier();
        // load the 64 x 64 window (wrapped) and its largest magnitude, then
        // stage it scaled by 2^a (largest magnitude below 2^14) as hi / lo
        f32x4 win[NWIN];
        float vmax = 0.f;
        const plane_t apl = plane(g.A + (size_t)s * HW, pb);
        // (the row offsets pass through an empty asm statement, so that the
        // 16 sums are formed here rather than kept live across the loop)
#pragma unroll
        for (int it = 0; it < NWIN; ++it) asm volatile("" : "+v"(wrow[it]));
#pragma unroll
        for (int it = 0; it < NWIN; ++it)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                win[it][j] = pld(apl, wrow[it] + wcol[j]);
                vmax = fmaxf(vmax, fabsf(win[it][j]));
            }
        vmax = wave_max(vmax);
        if (lane == 0) wmax[wave] = vmax;
        lds_barrier();
        vmax = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
        int ea = 0;
        (void)frexpf(vmax, &ea);                        // vmax < 2^ea
        const int a = (vmax > 0.f) ? min(max(14 - ea, -100), 100) : 0;
        const float sx = ldexpf(1.f, a);
        const float sout = ldexpf(1.f, -(a + kOutExp));
#pragma unroll
        for (int it = 0; it < NWIN; ++it) {
            const int i = threadIdx.x + 256 * it;
            const int r = i / (DT / 4), c4 = (i % (DT / 4)) * 4;
            st4_split<E>(xs_hi + r * XS_P + c4, xs_lo + r * XS_P + c4, win[it] * sx);
        }
        lds_barrier();
        // GEMM1: wave w computes rows 16w..16w+15 of Y, all 4 column blocks;
        // each k-step's eight B fragments are loaded before its products
        {
            f32x4 acc[4];
#pragma unroll
            for (int n = 0; n < 4; ++n) acc[n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const int k0 = 32 * ks + lk;
                ev8 bh[4], bl[4];
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    const uint32_t o = 2u * (uint32_t)((16 * n + lr) * DT + k0);
                    bh[n] = bld8<E>(f1r, o, zoff);
                    bl[n] = bld8<E>(f1r, o + 2u * DT * DT, zoff);
                }
                const ev8 ah = ld8(xs_hi + (16 * wave + lr) * XS_P + k0);
                const ev8 al = ld8(xs_lo + (16 * wave + lr) * XS_P + k0);
#pragma unroll
                for (int n = 0; n < 4; ++n) acc[n] = mma3<E>(ah, al, bh[n], bl[n], acc[n]);
            }
            if constexpr (FUSED) lds_barrier();    // every wave has read Xs, which Yt overlays
            // Y column c = 16n + lr, rows i = 16w + ld + j  ->  Yt[c % 32][64 (c / 32) + i]
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const int c = 16 * n + lr;
                const int off = (c % NB) * YT_P + DT * (c / NB) + 16 * wave + ld;
                st4_split<E>(yt_hi + off, yt_lo + off, acc[n] * ldexpf(1.f, kYExp));
            }
        }
        lds_barrier();
        // GEMM2: wave w computes row blocks 2w, 2w+1 of T, both column blocks;
        // the A fragments of two k-steps are loaded at a time
        {
            f32x4 acc[2][2];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int n = 0; n < 2; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kh = 0; kh < 2; ++kh) {
                ev8 ah[2][2], al[2][2];
#pragma unroll
                for (int kq = 0; kq < 2; ++kq)
#pragma unroll
                    for (int m = 0; m < 2; ++m) {
                        const int row = 16 * (2 * wave + m) + lr;
                        const uint32_t o = 2u * (uint32_t)(row * DT2 + 32 * (2 * kh + kq) + lk);
                        ah[kq][m] = bld8<E>(f2r, o, zoff);
                        al[kq][m] = bld8<E>(f2r, o + 2u * DT2 * DT2, zoff);
                    }
#pragma unroll
                for (int kq = 0; kq < 2; ++kq) {
                    const int k0 = 32 * (2 * kh + kq) + lk;
#pragma unroll
                    for (int n = 0; n < 2; ++n) {
                        const ev8 bh = ld8(yt_hi + (16 * n + lr) * YT_P + k0);
                        const ev8 bl = ld8(yt_lo + (16 * n + lr) * YT_P + k0);
#pragma unroll
                        for (int m = 0; m < 2; ++m) acc[m][n] = mma3<E>(ah[kq][m], al[kq][m], bh, bl, acc[m][n]);
                    }
                }
            }
            // T row r = 16 (2w + m) + ld + j (re: a, im: 64 + a), column b = 16n + lr  ->  th[b][r]
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int n = 0; n < 2; ++n) {
                    const int b = 16 * n + lr, r = 16 * (2 * wave + m) + ld;
                    *(f32x4*)(th + b * TH_P + r) = acc[m][n];
                }
        }
        lds_barrier();
#pragma unroll 1
        for (int j = 0; j < T::KPS; ++j) {
            const int k = T::kidx[s][j];
            if constexpr (FUSED) load_spectrum(k);
            // the spectral product U = Xh * Khat_k, split into LDS once for
            // all waves: real part at column a, imaginary part at 64 + a
            {
                const float* xr = th + sp_b * TH_P + sp_a8;
                const f32x4 r0 = *(const f32x4*)xr, r1 = *(const f32x4*)(xr + 4);
                const f32x4 i0 = *(const f32x4*)(xr + DT), i1 = *(const f32x4*)(xr + DT + 4);
                const f32x4 k0 = ks0, k1 = ks1;
                float ure[8], uim[8];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    ure[q] = r0[q] * k0[q];
                    ure[4 + q] = r1[q] * k1[q];
                    uim[q] = i0[q] * k0[q];
                    uim[4 + q] = i1[q] * k1[q];
                }
                if (sp_b == 0) {
                    // packed column: T[a] (K0 + K32) / 2 + conj(T[-a]) (K0 - K32) / 2
                    const f32x4 m0 = ks2, m1 = ks3;
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const float K0 = (q < 4) ? k0[q] : k1[q - 4];
                        const float K32 = (q < 4) ? m0[q] : m1[q - 4];
                        const float tr = (q < 4) ? r0[q] : r1[q - 4];
                        const float ti = (q < 4) ? i0[q] : i1[q - 4];
                        const int am = (DT - (sp_a8 + q)) & (DT - 1);
                        const float trm = th[am], tim = th[DT + am];
                        const float P = 0.5f * (K0 + K32), Q = 0.5f * (K0 - K32);
                        ure[q] = tr * P + trm * Q;
                        uim[q] = ti * P - tim * Q;
                    }
                }
                ev8 uh, ul;
                split8<E>(ure, uh, ul);
                *(ev8*)(ust_hi + sp_b * UST_P + sp_a8) = uh;
                *(ev8*)(ust_lo + sp_b * UST_P + sp_a8) = ul;
                split8<E>(uim, uh, ul);
                *(ev8*)(ust_hi + sp_b * UST_P + DT + sp_a8) = uh;
                *(ev8*)(ust_lo + sp_b * UST_P + DT + sp_a8) = ul;
            }
            // the next kernel's genes load while this one is transformed and
            // its cells computed (issued after the spectra are read, so that
            // no wait for those loads waits for the DMA too)
            const int pos = s * T::KPS + j;
            if constexpr (!FUSED)
                if (pos + 1 < T::NK) load_spectrum(T::kidx[(pos + 1) / T::KPS][(pos + 1) % T::KPS]);
            if constexpr (FUSED) {
                if (pos + 1 < T::NK) {
                    const int kn = T::kidx[(pos + 1) / T::KPS][(pos + 1) % T::KPS];
                    if ((pos + 1) & 1) stage_genes(kn, gstB);
                    else stage_genes(kn, gstA);
                }
            }
            lds_barrier();    // Ust is complete; the previous GEMM4 is done with Zc
            // GEMM3: Z^T (32 x 80) = Ust^T (32 x 128) F3^T
            {
                f32x4 acc[2], acc4 = f32x4{0.f, 0.f, 0.f, 0.f};
                acc[0] = acc[1] = acc4;
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int k0 = 32 * ks + lk;          // a, or 64 + a for the imaginary part
#pragma unroll
                    for (int m = 0; m < 2; ++m) {
                        const int b = 16 * m + lr;
                        const ev8 ah = ld8(ust_hi + b * UST_P + k0);
                        const ev8 al = ld8(ust_lo + b * UST_P + k0);
                        acc[m] = mma3<E>(ah, al, b3h[0][ks], b3l[0][ks], acc[m]);
                        if (m == wave) acc4 = mma3<E>(ah, al, b3h[1][ks], b3l[1][ks], acc4);
                    }
                }
                if constexpr (FUSED) lds_barrier();    // every wave has read Ust, which Zc overlays
                // Z^T row b = 16m + ld + j, column p' = 16 nt + lr -> Zc[p' mod V][32 (p' >= V) + b]
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    if (q == 2 && wave >= 2) break;
                    const int nt = (q < 2) ? wave : 4;
                    const int m = (q < 2) ? q : wave;
                    const int pp = 16 * nt + lr;
                    if (pp < 2 * V) {
                        const int p = (pp < V) ? pp : pp - V, col0 = (pp < V) ? 0 : NB;
                        const int off = p * ZC_P + col0 + 16 * m + ld;
                        st4_split<E>(zc_hi + off, zc_lo + off, ((q < 2) ? acc[q] : acc4) * ldexpf(1.f, kZExp));
                    }
                }
            }
            lds_barrier();    // Zc is complete; every wave has read Ust
            // GEMM4: u (48 x 48) = Zc (48 x 64) F4; wave w < 3 computes column block w
            if (wave < 3) {
                f32x4 o[3];
#pragma unroll
                for (int m = 0; m < 3; ++m) o[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const int k0 = 32 * ks + lk;
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        const int row = 16 * m + lr;
                        const ev8 ah = ld8(zc_hi + row * ZC_P + k0);
                        const ev8 al = ld8(zc_lo + row * ZC_P + k0);
                        o[m] = mma3<E>(ah, al, b4h[ks], b4l[ks], o[m]);
                    }
                }
                // u row p = 16m + ld + j, column q = 16w + lr
                const int qx = 16 * wave + lr;
                const int gx = x0 + qx;
                if constexpr (FUSED) {
                    if (qx < V) {
#pragma unroll
                        for (int m = 0; m < 3; ++m)
#pragma unroll
                            for (int jj = 0; jj < 4; ++jj) {
                                const int p = 16 * m + ld + jj;
                                if (p < V) ut[p * V + qx] = o[m][jj] * sout;
                            }
                    }
                } else if (qx < V && gx < W) {
                    float* uk = g.U + (size_t)k * HW;
#pragma unroll
                    for (int m = 0; m < 3; ++m)
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) {
                            const int p = 16 * m + ld + jj, gy = y0 + p;
                            if (p < V && gy < H) uk[(size_t)gy * W + gx] = o[m][jj] * sout;
                        }
                }
            }
            if constexpr (FUSED) {
                // diffusion, alpha test and growth of kernel k at this
                // thread's cells, from u_k and the staged genes; the new gene
                // values go out now (0 where alpha has failed)
                if (pos + 1 < T::NK) dma_barrier_keep<3 * NGI>();
                else dma_barrier();
                const int dk = T::dst[k];
                const float eps = wd.eps, cs = wd.cnt_scale, ncs = wd.cnt_bias;
                const plane_t o0 = plane(wd.P_out + (size_t)k * HW, pb);
                const plane_t o1 = plane(wd.P_out + (size_t)(T::NK + k) * HW, pb);
                const plane_t o2 = plane(wd.P_out + (size_t)(2 * T::NK + k) * HW, pb);
                // strip coordinates are formed here from an opaque thread
                // index (kept across the loop they would take registers the
                // transforms need)
                int tid = threadIdx.x;
                asm volatile("" : "+v"(tid));
                const int sgr = tid / V, sq = tid - sgr * V;
                const int p0 = min(SH * sgr, V - SH);
                const int cb = (p0 + 1) * HS + sq + 1;     // staged centre of the strip's first cell
                const float* ub = ut + p0 * V + sq;
                const uint32_t ob0 = 4u * ((uint32_t)(y0 + p0) * (uint32_t)W + (uint32_t)(x0 + sq));
                // the current kernel's genes are in buffer pos & 1.  Down the
                // strip, a cell's upper and centre disk values (and their
                // counts) are the previous cell's centre and lower ones; the
                // sums are formed in the per-cell order, so the result is
                // diffuse_disk's, bitwise.
                auto cells = [&](const float* gb) {
                float vu[3], nu[3], vc[3], nc[3];
#pragma unroll
                for (int pl = 0; pl < 3; ++pl) {
                    vu[pl] = gb[pl * GSLOT + cb - HS];
                    vc[pl] = gb[pl * GSLOT + cb];
                    nu[pl] = clip01(fmaf(vu[pl], cs, ncs));
                    nc[pl] = clip01(fmaf(vc[pl], cs, ncs));
                }
#pragma unroll
                for (int r = 0; r < SH; ++r) {
                    // branch-free: every slot runs the same instructions, and
                    // the selects keep what alpha allows; a slot that is not
                    // the thread's (dead_at < 0) stores past the plane, where
                    // the buffer store is dropped
                    const int c = cb + r * HS;
                    const bool live = dead_at[r] == kAlive;
                    const float u = ub[r * V];
                    float pd[3];
#pragma unroll
                    for (int pl = 0; pl < 3; ++pl) {
                        const float* gp = gb + pl * GSLOT;
                        const float vl = gp[c - 1], vr = gp[c + 1], vd = gp[c + HS];
                        const float nl = clip01(fmaf(vl, cs, ncs)), nr = clip01(fmaf(vr, cs, ncs));
                        const float nd = clip01(fmaf(vd, cs, ncs));
                        const float num = (((vu[pl] + vl) + vc[pl]) + vr) + vd;
                        const float n = (((nu[pl] + nl) + nc[pl]) + nr) + nd;
                        const float d = clip01(num * __builtin_amdgcn_rcpf(n));
                        pd[pl] = (n > 0.f) ? d : 0.f;
                        vu[pl] = vc[pl];
                        nu[pl] = nc[pl];
                        vc[pl] = vd;
                        nc[pl] = nd;
                    }
                    const bool ok = live && (u > eps) && (pd[0] > eps) && (pd[1] > eps) && (pd[2] > eps);
                    float cur = gsum[r][0];
#pragma unroll
                    for (int c3 = 1; c3 < T::C; ++c3) cur = (c3 == dk) ? gsum[r][c3] : cur;
                    const float gacc = growth_acc(cur, u, pd[0], pd[1], pd[2]);
#pragma unroll
                    for (int c3 = 0; c3 < T::C; ++c3)
                        gsum[r][c3] = (ok && c3 == dk) ? gacc : gsum[r][c3];
                    dead_at[r] = (live && !ok) ? pos : dead_at[r];
                    const uint32_t ob = (dead_at[r] >= 0) ? ob0 + (uint32_t)r * 4u * (uint32_t)W : 0xFFFFFFF0u;
                    pst_stream(o0, ob, ok ? pd[0] : 0.f);
                    pst_stream(o1, ob, ok ? pd[1] : 0.f);
                    pst_stream(o2, ob, ok ? pd[2] : 0.f);
                    // one cell at a time: hoisting every cell's LDS reads
                    // ahead would take more registers than the wave has
                    __builtin_amdgcn_sched_barrier(0);
                }
                };
                if (pos & 1) cells(gstB);
                else cells(gstA);
                lds_barrier();    // u_k and the staged genes are free again
            }
        }
    }
    if constexpr (FUSED) {
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        // cells whose alpha failed after the first kernel: the gene planes of
        // the kernels before that one hold diffused values, cleared here
        const int sgr = tid / V, sq = tid - sgr * V;
        const int p0 = min(SH * sgr, V - SH);
        const uint32_t ob0 = 4u * ((uint32_t)(y0 + p0) * (uint32_t)W + (uint32_t)(x0 + sq));
        int need = 0;
#pragma unroll
        for (int r = 0; r < SH; ++r) need |= (dead_at[r] > 0 && dead_at[r] < kAlive) ? 1 : 0;
        if (__any(need)) {
#pragma unroll 1
            for (int pos = 0; pos + 1 < T::NK; ++pos) {
                const int kk = T::kidx[pos / T::KPS][pos % T::KPS];
                const plane_t z0 = plane(wd.P_out + (size_t)kk * HW, pb);
                const plane_t z1 = plane(wd.P_out + (size_t)(T::NK + kk) * HW, pb);
                const plane_t z2 = plane(wd.P_out + (size_t)(2 * T::NK + kk) * HW, pb);
#pragma unroll
                for (int r = 0; r < SH; ++r) {
                    if (pos < dead_at[r] && dead_at[r] < kAlive) {
                        const uint32_t ob = ob0 + (uint32_t)r * 4u * (uint32_t)W;
                        pst_stream(z0, ob, 0.f);
                        pst_stream(z1, ob, 0.f);
                        pst_stream(z2, ob, 0.f);
                    }
                }
            }
        }
        // A' = clip01(A + dt * sum), the sum counting only where alpha holds
        // (one fused multiply-add, as the per-cell epilogue forms it; this
        // file compiles without contraction)
#pragma unroll
        for (int r = 0; r < SH; ++r) {
            if (dead_at[r] < 0) continue;
            const uint32_t ob = ob0 + (uint32_t)r * 4u * (uint32_t)W;
            const bool alive = dead_at[r] == kAlive;
#pragma unroll
            for (int c = 0; c < T::C; ++c) {
                const float a = pld(plane(wd.A + (size_t)c * HW, pb), ob);
                pst(plane(wd.A_out + (size_t)c * HW, pb), ob, clip01(fmaf(wd.dt, alive ? gsum[r][c] : 0.f, a)));
            }
        }
    }
}

template <class T, int R, class E, bool FUSED>
hipError_t launch_dft(const DftArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL((dft_conv_kernel<T, R, E, FUSED>), dim3(a.n_tiles), dim3(256), 0, s, a);
    return hipGetLastError();
}

typedef hipError_t (*dft_launch_fn)(const DftArgs&, hipStream_t);

template <class E, bool FUSED>
static dft_launch_fn find_dft_e(int table, int R)
{
    if (table == TABLE_3x15 && R == 12) return &launch_dft<Table3x15, 12, E, FUSED>;
    if (table == TABLE_3x15 && R == 13) return &launch_dft<Table3x15, 13, E, FUSED>;
    if (table == TABLE_1x1 && R == 12) return &launch_dft<Table1x1, 12, E, FUSED>;
    if (table == TABLE_1x1 && R == 13) return &launch_dft<Table1x1, 13, E, FUSED>;
    return nullptr;
}

static dft_launch_fn find_dft(int conv, int table, int R, bool fused = false)
{
    if (conv == LENIA_CONV_DFT_SPLIT_BF16)
        return fused ? find_dft_e<__bf16, true>(table, R) : find_dft_e<__bf16, false>(table, R);
    if (conv == LENIA_CONV_DFT_SPLIT_F16)
        return fused ? find_dft_e<_Float16, true>(table, R) : find_dft_e<_Float16, false>(table, R);
    return nullptr;
}

bool conv_is_dft(int conv) { return conv == LENIA_CONV_DFT_SPLIT_BF16 || conv == LENIA_CONV_DFT_SPLIT_F16; }

bool conv_form_supported(int conv, int table, int R) { return find_dft(conv, table, R) != nullptr; }

int dft_valid_side(int R) { return DT - 2 * R; }

// Round-to-nearest-even float -> bf16 bits, on the host.
static uint16_t bf16_bits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

static float bf16_value(uint16_t b)
{
    const uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Host tables of the DFT form: the four transform matrices (FP64, split into
// hi / lo parts in the plan's operand type) and the kernels' real spectra on
// the 64 x 64 torus, columns b = 0..32.
lenia_status build_dft_tables(lenia_plan_t p, WorldPlan& w, hipStream_t s,
                              std::vector<void*>& keep)
{
    const int R = w.R, V = DT - 2 * R;
    const double tw = 2.0 * M_PI / DT;
    auto C = [&](int f, int i) { return std::cos(tw * (double)((f * i) % DT)); };
    auto S = [&](int f, int i) { return std::sin(tw * (double)((f * i) % DT)); };
    std::vector<double> f1t(DT * DT), f2(DT2 * DT2), f3(F3_ROWS * DT2, 0.0), f4t(ZC_ROWS * DT, 0.0);
    for (int c = 0; c < DT; ++c)           // F1^T : row c, column j
        for (int j = 0; j < DT; ++j) {
            const int b = c % NB;
            double v;
            if (c < NB) v = C(b, j);
            else v = (b == 0) ? C(NB, j) : -S(b, j);
            f1t[c * DT + j] = v;
        }
    for (int r = 0; r < DT2; ++r)
        for (int k = 0; k < DT2; ++k) {
            const int rr = r % DT, kk = k % DT;
            double v;
            if (r < DT) v = (k < DT) ? C(rr, kk) : S(rr, kk);
            else v = (k < DT) ? -S(rr, kk) : C(rr, kk);
            f2[r * DT2 + k] = v;
        }
    for (int pp = 0; pp < 2 * V; ++pp)     // rows of [Z_re; Z_im]
        for (int k = 0; k < DT2; ++k) {
            const int p = pp % V, a = k % DT;
            const double c = C(a, R + p), sn = S(a, R + p);
            double v;
            if (pp < V) v = (k < DT) ? c : -sn;
            else v = (k < DT) ? sn : c;
            f3[pp * DT2 + k] = v;
        }
    for (int q = 0; q < V; ++q)            // F4^T : row q, column k (2 cos / -2 sin; 1 and (-1)^(q+R) at b = 0)
        for (int k = 0; k < DT; ++k) {
            const int b = k % NB;
            double v;
            if (k < NB) v = (b == 0) ? 1.0 : 2.0 * C(b, R + q);
            else v = (b == 0) ? C(NB, R + q) : -2.0 * S(b, R + q);
            f4t[q * DT + k] = v;
        }
    // hi = round(x), lo = round(x - hi) in the operand type of the plan's form
    const bool f16 = (p->conv == LENIA_CONV_DFT_SPLIT_F16);
    auto split = [&](const std::vector<double>& mu, int e) {
        std::vector<double> m(mu.size());
        for (size_t i = 0; i < m.size(); ++i) m[i] = std::ldexp(mu[i], e);
        uint16_t* out = new uint16_t[2 * m.size()];
        for (size_t i = 0; i < m.size(); ++i) {
            if (f16) {
                const _Float16 h = (_Float16)(float)m[i];
                const _Float16 l = (_Float16)(float)(m[i] - (double)(float)h);
                std::memcpy(&out[i], &h, 2);
                std::memcpy(&out[m.size() + i], &l, 2);
            } else {
                const uint16_t h = bf16_bits((float)m[i]);
                out[i] = h;
                out[m.size() + i] = bf16_bits((float)(m[i] - (double)bf16_value(h)));
            }
        }
        keep.push_back(out);
        return out;
    };
    // kernel spectra: Khat[k][b][a] = sum_d K~(d) cos(2 pi (a dy + b dx)/64) / 64^2, b <= 32
    constexpr int NBK = NB + 1;
    std::vector<double> kt((size_t)DT * DT);
    float* kh = new float[(size_t)w.NK * NBK * DT];
    keep.push_back(kh);
    for (int k = 0; k < w.NK; ++k) {
        const int B = w.n_shells[k];
        const double* beta = &w.beta[3 * k];
        const double z = raw_kernel_sum(R, B, beta);
        std::fill(kt.begin(), kt.end(), 0.0);
        for (int dy = -R; dy <= R; ++dy)
            for (int dx = -R; dx <= R; ++dx)
                kt[((dy + DT) % DT) * DT + (dx + DT) % DT] += raw_kernel_tap(R, B, beta, dy, dx) / z;
        // separable real DFT: first over dx (b), then dy (a); the kernel is even
        std::vector<double> t1((size_t)DT * NBK, 0.0);
        for (int y = 0; y < DT; ++y)
            for (int b = 0; b < NBK; ++b) {
                double acc = 0.0;
                for (int x = 0; x < DT; ++x) acc += kt[y * DT + x] * C(b, x);
                t1[y * NBK + b] = acc;
            }
        for (int b = 0; b < NBK; ++b)
            for (int a = 0; a < DT; ++a) {
                double acc = 0.0;
                for (int y = 0; y < DT; ++y) acc += t1[y * NBK + b] * C(a, y);
                kh[((size_t)k * NBK + b) * DT + a] = (float)std::ldexp(acc / (DT * DT), kUExp);
            }
    }
    const struct {
        const std::vector<double>* m;
        int e;
        void** dst;
    } mats[4] = {{&f1t, kMatExp, &w.dft_f1t}, {&f2, kMatExp, &w.dft_f2}, {&f3, kMatExp, &w.dft_f3},
                 {&f4t, kF4Exp, &w.dft_f4t}};
    for (const auto& mm : mats) {
        uint16_t* host = split(*mm.m, mm.e);
        const size_t bytes = 2 * mm.m->size() * sizeof(uint16_t);
        void* d = nullptr;
        if (device_alloc(&d, bytes) != hipSuccess)
            return set_error(LENIA_ERR_OUT_OF_MEMORY, "DFT tables");
        p->allocations.push_back(d);
        p->ws_bytes += bytes;
        *mm.dst = d;
        hipError_t e = hipMemcpyAsync(d, host, bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "uploading DFT tables");
    }
    const size_t kbytes = (size_t)w.NK * NBK * DT * sizeof(float);
    void* d = nullptr;
    if (device_alloc(&d, kbytes) != hipSuccess) return set_error(LENIA_ERR_OUT_OF_MEMORY, "spectra");
    p->allocations.push_back(d);
    p->ws_bytes += kbytes;
    w.dft_khat = (float*)d;
    hipError_t e = hipMemcpyAsync(d, kh, kbytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "uploading spectra");
    const size_t ubytes = (size_t)w.NK * w.cells() * sizeof(float);
    if (device_alloc(&d, ubytes) != hipSuccess) return set_error(LENIA_ERR_OUT_OF_MEMORY, "potentials");
    p->allocations.push_back(d);
    p->ws_bytes += ubytes;
    w.dft_u = (float*)d;
    return LENIA_OK;
}

hipError_t launch_dft_potentials(const lenia_plan_t p, const WorldPlan& w, const float* A,
                                 float* U, hipStream_t s)
{
    DftArgs a{};
    a.A = A;
    a.U = U;
    a.t.f1t = w.dft_f1t;
    a.t.f2 = w.dft_f2;
    a.t.f3 = w.dft_f3;
    a.t.f4t = w.dft_f4t;
    a.t.khat = w.dft_khat;
    a.H = w.H;
    a.W = w.W;
    const int V = DT - 2 * w.R;
    a.tiles_x = (w.W + V - 1) / V;
    a.n_tiles = a.tiles_x * ((w.H + V - 1) / V);
    dft_launch_fn fn = find_dft(p->conv, p->table, p->R);
    if (!fn) return hipErrorInvalidValue;
    return fn(a, s);
}

hipError_t launch_dft_step(const lenia_plan_t p, const WorldPlan& w, const WorldArgs& wa, hipStream_t s)
{
    DftArgs a{};
    a.A = wa.A;
    a.U = nullptr;
    a.t.f1t = w.dft_f1t;
    a.t.f2 = w.dft_f2;
    a.t.f3 = w.dft_f3;
    a.t.f4t = w.dft_f4t;
    a.t.khat = w.dft_khat;
    a.H = w.H;
    a.W = w.W;
    const int V = DT - 2 * w.R;
    a.tiles_x = (w.W + V - 1) / V;
    a.n_tiles = a.tiles_x * ((w.H + V - 1) / V);
    a.wd = wa;
    dft_launch_fn fn = find_dft(p->conv, p->table, p->R, true);
    if (!fn) return hipErrorInvalidValue;
    return fn(a, s);
}

}  // namespace lenia
