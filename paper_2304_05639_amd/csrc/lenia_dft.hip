// Potentials by tile-local DFT as matrix products on the MFMA units (gfx950).
//
// u_k = K~_k * A_src(k) is a circular convolution; on a 64 x 64 window of A
// (the 40 x 40 output tile plus an R-cell halo, R = 12) it equals the inverse
// DFT of DFT(window) times the kernel's DFT (Section 2.1 computes the
// convolution through the convolution theorem).  The kernel is even, so its
// DFT is real.  With C[f][i] = cos(2 pi f i / 64), S[f][i] = sin(2 pi f i / 64)
// and real-embedded complex matrices, per tile:
//   GEMM1  [Y_re | Y_im]     (64 x 128) = X (64 x 64) [C | -S]            per channel
//   GEMM2  [Xh_re; Xh_im]    (128 x 64) = [[C, S], [-S, C]] [Y_re; Y_im]  per channel
//          U = Xh * Khat_k (real, 1/64^2 folded in)                        per kernel
//   GEMM3  [Z_re; Z_im]^T    (64 x 2V)  = [U_re; U_im]^T [[C_V, -S_V], [S_V, C_V]]^T
//   GEMM4  u_k               (V x V)    = [Z_re | Z_im] [C'_V; -S'_V]
// where C_V / S_V keep the V output rows (columns) of the inverse transform.
// Two kernels k1, k2 reading the same channel share one inverse transform:
// Xh * Khat_k1 and Xh * Khat_k2 are each the spectrum of a real image, so the
// inverse transform of U = Xh * Khat_k1 + i Xh * Khat_k2 is u_k1 + i u_k2;
// GEMM3 runs once for the pair and GEMM4 forms both parts, the imaginary one
// with [S'_V; C'_V].  With five kernels per channel that is two pairs and one
// single kernel per channel.
// Every GEMM runs on v_mfma_f32_16x16x32_bf16 (or _f16) with FP32
// accumulation; each operand x is split as hi = e(x), lo = e(x - hi) in the
// operand type e and a product is hi*hi + hi*lo + lo*hi: about 16 significant
// bits with bf16 and 22 with fp16.  fp16 keeps those 22 bits only while lo
// stays a normal number, |x| >= 2^-3, so every operand is scaled by a power
// of two that puts its largest possible magnitude just below 2^14 (far from
// fp16's largest value, 65504): the DFT matrices (|x| <= 1) by 2^14 on the
// host, the window by 2^a from its largest magnitude, and each intermediate
// by the bound its GEMM implies (a K-term sum of products below 2^28).  An
// element then loses precision only below 2^-17 of that bound, where its
// absolute error (half of fp16's subnormal step) is 2^-39 of it.  The scales
// are exact, so they cancel in the result and leave the bf16 form's rounding
// unchanged.  The DFT matrices are built in FP64 on the host and split there;
// data operands are split here.
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

// Power-of-two scales of the operands (see the header): the DFT matrices
// carry 2^14; GEMM1's output (64 terms below 2^28) is split at 2^-20, the
// spectral product (the transformed channel, 128 terms below 2^28, times a
// spectrum of magnitude <= 2^-12) at 2^-9, folded into the spectra, and
// GEMM3's output (128 terms) at 2^-21.  With the window scaled by 2^a the
// potentials come out scaled by 2^(a + 6).
constexpr int kMatExp = 14;
constexpr int kYExp = -20;
constexpr int kUExp = -9;
constexpr int kZExp = -21;
constexpr int kOutExp = 6;

constexpr int DT = 64;                   // DFT tile
constexpr int DT2 = 128;                 // real-embedded complex dimension
constexpr int XS_P = DT + 8;             // LDS row pitches (bf16 / fp32 elements)
constexpr int YT_P = DT2 + 8;
constexpr int XH_P = DT2 + 4;
constexpr int ZC_P = DT2 + 8;
constexpr int ZC_ROWS = 48;
constexpr int UST_P = DT2 + 8;

struct DftTables {
    const void* f1t;      // [2][128][64]  hi, lo of [C | -S]^T
    const void* f2;       // [2][128][128] hi, lo of [[C, S], [-S, C]]
    const void* f3;       // [2][80][128]  hi, lo of [[C_V, -S_V], [S_V, C_V]] (rows >= 2V zero)
    const void* f4t;      // [2][48][128]  hi, lo of [C'_V; -S'_V]^T (rows >= V zero)
    const void* f4ti;     // [2][48][128]  hi, lo of [S'_V; C'_V]^T (imaginary part)
    const float* khat;    // [NK][64 f2][64 f1] real kernel spectra / 64^2, times 2^kUExp
};

struct DftArgs {
    const float* A;       // [C][H][W]
    float* U;             // [NK][H][W] potentials (output)
    DftTables t;
    int H, W, tiles_x, n_tiles;
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

template <class T, int R, class E>
__global__ __launch_bounds__(256) void dft_conv_kernel(DftArgs g)
{
    typedef typename Op<E>::v8 ev8;
    const E* f1t = (const E*)g.t.f1t;
    const E* f2m = (const E*)g.t.f2;
    const E* f3m = (const E*)g.t.f3;
    const E* f4t = (const E*)g.t.f4t;
    const E* f4ti = (const E*)g.t.f4ti;
    constexpr int V = DT - 2 * R;
    // LDS: the transformed channel being processed (fp32) + a scratch region
    // shared by the forward stages (Xs, Yt) and the inverse stages (Zc, and the
    // spectral product Ust of the current kernel, split once per workgroup)
    constexpr int XH_FLOATS = DT * XH_P;
    constexpr int FWD_E = 2 * DT * XS_P + 2 * DT * YT_P;
    constexpr int INV_E = 2 * ZC_ROWS * ZC_P + 2 * DT * UST_P;
    constexpr int SCRATCH_E = (FWD_E > INV_E) ? FWD_E : INV_E;
    __shared__ float xh[XH_FLOATS];
    __shared__ __attribute__((aligned(16))) E scr[SCRATCH_E];
    __shared__ float wmax[4];
    E* xs_hi = scr;
    E* xs_lo = scr + DT * XS_P;
    E* yt_hi = scr + 2 * DT * XS_P;
    E* yt_lo = yt_hi + DT * YT_P;
    E* zc_hi = scr;
    E* zc_lo = scr + ZC_ROWS * ZC_P;
    E* ust_hi = scr + 2 * ZC_ROWS * ZC_P;
    E* ust_lo = ust_hi + DT * UST_P;

    const int H = g.H, W = g.W;
    const size_t HW = (size_t)H * W;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tyi = tile / g.tiles_x, txi = tile - tyi * g.tiles_x;
    const int y0 = tyi * V, x0 = txi * V;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = (lane >> 4) * 8, ld = (lane >> 4) * 4;
    const bool single_wrap = (H >= DT) && (W >= DT);

    // ---- per kernel: spectral product and inverse transform -----------------
    // GEMM3 has 4 row blocks x 5 column blocks (2V rows of Z, padded to 80):
    // wave w computes column block w for every row block, and row block w of
    // column block 4, five tiles each; the B fragments of its two column
    // blocks stay in registers.
    constexpr int NB3 = (2 * V + 15) / 16;
    static_assert(NB3 == 5, "GEMM3 is laid out for 5 column blocks");
    ev8 b3h[2][4], b3l[2][4];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int nt = (q == 0) ? wave : 4;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int row = 16 * nt + lr, k0 = 32 * ks + lk;
            b3h[q][ks] = ld8(f3m + row * DT2 + k0);
            b3l[q][ks] = ld8(f3m + 80 * DT2 + row * DT2 + k0);
        }
    }
    // GEMM4: wave w < 3 handles output column block w; B fragments in registers
    ev8 b4h[4], b4l[4], b4ih[4], b4il[4];
    {
        const int row = 16 * (wave < 3 ? wave : 0) + lr;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            b4h[ks] = ld8(f4t + row * DT2 + 32 * ks + lk);
            b4l[ks] = ld8(f4t + ZC_ROWS * DT2 + row * DT2 + 32 * ks + lk);
            b4ih[ks] = ld8(f4ti + row * DT2 + 32 * ks + lk);
            b4il[ks] = ld8(f4ti + ZC_ROWS * DT2 + row * DT2 + 32 * ks + lk);
        }
    }

    // ---- per source channel: forward transform, then its kernels ------------
    for (int s = 0; s < T::C; ++s) {
        __syncthreads();
        // load the 64 x 64 window (wrapped) and its largest magnitude, then
        // stage it scaled by 2^a (largest magnitude below 2^14) as hi / lo
        constexpr int NWIN = DT * DT / 4 / 256;
        f32x4 win[NWIN];
        float vmax = 0.f;
#pragma unroll
        for (int it = 0; it < NWIN; ++it) {
            const int i = threadIdx.x + 256 * it;
            const int r = i / (DT / 4), c4 = (i % (DT / 4)) * 4;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int gy = y0 - R + r, gx = x0 - R + c4 + j;
                wrap2(gy, gx, H, W, single_wrap);
                win[it][j] = g.A[(size_t)s * HW + (size_t)gy * W + gx];
                vmax = fmaxf(vmax, fabsf(win[it][j]));
            }
        }
        vmax = wave_max(vmax);
        if (lane == 0) wmax[wave] = vmax;
        __syncthreads();
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
        __syncthreads();
        // GEMM1: wave w computes rows 16w..16w+15 of Y, all 8 column blocks
        {
            f32x4 acc[8];
#pragma unroll
            for (int n = 0; n < 8; ++n) acc[n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const int k0 = 32 * ks + lk;
                const ev8 ah = ld8(xs_hi + (16 * wave + lr) * XS_P + k0);
                const ev8 al = ld8(xs_lo + (16 * wave + lr) * XS_P + k0);
#pragma unroll
                for (int n = 0; n < 8; ++n) {
                    const int row = 16 * n + lr;
                    const ev8 bh = ld8(f1t + row * DT + k0);
                    const ev8 bl = ld8(f1t + DT2 * DT + row * DT + k0);
                    acc[n] = mma3<E>(ah, al, bh, bl, acc[n]);
                }
            }
            // Y column c = 16n + lr, rows i = 16w + ld + j  ->  Yt[c % 64][64 (c / 64) + i]
#pragma unroll
            for (int n = 0; n < 8; ++n) {
                const int c = 16 * n + lr;
                const int off = (c % DT) * YT_P + DT * (c / DT) + 16 * wave + ld;
                st4_split<E>(yt_hi + off, yt_lo + off, acc[n] * ldexpf(1.f, kYExp));
            }
        }
        __syncthreads();
        // GEMM2: wave w computes row blocks 2w, 2w+1 of Xh, all 4 column blocks
        {
            f32x4 acc[2][4];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int k0 = 32 * ks + lk;
                ev8 ah[2], al[2];
#pragma unroll
                for (int m = 0; m < 2; ++m) {
                    const int row = 16 * (2 * wave + m) + lr;
                    ah[m] = ld8(f2m + row * DT2 + k0);
                    al[m] = ld8(f2m + DT2 * DT2 + row * DT2 + k0);
                }
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    const ev8 bh = ld8(yt_hi + (16 * n + lr) * YT_P + k0);
                    const ev8 bl = ld8(yt_lo + (16 * n + lr) * YT_P + k0);
#pragma unroll
                    for (int m = 0; m < 2; ++m) acc[m][n] = mma3<E>(ah[m], al[m], bh, bl, acc[m][n]);
                }
            }
            // Xh row r = 16 (2w + m) + ld + j, column f2 = 16n + lr  ->  xh[s][f2][r]
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n) {
                    const int f2 = 16 * n + lr, r = 16 * (2 * wave + m) + ld;
                    *(f32x4*)(xh + f2 * XH_P + r) = acc[m][n];
                }
        }
        __syncthreads();
#pragma unroll 1
        for (int it = 0; it < (T::KPS + 1) / 2; ++it) {
            const int k = T::kidx[s][2 * it];
            const bool pair = (2 * it + 1 < T::KPS);
            const int k2 = pair ? T::kidx[s][2 * it + 1] : k;
            const float* kh = g.t.khat + (size_t)k * DT * DT;
            const float* kh2 = g.t.khat + (size_t)k2 * DT * DT;
            // the spectral product U = Xh * Khat_k (+ i Xh * Khat_k2 for a pair,
            // halved so that it keeps the bound of one product), split into LDS
            // once for all waves: 8 frequencies per thread and item, real part at
            // column c8, imaginary part at column 64 + c8
            const float ph = pair ? 0.5f : 1.f;
            for (int i = threadIdx.x; i < DT * (DT / 8); i += 256) {
                const int f2 = i / (DT / 8), c8 = (i % (DT / 8)) * 8;
                const float* xr = xh + f2 * XH_P + c8;
                const f32x4 r0 = *(const f32x4*)xr, r1 = *(const f32x4*)(xr + 4);
                const f32x4 i0 = *(const f32x4*)(xr + DT), i1 = *(const f32x4*)(xr + DT + 4);
                const f32x4 a0 = *(const f32x4*)(kh + f2 * DT + c8), a1 = *(const f32x4*)(kh + f2 * DT + c8 + 4);
                float ure[8], uim[8];
                if (pair) {
                    const f32x4 b0 = *(const f32x4*)(kh2 + f2 * DT + c8);
                    const f32x4 b1 = *(const f32x4*)(kh2 + f2 * DT + c8 + 4);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        ure[q] = (r0[q] * a0[q] - i0[q] * b0[q]) * ph;
                        ure[4 + q] = (r1[q] * a1[q] - i1[q] * b1[q]) * ph;
                        uim[q] = (i0[q] * a0[q] + r0[q] * b0[q]) * ph;
                        uim[4 + q] = (i1[q] * a1[q] + r1[q] * b1[q]) * ph;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        ure[q] = r0[q] * a0[q];
                        ure[4 + q] = r1[q] * a1[q];
                        uim[q] = i0[q] * a0[q];
                        uim[4 + q] = i1[q] * a1[q];
                    }
                }
                ev8 uh, ul;
                split8<E>(ure, uh, ul);
                *(ev8*)(ust_hi + f2 * UST_P + c8) = uh;
                *(ev8*)(ust_lo + f2 * UST_P + c8) = ul;
                split8<E>(uim, uh, ul);
                *(ev8*)(ust_hi + f2 * UST_P + DT + c8) = uh;
                *(ev8*)(ust_lo + f2 * UST_P + DT + c8) = ul;
            }
            __syncthreads();
            // GEMM3: Z^T (64 x 80) = Ust^T (64 x 128) F3^T; wave handles all 4 row blocks
            f32x4 acc[2][4];
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int m = 0; m < 4; ++m) acc[q][m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int k0 = 32 * ks + lk;          // f1 + 64 (im)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int f2 = 16 * m + lr;
                    const ev8 ah = ld8(ust_hi + f2 * UST_P + k0);
                    const ev8 al = ld8(ust_lo + f2 * UST_P + k0);
                    acc[0][m] = mma3<E>(ah, al, b3h[0][ks], b3l[0][ks], acc[0][m]);
                    if (m == wave) acc[1][0] = mma3<E>(ah, al, b3h[1][ks], b3l[1][ks], acc[1][0]);
                }
            }
            __syncthreads();    // every wave has read Ust; the previous GEMM4 is done with Zc
            // Z^T row f2 = 16m + ld + j, column p' = 16 nt + lr -> Zc[p' mod V][64 (p' >= V) + f2]
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int nt = (q == 0) ? wave : 4;
                const int pp = 16 * nt + lr;
                if (pp < 2 * V) {
                    const int p = (pp < V) ? pp : pp - V, col0 = (pp < V) ? 0 : DT;
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        if (q == 1 && m != 0) break;
                        // column block 4 holds row block `wave` only, in acc[1][0]
                        const int mm = (q == 0) ? m : wave;
                        const int off = p * ZC_P + col0 + 16 * mm + ld;
                        st4_split<E>(zc_hi + off, zc_lo + off, acc[q][m] * ldexpf(1.f, kZExp));
                    }
                }
            }
            __syncthreads();
            // GEMM4: u (48 x 48) = Zc (48 x 128) F4; wave w < 3 computes column block w
            if (wave < 3) {
                f32x4 o[3], o2[3];
#pragma unroll
                for (int m = 0; m < 3; ++m) o[m] = o2[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int k0 = 32 * ks + lk;
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        const int row = 16 * m + lr;
                        const ev8 ah = ld8(zc_hi + row * ZC_P + k0);
                        const ev8 al = ld8(zc_lo + row * ZC_P + k0);
                        o[m] = mma3<E>(ah, al, b4h[ks], b4l[ks], o[m]);
                        if (pair) o2[m] = mma3<E>(ah, al, b4ih[ks], b4il[ks], o2[m]);
                    }
                }
                // u row p = 16m + ld + j, column q = 16w + lr
                const int qx = 16 * wave + lr;
                const int gx = x0 + qx;
                if (qx < V && gx < W) {
                    const float so = pair ? 2.f * sout : sout;
                    float* uk = g.U + (size_t)k * HW;
                    float* uk2 = g.U + (size_t)k2 * HW;
#pragma unroll
                    for (int m = 0; m < 3; ++m)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int p = 16 * m + ld + j, gy = y0 + p;
                            if (p < V && gy < H) {
                                uk[(size_t)gy * W + gx] = o[m][j] * so;
                                if (pair) uk2[(size_t)gy * W + gx] = o2[m][j] * so;
                            }
                        }
                }
            }
        }
    }
}

template <class T, int R, class E>
hipError_t launch_dft(const DftArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL((dft_conv_kernel<T, R, E>), dim3(a.n_tiles), dim3(256), 0, s, a);
    return hipGetLastError();
}

typedef hipError_t (*dft_launch_fn)(const DftArgs&, hipStream_t);

template <class E>
static dft_launch_fn find_dft_e(int table, int R)
{
    if (table == TABLE_3x15 && R == 12) return &launch_dft<Table3x15, 12, E>;
    if (table == TABLE_3x15 && R == 13) return &launch_dft<Table3x15, 13, E>;
    if (table == TABLE_1x1 && R == 12) return &launch_dft<Table1x1, 12, E>;
    if (table == TABLE_1x1 && R == 13) return &launch_dft<Table1x1, 13, E>;
    return nullptr;
}

static dft_launch_fn find_dft(int conv, int table, int R)
{
    if (conv == LENIA_CONV_DFT_SPLIT_BF16) return find_dft_e<__bf16>(table, R);
    if (conv == LENIA_CONV_DFT_SPLIT_F16) return find_dft_e<_Float16>(table, R);
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
// bf16 hi / lo) and the kernels' real spectra on the 64 x 64 torus.
lenia_status build_dft_tables(lenia_plan_t p, WorldPlan& w, hipStream_t s,
                              std::vector<void*>& keep)
{
    const int R = w.R, V = DT - 2 * R;
    const double tw = 2.0 * M_PI / DT;
    auto C = [&](int f, int i) { return std::cos(tw * (double)((f * i) % DT)); };
    auto S = [&](int f, int i) { return std::sin(tw * (double)((f * i) % DT)); };
    std::vector<double> f1t(DT2 * DT), f2(DT2 * DT2), f3(80 * DT2, 0.0), f4t(ZC_ROWS * DT2, 0.0),
        f4ti(ZC_ROWS * DT2, 0.0);
    for (int c = 0; c < DT2; ++c)          // [C | -S]^T : row c, column j
        for (int j = 0; j < DT; ++j) f1t[c * DT + j] = (c < DT) ? C(c, j) : -S(c - DT, j);
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
            const int p = pp % V, f1 = k % DT;
            const double c = C(f1, R + p), sn = S(f1, R + p);
            double v;
            if (pp < V) v = (k < DT) ? c : -sn;
            else v = (k < DT) ? sn : c;
            f3[pp * DT2 + k] = v;
        }
    for (int q = 0; q < V; ++q)            // [C'_V; -S'_V]^T : row q, column k
        for (int k = 0; k < DT2; ++k) {
            const int f2i = k % DT;
            f4t[q * DT2 + k] = (k < DT) ? C(f2i, R + q) : -S(f2i, R + q);
            f4ti[q * DT2 + k] = (k < DT) ? S(f2i, R + q) : C(f2i, R + q);
        }
    // hi = round(x), lo = round(x - hi) in the operand type of the plan's form
    const bool f16 = (p->conv == LENIA_CONV_DFT_SPLIT_F16);
    auto split = [&](const std::vector<double>& mu) {
        std::vector<double> m(mu.size());
        for (size_t i = 0; i < m.size(); ++i) m[i] = std::ldexp(mu[i], kMatExp);
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
    // kernel spectra: Khat[k][f2][f1] = sum_d K~(d) cos(2 pi (f1 dy + f2 dx)/64) / 64^2
    std::vector<double> kt((size_t)DT * DT);
    float* kh = new float[(size_t)w.NK * DT * DT];
    keep.push_back(kh);
    for (int k = 0; k < w.NK; ++k) {
        const int B = w.n_shells[k];
        const double* beta = &w.beta[3 * k];
        const double z = raw_kernel_sum(R, B, beta);
        std::fill(kt.begin(), kt.end(), 0.0);
        for (int dy = -R; dy <= R; ++dy)
            for (int dx = -R; dx <= R; ++dx)
                kt[((dy + DT) % DT) * DT + (dx + DT) % DT] += raw_kernel_tap(R, B, beta, dy, dx) / z;
        // separable real DFT: first over dx (f2), then dy (f1); the kernel is even
        std::vector<double> t1((size_t)DT * DT, 0.0);
        for (int y = 0; y < DT; ++y)
            for (int f = 0; f < DT; ++f) {
                double acc = 0.0;
                for (int x = 0; x < DT; ++x) acc += kt[y * DT + x] * C(f, x);
                t1[y * DT + f] = acc;
            }
        for (int f2i = 0; f2i < DT; ++f2i)
            for (int f1 = 0; f1 < DT; ++f1) {
                double acc = 0.0;
                for (int y = 0; y < DT; ++y) acc += t1[y * DT + f2i] * C(f1, y);
                kh[((size_t)k * DT + f2i) * DT + f1] = (float)std::ldexp(acc / (DT * DT), kUExp);
            }
    }
    const struct {
        const std::vector<double>* m;
        void** dst;
    } mats[5] = {{&f1t, &w.dft_f1t}, {&f2, &w.dft_f2}, {&f3, &w.dft_f3}, {&f4t, &w.dft_f4t},
                 {&f4ti, &w.dft_f4ti}};
    for (const auto& mm : mats) {
        uint16_t* host = split(*mm.m);
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
    const size_t kbytes = (size_t)w.NK * DT * DT * sizeof(float);
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
    a.t.f4ti = w.dft_f4ti;
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

}  // namespace lenia
