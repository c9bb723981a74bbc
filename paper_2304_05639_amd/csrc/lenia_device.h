// Device helpers shared by the forward and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lenia {

// Kernel weights and other launch-uniform tables are read through the
// constant address space, so the loads become scalar loads whose results feed
// VALU instructions as SGPR operands.
typedef const __attribute__((address_space(4))) float cfloat;

// Block id -> tile id.  The dispatcher deals workgroups round-robin over the
// 8 XCDs (block b runs on XCD b & 7), each XCD with its own L2.  Tiles are
// grouped into runs of kTileRun consecutive tiles and run r goes to XCD r & 7:
// the tiles of a run share an L2, so their overlapping halos are re-read from
// it, and every XCD gets runs from all over the tile list, so regions of
// uneven cost (active creatures, empty space) are spread evenly.  Tiles past
// the last whole group of 8 runs map to themselves.
constexpr int kTileRun = 512;

__device__ __forceinline__ int xcd_tile(int bid, int nb)
{
    const int full = (nb / (8 * kTileRun)) * (8 * kTileRun);
    if (bid >= full) return bid;
    const int xcd = bid & 7, k = bid >> 3;
    const int run = (k / kTileRun) * 8 + xcd;
    return run * kTileRun + (k % kTileRun);
}

__device__ __forceinline__ float clip01(float x) { return fminf(fmaxf(x, 0.f), 1.f); }

// Raw buffer access to one plane: a descriptor (base address, size in bytes)
// held in scalar registers plus a 32-bit byte offset per lane, from which the
// memory unit forms the address.  An access past the plane's end reads 0 and a
// store there is dropped.  A plane is below 4 GiB.
typedef __amdgpu_buffer_rsrc_t plane_t;

__device__ __forceinline__ plane_t plane(const float* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)bytes,
                                            0x00020000);
}
__device__ __forceinline__ float pld(plane_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ void pst(plane_t r, uint32_t off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}

// A store with the non-temporal cache policy (bit 1 of the buffer
// instruction's cache policy on gfx950).  The new gene planes are written
// once and not read again by the kernel that writes them; as ordinary stores
// their 180 bytes per cell fill the L2 and push out the state rows that
// neighbouring tiles' halos re-read.  Measured on the dense 4096^2 step:
// 2.36 -> 2.13 ms, HBM bytes 517 -> 476 per cell (non-temporal loads of the
// genes as well made it 3.46 ms: the diffusion disks lose their L1 reuse).
__device__ __forceinline__ void pst_stream(plane_t r, uint32_t off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 2);
}

// Gaussian factor e = exp(-(u-m)^2 / (2 s^2)) of the growth mapping, with the
// hardware reciprocal and exponential (a few ulp; the exponent's error only
// matters where e is far below the state tolerance).
__device__ __forceinline__ float growth_bell(float d, float s)
{
    const float inv = __builtin_amdgcn_rcpf(2.f * s * s);
    return __expf(-(d * d) * inv);
}

// G(u; m, s, h) = h (2 exp(-(u-m)^2 / (2 s^2)) - 1)
__device__ __forceinline__ float growth(float u, float m, float s, float h)
{
    return h * fmaf(2.f, growth_bell(u - m, s), -1.f);
}

// acc + G(u; m, s, h), the last multiply and the add fused.  Every kernel that
// sums growth for the state update goes through this one expression, so the
// forms that must agree bitwise (the per-cell epilogue, the fused DFT step, the
// adjoint's recomputed update) round alike whatever the compiler's contraction
// setting in their file.
__device__ __forceinline__ float growth_acc(float acc, float u, float m, float s, float h)
{
    return fmaf(h, fmaf(2.f, growth_bell(u - m, s), -1.f), acc);
}

// LDS row pitch of a staged single-channel tile: tile width + halo, rounded up
// to a multiple of 64 floats so that every row offset is a ds_read2st64 offset.
template <int R, int TX>
constexpr int tile_pitch() { return ((TX + 2 * R + 63) / 64) * 64; }

// Wrapped global coordinates of a halo position.
__device__ __forceinline__ void wrap2(int& gy, int& gx, int H, int W, bool single_wrap)
{
    if (single_wrap) {
        gy += (gy < 0) ? H : 0;
        gy -= (gy >= H) ? H : 0;
        gx += (gx < 0) ? W : 0;
        gx -= (gx >= W) ? W : 0;
    } else {
        gy = ((gy % H) + H) % H;
        gx = ((gx % W) + W) % W;
    }
}

// Stages NPL planes (plane p at src[p], row-major H x W) of the tile whose
// top-left output cell is (y0, x0), plus a HALO-cell halo wrapped on the
// torus, into LDS: the values of position (yy, xx) of the padded tile go to
// L::store(dst, yy * (TX + 2 HALO) + xx, v).  NT threads, with all of a
// thread's loads in flight before the LDS writes.
// The first NM planes are masked: a position whose mask byte is 0 stages 0.
// Returns whether any of the thread's positions had a nonzero mask byte.
template <class L, int NPL, int HALO, int TY, int TX, int NT, int NM = 0>
__device__ __forceinline__ bool stage_planes(float* dst, const float* const (&src)[NPL], int H,
                                             int W, int y0, int x0,
                                             const uint8_t* mask = nullptr)
{
    bool any_kept = false;
    constexpr int PY = TY + 2 * HALO, PX = TX + 2 * HALO;
    constexpr int NG = PY * PX;
    constexpr int IT = (NG + NT - 1) / NT;
    const bool single_wrap = (H >= TY + HALO + 1) && (W >= TX + HALO + 1);
    plane_t pl[NPL];
#pragma unroll
    for (int p = 0; p < NPL; ++p) pl[p] = plane(src[p], 4u * (uint32_t)H * (uint32_t)W);
    float v[IT][NPL];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = threadIdx.x + it * NT;
        if (i < NG) {
            const int yy = i / PX;
            const int xx = i - yy * PX;
            int gy = y0 + yy - HALO, gx = x0 + xx - HALO;
            wrap2(gy, gx, H, W, single_wrap);
            const uint32_t o = (uint32_t)gy * (uint32_t)W + (uint32_t)gx;
            const bool keep = (NM == 0) || (mask[o] != 0);
            any_kept = any_kept || keep;
#pragma unroll
            for (int p = 0; p < NPL; ++p) v[it][p] = (p < NM && !keep) ? 0.f : pld(pl[p], 4u * o);
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = threadIdx.x + it * NT;
        if (i < NG) {
            L::store(dst, i, v[it]);
        }
    }
    return any_kept;
}

}  // namespace lenia

namespace lenia {

// Gene diffusion of one plane at one cell over the r = 1 disk (Section 2.3):
// num = sum of the 5 values, n = count of values above eps,
// v = clip01(num / n) (0 where n = 0).  Summation order up, left, centre,
// right, down.
struct Diffused {
    float v, num;
    int n;
};

// The same from the 5 values v = (up, left, centre, right, down).
__device__ __forceinline__ Diffused diffuse_vals(const float (&v)[5], float eps)
{
    Diffused r;
    r.num = (((v[0] + v[1]) + v[2]) + v[3]) + v[4];
    r.n = (v[0] > eps) + (v[1] > eps) + (v[2] > eps) + (v[3] > eps) + (v[4] > eps);
    r.v = (r.n > 0) ? clip01(r.num * __builtin_amdgcn_rcpf((float)r.n)) : 0.f;
    return r;
}

__device__ __forceinline__ Diffused diffuse5(const float* pl, uint32_t ou, uint32_t ol,
                                             uint32_t oc, uint32_t orr, uint32_t od, float eps)
{
    const float v[5] = {pl[ou], pl[ol], pl[oc], pl[orr], pl[od]};
    return diffuse_vals(v, eps);
}

// Diffusion of one plane with byte offsets of the 5 disk cells (as diffuse5,
// same summation order and result).  The count of values above eps is taken
// as sum_i clamp(cs * v_i + ncs) with cs = 2^100 and ncs = -cs * eps, one FMA
// per value: the product is exact and the FMA rounds once, so the term has
// the sign of v_i - eps; for eps >= 2^-64, v_i > eps means v_i - eps >=
// ulp(eps) >= 2^-87 and the clamped term is exactly 1, while v_i <= eps gives 0.
struct NbrB {
    uint32_t c, u, d, l, r;
};

// The 5 disk values of one plane, in the order up, left, centre, right, down.
__device__ __forceinline__ void load_disk(float (&v)[5], plane_t pl, const NbrB& o)
{
    v[0] = pld(pl, o.u);
    v[1] = pld(pl, o.l);
    v[2] = pld(pl, o.c);
    v[3] = pld(pl, o.r);
    v[4] = pld(pl, o.d);
}

__device__ __forceinline__ float diffuse_disk(const float (&v)[5], float cs, float ncs)
{
    const float num = (((v[0] + v[1]) + v[2]) + v[3]) + v[4];
    const float n = clip01(fmaf(v[0], cs, ncs)) + clip01(fmaf(v[1], cs, ncs)) +
                    clip01(fmaf(v[2], cs, ncs)) + clip01(fmaf(v[3], cs, ncs)) +
                    clip01(fmaf(v[4], cs, ncs));
    // evaluated unconditionally (n = 0 gives inf or NaN, which the select drops)
    const float d = clip01(num * __builtin_amdgcn_rcpf(n));
    return (n > 0.f) ? d : 0.f;
}

__device__ __forceinline__ float diffuse5b(plane_t pl, const NbrB& o, float cs, float ncs)
{
    float v[5];
    load_disk(v, pl, o);
    return diffuse_disk(v, cs, ncs);
}

__device__ __forceinline__ NbrB neighbour_bytes(int gy, int gx, int H, int W)
{
    const int ym = (gy == 0) ? H - 1 : gy - 1;
    const int yp = (gy == H - 1) ? 0 : gy + 1;
    const int xm = (gx == 0) ? W - 1 : gx - 1;
    const int xp = (gx == W - 1) ? 0 : gx + 1;
    const uint32_t row = (uint32_t)gy * (uint32_t)W;
    NbrB n;
    n.c = 4u * (row + gx);
    n.u = 4u * ((uint32_t)ym * (uint32_t)W + gx);
    n.d = 4u * ((uint32_t)yp * (uint32_t)W + gx);
    n.l = 4u * (row + xm);
    n.r = 4u * (row + xp);
    return n;
}

// 32-bit in-plane offsets of a cell and its 4 torus neighbours.
struct Nbr {
    uint32_t oc, ou, od, ol, orr;
};

__device__ __forceinline__ Nbr neighbours(int gy, int gx, int H, int W)
{
    const int ym = (gy == 0) ? H - 1 : gy - 1;
    const int yp = (gy == H - 1) ? 0 : gy + 1;
    const int xm = (gx == 0) ? W - 1 : gx - 1;
    const int xp = (gx == W - 1) ? 0 : gx + 1;
    Nbr n;
    n.oc = (uint32_t)gy * W + gx;
    n.ou = (uint32_t)ym * W + gx;
    n.od = (uint32_t)yp * W + gx;
    n.ol = (uint32_t)gy * W + xm;
    n.orr = (uint32_t)gy * W + xp;
    return n;
}

}  // namespace lenia
