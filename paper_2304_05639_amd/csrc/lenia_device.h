// Device helpers shared by the forward and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lenia {

// Kernel weights and other launch-uniform tables are read through the
// constant address space, so the loads become scalar loads whose results feed
// VALU instructions as SGPR operands.
typedef const __attribute__((address_space(4))) float cfloat;

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

__device__ __forceinline__ float clip01(float x) { return fminf(fmaxf(x, 0.f), 1.f); }

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
    return h * (2.f * growth_bell(u - m, s) - 1.f);
}

// LDS row pitch of a staged tile: tile width + halo, rounded up to a multiple
// of 64 floats so that every plane / row offset is a ds_read2st64 offset.
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
// top-left output cell is (y0, x0), plus an R-cell halo wrapped on the torus,
// into dst[p * CHS + yy * PITCH + xx], using NT threads with all of a thread's
// loads in flight before the LDS writes.
// The first NM planes are masked: a position whose mask byte is 0 stages 0.
template <int NPL, int R, int TY, int TX, int NT, int PITCH, int CHS, int NM = 0>
__device__ __forceinline__ void stage_planes(float* dst, const float* const (&src)[NPL], int H,
                                             int W, int y0, int x0,
                                             const uint8_t* mask = nullptr)
{
    constexpr int PY = TY + 2 * R, PX = TX + 2 * R;
    constexpr int NG = PY * PX;
    constexpr int IT = (NG + NT - 1) / NT;
    const bool single_wrap = (H >= TY + R) && (W >= TX + R);
    float v[IT][NPL];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = threadIdx.x + it * NT;
        if (i < NG) {
            const int yy = i / PX;
            const int xx = i - yy * PX;
            int gy = y0 + yy - R, gx = x0 + xx - R;
            wrap2(gy, gx, H, W, single_wrap);
            const uint32_t o = (uint32_t)gy * (uint32_t)W + (uint32_t)gx;
            const bool keep = (NM == 0) || (mask[o] != 0);
#pragma unroll
            for (int p = 0; p < NPL; ++p) v[it][p] = (p < NM && !keep) ? 0.f : src[p][o];
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = threadIdx.x + it * NT;
        if (i < NG) {
            const int yy = i / PX;
            const int xx = i - yy * PX;
#pragma unroll
            for (int p = 0; p < NPL; ++p) dst[p * CHS + yy * PITCH + xx] = v[it][p];
        }
    }
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

__device__ __forceinline__ Diffused diffuse5(const float* pl, uint32_t ou, uint32_t ol,
                                             uint32_t oc, uint32_t orr, uint32_t od, float eps)
{
    const float vu = pl[ou], vl = pl[ol], vc = pl[oc], vr = pl[orr], vd = pl[od];
    Diffused r;
    r.num = (((vu + vl) + vc) + vr) + vd;
    r.n = (vu > eps) + (vl > eps) + (vc > eps) + (vr > eps) + (vd > eps);
    r.v = (r.n > 0) ? clip01(r.num * __builtin_amdgcn_rcpf((float)r.n)) : 0.f;
    return r;
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
