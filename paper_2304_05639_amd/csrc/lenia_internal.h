// Internal declarations shared by the host plan code and the HIP kernels of
// liblenia.so.  Not part of the public ABI (include/lenia.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lenia {

// ---------------------------------------------------------------------------
// Kernel-offset orbits.  A ring-shell kernel depends on |d| only, so it is
// invariant under the 8 symmetries of the square lattice.  Offsets with
// 0 < |d| < R fall into orbits represented by (a, b), 0 <= b <= a:
//   b == 0 : (+-a, 0), (0, +-a)          4 offsets
//   b == a : (+-a, +-a)                  4 offsets
//   else   : (+-a, +-b), (+-b, +-a)      8 offsets
// The centre (0, 0) has weight 0 (the shell core vanishes at r = 0) and is
// not an orbit.  The convolution sums the cells of an orbit first and
// multiplies once per kernel.
// ---------------------------------------------------------------------------
template <int R>
struct Orbits {
    static constexpr int count()
    {
        int n = 0;
        for (int a = 0; a < R; ++a)
            for (int b = 0; b <= a; ++b)
                if (a * a + b * b > 0 && a * a + b * b < R * R) ++n;
        return n;
    }
    static constexpr int N = count();
    struct Tab {
        int a[N];
        int b[N];
    };
    static constexpr Tab make()
    {
        Tab t{};
        int n = 0;
        for (int a = 0; a < R; ++a)
            for (int b = 0; b <= a; ++b)
                if (a * a + b * b > 0 && a * a + b * b < R * R) {
                    t.a[n] = a;
                    t.b[n] = b;
                    ++n;
                }
        return t;
    }
    static constexpr Tab tab = make();
};

// ---------------------------------------------------------------------------
// The kernel core per orbit, at compile time.  A kernel with B shells and
// heights beta has the tap value beta_i K_C(rho - i), rho = B |d| / R,
// i = floor(rho) (Section 2.1), K_C(t) = exp(4 - 1 / (t (1 - t))).  So
//   u_k = (1 / z_k) sum_i beta_{k,i} sum_{o in shell i of B_k} K_C(rho_o - i) S(o)
// with S(o) the orbit sum of the source channel: the orbits' weighted sums
// for the six (B, i) pairs of B = 1, 2, 3 serve every kernel, and each kernel
// combines its B_k of them.  An orbit lies in one shell for each B, so it
// costs 3 multiply-adds per source channel instead of one per kernel.  The
// core values depend on R only; they are formed here, in double precision,
// and rounded to float, so that the step kernel carries them as instruction
// constants.  The host plan checks them against its own FP64 kernel.
// Orbits are listed in the step kernel's walk order: axis (a, 0) by a,
// diagonal (a, a) by a, then general (a, b), 0 < b < a, by a then b.
// ---------------------------------------------------------------------------
namespace cx {
constexpr double sqrt_pos(double x)
{
    if (!(x > 0.0)) return 0.0;
    double y = (x > 1.0) ? x : 1.0;   // Newton's iteration from above
    for (int i = 0; i < 200; ++i) {
        const double n = 0.5 * (y + x / y);
        if (!(n < y)) break;
        y = n;
    }
    return y;
}

// e^x for x <= 4: x = k ln 2 + f, |f| <= ln 2 / 2 (ln 2 in two parts, so
// that k ln 2 is exact to about 2^-80), e^f by its Taylor series, times 2^k.
constexpr double exp_le4(double x)
{
    if (x < -800.0) return 0.0;
    const double ln2_hi = 0.693147180369123816490, ln2_lo = 1.90821492927058770002e-10;
    const double kf = x * 1.44269504088896340736;
    const int k = (int)(kf < 0.0 ? kf - 0.5 : kf + 0.5);
    const double f = (x - k * ln2_hi) - k * ln2_lo;
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 30; ++n) {
        term *= f / n;
        sum += term;
    }
    for (int n = 0; n < k; ++n) sum *= 2.0;
    for (int n = 0; n > k; --n) sum *= 0.5;
    return sum;
}

constexpr double shell_core(double t)
{
    return (t > 0.0 && t < 1.0) ? exp_le4(4.0 - 1.0 / (t * (1.0 - t))) : 0.0;
}
}  // namespace cx

// index of the (B, shell i) pair among the six: B = 1: 0; B = 2: 1, 2; B = 3: 3..5
constexpr int shell_pair(int B, int i) { return B * (B - 1) / 2 + i; }

template <int R>
struct ShellBasis {
    static constexpr int NO = Orbits<R>::N;
    struct Tab {
        int a[NO], b[NO];
        int pair[NO][3];      // shell_pair(B, shell of the orbit) for B = 1, 2, 3
        float core[NO][3];    // K_C at the orbit for B = 1, 2, 3 (0 on a shell boundary)
    };
    static constexpr void put(Tab& t, int& n, int a, int b)
    {
        t.a[n] = a;
        t.b[n] = b;
        const int d2 = a * a + b * b;
        for (int B = 1; B <= 3; ++B) {
            // shell i: i^2 R^2 <= B^2 d2 < (i + 1)^2 R^2, in integers
            int i = 0;
            while ((i + 1) * (i + 1) * R * R <= B * B * d2) ++i;
            const double rho = B * cx::sqrt_pos((double)d2) / R;
            t.pair[n][B - 1] = shell_pair(B, i);
            t.core[n][B - 1] = (float)cx::shell_core(rho - i);
        }
        ++n;
    }
    static constexpr Tab make()
    {
        Tab t{};
        int n = 0;
        for (int a = 1; a < R; ++a) put(t, n, a, 0);
        for (int a = 1; 2 * a * a < R * R; ++a) put(t, n, a, a);
        for (int a = 2; a < R; ++a)
            for (int b = 1; b < a; ++b)
                if (a * a + b * b < R * R) put(t, n, a, b);
        return t;
    }
    static constexpr Tab tab = make();
};

inline int orbit_count(int R)
{
    int n = 0;
    for (int a = 0; a < R; ++a)
        for (int b = 0; b <= a; ++b)
            if (a * a + b * b > 0 && a * a + b * b < R * R) ++n;
    return n;
}

// ---------------------------------------------------------------------------
// Kernel tables compiled into the kernels: for each source channel the kernels
// reading it ("slots"), and each kernel's target channel.
// ---------------------------------------------------------------------------
struct Table1x1 {
    static constexpr int C = 1, NK = 1, KPS = 1, KPD = 1;
    static constexpr int kidx[1][1] = {{0}};
    static constexpr int kdst[1][1] = {{0}};     // kernels by target channel
    static constexpr int src[1] = {0};
    static constexpr int dst[1] = {0};
};

// 3 channels, 15 kernels: k = 0..8 self (channel k/3), k = 9..14 cross
// (0->1, 0->2, 1->0, 1->2, 2->0, 2->1).
struct Table3x15 {
    static constexpr int C = 3, NK = 15, KPS = 5, KPD = 5;
    static constexpr int kidx[3][5] = {{0, 1, 2, 9, 10}, {3, 4, 5, 11, 12}, {6, 7, 8, 13, 14}};
    // kernels by target channel, in the order the step sums their growth
    // (by source channel, each channel's kernels as in kidx)
    static constexpr int kdst[3][5] = {{0, 1, 2, 11, 13}, {9, 3, 4, 5, 14}, {10, 12, 6, 7, 8}};
    static constexpr int src[15] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 0, 0, 1, 1, 2, 2};
    static constexpr int dst[15] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 1, 2, 0, 2, 0, 1};
};

enum TableId { TABLE_1x1 = 0, TABLE_3x15 = 1 };

enum Mode { MODE_GLOBAL = 0, MODE_LOCAL_READONLY = 1, MODE_LOCAL_UPDATE = 2,
            MODE_POTENTIALS = 3 /* write u_k to U_save only */ };

constexpr int kMaxK = 16;

// One world as seen by the step kernels.
struct WorldArgs {
    const float* A;        // [C][H][W]
    const float* P;        // [3][NK][H][W] or null
    float* A_out;
    float* P_out;          // null when genes are read-only
    float* U_save;         // [NK][H][W] or null
    uint8_t* alpha_save;   // [H][W] or null
    uint8_t* flags_out;    // [H][W] or null: bit 0 alpha, bit 1 sum_k u_k > eps (the
                           // organic-matter mask of the penalization); disables the
                           // tile shortcuts, which never form the potentials
    uint8_t* p_zero;       // [n_tiles] or null: 1 where P_out is known to hold 0 on the
                           // tile in every gene plane (set by a tile that writes its
                           // genes as 0, cleared by one that writes them otherwise)
    const float* w;        // [NK][n_orbits] orbit weights of K~_k (FP32)
    const float* wt;       // [n_orbits][wt_stride] the same weights by orbit, packed as
                           // source * KPS + slot (one scalar load per orbit); the
                           // single-kernel table's step reads these
    const float* shc;      // [C][KPS][8] shell coefficients beta_{k,i} / z_k of slot
                           // (source, j) at shell_pair(B_k, i), 0 elsewhere; the
                           // 15-kernel table's step combines the shell sums with these
    int H, W;
    int tiles_x, n_tiles;  // tile grid of this world
    float dt;
    float eps;             // the largest float <= the descriptor's eps, so that
                           // (float x > eps) == ((double)x > eps_double)
    float cnt_scale;       // 2^100: threshold count by FMA + clamp (needs eps >= 2^-64)
    float cnt_bias;        // -cnt_scale * eps (exact)
    float skip_thr;        // eps * (1 - 2^-10), rounded down: a tile whose window of one
                           // source channel stays <= skip_thr has alpha = 0 everywhere
    float org_thr;         // skip_thr / NK, rounded down: a tile whose window stays
                           // <= org_thr in every channel has sum_k u_k < eps everywhere
    float gm[kMaxK], gs[kMaxK], gh[kMaxK];   // global genes (MODE_GLOBAL)
};

// Work list of a batched step: item i is tile items[i].y of world items[i].x.
struct BatchList {
    const WorldArgs* worlds;
    const int2* items;
    int n_items;
};

// Launchers (defined in lenia_step.hip).  Return hipSuccess or the launch error.
typedef hipError_t (*step_launch_fn)(const WorldArgs& w, int mode, hipStream_t s);
// one workgroup per work item (grid = b.n_items)
typedef hipError_t (*batch_launch_fn)(const BatchList& b, int mode, hipStream_t s);

step_launch_fn find_step_launcher(int table, int R, int ty, int tx);
// the ring-decomposed kernel form (genes P[9][NK][H][W]); null if not compiled
step_launch_fn find_ring_step_launcher(int table, int R, int ty, int tx);
batch_launch_fn find_batch_launcher(int table, int R, int ty, int tx);
// candidate tiles compiled for (table, R); returns count, fills up to max pairs
int step_tile_candidates(int table, int R, int* ty, int* tx, int max);
hipError_t launch_fill_synthetic(float* A, size_t nA, float* P, size_t plane, int nk,
                                 hipStream_t s);
// hipMalloc through the library's allocation-failure test hook; *ptr is null
// on failure
hipError_t device_alloc(void** ptr, size_t bytes);
// *flag |= bit if x[0, n) holds a NaN or an infinity
hipError_t launch_find_nonfinite(const float* x, size_t n, uint32_t* flag, uint32_t bit,
                                 hipStream_t s);
// p[0, n) = 0 (a kernel, so that the call can sit in a captured graph)
hipError_t launch_clear_bytes(uint8_t* p, uint32_t n, hipStream_t s);

}  // namespace lenia
