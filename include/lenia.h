/*
 * lenia.h - C ABI of the MI355X (gfx950) multi-channel Lenia library.
 *
 * One step of 2-D, multi-channel Lenia on a torus with per-cell ("localized")
 * growth genes, following Chan, "Towards Large-Scale Simulations of
 * Open-Ended Evolution in Continuous Cellular Automata" (GECCO 2023):
 *   Section 2.1  3 channels, 15 kernels (3 self-kernels per channel, 2 cross-
 *                kernels per channel pair), normalized kernels K~ = K/sum(K),
 *                clipped update A <- clip01(A + sum_k G_k(K~_k * A)).
 *   Section 2.2  genes in a tensor P[p][k][y][x]; alpha mask = all potentials
 *                above the cutoff eps AND all genes above eps; P <- P * alpha.
 *   Section 2.3  gene diffusion: P <- clip01((P * Kdiff) / (count of
 *                above-eps neighbours within Kdiff)), Kdiff a disk.
 *   Section 2.4  growth of kernel k at a cell uses that cell's m, s, h genes.
 *   Algorithm 2  order per step: diffuse -> convolve -> alpha -> mask -> grow.
 * Readings taken where the paper is silent (see the design notes):
 *   kernel of kernel k: K(d) = beta_{k,i} * exp(4 - 1/(r(1-r))) for |d| < R,
 *     i = floor(B_k |d|/R), r = B_k |d|/R - i (ring shells, B_k in 1..3);
 *   growth G(u; m,s,h) = h * (2 exp(-(u-m)^2/(2 s^2)) - 1);
 *   update A' = clip01(A + dt * sum_{k: dst(k)=c} g_k), summed in ascending k;
 *   the alpha mask thresholds the potentials u_k = K~_k * A (strict > eps);
 *   the diffusion disk is |d| <= r_diff; a cell with no above-eps neighbour
 *   gets gene 0; only m, s, h are localized (kernel heights are global).
 *
 * Layouts (all row-major FP32, device memory, 4-byte aligned):
 *   A  float[C][H][W]             cell states
 *   P  float[3][NK][H][W]         gene planes m (k = 0..NK-1), then s, then h
 *      float[9][NK][H][W]         with n_ring > 0: r1, w1, b1, r2, w2, b2, m, s, h
 *                                 (the two kernel-function bumps, then growth)
 * Ownership: the caller owns every state, gene, gradient and `saved` buffer;
 * a plan owns its workspaces and tables and frees them in lenia_plan_destroy.
 * Streams: every call only enqueues work on `stream` (a hipStream_t, NULL =
 * the null stream) and returns without synchronizing; device faults surface at
 * the caller's next synchronization.  A plan must not be used from two host
 * threads at once; distinct plans are independent.
 * Errors: arguments are validated before anything is enqueued; on error no
 * work is enqueued and caller buffers are untouched.  No C++ exception crosses
 * this ABI; lenia_last_error() gives a thread-local detail string.
 */
#ifndef LENIA_H
#define LENIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LENIA_API __attribute__((visibility("default")))

typedef enum {
    LENIA_OK = 0,
    LENIA_ERR_INVALID_ARG = 1,   /* malformed descriptor or call arguments   */
    LENIA_ERR_UNSUPPORTED = 2,   /* valid, but outside what the kernels build */
    LENIA_ERR_OUT_OF_MEMORY = 3, /* device allocation failed                  */
    LENIA_ERR_HIP = 4,           /* a HIP runtime call or launch failed       */
    LENIA_ERR_STATE = 5,         /* call not valid for this plan              */
    LENIA_ERR_NONFINITE = 6      /* LENIA_FLAG_CHECK_FINITE found a NaN or an
                                    infinity in an input buffer              */
} lenia_status;

/* How the potentials u_k = K~_k * A are computed.  Every form computes the
 * same circular convolution; they differ in arithmetic and speed. */
typedef enum {
    LENIA_CONV_AUTO = 0,             /* library choice (currently DIRECT_F32)       */
    LENIA_CONV_DIRECT_F32 = 1,       /* direct torus sum in FP32, taps folded by the
                                        kernel's 8-fold lattice symmetry              */
    LENIA_CONV_DFT_SPLIT_BF16 = 2,   /* tile-local DFT as matrix products on MFMA,
                                        bf16 hi+lo operands, FP32 accumulation       */
    LENIA_CONV_DFT_SPLIT_F16 = 3     /* as above with fp16 hi+lo operands            */
} lenia_conv;

#define LENIA_MAX_CHANNELS 3
#define LENIA_MAX_KERNELS 15
#define LENIA_MAX_SHELLS 3

/* Descriptor of one world.  All pointers are host pointers read only during
 * lenia_plan / lenia_plan_batched / lenia_desc_validate. */
typedef struct {
    int32_t H, W;               /* torus rows, columns: each in [1, 65536] and   */
                                /* H * W < 2^30 (a plane below 4 GiB)            */
    int32_t n_channels;         /* C: 1 or 3                                     */
    int32_t n_kernels;          /* NK: 1 (with C = 1) or 15 (with C = 3)         */
    const int32_t* src;         /* [NK] source channel of each kernel            */
    const int32_t* dst;         /* [NK] target channel of each kernel            */
    int32_t R;                  /* kernel radius in cells (12 or 13)             */
    const int32_t* n_shells;    /* [NK] B_k in 1..3                              */
    const double* beta;         /* [NK][3] shell heights; the first B_k are used */
    double dt;                  /* time step, > 0                                */
    int32_t localized;          /* 0: global genes m,s,h below; 1: genes in P    */
    int32_t genotype_update;    /* 1: diffuse + alpha-mask P each step (needs
                                   localized); 0: genes are read-only            */
    const double* m;            /* [NK] global genes, used iff localized == 0    */
    const double* s;            /*      (s > 0)                                  */
    const double* h;
    double eps;                 /* mask cutoff (0.01), in [0, 1); >= 2^-64 when  */
                                /* genotype_update is set                        */
    int32_t r_diff;             /* diffusion disk radius (1)                     */
    int32_t conv;               /* lenia_conv                                    */
    int32_t tile_y, tile_x;     /* output tile of the fused step kernel; 0,0 =
                                   the autotuned / default choice                */
    uint32_t flags;             /* LENIA_FLAG_*                                  */
    int32_t n_ring;             /* 0: the ring-shell kernels above (beta, shells);
                                   > 0: ring-decomposed kernels with localized
                                   kernel genes (Section 2.4): the disk |d| < R
                                   split into n_ring rings, ring j = the offsets
                                   with floor(n_ring |d| / R) = j, weighted per
                                   cell by the two bumps b exp(-(j/n_ring -
                                   r)^2 / (2 w^2)) of each kernel's genes; then
                                   u_k = sum_j kw_j (ring-j sum of A_src) /
                                   sum_j kw_j (ring-j size), 0 if that is 0.
                                   Needs localized and genotype_update; P has 9
                                   gene types (below); n_shells / beta unused
                                   (may be NULL).  Compiled: 3 channels / 15
                                   kernels, R = 12, n_ring = 24, lenia_step
                                   only (no saved buffer, batched plan,
                                   potentials, adjoint, autotune, DFT form).  */
} lenia_desc;

#define LENIA_FLAG_AUTOTUNE 1u  /* time the tile candidates at plan time and
                                   cache the winner per (H, W, R, C, mode)       */
#define LENIA_FLAG_CHECK_FINITE 2u
                                /* debug checks on every call of the plan, before
                                   anything else is enqueued: each caller buffer
                                   must lie inside the device allocation that
                                   holds it (host-side, from the allocation's
                                   address range: LENIA_ERR_INVALID_ARG), and
                                   every value of the input buffers (state,
                                   genes, cotangents) must be finite (a device
                                   scan, after which the call waits for its
                                   stream: LENIA_ERR_NONFINITE).  The steps
                                   assume finite inputs and do not check them
                                   otherwise (a NaN fails every comparison and
                                   the clips pass it on).                        */
#define LENIA_FLAG_DFT_FUSED 4u
                                /* DFT forms: run every step that can be fused
                                   (localized genes updated each step, no saved
                                   buffer) as one kernel, whatever the world's
                                   size.  By default a plan fuses only when the
                                   world has at least 4 DFT tiles per compute
                                   unit: below that the one-kernel step's few
                                   workgroups run the 15 kernels' transforms one
                                   after another, and the two-kernel step (the
                                   potentials, then a per-cell epilogue spread
                                   over the whole GPU) is faster (at 256^2, 57
                                   against 104 us per step).  Both give
                                   identical results.  Ignored by the direct and
                                   ring forms.                                   */

typedef struct lenia_plan_* lenia_plan_t;

/* Information about a plan (what the library chose). */
typedef struct {
    int32_t conv;               /* lenia_conv actually used                      */
    int32_t tile_y, tile_x;     /* tile of the fused step kernel                 */
    int32_t n_worlds;           /* 1, or the batch size of a batched plan        */
    int64_t cells;              /* sum of H*W over worlds                        */
    size_t workspace_bytes;     /* device memory owned by the plan               */
    size_t saved_bytes;         /* lenia_saved_bytes()                           */
} lenia_plan_info;

/* Checks a descriptor on the host only (no device call): LENIA_OK,
 * LENIA_ERR_INVALID_ARG (malformed) or LENIA_ERR_UNSUPPORTED. */
LENIA_API lenia_status lenia_desc_validate(const lenia_desc* d);

/* The normalized kernel K~_k (Section 2.1) that a plan for `d` uses, in FP64
 * on the (2R+1)x(2R+1) offset grid, index [(dy+R)*(2R+1) + (dx+R)], computed
 * on the host before rounding to FP32.  `out` holds (2R+1)^2 doubles. */
LENIA_API lenia_status lenia_kernel_taps(const lenia_desc* d, int32_t k, double* out);

/* Builds a plan for one world: kernel tables (FP64 on the host, rounded to
 * FP32), device workspaces, tile choice.  Uploads on `stream`. */
LENIA_API lenia_status lenia_plan(const lenia_desc* d, void* stream, lenia_plan_t* out);

/* Builds a plan for n_worlds independent worlds (sizes may differ; each has
 * its own kernels and genes), stepped together by lenia_step_batched. */
LENIA_API lenia_status lenia_plan_batched(const lenia_desc* descs, int32_t n_worlds, void* stream,
                                lenia_plan_t* out);

/*
 * Advances one world by n_steps >= 0 steps (Algorithm 2 without its random
 * operators): from (A_in, P_in) to (A_out, P_out).  A_out may equal A_in and
 * P_out may equal P_in (in place); otherwise the buffers must not overlap.
 * P_in / P_out are ignored (may be NULL) when localized == 0; P_out is not
 * written when genotype_update == 0 (genes read-only).
 * saved: NULL, or (only with n_steps == 1) a device buffer of
 * lenia_saved_bytes() bytes that receives the step's potentials u_k
 * (float[NK][H][W]) followed by the alpha mask (uint8[H][W]), for
 * lenia_backward.
 * A call of more than two steps that updates genes keeps one byte per tile
 * and output buffer (2 bytes per tile, allocated on first use, cleared at the
 * start of the call): a tile whose genes are provably 0 does not rewrite gene
 * planes that this call already wrote as 0 there.  The results are the same
 * as with every plane written.
 */
LENIA_API lenia_status lenia_step(lenia_plan_t p, const float* A_in, const float* P_in,
                        float* A_out, float* P_out, int32_t n_steps, void* saved,
                        void* stream);

/* Advances every world of a batched plan by n_steps, in place: A[i], P[i] are
 * device pointers of world i (host arrays of n_worlds pointers).  The steps
 * run as one launch per step over a (world, tile) work list,
 * captured once into a HIP graph per pointer set and replayed.  The
 * zero-gene tile bytes of lenia_step (2 per tile of every world, allocated
 * on the first call) are cleared by a kernel before the replays. */
LENIA_API lenia_status lenia_step_batched(lenia_plan_t p, float* const* A, float* const* P,
                                int32_t n_steps, void* stream);

/* The potentials u_k = K~_k * A_src(k) (Section 2.1's normalized kernels;
 * the "potential" of Section 2.2) of the state A of a single-world plan, with
 * the plan's convolution form, into U float[NK][H][W] (device, not aliasing
 * A).  No gene or state update. */
LENIA_API lenia_status lenia_potentials(lenia_plan_t p, const float* A, float* U, void* stream);

/* Bytes of the `saved` buffer of lenia_step / lenia_backward. */
LENIA_API size_t lenia_saved_bytes(lenia_plan_t p);

/*
 * Vector-Jacobian product of one step (A_t, P_t) -> (A_{t+1}, P_{t+1}) of a
 * single-world plan with localized == 1.  `saved` is what lenia_step(...,
 * n_steps = 1, saved) wrote for this (A_t, P_t).  Given gA_next, gP_next
 * (cotangents of A_{t+1}, P_{t+1}; gP_next may be NULL = zero), writes
 *   gA_t  float[C][H][W]        (overwritten)
 *   gP_t  float[3][NK][H][W]    (overwritten)
 * and ADDS the shell-height gradient into gbeta float[NK][3] (entries
 * >= B_k untouched).  The alpha mask and diffusion counts are piecewise
 * constant and carry no gradient; clips use the inclusive subgradient.
 * gA_t / gP_t must not alias any input.
 */
LENIA_API lenia_status lenia_backward(lenia_plan_t p, const float* A_t, const float* P_t,
                            const void* saved, const float* gA_next, const float* gP_next,
                            float* gA_t, float* gP_t, float* gbeta, void* stream);

/*
 * lenia_backward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and arguments, with their workspaces (the potential and
 * diffusion cotangents and the per-tile shell-height partials, about
 * 240 B per cell with 15 kernels) in one static device array of
 * LENIA_NOALLOC_WORKSPACE_BYTES per GPU instead of plan-owned memory.  The
 * array is created with the library's code object on each GPU it runs on and
 * lives until the process ends; its address is looked up on the first call
 * on a device.  Worlds that need more than the array holds (above about
 * 2.7e5 cells with 15 kernels) get LENIA_ERR_UNSUPPORTED, and a plan whose
 * device is not current gets LENIA_ERR_STATE.  Results are bitwise those of
 * lenia_backward.  All calls on one GPU share the array: calls that overlap
 * in time on one GPU (two streams, two threads) race and must be serialized
 * by the caller.  The call itself allocates nothing.
 */
#define LENIA_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
LENIA_API lenia_status lenia_backward_noalloc(lenia_plan_t p, const float* A_t, const float* P_t,
                                              const void* saved, const float* gA_next,
                                              const float* gP_next, float* gA_t, float* gP_t,
                                              float* gbeta, void* stream);

/*
 * The environmental and random operators of Algorithm 2 around each step of
 * a single-world plan with localized, updated genes (shell form):
 *   1. walls (Section 2.7): A and P are set to 0 on the wall cells of the
 *      state the step starts from;
 *   2. the step of lenia_step;
 *   3. the penalizing area (Section 2.6): organic matter = the cells where
 *      sum_k u_k > eps; E_oxy = the cells with a non-organic cell within the
 *      disk |d| <= r_oxy; E_pen = the cells with a cell outside E_oxy within
 *      that disk (both convolutions read as "any cell of the disk");
 *   4. mutation (Section 2.5): gene plane (mut_p, mut_k) += gamma_mut *
 *      mut_delta on the square of side 2 mut_half, rows mut_y0 - mut_half ..
 *      mut_y0 + mut_half - 1 and columns likewise (wrapped), where alpha = 1;
 *   5. penalization (Section 2.6): gene plane (pen_p, pen_k) += gamma_pen *
 *      pen_delta where E_pen and alpha hold.
 * No clip follows 4 and 5 (the next step's diffusion clips).  The random
 * draws of each iteration are the caller's: one lenia_event per step.
 */
typedef struct {
    const uint8_t* walls;       /* device uint8[H][W], nonzero = wall; or NULL   */
    double gamma_mut;           /* mutation rate (the paper runs 1 and 5); 0 = off */
    int32_t mut_half;           /* half side s of the mutated square; 2s <= H, W */
    double gamma_pen;           /* penalization rate (the paper runs 0.2); 0 = off */
    int32_t r_oxy;              /* oxygen disk radius, 0..16                      */
} lenia_evolution;

typedef struct {
    int32_t mut_p, mut_k;       /* mutated gene type (0 m, 1 s, 2 h) and kernel  */
    float mut_delta;            /* the mutation's delta                           */
    int32_t mut_y0, mut_x0;     /* centre of the square (|.| <= 2^30, wrapped)    */
    int32_t pen_p, pen_k;       /* penalized gene type (0 m or 1 s) and kernel    */
    float pen_delta;            /* the penalty's delta (its sign is the caller's) */
} lenia_event;

/*
 * n_steps iterations of the above.  Buffers as for lenia_step (in place or
 * out of place), except that the wall cells of (A_in, P_in) are zeroed in
 * place first.  events: host array of n_steps entries (may be NULL when both
 * rates are 0).  Workspace of 3 bytes per cell allocated on first use, and the
 * tile bytes of lenia_step for calls of more than two steps.
 * Ring-decomposed kernels and batched plans: LENIA_ERR_UNSUPPORTED.
 */
LENIA_API lenia_status lenia_step_evolve(lenia_plan_t p, float* A_in, float* P_in, float* A_out,
                                         float* P_out, int32_t n_steps, const lenia_evolution* evo,
                                         const lenia_event* events, void* stream);

/*
 * Test hook for the failure paths of device allocation (not for production
 * use): from now on, in this process, let `after` device allocations of the
 * library through and make the `count` after them fail as if the device were
 * out of memory (the call then returns LENIA_ERR_OUT_OF_MEMORY and leaves its
 * plan as it was).  count <= 0 turns the hook off.
 */
LENIA_API void lenia_debug_fail_alloc(int32_t after, int32_t count);

LENIA_API lenia_status lenia_plan_get_info(lenia_plan_t p, lenia_plan_info* info);
LENIA_API lenia_status lenia_plan_destroy(lenia_plan_t p);
LENIA_API const char* lenia_status_str(lenia_status s);
LENIA_API const char* lenia_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LENIA_H */
