/*
 * Plain FP64 CPU oracle for one step of multi-channel Lenia with localized
 * growth genes, and for that step's vector-Jacobian product.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the HIP library and is written from the paper's definitions, not for speed:
 * the convolution is the direct spatial sum over kernel taps on the torus
 * (the paper's FFT route reaches the same result up to rounding).
 *
 * Definitions followed (Chan 2023, "Towards Large-Scale Simulations of
 * Open-Ended Evolution in Continuous Cellular Automata"):
 *   - Section 2.1 / Algorithm 1: normalized kernels K~ = K / sum(K), update
 *     A <- clip01(A + sum_k G_k(K~_k * A)), clip [x]_a^b = max(min(x,b),a);
 *   - Section 2.2: Delta masks with cutoff eps, alpha = Delta_all(U) and
 *     Delta_all(P), P <- P (.) alpha;
 *   - Section 2.3: P <- clip01((P * K_diff) / (Delta_same(P) * K_diff)) with a
 *     disk K_diff of radius r_diff;
 *   - Section 2.4: growth read from the local genes (m, s, h) of kernel k;
 *   - Algorithm 2: order diffuse -> convolve -> alpha -> mask -> grow/update.
 * Readings where the paper is silent or its printed form is contradicted by its
 * own behaviour (all listed with reasons in the design notes):
 *   - kernel shell: K(D) = beta_i * exp(4 - 1/(r(1-r))), D = |d|/R < 1,
 *     i = floor(B*D), r = B*D - i (classic Lenia ring shell, cited by the paper);
 *   - growth G(u; m,s,h) = h * (2 exp(-(u-m)^2 / (2 s^2)) - 1);
 *   - update with a time step: A' = clip01(A + dt * sum_k g_k), ascending k;
 *   - U in the alpha mask is the normalized potential u_k = K~_k * A;
 *   - diffusion disk |d| <= r_diff inclusive; output 0 where the count is 0;
 *   - thresholds are strict (> eps); only the m, s, h genes are localized.
 * The ring-decomposed kernels of Section 2.4, whose kernel genes are localized
 * too, are a second step function, oracle_ring_step; the walls, mutation and
 * penalization operators of Sections 2.5-2.7 around a step are
 * oracle_evolve_step (both at the end of the file).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_EXPORT __attribute__((visibility("default")))

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the OpenMP loops (for timing the oracle on one core or all). */
ORACLE_EXPORT void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static double core_fn(double r)
{
    if (r <= 0.0 || r >= 1.0) return 0.0;
    return exp(4.0 - 1.0 / (r * (1.0 - r)));
}

/* Shell index and shell-local radius of offset (dy,dx); returns -1 outside the
 * open disk |d| < R. */
static int shell_of(int R, int B, int dy, int dx, double* r_local)
{
    long d2 = (long)dy * dy + (long)dx * dx;
    if (d2 >= (long)R * R) return -1;
    double BD = (double)B * sqrt((double)d2) / (double)R;
    int i = (int)floor(BD);
    if (i >= B) return -1;
    *r_local = BD - (double)i;
    return i;
}

/* Unnormalized shell basis S_i(d) (the core evaluated in shell i, 0 elsewhere). */
ORACLE_EXPORT double oracle_shell_basis(int R, int B, int i, int dy, int dx)
{
    double r = 0.0;
    int s = shell_of(R, B, dy, dx, &r);
    return (s == i) ? core_fn(r) : 0.0;
}

/* Normalized kernel K~ on the (2R+1)x(2R+1) offset grid, index
 * [(dy+R)*(2R+1) + (dx+R)].  Returns the normalizer Z = sum of the raw kernel
 * (0 if the kernel is identically zero, in which case K is left zero). */
ORACLE_EXPORT double oracle_kernel(int R, int B, const double* beta, double* K)
{
    int S = 2 * R + 1;
    double Z = 0.0;
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
            double v = 0.0;
            for (int i = 0; i < B; ++i) v += beta[i] * oracle_shell_basis(R, B, i, dy, dx);
            K[(dy + R) * S + (dx + R)] = v;
            Z += v;
        }
    if (Z == 0.0) return 0.0;
    for (int t = 0; t < S * S; ++t) K[t] /= Z;
    return Z;
}

static inline long wrap(long i, long n)
{
    long r = i % n;
    return r < 0 ? r + n : r;
}

/* Section 2.3: P_d = clip01((P * K_diff) / (Delta_same(P) * K_diff)) for NP
 * planes, K_diff the disk |d| <= r_diff, 0 where no disk value exceeds eps.
 * num, cnt receive the numerator and the count (may be NULL). */
static void diffuse_planes(int H, int W, int NP, int rd, double eps, const double* P,
                           double* num_out, double* cnt_out, double* Pd)
{
    const long N = (long)H * W;
    #pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (int pk = 0; pk < NP; ++pk)
            for (long x = 0; x < W; ++x) {
                double num = 0.0, n = 0.0;
                for (int dy = -rd; dy <= rd; ++dy)
                    for (int dx = -rd; dx <= rd; ++dx) {
                        if (dy * dy + dx * dx > rd * rd) continue;
                        double v = P[(long)pk * N + wrap(y + dy, H) * W + wrap(x + dx, W)];
                        num += v;
                        if (v > eps) n += 1.0;
                    }
                long o = (long)pk * N + y * W + x;
                if (num_out) num_out[o] = num;
                if (cnt_out) cnt_out[o] = n;
                double q = (n > 0.0) ? num / n : 0.0;
                Pd[o] = (n > 0.0) ? fmax(fmin(q, 1.0), 0.0) : 0.0;
            }
}

/* Forward internals of one step at every cell, shared by step and VJP. */
typedef struct {
    int H, W, C, NK, R, localized, genotype_update, r_diff;
    const int *src, *dst;
    const double* K;        /* NK * (2R+1)^2 */
    double dt, eps, tau;
    const double *gm, *gs, *gh;
    const double *A, *P;
    /* outputs of the forward pass */
    double* num;            /* 3*NK*H*W (diffusion numerator)   */
    double* cnt;            /* 3*NK*H*W (diffusion count n)      */
    double* Pd;             /* 3*NK*H*W diffused genes (or P)    */
    double* U;              /* NK*H*W potentials                 */
    uint8_t* alpha;         /* H*W                               */
    double* Z;              /* C*H*W pre-clip update             */
} fwd_t;

static void forward_internals(fwd_t* f)
{
    const long N = (long)f->H * f->W;
    const int S = 2 * f->R + 1;
    const int NP = 3 * f->NK;

    /* Section 2.3: diffusion of every gene plane (only when genes are updated). */
    if (f->localized) {
        if (f->genotype_update) {
            diffuse_planes(f->H, f->W, NP, f->r_diff, f->eps, f->P, f->num, f->cnt, f->Pd);
        } else {
            memcpy(f->Pd, f->P, sizeof(double) * NP * N);
        }
    }

    /* Potentials u_k(x) = sum_d K~_k(d) A_src(x + d), direct torus sum. */
    #pragma omp parallel for schedule(static)
    for (long y = 0; y < f->H; ++y)
        for (int k = 0; k < f->NK; ++k) {
            const double* Ks = f->K + (long)k * S * S;
            const double* As = f->A + (long)f->src[k] * N;
            for (long x = 0; x < f->W; ++x) {
                double u = 0.0;
                for (int dy = -f->R; dy <= f->R; ++dy) {
                    const double* row = As + wrap(y + dy, f->H) * f->W;
                    const double* krow = Ks + (long)(dy + f->R) * S + f->R;
                    for (int dx = -f->R; dx <= f->R; ++dx) {
                        double kv = krow[dx];
                        if (kv != 0.0) u += kv * row[wrap(x + dx, f->W)];
                    }
                }
                f->U[(long)k * N + y * f->W + x] = u;
            }
        }

    /* Section 2.2 alpha mask and Algorithm 2 growth / update. */
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
        int a = 1;
        if (f->localized && f->genotype_update) {
            for (int k = 0; k < f->NK; ++k) if (!(f->U[(long)k * N + c] > f->eps)) a = 0;
            for (int pk = 0; pk < NP; ++pk) if (!(f->Pd[(long)pk * N + c] > f->eps)) a = 0;
        }
        f->alpha[c] = (uint8_t)a;
        for (int ch = 0; ch < f->C; ++ch) {
            double sum = 0.0;
            for (int k = 0; k < f->NK; ++k) {
                if (f->dst[k] != ch) continue;
                double g = 0.0;
                if (a) {
                    double m, s, h;
                    if (f->localized) {
                        m = f->Pd[(long)(0 * f->NK + k) * N + c];
                        s = f->Pd[(long)(1 * f->NK + k) * N + c];
                        h = f->Pd[(long)(2 * f->NK + k) * N + c];
                    } else {
                        m = f->gm[k]; s = f->gs[k]; h = f->gh[k];
                    }
                    double d = f->U[(long)k * N + c] - m;
                    g = h * (2.0 * exp(-d * d / (2.0 * s * s)) - 1.0);
                }
                sum += g;
            }
            f->Z[(long)ch * N + c] = f->A[(long)ch * N + c] + f->dt * sum;
        }
    }
}

static int alloc_fwd(fwd_t* f)
{
    const long N = (long)f->H * f->W;
    const long NPN = 3L * f->NK * N;
    f->num = f->cnt = f->Pd = NULL;
    if (f->localized) {
        f->num = (double*)calloc(NPN, sizeof(double));
        f->cnt = (double*)calloc(NPN, sizeof(double));
        f->Pd = (double*)calloc(NPN, sizeof(double));
    }
    f->U = (double*)calloc((long)f->NK * N, sizeof(double));
    f->alpha = (uint8_t*)calloc(N, 1);
    f->Z = (double*)calloc((long)f->C * N, sizeof(double));
    if (!f->U || !f->alpha || !f->Z || (f->localized && (!f->num || !f->cnt || !f->Pd))) return -1;
    return 0;
}

static void free_fwd(fwd_t* f)
{
    free(f->num); free(f->cnt); free(f->Pd); free(f->U); free(f->alpha); free(f->Z);
}

/* Ambiguity bits per cell: bit 0 = a thresholded quantity (u_k or diffused
 * gene) lies within tau of eps, so either branch of alpha is correct; bit 1 =
 * a clipped quantity (pre-clip update z, diffusion quotient q) lies within tau
 * of a clip bound, so either side of the subgradient is correct. */
static void ambiguity(const fwd_t* f, uint8_t* amb)
{
    const long N = (long)f->H * f->W;
    const int NP = 3 * f->NK;
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
        uint8_t b = 0;
        if (f->localized && f->genotype_update) {
            for (int k = 0; k < f->NK; ++k)
                if (fabs(f->U[(long)k * N + c] - f->eps) <= f->tau) b |= 1;
            for (int pk = 0; pk < NP; ++pk)
                if (fabs(f->Pd[(long)pk * N + c] - f->eps) <= f->tau) b |= 1;
            for (int pk = 0; pk < NP; ++pk) {
                double n = f->cnt[(long)pk * N + c];
                if (n > 0.0) {
                    double q = f->num[(long)pk * N + c] / n;
                    if (fabs(q) <= f->tau || fabs(q - 1.0) <= f->tau) b |= 2;
                }
            }
        }
        for (int ch = 0; ch < f->C; ++ch) {
            double z = f->Z[(long)ch * N + c];
            if (fabs(z) <= f->tau || fabs(z - 1.0) <= f->tau) b |= 2;
        }
        amb[c] = b;
    }
}

/*
 * One step.  Arrays are row-major: A[C][H][W], P[3][NK][H][W] (planes m, s, h,
 * each ordered by kernel), K[NK][(2R+1)^2] normalized kernels.
 * Outputs: A_out, P_out (P_out ignored when not localized); optional U_out
 * [NK][H][W], alpha_out [H][W], amb_out [H][W] (may be NULL).
 * Returns 0 on success, -1 on allocation failure.
 */
ORACLE_EXPORT int oracle_step(int H, int W, int C, int NK, const int* src, const int* dst,
                              int R, const double* K, double dt, int localized,
                              const double* gm, const double* gs, const double* gh,
                              int genotype_update, double eps, int r_diff, double tau,
                              const double* A, const double* P,
                              double* A_out, double* P_out, double* U_out,
                              uint8_t* alpha_out, uint8_t* amb_out)
{
    fwd_t f = {H, W, C, NK, R, localized, localized ? genotype_update : 0, r_diff,
               src, dst, K, dt, eps, tau, gm, gs, gh, A, P};
    if (alloc_fwd(&f)) { free_fwd(&f); return -1; }
    forward_internals(&f);
    const long N = (long)H * W;
    for (long i = 0; i < (long)C * N; ++i) A_out[i] = fmax(fmin(f.Z[i], 1.0), 0.0);
    if (localized && P_out) {
        for (long pk = 0; pk < 3L * NK; ++pk)
            for (long c = 0; c < N; ++c)
                P_out[pk * N + c] = f.genotype_update ? (f.alpha[c] ? f.Pd[pk * N + c] : 0.0)
                                                      : P[pk * N + c];
    }
    if (U_out) memcpy(U_out, f.U, sizeof(double) * NK * N);
    if (alpha_out) memcpy(alpha_out, f.alpha, N);
    if (amb_out) ambiguity(&f, amb_out);
    free_fwd(&f);
    return 0;
}

/*
 * Vector-Jacobian product of one step.  Given the cotangents gA_next [C][H][W]
 * and gP_next [3][NK][H][W] of (A', P'), returns
 *   gA [C][H][W]      d<gA',A'> + <gP',P'> / dA
 *   gP [3][NK][H][W]  ... / dP                       (localized only)
 *   gK [NK][(2R+1)^2] ... / dK~ (normalized kernel taps)
 *   gm, gs, gh [NK]   ... / d(global genes)           (global mode only)
 * Piecewise-constant parts (alpha, the diffusion count n) carry no gradient;
 * clips use the inclusive subgradient [lo <= x <= hi].
 */
ORACLE_EXPORT int oracle_step_vjp(int H, int W, int C, int NK, const int* src, const int* dst,
                                  int R, const double* K, double dt, int localized,
                                  const double* gm_in, const double* gs_in, const double* gh_in,
                                  int genotype_update, double eps, int r_diff, double tau,
                                  const double* A, const double* P,
                                  const double* gA_next, const double* gP_next,
                                  double* gA, double* gP, double* gK,
                                  double* gm, double* gs, double* gh, uint8_t* amb_out)
{
    fwd_t f = {H, W, C, NK, R, localized, localized ? genotype_update : 0, r_diff,
               src, dst, K, dt, eps, tau, gm_in, gs_in, gh_in, A, P};
    if (alloc_fwd(&f)) { free_fwd(&f); return -1; }
    forward_internals(&f);
    const long N = (long)H * W;
    const int S = 2 * R + 1;
    const int NP = 3 * NK;

    double* zbar = (double*)calloc((long)C * N, sizeof(double));
    double* ubar = (double*)calloc((long)NK * N, sizeof(double));
    double* gPd = localized ? (double*)calloc((long)NP * N, sizeof(double)) : NULL;
    if (!zbar || !ubar || (localized && !gPd)) {
        free(zbar); free(ubar); free(gPd); free_fwd(&f); return -1;
    }

    /* clip of the state update (inclusive subgradient) */
    for (long i = 0; i < (long)C * N; ++i) {
        double z = f.Z[i];
        zbar[i] = (z >= 0.0 && z <= 1.0) ? gA_next[i] : 0.0;
        gA[i] = zbar[i];
    }
    if (!localized)
        for (int k = 0; k < NK; ++k) { gm[k] = 0.0; gs[k] = 0.0; gh[k] = 0.0; }

    /* growth derivatives */
    for (int k = 0; k < NK; ++k) {
        double am = 0.0, as = 0.0, ah = 0.0;
        for (long c = 0; c < N; ++c) {
            if (!f.alpha[c]) continue;
            double m, s, h;
            if (localized) {
                m = f.Pd[(long)(0 * NK + k) * N + c];
                s = f.Pd[(long)(1 * NK + k) * N + c];
                h = f.Pd[(long)(2 * NK + k) * N + c];
            } else {
                m = gm_in[k]; s = gs_in[k]; h = gh_in[k];
            }
            double u = f.U[(long)k * N + c];
            double d = u - m;
            double e = exp(-d * d / (2.0 * s * s));
            double gb = dt * zbar[(long)dst[k] * N + c];
            double dgdu = -2.0 * h * e * d / (s * s);
            ubar[(long)k * N + c] = gb * dgdu;
            double dm = gb * (2.0 * h * e * d / (s * s));
            double ds = gb * (2.0 * h * e * d * d / (s * s * s));
            double dh = gb * (2.0 * e - 1.0);
            if (localized) {
                gPd[(long)(0 * NK + k) * N + c] += dm;
                gPd[(long)(1 * NK + k) * N + c] += ds;
                gPd[(long)(2 * NK + k) * N + c] += dh;
            } else {
                am += dm; as += ds; ah += dh;
            }
        }
        if (!localized) { gm[k] = am; gs[k] = as; gh[k] = ah; }
    }

    /* transpose of u_k(x) = sum_d K(d) A(x+d): A_bar(y) += sum_d K(d) ubar(y-d);
     * and dL/dK(d) = sum_x ubar(x) A(x+d). */
    for (int ch = 0; ch < C; ++ch) {
        #pragma omp parallel for schedule(static)
        for (long y = 0; y < H; ++y)
            for (long x = 0; x < W; ++x) {
                double acc = 0.0;
                for (int k = 0; k < NK; ++k) {
                    if (src[k] != ch) continue;
                    const double* Ks = K + (long)k * S * S;
                    const double* Ub = ubar + (long)k * N;
                    for (int dy = -R; dy <= R; ++dy)
                        for (int dx = -R; dx <= R; ++dx) {
                            double kv = Ks[(dy + R) * S + (dx + R)];
                            if (kv != 0.0) acc += kv * Ub[wrap(y - dy, H) * W + wrap(x - dx, W)];
                        }
                }
                gA[(long)ch * N + y * W + x] += acc;
            }
    }
    for (int k = 0; k < NK; ++k) {
        const double* As = A + (long)src[k] * N;
        const double* Ub = ubar + (long)k * N;
        #pragma omp parallel for schedule(static)
        for (int t = 0; t < S * S; ++t) {
            int dy = t / S - R, dx = t % S - R;
            double acc = 0.0;
            for (long y = 0; y < H; ++y) {
                const double* row = As + wrap(y + dy, H) * W;
                for (long x = 0; x < W; ++x) acc += Ub[y * W + x] * row[wrap(x + dx, W)];
            }
            gK[(long)k * S * S + t] = acc;
        }
    }

    if (localized) {
        if (f.genotype_update) {
            /* mask P' = alpha * Pd, then the diffusion clip and quotient */
            double* numbar = (double*)calloc((long)NP * N, sizeof(double));
            if (!numbar) { free(zbar); free(ubar); free(gPd); free_fwd(&f); return -1; }
            for (long pk = 0; pk < NP; ++pk)
                for (long c = 0; c < N; ++c) {
                    long o = pk * N + c;
                    double pd_bar = f.alpha[c] ? (gP_next[o] + gPd[o]) : 0.0;
                    double n = f.cnt[o];
                    if (n > 0.0) {
                        double q = f.num[o] / n;
                        if (q >= 0.0 && q <= 1.0) numbar[o] = pd_bar / n;
                    }
                }
            int rd = r_diff;
            #pragma omp parallel for schedule(static)
            for (long y = 0; y < H; ++y)
                for (int pk = 0; pk < NP; ++pk)
                    for (long x = 0; x < W; ++x) {
                        double acc = 0.0;
                        for (int dy = -rd; dy <= rd; ++dy)
                            for (int dx = -rd; dx <= rd; ++dx) {
                                if (dy * dy + dx * dx > rd * rd) continue;
                                acc += numbar[(long)pk * N + wrap(y - dy, H) * W + wrap(x - dx, W)];
                            }
                        gP[(long)pk * N + y * W + x] = acc;
                    }
            free(numbar);
        } else {
            for (long i = 0; i < (long)NP * N; ++i) gP[i] = gP_next[i] + gPd[i];
        }
    }
    if (amb_out) ambiguity(&f, amb_out);
    free(zbar); free(ubar); free(gPd); free_fwd(&f);
    return 0;
}

/*
 * Gradient of the loss with respect to the shell heights beta_i of one kernel,
 * through K~ = (sum_i beta_i S_i) / Z, Z = sum_i beta_i |S_i|:
 *   dL/dbeta_i = (<gK, S_i> - |S_i| <gK, K~>) / Z.
 * gK is dL/dK~ on the (2R+1)^2 grid; writes B values to gbeta.
 */
ORACLE_EXPORT int oracle_beta_grad(int R, int B, const double* beta, const double* gK, double* gbeta)
{
    int S = 2 * R + 1;
    double* Kn = (double*)calloc((long)S * S, sizeof(double));
    if (!Kn) return -1;
    double Z = oracle_kernel(R, B, beta, Kn);
    double gk_dot_k = 0.0;
    for (int t = 0; t < S * S; ++t) gk_dot_k += gK[t] * Kn[t];
    for (int i = 0; i < B; ++i) {
        double dot = 0.0, size = 0.0;
        for (int dy = -R; dy <= R; ++dy)
            for (int dx = -R; dx <= R; ++dx) {
                double sv = oracle_shell_basis(R, B, i, dy, dx);
                dot += gK[(dy + R) * S + (dx + R)] * sv;
                size += sv;
            }
        gbeta[i] = (Z != 0.0) ? (dot - size * gk_dot_k) / Z : 0.0;
    }
    free(Kn);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Ring-decomposed localized kernels (Section 2.4).  Each kernel k carries, per
 * cell, two bumps (r_i, w_i, b_i), i = 0, 1, of the kernel function
 * kf(x; r, w, b) = b exp(-(x - r)^2 / (2 w^2)).  The disk |d| < R is split into
 * n_ring rings; ring j holds the offsets with floor(n_ring |d| / R) = j and
 * gets the weight kw_j = sum_i kf(j / n_ring; r_i, w_i, b_i) of the genes at
 * the output cell.  The normalized potential is
 *   u_k = sum_j kw_j (K_j * A_src(k)) / sum_j kw_j (K_j * 1),
 * K_j the indicator of ring j, so K_j * 1 is the ring's number of offsets (a
 * ring without lattice offsets adds nothing to either sum).  Gene tensor
 * P[9][NK][H][W] in the paper's parameter order r1, w1, b1, r2, w2, b2, m, s,
 * h.  Algorithm 2 otherwise as in the step above: every gene plane diffused,
 * alpha = all u_k > eps and all diffused genes > eps, P' = alpha P_d, growth
 * from the diffused m, s, h, A' = clip01(A + dt sum_k g_k) in ascending k.
 * Readings: ring index by floor (the paper numbers rings r = 0 .. n_ring-1
 * and evaluates the kernel function at r / n_ring); a bump with w <= 0
 * contributes 0; u_k = 0 where the denominator is 0.
 * ------------------------------------------------------------------------- */

/* Ring of offset (dy, dx), -1 outside the open disk |d| < R. */
ORACLE_EXPORT int oracle_ring_of(int R, int n_ring, int dy, int dx)
{
    long d2 = (long)dy * dy + (long)dx * dx;
    if (d2 >= (long)R * R) return -1;
    int j = (int)floor((double)n_ring * sqrt((double)d2) / (double)R);
    return (j < n_ring) ? j : -1;
}

/* Number of offsets in each ring: n_r[j], j = 0 .. n_ring-1. */
ORACLE_EXPORT void oracle_ring_sizes(int R, int n_ring, double* n_r)
{
    for (int j = 0; j < n_ring; ++j) n_r[j] = 0.0;
    for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
            int j = oracle_ring_of(R, n_ring, dy, dx);
            if (j >= 0) n_r[j] += 1.0;
        }
}

static double kernel_fn(double x, double r, double w, double b)
{
    if (!(w > 0.0)) return 0.0;
    return b * exp(-(x - r) * (x - r) / (2.0 * w * w));
}

/*
 * One step with ring kernels.  A[C][H][W], P[9][NK][H][W] (see above).
 * Outputs A_out, P_out; optional U_out [NK][H][W], alpha_out, amb_out [H][W]
 * (amb as for oracle_step).  Returns 0, or -1 on allocation failure.
 */
ORACLE_EXPORT int oracle_ring_step(int H, int W, int C, int NK, const int* src, const int* dst,
                                   int R, int n_ring, double dt, double eps, int r_diff,
                                   double tau, const double* A, const double* P,
                                   double* A_out, double* P_out, double* U_out,
                                   uint8_t* alpha_out, uint8_t* amb_out)
{
    const long N = (long)H * W;
    const int NP = 9 * NK;
    double* num = (double*)calloc((long)NP * N, sizeof(double));
    double* cnt = (double*)calloc((long)NP * N, sizeof(double));
    double* Pd = (double*)calloc((long)NP * N, sizeof(double));
    double* ringsum = (double*)calloc((long)C * n_ring * N, sizeof(double));
    double* U = (double*)calloc((long)NK * N, sizeof(double));
    double* n_r = (double*)calloc(n_ring, sizeof(double));
    if (!num || !cnt || !Pd || !ringsum || !U || !n_r) {
        free(num); free(cnt); free(Pd); free(ringsum); free(U); free(n_r);
        return -1;
    }
    /* Section 2.3: every gene plane is diffused */
    diffuse_planes(H, W, NP, r_diff, eps, P, num, cnt, Pd);
    oracle_ring_sizes(R, n_ring, n_r);

    /* K_j * A_c: the sum of A_c over ring j around each cell (direct torus sum) */
    #pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (int c = 0; c < C; ++c)
            for (long x = 0; x < W; ++x) {
                double* rs = ringsum + ((long)c * n_ring) * N + y * W + x;
                for (int dy = -R; dy <= R; ++dy)
                    for (int dx = -R; dx <= R; ++dx) {
                        int j = oracle_ring_of(R, n_ring, dy, dx);
                        if (j < 0) continue;
                        rs[(long)j * N] += A[(long)c * N + wrap(y + dy, H) * W + wrap(x + dx, W)];
                    }
            }

    /* per-cell ring weights from the diffused genes, recombined potentials */
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c)
        for (int k = 0; k < NK; ++k) {
            double g[6];
            for (int p = 0; p < 6; ++p) g[p] = Pd[(long)(p * NK + k) * N + c];
            double nu = 0.0, de = 0.0;
            for (int j = 0; j < n_ring; ++j) {
                double x = (double)j / (double)n_ring;
                double kw = kernel_fn(x, g[0], g[1], g[2]) + kernel_fn(x, g[3], g[4], g[5]);
                nu += kw * ringsum[((long)src[k] * n_ring + j) * N + c];
                de += kw * n_r[j];
            }
            U[(long)k * N + c] = (de > 0.0) ? nu / de : 0.0;
        }

    /* Section 2.2 alpha, Algorithm 2 mask, growth and clipped update */
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
        int a = 1;
        uint8_t b = 0;
        for (int k = 0; k < NK; ++k) {
            double u = U[(long)k * N + c];
            if (!(u > eps)) a = 0;
            if (fabs(u - eps) <= tau) b |= 1;
        }
        for (int pk = 0; pk < NP; ++pk) {
            double v = Pd[(long)pk * N + c];
            if (!(v > eps)) a = 0;
            if (fabs(v - eps) <= tau) b |= 1;
            double n = cnt[(long)pk * N + c];
            if (n > 0.0) {
                double q = num[(long)pk * N + c] / n;
                if (fabs(q) <= tau || fabs(q - 1.0) <= tau) b |= 2;
            }
        }
        for (int ch = 0; ch < C; ++ch) {
            double sum = 0.0;
            for (int k = 0; k < NK; ++k) {
                if (dst[k] != ch || !a) continue;
                double m = Pd[(long)(6 * NK + k) * N + c];
                double s = Pd[(long)(7 * NK + k) * N + c];
                double h = Pd[(long)(8 * NK + k) * N + c];
                double d = U[(long)k * N + c] - m;
                sum += h * (2.0 * exp(-d * d / (2.0 * s * s)) - 1.0);
            }
            double z = A[(long)ch * N + c] + dt * sum;
            if (fabs(z) <= tau || fabs(z - 1.0) <= tau) b |= 2;
            A_out[(long)ch * N + c] = fmax(fmin(z, 1.0), 0.0);
        }
        for (int pk = 0; pk < NP; ++pk) P_out[(long)pk * N + c] = a ? Pd[(long)pk * N + c] : 0.0;
        if (alpha_out) alpha_out[c] = (uint8_t)a;
        if (amb_out) amb_out[c] = b;
    }
    if (U_out) memcpy(U_out, U, sizeof(double) * NK * N);
    free(num); free(cnt); free(Pd); free(ringsum); free(U); free(n_r);
    return 0;
}

/*
 * The cast form of the same localized kernels, the reference Section 2.4
 * recombines its rings against: at each cell, kernel k is the two-bump kernel
 * function of the cell's diffused genes (the r1, w1, b1, r2, w2, b2 planes,
 * diffused as in oracle_ring_step, unmasked) evaluated at each offset's own
 * radius |d| / R over the open disk |d| < R, and
 *   u_k = sum_d K(|d|/R) A_src(x + d) / sum_d K(|d|/R),   0 if that is 0.
 * The ring form evaluates the same function at the inner radius j / n_ring of
 * the offset's ring instead.  U[NK][H][W].  Returns 0, or -1 on allocation
 * failure.
 */
ORACLE_EXPORT int oracle_cast_potentials(int H, int W, int C, int NK, const int* src, int R,
                                         double eps, int r_diff, const double* A, const double* P,
                                         double* U)
{
    const long N = (long)H * W;
    const int NP = 9 * NK;
    double* Pd = (double*)calloc((long)NP * N, sizeof(double));
    if (!Pd) return -1;
    (void)C;
    diffuse_planes(H, W, NP, r_diff, eps, P, NULL, NULL, Pd);
    #pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (int k = 0; k < NK; ++k)
            for (long x = 0; x < W; ++x) {
                const long c = y * W + x;
                double g[6];
                for (int p = 0; p < 6; ++p) g[p] = Pd[(long)(p * NK + k) * N + c];
                const double* As = A + (long)src[k] * N;
                double nu = 0.0, de = 0.0;
                for (int dy = -R; dy <= R; ++dy)
                    for (int dx = -R; dx <= R; ++dx) {
                        const long d2 = (long)dy * dy + (long)dx * dx;
                        if (d2 >= (long)R * R) continue;
                        const double rho = sqrt((double)d2) / (double)R;
                        const double kw = kernel_fn(rho, g[0], g[1], g[2]) + kernel_fn(rho, g[3], g[4], g[5]);
                        nu += kw * As[wrap(y + dy, H) * W + wrap(x + dx, W)];
                        de += kw;
                    }
                U[(long)k * N + c] = (de > 0.0) ? nu / de : 0.0;
            }
    free(Pd);
    return 0;
}

/* ---------------------------------------------------------------------------
 * The random and environmental operators of Algorithm 2 around one step:
 * walls (Section 2.7), mutation (Section 2.5) and the penalization of
 * exploding patterns (Section 2.6), for the shell form with localized genes
 * that are updated.  The random draws of the iteration are inputs.
 *   1. walls: A and P are set to 0 on the wall cells (of the input state);
 *   2. the step of oracle_step (diffusion, potentials, alpha, mask, growth);
 *   3. organic matter = Delta_sum(U): the cells where the sum over kernels of
 *      the potentials exceeds eps; E_oxy = the cells with a non-organic cell
 *      within the disk |d| <= r_oxy; E_pen = the cells with a cell outside
 *      E_oxy within that disk (the oxygenated area, then the area around what
 *      it does not reach);
 *   4. mutation: P[mut_p][mut_k] += gamma_mut * mut_delta on the square of
 *      side 2s (rows y0 - s .. y0 + s - 1, columns likewise, on the torus)
 *      where alpha = 1;
 *   5. penalization: P[pen_p][pen_k] += gamma_pen * pen_delta where E_pen and
 *      alpha hold.
 * Readings: the disk K_oxy is |d| <= r_oxy; the two convolutions of the
 * paper are read as set operations (any cell of the disk); no clip after the
 * two additions (the next diffusion clips).  A, P are updated in place.
 * flags_out[H][W]: bit 0 alpha, bit 1 organic; epen_out[H][W]: E_pen;
 * amb_out as oracle_step, plus bit 2 where the organic sum is within tau of
 * eps.  Returns 0, or -1 on allocation failure.
 * ------------------------------------------------------------------------- */
static void disk_any(int H, int W, int r, const uint8_t* in, uint8_t want, uint8_t* out)
{
    #pragma omp parallel for schedule(static)
    for (long y = 0; y < H; ++y)
        for (long x = 0; x < W; ++x) {
            uint8_t hit = 0;
            for (int dy = -r; dy <= r && !hit; ++dy)
                for (int dx = -r; dx <= r; ++dx) {
                    if (dy * dy + dx * dx > r * r) continue;
                    if (in[wrap(y + dy, H) * W + wrap(x + dx, W)] == want) { hit = 1; break; }
                }
            out[y * W + x] = hit;
        }
}

ORACLE_EXPORT int oracle_evolve_step(int H, int W, int C, int NK, const int* src, const int* dst,
                                     int R, const double* K, double dt, double eps, int r_diff,
                                     double tau, const uint8_t* walls, double gamma_mut,
                                     int mut_half, double gamma_pen, int r_oxy, int mut_p,
                                     int mut_k, double mut_delta, int mut_y0, int mut_x0,
                                     int pen_p, int pen_k, double pen_delta, double* A, double* P,
                                     uint8_t* flags_out, uint8_t* epen_out, uint8_t* amb_out)
{
    const long N = (long)H * W;
    const int NP = 3 * NK;
    if (walls)
        for (long c = 0; c < N; ++c)
            if (walls[c]) {
                for (int ch = 0; ch < C; ++ch) A[(long)ch * N + c] = 0.0;
                for (int pk = 0; pk < NP; ++pk) P[(long)pk * N + c] = 0.0;
            }
    double* A1 = (double*)malloc(sizeof(double) * C * N);
    double* P1 = (double*)malloc(sizeof(double) * NP * N);
    double* U = (double*)malloc(sizeof(double) * NK * N);
    uint8_t* alpha = (uint8_t*)malloc(N);
    uint8_t* organic = (uint8_t*)malloc(N);
    uint8_t* eoxy = (uint8_t*)malloc(N);
    uint8_t* epen = (uint8_t*)malloc(N);
    int rc = (A1 && P1 && U && alpha && organic && eoxy && epen) ? 0 : -1;
    if (rc == 0)
        rc = oracle_step(H, W, C, NK, src, dst, R, K, dt, 1, NULL, NULL, NULL, 1, eps, r_diff, tau,
                         A, P, A1, P1, U, alpha, amb_out);
    if (rc == 0) {
        for (long c = 0; c < N; ++c) {
            double su = 0.0;
            for (int k = 0; k < NK; ++k) su += U[(long)k * N + c];
            organic[c] = (su > eps) ? 1 : 0;
            if (amb_out && fabs(su - eps) <= tau) amb_out[c] |= 4;
        }
        disk_any(H, W, r_oxy, organic, 0, eoxy);   /* oxygenated: empty space in reach */
        disk_any(H, W, r_oxy, eoxy, 0, epen);      /* around what oxygen does not reach */
        if (gamma_mut != 0.0)
            for (int i = 0; i < 2 * mut_half; ++i)
                for (int j = 0; j < 2 * mut_half; ++j) {
                    long c = wrap(mut_y0 - mut_half + i, H) * W + wrap(mut_x0 - mut_half + j, W);
                    if (alpha[c]) P1[(long)(mut_p * NK + mut_k) * N + c] += gamma_mut * mut_delta;
                }
        if (gamma_pen != 0.0)
            for (long c = 0; c < N; ++c)
                if (epen[c] && alpha[c]) P1[(long)(pen_p * NK + pen_k) * N + c] += gamma_pen * pen_delta;
        memcpy(A, A1, sizeof(double) * C * N);
        memcpy(P, P1, sizeof(double) * NP * N);
        for (long c = 0; c < N; ++c) {
            if (flags_out) flags_out[c] = (uint8_t)(alpha[c] | (organic[c] << 1));
            if (epen_out) epen_out[c] = epen[c];
        }
    }
    free(A1); free(P1); free(U); free(alpha); free(organic); free(eoxy); free(epen);
    return rc;
}
