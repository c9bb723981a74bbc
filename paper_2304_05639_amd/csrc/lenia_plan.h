// Plan object behind the opaque lenia_plan_t handle (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "lenia.h"
#include "lenia_internal.h"

namespace lenia {

lenia_status set_error(lenia_status s, const std::string& msg);
lenia_status hip_fail(hipError_t e, const char* what);
lenia_status validate(const lenia_desc* d);
int table_of(const lenia_desc* d);
int mode_of(const lenia_desc* d);
float eps_below(double eps);
double raw_kernel_tap(int R, int B, const double* beta, int dy, int dx);
double raw_kernel_sum(int R, int B, const double* beta);
void orbit_list(int R, std::vector<int>& a, std::vector<int>& b);
int orbit_size(int a, int b);
bool conv_form_supported(int conv, int table, int R);
bool conv_is_dft(int conv);   // one of the split DFT-as-GEMM forms
int dft_valid_side(int R);
struct WorldPlan;
lenia_status build_dft_tables(lenia_plan_t p, WorldPlan& w, hipStream_t s, std::vector<void*>& keep);
hipError_t launch_dft_potentials(const lenia_plan_t p, const WorldPlan& w, const float* A, float* U,
                                 hipStream_t s);
// The whole step of the DFT forms in one kernel (MODE_LOCAL_UPDATE, no saved
// potentials, alpha or flags): potentials on the MFMA units, then diffusion,
// alpha test, growth and update of every cell of the tile.
hipError_t launch_dft_step(const lenia_plan_t p, const WorldPlan& w, const WorldArgs& wa, hipStream_t s);

// One world of a plan, with its descriptor arrays copied.
struct WorldPlan {
    int H = 0, W = 0, C = 0, NK = 0, R = 0, mode = 0;
    double dt = 0, eps = 0;
    std::vector<int> n_shells;
    std::vector<double> beta;      // [NK][3]
    std::vector<double> gm, gs, gh;
    int n_orbits = 0;
    int table = 0;
    int gene_types = 3;            // gene planes per kernel: 3 (m, s, h) or 9 (ring form)
    float* d_w = nullptr;          // [NK][n_orbits] orbit weights of K~_k
    float* d_wt = nullptr;         // [n_orbits][C][8] by (orbit, source, slot)
    float* d_wtp = nullptr;        // [n_orbits][wt_stride] packed: source * KPS + slot
    float* d_shc = nullptr;        // [C][KPS][8] shell coefficients (15-kernel table)
    float* d_bcoef = nullptr;      // [NK][3][n_orbits] beta-gradient coefficients
    float* d_bt = nullptr;         // the same in the step kernel's orbit order
    int* d_nshells = nullptr;      // [NK]
    void* dft_f1t = nullptr;       // DFT forms: transform matrices (hi / lo parts),
    void* dft_f2 = nullptr;        //   kernel spectra and the potentials workspace
    void* dft_f3 = nullptr;
    void* dft_f4t = nullptr;
    float* dft_khat = nullptr;
    float* dft_u = nullptr;        // [NK][H][W]
    bool dft_fused = false;        // DFT forms: eligible steps run as one kernel
    float* ws_A = nullptr;         // ping-pong state workspace [C][H][W]
    float* ws_P = nullptr;         // [gene_types][NK][H][W] (gene update only)
    uint8_t* p_zero = nullptr;     // [2][tiles] zero-gene tile flags of the caller's P
                                   //   output and of ws_P (allocated on first use)
    size_t cells() const { return (size_t)H * W; }
    size_t a_elems() const { return (size_t)C * H * W; }
    size_t p_elems() const { return (size_t)gene_types * NK * H * W; }
    WorldArgs args_template() const;
};

struct BackwardWs {
    float* ubar = nullptr;         // [NK][H][W]
    float* numbar = nullptr;       // [3NK][H][W]
    float* part = nullptr;         // [n_tiles][NK][3] beta-gradient partials
    int n_part = 0;
};

// LENIA_FLAG_CHECK_FINITE: one caller buffer of a call.  Every buffer must lie
// inside the device allocation that holds it; those with `scan` set must hold
// finite floats only.
struct DebugBuf {
    const void* ptr;       // may be NULL (skipped)
    size_t bytes;
    const char* name;
    bool scan;             // input buffer of floats: checked for NaN / infinity
};
// No-op unless the plan was made with LENIA_FLAG_CHECK_FINITE; otherwise the
// checks above (the scan waits for the stream).
lenia_status debug_checks(lenia_plan_t p, const DebugBuf* bufs, int n, hipStream_t s);

typedef hipError_t (*epilogue_launch_fn)(const WorldArgs& w, const float* U, int mode,
                                         hipStream_t s);
epilogue_launch_fn find_epilogue_launcher(int table);

}  // namespace lenia

struct lenia_plan_ {
    std::vector<lenia::WorldPlan> worlds;
    bool batched = false;
    int table = 0, mode = 0, R = 0, conv = LENIA_CONV_DIRECT_F32;
    bool rings = false;            // ring-decomposed kernels (n_ring > 0)
    int tile_y = 0, tile_x = 0;
    lenia::step_launch_fn step_fn = nullptr;
    lenia::batch_launch_fn batch_fn = nullptr;
    size_t ws_bytes = 0;
    int device = 0;
    // batched execution
    lenia::WorldArgs* d_tables[2] = {nullptr, nullptr};   // phase 0: X -> ws, 1: ws -> X
    int2* d_items = nullptr;
    int n_items = 0;
    uint8_t* batch_zero = nullptr;    // zero-gene tile flags of every world's two output
    size_t batch_zero_bytes = 0;      //   buffers (ws in phase 0, the caller's in phase 1)
    std::vector<float*> graph_A, graph_P;                 // pointer set of the graph
    hipGraphExec_t graph = nullptr;
    hipStream_t capture_stream = nullptr;                 // private stream used for capture
    // adjoint
    lenia::BackwardWs bw;
    // operators around the step (lenia_step_evolve): per-cell flags (alpha,
    // organic), the oxygenated area and the penalizing area
    uint8_t* evo_flags = nullptr;
    uint8_t* evo_eoxy = nullptr;
    uint8_t* evo_epen = nullptr;
    // LENIA_FLAG_CHECK_FINITE: one bit per scanned buffer of a call
    bool check_finite = false;
    uint32_t* d_nonfinite = nullptr;
    std::vector<void*> allocations;
};
