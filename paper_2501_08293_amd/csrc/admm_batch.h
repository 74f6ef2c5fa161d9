// Batched same-topology scenarios (internal header; see admm_batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace opf {

constexpr int kBatchKernelRev = 8;   // revision of the step kernel (tuning decisions are kept per revision)
constexpr int kBatchCopies = 6;    // copies per variable gathered from the slot record (more: from the copy list)

// ---- batched same-topology scenarios (see admm_batch.hip)
struct BatchCtrl {
    long long iter;         // completed iterations
    long long max_iter;
    int stop;               // 1: every scenario has stopped (later launches return)
    int done;               // scenarios stopped so far
    unsigned arrive;        // last-workgroup counter of the reduction launch
    int pad;
};

struct BatchArgs {
    const uint16_t* Fp;     // [terms][W][64][64] bfloat16 planes of the block-diagonal factors
    int terms;              // 2 or 3
    const int* wave_var;    // [W] index among the scenario-varying wavefronts or -1 (null: none)
    const float* Fv;        // [varying wave][fv_cols][64][Kp] per-scenario factors (FP32)
    int fv_cols;
    int vary_waves;         // the varying wavefronts lie in [0, vary_waves) of the packing (0: none)
    const int4* sdesc;      // [LP] per slot: variable (-1: padding), copies, first copy in clist, owner
    const float4* sval;     // [LP] per slot: cost, lower bound, upper bound, 0
    const int4* scopy;      // [LP][2] per slot: its variable's first kBatchCopies copies (then the slot itself)
    const int* meta;        // base lane | n_s << 8 | owner << 16
    const int* clist;
    // scenario state, chunk-major: 64-scenario chunk c of slot d at (c LP + d) 64
    const float* bbar;      // [Kp / 64][LP][64]
    float* z0; float* z1;   // [Kp / 64][LP][64] ping-pong
    float* l0; float* l1;
    float* x0; float* x1;   // [Kp / 64][n][64]
    double* part;           // [5][Kp][W] per-wavefront residual partials
    BatchCtrl* ctrl;
    int W, Kp, K, n;
    float rho, inv_rho;
    int order;              // workgroup order: bit 0 XCD-contiguous packing ranges, bit 1 chunk-major
    int c0, nc;             // this launch's 64-scenario chunks: [c0, c0 + nc)
};

struct BatchRedArgs {
    const double* part;
    BatchCtrl* ctrl;
    int* state;             // [K] 0 running, 1 converged, 2 stopped at max_iter, 3 NaN/Inf
    long long* iters;       // [K]
    double* res;            // [K][4]
    double* objective;      // [K]
    double* xout;           // [K][n] snapshot at the scenario's stop iteration
    const float* x0; const float* x1;
    const double* c;
    int W, Kp, K, n;
    double rho, eps_rel;
    int k0;                 // this launch's scenarios: [k0, k0 + gridDim.x)
};


// One iteration of the scenario group whose chunks a.c0 .. a.c0 + a.nc - 1
// and scenarios r.k0 .. r.k0 + kn - 1 are given (kn: its scenarios below K).
hipError_t launch_batch_iteration(const BatchArgs& a, const BatchRedArgs& r, int kn, hipStream_t st);
// State of every scenario at the default start, and the control blocks of
// the `groups` scenario groups.
hipError_t launch_batch_init(const double* z0, float* z, float* l, int LP, int Kp, BatchCtrl* ctrl, int groups,
                             int* state, int K, long long max_iter, hipStream_t st);

}  // namespace opf
