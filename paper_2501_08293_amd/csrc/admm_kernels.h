// Device-side structures shared by the iteration kernels and the C-ABI
// implementation (internal header).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace opf {

// ---- arithmetic of one iteration, shared by every schedule (single-instance
// step and persistent kernels, serving kernel) with explicit fused
// multiply-adds, so that all schedules round identically.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// term of one copy in the consensus sum of global_sparse: z_e - lambda_e / rho
template <typename T>
__device__ __forceinline__ T copy_term(T z, T l, T inv_rho) {
    return fmadd(-l, inv_rho, z);
}
// global_sparse: clipped average of the copy terms, shifted by the cost term
template <typename T>
__device__ __forceinline__ T consensus_value(T acc, T cost, T inv_rho, int copies, T lo, T hi) {
    const T xh = fmadd(-cost, inv_rho, acc) / (T)copies;
    return xh < lo ? lo : (xh > hi ? hi : xh);
}
// input of the local projection closed_2: B_s x + lambda_s / rho
template <typename T>
__device__ __forceinline__ T projection_input(T x, T l, T inv_rho) {
    return fmadd(l, inv_rho, x);
}
// local projection closed_2 for one slot: acc + sum_k F[k][lane] v[(base + k) & 63]
// over k ascending (F column-blocked [k][lane]); the loads of eight columns are
// issued ahead of their dependent fused multiply-adds
template <typename T>
__device__ __forceinline__ T project_row(const T* F, const T* v, int base, int lane, int ncols, T acc) {
    int k = 0;
    for (; k + 8 <= ncols; k += 8) {
        T f[8], x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            f[j] = F[(k + j) * 64 + lane];
            x[j] = v[(base + k + j) & 63];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) acc = fmadd(f[j], x[j], acc);
    }
    for (; k < ncols; ++k) acc = fmadd(F[k * 64 + lane], v[(base + k) & 63], acc);
    return acc;
}
// Sum of a double over the 64 lanes of a wavefront, in one fixed order, with
// DPP lane moves (no LDS traffic): an inclusive scan inside each row of 16
// lanes (shifts 1, 2, 4, 8), then row 0 into row 1 and row 2 into row 3, then
// rows 0-1 into rows 2-3; lane 63 ends with the total, which every lane
// receives.  Used by every schedule, so all reduce in the same order.  Lanes
// without a source lane read 0 (bound_ctrl), so no move needs a zeroed
// destination; the broadcasts also add into rows whose sums lane 63 never
// reads again (row 2 at the first, rows 0 and 1 at the second).
__device__ __forceinline__ double dpp_move(double v, int ctrl_id) {
    const long long b = __double_as_longlong(v);
    int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
    switch (ctrl_id) {
        case 0: lo = __builtin_amdgcn_mov_dpp(lo, 0x111, 0xf, 0xf, true);
                hi = __builtin_amdgcn_mov_dpp(hi, 0x111, 0xf, 0xf, true); break;   // row_shr:1
        case 1: lo = __builtin_amdgcn_mov_dpp(lo, 0x112, 0xf, 0xf, true);
                hi = __builtin_amdgcn_mov_dpp(hi, 0x112, 0xf, 0xf, true); break;   // row_shr:2
        case 2: lo = __builtin_amdgcn_mov_dpp(lo, 0x114, 0xf, 0xf, true);
                hi = __builtin_amdgcn_mov_dpp(hi, 0x114, 0xf, 0xf, true); break;   // row_shr:4
        case 3: lo = __builtin_amdgcn_mov_dpp(lo, 0x118, 0xf, 0xf, true);
                hi = __builtin_amdgcn_mov_dpp(hi, 0x118, 0xf, 0xf, true); break;   // row_shr:8
        case 4: lo = __builtin_amdgcn_mov_dpp(lo, 0x142, 0xf, 0xf, true);
                hi = __builtin_amdgcn_mov_dpp(hi, 0x142, 0xf, 0xf, true); break;   // row_bcast:15
        default: lo = __builtin_amdgcn_mov_dpp(lo, 0x143, 0xf, 0xf, true);
                 hi = __builtin_amdgcn_mov_dpp(hi, 0x143, 0xf, 0xf, true); break;  // row_bcast:31
    }
    return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
    for (int c = 0; c < 6; ++c) v += dpp_move(v, c);
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)(unsigned)hi << 32) | (unsigned)lo);
}

// dual update ADMM-3: lambda_s + rho (B_s x - x_s)
template <typename T>
__device__ __forceinline__ T dual_step(T l, T rho, T x, T z) {
    return fmadd(rho, x - z, l);
}

// Residual balancing of the penalty (the acceleration of Section III-D, in
// Wohlberg's form).  The penalty of iteration k lives in Ctrl::rho[k %
// kRhoRing]; the decision taken on the residuals of iteration u writes the
// penalty of iteration u + kRhoLag.  The persistent kernel learns the
// decision of u only at the start of u + kDecisionLag, and the consensus
// term it publishes at the end of that iteration already carries the next
// iteration's 1/rho, hence one iteration more than the decision lag.
constexpr int kRhoRing = 8;
constexpr int kRhoLag = 4;

struct RhoRule {
    int every;             // 0: fixed penalty; else decide after every `every`-th iteration
    int mode;              // 0: residuals relative to their tolerances; 1: plain residuals
    double mu, tau, lo, hi;
};

// Factor of one balancing decision: tau when the primal residual exceeds mu
// times the dual one, 1/tau in the opposite case, else 1.
__host__ __device__ __forceinline__ double rho_factor(const RhoRule& r, double pres, double dres, double ep,
                                                      double ed) {
    double a = pres, b = dres;
    if (r.mode == 0) {
        a = ep > 0.0 ? pres / ep : __builtin_huge_val();
        b = ed > 0.0 ? dres / ed : __builtin_huge_val();
    }
    if (a > r.mu * b) return r.tau;
    if (b > r.mu * a) return 1.0 / r.tau;
    return 1.0;
}
// Penalty of iteration u + kRhoLag from the one of u + kRhoLag - 1 and the
// residuals of iteration u.
__host__ __device__ __forceinline__ double rho_decide(const RhoRule& r, double prev, long long u, double pres,
                                                      double dres, double ep, double ed) {
    if (u % r.every != 0) return prev;
    const double v = prev * rho_factor(r, pres, dres, ep, ed);
    return v < r.lo ? r.lo : (v > r.hi ? r.hi : v);
}

// Workgroups of kernel `fn` that one compute unit holds at once with `dyn`
// bytes of dynamic shared memory: the occupancy query, further bounded by
// counting each workgroup's LDS (static and dynamic) in whole 4 KiB blocks.
// The query counts bytes: a grid it admitted at three workgroups per compute
// unit, 2.3 KiB short of the LDS, was not co-resident on gfx950, while grids
// whose workgroups fit the LDS in whole 4 KiB blocks have been (a persistent
// grid that is not co-resident can only end by its bounded waits).  The
// bound applies only where the device's LDS size agrees with the query.
constexpr size_t kLdsBlock = 4096;
inline hipError_t resident_per_cu(int* per, const void* fn, int threads, size_t dyn) {
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per, fn, threads, dyn);
    if (e != hipSuccess) return e;
    hipFuncAttributes at;
    int dev = 0, lds = 0;
    if ((e = hipFuncGetAttributes(&at, fn)) != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev)) != hipSuccess)
        return e;
    const size_t bytes = at.sharedSizeBytes + dyn;
    const size_t need = (bytes + kLdsBlock - 1) / kLdsBlock * kLdsBlock;
    if (bytes > 0 && *per > 0 && (size_t)lds >= (size_t)*per * bytes) {
        const int fit = (int)((size_t)lds / need);
        if (fit < *per) *per = fit;
    }
    return hipSuccess;
}

// Control block in device memory; written by the last workgroup of each
// iteration, read by the host between launches and by the next iteration.
struct Ctrl {
    long long iter;        // completed iterations
    long long max_iter;    // stop when iter reaches this value
    int stop;              // 1: later launches return at once
    int status;            // OPF_OK / OPF_NOT_CONVERGED / OPF_ENUMERIC / OPF_EHANG at stop
    int check;             // 1: apply the termination test
    unsigned int arrive;   // last-workgroup-done counter (returns to 0)
    double res[4];         // pres, dres, eps_prim, eps_dual of iteration `iter`
    double objective;      // c^T x (written by the output kernel)
    double rho[kRhoRing];  // penalty of iteration k at rho[k % kRhoRing] (residual balancing only)
    long long pad[4];
};

// Arguments of one iteration kernel, for state/factor type T (double or float).
// Device slot d = wave * 64 + lane.  Ping-pong state: iteration t reads buffer
// (t-1)&1 and writes buffer t&1.
template <typename T>
struct IterArgs {
    const T* F;                 // packed factors, [k][lane] per wave
    const int2* winfo;          // per wave: (columns stored, factor offset / 64)
    const int* var;             // per slot: global variable, -1 for padding
    const int* meta;            // base lane | n_s << 8 | owner << 16
    const int* cstart;          // per slot: offset of its variable's copy list
    const int* ccnt;            // per slot: copies of its variable (N_i)
    const int* clist;           // copy lists (device slots, ascending)
    const T* bbar;              // per slot
    const T* lo;                // per slot: bound of its variable
    const T* hi;
    const T* cost;              // per slot: objective coefficient of its variable
    T* z0; T* z1;               // local copies x_s (stacked), ping-pong
    T* l0; T* l1;               // duals lambda_s (stacked), ping-pong
    T* x0; T* x1;               // global variables, ping-pong (written by owner slots)
    double* partials;           // [grid][5] per-workgroup residual sums
    Ctrl* ctrl;
    double* hist;               // [hist_cap][4]
    int hist_cap;
    int waves;
    T rho, inv_rho;             // rho: the dual step length (local_updates x penalty)
    double rho_d, eps_rel;      // rho_d: the penalty
    RhoRule rule;               // rule.every == 0: rho fixed at rho_d
    double local_updates;       // local updates per global update (dual step = local_updates x penalty)
};

// Extra state of the persistent kernel (see admm_persistent.hip).
struct PersistArgs {
    unsigned long long* pub;    // [2][LP][words] published copy terms with iteration tags
    unsigned long long* records;// [kDecisionLag][10][G] tagged residual partial sums (word-major)
    long long* dec_iter;        // last iteration the reducer has decided
    long long* dec_stop;        // stop iteration, -1 while running
    int* error;                 // OPF_EHANG when a bounded wait ran out
    long long spin_limit;       // polls before a wait gives up
    long long max_iter;         // stop when this iteration count is reached
    int check;                  // 1: apply the termination test
    int lds_factors;            // 0: factors read from memory; FP32: 1 = every workgroup's factors in LDS;
                                // FP64: the column budget (workgroups within it hold theirs in LDS)
    int lds_factor_cols;        // columns of dynamic shared memory per workgroup
    int xcd_remap;              // 1: consecutive workgroups of the packing share an XCD
};

// Extra state of the tiled persistent schedule (see admm_persistent.hip): the
// state of the last kStateRing iterations, in the iteration kernel's element
// type, and the number of workgroup tiles of the packing.
constexpr int kStateRing = 4;
struct TiledArgs {
    void* zr;                   // [kStateRing][LP] local copies
    void* lr;                   // [kStateRing][LP] duals
    void* xr;                   // [kStateRing][n] global variables (written by owner slots)
    int tiles;                  // workgroup tiles of the packing (block_waves wavefronts each)
    int n;
    int pair;                   // 1: at most two tiles per workgroup, both in flight (admm_tiled_pair_kernel)
    int lds_cols;               // two-tile kernel: factor columns of dynamic shared memory per workgroup; a
                                // workgroup whose tiles' columns fit keeps their factors there (0: none)
};

// Iterations between a residual reduction and the moment workgroups act on
// its stop decision (also the depth of the partial-sum ring and of the state
// history each slot keeps in registers).
constexpr int kDecisionLag = 3;

// Position of a workgroup in the packing.  With remap, hardware workgroup ids
// (dealt round-robin over the 8 XCDs) are renumbered so that each XCD runs a
// contiguous range of the packing (a permutation of [0, nb)): neighbouring
// workgroups then share data through one XCD's L2.
__device__ __forceinline__ int logical_block(int bx, int nb, int remap) {
    if (!remap) return bx;
    const int x = bx & 7, j = bx >> 3;
    const int full = nb >> 3, rem = nb & 7;
    return x * full + (x < rem ? x : rem) + j;
}

// ---- serving runtime: one resident solve (see admm_multi.hip, admm_persistent.hip)
struct InstDesc {
    const int2* winfo;
    const int* var;
    const int* meta;
    const int* cstart;
    const int* ccnt;
    const int* clist;
    const int* user_slot;
    const double* F;
    const double* bbar;
    const double* lo;
    const double* hi;
    const double* cost;
    double* z0; double* z1;
    double* l0; double* l1;
    double* x0; double* x1;
    // FP32 copies for the bulk phase of a mixed-precision solve (null otherwise)
    const float* Ff;
    const float* bbarf;
    const float* lof;
    const float* hif;
    const float* costf;
    float* z0f; float* z1f;
    float* l0f; float* l1f;
    float* x0f; float* x1f;
    unsigned long long* records;// [kDecisionLag][10][blocks] tagged residual partial sums (word-major)
    unsigned long long* pub;    // [2][lanes][2] published copy terms (persistent schedule)
    long long* dec;             // [2]: last decided iteration, stop iteration
    Ctrl* ctrl;
    int blocks;                 // workgroups of this solve
    int lanes;                  // blocks * WPB * 64
    int n;
    double rho, eps_rel;
};

// Launch-wide arguments of the persistent serving kernel.
struct ServeArgs {
    int* error;                 // OPF_EHANG when a bounded wait ran out (shared by all solves)
    long long spin_limit;
    long long chunk;            // iterations per launch before a solve pauses
    int xcd_remap;
    int lds_cols;               // factor columns of the dynamic LDS budget per workgroup; a workgroup
                                // whose factors fit holds them in LDS, the others read them from memory
};

// fp32 = 1: the launch runs the FP32 bulk phase of its solves, else FP64.  The
// caller clears s.error before the launches of one round (a hang reported by
// one launch makes the later ones of the round end early).
hipError_t launch_serve_persistent(const InstDesc* descs, const int2* work, int nwork, const ServeArgs& s,
                                   int fp32, hipStream_t st);
int serve_capacity(size_t lds_bytes, int fp32);

// Control block reset; with narrow = 1 also the FP32 start state from the FP64 one.
hipError_t launch_multi_init(InstDesc* descs, int slot, int lanes, long long max_iter, int narrow, hipStream_t st);
// Outputs of the FP64 state, or (fp32 = 1) of the FP32 state of a solve that ends unpolished.
hipError_t launch_multi_output(const InstDesc* descs, int slot, double* xo, double* zo, double* lo, int fp32,
                               hipStream_t st);
hipError_t launch_warm_gather(const int4* plan, int nplan, const double* rz, const double* rl, double* zu,
                              double* lu, hipStream_t st);
hipError_t launch_to_device_order(const double* zu, const double* lu, const int* user_slot, int lanes,
                                  const double* zdef, double* zd, double* ld, int use_warm, hipStream_t st);

}  // namespace opf
