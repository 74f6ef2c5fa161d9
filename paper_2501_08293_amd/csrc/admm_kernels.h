// Device-side structures shared by the iteration kernels and the C-ABI
// implementation (internal header).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace opf {

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
    T rho, inv_rho;
    double rho_d, eps_rel;
};

}  // namespace opf
