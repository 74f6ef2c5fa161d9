// Iteration kernels of the solver-free componentwise ADMM for gfx950.
//
// One launch performs one full iteration of Algorithm 1 for every component:
//   global update (global_sparse): each slot recomputes the clipped consensus
//       average of its variable from all copies of that variable, in one fixed
//       order, so every copy obtains the same x_i bit for bit;
//   local update (closed_2): x_s = F_s (B_s x + lambda_s / rho) + bbar_s as a
//       64-lane wavefront matvec, the input vector staged in LDS;
//   dual update (ADMM-3): lambda_s += rho (B_s x - x_s);
//   residual sums of the termination test, accumulated in FP64 in fixed order
//       (wavefront shuffles, then workgroup, then the last workgroup to finish
//       reduces all workgroup partials and takes the stop decision).
// Recomputing x per slot removes the grid-wide dependency between the global
// and the local step, so an iteration is a single launch.
#include "admm_kernels.h"

#include "../../include/opf_admm.h"

namespace opf {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Arrival counters of the step kernel: workgroup b arrives on counter
// b % kArriveGroups, and the last arrival of each group on ctrl->arrive, so
// that no single address takes one atomic per workgroup.  They live after the
// residual partials: [G][5] doubles, 16 doubles of slack, then the counters.
constexpr int kArriveGroups = 32;
__host__ __device__ constexpr size_t step_partials_doubles(size_t G) { return G * 5 + 16 + kArriveGroups / 2; }

// Residual sums of a workgroup -> global partials; the last workgroup reduces
// them and writes the control block.  All threads of the block must call it.
template <int NT>
__device__ __forceinline__ void finish_iteration(const double (&s)[5], double* partials, Ctrl* ctrl,
                                                 double* hist, int hist_cap, long long t,
                                                 double rho, double eps_rel, const RhoRule& rule) {
    unsigned* grp = reinterpret_cast<unsigned*>(partials + (size_t)gridDim.x * 5 + 16);
    __shared__ double red[NT / 64][5];
    __shared__ int is_last;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double r[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) r[i] = wave_total(s[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 5; ++i) red[wv][i] = r[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b[5] = {0, 0, 0, 0, 0};
        for (int w = 0; w < NT / 64; ++w)
#pragma unroll
            for (int i = 0; i < 5; ++i) b[i] += red[w][i];
        // write-through (agent-scope) stores, then wait for them to complete
        // before arriving; an agent-scope fence would write back the L2 instead
#pragma unroll
        for (int i = 0; i < 5; ++i)
            __hip_atomic_store(&partials[(size_t)blockIdx.x * 5 + i], b[i], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const unsigned ng = gridDim.x < (unsigned)kArriveGroups ? gridDim.x : (unsigned)kArriveGroups;
        const unsigned gi = blockIdx.x % ng;
        const unsigned in_group = (gridDim.x - gi + ng - 1) / ng;
        const unsigned og = __hip_atomic_fetch_add(&grp[gi], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int last = 0;
        if (og == in_group - 1) {
            // last of its group: every member's partials are complete; the
            // counter returns to 0 for the next iteration (a later launch)
            __hip_atomic_store(&grp[gi], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned old = __hip_atomic_fetch_add(&ctrl->arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = (old == ng - 1);
        }
        is_last = last;
    }
    __syncthreads();
    if (!is_last) return;
    double a[5] = {0, 0, 0, 0, 0};
    for (unsigned bidx = threadIdx.x; bidx < gridDim.x; bidx += NT)
#pragma unroll
        for (int i = 0; i < 5; ++i)
            a[i] += __hip_atomic_load(&partials[(size_t)bidx * 5 + i], __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int i = 0; i < 5; ++i) a[i] = wave_total(a[i]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 5; ++i) red[wv][i] = a[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        double S[5] = {0, 0, 0, 0, 0};
        for (int w = 0; w < NT / 64; ++w)
#pragma unroll
            for (int i = 0; i < 5; ++i) S[i] += red[w][i];
        const double pres = sqrt(S[0]);
        const double dres = rho * sqrt(S[1]);
        const double ep = eps_rel * fmax(sqrt(S[2]), sqrt(S[3]));
        const double ed = eps_rel * sqrt(S[4]);
        if (t - 1 < hist_cap) {
            hist[(t - 1) * 4 + 0] = pres;
            hist[(t - 1) * 4 + 1] = dres;
            hist[(t - 1) * 4 + 2] = ep;
            hist[(t - 1) * 4 + 3] = ed;
        }
        ctrl->res[0] = pres;
        ctrl->res[1] = dres;
        ctrl->res[2] = ep;
        ctrl->res[3] = ed;
        ctrl->iter = t;
        int stop = 0, status = OPF_OK;
        if (!(isfinite(pres) && isfinite(dres) && isfinite(ep) && isfinite(ed))) {
            stop = 1;
            status = OPF_ENUMERIC;
        } else if (ctrl->check && pres <= ep && dres <= ed) {
            stop = 1;
            status = OPF_OK;
        } else if (t >= ctrl->max_iter) {
            stop = 1;
            status = ctrl->check ? OPF_NOT_CONVERGED : OPF_OK;
        }
        ctrl->status = status;
        ctrl->stop = stop;
        ctrl->arrive = 0u;
        if (rule.every)
            ctrl->rho[(t + kRhoLag) % kRhoRing] =
                rho_decide(rule, ctrl->rho[(t + kRhoLag - 1) % kRhoRing], t, pres, dres, ep, ed);
    }
}

// One ADMM iteration (global + local + dual + residual sums).  Workgroup =
// WPB wavefronts; wavefront w of the grid processes packed wave w.
template <typename T, int WPB>
__global__ __launch_bounds__(WPB * 64) void admm_step_kernel(IterArgs<T> a) {
    Ctrl* ctrl = a.ctrl;
    if (ctrl->stop) return;
    const long long t = ctrl->iter + 1;
    const bool odd = (t & 1) != 0;                 // write buffer 1 on odd t
    const T* zp = odd ? a.z0 : a.z1;
    const T* lp = odd ? a.l0 : a.l1;
    T* zq = odd ? a.z1 : a.z0;
    T* lq = odd ? a.l1 : a.l0;
    T* xq = odd ? a.x1 : a.x0;
    // penalty of this iteration (residual balancing: from the control block)
    T rho = a.rho, inv_rho = a.inv_rho;
    double rho_d = a.rho_d;
    if (a.rule.every) {
        rho_d = ctrl->rho[t % kRhoRing];
        rho = (T)(a.local_updates * rho_d);
        inv_rho = (T)(1.0 / rho_d);
    }

    __shared__ T vsh[WPB][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int w = blockIdx.x * WPB + wv;
    const int d = w * 64 + lane;
    int g = -1, meta = 0;
    T xg = 0, zold = 0, lold = 0;
    if (w < a.waves) {
        g = a.var[d];
        if (g >= 0) {
            meta = a.meta[d];
            const int cs = a.cstart[d], cn = a.ccnt[d];
            T acc = 0;
            for (int k = 0; k < cn; ++k) {
                const int e = a.clist[cs + k];
                acc += copy_term(zp[e], lp[e], inv_rho);
            }
            xg = consensus_value(acc, a.cost[d], inv_rho, cn, a.lo[d], a.hi[d]);
            zold = zp[d];
            lold = lp[d];
        }
        vsh[wv][lane] = (g >= 0) ? projection_input(xg, lold, inv_rho) : (T)0;
    }
    __syncthreads();
    double s[5] = {0, 0, 0, 0, 0};
    if (w < a.waves && g >= 0) {
        const int2 wi = a.winfo[w];
        const T* Fw = a.F + (size_t)wi.y * 64;
        const int base = meta & 255;
        const T zn = project_row(Fw, vsh[wv], base, lane, wi.x, a.bbar[d]);
        const T ln = dual_step(lold, rho, xg, zn);
        zq[d] = zn;
        lq[d] = ln;
        if (meta & (1 << 16)) xq[g] = xg;
        const double xd = (double)xg, zd = (double)zn;
        s[0] = (xd - zd) * (xd - zd);
        s[1] = (zd - (double)zold) * (zd - (double)zold);
        s[2] = xd * xd;
        s[3] = zd * zd;
        s[4] = (double)ln * (double)ln;
    }
    finish_iteration<WPB * 64>(s, a.partials, ctrl, a.hist, a.hist_cap, t, rho_d, a.eps_rel, a.rule);
}

// Initial state: buffer 0 holds the start point (z0, lambda0) in device order.
template <typename T>
__global__ void init_state_kernel(const double* z0, const double* lam0, T* z, T* l, int LP,
                                  Ctrl* ctrl, long long max_iter, int check, double rho0) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d < LP) {
        z[d] = (T)z0[d];
        l[d] = lam0 ? (T)lam0[d] : (T)0;
    }
    if (d == 0) {
        ctrl->iter = 0;
        ctrl->max_iter = max_iter;
        ctrl->stop = 0;
        ctrl->status = OPF_OK;
        ctrl->check = check;
        ctrl->arrive = 0u;
        ctrl->res[0] = ctrl->res[1] = ctrl->res[2] = ctrl->res[3] = 0.0;
        for (int k = 0; k < kRhoRing; ++k) ctrl->rho[k] = rho0;
    }
}

// FP32 -> FP64 hand-over of the state at the last completed iteration (polish).
__global__ void promote_state_kernel(const float* z32a, const float* z32b, const float* l32a,
                                     const float* l32b, double* z64a, double* z64b, double* l64a,
                                     double* l64b, int LP, Ctrl* ctrl, long long max_iter) {
    const long long t = ctrl->iter;
    const bool odd = (t & 1) != 0;
    const float* zs = odd ? z32b : z32a;
    const float* ls = odd ? l32b : l32a;
    double* zd = odd ? z64b : z64a;
    double* ld = odd ? l64b : l64a;
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d < LP) {
        zd[d] = (double)zs[d];
        ld[d] = (double)ls[d];
    }
}

// Re-arms the control block for another phase (after promote_state_kernel).
__global__ void rearm_kernel(Ctrl* ctrl, long long max_iter, int check) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctrl->max_iter = max_iter;
        ctrl->stop = 0;
        ctrl->status = OPF_OK;
        ctrl->check = check;
        ctrl->arrive = 0u;
    }
}

// Outputs in user order and in FP64; objective c^T x by one workgroup.
template <typename T>
__global__ void output_kernel(const T* z0, const T* z1, const T* l0, const T* l1, const T* x0,
                              const T* x1, const int* user_slot, int LP, int n, const double* c,
                              double* xo, double* zo, double* lo, Ctrl* ctrl) {
    const long long t = ctrl->iter;
    const bool odd = (t & 1) != 0;
    const T* zs = odd ? z1 : z0;
    const T* ls = odd ? l1 : l0;
    const T* xs = odd ? x1 : x0;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nth = gridDim.x * blockDim.x;
    for (int d = gid; d < LP; d += nth) {
        const int u = user_slot[d];
        if (u >= 0) {
            if (zo) zo[u] = (double)zs[d];
            if (lo) lo[u] = (double)ls[d];
        }
    }
    for (int i = gid; i < n; i += nth) xo[i] = (double)xs[i];
}

__global__ void objective_kernel(const double* x, const double* c, int n, Ctrl* ctrl) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += c[i] * x[i];
    s = wave_sum(s);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) a += red[w];
        ctrl->objective = a;
    }
}

// ---- launch helpers (host) -------------------------------------------------

template <typename T>
hipError_t launch_step(const IterArgs<T>& a, int wpb, hipStream_t st) {
    const int grid_w = wpb;
    const int blocks = (a.waves + grid_w - 1) / grid_w;
    switch (wpb) {
        case 1: hipLaunchKernelGGL((admm_step_kernel<T, 1>), dim3(blocks), dim3(64), 0, st, a); break;
        case 2: hipLaunchKernelGGL((admm_step_kernel<T, 2>), dim3(blocks), dim3(128), 0, st, a); break;
        case 8: hipLaunchKernelGGL((admm_step_kernel<T, 8>), dim3(blocks), dim3(512), 0, st, a); break;
        default: hipLaunchKernelGGL((admm_step_kernel<T, 4>), dim3(blocks), dim3(256), 0, st, a); break;
    }
    return hipGetLastError();
}

template hipError_t launch_step<double>(const IterArgs<double>&, int, hipStream_t);
template hipError_t launch_step<float>(const IterArgs<float>&, int, hipStream_t);

template <typename T>
hipError_t launch_init(const double* z0, const double* lam0, T* z, T* l, int LP, Ctrl* ctrl,
                       long long max_iter, int check, double rho0, hipStream_t st) {
    hipLaunchKernelGGL((init_state_kernel<T>), dim3((LP + 255) / 256), dim3(256), 0, st, z0, lam0, z, l,
                       LP, ctrl, max_iter, check, rho0);
    return hipGetLastError();
}
template hipError_t launch_init<double>(const double*, const double*, double*, double*, int, Ctrl*,
                                        long long, int, double, hipStream_t);
template hipError_t launch_init<float>(const double*, const double*, float*, float*, int, Ctrl*,
                                       long long, int, double, hipStream_t);

hipError_t launch_promote(const float* z32a, const float* z32b, const float* l32a, const float* l32b,
                          double* z64a, double* z64b, double* l64a, double* l64b, int LP, Ctrl* ctrl,
                          long long max_iter, int check, hipStream_t st) {
    hipLaunchKernelGGL(promote_state_kernel, dim3((LP + 255) / 256), dim3(256), 0, st, z32a, z32b, l32a,
                       l32b, z64a, z64b, l64a, l64b, LP, ctrl, max_iter);
    hipLaunchKernelGGL(rearm_kernel, dim3(1), dim3(64), 0, st, ctrl, max_iter, check);
    return hipGetLastError();
}

size_t step_partials_count(int G) { return step_partials_doubles((size_t)G); }

hipError_t launch_rearm(Ctrl* ctrl, long long max_iter, int check, hipStream_t st) {
    hipLaunchKernelGGL(rearm_kernel, dim3(1), dim3(64), 0, st, ctrl, max_iter, check);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_output(const T* z0, const T* z1, const T* l0, const T* l1, const T* x0, const T* x1,
                         const int* user_slot, int LP, int n, const double* c, double* xo, double* zo,
                         double* lo, Ctrl* ctrl, hipStream_t st) {
    hipLaunchKernelGGL((output_kernel<T>), dim3(256), dim3(256), 0, st, z0, z1, l0, l1, x0, x1, user_slot,
                       LP, n, c, xo, zo, lo, ctrl);
    hipLaunchKernelGGL(objective_kernel, dim3(1), dim3(1024), 0, st, xo, c, n, ctrl);
    return hipGetLastError();
}
template hipError_t launch_output<double>(const double*, const double*, const double*, const double*,
                                          const double*, const double*, const int*, int, int,
                                          const double*, double*, double*, double*, Ctrl*, hipStream_t);
template hipError_t launch_output<float>(const float*, const float*, const float*, const float*,
                                         const float*, const float*, const int*, int, int, const double*,
                                         double*, double*, double*, Ctrl*, hipStream_t);

}  // namespace opf
