// Multi-instance fused iteration for the serving runtime (gfx950).
//
// Independent solves of different sizes share one launch: the launch's
// workgroups are dealt out by a device work list of (instance slot, local
// workgroup) pairs, and each instance keeps its own iteration counter,
// ping-pong parity, residual reduction and stop decision in its descriptor.
// The arithmetic of an instance is exactly that of the single-instance step
// kernel (same slot order, same reduction order), so a solve returns the same
// bits alone and in any mix.  The launch has a fixed grid; workgroups past
// the current work list return at once, so one captured graph serves every
// membership of the mix.
#include "admm_kernels.h"

#include "../../include/opf_admm.h"

namespace opf {

__device__ __forceinline__ double wave_sum_m(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int WPB>
__global__ __launch_bounds__(WPB * 64) void admm_multi_step_kernel(const InstDesc* __restrict__ descs,
                                                                   const int2* __restrict__ work,
                                                                   const int* __restrict__ nwork) {
    constexpr int NT = WPB * 64;
    if ((int)blockIdx.x >= *nwork) return;
    const int2 wk = work[blockIdx.x];
    const InstDesc& D = descs[wk.x];
    Ctrl* ctrl = D.ctrl;
    if (ctrl->stop) return;
    const long long t = ctrl->iter + 1;
    const bool odd = (t & 1) != 0;
    const double* zp = odd ? D.z0 : D.z1;
    const double* lp = odd ? D.l0 : D.l1;
    double* zq = odd ? D.z1 : D.z0;
    double* lq = odd ? D.l1 : D.l0;
    double* xq = odd ? D.x1 : D.x0;
    const double rho = D.rho, inv_rho = 1.0 / D.rho;

    __shared__ double vsh[WPB][64];
    __shared__ double red[WPB][5];
    __shared__ int is_last;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int w = wk.y * WPB + wv;           // wavefront inside the instance
    const int d = w * 64 + lane;
    int g = -1, meta = 0;
    double xg = 0, zold = 0, lold = 0;
    g = D.var[d];
    if (g >= 0) {
        meta = D.meta[d];
        const int cs = D.cstart[d], cn = D.ccnt[d];
        double acc = 0;
        for (int k = 0; k < cn; ++k) {
            const int e = D.clist[cs + k];
            acc += zp[e] - lp[e] * inv_rho;
        }
        const double xh = (acc - D.cost[d] * inv_rho) / (double)cn;
        xg = xh < D.lo[d] ? D.lo[d] : (xh > D.hi[d] ? D.hi[d] : xh);
        zold = zp[d];
        lold = lp[d];
    }
    vsh[wv][lane] = (g >= 0) ? xg + lold * inv_rho : 0.0;
    __syncthreads();
    double s[5] = {0, 0, 0, 0, 0};
    if (g >= 0) {
        const int2 wi = D.winfo[w];
        const double* Fw = D.F + (size_t)wi.y * 64;
        const int base = meta & 255;
        double acc = D.bbar[d];
        for (int k = 0; k < wi.x; ++k) acc += Fw[k * 64 + lane] * vsh[wv][(base + k) & 63];
        const double zn = acc;
        const double ln = lold + rho * (xg - zn);
        zq[d] = zn;
        lq[d] = ln;
        if (meta & (1 << 16)) xq[g] = xg;
        s[0] = (xg - zn) * (xg - zn);
        s[1] = (zn - zold) * (zn - zold);
        s[2] = xg * xg;
        s[3] = zn * zn;
        s[4] = ln * ln;
    }
    // ---- residual partial of this workgroup; the instance's last workgroup decides
#pragma unroll
    for (int i = 0; i < 5; ++i) s[i] = wave_sum_m(s[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 5; ++i) red[wv][i] = s[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        double b[5] = {0, 0, 0, 0, 0};
        for (int q = 0; q < WPB; ++q)
#pragma unroll
            for (int i = 0; i < 5; ++i) b[i] += red[q][i];
#pragma unroll
        for (int i = 0; i < 5; ++i)
            __hip_atomic_store(&D.partials[(size_t)wk.y * 5 + i], b[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const unsigned old = __hip_atomic_fetch_add(&ctrl->arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        is_last = (old == (unsigned)D.blocks - 1);
    }
    __syncthreads();
    if (!is_last) return;
    double a[5] = {0, 0, 0, 0, 0};
    for (int q = threadIdx.x; q < D.blocks; q += NT)
#pragma unroll
        for (int i = 0; i < 5; ++i)
            a[i] += __hip_atomic_load(&D.partials[(size_t)q * 5 + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int i = 0; i < 5; ++i) a[i] = wave_sum_m(a[i]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 5; ++i) red[wv][i] = a[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        double S[5] = {0, 0, 0, 0, 0};
        for (int q = 0; q < WPB; ++q)
#pragma unroll
            for (int i = 0; i < 5; ++i) S[i] += red[q][i];
        const double pres = sqrt(S[0]);
        const double dres = rho * sqrt(S[1]);
        const double ep = D.eps_rel * fmax(sqrt(S[2]), sqrt(S[3]));
        const double ed = D.eps_rel * sqrt(S[4]);
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
        } else if (t >= ctrl->max_iter) {
            stop = 1;
            status = ctrl->check ? OPF_NOT_CONVERGED : OPF_OK;
        }
        ctrl->status = status;
        ctrl->stop = stop;
        ctrl->arrive = 0u;
    }
}

// Start state of one instance: z from (default start or warm values) in device
// order, lambda likewise, control block reset.
__global__ void multi_init_kernel(InstDesc* descs, int slot, const double* z0, const double* l0, long long max_iter) {
    InstDesc& D = descs[slot];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < D.lanes && z0) {
        D.z0[i] = z0[i];
        D.l0[i] = l0 ? l0[i] : 0.0;
    }
    if (i == 0) {
        D.ctrl->iter = 0;
        D.ctrl->max_iter = max_iter;
        D.ctrl->stop = 0;
        D.ctrl->status = OPF_OK;
        D.ctrl->check = 1;
        D.ctrl->arrive = 0u;
    }
}

// Outputs of a finished instance in user order: x, and z / lambda (kept for
// warm starts of later solves of the same feeder family).
__global__ void multi_output_kernel(const InstDesc* descs, int slot, double* xo, double* zo, double* lo) {
    const InstDesc& D = descs[slot];
    const long long t = D.ctrl->iter;
    const bool odd = (t & 1) != 0;
    const double* zs = odd ? D.z1 : D.z0;
    const double* ls = odd ? D.l1 : D.l0;
    const double* xs = odd ? D.x1 : D.x0;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x, nth = gridDim.x * blockDim.x;
    for (int d = gid; d < D.lanes; d += nth) {
        const int u = D.user_slot[d];
        if (u >= 0) {
            zo[u] = zs[d];
            lo[u] = ls[d];
        }
    }
    for (int i = gid; i < D.n; i += nth) xo[i] = xs[i];
}

// Copies warm-start values of matching components: for each pair
// (src user offset, dst user offset, length) of `plan`, z/lambda of the
// resident state go to the new instance's start vectors (user order).
__global__ void warm_gather_kernel(const int4* plan, int nplan, const double* rz, const double* rl, double* zu,
                                   double* lu) {
    const int p = blockIdx.x;
    if (p >= nplan) return;
    const int4 e = plan[p];
    for (int j = threadIdx.x; j < e.z; j += blockDim.x) {
        zu[e.y + j] = rz[e.x + j];
        lu[e.y + j] = rl[e.x + j];
    }
}

// user order -> device order for the start vectors; padding lanes get 0
__global__ void to_device_order_kernel(const double* zu, const double* lu, const int* user_slot, int lanes,
                                       const double* zdef, double* zd, double* ld, int use_warm) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= lanes) return;
    const int u = user_slot[d];
    if (u < 0) {
        zd[d] = 0.0;
        ld[d] = 0.0;
    } else if (use_warm) {
        zd[d] = zu[u];
        ld[d] = lu[u];
    } else {
        zd[d] = zdef[d];
        ld[d] = 0.0;
    }
}

hipError_t launch_multi_step(const InstDesc* descs, const int2* work, const int* nwork, int grid, int wpb,
                             hipStream_t st) {
    switch (wpb) {
        case 1: hipLaunchKernelGGL(admm_multi_step_kernel<1>, dim3(grid), dim3(64), 0, st, descs, work, nwork); break;
        case 2: hipLaunchKernelGGL(admm_multi_step_kernel<2>, dim3(grid), dim3(128), 0, st, descs, work, nwork); break;
        default: hipLaunchKernelGGL(admm_multi_step_kernel<4>, dim3(grid), dim3(256), 0, st, descs, work, nwork); break;
    }
    return hipGetLastError();
}

hipError_t launch_multi_init(InstDesc* descs, int slot, int lanes, const double* z0, const double* l0,
                             long long max_iter, hipStream_t st) {
    hipLaunchKernelGGL(multi_init_kernel, dim3((lanes + 255) / 256), dim3(256), 0, st, descs, slot, z0, l0, max_iter);
    return hipGetLastError();
}

hipError_t launch_multi_output(const InstDesc* descs, int slot, double* xo, double* zo, double* lo,
                               hipStream_t st) {
    hipLaunchKernelGGL(multi_output_kernel, dim3(64), dim3(256), 0, st, descs, slot, xo, zo, lo);
    return hipGetLastError();
}

hipError_t launch_warm_gather(const int4* plan, int nplan, const double* rz, const double* rl, double* zu,
                              double* lu, hipStream_t st) {
    if (nplan > 0) hipLaunchKernelGGL(warm_gather_kernel, dim3(nplan), dim3(64), 0, st, plan, nplan, rz, rl, zu, lu);
    return hipGetLastError();
}

hipError_t launch_to_device_order(const double* zu, const double* lu, const int* user_slot, int lanes,
                                  const double* zdef, double* zd, double* ld, int use_warm, hipStream_t st) {
    hipLaunchKernelGGL(to_device_order_kernel, dim3((lanes + 255) / 256), dim3(256), 0, st, zu, lu, user_slot, lanes,
                       zdef, zd, ld, use_warm);
    return hipGetLastError();
}

}  // namespace opf
