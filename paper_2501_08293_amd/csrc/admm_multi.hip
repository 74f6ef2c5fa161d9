// Per-solve helper kernels of the serving runtime (gfx950): start state,
// warm-start gathers, outputs.  The shared iteration itself is the persistent
// serving kernel (admm_persistent.hip).
#include "admm_kernels.h"

#include "../../include/opf_admm.h"

namespace opf {

// Control block of one instance reset for a new solve; with `narrow` the FP32
// start state of the bulk phase is rounded from the FP64 start state.
__global__ void multi_init_kernel(InstDesc* descs, int slot, long long max_iter, int narrow) {
    InstDesc& D = descs[slot];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (narrow && i < D.lanes) {
        D.z0f[i] = (float)D.z0[i];
        D.l0f[i] = (float)D.l0[i];
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

template <typename T>
__device__ void write_outputs(const InstDesc& D, const T* z0, const T* z1, const T* l0, const T* l1, const T* x0,
                              const T* x1, double* xo, double* zo, double* lo) {
    const long long t = D.ctrl->iter;
    const bool odd = (t & 1) != 0;
    const T* zs = odd ? z1 : z0;
    const T* ls = odd ? l1 : l0;
    const T* xs = odd ? x1 : x0;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x, nth = gridDim.x * blockDim.x;
    for (int d = gid; d < D.lanes; d += nth) {
        const int u = D.user_slot[d];
        if (u >= 0) {
            zo[u] = (double)zs[d];
            lo[u] = (double)ls[d];
        }
    }
    for (int i = gid; i < D.n; i += nth) xo[i] = (double)xs[i];
}

// Outputs of a finished instance in user order: x, and z / lambda (kept for
// warm starts of later solves of the same feeder family).
__global__ void multi_output_kernel(const InstDesc* descs, int slot, double* xo, double* zo, double* lo, int fp32) {
    const InstDesc& D = descs[slot];
    if (fp32) write_outputs<float>(D, D.z0f, D.z1f, D.l0f, D.l1f, D.x0f, D.x1f, xo, zo, lo);
    else write_outputs<double>(D, D.z0, D.z1, D.l0, D.l1, D.x0, D.x1, xo, zo, lo);
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

hipError_t launch_multi_init(InstDesc* descs, int slot, int lanes, long long max_iter, int narrow, hipStream_t st) {
    hipLaunchKernelGGL(multi_init_kernel, dim3((lanes + 255) / 256), dim3(256), 0, st, descs, slot, max_iter, narrow);
    return hipGetLastError();
}

hipError_t launch_multi_output(const InstDesc* descs, int slot, double* xo, double* zo, double* lo, int fp32,
                               hipStream_t st) {
    hipLaunchKernelGGL(multi_output_kernel, dim3(64), dim3(256), 0, st, descs, slot, xo, zo, lo, fp32);
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
