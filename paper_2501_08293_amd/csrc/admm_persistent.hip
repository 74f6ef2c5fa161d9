// Persistent form of the fused ADMM iteration for gfx950: one cooperative
// launch runs every iteration of Algorithm 1 until the termination test holds.
//
// Work split: workgroup b owns `WPB` packed wavefronts (a contiguous run of the
// component graph) and keeps its slots' static data and its own local copy
// and dual in registers across iterations.  Synchronisation is local:
//   * before iteration t+1, workgroup b waits until every workgroup owning a
//     copy of one of its variables ("neighbour") has published iteration t
//     (a per-workgroup iteration flag);
//   * the stacked z and lambda live in two buffers (iteration parity); a
//     neighbour has finished reading buffer (t-1)&1 once it publishes t, so
//     writing buffer (t+1)&1 is safe after the same wait;
//   * every workgroup publishes its residual partial sums of iteration t with
//     its flag; one extra workgroup (the reducer, the last of the grid) waits
//     for all flags to reach t, reduces the partials in a fixed order and
//     publishes the stop decision for t.  Workgroups consult it one iteration
//     later (before starting t+2), so the reduction is hidden behind
//     iteration t+1, whose writes go to the other buffer and leave the state
//     of t intact.  No read-modify-write atomics are on the compute path.
// Cross-workgroup data moves through agent-scope atomic loads and stores
// (coherent across the chip's L2 slices without write-back fences); ordering
// between a workgroup's data stores and its flag store is an explicit wait for
// outstanding memory operations followed by a workgroup barrier.
// Every wait is bounded: a wait that runs out sets OPF_EHANG and every
// workgroup leaves the loop, so the grid always drains.
#include "admm_kernels.h"

#include "../../include/opf_admm.h"

namespace opf {

template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until every memory operation this thread issued has completed.
__device__ __forceinline__ void drain_memory() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ double wave_sum_p(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kCopyRegs = 8;
constexpr int kBatch = 8;      // loads the reducer keeps in flight per thread

// Reducer workgroup: decision of every iteration from the published partials.
template <int NT>
__device__ void reducer_loop(const IterArgs<double>& ad, Ctrl* ctrl, const PersistArgs& p, int G,
                             long long t0, double rho, double eps_rel, double* hist, int hist_cap) {
    __shared__ double rred[NT / 64][5];
    __shared__ int rstop;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    (void)ad;
    long long t = t0;
    for (;;) {
        const long long tn = t + 1;
        long long spins = 0;
        for (;;) {
            // up to kBatch flags per thread in flight at once
            int mine = 1;
            for (int q0 = threadIdx.x; q0 < G; q0 += kBatch * NT) {
                long long f[kBatch];
#pragma unroll
                for (int k = 0; k < kBatch; ++k) {
                    const int q = q0 + k * NT;
                    f[k] = q < G ? ld_agent(&p.flags[q]) : tn;
                }
#pragma unroll
                for (int k = 0; k < kBatch; ++k) mine &= (f[k] >= tn);
            }
            if (__syncthreads_and(mine)) break;
            int bad = 0;
            if (threadIdx.x == 0) bad = (ld_agent(p.error) != 0) || (++spins > p.spin_limit);
            if (__syncthreads_or(bad)) {
                if (threadIdx.x == 0) st_agent(p.error, (int)OPF_EHANG);
                return;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        const int par = (int)(tn & 1);
        double acc5[5] = {0, 0, 0, 0, 0};
        for (int q0 = threadIdx.x; q0 < G; q0 += kBatch * NT) {
            double v[kBatch][5];
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int q = q0 + k * NT;
                const double* pp = p.partials + ((size_t)par * G + (q < G ? q : 0)) * 5;
#pragma unroll
                for (int i = 0; i < 5; ++i) v[k][i] = q < G ? ld_agent(&pp[i]) : 0.0;
            }
            // same summation order as a plain strided loop over q
#pragma unroll
            for (int k = 0; k < kBatch; ++k)
#pragma unroll
                for (int i = 0; i < 5; ++i)
                    if (q0 + k * NT < G) acc5[i] += v[k][i];
        }
#pragma unroll
        for (int i = 0; i < 5; ++i) acc5[i] = wave_sum_p(acc5[i]);
        if (lane == 0)
#pragma unroll
            for (int i = 0; i < 5; ++i) rred[wv][i] = acc5[i];
        __syncthreads();
        if (threadIdx.x == 0) {
            double S[5] = {0, 0, 0, 0, 0};
            for (int q = 0; q < NT / 64; ++q)
#pragma unroll
                for (int i = 0; i < 5; ++i) S[i] += rred[q][i];
            const double pres = sqrt(S[0]);
            const double dres = rho * sqrt(S[1]);
            const double ep = eps_rel * fmax(sqrt(S[2]), sqrt(S[3]));
            const double ed = eps_rel * sqrt(S[4]);
            if (tn - 1 < hist_cap) {
                hist[(tn - 1) * 4 + 0] = pres;
                hist[(tn - 1) * 4 + 1] = dres;
                hist[(tn - 1) * 4 + 2] = ep;
                hist[(tn - 1) * 4 + 3] = ed;
            }
            int stop = 0, status = OPF_OK;
            if (!(isfinite(pres) && isfinite(dres) && isfinite(ep) && isfinite(ed))) {
                stop = 1;
                status = OPF_ENUMERIC;
            } else if (p.check && pres <= ep && dres <= ed) {
                stop = 1;
            } else if (tn >= p.max_iter) {
                stop = 1;
                status = p.check ? OPF_NOT_CONVERGED : OPF_OK;
            }
            if (stop) {
                // the final state is that of iteration tn (buffer tn & 1)
                ctrl->iter = tn;
                ctrl->status = status;
                ctrl->res[0] = pres;
                ctrl->res[1] = dres;
                ctrl->res[2] = ep;
                ctrl->res[3] = ed;
                ctrl->stop = 1;
            }
            st_agent(&p.dec_stop[par], stop);
            drain_memory();
            st_agent(&p.dec_iter[par], tn);
            rstop = stop;
        }
        __syncthreads();
        if (rstop) return;
        t = tn;
    }
}

template <typename T, int WPB>
__global__ __launch_bounds__(WPB * 64) void admm_persistent_kernel(IterArgs<T> a, PersistArgs p) {
    constexpr int NT = WPB * 64;
    __shared__ T vsh[WPB][64];
    __shared__ double red[WPB][5];
    __shared__ int sh_flag;

    const int G = (int)gridDim.x - 1;      // compute workgroups; the last one reduces
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int b = blockIdx.x;
    Ctrl* ctrl = a.ctrl;
    const long long t0 = ctrl->iter;
    if (b == G) {
        IterArgs<double> dummy{};
        reducer_loop<NT>(dummy, ctrl, p, G, t0, a.rho_d, a.eps_rel, a.hist, a.hist_cap);
        return;
    }
    const int w = b * WPB + wv;
    const int d = w * 64 + lane;

    // ---- static per-slot data, kept in registers
    const int g = a.var[d];
    const bool live = g >= 0;
    int meta = 0, cs = 0, cn = 1;
    int cp[kCopyRegs];
    T bb = 0, lo = 0, hi = 0, cterm = 0;
    if (live) {
        meta = a.meta[d];
        cs = a.cstart[d];
        cn = a.ccnt[d];
#pragma unroll
        for (int k = 0; k < kCopyRegs; ++k) cp[k] = k < cn ? a.clist[cs + k] : d;
        bb = a.bbar[d];
        lo = a.lo[d];
        hi = a.hi[d];
        cterm = a.cost[d] * a.inv_rho;
    }
    const int2 wi = a.winfo[w];
    const T* Fw = a.F + (size_t)wi.y * 64;
    if (p.lds_factors) {
        // static factors of this workgroup's wavefronts, copied once into LDS
        extern __shared__ __align__(16) unsigned char dyn_lds[];
        T* Fl = reinterpret_cast<T*>(dyn_lds);
        int off = 0;
        for (int q = 0; q < wv; ++q) off += a.winfo[b * WPB + q].x;
        Fl += (size_t)off * 64;
        for (int k = 0; k < wi.x; ++k) Fl[k * 64 + lane] = Fw[k * 64 + lane];
        Fw = Fl;
    }
    const int base = meta & 255;
    const bool owner = (meta >> 16) & 1;
    // current local copy and dual of this slot (state of iteration t0)
    T zc = 0, lc = 0;
    if (live) {
        zc = (t0 & 1) ? a.z1[d] : a.z0[d];
        lc = (t0 & 1) ? a.l1[d] : a.l0[d];
    }
    const int nb0 = p.nbr_ptr[b], nbn = p.nbr_ptr[b + 1] - nb0;

    long long t = t0;
    for (;;) {
        const long long tn = t + 1;
        // ---- thread 0: stop decision of iteration tn - 2 (published one
        // iteration late); other threads: neighbours have published iteration t
        if (threadIdx.x == 0) {
            int stop = 0;
            if (tn - 2 > t0) {
                const int slot = (int)((tn - 2) & 1);
                long long spins = 0;
                while (ld_agent(&p.dec_iter[slot]) != tn - 2) {
                    if (ld_agent(p.error) != 0 || ++spins > p.spin_limit) {
                        st_agent(p.error, (int)OPF_EHANG);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                stop = ld_agent(&p.dec_stop[slot]);
            }
            if (ld_agent(p.error) != 0) stop = 1;
            sh_flag = stop;
        } else {
            for (int q = threadIdx.x - 1; q < nbn; q += NT - 1) {
                const int nbk = p.nbr_list[nb0 + q];
                long long spins = 0;
                while (ld_agent(&p.flags[nbk]) < t) {
                    if (ld_agent(p.error) != 0 || ++spins > p.spin_limit) {
                        st_agent(p.error, (int)OPF_EHANG);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
        }
        __syncthreads();
        if (sh_flag) break;
        // ---- global update for this slot's variable (all copies, fixed order)
        const bool odd = (tn & 1) != 0;
        const T* zp = odd ? a.z0 : a.z1;
        const T* lp = odd ? a.l0 : a.l1;
        T* zq = odd ? a.z1 : a.z0;
        T* lq = odd ? a.l1 : a.l0;
        T* xq = odd ? a.x1 : a.x0;
        T xg = 0;
        if (live) {
            T acc = 0;
#pragma unroll
            for (int k = 0; k < kCopyRegs; ++k) {
                if (k < cn) {
                    const int e = cp[k];
                    const T ze = (e == d) ? zc : ld_agent(&zp[e]);
                    const T le = (e == d) ? lc : ld_agent(&lp[e]);
                    acc += ze - le * a.inv_rho;
                }
            }
            for (int k = kCopyRegs; k < cn; ++k) {
                const int e = a.clist[cs + k];
                acc += ld_agent(&zp[e]) - ld_agent(&lp[e]) * a.inv_rho;
            }
            const T xh = (acc - cterm) / (T)cn;
            xg = xh < lo ? lo : (xh > hi ? hi : xh);
        }
        vsh[wv][lane] = live ? xg + lc * a.inv_rho : (T)0;
        __syncthreads();
        // ---- local projection, dual update, residual terms
        double s[5] = {0, 0, 0, 0, 0};
        if (live) {
            T acc = bb;
            for (int k = 0; k < wi.x; ++k) acc += Fw[k * 64 + lane] * vsh[wv][(base + k) & 63];
            const T zn = acc;
            const T ln = lc + a.rho * (xg - zn);
            st_agent(&zq[d], zn);
            st_agent(&lq[d], ln);
            if (owner) xq[g] = xg;
            const double xd = (double)xg, zd = (double)zn;
            s[0] = (xd - zd) * (xd - zd);
            s[1] = (zd - (double)zc) * (zd - (double)zc);
            s[2] = xd * xd;
            s[3] = zd * zd;
            s[4] = (double)ln * (double)ln;
            zc = zn;
            lc = ln;
        }
        // ---- workgroup residual partial, then publish iteration tn
#pragma unroll
        for (int i = 0; i < 5; ++i) s[i] = wave_sum_p(s[i]);
        if (lane == 0)
#pragma unroll
            for (int i = 0; i < 5; ++i) red[wv][i] = s[i];
        __syncthreads();
        if (threadIdx.x == 0) {
            double bsum[5] = {0, 0, 0, 0, 0};
            for (int q = 0; q < WPB; ++q)
#pragma unroll
                for (int i = 0; i < 5; ++i) bsum[i] += red[q][i];
            double* pp = p.partials + ((size_t)(tn & 1) * G + b) * 5;
#pragma unroll
            for (int i = 0; i < 5; ++i) st_agent(&pp[i], bsum[i]);
        }
        drain_memory();          // this thread's z / lambda (and partial) stores are complete
        __syncthreads();
        if (threadIdx.x == 0) st_agent(&p.flags[b], tn);   // state and partials of tn are visible
        t = tn;
    }
}

template <typename T>
__global__ void persistent_prepare_kernel(PersistArgs p, int G, Ctrl* ctrl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const long long t0 = ctrl->iter;
    if (i < G) p.flags[i] = t0;
    if (i < 2) {
        p.arrive[i] = 0u;
        p.dec_iter[i] = -1;
        p.dec_stop[i] = 0;
    }
    if (i == 0) {
        *p.error = 0;
        *p.stopped = 0;
    }
}

template <typename T>
hipError_t launch_persistent(const IterArgs<T>& a, PersistArgs p, int wpb, int G, hipStream_t st) {
    const size_t lds = p.lds_factors ? (size_t)p.lds_factor_cols * 64 * sizeof(T) : 0;
    hipLaunchKernelGGL((persistent_prepare_kernel<T>), dim3((G + 255) / 256), dim3(256), 0, st, p, G, a.ctrl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* args[] = {(void*)&a, (void*)&p};
    switch (wpb) {
        case 1: return hipLaunchCooperativeKernel((const void*)admm_persistent_kernel<T, 1>, dim3(G + 1), dim3(64), args, lds, st);
        case 2: return hipLaunchCooperativeKernel((const void*)admm_persistent_kernel<T, 2>, dim3(G + 1), dim3(128), args, lds, st);
        case 8: return hipLaunchCooperativeKernel((const void*)admm_persistent_kernel<T, 8>, dim3(G + 1), dim3(512), args, lds, st);
        default: return hipLaunchCooperativeKernel((const void*)admm_persistent_kernel<T, 4>, dim3(G + 1), dim3(256), args, lds, st);
    }
}
template hipError_t launch_persistent<double>(const IterArgs<double>&, PersistArgs, int, int, hipStream_t);
template hipError_t launch_persistent<float>(const IterArgs<float>&, PersistArgs, int, int, hipStream_t);

// Largest co-resident grid for the persistent kernel (0 on error); the grid
// holds one workgroup more than the compute workgroups (the reducer).
template <typename T>
int persistent_capacity(int wpb, size_t lds_bytes) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e;
    switch (wpb) {
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, admm_persistent_kernel<T, 1>, 64, lds_bytes); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, admm_persistent_kernel<T, 2>, 128, lds_bytes); break;
        case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, admm_persistent_kernel<T, 8>, 512, lds_bytes); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, admm_persistent_kernel<T, 4>, 256, lds_bytes); break;
    }
    if (e != hipSuccess) return 0;
    return per * cus;
}
template int persistent_capacity<double>(int, size_t);
template int persistent_capacity<float>(int, size_t);

}  // namespace opf
