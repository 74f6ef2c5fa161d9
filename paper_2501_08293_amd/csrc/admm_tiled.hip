// Tiled persistent schedule of the fused ADMM iteration for gfx950 (see the
// kernel's comment): for packings with more workgroup tiles than the device
// holds at once.
#include <algorithm>

#include "admm_kernels.h"
#include "admm_sync.h"

#include "../../include/opf_admm.h"

namespace opf {

template <typename T>
hipError_t launch_prepare(const IterArgs<T>& a, PersistArgs p, int G, hipStream_t st);

// Tiled persistent schedule, for packings with more workgroups than the device
// holds at once: G compute workgroups (and the reducer) share the `tiles`
// workgroup tiles of the packing, workgroup b taking tiles b, b + G, ... in
// turn every iteration.  The per-slot state lives in memory, in a ring of the
// last kStateRing iterations (a stop decision reaches the workgroups
// kDecisionLag iterations late, so the decided iteration's state must outlive
// two more), and static slot data and factors are read through the caches
// every iteration; a slot is always computed by the same thread, so the ring
// needs no synchronisation.  Exchange (tagged consensus terms), residual
// records, reducer and decisions are those of the persistent kernel.  No wait
// can deadlock: a workgroup finishes every tile of an iteration before it
// starts the next, so the slowest workgroup always finds the terms it waits for.
template <typename T, int WPB>
__global__ __launch_bounds__(WPB * 64) void admm_tiled_kernel(IterArgs<T> a, PersistArgs p, TiledArgs ta) {
    constexpr int NT = WPB * 64;
    constexpr int W = Tag<T>::W;
    constexpr int LAG = kDecisionLag;
    const int G = (int)gridDim.x - 1;
    const int b = (int)blockIdx.x;
    int* error = p.error;
    Ctrl* ctrl = a.ctrl;
    const long long t0 = ctrl->iter;
    if (b == G) {
        const InstanceView<T> v = view_of(a, p);
        reducer_loop<T, NT, false>(v, G, t0, error, p.spin_limit);
        return;
    }
    __shared__ T vsh[WPB][64];
    __shared__ double red[WPB][5];
    __shared__ int sh_flag;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const size_t LP = (size_t)a.waves * 64;
    T* zr = static_cast<T*>(ta.zr);
    T* lr = static_cast<T*>(ta.lr);
    T* xr = static_cast<T*>(ta.xr);
    const T inv_rho = a.inv_rho, rho = a.rho;
    long long t = t0;
    for (;;) {
        const long long tn = t + 1;
        // ---- decision of iteration tn - LAG
        if (threadIdx.x == 0) {
            long long spins = 0;
            int bad = 0;
            long long dseen = ld_agent(p.dec_iter);
            int errseen = ld_agent(error);
            while (dseen < tn - LAG && !bad && !errseen) {
                __builtin_amdgcn_s_sleep(1);
                dseen = ld_agent(p.dec_iter);
                errseen = ld_agent(error);
                if (++spins > p.spin_limit) bad = 1;
            }
            int stop = 0;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);   // dec_stop is read after dec_iter
            if (!bad && !errseen && tn - LAG > t0) stop = ld_agent(p.dec_stop) == tn - LAG;
            if (bad) st_agent(error, (int)OPF_EHANG);
            sh_flag = stop | ((errseen || bad) ? 2 : 0);
        }
        __syncthreads();
        const int flag = sh_flag;
        if (flag) {
            if (flag == 1) {
                // state of the end iteration ts into the iteration-parity buffers
                const long long ts = tn - LAG;
                const size_t rs = (size_t)(ts % kStateRing);
                T* zo = (ts & 1) ? a.z1 : a.z0;
                T* lo_ = (ts & 1) ? a.l1 : a.l0;
                T* xo = (ts & 1) ? a.x1 : a.x0;
                for (int j = b; j < ta.tiles; j += G) {
                    const int d = (j * WPB + wv) * 64 + lane;
                    const int g = a.var[d];
                    if (g >= 0) {
                        zo[d] = zr[rs * LP + d];
                        lo_[d] = lr[rs * LP + d];
                        if ((a.meta[d] >> 16) & 1) xo[g] = xr[rs * ta.n + g];
                    }
                }
            }
            break;
        }
        const unsigned tag = (unsigned)t;
        const u64* pubr = p.pub + (size_t)(t & 1) * LP * W;
        u64* pubw = p.pub + (size_t)(tn & 1) * LP * W;
        const size_t rsrc = (size_t)(t % kStateRing), rdst = (size_t)(tn % kStateRing);
        double s[5] = {0, 0, 0, 0, 0};
        int bad = 0;
        long long spins = 0;
        for (int j = b; j < ta.tiles; j += G) {
            const int w = j * WPB + wv;
            const int d = w * 64 + lane;
            const int g = a.var[d];
            const bool live = g >= 0;
            T acc = 0, zold = 0, lold = 0;
            int meta = 0, cn = 1;
            if (live) {
                meta = a.meta[d];
                const int cs = a.cstart[d];
                cn = a.ccnt[d];
                zold = zr[rsrc * LP + d];
                lold = lr[rsrc * LP + d];
                int cp[kCopyRegs];
                u64 wd[kCopyRegs][W];
                unsigned pending = 0;
#pragma unroll
                for (int k = 0; k < kCopyRegs; ++k) {
                    cp[k] = k < cn ? a.clist[cs + k] : d;
                    if (k < cn && cp[k] != d) {
                        load_words<W>(pubr + (size_t)cp[k] * W, wd[k]);
                        pending |= 1u << k;
                    }
                }
                for (;;) {
                    unsigned stale = 0;
#pragma unroll
                    for (int k = 0; k < kCopyRegs; ++k)
                        if (((pending >> k) & 1u) && !tags_are<W>(wd[k], tag)) stale |= 1u << k;
                    if (!stale || bad) break;
                    __builtin_amdgcn_s_sleep(1);
#pragma unroll
                    for (int k = 0; k < kCopyRegs; ++k)
                        if ((stale >> k) & 1u) load_words<W>(pubr + (size_t)cp[k] * W, wd[k]);
                    pending = stale;
                    bad = wait_expired(++spins, error, p.spin_limit);
                }
#pragma unroll
                for (int k = 0; k < kCopyRegs; ++k)
                    if (k < cn) acc += (cp[k] == d) ? copy_term(zold, lold, inv_rho) : Tag<T>::unpack(wd[k]);
                for (int k = kCopyRegs; k < cn; ++k) {
                    const int e = a.clist[cs + k];
                    u64 we[W];
                    load_words<W>(pubr + (size_t)e * W, we);
                    while (!tags_are<W>(we, tag) && !bad) {
                        __builtin_amdgcn_s_sleep(1);
                        load_words<W>(pubr + (size_t)e * W, we);
                        bad = wait_expired(++spins, error, p.spin_limit);
                    }
                    acc += Tag<T>::unpack(we);
                }
            }
            T xg = 0;
            if (live) xg = consensus_value(acc, a.cost[d], inv_rho, cn, a.lo[d], a.hi[d]);
            vsh[wv][lane] = live ? projection_input(xg, lold, inv_rho) : (T)0;
            __builtin_amdgcn_wave_barrier();
            if (live) {
                const int2 wi = a.winfo[w];
                const T z = project_row(a.F + (size_t)wi.y * 64, vsh[wv], meta & 255, lane, wi.x, a.bbar[d]);
                const T ln = dual_step(lold, rho, xg, z);
                u64 wout[W];
                Tag<T>::pack(copy_term(z, ln, inv_rho), (unsigned)tn, wout);
#pragma unroll
                for (int h = 0; h < W; ++h) st_agent(pubw + (size_t)d * W + h, wout[h]);
                zr[rdst * LP + d] = z;
                lr[rdst * LP + d] = ln;
                if ((meta >> 16) & 1) xr[rdst * ta.n + g] = xg;
                const double xd = (double)xg, zd = (double)z;
                s[0] += (xd - zd) * (xd - zd);
                s[1] += (zd - (double)zold) * (zd - (double)zold);
                s[2] += xd * xd;
                s[3] += zd * zd;
                s[4] += (double)ln * (double)ln;
            }
            // the next tile rewrites this wavefront's LDS row after every lane has read it
            __builtin_amdgcn_wave_barrier();
        }
        if (__syncthreads_or(bad)) {
            if (threadIdx.x == 0) st_agent(error, (int)OPF_EHANG);
            break;
        }
        // ---- workgroup residual record of iteration tn (as the persistent kernel)
#pragma unroll
        for (int i = 0; i < 5; ++i) s[i] = wave_total(s[i]);
        if (lane == 0)
#pragma unroll
            for (int i = 0; i < 5; ++i) red[wv][i] = s[i];
        __syncthreads();
        if (threadIdx.x < 5) {
            const int i = threadIdx.x;
            double bsum = 0.0;
            for (int q = 0; q < WPB; ++q) bsum += red[q][i];
            u64 two[2];
            Tag<double>::pack(bsum, (unsigned)tn, two);
            u64* rw = p.records + ((size_t)(tn % LAG) * kRec + 2 * i) * G + b;
            st_agent(rw, two[0]);
            st_agent(rw + G, two[1]);
        }
        t = tn;
    }
}

// The state of the start iteration t0 into its ring position.
template <typename T>
__global__ void tiled_ring_init_kernel(IterArgs<T> a, TiledArgs ta) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const long long t0 = a.ctrl->iter;
    const size_t LP = (size_t)a.waves * 64;
    const size_t r = (size_t)(t0 % kStateRing);
    T* zr = static_cast<T*>(ta.zr);
    T* lr = static_cast<T*>(ta.lr);
    T* xr = static_cast<T*>(ta.xr);
    if (i < LP) {
        zr[r * LP + i] = (t0 & 1) ? a.z1[i] : a.z0[i];
        lr[r * LP + i] = (t0 & 1) ? a.l1[i] : a.l0[i];
    }
    if (i < (size_t)ta.n) xr[r * ta.n + i] = (t0 & 1) ? a.x1[i] : a.x0[i];
}

// Tiled schedule: G compute workgroups (plus the reducer) over ta.tiles tiles.
template <typename T>
hipError_t launch_tiled(const IterArgs<T>& a, PersistArgs p, const TiledArgs& ta, int wpb, int G, hipStream_t st) {
    const size_t LP = (size_t)a.waves * 64;
    hipError_t e0 = launch_prepare<T>(a, p, G, st);
    if (e0 != hipSuccess) return e0;
    const size_t m = std::max<size_t>(LP, (size_t)ta.n);
    hipLaunchKernelGGL((tiled_ring_init_kernel<T>), dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, a, ta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    TiledArgs t = ta;
    void* args[] = {(void*)&a, (void*)&p, (void*)&t};
    switch (wpb) {
        case 1: return hipLaunchCooperativeKernel((const void*)admm_tiled_kernel<T, 1>, dim3(G + 1), dim3(64), args, 0, st);
        case 2: return hipLaunchCooperativeKernel((const void*)admm_tiled_kernel<T, 2>, dim3(G + 1), dim3(128), args, 0, st);
        case 8: return hipLaunchCooperativeKernel((const void*)admm_tiled_kernel<T, 8>, dim3(G + 1), dim3(512), args, 0, st);
        default: return hipLaunchCooperativeKernel((const void*)admm_tiled_kernel<T, 4>, dim3(G + 1), dim3(256), args, 0, st);
    }
}
template hipError_t launch_tiled<double>(const IterArgs<double>&, PersistArgs, const TiledArgs&, int, int, hipStream_t);
template hipError_t launch_tiled<float>(const IterArgs<float>&, PersistArgs, const TiledArgs&, int, int, hipStream_t);

// Co-resident workgroups of the tiled kernel (0 on error).
template <typename T>
int tiled_capacity(int wpb) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e;
    switch (wpb) {
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, admm_tiled_kernel<T, 1>, 64, 0); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, admm_tiled_kernel<T, 2>, 128, 0); break;
        case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, admm_tiled_kernel<T, 8>, 512, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, admm_tiled_kernel<T, 4>, 256, 0); break;
    }
    if (e != hipSuccess) return 0;
    return per * cus;
}
template int tiled_capacity<double>(int);
template int tiled_capacity<float>(int);

}  // namespace opf
