// Persistent form of the fused ADMM iteration for gfx950: one cooperative
// launch runs every iteration of Algorithm 1 until the termination test holds.
//
// Work split: workgroup b owns `WPB` packed wavefronts (a contiguous run of the
// component graph) and keeps its slots' static data, its factors (in LDS when
// they fit) and its own local copy and dual in registers across iterations.
//
// Data exchange without barriers or flags on the compute path: after
// iteration t every slot publishes the one value other copies of its variable
// need, its consensus term z - lambda / rho, as 64-bit words that carry the
// iteration number t in their upper half (one word for FP32, two for FP64).
// A consumer loads the words of all copies of its variable at once and only
// re-loads those whose tag is not yet t.  Two buffers (iteration parity)
// suffice: a slot can publish t + 1 only after it has read every neighbour's
// term of t, which each neighbour computed after reading the old term of
// t - 1 that t + 1 overwrites.
//
// Termination: each workgroup writes its five FP64 residual partial sums of
// iteration t, split into tagged 64-bit words like the copy terms, into a ring
// of kDecisionLag records.  One extra workgroup (the reducer, last of the
// grid) polls the records of iteration t until every tag is t, reduces them in
// a fixed order and publishes the last decided iteration and, on a stop, the
// stop iteration ts.  A workgroup acts
// on the decision of iteration tn - kDecisionLag at the start of tn, so every
// workgroup computes exactly the iterations up to ts + kDecisionLag - 1 (no
// wait can outlive its producer), and keeps the state of its last
// kDecisionLag iterations in registers to write out the state of ts.
// Cross-workgroup data moves through agent-scope atomic loads and stores
// (coherent across the chip's L2 slices without write-back fences).  Every
// wait is bounded: a wait that runs out sets OPF_EHANG and every workgroup
// leaves the loop, so the grid always drains.
#include <algorithm>

#include "admm_kernels.h"
#include "admm_sync.h"

#include "../../include/opf_admm.h"

namespace opf {

// The persistent loop of one solve for workgroup b of its G compute
// workgroups (b == G: its reducer).
// PER_WG_LDS: each workgroup checks its own factor columns against the LDS
// budget (serving, where one launch holds several solves); otherwise the
// budget covers every workgroup of the launch.  ADAPT: the penalty follows
// the residual-balancing ring of the control block (a separate instantiation,
// so the fixed-penalty kernel keeps its registers).  RB: workgroup records
// the reducer's threads load at once.
template <typename T, int WPB, bool PER_WG_LDS, bool ADAPT, int RB = kBatch>
__device__ void persistent_instance(const InstanceView<T>& a, int b, int G, int* error, long long spin_limit) {
    constexpr int NT = WPB * 64;
    constexpr int W = Tag<T>::W;
    constexpr int LAG = kDecisionLag;
    __shared__ T vsh[WPB][64];
    __shared__ double red[WPB][5];
    __shared__ int sh_flag;
    __shared__ double sh_rho;

    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    Ctrl* ctrl = a.ctrl;
    const long long t0 = ctrl->iter;
    if (b == G) {
        reducer_loop<T, NT, ADAPT, RB>(a, G, t0, error, spin_limit);
        return;
    }
    const int w = b * WPB + wv;
    const int d = w * 64 + lane;
    const size_t LP = (size_t)a.waves * 64;

    // ---- static per-slot data, kept in registers
    const int g = a.var[d];
    const bool live = g >= 0;
    int meta = 0, cs = 0, cn = 1;
    int cp[kCopyRegs];
    T bb = 0, lo = 0, hi = 0, cost = 0;
    if (live) {
        meta = a.meta[d];
        cs = a.cstart[d];
        cn = a.ccnt[d];
#pragma unroll
        for (int k = 0; k < kCopyRegs; ++k) cp[k] = k < cn ? a.clist[cs + k] : d;
        bb = a.bbar[d];
        lo = a.lo[d];
        hi = a.hi[d];
        cost = a.cost[d];
    }
    const int2 wi = a.winfo[w];
    const T* Fg = a.F + (size_t)wi.y * 64;
    // static factors of this workgroup's wavefronts, copied once into LDS when
    // they fit (kept as a separate pointer so the loads stay LDS loads)
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    T* Fl = reinterpret_cast<T*>(dyn_lds);
    // (the same decision for all threads of the workgroup)
    bool in_lds = a.lds_factors != 0;
    if (PER_WG_LDS) {
        int wg_cols = 0;
        for (int q = 0; q < WPB; ++q) wg_cols += a.winfo[b * WPB + q].x;
        in_lds = in_lds && wg_cols <= a.lds_factors;
    }
    if (in_lds) {
        int off = 0;
        for (int q = 0; q < wv; ++q) off += a.winfo[b * WPB + q].x;
        Fl += (size_t)off * 64;
        for (int k = 0; k < wi.x; ++k) Fl[k * 64 + lane] = Fg[k * 64 + lane];
    }
    const int base = meta & 255;
    const bool owner = (meta >> 16) & 1;
    // penalty of the iteration being computed (residual balancing: from the
    // ring, where the decision of tn - LAG put the penalty of tn + 1)
    T inv_rho = a.inv_rho, rho = a.rho;
    if (ADAPT) {
        const double r0 = ld_agent(&ctrl->rho[(t0 + 1) % kRhoRing]);
        rho = (T)(a.local_updates * r0);
        inv_rho = (T)(1.0 / r0);
    }
    // state of the last LAG iterations: index 0 = current iteration t
    T zh[LAG], lh[LAG], xh[LAG];
#pragma unroll
    for (int k = 0; k < LAG; ++k) zh[k] = lh[k] = xh[k] = 0;
    if (live) {
        zh[0] = (t0 & 1) ? a.z1[d] : a.z0[d];
        lh[0] = (t0 & 1) ? a.l1[d] : a.l0[d];
    }

    long long t = t0;
    int bad = 0;
    for (;;) {
        const long long tn = t + 1;
        long long spins = 0;            // polls of the waits of this iteration
        // ---- thread 0: decision of iteration tn - LAG (issued first, checked after the gathers)
        long long dseen = 0;
        int errseen = 0;
        if (threadIdx.x == 0) {
            dseen = ld_agent(a.dec_iter);
            errseen = ld_agent(error);
        }
        // ---- gather the terms of iteration t of every copy of this slot's variable
        const unsigned tag = (unsigned)t;
        const u64* pubr = a.pub + (size_t)(t & 1) * LP * W;
        T acc = 0;
        if (live) {
            // issue priority: low while waiting for the neighbours' terms, high
            // once they are in, so that a workgroup that can compute goes ahead
            // of the polling ones sharing its SIMDs
            __builtin_amdgcn_s_setprio(0);
            u64 wd[kCopyRegs][W];
            unsigned pending = 0;       // copies whose word of iteration t has not arrived
#pragma unroll
            for (int k = 0; k < kCopyRegs; ++k) {
                if (k < cn && cp[k] != d) {
                    load_words<W>(pubr + (size_t)cp[k] * W, wd[k]);
                    pending |= 1u << k;
                }
            }
            // re-load every stale copy at once, so one round trip covers them all
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
                bad = wait_expired(++spins, error, spin_limit);
            }
#pragma unroll
            for (int k = 0; k < kCopyRegs; ++k) {
                if (k < cn) acc += (cp[k] == d) ? copy_term(zh[0], lh[0], inv_rho) : Tag<T>::unpack(wd[k]);
            }
            for (int k = kCopyRegs; k < cn; ++k) {
                const int e = a.clist[cs + k];
                u64 we[W];
                load_words<W>(pubr + (size_t)e * W, we);
                while (!tags_are<W>(we, tag) && !bad) {
                    __builtin_amdgcn_s_sleep(1);
                    load_words<W>(pubr + (size_t)e * W, we);
                    bad = wait_expired(++spins, error, spin_limit);
                }
                acc += Tag<T>::unpack(we);
            }
            __builtin_amdgcn_s_setprio(2);
        }
        if (threadIdx.x == 0) {
            while (dseen < tn - LAG && !bad && !errseen) {
                __builtin_amdgcn_s_sleep(1);
                dseen = ld_agent(a.dec_iter);
                errseen = ld_agent(error);
                if (++spins > spin_limit) bad = 1;
            }
            int stop = 0;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);   // dec_stop and the penalty are read after dec_iter
            if (!bad && !errseen && tn - LAG > t0) stop = ld_agent(a.dec_stop) == tn - LAG;
            if (ADAPT && !bad && !errseen) sh_rho = ld_agent(&ctrl->rho[(tn + 1) % kRhoRing]);
            sh_flag = stop | (errseen ? 2 : 0);
        }
        if (__syncthreads_or(bad)) {
            if (threadIdx.x == 0) st_agent(error, (int)OPF_EHANG);
            break;
        }
        if (sh_flag) {
            if (sh_flag == 1 && live) {
                // state of the end iteration ts = tn - LAG = t - (LAG - 1)
                const long long ts = tn - LAG;
                T* zo = (ts & 1) ? a.z1 : a.z0;
                T* lo_ = (ts & 1) ? a.l1 : a.l0;
                T* xo = (ts & 1) ? a.x1 : a.x0;
                zo[d] = zh[LAG - 1];
                lo_[d] = lh[LAG - 1];
                if (owner) xo[g] = xh[LAG - 1];
            }
            break;
        }
        // ---- global update, local projection, dual update, residual terms.
        // The projection input is exchanged through this wavefront's own LDS
        // row only, and a wavefront's LDS operations complete in order, so a
        // wavefront barrier suffices here.
        // 1/rho of iteration tn + 1, carried by the published consensus term
        T inv_next = inv_rho;
        double rho_next = 0.0;
        if (ADAPT) {
            rho_next = sh_rho;
            inv_next = (T)(1.0 / rho_next);
        }
        T xg = 0;
        if (live) xg = consensus_value(acc, cost, inv_rho, cn, lo, hi);
        vsh[wv][lane] = live ? projection_input(xg, lh[0], inv_rho) : (T)0;
        __builtin_amdgcn_wave_barrier();
        double s[5] = {0, 0, 0, 0, 0};
        if (live) {
            const T z = in_lds ? project_row(Fl, vsh[wv], base, lane, wi.x, bb)
                               : project_row(Fg, vsh[wv], base, lane, wi.x, bb);
            const T ln = dual_step(lh[0], rho, xg, z);
            u64 wout[W];
            Tag<T>::pack(copy_term(z, ln, inv_next), (unsigned)tn, wout);
            u64* pubw = a.pub + (size_t)(tn & 1) * LP * W + (size_t)d * W;
#pragma unroll
            for (int h = 0; h < W; ++h) st_agent(pubw + h, wout[h]);
            // the term the neighbours wait for is out; the residual tail yields
            // to workgroups still on their way to publishing
            __builtin_amdgcn_s_setprio(1);
            const double xd = (double)xg, zd = (double)z;
            s[0] = (xd - zd) * (xd - zd);
            s[1] = (zd - (double)zh[0]) * (zd - (double)zh[0]);
            s[2] = xd * xd;
            s[3] = zd * zd;
            s[4] = (double)ln * (double)ln;
#pragma unroll
            for (int k = LAG - 1; k > 0; --k) {
                zh[k] = zh[k - 1];
                lh[k] = lh[k - 1];
                xh[k] = xh[k - 1];
            }
            zh[0] = z;
            lh[0] = ln;
            xh[0] = xg;
        }
        // ---- workgroup residual record of iteration tn: sum i over the
        // wavefronts in order (thread i), two tagged words per sum
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
            u64* rw = a.records + ((size_t)(tn % LAG) * kRec + 2 * i) * G + b;
            st_agent(rw, two[0]);
            st_agent(rw + G, two[1]);
        }
        if (ADAPT) {
            rho = (T)(a.local_updates * rho_next);
            inv_rho = inv_next;
        }
        t = tn;
    }
}


// FP64: each workgroup keeps its factors in LDS when their columns fit the
// launch's column budget (p.lds_factors), so that a problem whose largest
// workgroups would not let the grid fit still holds most of its factors in
// LDS; FP32: all workgroups or none (every FP32 problem here fits).
template <typename T, int WPB, bool ADAPT>
__global__ __launch_bounds__(WPB * 64) void admm_persistent_kernel(IterArgs<T> a, PersistArgs p) {
    const InstanceView<T> v = view_of(a, p);
    const int b = logical_block((int)blockIdx.x, (int)gridDim.x, p.xcd_remap);
    persistent_instance<T, WPB, (sizeof(T) == 8), ADAPT>(v, b, (int)gridDim.x - 1, p.error, p.spin_limit);
}

// Serving: the launch's workgroups are dealt to the resident solves by a work
// list of (slot, workgroup of the solve; == blocks for its reducer).  Each
// solve runs the single-instance persistent loop on its own state, for at
// most `chunk` iterations, so every solve returns the same bits alone and in
// any mix.  One launch runs one precision: the FP32 bulk phase of mixed
// solves, or FP64 (plain solves and the polish phase).
template <typename T>
struct DescState;

template <>
struct DescState<double> {
    static __device__ __forceinline__ void set(InstanceView<double>& v, const InstDesc& D) {
        v.F = D.F; v.bbar = D.bbar; v.lo = D.lo; v.hi = D.hi; v.cost = D.cost;
        v.z0 = D.z0; v.z1 = D.z1; v.l0 = D.l0; v.l1 = D.l1; v.x0 = D.x0; v.x1 = D.x1;
    }
    static __device__ __forceinline__ const double* z(const InstDesc& D, bool odd) { return odd ? D.z1 : D.z0; }
    static __device__ __forceinline__ const double* l(const InstDesc& D, bool odd) { return odd ? D.l1 : D.l0; }
};

template <>
struct DescState<float> {
    static __device__ __forceinline__ void set(InstanceView<float>& v, const InstDesc& D) {
        v.F = D.Ff; v.bbar = D.bbarf; v.lo = D.lof; v.hi = D.hif; v.cost = D.costf;
        v.z0 = D.z0f; v.z1 = D.z1f; v.l0 = D.l0f; v.l1 = D.l1f; v.x0 = D.x0f; v.x1 = D.x1f;
    }
    static __device__ __forceinline__ const float* z(const InstDesc& D, bool odd) { return odd ? D.z1f : D.z0f; }
    static __device__ __forceinline__ const float* l(const InstDesc& D, bool odd) { return odd ? D.l1f : D.l0f; }
};

template <typename T>
__device__ __forceinline__ InstanceView<T> view_of(const InstDesc& D, const ServeArgs& s) {
    InstanceView<T> v;
    DescState<T>::set(v, D);
    v.winfo = D.winfo; v.var = D.var; v.meta = D.meta; v.cstart = D.cstart; v.ccnt = D.ccnt; v.clist = D.clist;
    v.pub = D.pub; v.records = D.records; v.dec_iter = D.dec; v.dec_stop = D.dec + 1;
    v.ctrl = D.ctrl; v.hist = nullptr; v.hist_cap = 0; v.waves = D.lanes / 64; v.check = D.ctrl->check;
    v.lds_factors = s.lds_cols; v.rho = (T)D.rho; v.inv_rho = (T)(1.0 / D.rho); v.rho_d = D.rho;
    v.eps_rel = D.eps_rel; v.rule = RhoRule{0, 0, 0.0, 0.0, 0.0, 0.0}; v.local_updates = 1.0;
    v.max_iter = D.ctrl->max_iter; v.chunk = s.chunk;
    return v;
}

constexpr int kServeWPB = 4;

template <typename T>
__global__ __launch_bounds__(kServeWPB * 64) void admm_serve_kernel(const InstDesc* descs, const int2* work,
                                                                     ServeArgs s) {
    const int q = logical_block((int)blockIdx.x, (int)gridDim.x, s.xcd_remap);
    const int2 wk = work[q];
    const InstDesc& D = descs[wk.x];
    if (D.ctrl->stop) return;               // finished solves stay resident until retired
    const InstanceView<T> v = view_of<T>(D, s);
    // the reducer loads two records per thread at once (three: 136 instead of
    // 118 VGPRs in FP32, one workgroup fewer per compute unit)
    persistent_instance<T, kServeWPB, true, false, 2>(v, wk.y, D.blocks, s.error, s.spin_limit);
}

// Before a serving launch: each work item prepares its own part of its solve
// (published terms of the start iteration, residual records; the reducer item resets the
// decisions).
template <typename T>
__global__ void serve_prepare_kernel(const InstDesc* descs, const int2* work) {
    constexpr int W = Tag<T>::W;
    const int2 wk = work[blockIdx.x];
    const InstDesc& D = descs[wk.x];
    const long long t0 = D.ctrl->iter;
    const size_t LP = (size_t)D.lanes;
    if (wk.y < D.blocks) {
        const size_t d = (size_t)wk.y * blockDim.x + threadIdx.x;
        const bool odd = (t0 & 1) != 0;
        const T z = DescState<T>::z(D, odd)[d];
        const T l = DescState<T>::l(D, odd)[d];
        u64 w[W];
        Tag<T>::pack(copy_term(z, l, (T)(1.0 / D.rho)), (unsigned)t0, w);
#pragma unroll
        for (int h = 0; h < W; ++h) {
            D.pub[d * W + h] = w[h];
            D.pub[(LP + d) * W + h] = w[h];
        }
        // residual records of this workgroup: tag t0 matches no iteration of the launch
        for (int q = threadIdx.x; q < kDecisionLag * kRec; q += blockDim.x)
            D.records[(size_t)q * D.blocks + wk.y] = (u64)(unsigned)t0 << 32;
    } else if (threadIdx.x == 0) {
        D.dec[0] = t0;
        D.dec[1] = -1;
    }
}

template <typename T>
hipError_t launch_serve(const InstDesc* descs, const int2* work, int nwork, const ServeArgs& s, hipStream_t st) {
    hipLaunchKernelGGL(serve_prepare_kernel<T>, dim3(nwork), dim3(kServeWPB * 64), 0, st, descs, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ServeArgs sa = s;
    void* args[] = {(void*)&descs, (void*)&work, (void*)&sa};
    const size_t lds = (size_t)s.lds_cols * 64 * sizeof(T);
    return hipLaunchCooperativeKernel((const void*)admm_serve_kernel<T>, dim3(nwork), dim3(kServeWPB * 64), args,
                                      lds, st);
}

hipError_t launch_serve_persistent(const InstDesc* descs, const int2* work, int nwork, const ServeArgs& s, int fp32,
                                   hipStream_t st) {
    if (nwork < 1) return hipSuccess;
    return fp32 ? launch_serve<float>(descs, work, nwork, s, st) : launch_serve<double>(descs, work, nwork, s, st);
}

int serve_capacity(size_t lds_bytes, int fp32) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const void* k = fp32 ? (const void*)admm_serve_kernel<float> : (const void*)admm_serve_kernel<double>;
    if (resident_per_cu(&per, k, kServeWPB * 64, lds_bytes) != hipSuccess) return 0;
    return per * cus;
}

// Before a launch: the published terms of the start iteration t0 (both parity
// buffers, tag t0; the other buffer's tag t0 never matches a later
// iteration), residual records tagged t0 (stale), decisions at t0, error
// cleared.
template <typename T>
__global__ void persistent_prepare_kernel(IterArgs<T> a, PersistArgs p, int G) {
    constexpr int W = Tag<T>::W;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const long long t0 = a.ctrl->iter;
    const size_t LP = (size_t)a.waves * 64;
    if ((size_t)i < LP) {
        const T z = (t0 & 1) ? a.z1[i] : a.z0[i];
        const T l = (t0 & 1) ? a.l1[i] : a.l0[i];
        const T inv = a.rule.every ? (T)(1.0 / a.ctrl->rho[(t0 + 1) % kRhoRing]) : a.inv_rho;
        u64 w[W];
        Tag<T>::pack(copy_term(z, l, inv), (unsigned)t0, w);
#pragma unroll
        for (int h = 0; h < W; ++h) {
            p.pub[(size_t)i * W + h] = w[h];
            p.pub[(LP + i) * W + h] = w[h];
        }
    }
    if ((size_t)i < (size_t)kDecisionLag * G * kRec) p.records[i] = (u64)(unsigned)t0 << 32;
    if (i == 0) {
        *p.dec_iter = t0;
        *p.dec_stop = -1;
        *p.error = 0;
    }
}

// The prepare kernel alone (the tiled schedule's launch starts with it).
template <typename T>
hipError_t launch_prepare(const IterArgs<T>& a, PersistArgs p, int G, hipStream_t st) {
    const size_t LP = (size_t)a.waves * 64;
    const int n = (int)std::max<size_t>(LP, (size_t)kDecisionLag * G * kRec);
    hipLaunchKernelGGL((persistent_prepare_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, st, a, p, G);
    return hipGetLastError();
}
template hipError_t launch_prepare<double>(const IterArgs<double>&, PersistArgs, int, hipStream_t);
template hipError_t launch_prepare<float>(const IterArgs<float>&, PersistArgs, int, hipStream_t);

template <typename T, bool ADAPT>
hipError_t launch_persistent_as(const IterArgs<T>& a, PersistArgs p, int wpb, int G, size_t lds, hipStream_t st) {
    void* args[] = {(void*)&a, (void*)&p};
    switch (wpb) {
        case 1: return hipLaunchCooperativeKernel((const void*)admm_persistent_kernel<T, 1, ADAPT>, dim3(G + 1), dim3(64), args, lds, st);
        case 2: return hipLaunchCooperativeKernel((const void*)admm_persistent_kernel<T, 2, ADAPT>, dim3(G + 1), dim3(128), args, lds, st);
        case 8: return hipLaunchCooperativeKernel((const void*)admm_persistent_kernel<T, 8, ADAPT>, dim3(G + 1), dim3(512), args, lds, st);
        default: return hipLaunchCooperativeKernel((const void*)admm_persistent_kernel<T, 4, ADAPT>, dim3(G + 1), dim3(256), args, lds, st);
    }
}

template <typename T>
hipError_t launch_persistent(const IterArgs<T>& a, PersistArgs p, int wpb, int G, hipStream_t st) {
    const size_t lds = p.lds_factors ? (size_t)p.lds_factor_cols * 64 * sizeof(T) : 0;
    const size_t LP = (size_t)a.waves * 64;
    const int n = (int)std::max<size_t>(LP, (size_t)kDecisionLag * G * kRec);
    hipLaunchKernelGGL((persistent_prepare_kernel<T>), dim3((n + 255) / 256), dim3(256), 0, st, a, p, G);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return a.rule.every ? launch_persistent_as<T, true>(a, p, wpb, G, lds, st)
                        : launch_persistent_as<T, false>(a, p, wpb, G, lds, st);
}
template hipError_t launch_persistent<double>(const IterArgs<double>&, PersistArgs, int, int, hipStream_t);
template hipError_t launch_persistent<float>(const IterArgs<float>&, PersistArgs, int, int, hipStream_t);

template <typename T, bool ADAPT>
int persistent_capacity_as(int wpb, size_t lds_bytes) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e;
    switch (wpb) {
        case 1: e = resident_per_cu(&per, (const void*)admm_persistent_kernel<T, 1, ADAPT>, 64, lds_bytes); break;
        case 2: e = resident_per_cu(&per, (const void*)admm_persistent_kernel<T, 2, ADAPT>, 128, lds_bytes); break;
        case 8: e = resident_per_cu(&per, (const void*)admm_persistent_kernel<T, 8, ADAPT>, 512, lds_bytes); break;
        default: e = resident_per_cu(&per, (const void*)admm_persistent_kernel<T, 4, ADAPT>, 256, lds_bytes); break;
    }
    if (e != hipSuccess) return 0;
    return per * cus;
}

// Largest co-resident grid for the persistent kernel (0 on error); the grid
// holds one workgroup more than the compute workgroups (the reducer).
// adapt = 1: the residual-balancing instantiation.
template <typename T>
int persistent_capacity(int wpb, size_t lds_bytes, int adapt) {
    return adapt ? persistent_capacity_as<T, true>(wpb, lds_bytes) : persistent_capacity_as<T, false>(wpb, lds_bytes);
}
template int persistent_capacity<double>(int, size_t, int);
template int persistent_capacity<float>(int, size_t, int);

}  // namespace opf
