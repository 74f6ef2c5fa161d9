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

// ---- two tiles per workgroup, both in flight ------------------------------
// When every workgroup holds at most two tiles, workgroup b owns tiles b and
// b + G (if it exists) for the whole launch, and each thread keeps the static
// data and the current local copy and dual of its two slots in registers (the
// ring in memory only serves the stop decision's write-out).  Every iteration
// issues the neighbour-term loads of both slots before waiting on either, and
// computes the two projections with the factor columns of both loaded
// together, so the two slots share one chain of memory round trips.  The
// arithmetic is that of every other schedule, step for step.
constexpr int kPairCopies = 4;   // copies of a slot's variable gathered in registers (more: one by one)

template <typename T>
struct PairSlot {
    int d, g, meta, cs, cn;
    int cp[kPairCopies];
    int2 wi;
    T cost, lo, hi, bb, z, l;
};

// acc_q + sum_k F_q[k][lane] v_q[(base_q + k) & 63] for two slots, columns
// ascending, the loads of eight columns of both issued ahead of their
// fused multiply-adds (the rounding of project_row for each slot).
template <typename T>
__device__ __forceinline__ void project_rows2(const T* F0, const T* v0, int base0, int n0, T& acc0,
                                              const T* F1, const T* v1, int base1, int n1, T& acc1, int lane) {
    const int nmax = n0 > n1 ? n0 : n1;
    for (int k = 0; k < nmax; k += 8) {
        T f0[8], x0[8], f1[8], x1[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int c = k + j;
            f0[j] = c < n0 ? F0[c * 64 + lane] : (T)0;
            x0[j] = v0[(base0 + c) & 63];
            f1[j] = c < n1 ? F1[c * 64 + lane] : (T)0;
            x1[j] = v1[(base1 + c) & 63];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (k + j < n0) acc0 = fmadd(f0[j], x0[j], acc0);
            if (k + j < n1) acc1 = fmadd(f1[j], x1[j], acc1);
        }
    }
}

template <typename T, int WPB>
__global__ __launch_bounds__(WPB * 64) void admm_tiled_pair_kernel(IterArgs<T> a, PersistArgs p, TiledArgs ta) {
    constexpr int NT = WPB * 64;
    constexpr int W = Tag<T>::W;
    constexpr int LAG = kDecisionLag;
    const int G = (int)gridDim.x - 1;
    const int b = (int)blockIdx.x;
    int* error = p.error;
    Ctrl* ctrl = a.ctrl;
    const long long t0 = ctrl->iter;
    if (b == G) {
        // one workgroup's record per poll keeps the reducer's registers (and
        // so the kernel's) within four wavefronts per SIMD
        const InstanceView<T> v = view_of(a, p);
        reducer_loop<T, NT, false, 1>(v, G, t0, error, p.spin_limit);
        return;
    }
    __shared__ T vsh[2][WPB][64];
    __shared__ double red[WPB][5];
    __shared__ int sh_flag;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const size_t LP = (size_t)a.waves * 64;
    T* zr = static_cast<T*>(ta.zr);
    T* lr = static_cast<T*>(ta.lr);
    T* xr = static_cast<T*>(ta.xr);
    const T inv_rho = a.inv_rho, rho = a.rho;
    const int ntile = b + G < ta.tiles ? 2 : 1;          // the same for the whole workgroup
    // factors of this workgroup's wavefronts (tile 0's, then tile 1's) copied
    // once into LDS when their columns fit the launch's budget; each lane
    // reads back only what it wrote, so no barrier is needed
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    T* Fl = reinterpret_cast<T*>(dyn_lds);
    int wg_cols = 0, off_cols[2] = {0, 0};
    for (int q = 0; q < ntile; ++q)
        for (int v = 0; v < WPB; ++v) {
            const int c = a.winfo[(b + q * G) * WPB + v].x;
            if (v == wv) off_cols[q] = wg_cols;
            wg_cols += c;
        }
    const bool in_lds = ta.lds_cols > 0 && wg_cols <= ta.lds_cols;
    PairSlot<T> S[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        PairSlot<T>& u = S[q];
        const int w = (b + q * G) * WPB + wv;
        u.d = w * 64 + lane;
        u.g = -1; u.meta = 0; u.cs = 0; u.cn = 1;
        u.wi = make_int2(0, 0);
        u.cost = u.lo = u.hi = u.bb = u.z = u.l = (T)0;
#pragma unroll
        for (int k = 0; k < kPairCopies; ++k) u.cp[k] = u.d;
        if (q < ntile) {
            u.g = a.var[u.d];
            u.wi = a.winfo[w];
            if (u.g >= 0) {
                u.meta = a.meta[u.d];
                u.cs = a.cstart[u.d];
                u.cn = a.ccnt[u.d];
#pragma unroll
                for (int k = 0; k < kPairCopies; ++k) u.cp[k] = k < u.cn ? a.clist[u.cs + k] : u.d;
                u.cost = a.cost[u.d];
                u.lo = a.lo[u.d];
                u.hi = a.hi[u.d];
                u.bb = a.bbar[u.d];
                const size_t r0 = (size_t)(t0 % kStateRing);
                u.z = zr[r0 * LP + u.d];
                u.l = lr[r0 * LP + u.d];
            }
        }
    }
    const T* Fsrc[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        Fsrc[q] = a.F + (size_t)S[q].wi.y * 64;
        if (in_lds && q < ntile) {
            T* dst = Fl + (size_t)off_cols[q] * 64;
            for (int k = 0; k < S[q].wi.x; ++k) dst[k * 64 + lane] = Fsrc[q][k * 64 + lane];
            Fsrc[q] = dst;
        }
    }
    long long t = t0;
    int bad = 0;
    for (;;) {
        const long long tn = t + 1;
        long long dseen = 0;
        int errseen = 0;
        if (threadIdx.x == 0) {
            dseen = ld_agent(p.dec_iter);
            errseen = ld_agent(error);
        }
        const unsigned tag = (unsigned)t;
        const u64* pubr = p.pub + (size_t)(t & 1) * LP * W;
        u64* pubw = p.pub + (size_t)(tn & 1) * LP * W;
        const size_t rdst = (size_t)(tn % kStateRing);
        long long spins = 0;
        // ---- the neighbour terms of both slots, all loads in flight at once
        u64 wd[2][kPairCopies][W];
        unsigned pending[2] = {0u, 0u};
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int k = 0; k < kPairCopies; ++k)
                if (S[q].g >= 0 && k < S[q].cn && S[q].cp[k] != S[q].d) {
                    load_words<W>(pubr + (size_t)S[q].cp[k] * W, wd[q][k]);
                    pending[q] |= 1u << k;
                }
        for (;;) {
            unsigned stale[2] = {0u, 0u};
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int k = 0; k < kPairCopies; ++k)
                    if (((pending[q] >> k) & 1u) && !tags_are<W>(wd[q][k], tag)) stale[q] |= 1u << k;
            if (!(stale[0] | stale[1]) || bad) break;
            __builtin_amdgcn_s_sleep(1);
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int k = 0; k < kPairCopies; ++k)
                    if ((stale[q] >> k) & 1u) load_words<W>(pubr + (size_t)S[q].cp[k] * W, wd[q][k]);
            pending[0] = stale[0];
            pending[1] = stale[1];
            bad = wait_expired(++spins, error, p.spin_limit);
        }
        T acc[2] = {(T)0, (T)0};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (S[q].g < 0) continue;
#pragma unroll
            for (int k = 0; k < kPairCopies; ++k)
                if (k < S[q].cn)
                    acc[q] += (S[q].cp[k] == S[q].d) ? copy_term(S[q].z, S[q].l, inv_rho) : Tag<T>::unpack(wd[q][k]);
            for (int k = kPairCopies; k < S[q].cn; ++k) {
                const int e = a.clist[S[q].cs + k];
                u64 we[W];
                load_words<W>(pubr + (size_t)e * W, we);
                while (!tags_are<W>(we, tag) && !bad) {
                    __builtin_amdgcn_s_sleep(1);
                    load_words<W>(pubr + (size_t)e * W, we);
                    bad = wait_expired(++spins, error, p.spin_limit);
                }
                acc[q] += Tag<T>::unpack(we);
            }
        }
        // ---- the decision of tn - LAG (every workgroup computed every
        // iteration up to it + LAG - 1, so the gathers above ended)
        if (threadIdx.x == 0) {
            long long sp = 0;
            int late = 0;
            while (dseen < tn - LAG && !late && !errseen) {
                __builtin_amdgcn_s_sleep(1);
                dseen = ld_agent(p.dec_iter);
                errseen = ld_agent(error);
                if (++sp > p.spin_limit) late = 1;
            }
            int stop = 0;
            __atomic_signal_fence(__ATOMIC_SEQ_CST);   // dec_stop is read after dec_iter
            if (!late && !errseen && tn - LAG > t0) stop = ld_agent(p.dec_stop) == tn - LAG;
            sh_flag = stop | ((errseen || late) ? 2 : 0);
        }
        const int flag = __syncthreads_or(bad) ? 2 : sh_flag;
        if (flag) {
            if (flag == 1) {
                // state of the end iteration ts into the iteration-parity buffers
                const long long ts = tn - LAG;
                const size_t rs = (size_t)(ts % kStateRing);
                T* zo = (ts & 1) ? a.z1 : a.z0;
                T* lo_ = (ts & 1) ? a.l1 : a.l0;
                T* xo = (ts & 1) ? a.x1 : a.x0;
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    if (S[q].g >= 0) {
                        zo[S[q].d] = zr[rs * LP + S[q].d];
                        lo_[S[q].d] = lr[rs * LP + S[q].d];
                        if ((S[q].meta >> 16) & 1) xo[S[q].g] = xr[rs * ta.n + S[q].g];
                    }
            } else if (threadIdx.x == 0) {
                st_agent(error, (int)OPF_EHANG);
            }
            break;
        }
        // ---- global update, both projections, dual updates, residual terms
        T xg[2] = {(T)0, (T)0};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (S[q].g >= 0) xg[q] = consensus_value(acc[q], S[q].cost, inv_rho, S[q].cn, S[q].lo, S[q].hi);
            vsh[q][wv][lane] = S[q].g >= 0 ? projection_input(xg[q], S[q].l, inv_rho) : (T)0;
        }
        __builtin_amdgcn_wave_barrier();
        T zn[2] = {S[0].bb, S[1].bb};
        project_rows2(Fsrc[0], vsh[0][wv], S[0].meta & 255, S[0].g >= 0 ? S[0].wi.x : 0, zn[0],
                      Fsrc[1], vsh[1][wv], S[1].meta & 255, S[1].g >= 0 ? S[1].wi.x : 0, zn[1], lane);
        double s[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (S[q].g < 0) continue;
            const T z = zn[q];
            const T ln = dual_step(S[q].l, rho, xg[q], z);
            u64 wout[W];
            Tag<T>::pack(copy_term(z, ln, inv_rho), (unsigned)tn, wout);
#pragma unroll
            for (int h = 0; h < W; ++h) st_agent(pubw + (size_t)S[q].d * W + h, wout[h]);
            zr[rdst * LP + S[q].d] = z;
            lr[rdst * LP + S[q].d] = ln;
            if ((S[q].meta >> 16) & 1) xr[rdst * ta.n + S[q].g] = xg[q];
            const double xd = (double)xg[q], zd = (double)z;
            s[0] += (xd - zd) * (xd - zd);
            s[1] += (zd - (double)S[q].z) * (zd - (double)S[q].z);
            s[2] += xd * xd;
            s[3] += zd * zd;
            s[4] += (double)ln * (double)ln;
            S[q].z = z;
            S[q].l = ln;
        }
        // the next iteration rewrites the wavefront's LDS rows after every lane has read them
        __builtin_amdgcn_wave_barrier();
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
    if (ta.pair) {
        const size_t lds = (size_t)ta.lds_cols * 64 * sizeof(T);
        switch (wpb) {
            case 1: return hipLaunchCooperativeKernel((const void*)admm_tiled_pair_kernel<T, 1>, dim3(G + 1), dim3(64), args, lds, st);
            case 2: return hipLaunchCooperativeKernel((const void*)admm_tiled_pair_kernel<T, 2>, dim3(G + 1), dim3(128), args, lds, st);
            case 8: return hipLaunchCooperativeKernel((const void*)admm_tiled_pair_kernel<T, 8>, dim3(G + 1), dim3(512), args, lds, st);
            default: return hipLaunchCooperativeKernel((const void*)admm_tiled_pair_kernel<T, 4>, dim3(G + 1), dim3(256), args, lds, st);
        }
    }
    switch (wpb) {
        case 1: return hipLaunchCooperativeKernel((const void*)admm_tiled_kernel<T, 1>, dim3(G + 1), dim3(64), args, 0, st);
        case 2: return hipLaunchCooperativeKernel((const void*)admm_tiled_kernel<T, 2>, dim3(G + 1), dim3(128), args, 0, st);
        case 8: return hipLaunchCooperativeKernel((const void*)admm_tiled_kernel<T, 8>, dim3(G + 1), dim3(512), args, 0, st);
        default: return hipLaunchCooperativeKernel((const void*)admm_tiled_kernel<T, 4>, dim3(G + 1), dim3(256), args, 0, st);
    }
}
template hipError_t launch_tiled<double>(const IterArgs<double>&, PersistArgs, const TiledArgs&, int, int, hipStream_t);
template hipError_t launch_tiled<float>(const IterArgs<float>&, PersistArgs, const TiledArgs&, int, int, hipStream_t);

// Co-resident workgroups of the tiled kernel (pair = 1: the two-tile kernel,
// with lds_bytes of dynamic shared memory per workgroup) (0 on error).
template <typename T>
int tiled_capacity(int wpb, int pair, size_t lds_bytes) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e;
    if (pair) {
        switch (wpb) {
            case 1: e = resident_per_cu(&per, (const void*)admm_tiled_pair_kernel<T, 1>, 64, lds_bytes); break;
            case 2: e = resident_per_cu(&per, (const void*)admm_tiled_pair_kernel<T, 2>, 128, lds_bytes); break;
            case 8: e = resident_per_cu(&per, (const void*)admm_tiled_pair_kernel<T, 8>, 512, lds_bytes); break;
            default: e = resident_per_cu(&per, (const void*)admm_tiled_pair_kernel<T, 4>, 256, lds_bytes); break;
        }
    } else {
        switch (wpb) {
            case 1: e = resident_per_cu(&per, (const void*)admm_tiled_kernel<T, 1>, 64, 0); break;
            case 2: e = resident_per_cu(&per, (const void*)admm_tiled_kernel<T, 2>, 128, 0); break;
            case 8: e = resident_per_cu(&per, (const void*)admm_tiled_kernel<T, 8>, 512, 0); break;
            default: e = resident_per_cu(&per, (const void*)admm_tiled_kernel<T, 4>, 256, 0); break;
        }
    }
    if (e != hipSuccess) return 0;
    return per * cus;
}
template int tiled_capacity<double>(int, int, size_t);
template int tiled_capacity<float>(int, int, size_t);

}  // namespace opf
