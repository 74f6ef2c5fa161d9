// Cross-workgroup synchronisation helpers shared by the persistent, serving
// and tiled schedules (internal header): agent-scope loads and stores, tagged
// words, bounded waits, the view of one solve's buffers and the reducer
// workgroup that takes the stop decisions.
#pragma once

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

__device__ __forceinline__ long long wave_min_p(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const long long u = __shfl_xor(v, o, 64);
        v = u < v ? u : v;
    }
    return v;
}

// ---- tagged words: payload in the low 32 bits, iteration tag in the high 32
typedef unsigned long long u64;
template <typename T>
struct Tag;
template <>
struct Tag<float> {
    static constexpr int W = 1;
    __device__ static void pack(float v, unsigned tag, u64 (&w)[1]) {
        w[0] = (u64)__float_as_uint(v) | ((u64)tag << 32);
    }
    __device__ static float unpack(const u64 (&w)[1]) { return __uint_as_float((unsigned)w[0]); }
};
template <>
struct Tag<double> {
    static constexpr int W = 2;
    __device__ static void pack(double v, unsigned tag, u64 (&w)[2]) {
        const u64 bits = (u64)__double_as_longlong(v);
        w[0] = (bits & 0xffffffffull) | ((u64)tag << 32);
        w[1] = (bits >> 32) | ((u64)tag << 32);
    }
    __device__ static double unpack(const u64 (&w)[2]) {
        return __longlong_as_double((long long)((w[0] & 0xffffffffull) | (w[1] << 32)));
    }
};
template <int W>
__device__ __forceinline__ bool tags_are(const u64 (&w)[W], unsigned tag) {
    bool ok = true;
#pragma unroll
    for (int h = 0; h < W; ++h) ok &= (unsigned)(w[h] >> 32) == tag;
    return ok;
}
template <int W>
__device__ __forceinline__ void load_words(const u64* p, u64 (&w)[W]) {
#pragma unroll
    for (int h = 0; h < W; ++h) w[h] = ld_agent(p + h);
}

// A wait gives up after spin_limit polls, or early once another workgroup
// has reported an error (checked every 1024 polls).
__device__ __forceinline__ int wait_expired(long long spins, int* error, long long spin_limit) {
    if (spins > spin_limit) return 1;
    return (spins & 1023) == 0 && ld_agent(error) != 0;
}

constexpr int kCopyRegs = 8;
constexpr int kBatch = 3;      // workgroups whose records a reducer thread loads at once (default)
constexpr int kRec = 10;       // words of one residual record (5 doubles, two tagged halves each)

// Everything one solve's persistent loop touches, for the single-instance
// kernel and for each solve of the serving kernel.
template <typename T>
struct InstanceView {
    const T* F;
    const int2* winfo;
    const int* var;
    const int* meta;
    const int* cstart;
    const int* ccnt;
    const int* clist;
    const T* bbar;
    const T* lo;
    const T* hi;
    const T* cost;
    T* z0; T* z1;
    T* l0; T* l1;
    T* x0; T* x1;
    u64* pub;
    u64* records;
    long long* dec_iter;
    long long* dec_stop;
    Ctrl* ctrl;
    double* hist;
    int hist_cap;
    int waves;
    int check;
    int lds_factors;           // 0: factors read from memory; otherwise 1 (every workgroup's factors
                               // fit the launch's LDS), or with per-workgroup checks the column budget
    T rho, inv_rho;            // rho: the dual step length (local_updates x penalty)
    double rho_d, eps_rel;
    RhoRule rule;              // rule.every == 0: fixed penalty; else the ring of ctrl->rho
    double local_updates;
    long long max_iter;
    long long chunk;           // the launch ends for this solve after this many iterations
};

// Reducer workgroup of one solve: stop decisions of every iteration.  A
// decision ends the launch for the solve when the test holds, on a NaN/Inf,
// at max_iter, or after `chunk` iterations of this launch (a pause: the solve
// continues in the next launch from the state written at the pause).  BATCH:
// workgroups whose records one thread loads at once (fewer: fewer registers).
template <typename T, int NT, bool ADAPT, int BATCH = kBatch>
__device__ void reducer_loop(const InstanceView<T>& v, int G, long long t0, int* error, long long spin_limit) {
    __shared__ double rred[NT / 64][5];
    __shared__ int rstop;
    // the reducer shares a compute unit with iteration workgroups: its waves
    // issue first, so that the decisions keep pace with the iterations
    __builtin_amdgcn_s_setprio(3);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    Ctrl* ctrl = v.ctrl;
    for (long long u = t0 + 1;; ++u) {
        // ---- records of iteration u of every workgroup, summed in a fixed order
        // (per thread over q = tid, tid + NT, ..., then across lanes and waves)
        const unsigned tag = (unsigned)u;
        // word w of workgroup q at rec[w * G + q]: one load instruction per
        // word covers 64 consecutive workgroups
        const u64* rec = v.records + (size_t)(u % kDecisionLag) * G * kRec;
        double acc5[5] = {0, 0, 0, 0, 0};
        int bad = 0;
        long long spins = 0;
        for (int q0 = threadIdx.x; q0 < G; q0 += BATCH * NT) {
            u64 wd[BATCH][kRec];
            unsigned pending = 0;
#pragma unroll
            for (int k = 0; k < BATCH; ++k) {
                const int q = q0 + k * NT;
                if (q < G) {
#pragma unroll
                    for (int h = 0; h < kRec; ++h) wd[k][h] = ld_agent(rec + (size_t)h * G + q);
                    pending |= 1u << k;
                }
            }
            for (;;) {
                unsigned stale = 0;
#pragma unroll
                for (int k = 0; k < BATCH; ++k)
                    if (((pending >> k) & 1u) && !tags_are<kRec>(wd[k], tag)) stale |= 1u << k;
                if (!stale || bad) break;
                __builtin_amdgcn_s_sleep(1);
#pragma unroll
                for (int k = 0; k < BATCH; ++k)
                    if ((stale >> k) & 1u)
#pragma unroll
                        for (int h = 0; h < kRec; ++h) wd[k][h] = ld_agent(rec + (size_t)h * G + q0 + k * NT);
                pending = stale;
                bad = wait_expired(++spins, error, spin_limit);
            }
#pragma unroll
            for (int k = 0; k < BATCH; ++k)
                if (q0 + k * NT < G)
#pragma unroll
                    for (int i = 0; i < 5; ++i) {
                        const u64 two[2] = {wd[k][2 * i], wd[k][2 * i + 1]};
                        acc5[i] += Tag<double>::unpack(two);
                    }
        }
        if (__syncthreads_or(bad)) {
            if (threadIdx.x == 0) st_agent(error, (int)OPF_EHANG);
            return;
        }
#pragma unroll
        for (int i = 0; i < 5; ++i) acc5[i] = wave_total(acc5[i]);
        if (lane == 0)
#pragma unroll
            for (int i = 0; i < 5; ++i) rred[wv][i] = acc5[i];
        __syncthreads();
        if (threadIdx.x == 0) {
            double S[5] = {0, 0, 0, 0, 0};
            for (int q = 0; q < NT / 64; ++q)
#pragma unroll
                for (int i = 0; i < 5; ++i) S[i] += rred[q][i];
            const double rho_u = ADAPT ? ld_agent(&ctrl->rho[u % kRhoRing]) : v.rho_d;
            const double pres = sqrt(S[0]);
            const double dres = rho_u * sqrt(S[1]);
            const double ep = v.eps_rel * fmax(sqrt(S[2]), sqrt(S[3]));
            const double ed = v.eps_rel * sqrt(S[4]);
            if (ADAPT) {
                // penalty of iteration u + kRhoLag, visible before the decision of u is
                const double nxt = rho_decide(v.rule, ld_agent(&ctrl->rho[(u + kRhoLag - 1) % kRhoRing]), u,
                                              pres, dres, ep, ed);
                st_agent(&ctrl->rho[(u + kRhoLag) % kRhoRing], nxt);
                drain_memory();
            }
            if (u - 1 < v.hist_cap) {
                v.hist[(u - 1) * 4 + 0] = pres;
                v.hist[(u - 1) * 4 + 1] = dres;
                v.hist[(u - 1) * 4 + 2] = ep;
                v.hist[(u - 1) * 4 + 3] = ed;
            }
            int end = 1, finished = 1, status = OPF_OK;
            if (!(isfinite(pres) && isfinite(dres) && isfinite(ep) && isfinite(ed))) {
                status = OPF_ENUMERIC;
            } else if (v.check && pres <= ep && dres <= ed) {
                status = OPF_OK;
            } else if (u >= v.max_iter) {
                status = v.check ? OPF_NOT_CONVERGED : OPF_OK;
            } else if (u >= t0 + v.chunk) {
                finished = 0;                      // pause
            } else {
                end = 0;
            }
            if (end) {
                ctrl->iter = u;
                ctrl->status = status;
                ctrl->res[0] = pres;
                ctrl->res[1] = dres;
                ctrl->res[2] = ep;
                ctrl->res[3] = ed;
                ctrl->stop = finished;
                st_agent(v.dec_stop, u);
                drain_memory();          // the end iteration is visible before dec_iter reaches it
            }
            st_agent(v.dec_iter, u);
            rstop = end;
        }
        __syncthreads();
        if (rstop) return;
    }
}

template <typename T>
__device__ __forceinline__ InstanceView<T> view_of(const IterArgs<T>& a, const PersistArgs& p) {
    InstanceView<T> v;
    v.F = a.F; v.winfo = a.winfo; v.var = a.var; v.meta = a.meta; v.cstart = a.cstart; v.ccnt = a.ccnt;
    v.clist = a.clist; v.bbar = a.bbar; v.lo = a.lo; v.hi = a.hi; v.cost = a.cost;
    v.z0 = a.z0; v.z1 = a.z1; v.l0 = a.l0; v.l1 = a.l1; v.x0 = a.x0; v.x1 = a.x1;
    v.pub = p.pub; v.records = p.records; v.dec_iter = p.dec_iter; v.dec_stop = p.dec_stop;
    v.ctrl = a.ctrl; v.hist = a.hist; v.hist_cap = a.hist_cap; v.waves = a.waves; v.check = p.check;
    v.lds_factors = p.lds_factors; v.rho = a.rho; v.inv_rho = a.inv_rho; v.rho_d = a.rho_d;
    v.eps_rel = a.eps_rel; v.rule = a.rule; v.local_updates = a.local_updates; v.max_iter = p.max_iter;
    v.chunk = 0x3fffffffffffffffll;
    return v;
}

}  // namespace opf
