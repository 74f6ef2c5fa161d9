// C-ABI of the batched same-topology path (K load scenarios sharing A_s).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/opf_admm.h"
#include "metrics.h"
#include "tune_cache.h"
#include "admm_batch.h"
#include "admm_kernels.h"
#include "opf_layout.h"


using namespace opf;

namespace {
std::mutex g_berr_mu;
std::string g_batch_setup_err;
}  // namespace

constexpr int kMaxGroups = 4;

struct opf_admm_batch {
    opf_admm_options opt;
    hipStream_t user_stream = nullptr;
    hipStream_t stream = nullptr;
    HostLayout lay;
    int K = 0, Kp = 0, LP = 0, terms = 3;
    std::vector<void*> bufs;
    size_t device_bytes = 0;
    double setup_ms = 0;
    std::string err;
    uint16_t* Fp = nullptr;
    int* wave_var = nullptr;        // per wavefront: index among the scenario-varying wavefronts, or -1
    float* Fv = nullptr;            // per-scenario factors of the varying wavefronts
    int fv_cols = 0;
    int vary_waves = 0;             // end of the prefix of wavefronts holding the varying components
    int *sdesc = nullptr, *scopy = nullptr, *meta = nullptr, *clist = nullptr;   // see BatchArgs
    float *sval = nullptr, *bbar = nullptr;
    float* z[2] = {nullptr, nullptr};
    float* l[2] = {nullptr, nullptr};
    float* x[2] = {nullptr, nullptr};
    double* part = nullptr;
    double* z0 = nullptr;
    double* c = nullptr;
    BatchCtrl* ctrl = nullptr;          // [kMaxGroups] one control block per scenario group
    BatchCtrl* ctrl_host = nullptr;     // [kMaxGroups] pinned copies
    int* state = nullptr;
    long long* iters = nullptr;
    double* res = nullptr;
    double* objective = nullptr;
    double* xout = nullptr;
    // Scenario groups: the 64-scenario chunks split into `groups` contiguous
    // ranges, each iterated by its own launches on its own stream (streams[0]
    // is the handle's stream), so that one group's launch fills the compute
    // units the other's ending launch leaves idle.  Scenarios are independent:
    // every grouping computes the same values.
    int groups = 1;
    hipStream_t streams[kMaxGroups] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kMaxGroups] = {};
    hipGraphExec_t graph[kMaxGroups] = {};
    int graph_k = 0, graph_groups = 0, graph_order = -1;
    int order = 1;                  // workgroup order of the step kernel (BatchArgs::order)
};

namespace {

int berr(opf_admm_batch* h, int code, const std::string& m) {
    if (h) h->err = m;
    else {
        std::lock_guard<std::mutex> lk(g_berr_mu);
        g_batch_setup_err = m;
    }
    return code;
}

#define BHIP(expr)                                                                         \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess) return berr(h, OPF_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

template <typename P>
int balloc(opf_admm_batch* h, P** out, size_t count) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(count * sizeof(P), 256);
    if (hipMalloc(&p, bytes) != hipSuccess) return berr(h, OPF_ENOMEM, "hipMalloc failed");
    h->bufs.push_back(p);
    h->device_bytes += bytes;
    *out = static_cast<P*>(p);
    return 0;
}

template <typename P, typename Q>
int bupload(opf_admm_batch* h, P** out, const std::vector<Q>& src) {
    std::vector<P> tmp(src.begin(), src.end());
    int rc = balloc(h, out, std::max<size_t>(tmp.size(), 1));
    if (rc) return rc;
    if (!tmp.empty()) BHIP(hipMemcpyAsync(*out, tmp.data(), tmp.size() * sizeof(P), hipMemcpyHostToDevice, h->stream));
    BHIP(hipStreamSynchronize(h->stream));
    return 0;
}

// Chunks [c0, c0 + nc) and scenarios [k0, k0 + kn) of group g of G.
void group_range(const opf_admm_batch* h, int g, int G, int* c0, int* nc, int* k0, int* kn) {
    const int KB = h->Kp / 64;
    const int a = g * KB / G, b = (g + 1) * KB / G;
    *c0 = a;
    *nc = b - a;
    *k0 = a * 64;
    *kn = std::min(h->K, b * 64) - a * 64;
}

void args_of(opf_admm_batch* h, BatchArgs& a, BatchRedArgs& r) {
    a.Fp = h->Fp; a.terms = h->terms;
    a.wave_var = h->wave_var; a.Fv = h->Fv; a.fv_cols = h->fv_cols; a.vary_waves = h->vary_waves;
    a.sdesc = reinterpret_cast<const int4*>(h->sdesc); a.sval = reinterpret_cast<const float4*>(h->sval);
    a.scopy = reinterpret_cast<const int4*>(h->scopy); a.meta = h->meta; a.clist = h->clist; a.bbar = h->bbar;
    a.z0 = h->z[0]; a.z1 = h->z[1]; a.l0 = h->l[0]; a.l1 = h->l[1]; a.x0 = h->x[0]; a.x1 = h->x[1];
    a.part = h->part; a.ctrl = h->ctrl;
    a.W = h->lay.waves; a.Kp = h->Kp; a.K = h->K; a.n = h->lay.n;
    a.rho = (float)h->opt.rho; a.inv_rho = (float)(1.0 / h->opt.rho);
    a.order = h->order;
    a.c0 = 0; a.nc = h->Kp / 64;
    r.k0 = 0;
    r.part = h->part; r.ctrl = h->ctrl; r.state = h->state; r.iters = h->iters; r.res = h->res;
    r.objective = h->objective; r.xout = h->xout; r.x0 = h->x[0]; r.x1 = h->x[1]; r.c = h->c;
    r.W = h->lay.waves; r.Kp = h->Kp; r.K = h->K; r.n = h->lay.n;
    r.rho = h->opt.rho; r.eps_rel = h->opt.eps_rel;
}

// Arguments of group g of G; *kn receives its scenario count.
void group_args(opf_admm_batch* h, int g, int G, BatchArgs& a, BatchRedArgs& r, int* kn) {
    args_of(h, a, r);
    int c0, nc, k0;
    group_range(h, g, G, &c0, &nc, &k0, kn);
    a.c0 = c0; a.nc = nc; a.ctrl = h->ctrl + g;
    r.k0 = k0; r.ctrl = h->ctrl + g;
}

// The extra streams of groups 1.. wait for the handle's stream (fork), and
// the handle's stream for all of them (join).
int fork_groups(opf_admm_batch* h, int G) {
    BHIP(hipEventRecord(h->fork, h->stream));
    for (int g = 1; g < G; ++g) BHIP(hipStreamWaitEvent(h->streams[g], h->fork, 0));
    return 0;
}
int join_groups(opf_admm_batch* h, int G) {
    for (int g = 1; g < G; ++g) {
        BHIP(hipEventRecord(h->join[g], h->streams[g]));
        BHIP(hipStreamWaitEvent(h->stream, h->join[g], 0));
    }
    return 0;
}

// One graph of k iterations per group of G, captured on the group's stream
// for the current workgroup order; kept until k, G or the order change.
int build_graphs(opf_admm_batch* h, int G, int k) {
    if (h->graph_k == k && h->graph_groups == G && h->graph_order == h->order) return 0;
    for (auto& gr : h->graph)
        if (gr) { (void)hipGraphExecDestroy(gr); gr = nullptr; }
    h->graph_k = 0;                     // no valid graphs until every group's is built
    for (int g = 0; g < G; ++g) {
        BatchArgs a;
        BatchRedArgs rr;
        int kn = 0;
        group_args(h, g, G, a, rr, &kn);
        hipGraph_t gph = nullptr;
        BHIP(hipStreamBeginCapture(h->streams[g], hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < k; ++i) {
            hipError_t e = launch_batch_iteration(a, rr, kn, h->streams[g]);
            if (e != hipSuccess) {
                (void)hipStreamEndCapture(h->streams[g], &gph);
                if (gph) (void)hipGraphDestroy(gph);
                return berr(h, OPF_EHIP, std::string("launch during capture: ") + hipGetErrorString(e));
            }
        }
        BHIP(hipStreamEndCapture(h->streams[g], &gph));
        hipError_t e = hipGraphInstantiate(&h->graph[g], gph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gph);
        if (e != hipSuccess) return berr(h, OPF_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    h->graph_k = k;
    h->graph_groups = G;
    h->graph_order = h->order;
    return 0;
}

}  // namespace

// Autotuner of the batched iteration: each workgroup order of the step
// kernel (XCD-contiguous or hardware order, wavefront- or chunk-major) with
// each number of scenario groups on concurrent streams (1, 2, 4, at most one
// per 64-scenario chunk) is timed as the solve runs it, over two replays of
// each group's graph of 32 iterations after one untimed replay, on this
// problem, in two passes over all candidates (its faster pass counts),
// and the fastest kept; decisions are cached per problem shape and kernel
// revision (tune_cache.h).  All choices compute the same values.
constexpr int kTuneGraph = 32;          // iterations per group graph while tuning
int tune_batch(opf_admm_batch* h) {
    const std::string key = "batch/r" + std::to_string(kBatchKernelRev) + "/" + std::to_string(h->lay.waves) + "/" + std::to_string(h->Kp) + "/" +
                            std::to_string(h->terms) + "/" + std::to_string(h->vary_waves) + "/" +
                            std::to_string(h->lay.L) + "/" + std::to_string(h->lay.sum_ns2);
    std::vector<int> got;
    const int KB = h->Kp / 64;
    if (tune_cache_get(key, got) && got.size() == 2 && got[1] >= 1 && got[1] <= std::min(KB, kMaxGroups)) {
        h->order = got[0];
        h->groups = got[1];
        return 0;
    }
    struct Events {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } ev;
    BHIP(hipEventCreate(&ev.e0));
    BHIP(hipEventCreate(&ev.e1));
    // two passes: one alone leaves choices a few per cent apart to noise
    const int orders[4] = {1, 0, 3, 2};
    const int group_counts[3] = {1, 2, 4};
    float t_best[3][4];
    for (auto& row : t_best)
        for (float& v : row) v = 1e30f;
    for (int pass = 0; pass < 2; ++pass)
    for (int gi = 0; gi < 3; ++gi) {
        const int G = group_counts[gi];
        if (G > std::min(KB, kMaxGroups)) continue;
        for (int oi = 0; oi < 4; ++oi) {
            const int order = orders[oi];
            h->order = order;
            int rc = build_graphs(h, G, kTuneGraph);
            if (rc) return rc;
            BHIP(launch_batch_init(h->z0, h->z[0], h->l[0], h->LP, h->Kp, h->ctrl, kMaxGroups, h->state, h->K,
                                   1LL << 40, h->stream));
            // as the solve runs them: one untimed replay per group, then two timed
            for (int phase = 0; phase < 2; ++phase) {
                if (phase == 1) BHIP(hipEventRecord(ev.e0, h->stream));
                if ((rc = fork_groups(h, G))) return rc;
                for (int g = 0; g < G; ++g)
                    for (int rep = 0; rep < (phase ? 2 : 1); ++rep) BHIP(hipGraphLaunch(h->graph[g], h->streams[g]));
                if ((rc = join_groups(h, G))) return rc;
            }
            BHIP(hipEventRecord(ev.e1, h->stream));
            BHIP(hipStreamSynchronize(h->stream));
            float ms = 0.0f;
            BHIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
            t_best[gi][oi] = std::min(t_best[gi][oi], ms);
        }
    }
    float best = 1e30f;
    int bo = 1, bg = 1;
    for (int gi = 0; gi < 3; ++gi)
        for (int oi = 0; oi < 4; ++oi)
            if (t_best[gi][oi] < best) {
                best = t_best[gi][oi];
                bo = orders[oi];
                bg = group_counts[gi];
            }
    h->order = bo;
    h->groups = bg;
    tune_cache_put(key, {bo, bg});
    return 0;
}

extern "C" {

int opf_admm_setup_batch(const opf_problem* p, const double* b_scen, int32_t K, const opf_admm_options* o,
                         void* hip_stream, opf_admm_batch** out) {
    return opf_admm_setup_batch_ex(p, b_scen, K, 0, nullptr, nullptr, o, hip_stream, out);
}

int opf_admm_setup_batch_ex(const opf_problem* p, const double* b_scen, int32_t K, int64_t nv, const int64_t* a_pos,
                            const double* a_scen, const opf_admm_options* o, void* hip_stream,
                            opf_admm_batch** out) {
    if (out) *out = nullptr;
    if (!p || !b_scen || !out) return berr(nullptr, OPF_EINVAL, "null argument");
    if (K < 1 || K > 4096) return berr(nullptr, OPF_EINVAL, "K must be in [1, 4096]");
    if (nv < 0 || (nv > 0 && (!a_pos || !a_scen))) return berr(nullptr, OPF_EINVAL, "bad scenario-varying A entries");
    if (p->S < 1 || !p->comp_m || !p->comp_n || !p->A_vals) return berr(nullptr, OPF_EINVAL, "incomplete problem");
    // components whose A_s changes with the scenario
    std::vector<int64_t> aoff(p->S + 1, 0);
    for (int q = 0; q < p->S; ++q) {
        if (p->comp_m[q] < 0 || p->comp_n[q] < 1) return berr(nullptr, OPF_EINVAL, "bad component size");
        aoff[q + 1] = aoff[q] + (int64_t)p->comp_m[q] * p->comp_n[q];
    }
    std::vector<int8_t> varying;
    std::vector<int> pos_comp(nv);
    if (nv > 0) {
        varying.assign(p->S, 0);
        for (int64_t j = 0; j < nv; ++j) {
            if (a_pos[j] < 0 || a_pos[j] >= aoff[p->S]) return berr(nullptr, OPF_EINVAL, "A position out of range");
            const int c = (int)(std::upper_bound(aoff.begin(), aoff.end(), a_pos[j]) - aoff.begin()) - 1;
            pos_comp[j] = c;
            varying[c] = 1;
        }
        for (int64_t q = 0; q < nv * K; ++q)
            if (!std::isfinite(a_scen[q])) return berr(nullptr, OPF_EINVAL, "non-finite scenario A entry");
    }
    opf_admm_options opt;
    if (o) opt = *o;
    else opf_admm_default_options(&opt);
    if (!(opt.rho > 0.0) || !(opt.eps_rel > 0.0) || opt.max_iter < 1)
        return berr(nullptr, OPF_EINVAL, "rho, eps_rel and max_iter must be positive");
    if (opt.rho_every != 0 || opt.local_updates > 1)
        return berr(nullptr, OPF_EINVAL, "the batched path runs Algorithm 1 with a fixed penalty "
                                         "(rho_every 0, one local update)");
    if (opt.check_every < 1) opt.check_every = 64;
    auto t0 = std::chrono::steady_clock::now();
    opf_admm_batch* h = new opf_admm_batch();
    h->opt = opt;
    h->K = K;
    h->Kp = (K + 63) / 64 * 64;
    h->terms = (opt.split_terms == 2) ? 2 : 3;
    ProblemView v;
    v.n = p->n; v.S = p->S; v.c = p->c; v.lb = p->lb; v.ub = p->ub; v.var_kind = p->var_kind;
    v.comp_m = p->comp_m; v.comp_n = p->comp_n; v.A = p->A_vals; v.b = p->b_vals ? p->b_vals : b_scen;
    v.idx = p->idx;
    h->lay.block_waves = 1;
    h->lay.comp_group = varying;
    std::string err;
    const int threads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    int rc = build_layout(v, h->lay, err, threads);
    std::vector<float> bb;
    if (!rc) rc = build_batch_rhs(v, h->lay, b_scen, K, h->Kp, bb, err, threads, nv > 0 ? &varying : nullptr);
    // per-scenario factors of the varying components (Section IV-B row
    // reduction and closed_2 for each scenario's A_s), FP32, laid out
    // [varying wave][column][lane][scenario]
    std::vector<int> wave_var;
    std::vector<float> Fv;
    if (!rc && nv > 0) {
        const HostLayout& L = h->lay;
        std::vector<int64_t> ioff(p->S + 1, 0), boff(p->S + 1, 0);
        for (int q = 0; q < p->S; ++q) {
            ioff[q + 1] = ioff[q] + p->comp_n[q];
            boff[q + 1] = boff[q] + p->comp_m[q];
        }
        wave_var.assign(L.waves, -1);
        int nvw = 0;
        for (int q = 0; q < p->S; ++q) {
            if (!varying[q]) continue;
            const int w = L.user_to_dev[ioff[q]] / 64;
            if (wave_var[w] < 0) wave_var[w] = nvw++;
            h->fv_cols = std::max(h->fv_cols, L.wave_maxn[w]);
            h->vary_waves = std::max(h->vary_waves, w + 1);
        }
        std::vector<std::vector<int64_t>> cpos(p->S);   // varying entries of each component
        for (int64_t j = 0; j < nv; ++j) cpos[pos_comp[j]].push_back(j);
        const size_t Kp = (size_t)h->Kp, C = (size_t)h->fv_cols;
        Fv.assign((size_t)nvw * C * 64 * Kp, 0.0f);
        std::vector<int> vlist;
        for (int q = 0; q < p->S; ++q)
            if (varying[q]) vlist.push_back(q);
        std::atomic<int> next(0), bad(-1);
        const int64_t M = boff[p->S];
        auto work = [&]() {
            std::vector<double> A, F, bbar;
            for (;;) {
                const int t = next.fetch_add(1);
                if (t >= (int)vlist.size() * K) break;
                const int q = vlist[t / K], k = t % K;
                const int m = p->comp_m[q], n = p->comp_n[q];
                A.assign(p->A_vals + aoff[q], p->A_vals + aoff[q + 1]);
                for (int64_t j : cpos[q]) A[a_pos[j] - aoff[q]] = a_scen[(size_t)k * nv + j];
                F.assign((size_t)n * n, 0.0);
                bbar.assign(n, 0.0);
                int rank = 0;
                if (component_factor(m, n, A.data(), b_scen + (size_t)k * M + boff[q], F.data(), bbar.data(), &rank)) {
                    bad.store(q);
                    continue;
                }
                const int d0 = L.user_to_dev[ioff[q]];
                const int vw = wave_var[d0 / 64], base = d0 % 64;
                for (int i = 0; i < n; ++i) {
                    bb[(size_t)(d0 + i) * Kp + k] = (float)bbar[i];
                    for (int jc = 0; jc < n; ++jc)
                        Fv[(((size_t)vw * C + jc) * 64 + base + i) * Kp + k] = (float)F[(size_t)i * n + jc];
                }
            }
        };
        std::vector<std::thread> pool;
        for (int tt = 1; tt < threads; ++tt) pool.emplace_back(work);
        work();
        for (auto& th : pool) th.join();
        if (bad.load() >= 0) {
            rc = OPF_EINFEASIBLE_COMPONENT;
            err = "a scenario's equations are inconsistent in component " + std::to_string(bad.load());
        }
    }
    if (rc) {
        delete h;
        return berr(nullptr, rc, err);
    }
    h->LP = h->lay.waves * 64;
    h->user_stream = (hipStream_t)hip_stream;
    auto fail = [&](int code) {
        std::string m = h->err;
        opf_admm_destroy_batch(h);
        return berr(nullptr, code, m);
    };
    // the step kernel addresses one 64-scenario chunk of the state with 32-bit byte offsets
    if ((size_t)h->LP * 256 > 0xffffffffull || (size_t)h->lay.n * 256 > 0xffffffffull)
        return fail(berr(h, OPF_EINVAL, "batched scenarios: more than 16M slots or variables"));
    if (h->user_stream) h->stream = h->user_stream;
    else if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess)
        return fail(berr(h, OPF_EHIP, "hipStreamCreate failed"));
    if (hipHostMalloc((void**)&h->ctrl_host, sizeof(BatchCtrl) * kMaxGroups, hipHostMallocDefault) != hipSuccess)
        return fail(berr(h, OPF_ENOMEM, "hipHostMalloc failed"));
    // streams of the scenario groups (default priority) and their fork / join events
    h->streams[0] = h->stream;
    for (int g = 1; g < std::min(h->Kp / 64, kMaxGroups); ++g)
        if (hipStreamCreateWithFlags(&h->streams[g], hipStreamNonBlocking) != hipSuccess)
            return fail(berr(h, OPF_EHIP, "hipStreamCreate failed"));
    if (hipEventCreateWithFlags(&h->fork, hipEventDisableTiming) != hipSuccess)
        return fail(berr(h, OPF_EHIP, "hipEventCreate failed"));
    for (int g = 1; g < kMaxGroups; ++g)
        if (hipEventCreateWithFlags(&h->join[g], hipEventDisableTiming) != hipSuccess)
            return fail(berr(h, OPF_EHIP, "hipEventCreate failed"));
    const HostLayout& L = h->lay;
    std::vector<uint16_t> planes;
    build_dense_planes(L, h->terms, planes);
    if ((rc = bupload(h, &h->Fp, planes))) return fail(rc);
    if (nv > 0) {
        if ((rc = bupload(h, &h->wave_var, wave_var))) return fail(rc);
        if ((rc = bupload(h, &h->Fv, Fv))) return fail(rc);
    }
    {
        // per-slot records of the step kernel (one 16-byte load each, no
        // dependent loads): variable, copies, copy-list offset, owner; cost and
        // bounds; the first kBatchCopies copies, then the slot itself
        const size_t LPs = (size_t)h->LP;
        std::vector<int> sd(LPs * 4, 0), sc(LPs * 8);
        std::vector<float> sv(LPs * 4, 0.0f);
        for (size_t d = 0; d < LPs; ++d) {
            const int g = L.var[d];
            const int cn = g >= 0 ? L.copy_cnt[d] : 0, cs = g >= 0 ? L.copy_start[d] : 0;
            sd[4 * d + 0] = g;
            sd[4 * d + 1] = cn;
            sd[4 * d + 2] = cs;
            sd[4 * d + 3] = g >= 0 ? (L.meta[d] >> 16) & 1 : 0;
            if (g >= 0) {
                sv[4 * d + 0] = (float)L.cost[d];
                sv[4 * d + 1] = (float)L.lo[d];
                sv[4 * d + 2] = (float)L.hi[d];
            }
            for (int q = 0; q < 8; ++q) sc[8 * d + q] = q < std::min(cn, kBatchCopies) ? L.copy_list[cs + q] : (int)d;
        }
        if ((rc = bupload(h, &h->sdesc, sd))) return fail(rc);
        if ((rc = bupload(h, &h->sval, sv))) return fail(rc);
        if ((rc = bupload(h, &h->scopy, sc))) return fail(rc);
    }
    if ((rc = bupload(h, &h->meta, L.meta))) return fail(rc);
    if ((rc = bupload(h, &h->clist, L.copy_list))) return fail(rc);
    {
        // b-bar per slot and scenario, [LP][Kp] -> chunk-major [Kp / 64][LP][64]
        const size_t LPs = (size_t)h->LP, Kp = (size_t)h->Kp;
        std::vector<float> cm(bb.size());
        for (size_t d = 0; d < LPs; ++d)
            for (size_t k = 0; k < Kp; ++k) cm[((k >> 6) * LPs + d) * 64 + (k & 63)] = bb[d * Kp + k];
        if ((rc = bupload(h, &h->bbar, cm))) return fail(rc);
    }
    if ((rc = bupload(h, &h->z0, L.z0))) return fail(rc);
    if ((rc = bupload(h, &h->c, L.c_full))) return fail(rc);
    const size_t st = (size_t)h->LP * h->Kp;
    for (int b = 0; b < 2; ++b) {
        if ((rc = balloc(h, &h->z[b], st))) return fail(rc);
        if ((rc = balloc(h, &h->l[b], st))) return fail(rc);
        if ((rc = balloc(h, &h->x[b], (size_t)L.n * h->Kp))) return fail(rc);
        if (hipMemsetAsync(h->x[b], 0, sizeof(float) * (size_t)L.n * h->Kp, h->stream) != hipSuccess)
            return fail(berr(h, OPF_EHIP, "memset"));
    }
    if ((rc = balloc(h, &h->part, (size_t)5 * h->Kp * L.waves))) return fail(rc);
    if ((rc = balloc(h, &h->ctrl, kMaxGroups))) return fail(rc);
    if ((rc = balloc(h, &h->state, K))) return fail(rc);
    if ((rc = balloc(h, &h->iters, K))) return fail(rc);
    if ((rc = balloc(h, &h->res, (size_t)4 * K))) return fail(rc);
    if ((rc = balloc(h, &h->objective, K))) return fail(rc);
    if ((rc = balloc(h, &h->xout, (size_t)K * L.n))) return fail(rc);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(berr(h, OPF_EHIP, "sync"));
    if (opt.autotune && (rc = tune_batch(h))) return fail(rc);
    h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h;
    return OPF_OK;
}

int opf_admm_solve_batch(opf_admm_batch* h, opf_batch_result* r) {
    if (!h || !r || !r->x) return berr(h, OPF_EINVAL, "null handle, result or x");
    auto t0 = std::chrono::steady_clock::now();
    if (h->user_stream != h->stream && h->user_stream) BHIP(hipStreamSynchronize(h->user_stream));
    const int G = h->groups;
    const int k = std::max(1, h->opt.check_every);
    int rc = build_graphs(h, G, k);
    if (rc) return rc;
    BHIP(launch_batch_init(h->z0, h->z[0], h->l[0], h->LP, h->Kp, h->ctrl, G, h->state, h->K, h->opt.max_iter,
                           h->stream));
    if ((rc = fork_groups(h, G))) return rc;
    bool stopped[kMaxGroups] = {};
    for (int left = G; left > 0;) {
        for (int g = 0; g < G; ++g) {
            if (stopped[g]) continue;
            BHIP(hipGraphLaunch(h->graph[g], h->streams[g]));
            BHIP(hipMemcpyAsync(h->ctrl_host + g, h->ctrl + g, sizeof(BatchCtrl), hipMemcpyDeviceToHost,
                                h->streams[g]));
        }
        for (int g = 0; g < G; ++g) {
            if (stopped[g]) continue;
            BHIP(hipStreamSynchronize(h->streams[g]));
            if (h->ctrl_host[g].stop) {
                stopped[g] = true;
                --left;
            }
        }
    }
    if ((rc = join_groups(h, G))) return rc;
    long long total = 0;
    for (int g = 0; g < G; ++g) total = std::max(total, (long long)h->ctrl_host[g].iter);
    const int K = h->K, n = h->lay.n;
    std::vector<int> st(K);
    std::vector<long long> it(K);
    std::vector<double> res((size_t)4 * K), obj(K);
    BHIP(hipMemcpyAsync(st.data(), h->state, sizeof(int) * K, hipMemcpyDeviceToHost, h->stream));
    BHIP(hipMemcpyAsync(it.data(), h->iters, sizeof(long long) * K, hipMemcpyDeviceToHost, h->stream));
    BHIP(hipMemcpyAsync(res.data(), h->res, sizeof(double) * 4 * K, hipMemcpyDeviceToHost, h->stream));
    BHIP(hipMemcpyAsync(obj.data(), h->objective, sizeof(double) * K, hipMemcpyDeviceToHost, h->stream));
    BHIP(hipMemcpyAsync(r->x, h->xout, sizeof(double) * (size_t)K * n,
                        r->outputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
    BHIP(hipStreamSynchronize(h->stream));
    int converged = 0, status = OPF_OK;
    for (int q = 0; q < K; ++q) {
        const int code = st[q] == 1 ? OPF_OK : (st[q] == 3 ? OPF_ENUMERIC : OPF_NOT_CONVERGED);
        if (st[q] == 1) ++converged;
        if (code == OPF_ENUMERIC) status = OPF_ENUMERIC;
        else if (code == OPF_NOT_CONVERGED && status == OPF_OK) status = OPF_NOT_CONVERGED;
        if (r->iterations) r->iterations[q] = it[q];
        if (r->objective) r->objective[q] = obj[q];
        if (r->status) r->status[q] = code;
        if (r->pres) r->pres[q] = res[(size_t)4 * q + 0];
        if (r->dres) r->dres[q] = res[(size_t)4 * q + 1];
        if (r->eps_prim) r->eps_prim[q] = res[(size_t)4 * q + 2];
        if (r->eps_dual) r->eps_dual[q] = res[(size_t)4 * q + 3];
    }
    r->total_iterations = total;
    r->converged = converged;
    r->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (metrics_on()) {
        // algorithmic bytes of one batch iteration: the shared FP64 factors once,
        // and per slot and scenario (FP32 state) z and lambda read and written,
        // the x gather and b-bar
        const double bytes = 8.0 * (double)h->lay.sum_ns2 + 24.0 * (double)K * (double)h->lay.L;
        JsonLine j;
        j.str("kind", "batch").integer("n", n).integer("S", h->lay.S).integer("L", h->lay.L).integer("K", K)
            .integer("status", status).integer("converged", converged).integer("total_iterations", total)
            .num("solve_ms", r->solve_ms).num("us_per_iteration", total > 0 ? 1e3 * r->solve_ms / (double)total : 0.0)
            .num("bytes_per_iteration", bytes)
            .num("effective_gbs", r->solve_ms > 0 ? bytes * (double)total / (r->solve_ms * 1e-3) / 1e9 : 0.0)
            .integer("order", h->order).integer("groups", G);
        metrics_write(j);
    }
    if (status == OPF_ENUMERIC) berr(h, OPF_ENUMERIC, "NaN/Inf in the residuals of a scenario");
    return status;
}

int opf_admm_batch_info(const opf_admm_batch* h, opf_admm_info* info) {
    if (!h || !info) return OPF_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->n = h->lay.n;
    info->S = h->lay.S;
    info->L = h->lay.L;
    info->waves = h->lay.waves;
    info->lanes = h->LP;
    info->max_ns = h->lay.max_ns;
    info->max_copies = h->lay.max_copies;
    info->sum_ns2 = h->lay.sum_ns2;
    info->factor_bytes_fp64 = (int64_t)h->lay.F.size() * 8;
    info->device_bytes = (int64_t)h->device_bytes;
    info->setup_ms = h->setup_ms;
    info->grid_blocks = h->lay.waves * (h->Kp / 64);
    info->block_waves = 4;
    info->kernel = OPF_KERNEL_STEP;
    info->batch_order = h->order;
    info->batch_groups = h->groups;
    return 0;
}

void opf_admm_destroy_batch(opf_admm_batch* h) {
    if (!h) return;
    for (int g = 0; g < kMaxGroups; ++g)
        if (h->streams[g]) (void)hipStreamSynchronize(h->streams[g]);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (auto& gr : h->graph)
        if (gr) (void)hipGraphExecDestroy(gr);
    for (void* p : h->bufs) (void)hipFree(p);
    if (h->ctrl_host) (void)hipHostFree(h->ctrl_host);
    for (int g = 1; g < kMaxGroups; ++g) {
        if (h->streams[g]) (void)hipStreamDestroy(h->streams[g]);
        if (h->join[g]) (void)hipEventDestroy(h->join[g]);
    }
    if (h->fork) (void)hipEventDestroy(h->fork);
    if (h->stream && h->stream != h->user_stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

const char* opf_admm_batch_last_error(const opf_admm_batch* h) {
    if (h) return h->err.c_str();
    std::lock_guard<std::mutex> lk(g_berr_mu);
    return g_batch_setup_err.c_str();
}

}  // extern "C"
