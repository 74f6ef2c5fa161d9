// Serving runtime: continuous batching of independent solves on one GPU.
//
// Threads: set-up workers (validation, row reduction, factors, packing of a
// submitted problem into a contiguous device image) and one GPU worker that
// admits ready solves into the device arena while their footprint (HBM) and
// their workgroups (co-resident capacity) fit, runs all resident solves in one
// persistent launch for a chunk of iterations each, polls the per-solve stop
// flags, and retires finished solves (outputs, warm-start state).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/opf_admm.h"
#include "admm_kernels.h"
#include "metrics.h"
#include "opf_layout.h"

namespace opf {
hipError_t launch_promote(const float* z32a, const float* z32b, const float* l32a, const float* l32b,
                          double* z64a, double* z64b, double* l64a, double* l64b, int LP, Ctrl* ctrl,
                          long long max_iter, int check, hipStream_t st);
}  // namespace opf

using namespace opf;

namespace {

using clk = std::chrono::steady_clock;
constexpr int kWPB = 4;              // wavefronts per workgroup of the shared launch
// factor columns per workgroup held in LDS.  FP64 (147 VGPRs, three
// workgroups per compute unit): 48 KiB.  FP32 (118 VGPRs, four workgroups per
// compute unit): 38 KiB, which with the kernel's own 1.6 KiB keeps four
// workgroups within the 160 KiB of one compute unit
constexpr int kServeLdsCols64 = 96;
constexpr int kServeLdsCols32 = 152;
constexpr size_t kAlign = 256;

size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Offsets of the arrays of one resident solve inside its arena region (the
// FP32 arrays only for mixed precision).
struct Image {
    size_t winfo, var, meta, cstart, ccnt, clist, user_slot, F, bbar, lo, hi, cost, zdef, zdef_user;
    size_t Ff, bbarf, lof, hif, costf;
    size_t z0, z1, l0, l1, x0, x1, records, pub, dec, zu, lu, xo, plan;
    size_t z0f, z1f, l0f, l1f, x0f, x1f, total;
};

struct Request {
    int64_t id = 0;
    uint64_t family = 0;
    std::vector<uint64_t> keys;
    int n = 0, S = 0;
    std::vector<double> c, lb, ub, A, b;
    std::vector<uint8_t> kind;
    std::vector<int32_t> cm, cn, idx;
    double* x_out = nullptr;
    HostLayout lay;
    int rc = 0;
    std::string err;
    Image img{};
    std::vector<unsigned char> bytes;       // static part of the region image
    std::vector<int32_t> comp_off;          // user-order offset of each component
    clk::time_point t_submit, t_admit;
};

struct WarmState {
    double* z = nullptr;
    double* l = nullptr;
    size_t L = 0;
    std::unordered_map<uint64_t, std::pair<int32_t, int32_t>> key_to;   // key -> (user offset, n_s)
    uint64_t tick = 0;
};

struct Slot {
    bool used = false;
    std::unique_ptr<Request> req;
    size_t off = 0, len = 0;
    InstDesc desc{};
    int warm = 0;
    int fp32 = 0;            // 1: in the FP32 bulk phase of a mixed-precision solve
    int waiting = 0;         // 1: bulk phase done, waiting for room in the FP64 launch
    long long it32 = 0;      // iterations of the bulk phase
    double q_prev = 0;       // stall watch of the bulk phase: residual ratio at the last check
    long long next_check = 0;
};

// First-fit allocator over one device buffer (offsets).
struct Arena {
    size_t size = 0;
    std::map<size_t, size_t> free_;          // offset -> length
    size_t used = 0;
    void init(size_t s) { size = s; free_.clear(); free_[0] = s; used = 0; }
    bool alloc(size_t len, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= len) {
                *off = it->first;
                const size_t rest = it->second - len;
                const size_t noff = it->first + len;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                used += len;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t len) {
        used -= len;
        auto it = free_.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

Image plan_image(const HostLayout& L, bool mixed) {
    Image im{};
    const size_t LP = (size_t)L.waves * kWave;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t r = o; o += up(std::max<size_t>(bytes, 1)); return r; };
    im.winfo = take(sizeof(int2) * L.waves);
    im.var = take(4 * LP);
    im.meta = take(4 * LP);
    im.cstart = take(4 * LP);
    im.ccnt = take(4 * LP);
    im.clist = take(4 * (size_t)L.L);
    im.user_slot = take(4 * LP);
    im.F = take(8 * L.F.size());
    im.bbar = take(8 * LP);
    im.lo = take(8 * LP);
    im.hi = take(8 * LP);
    im.cost = take(8 * LP);
    im.zdef = take(8 * LP);
    im.zdef_user = take(8 * (size_t)L.L);
    const size_t h = mixed ? 1 : 0;
    im.Ff = take(h * 4 * L.F.size());
    im.bbarf = take(h * 4 * LP);
    im.lof = take(h * 4 * LP);
    im.hif = take(h * 4 * LP);
    im.costf = take(h * 4 * LP);
    const size_t static_end = o;
    im.z0 = take(8 * LP);
    im.z1 = take(8 * LP);
    im.l0 = take(8 * LP);
    im.l1 = take(8 * LP);
    im.x0 = take(8 * (size_t)L.n);
    im.x1 = take(8 * (size_t)L.n);
    im.records = take(8 * 10 * (size_t)L.blocks * kDecisionLag);
    im.pub = take(8 * 2 * 2 * LP);
    im.dec = take(16);
    im.zu = take(8 * (size_t)L.L);
    im.lu = take(8 * (size_t)L.L);
    im.xo = take(8 * (size_t)L.n);
    im.plan = take(16 * (size_t)L.S);
    im.z0f = take(h * 4 * LP);
    im.z1f = take(h * 4 * LP);
    im.l0f = take(h * 4 * LP);
    im.l1f = take(h * 4 * LP);
    im.x0f = take(h * 4 * (size_t)L.n);
    im.x1f = take(h * 4 * (size_t)L.n);
    im.total = o;
    (void)static_end;
    return im;
}

template <typename T>
void put(std::vector<unsigned char>& buf, size_t off, const std::vector<T>& v) {
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(T));
}

// FP32 copy (round to nearest) of an FP64 array.
void put_narrow(std::vector<unsigned char>& buf, size_t off, const std::vector<double>& v) {
    float* d = reinterpret_cast<float*>(buf.data() + off);
    for (size_t i = 0; i < v.size(); ++i) d[i] = (float)v[i];
}

}  // namespace

struct opf_server {
    opf_server_options opt;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    unsigned char* arena_base = nullptr;
    Arena arena;
    InstDesc* d_descs = nullptr;
    int2* d_work = nullptr;
    Ctrl* d_ctrls = nullptr;
    Ctrl* h_ctrls = nullptr;
    int2* h_work = nullptr;
    int work_cap = 0;                      // entries of h_work / d_work
    int nwork = 0;
    int* d_error = nullptr;
    int* h_error = nullptr;
    bool mixed = false;                    // FP32 bulk phase + FP64 polish
    int cap32 = 0, cap64 = 0;              // co-resident workgroups of the FP32 / FP64 serving kernel
    std::vector<Slot> slots;
    int active = 0;                        // resident solves
    int blocks32 = 0, blocks64 = 0;        // workgroups (reducers included) in the FP32 / FP64 launch
    int nwork32 = 0;                       // the FP32 launch's items come first in the work list
    bool dirty = true;
    std::mutex mu;
    std::condition_variable cv_setup, cv_work, cv_result;
    std::deque<std::unique_ptr<Request>> submitted, ready;
    std::set<int64_t> live;                // submitted and not yet answered
    std::set<int64_t> cancel;              // cancellations of requests in set-up or resident
    std::deque<opf_served> results;
    std::map<uint64_t, WarmState> warm;
    size_t warm_used = 0;
    uint64_t tick = 0;
    std::atomic<bool> quit{false};
    std::vector<std::thread> setup_threads;
    std::thread worker;
    std::string err;
    int64_t next_id = 1, n_submitted = 0, n_completed = 0, n_rejected = 0, launches = 0;
    double busy_ms = 0;
};

namespace {

std::mutex g_serr_mu;
std::string g_server_err;

int serr(opf_server* s, int code, const std::string& m) {
    if (s) s->err = m;
    else {
        std::lock_guard<std::mutex> lk(g_serr_mu);
        g_server_err = m;
    }
    return code;
}

double ms_since(clk::time_point a, clk::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

void push_result(opf_server* s, Request& r, int status, const Ctrl* c, int warm_comps, long long it32 = 0) {
    opf_served o{};
    o.request_id = r.id;
    o.status = status;
    o.warm_components = warm_comps;
    o.x = r.x_out;
    const auto now = clk::now();
    o.latency_ms = ms_since(r.t_submit, now);
    o.queue_ms = r.t_admit.time_since_epoch().count() ? ms_since(r.t_submit, r.t_admit) : o.latency_ms;
    if (c) {
        o.iterations = c->iter;
        o.iterations_fp32 = it32;
        o.pres = c->res[0];
        o.dres = c->res[1];
        o.eps_prim = c->res[2];
        o.eps_dual = c->res[3];
        double obj = 0.0;
        for (int i = 0; i < r.n; ++i) obj += r.c[i] * r.x_out[i];
        o.objective = obj;
    }
    if (metrics_on()) {
        JsonLine j;
        j.str("kind", "served").integer("request_id", o.request_id).integer("family", (long long)r.family)
            .integer("n", r.n).integer("S", r.S).integer("status", status).integer("warm_components", warm_comps)
            .integer("iterations", o.iterations).integer("iterations_fp32", o.iterations_fp32)
            .num("objective", o.objective).num("pres", o.pres).num("dres", o.dres).num("eps_prim", o.eps_prim)
            .num("eps_dual", o.eps_dual).num("queue_ms", o.queue_ms).num("latency_ms", o.latency_ms);
        metrics_write(j);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->results.push_back(o);
        s->live.erase(r.id);
        s->cancel.erase(r.id);
        if (status < 0) s->n_rejected++;
        else s->n_completed++;
    }
    s->cv_result.notify_all();
}

void setup_loop(opf_server* s) {
    for (;;) {
        std::unique_ptr<Request> r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_setup.wait(lk, [&] { return s->quit.load() || !s->submitted.empty(); });
            if (s->quit.load()) return;
            r = std::move(s->submitted.front());
            s->submitted.pop_front();
        }
        ProblemView v;
        v.n = r->n; v.S = r->S; v.c = r->c.data(); v.lb = r->lb.data(); v.ub = r->ub.data();
        v.var_kind = r->kind.data(); v.comp_m = r->cm.data(); v.comp_n = r->cn.data(); v.A = r->A.data();
        v.b = r->b.data(); v.idx = r->idx.data();
        r->lay.block_waves = kWPB;
        r->rc = build_layout(v, r->lay, r->err, 1);
        if (!r->rc) {
            const HostLayout& L = r->lay;
            r->img = plan_image(L, s->mixed);
            if (r->img.total > s->arena.size) {
                r->rc = OPF_ENOMEM;
                r->err = "footprint larger than the arena";
            } else {
                Image& im = r->img;
                r->bytes.assign(im.z0, 0);
                std::vector<int2> wi(L.waves);
                for (int w = 0; w < L.waves; ++w) wi[w] = make_int2(L.wave_maxn[w], (int)(L.wave_foff[w] / kWave));
                put(r->bytes, im.winfo, wi);
                put(r->bytes, im.var, L.var);
                put(r->bytes, im.meta, L.meta);
                put(r->bytes, im.cstart, L.copy_start);
                put(r->bytes, im.ccnt, L.copy_cnt);
                put(r->bytes, im.clist, L.copy_list);
                put(r->bytes, im.user_slot, L.user_slot);
                put(r->bytes, im.F, L.F);
                put(r->bytes, im.bbar, L.bbar);
                put(r->bytes, im.lo, L.lo);
                put(r->bytes, im.hi, L.hi);
                put(r->bytes, im.cost, L.cost);
                put(r->bytes, im.zdef, L.z0);
                std::vector<double> zu(L.L, 0.0);
                for (size_t d = 0; d < L.user_slot.size(); ++d)
                    if (L.user_slot[d] >= 0) zu[L.user_slot[d]] = L.z0[d];
                put(r->bytes, im.zdef_user, zu);
                if (s->mixed) {
                    put_narrow(r->bytes, im.Ff, L.F);
                    put_narrow(r->bytes, im.bbarf, L.bbar);
                    put_narrow(r->bytes, im.lof, L.lo);
                    put_narrow(r->bytes, im.hif, L.hi);
                    put_narrow(r->bytes, im.costf, L.cost);
                }
                r->comp_off.assign(r->S, 0);
                for (int q = 1; q < r->S; ++q) r->comp_off[q] = r->comp_off[q - 1] + r->cn[q - 1];
            }
        }
        if (r->rc) {
            push_result(s, *r, r->rc, nullptr, 0);
            continue;
        }
        bool cancelled;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            cancelled = s->cancel.count(r->id) > 0;
            if (!cancelled) s->ready.push_back(std::move(r));
        }
        if (cancelled) {
            push_result(s, *r, OPF_ECANCELED, nullptr, 0);
            continue;
        }
        s->cv_work.notify_all();
    }
}

// ---- GPU worker ---------------------------------------------------------------

#define SHIP(expr)                                                                      \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess) {                                                         \
            serr(s, OPF_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));       \
            return false;                                                               \
        }                                                                               \
    } while (0)

#define SHIPI(expr)                                                                     \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess) {                                                         \
            serr(s, OPF_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));       \
            return -1;                                                                  \
        }                                                                               \
    } while (0)

void evict_for(opf_server* s, size_t need) {
    while (s->warm_used + need > (size_t)s->opt.warm_bytes && !s->warm.empty()) {
        auto victim = s->warm.begin();
        for (auto it = s->warm.begin(); it != s->warm.end(); ++it)
            if (it->second.tick < victim->second.tick) victim = it;
        (void)hipFree(victim->second.z);
        (void)hipFree(victim->second.l);
        s->warm_used -= 16 * victim->second.L;
        s->warm.erase(victim);
    }
}

int admit_one(opf_server* s, std::unique_ptr<Request>& r, int slot_id) {
    Request& q = *r;
    const HostLayout& L = q.lay;
    size_t off = 0;
    if (!s->arena.alloc(q.img.total, &off)) return 0;
    Slot& sl = s->slots[slot_id];
    unsigned char* base = s->arena_base + off;
    SHIPI(hipMemcpyAsync(base, q.bytes.data(), q.bytes.size(), hipMemcpyHostToDevice, s->stream));
    const Image& im = q.img;
    InstDesc D{};
    D.winfo = reinterpret_cast<const int2*>(base + im.winfo);
    D.var = reinterpret_cast<const int*>(base + im.var);
    D.meta = reinterpret_cast<const int*>(base + im.meta);
    D.cstart = reinterpret_cast<const int*>(base + im.cstart);
    D.ccnt = reinterpret_cast<const int*>(base + im.ccnt);
    D.clist = reinterpret_cast<const int*>(base + im.clist);
    D.user_slot = reinterpret_cast<const int*>(base + im.user_slot);
    D.F = reinterpret_cast<const double*>(base + im.F);
    D.bbar = reinterpret_cast<const double*>(base + im.bbar);
    D.lo = reinterpret_cast<const double*>(base + im.lo);
    D.hi = reinterpret_cast<const double*>(base + im.hi);
    D.cost = reinterpret_cast<const double*>(base + im.cost);
    D.z0 = reinterpret_cast<double*>(base + im.z0);
    D.z1 = reinterpret_cast<double*>(base + im.z1);
    D.l0 = reinterpret_cast<double*>(base + im.l0);
    D.l1 = reinterpret_cast<double*>(base + im.l1);
    D.x0 = reinterpret_cast<double*>(base + im.x0);
    D.x1 = reinterpret_cast<double*>(base + im.x1);
    if (s->mixed) {
        D.Ff = reinterpret_cast<const float*>(base + im.Ff);
        D.bbarf = reinterpret_cast<const float*>(base + im.bbarf);
        D.lof = reinterpret_cast<const float*>(base + im.lof);
        D.hif = reinterpret_cast<const float*>(base + im.hif);
        D.costf = reinterpret_cast<const float*>(base + im.costf);
        D.z0f = reinterpret_cast<float*>(base + im.z0f);
        D.z1f = reinterpret_cast<float*>(base + im.z1f);
        D.l0f = reinterpret_cast<float*>(base + im.l0f);
        D.l1f = reinterpret_cast<float*>(base + im.l1f);
        D.x0f = reinterpret_cast<float*>(base + im.x0f);
        D.x1f = reinterpret_cast<float*>(base + im.x1f);
    }
    D.records = reinterpret_cast<unsigned long long*>(base + im.records);
    D.pub = reinterpret_cast<unsigned long long*>(base + im.pub);
    D.dec = reinterpret_cast<long long*>(base + im.dec);
    D.ctrl = s->d_ctrls + slot_id;
    D.blocks = L.blocks;
    D.lanes = L.waves * kWave;
    D.n = L.n;
    D.rho = s->opt.admm.rho;
    D.eps_rel = s->opt.admm.eps_rel;
    SHIPI(hipMemcpyAsync(s->d_descs + slot_id, &D, sizeof(InstDesc), hipMemcpyHostToDevice, s->stream));
    // start point: default, or resident state of the family for matching components
    int warm_comps = 0;
    double* zu = reinterpret_cast<double*>(base + im.zu);
    double* lu = reinterpret_cast<double*>(base + im.lu);
    auto wit = s->warm.end();
    if (s->opt.warm_start && !q.keys.empty()) wit = s->warm.find(q.family);
    if (wit != s->warm.end()) {
        std::vector<int4> plan;
        for (int c = 0; c < q.S; ++c) {
            auto f = wit->second.key_to.find(q.keys[c]);
            if (f != wit->second.key_to.end() && f->second.second == q.cn[c])
                plan.push_back(make_int4(f->second.first, q.comp_off[c], q.cn[c], 0));
        }
        warm_comps = (int)plan.size();
        wit->second.tick = ++s->tick;
        if (warm_comps) {
            int4* dplan = reinterpret_cast<int4*>(base + im.plan);
            SHIPI(hipMemcpyAsync(zu, reinterpret_cast<double*>(base + im.zdef_user), 8 * (size_t)L.L,
                                hipMemcpyDeviceToDevice, s->stream));
            SHIPI(hipMemsetAsync(lu, 0, 8 * (size_t)L.L, s->stream));
            SHIPI(hipMemcpyAsync(dplan, plan.data(), sizeof(int4) * plan.size(), hipMemcpyHostToDevice, s->stream));
            SHIPI(launch_warm_gather(dplan, (int)plan.size(), wit->second.z, wit->second.l, zu, lu, s->stream));
        }
    }
    SHIPI(launch_to_device_order(zu, lu, D.user_slot, D.lanes, reinterpret_cast<const double*>(base + im.zdef),
                                D.z0, D.l0, warm_comps > 0 ? 1 : 0, s->stream));
    SHIPI(launch_multi_init(s->d_descs, slot_id, D.lanes, s->opt.admm.max_iter, s->mixed ? 1 : 0, s->stream));
    s->h_ctrls[slot_id] = Ctrl{};              // no round has run for this solve yet
    sl.used = true;
    sl.off = off;
    sl.len = q.img.total;
    sl.desc = D;
    sl.warm = warm_comps;
    sl.fp32 = s->mixed ? 1 : 0;
    sl.waiting = 0;
    sl.it32 = 0;
    sl.q_prev = HUGE_VAL;
    sl.next_check = OPF_MIXED_STALL_WINDOW;
    q.t_admit = clk::now();
    sl.req = std::move(r);
    s->active++;
    (s->mixed ? s->blocks32 : s->blocks64) += L.blocks + 1;
    s->dirty = true;
    return 1;
}

bool admit_ready(opf_server* s) {
    std::deque<std::unique_ptr<Request>> cand, keep;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        cand.swap(s->ready);
    }
    // offer order (requests left waiting keep their arrival order)
    std::vector<size_t> order(cand.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    if (s->opt.admission == OPF_ADMIT_LARGEST_FIRST)
        std::stable_sort(order.begin(), order.end(),
                         [&](size_t a, size_t b) { return cand[a]->lay.blocks > cand[b]->lay.blocks; });
    std::vector<char> waiting(cand.size(), 0);
    // starvation guard: the largest request that has waited max_wait_ms and
    // does not fit, when only smaller solves hold the capacity it needs
    const int limit_run = std::min(s->opt.max_workgroups, s->mixed ? s->cap32 : s->cap64);
    const int used_run = s->mixed ? s->blocks32 : s->blocks64;
    const Request* hold_for = nullptr;
    if (s->opt.max_wait_ms > 0) {
        const auto now = clk::now();
        for (auto& r : cand) {
            const int need = r->lay.blocks + 1;
            if (used_run + need <= limit_run || need > limit_run || ms_since(r->t_submit, now) < s->opt.max_wait_ms)
                continue;
            if (!hold_for || need > hold_for->lay.blocks + 1) hold_for = r.get();
        }
        if (hold_for) {
            const int need = hold_for->lay.blocks + 1;
            int smaller = 0;                      // capacity held by smaller solves of the same launch
            for (const Slot& sl : s->slots)
                if (sl.used && !sl.waiting && (sl.fp32 != 0) == s->mixed && sl.desc.blocks + 1 < need)
                    smaller += sl.desc.blocks + 1;
            if (limit_run - used_run + smaller < need) hold_for = nullptr;   // larger solves block it: no hold
        }
    }
    for (size_t oi : order) {
        auto& r = cand[oi];
        if (hold_for && r.get() != hold_for) {
            waiting[oi] = 1;
            continue;
        }
        int free_slot = -1;
        for (int q = 0; q < (int)s->slots.size(); ++q)
            if (!s->slots[q].used) { free_slot = q; break; }
        const int need = r->lay.blocks + 1;        // compute workgroups + reducer
        // every phase of the solve must be able to run: the FP64 launch (plain
        // solves, polish) and, for mixed precision, the FP32 launch
        const int limit64 = std::min(s->opt.max_workgroups, s->cap64);
        const int limit32 = std::min(s->opt.max_workgroups, s->cap32);
        if (need > limit64 || (s->mixed && need > limit32)) {
            push_result(s, *r, OPF_ENOMEM, nullptr, 0);   // can never be co-resident on this device
            continue;
        }
        const bool room = s->mixed ? s->blocks32 + need <= limit32 : s->blocks64 + need <= limit64;
        int rc = 0;
        if (free_slot >= 0 && room)
            rc = admit_one(s, r, free_slot);
        if (rc < 0) {
            push_result(s, *r, OPF_EHIP, nullptr, 0);   // device failure: report and drop
            continue;
        }
        if (rc == 0) waiting[oi] = 1;                      // no room now; later ones may fit
    }
    for (size_t i = 0; i < cand.size(); ++i)
        if (waiting[i]) keep.push_back(std::move(cand[i]));
    if (!keep.empty()) {
        std::lock_guard<std::mutex> lk(s->mu);
        while (!keep.empty()) {
            s->ready.push_front(std::move(keep.back()));
            keep.pop_back();
        }
    }
    return true;
}

bool retire(opf_server* s, int slot_id) {
    Slot& sl = s->slots[slot_id];
    Request& q = *sl.req;
    const HostLayout& L = q.lay;
    const Ctrl c = s->h_ctrls[slot_id];
    unsigned char* base = s->arena_base + sl.off;
    double* xo = reinterpret_cast<double*>(base + q.img.xo);
    // resident state of the family for later warm starts
    WarmState ws;
    ws.L = L.L;
    double* zo = reinterpret_cast<double*>(base + q.img.zu);
    double* lo = reinterpret_cast<double*>(base + q.img.lu);
    bool keep = s->opt.warm_start && !q.keys.empty() && c.status >= 0 &&
                16 * (size_t)L.L <= (size_t)s->opt.warm_bytes;
    if (keep) {
        auto old = s->warm.find(q.family);
        if (old != s->warm.end()) {
            (void)hipFree(old->second.z);
            (void)hipFree(old->second.l);
            s->warm_used -= 16 * old->second.L;
            s->warm.erase(old);
        }
        evict_for(s, 16 * (size_t)L.L);
        if (hipMalloc(&ws.z, 8 * (size_t)L.L) != hipSuccess || hipMalloc(&ws.l, 8 * (size_t)L.L) != hipSuccess) {
            if (ws.z) (void)hipFree(ws.z);
            keep = false;
        } else {
            zo = ws.z;
            lo = ws.l;
        }
    }
    SHIP(launch_multi_output(s->d_descs, slot_id, xo, zo, lo, sl.fp32, s->stream));
    SHIP(hipMemcpyAsync(q.x_out, xo, 8 * (size_t)L.n, hipMemcpyDeviceToHost, s->stream));
    SHIP(hipStreamSynchronize(s->stream));
    if (keep) {
        for (int cc = 0; cc < q.S; ++cc) ws.key_to[q.keys[cc]] = {q.comp_off[cc], q.cn[cc]};
        ws.tick = ++s->tick;
        s->warm_used += 16 * ws.L;
        s->warm[q.family] = std::move(ws);
    }
    push_result(s, q, c.status, &c, sl.warm, sl.fp32 ? c.iter : sl.it32);
    s->arena.release(sl.off, sl.len);
    s->active--;
    if (!sl.waiting) (sl.fp32 ? s->blocks32 : s->blocks64) -= L.blocks + 1;
    sl.waiting = 0;
    sl.used = false;
    sl.req.reset();
    s->dirty = true;
    return true;
}

// A mixed-precision solve whose FP32 bulk phase has ended moves to the FP64
// launch for the polish phase (the FP32 state of its last iteration widened,
// as in the single-instance solver) once that launch has room; until then it
// waits outside both launches.
bool promote(opf_server* s, int q) {
    Slot& sl = s->slots[q];
    const InstDesc& D = sl.desc;
    const int need = D.blocks + 1;
    if (!sl.waiting) {
        s->blocks32 -= need;
        sl.it32 = s->h_ctrls[q].iter;
        sl.waiting = 1;
        s->dirty = true;
    }
    if (s->blocks64 + need > std::min(s->opt.max_workgroups, s->cap64)) return true;
    SHIP(launch_promote(D.z0f, D.z1f, D.l0f, D.l1f, D.z0, D.z1, D.l0, D.l1, D.lanes, D.ctrl,
                        sl.it32 + s->opt.admm.max_iter, 1, s->stream));
    sl.fp32 = 0;
    sl.waiting = 0;
    s->blocks64 += need;
    s->dirty = true;
    return true;
}

// Work list: the FP32 launch's items, then the FP64 launch's.
bool upload_work(opf_server* s) {
    int nw = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int q = 0; q < (int)s->slots.size(); ++q) {
            const Slot& sl = s->slots[q];
            if (!sl.used || sl.waiting || sl.fp32 != (pass == 0 ? 1 : 0)) continue;
            if (nw + sl.desc.blocks + 1 > s->work_cap) {
                serr(s, OPF_EHIP, "work list overflow");
                return false;
            }
            for (int b = 0; b <= sl.desc.blocks; ++b) s->h_work[nw++] = make_int2(q, b);
        }
        if (pass == 0) s->nwork32 = nw;
    }
    s->nwork = nw;
    if (hipMemcpyAsync(s->d_work, s->h_work, sizeof(int2) * std::max(nw, 1), hipMemcpyHostToDevice, s->stream) !=
        hipSuccess) {
        serr(s, OPF_EHIP, "work list upload failed");
        return false;
    }
    s->dirty = false;
    return true;
}

void worker_loop(opf_server* s) {
    ServeArgs sa{};
    sa.error = s->d_error;
    sa.spin_limit = s->opt.admm.spin_limit > 0 ? s->opt.admm.spin_limit : 4000000LL;
    sa.chunk = std::max(1, s->opt.iters_per_poll);
    sa.xcd_remap = s->opt.admm.workgroup_order == 1 ? 1 : 0;
    ServeArgs sa32 = sa;
    sa.lds_cols = kServeLdsCols64;
    sa32.lds_cols = kServeLdsCols32;
    const bool polish = s->opt.admm.polish != 0;
    const bool watch = s->mixed && polish && s->opt.admm.eps_rel < OPF_MIXED_STALL_BELOW;
    for (;;) {
        if (s->quit.load()) return;
        admit_ready(s);
        // cancelled resident solves end before the round with their current iterate
        std::vector<int64_t> cids;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            cids.assign(s->cancel.begin(), s->cancel.end());
        }
        for (int q = 0; q < (int)s->slots.size() && !cids.empty(); ++q) {
            Slot& sl = s->slots[q];
            if (!sl.used || !std::binary_search(cids.begin(), cids.end(), sl.req->id)) continue;
            s->h_ctrls[q].status = OPF_ECANCELED;
            if (!retire(s, q)) return;
        }
        if (s->active == 0) {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait_for(lk, std::chrono::milliseconds(2),
                                [&] { return s->quit.load() || !s->ready.empty(); });
            continue;
        }
        if (s->dirty && !upload_work(s)) return;
        const auto t0 = clk::now();
        const int n64 = s->nwork - s->nwork32;
        // the two launches run one after the other on the stream; a hang in
        // the first leaves the error flag set and the second ends early
        bool ok = hipMemsetAsync(s->d_error, 0, sizeof(int), s->stream) == hipSuccess;
        if (ok && s->nwork32 > 0)
            ok = launch_serve_persistent(s->d_descs, s->d_work, s->nwork32, sa32, 1, s->stream) == hipSuccess;
        if (ok && n64 > 0)
            ok = launch_serve_persistent(s->d_descs, s->d_work + s->nwork32, n64, sa, 0, s->stream) == hipSuccess;
        if (!ok ||
            hipMemcpyAsync(s->h_ctrls, s->d_ctrls, sizeof(Ctrl) * s->slots.size(), hipMemcpyDeviceToHost,
                           s->stream) != hipSuccess ||
            hipMemcpyAsync(s->h_error, s->d_error, sizeof(int), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
            hipStreamSynchronize(s->stream) != hipSuccess) {
            serr(s, OPF_EHIP, "shared iteration launch failed");
            return;
        }
        s->busy_ms += ms_since(t0, clk::now());
        s->launches += 1;
        const bool hang = *s->h_error != 0;
        for (int q = 0; q < (int)s->slots.size(); ++q) {
            Slot& sl = s->slots[q];
            if (!sl.used) continue;
            if (hang) {
                s->h_ctrls[q].status = OPF_EHANG;           // a bounded wait ran out: end every resident solve
                if (!retire(s, q)) return;
                continue;
            }
            const Ctrl& c = s->h_ctrls[q];
            bool stalled = false;
            if (watch && sl.fp32 && !sl.waiting && !c.stop && c.iter >= sl.next_check) {
                // the bulk phase's stall watch, as in the single-instance solver
                const double r = std::max(c.res[0] / c.res[2], c.res[1] / c.res[3]);
                if (!(r < 0.5 * sl.q_prev)) stalled = true;
                sl.q_prev = r;
                sl.next_check += OPF_MIXED_STALL_WINDOW;
            }
            if (!sl.waiting && !c.stop && !stalled) continue;
            if (sl.fp32 && polish && s->h_ctrls[q].status != OPF_ENUMERIC) {
                if (!promote(s, q)) return;
            } else if (!sl.waiting) {
                if (!retire(s, q)) return;
            }
        }
    }
}

}  // namespace

extern "C" {

void opf_server_default_options(opf_server_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    opf_admm_default_options(&o->admm);
    o->arena_bytes = (int64_t)4 << 30;
    o->warm_bytes = (int64_t)1 << 30;
    o->max_slots = 256;
    o->max_workgroups = 8192;
    o->iters_per_poll = 256;
    o->setup_threads = 4;
    o->warm_start = 1;
    o->admission = OPF_ADMIT_LARGEST_FIRST;
    o->max_wait_ms = 500;
}

int opf_server_create(const opf_server_options* o, void* hip_stream, opf_server** out) {
    if (out) *out = nullptr;
    if (!out) return serr(nullptr, OPF_EINVAL, "null output");
    opf_server_options opt;
    if (o) opt = *o;
    else opf_server_default_options(&opt);
    if (!(opt.admm.rho > 0) || !(opt.admm.eps_rel > 0) || opt.admm.max_iter < 1 || opt.arena_bytes < (1 << 20) ||
        opt.max_slots < 1 || opt.max_workgroups < 1 || opt.iters_per_poll < 1 ||
        (opt.admission != OPF_ADMIT_LARGEST_FIRST && opt.admission != OPF_ADMIT_ARRIVAL) || opt.max_wait_ms < 0 ||
        (opt.admm.precision != OPF_PREC_FP64 && opt.admm.precision != OPF_PREC_MIXED))
        return serr(nullptr, OPF_EINVAL, "invalid server options");
    if (opt.admm.rho_every != 0 || opt.admm.local_updates > 1)
        return serr(nullptr, OPF_EINVAL, "served solves run Algorithm 1 with a fixed penalty "
                                         "(rho_every 0, one local update)");
    auto s = std::make_unique<opf_server>();
    s->opt = opt;
    if (opt.setup_threads < 1) s->opt.setup_threads = 1;
    if (hip_stream) s->stream = (hipStream_t)hip_stream;
    else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
            return serr(nullptr, OPF_EHIP, "hipStreamCreate failed");
        s->own_stream = true;
    }
    auto fail = [&](int code, const char* m) {
        opf_server* raw = s.release();
        opf_server_destroy(raw);
        return serr(nullptr, code, m);
    };
    if (hipMalloc((void**)&s->arena_base, (size_t)opt.arena_bytes) != hipSuccess) return fail(OPF_ENOMEM, "arena allocation failed");
    s->arena.init((size_t)opt.arena_bytes);
    // work list: up to max_workgroups items in each of the two launches of a round
    const int MS = opt.max_slots, MW = 2 * opt.max_workgroups;
    if (hipMalloc((void**)&s->d_descs, sizeof(InstDesc) * MS) != hipSuccess ||
        hipMalloc((void**)&s->d_work, sizeof(int2) * MW) != hipSuccess ||
        hipMalloc((void**)&s->d_error, sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&s->d_ctrls, sizeof(Ctrl) * MS) != hipSuccess)
        return fail(OPF_ENOMEM, "device allocation failed");
    if (hipHostMalloc((void**)&s->h_ctrls, sizeof(Ctrl) * MS, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&s->h_work, sizeof(int2) * MW, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&s->h_error, sizeof(int), hipHostMallocDefault) != hipSuccess)
        return fail(OPF_ENOMEM, "pinned allocation failed");
    s->work_cap = MW;
    *s->h_error = 0;
    if (hipMemsetAsync(s->d_error, 0, sizeof(int), s->stream) != hipSuccess ||
        hipMemsetAsync(s->d_ctrls, 0, sizeof(Ctrl) * MS, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return fail(OPF_EHIP, "device initialisation failed");
    s->mixed = opt.admm.precision == OPF_PREC_MIXED;
    s->cap64 = serve_capacity((size_t)kServeLdsCols64 * 64 * sizeof(double), 0);
    s->cap32 = s->mixed ? serve_capacity((size_t)kServeLdsCols32 * 64 * sizeof(float), 1) : 0;
    if (s->cap64 < 2 || (s->mixed && s->cap32 < 2))
        return fail(OPF_EHIP, "the serving kernel cannot be resident on this device");
    s->slots.resize(MS);
    opf_server* raw = s.release();
    for (int t = 0; t < raw->opt.setup_threads; ++t) raw->setup_threads.emplace_back(setup_loop, raw);
    raw->worker = std::thread(worker_loop, raw);
    *out = raw;
    return OPF_OK;
}

int opf_server_submit(opf_server* s, const opf_problem* p, uint64_t family, const uint64_t* comp_keys,
                      double* x_out, int64_t* request_id) {
    if (!s || !p || !x_out) return serr(s, OPF_EINVAL, "null argument");
    if (p->n < 1 || p->S < 1 || !p->c || !p->lb || !p->ub || !p->comp_m || !p->comp_n || !p->A_vals ||
        !p->b_vals || !p->idx)
        return serr(s, OPF_EINVAL, "incomplete problem");
    auto r = std::make_unique<Request>();
    r->family = family;
    r->n = p->n;
    r->S = p->S;
    r->x_out = x_out;
    r->c.assign(p->c, p->c + p->n);
    r->lb.assign(p->lb, p->lb + p->n);
    r->ub.assign(p->ub, p->ub + p->n);
    if (p->var_kind) r->kind.assign(p->var_kind, p->var_kind + p->n);
    else r->kind.assign(p->n, 0);
    r->cm.assign(p->comp_m, p->comp_m + p->S);
    r->cn.assign(p->comp_n, p->comp_n + p->S);
    int64_t na = 0, nb = 0, ni = 0;
    for (int q = 0; q < p->S; ++q) {
        if (p->comp_m[q] < 0 || p->comp_n[q] < 1 || p->comp_n[q] > 64) return serr(s, OPF_EINVAL, "bad component size");
        na += (int64_t)p->comp_m[q] * p->comp_n[q];
        nb += p->comp_m[q];
        ni += p->comp_n[q];
    }
    r->A.assign(p->A_vals, p->A_vals + na);
    r->b.assign(p->b_vals, p->b_vals + nb);
    r->idx.assign(p->idx, p->idx + ni);
    if (comp_keys) r->keys.assign(comp_keys, comp_keys + p->S);
    r->t_submit = clk::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->id = s->next_id++;
        if (request_id) *request_id = r->id;
        s->live.insert(r->id);
        s->n_submitted++;
        s->submitted.push_back(std::move(r));
    }
    s->cv_setup.notify_one();
    return OPF_OK;
}

int opf_server_cancel(opf_server* s, int64_t request_id) {
    if (!s) return serr(s, OPF_EINVAL, "null server");
    std::unique_ptr<Request> hit;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->live.count(request_id)) return serr(s, OPF_EINVAL, "unknown or already answered request");
        for (auto* dq : {&s->submitted, &s->ready}) {
            for (auto it = dq->begin(); it != dq->end(); ++it)
                if ((*it)->id == request_id) {
                    hit = std::move(*it);
                    dq->erase(it);
                    break;
                }
            if (hit) break;
        }
        if (!hit) s->cancel.insert(request_id);       // in set-up or resident: ended by its owner thread
    }
    if (hit) push_result(s, *hit, OPF_ECANCELED, nullptr, 0);
    return OPF_OK;
}

int opf_server_poll(opf_server* s, opf_served* out, int max_out, int wait_ms) {
    if (!s || !out || max_out < 1) return serr(s, OPF_EINVAL, "bad poll arguments");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->results.empty() && wait_ms > 0)
        s->cv_result.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->results.empty(); });
    int k = 0;
    while (k < max_out && !s->results.empty()) {
        out[k++] = s->results.front();
        s->results.pop_front();
    }
    return k;
}

int opf_server_get_stats(const opf_server* sc, opf_server_stats* st) {
    opf_server* s = const_cast<opf_server*>(sc);
    if (!s || !st) return OPF_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    st->submitted = s->n_submitted;
    st->completed = s->n_completed;
    st->rejected = s->n_rejected;
    st->resident = s->active;
    st->queued = (int32_t)(s->submitted.size() + s->ready.size());
    st->arena_used = (int64_t)s->arena.used;
    st->arena_bytes = (int64_t)s->arena.size;
    st->warm_used = (int64_t)s->warm_used;
    st->launches = s->launches;
    st->busy_ms = s->busy_ms;
    return 0;
}

void opf_server_destroy(opf_server* s) {
    if (!s) return;
    s->quit.store(true);
    s->cv_setup.notify_all();
    s->cv_work.notify_all();
    for (auto& t : s->setup_threads)
        if (t.joinable()) t.join();
    if (s->worker.joinable()) s->worker.join();
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto& w : s->warm) {
        (void)hipFree(w.second.z);
        (void)hipFree(w.second.l);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    if (s->d_descs) (void)hipFree(s->d_descs);
    if (s->d_work) (void)hipFree(s->d_work);
    if (s->d_error) (void)hipFree(s->d_error);
    if (s->d_ctrls) (void)hipFree(s->d_ctrls);
    if (s->h_ctrls) (void)hipHostFree(s->h_ctrls);
    if (s->h_work) (void)hipHostFree(s->h_work);
    if (s->h_error) (void)hipHostFree(s->h_error);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

const char* opf_server_last_error(const opf_server* s) {
    if (s) return s->err.c_str();
    std::lock_guard<std::mutex> lk(g_serr_mu);
    return g_server_err.c_str();
}

}  // extern "C"
