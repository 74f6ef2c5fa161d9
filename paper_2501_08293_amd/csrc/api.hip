// C-ABI implementation: handle life cycle, device buffers, solve drivers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/opf_admm.h"
#include "admm_kernels.h"
#include "setup_device.h"
#include "metrics.h"
#include "tune_cache.h"
#include "opf_layout.h"

namespace opf {
template <typename T> hipError_t launch_step(const IterArgs<T>& a, int wpb, hipStream_t st);
template <typename T>
hipError_t launch_init(const double* z0, const double* lam0, T* z, T* l, int LP, Ctrl* ctrl,
                       long long max_iter, int check, double rho0, hipStream_t st);
hipError_t launch_promote(const float* z32a, const float* z32b, const float* l32a, const float* l32b,
                          double* z64a, double* z64b, double* l64a, double* l64b, int LP, Ctrl* ctrl,
                          long long max_iter, int check, hipStream_t st);
hipError_t launch_rearm(Ctrl* ctrl, long long max_iter, int check, hipStream_t st);
size_t step_partials_count(int G);
template <typename T>
hipError_t launch_persistent(const IterArgs<T>& a, PersistArgs p, int wpb, int G, hipStream_t st);
template <typename T> int persistent_capacity(int wpb, size_t lds_bytes, int adapt);
template <typename T>
hipError_t launch_tiled(const IterArgs<T>& a, PersistArgs p, const TiledArgs& ta, int wpb, int G, hipStream_t st);
template <typename T> int tiled_capacity(int wpb, int pair, size_t lds_bytes = 0);
template <typename T>
hipError_t launch_output(const T* z0, const T* z1, const T* l0, const T* l1, const T* x0, const T* x1,
                         const int* user_slot, int LP, int n, const double* c, double* xo, double* zo,
                         double* lo, Ctrl* ctrl, hipStream_t st);
}  // namespace opf

using namespace opf;

static_assert(kRhoLag == OPF_RHO_LAG, "the balancing lag of the kernels is the one the header states");

namespace {

std::mutex g_err_mu;
std::string g_setup_err;
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, int>> g_tune;   // problem shape -> (schedule, workgroup waves)

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Per-precision device state and static per-slot data.
template <typename T>
struct PrecState {
    T* F = nullptr;
    T* bbar = nullptr;
    T* lo = nullptr;
    T* hi = nullptr;
    T* cost = nullptr;
    T* z[2] = {nullptr, nullptr};
    T* l[2] = {nullptr, nullptr};
    T* x[2] = {nullptr, nullptr};
    T* zr = nullptr;                 // tiled schedule: state of the last kStateRing iterations
    T* lr = nullptr;
    T* xr = nullptr;
};

// Scratch of the iteration kernels: the step kernel's residual partials and
// arrival counters, the persistent kernel's published terms, residual
// records, decision words and error flag.  A handle owns one set; the
// allocation-free solve points the kernels at the static device array instead.
struct Work {
    double* partials = nullptr;
    unsigned long long* pub = nullptr;     // published copy terms [2][LP][2] (tagged words)
    unsigned long long* records = nullptr; // persistent residual records [lag][10][blocks]
    long long* dec_iter = nullptr;
    long long* dec_stop = nullptr;
    int* dev_error = nullptr;
    bool graphs = true;                    // step schedule: replay captured graphs (false: direct launches)
};

}  // namespace

struct opf_admm_handle {
    opf_admm_options opt;
    hipStream_t user_stream = nullptr;
    hipStream_t stream = nullptr;   // private stream; calls are synchronous
    int device = 0;
    HostLayout lay;
    int LP = 0;
    std::vector<DevBuf> bufs;
    // static layout on device
    int2* winfo = nullptr;
    int* var = nullptr;
    int* meta = nullptr;
    int* cstart = nullptr;
    int* ccnt = nullptr;
    int* clist = nullptr;
    int* user_slot = nullptr;
    int* user_to_dev = nullptr;
    double* z0 = nullptr;          // default initial local copies (device order)
    double* c = nullptr;           // [n]
    double* warm_z = nullptr;      // staging for warm starts (device order)
    double* warm_l = nullptr;
    double* user_z = nullptr;      // staging for user-order inputs/outputs
    double* user_l = nullptr;
    double* xo = nullptr;          // FP64 x output staging [n]
    double* partials = nullptr;
    double* hist = nullptr;
    Ctrl* ctrl = nullptr;
    Ctrl* ctrl_host = nullptr;     // pinned
    PrecState<double> s64;
    PrecState<float> s32;
    bool has32 = false;
    int wpb = 4;
    int grid_blocks = 0;
    size_t device_bytes = 0;
    double setup_ms = 0;
    long long last_iter = 0;
    int last_prec = OPF_PREC_FP64;
    std::string err;
    // graph of `check_every` step launches per precision
    hipGraphExec_t graph64 = nullptr, graph32 = nullptr;
    int graph_k = 0;
    // persistent schedule
    int kernel = OPF_KERNEL_STEP;
    int capacity = 0;
    int tiled_G = 0;               // tiled schedule: compute workgroups of the FP64 kernel (tiles = lay.blocks)
    int tiled_G32 = 0;             // and of the FP32 kernel
    int tiled_pair64 = 0, tiled_pair32 = 0;   // the two-tile kernel runs (per precision)
    int tiled_lds64 = 0, tiled_lds32 = 0;     // its factor column budget in LDS (0: factors from memory)
    Work work;                     // the handle's own kernel scratch
    int xcd_remap = 1;
    int* error_host = nullptr;     // pinned
    double* devF = nullptr;        // factors from the device set-up (FP64, packed), else null
    double* devBbar = nullptr;
    int64_t devF_count = 0;
    int lds_cols = 0;              // factor columns of the largest workgroup
    int lds32 = 0, lds64 = 0;      // factors in LDS: FP32 all (1) or none; FP64 column budget (0: none)
    int lds64_cols = 0;            // dynamic LDS columns of the FP64 launch
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double kernel_ms = 0;          // device time of iteration kernels in the current solve
    long long kernel_launches = 0;
};

namespace {

int set_err(opf_admm_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    else {
        std::lock_guard<std::mutex> lk(g_err_mu);
        g_setup_err = msg;
    }
    return code;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t _e = (expr);                                                           \
        if (_e != hipSuccess)                                                             \
            return set_err(h, OPF_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

template <typename P>
int dalloc(opf_admm_handle* h, P** out, size_t count) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(count * sizeof(P), 256);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return set_err(h, OPF_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    h->bufs.push_back({p, bytes});
    h->device_bytes += bytes;
    *out = static_cast<P*>(p);
    return 0;
}

template <typename P, typename Q>
int upload(opf_admm_handle* h, P** out, const std::vector<Q>& src) {
    std::vector<P> tmp(src.begin(), src.end());
    int rc = dalloc(h, out, std::max<size_t>(tmp.size(), 1));
    if (rc) return rc;
    if (!tmp.empty()) HIPCHK(hipMemcpyAsync(*out, tmp.data(), tmp.size() * sizeof(P), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return 0;
}

template <typename T>
int make_prec(opf_admm_handle* h, PrecState<T>& s) {
    const HostLayout& L = h->lay;
    int rc;
    if (h->devF) {
        // factors computed by the device set-up (FP64); narrowed for FP32
        if (sizeof(T) == 8) {
            s.F = reinterpret_cast<T*>(h->devF);
            s.bbar = reinterpret_cast<T*>(h->devBbar);
        } else {
            if ((rc = dalloc(h, &s.F, (size_t)h->devF_count))) return rc;
            if ((rc = dalloc(h, &s.bbar, (size_t)h->LP))) return rc;
            HIPCHK(launch_narrow(h->devF, reinterpret_cast<float*>(s.F), h->devF_count, h->stream));
            HIPCHK(launch_narrow(h->devBbar, reinterpret_cast<float*>(s.bbar), h->LP, h->stream));
        }
    } else {
        if ((rc = upload(h, &s.F, L.F))) return rc;
        if ((rc = upload(h, &s.bbar, L.bbar))) return rc;
    }
    if ((rc = upload(h, &s.lo, L.lo))) return rc;
    if ((rc = upload(h, &s.hi, L.hi))) return rc;
    if ((rc = upload(h, &s.cost, L.cost))) return rc;
    if (h->kernel == OPF_KERNEL_TILED) {
        if ((rc = dalloc(h, &s.zr, (size_t)kStateRing * h->LP))) return rc;
        if ((rc = dalloc(h, &s.lr, (size_t)kStateRing * h->LP))) return rc;
        if ((rc = dalloc(h, &s.xr, (size_t)kStateRing * L.n))) return rc;
    }
    for (int b = 0; b < 2; ++b) {
        if ((rc = dalloc(h, &s.z[b], h->LP))) return rc;
        if ((rc = dalloc(h, &s.l[b], h->LP))) return rc;
        if ((rc = dalloc(h, &s.x[b], L.n))) return rc;
        HIPCHK(hipMemsetAsync(s.z[b], 0, sizeof(T) * h->LP, h->stream));
        HIPCHK(hipMemsetAsync(s.l[b], 0, sizeof(T) * h->LP, h->stream));
        HIPCHK(hipMemsetAsync(s.x[b], 0, sizeof(T) * L.n, h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return 0;
}

template <typename T>
IterArgs<T> iter_args(opf_admm_handle* h, PrecState<T>& s, const Work& w) {
    IterArgs<T> a;
    a.F = s.F;
    a.winfo = h->winfo;
    a.var = h->var;
    a.meta = h->meta;
    a.cstart = h->cstart;
    a.ccnt = h->ccnt;
    a.clist = h->clist;
    a.bbar = s.bbar;
    a.lo = s.lo;
    a.hi = s.hi;
    a.cost = s.cost;
    a.z0 = s.z[0];
    a.z1 = s.z[1];
    a.l0 = s.l[0];
    a.l1 = s.l[1];
    a.x0 = s.x[0];
    a.x1 = s.x[1];
    a.partials = w.partials;
    a.ctrl = h->ctrl;
    a.hist = h->hist;
    a.hist_cap = h->opt.history_cap;
    a.waves = h->lay.waves;
    a.rho = (T)(h->opt.local_updates * h->opt.rho);    // dual step length
    a.inv_rho = (T)(1.0 / h->opt.rho);
    a.local_updates = (double)h->opt.local_updates;
    a.rho_d = h->opt.rho;
    a.eps_rel = h->opt.eps_rel;
    a.rule = RhoRule{h->opt.rho_every, h->opt.rho_mode, h->opt.rho_mu, h->opt.rho_tau, h->opt.rho_min,
                     h->opt.rho_max};
    return a;
}

// Captures `k` consecutive step launches into an executable graph.
template <typename T>
int capture_steps(opf_admm_handle* h, PrecState<T>& s, int k, hipGraphExec_t* out) {
    IterArgs<T> a = iter_args(h, s, h->work);
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < k; ++i) {
        hipError_t e = launch_step<T>(a, h->wpb, h->stream);
        if (e != hipSuccess) {
            (void)hipStreamEndCapture(h->stream, &g);
            if (g) (void)hipGraphDestroy(g);
            return set_err(h, OPF_EHIP, std::string("launch during capture: ") + hipGetErrorString(e));
        }
    }
    HIPCHK(hipStreamEndCapture(h->stream, &g));
    hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return set_err(h, OPF_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return 0;
}

// Runs step launches until the device stop flag is set.  Returns 0 or error.
// Without graphs the `check_every` launches between host checks are issued
// one by one (nothing is instantiated).
template <typename T>
int run_phase(opf_admm_handle* h, PrecState<T>& s, hipGraphExec_t* graph, const Work& w) {
    const int k = std::max(1, h->opt.check_every);
    if (!w.graphs) {
        const IterArgs<T> a = iter_args(h, s, w);
        const long long before = h->ctrl_host->iter;
        for (;;) {
            HIPCHK(hipEventRecord(h->ev0, h->stream));
            for (int i = 0; i < k; ++i) HIPCHK(launch_step<T>(a, h->wpb, h->stream));
            HIPCHK(hipEventRecord(h->ev1, h->stream));
            HIPCHK(hipMemcpyAsync(h->ctrl_host, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
            h->kernel_ms += ms;
            if (h->ctrl_host->stop) break;
        }
        h->kernel_launches += h->ctrl_host->iter - before;
        return 0;
    }
    if (!*graph || h->graph_k != k) {
        if (*graph) { (void)hipGraphExecDestroy(*graph); *graph = nullptr; }
        int rc = capture_steps(h, s, k, graph);
        if (rc) return rc;
        h->graph_k = k;
    }
    const long long before = h->ctrl_host->iter;
    long long t_prev = -1;
    for (;;) {
        HIPCHK(hipEventRecord(h->ev0, h->stream));
        HIPCHK(hipGraphLaunch(*graph, h->stream));
        HIPCHK(hipEventRecord(h->ev1, h->stream));
        HIPCHK(hipMemcpyAsync(h->ctrl_host, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
        h->kernel_ms += ms;
        if (h->ctrl_host->stop) break;
        t_prev = h->ctrl_host->iter;
    }
    (void)t_prev;
    h->kernel_launches += h->ctrl_host->iter - before;
    return 0;
}

template <typename T>
int run_phase_persistent(opf_admm_handle* h, PrecState<T>& s, long long max_iter, int check, const Work& w) {
    IterArgs<T> a = iter_args(h, s, w);
    PersistArgs p;
    p.pub = w.pub;
    p.records = w.records;
    p.dec_iter = w.dec_iter;
    p.dec_stop = w.dec_stop;
    p.error = w.dev_error;
    p.xcd_remap = h->xcd_remap;
    p.spin_limit = h->opt.spin_limit > 0 ? h->opt.spin_limit : 4000000LL;
    p.max_iter = max_iter;
    p.check = check;
    p.lds_factor_cols = sizeof(T) == 8 ? h->lds64_cols : h->lds_cols;
    p.lds_factors = sizeof(T) == 8 ? h->lds64 : h->lds32;
    HIPCHK(hipEventRecord(h->ev0, h->stream));
    HIPCHK(launch_persistent<T>(a, p, h->wpb, h->lay.blocks, h->stream));
    HIPCHK(hipEventRecord(h->ev1, h->stream));
    HIPCHK(hipMemcpyAsync(h->ctrl_host, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(h->error_host, w.dev_error, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    h->kernel_ms += ms;
    h->kernel_launches += 1;
    if (*h->error_host) {
        h->ctrl_host->status = OPF_EHANG;
        return set_err(h, OPF_EHANG, "a bounded device-side wait ran out in the persistent kernel");
    }
    return 0;
}

template <typename T>
int run_phase_tiled(opf_admm_handle* h, PrecState<T>& s, long long max_iter, int check, const Work& w) {
    IterArgs<T> a = iter_args(h, s, w);
    PersistArgs p;
    p.pub = w.pub;
    p.records = w.records;
    p.dec_iter = w.dec_iter;
    p.dec_stop = w.dec_stop;
    p.error = w.dev_error;
    p.xcd_remap = 0;
    p.spin_limit = h->opt.spin_limit > 0 ? h->opt.spin_limit : 4000000LL;
    p.max_iter = max_iter;
    p.check = check;
    p.lds_factor_cols = 0;
    p.lds_factors = 0;
    TiledArgs ta;
    ta.zr = s.zr;
    ta.lr = s.lr;
    ta.xr = s.xr;
    ta.tiles = h->lay.blocks;
    ta.n = h->lay.n;
    ta.pair = sizeof(T) == 4 ? h->tiled_pair32 : h->tiled_pair64;
    ta.lds_cols = sizeof(T) == 4 ? h->tiled_lds32 : h->tiled_lds64;
    HIPCHK(hipEventRecord(h->ev0, h->stream));
    HIPCHK(launch_tiled<T>(a, p, ta, h->wpb, sizeof(T) == 4 ? h->tiled_G32 : h->tiled_G, h->stream));
    HIPCHK(hipEventRecord(h->ev1, h->stream));
    HIPCHK(hipMemcpyAsync(h->ctrl_host, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(h->error_host, w.dev_error, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    h->kernel_ms += ms;
    h->kernel_launches += 1;
    if (*h->error_host) {
        h->ctrl_host->status = OPF_EHANG;
        return set_err(h, OPF_EHANG, "a bounded device-side wait ran out in the tiled persistent kernel");
    }
    return 0;
}

template <typename T>
int run_any(opf_admm_handle* h, PrecState<T>& s, hipGraphExec_t* graph, long long max_iter, int check,
            const Work& w) {
    if (h->kernel == OPF_KERNEL_PERSISTENT) return run_phase_persistent<T>(h, s, max_iter, check, w);
    if (h->kernel == OPF_KERNEL_TILED) return run_phase_tiled<T>(h, s, max_iter, check, w);
    return run_phase<T>(h, s, graph, w);
}

template <typename T>
int finish_outputs(opf_admm_handle* h, PrecState<T>& s, opf_result* r) {
    const int n = h->lay.n, L = h->lay.L;
    double* xo = r->outputs_on_device ? r->x : h->xo;
    double* zo = r->z ? (r->outputs_on_device ? r->z : h->user_z) : nullptr;
    double* lo = r->lam ? (r->outputs_on_device ? r->lam : h->user_l) : nullptr;
    HIPCHK(launch_output<T>(s.z[0], s.z[1], s.l[0], s.l[1], s.x[0], s.x[1], h->user_slot, h->LP, n, h->c, xo,
                            zo, lo, h->ctrl, h->stream));
    HIPCHK(hipMemcpyAsync(h->ctrl_host, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    if (!r->outputs_on_device) {
        HIPCHK(hipMemcpyAsync(r->x, h->xo, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
        if (r->z) HIPCHK(hipMemcpyAsync(r->z, h->user_z, sizeof(double) * L, hipMemcpyDeviceToHost, h->stream));
        if (r->lam) HIPCHK(hipMemcpyAsync(r->lam, h->user_l, sizeof(double) * L, hipMemcpyDeviceToHost, h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return 0;
}

__global__ void scatter_user_kernel(const double* zu, const double* lu, const int* user_to_dev, int L,
                                    double* zd, double* ld) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u < L) {
        const int d = user_to_dev[u];
        zd[d] = zu[u];
        ld[d] = lu[u];
    }
}

// Start point in device order (default or warm), as FP64 arrays.
int prepare_start(opf_admm_handle* h, const opf_warm* warm, const double** z0, const double** l0) {
    if (!warm) {
        *z0 = h->z0;
        *l0 = nullptr;
        return 0;
    }
    if (!warm->z || !warm->lam) return set_err(h, OPF_EINVAL, "warm start needs both z and lam");
    const int L = h->lay.L;
    const double* zu = warm->z;
    const double* lu = warm->lam;
    if (!warm->on_device) {
        HIPCHK(hipMemcpyAsync(h->user_z, warm->z, sizeof(double) * L, hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->user_l, warm->lam, sizeof(double) * L, hipMemcpyHostToDevice, h->stream));
        zu = h->user_z;
        lu = h->user_l;
    }
    HIPCHK(hipMemsetAsync(h->warm_z, 0, sizeof(double) * h->LP, h->stream));
    HIPCHK(hipMemsetAsync(h->warm_l, 0, sizeof(double) * h->LP, h->stream));
    hipLaunchKernelGGL(scatter_user_kernel, dim3((L + 255) / 256), dim3(256), 0, h->stream, zu, lu,
                       h->user_to_dev, L, h->warm_z, h->warm_l);
    HIPCHK(hipGetLastError());
    *z0 = h->warm_z;
    *l0 = h->warm_l;
    return 0;
}

// The metrics record of one solve (OPF_ADMM_METRICS): sizes, schedule,
// status, iterations, residuals, times, the iteration rate and the effective
// rate of the algorithmic bytes of the bulk precision; with a residual history
// on the device, up to 64 evenly spaced (pres, dres) pairs of it.
void record_solve(opf_admm_handle* h, const opf_result* r, const char* kind) {
    const HostLayout& L = h->lay;
    const bool mixed = h->opt.precision == OPF_PREC_MIXED;
    const double e = mixed ? 4.0 : 8.0;
    const double bytes = e * (double)L.sum_ns2 + (7 * e + 8) * (double)L.L + (4 * e + 4) * (double)L.n;
    const long long it_bulk = mixed ? r->iterations_fp32 : r->iterations;
    const double ms_bulk = mixed ? r->kernel_ms_fp32 : r->kernel_ms;
    static const char* kname[] = {"auto", "step", "persistent", "tiled"};
    JsonLine j;
    j.str("kind", kind).integer("n", L.n).integer("S", L.S).integer("L", L.L)
        .str("precision", mixed ? "mixed" : "fp64").str("kernel", kname[std::min(std::max(h->kernel, 0), 3)])
        .integer("block_waves", h->wpb).integer("status", r->status).integer("iterations", r->iterations)
        .integer("iterations_fp32", r->iterations_fp32).num("objective", r->objective).num("pres", r->pres)
        .num("dres", r->dres).num("eps_prim", r->eps_prim).num("eps_dual", r->eps_dual)
        .num("rho_final", r->rho_final).num("solve_ms", r->solve_ms).num("kernel_ms", r->kernel_ms)
        .num("iters_per_s", r->solve_ms > 0 ? 1e3 * (double)r->iterations / r->solve_ms : 0.0)
        .num("bytes_per_iteration", bytes)
        .num("effective_gbs", ms_bulk > 0 ? bytes * (double)it_bulk / (ms_bulk * 1e-3) / 1e9 : 0.0);
    const long long rows = std::min<long long>(h->opt.history_cap, r->iterations);
    if (rows > 0) {
        std::vector<double> hb((size_t)rows * 4);
        if (hipMemcpyAsync(hb.data(), h->hist, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, h->stream) ==
                hipSuccess && hipStreamSynchronize(h->stream) == hipSuccess) {
            std::vector<std::pair<double, double>> hs;
            const long long step = std::max<long long>(1, (rows + 63) / 64);
            for (long long u = 0; u < rows; u += step) hs.push_back({hb[(size_t)u * 4], hb[(size_t)u * 4 + 1]});
            j.integer("history_every", step).pairs("history", hs);
        }
    }
    metrics_write(j);
}

// FP64 iterations up to the absolute cap `cap` (the control block already
// armed for them), with the stall watch when it is on: windows of
// stall_window iterations, the merit pres^2 + (dres / rho)^2 of each
// window's last iteration against the previous one.  Sets *status.
int run_fp64_watched(opf_admm_handle* h, long long cap, const Work& w, int* status) {
    const long long W = h->opt.stall_window;
    if (W <= 0) {
        int rc = run_any<double>(h, h->s64, &h->graph64, cap, 1, w);
        if (rc) return rc;
        *status = h->ctrl_host->status;
        return 0;
    }
    long long stop_at = std::min<long long>(h->ctrl_host->iter + W, cap);
    HIPCHK(launch_rearm(h->ctrl, stop_at, 1, h->stream));
    int rc = run_any<double>(h, h->s64, &h->graph64, stop_at, 1, w);
    if (rc) return rc;
    double m_prev = HUGE_VAL;
    int flat = 0;
    while (h->ctrl_host->status == OPF_NOT_CONVERGED && h->ctrl_host->iter < cap) {
        const Ctrl& c = *h->ctrl_host;
        const double rho_t = h->opt.rho_every ? c.rho[c.iter % kRhoRing] : h->opt.rho;
        const double m = c.res[0] * c.res[0] + (c.res[1] / rho_t) * (c.res[1] / rho_t);
        flat = m > (1.0 - h->opt.stall_delta) * m_prev ? flat + 1 : 0;
        m_prev = m;
        if (flat >= h->opt.stall_checks) {
            *status = OPF_STALLED;
            return 0;
        }
        stop_at = std::min<long long>(c.iter + W, cap);
        HIPCHK(launch_rearm(h->ctrl, stop_at, 1, h->stream));
        if ((rc = run_any<double>(h, h->s64, &h->graph64, stop_at, 1, w))) return rc;
    }
    *status = h->ctrl_host->status;
    return 0;
}

int solve_impl(opf_admm_handle* h, const opf_warm* warm, opf_result* r, long long fixed_iters, const Work& w) {
    if (!h || !r || !r->x) return set_err(h, OPF_EINVAL, "null handle, result or x");
    auto t0 = std::chrono::steady_clock::now();
    if (h->user_stream != h->stream) HIPCHK(hipStreamSynchronize(h->user_stream));
    const double* z0;
    const double* l0;
    int rc = prepare_start(h, warm, &z0, &l0);
    if (rc) return rc;
    const bool fixed = fixed_iters > 0;
    const long long max_iter = fixed ? fixed_iters : h->opt.max_iter;
    const int check = fixed ? 0 : 1;
    int status = OPF_OK;
    long long it32 = 0;
    bool final64 = true;
    h->kernel_ms = 0;
    h->kernel_launches = 0;
    h->ctrl_host->iter = 0;
    r->kernel_ms_fp32 = 0;
    if (h->opt.precision == OPF_PREC_MIXED) {
        // below OPF_MIXED_STALL_BELOW the bulk phase runs in windows and ends
        // early when the residual ratio stops halving from window to window
        const bool watch = h->opt.polish && !fixed && h->opt.eps_rel < OPF_MIXED_STALL_BELOW;
        long long stop_at = watch ? std::min<long long>(OPF_MIXED_STALL_WINDOW, max_iter) : max_iter;
        HIPCHK(launch_init<float>(z0, l0, h->s32.z[0], h->s32.l[0], h->LP, h->ctrl, stop_at, check, h->opt.rho,
                                  h->stream));
        rc = run_any<float>(h, h->s32, &h->graph32, stop_at, check, w);
        if (rc) return rc;
        double q_prev = HUGE_VAL;
        while (watch && h->ctrl_host->status == OPF_NOT_CONVERGED && h->ctrl_host->iter < max_iter) {
            const Ctrl& c = *h->ctrl_host;
            const double q = std::max(c.res[0] / c.res[2], c.res[1] / c.res[3]);
            if (!(q < 0.5 * q_prev)) break;          // stalled: on to the polish
            q_prev = q;
            stop_at = std::min<long long>(c.iter + OPF_MIXED_STALL_WINDOW, max_iter);
            HIPCHK(launch_rearm(h->ctrl, stop_at, check, h->stream));
            rc = run_any<float>(h, h->s32, &h->graph32, stop_at, check, w);
            if (rc) return rc;
        }
        it32 = h->ctrl_host->iter;
        status = h->ctrl_host->status;
        r->kernel_ms_fp32 = h->kernel_ms;
        const bool polish = h->opt.polish && !fixed && status != OPF_ENUMERIC;
        if (polish) {
            HIPCHK(launch_promote(h->s32.z[0], h->s32.z[1], h->s32.l[0], h->s32.l[1], h->s64.z[0], h->s64.z[1],
                                  h->s64.l[0], h->s64.l[1], h->LP, h->ctrl, it32 + h->opt.max_iter, 1, h->stream));
            if ((rc = run_fp64_watched(h, it32 + h->opt.max_iter, w, &status))) return rc;
        } else {
            final64 = false;
        }
    } else {
        HIPCHK(launch_init<double>(z0, l0, h->s64.z[0], h->s64.l[0], h->LP, h->ctrl, max_iter, check, h->opt.rho,
                                   h->stream));
        if (fixed) {
            if ((rc = run_any<double>(h, h->s64, &h->graph64, max_iter, check, w))) return rc;
            status = h->ctrl_host->status;
        } else if ((rc = run_fp64_watched(h, max_iter, w, &status))) {
            return rc;
        }
    }
    rc = final64 ? finish_outputs<double>(h, h->s64, r) : finish_outputs<float>(h, h->s32, r);
    if (rc) return rc;
    const Ctrl& c = *h->ctrl_host;
    r->iterations = c.iter;
    r->iterations_fp32 = it32;
    r->objective = c.objective;
    r->pres = c.res[0];
    r->dres = c.res[1];
    r->eps_prim = c.res[2];
    r->eps_dual = c.res[3];
    r->status = status;
    r->kernel_ms = h->kernel_ms;
    r->kernel_launches = h->kernel_launches;
    r->rho_final = h->opt.rho_every ? c.rho[(c.iter + 1) % kRhoRing] : h->opt.rho;
    h->last_iter = c.iter;
    h->last_prec = final64 ? OPF_PREC_FP64 : OPF_PREC_MIXED;
    r->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (status == OPF_ENUMERIC) set_err(h, OPF_ENUMERIC, "NaN/Inf in the residuals");
    return status;
}

// ---- allocation-free solve: kernel scratch in a static device array ----------
//
// One array per device for the life of the process (the code object's
// static data); its address on each device is looked up once, with that
// device current, and kept.  Every allocation-free solve on a device shares
// it, so such solves must not overlap on one device.
constexpr size_t kScratchBytes = OPF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

__global__ void zero_words_kernel(unsigned* p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of scratch the handle's kernels need (both schedules, both precisions).
size_t static_work_bytes(const opf_admm_handle* h) {
    const size_t G = (size_t)h->lay.blocks;
    return round256((size_t)h->LP * 4 * sizeof(unsigned long long)) +
           round256(G * 10 * kDecisionLag * sizeof(unsigned long long)) + 3 * 256 +
           round256(step_partials_count((int)G) * sizeof(double));
}

// Points w at the static array of the handle's device; the step kernel's
// arrival counters (behind its residual partials) are cleared, the persistent
// kernel's words are prepared by its own launch.
int static_work(opf_admm_handle* h, Work* w) {
    const size_t need = static_work_bytes(h);
    if (need > kScratchBytes)
        return set_err(h, OPF_EINVAL, "the allocation-free solve needs " + std::to_string(need) +
                                          " bytes of kernel scratch; the static array holds " +
                                          std::to_string(kScratchBytes));
    if (h->device < 0 || h->device >= kMaxDevices) return set_err(h, OPF_EINVAL, "device id out of range");
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = g_scratch_ptr[h->device];
        if (!base) {
            int cur = 0;
            HIPCHK(hipGetDevice(&cur));
            if (cur != h->device) HIPCHK(hipSetDevice(h->device));
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (cur != h->device) (void)hipSetDevice(cur);
            if (e != hipSuccess)
                return set_err(h, OPF_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            base = static_cast<unsigned char*>(p);
            g_scratch_ptr[h->device] = base;
        }
    }
    const size_t G = (size_t)h->lay.blocks;
    size_t off = 0;
    w->pub = reinterpret_cast<unsigned long long*>(base + off);
    off += round256((size_t)h->LP * 4 * sizeof(unsigned long long));
    w->records = reinterpret_cast<unsigned long long*>(base + off);
    off += round256(G * 10 * kDecisionLag * sizeof(unsigned long long));
    w->dec_iter = reinterpret_cast<long long*>(base + off);
    off += 256;
    w->dec_stop = reinterpret_cast<long long*>(base + off);
    off += 256;
    w->dev_error = reinterpret_cast<int*>(base + off);
    off += 256;
    w->partials = reinterpret_cast<double*>(base + off);
    w->graphs = false;
    const size_t words = step_partials_count((int)G) * 2;
    hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, h->stream,
                       reinterpret_cast<unsigned*>(w->partials), words);
    HIPCHK(hipGetLastError());
    return 0;
}

}  // namespace

// Device set-up: row reduction and factors of every component on the GPU,
// written into the packed layout (FP64); any component found infeasible fails
// the set-up as on the host.
int device_factors(opf_admm_handle* h, const opf_problem* p) {
    const HostLayout& L = h->lay;
    const int S = L.S;
    size_t lds = 0;
    int64_t na = 0, nb = 0;
    for (int q = 0; q < S; ++q) {
        lds = std::max(lds, factor_lds_bytes(p->comp_m[q], p->comp_n[q]));
        na += (int64_t)p->comp_m[q] * p->comp_n[q];
        nb += p->comp_m[q];
    }
    if (lds > 64 * 1024)
        return set_err(h, OPF_EINVAL, "device set-up: a component needs more than 64 KiB of LDS; use the host set-up");
    const int W = L.waves;
    h->devF_count = W ? L.wave_foff[W - 1] + (int64_t)L.wave_maxn[W - 1] * kWave : 0;
    int rc;
    double *dA = nullptr, *db = nullptr;
    int64_t *daoff = nullptr, *dboff = nullptr, *dfoff = nullptr;
    int *dm = nullptr, *dn = nullptr, *ddev = nullptr, *dstatus = nullptr;
    if ((rc = dalloc(h, &h->devF, (size_t)std::max<int64_t>(h->devF_count, 1)))) return rc;
    if ((rc = dalloc(h, &h->devBbar, (size_t)h->LP))) return rc;
    HIPCHK(hipMemsetAsync(h->devF, 0, sizeof(double) * std::max<int64_t>(h->devF_count, 1), h->stream));
    HIPCHK(hipMemsetAsync(h->devBbar, 0, sizeof(double) * h->LP, h->stream));
    std::vector<double> A(p->A_vals, p->A_vals + na), b(p->b_vals, p->b_vals + nb);
    std::vector<int32_t> m(p->comp_m, p->comp_m + S), n(p->comp_n, p->comp_n + S);
    if ((rc = upload(h, &dA, A)) || (rc = upload(h, &db, b)) || (rc = upload(h, &daoff, L.comp_aoff)) ||
        (rc = upload(h, &dboff, L.comp_boff)) || (rc = upload(h, &dfoff, L.wave_foff)) || (rc = upload(h, &dm, m)) ||
        (rc = upload(h, &dn, n)) || (rc = upload(h, &ddev, L.comp_dev)) || (rc = dalloc(h, &dstatus, (size_t)S)))
        return rc;
    FactorJob job{dA, db, daoff, dboff, dm, dn, ddev, dfoff, h->devF, h->devBbar, dstatus, S};
    HIPCHK(launch_factors(job, lds, h->stream));
    std::vector<int> status(S, 0);
    HIPCHK(hipMemcpyAsync(status.data(), dstatus, sizeof(int) * S, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int q = 0; q < S; ++q)
        if (status[q] != 0)
            return set_err(h, status[q], "row reduction found 0 = nonzero (inconsistent equations) in component " +
                                             std::to_string(q));
    return 0;
}

extern "C" {

void opf_admm_default_options(opf_admm_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->rho = 100.0;
    o->eps_rel = 1e-3;
    o->max_iter = 1000000;
    o->precision = OPF_PREC_FP64;
    o->polish = 1;
    o->check_every = 256;
    o->kernel = OPF_KERNEL_AUTO;
    o->history_cap = 0;
    o->block_waves = 0;
}

int opf_admm_setup(const opf_problem* p, const opf_admm_options* o, void* hip_stream, opf_admm_handle** out) {
    opf_admm_handle* h = nullptr;
    if (out) *out = nullptr;
    if (!p || !out) return set_err(nullptr, OPF_EINVAL, "null problem or output pointer");
    opf_admm_options opt;
    if (o) opt = *o;
    else opf_admm_default_options(&opt);
    if (opt.autotune && opt.kernel == OPF_KERNEL_AUTO && opt.block_waves == 0 && p->S > 0 && p->comp_n) {
        // ---- autotuner: time each (schedule, workgroup shape) on this problem
        int64_t L = 0, n2 = 0;
        for (int s2 = 0; s2 < p->S; ++s2) { L += p->comp_n[s2]; n2 += (int64_t)p->comp_n[s2] * p->comp_n[s2]; }
        const std::string key = std::to_string(p->n) + "/" + std::to_string(p->S) + "/" + std::to_string(L) + "/" +
                                std::to_string(n2) + "/" + std::to_string(opt.precision);
        std::pair<int, int> choice{0, 0};
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune.find(key);
            if (it != g_tune.end()) choice = it->second;
        }
        std::vector<int> cached;
        if (!choice.first && tune_cache_get("single/" + key, cached) && cached.size() == 2)
            choice = {cached[0], cached[1]};
        if (!choice.first) {
            double best = 1e300;
            const int cands[][2] = {{OPF_KERNEL_PERSISTENT, 2}, {OPF_KERNEL_PERSISTENT, 4}, {OPF_KERNEL_PERSISTENT, 8},
                                    {OPF_KERNEL_TILED, 4}, {OPF_KERNEL_STEP, 4}, {OPF_KERNEL_STEP, 8}};
            for (const auto& c : cands) {
                opf_admm_options t = opt;
                t.autotune = 0;
                t.kernel = c[0];
                t.block_waves = c[1];
                t.history_cap = 0;
                t.check_every = 128;
                opf_admm_handle* th = nullptr;
                if (opf_admm_setup(p, &t, hip_stream, &th) != OPF_OK) continue;
                std::vector<double> xs(p->n);
                opf_result r{};
                r.x = xs.data();
                double ms = 1e300;
                if (opf_admm_run_fixed(th, nullptr, 64, &r) >= 0 && opf_admm_run_fixed(th, nullptr, 512, &r) >= 0)
                    ms = r.kernel_ms;
                opf_admm_destroy(th);
                if (ms < best) { best = ms; choice = {c[0], c[1]}; }
            }
            if (!choice.first) choice = {OPF_KERNEL_AUTO, 4};
            else tune_cache_put("single/" + key, {choice.first, choice.second});
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune[key] = choice;
        }
        opt.autotune = 0;
        opt.kernel = choice.first;
        opt.block_waves = choice.second;
        return opf_admm_setup(p, &opt, hip_stream, out);
    }
    if (!(opt.rho > 0.0) || !std::isfinite(opt.rho)) return set_err(nullptr, OPF_EINVAL, "rho must be positive");
    if (!(opt.eps_rel > 0.0)) return set_err(nullptr, OPF_EINVAL, "eps_rel must be positive");
    if (opt.max_iter < 1) return set_err(nullptr, OPF_EINVAL, "max_iter must be >= 1");
    if (opt.precision != OPF_PREC_FP64 && opt.precision != OPF_PREC_MIXED)
        return set_err(nullptr, OPF_EINVAL, "unknown precision");
    if (opt.history_cap < 0) return set_err(nullptr, OPF_EINVAL, "history_cap must be >= 0");
    if (opt.rho_every < 0) return set_err(nullptr, OPF_EINVAL, "rho_every must be >= 0");
    if (opt.stall_window < 0 || opt.stall_checks < 0 || opt.stall_delta < 0 || opt.stall_delta >= 1)
        return set_err(nullptr, OPF_EINVAL, "stall watch: window, checks >= 0 and delta in [0, 1)");
    if (opt.stall_window > 0) {
        if (opt.stall_checks == 0) opt.stall_checks = 3;
        if (opt.stall_delta == 0) opt.stall_delta = 1e-3;
    }
    if (opt.local_updates < 0) return set_err(nullptr, OPF_EINVAL, "local_updates must be >= 0");
    if (opt.local_updates == 0) opt.local_updates = 1;
    if (opt.rho_every > 0) {
        if (opt.rho_mu == 0.0) opt.rho_mu = 10.0;
        if (opt.rho_tau == 0.0) opt.rho_tau = 2.0;
        if (opt.rho_min == 0.0) opt.rho_min = opt.rho / 10.0;
        if (opt.rho_max == 0.0) opt.rho_max = opt.rho * 10.0;
        if (opt.rho_mode != OPF_RHO_RELATIVE && opt.rho_mode != OPF_RHO_PLAIN)
            return set_err(nullptr, OPF_EINVAL, "unknown rho_mode");
        if (!(opt.rho_mu >= 1.0) || !(opt.rho_tau > 1.0) || !std::isfinite(opt.rho_mu) || !std::isfinite(opt.rho_tau))
            return set_err(nullptr, OPF_EINVAL, "residual balancing needs rho_mu >= 1 and rho_tau > 1");
        if (!(opt.rho_min > 0.0) || !(opt.rho_min <= opt.rho) || !(opt.rho <= opt.rho_max) || !std::isfinite(opt.rho_max))
            return set_err(nullptr, OPF_EINVAL, "residual balancing needs 0 < rho_min <= rho <= rho_max < inf");
    }
    if (opt.check_every < 1) opt.check_every = 256;
    auto t0 = std::chrono::steady_clock::now();
    ProblemView v;
    v.n = p->n; v.S = p->S; v.c = p->c; v.lb = p->lb; v.ub = p->ub; v.var_kind = p->var_kind;
    v.comp_m = p->comp_m; v.comp_n = p->comp_n; v.A = p->A_vals; v.b = p->b_vals; v.idx = p->idx;
    h = new opf_admm_handle();
    h->opt = opt;
    std::string err;
    const int threads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    h->lay.block_waves = (opt.block_waves == 1 || opt.block_waves == 2 || opt.block_waves == 4 ||
                          opt.block_waves == 8) ? opt.block_waves : 4;
    h->lay.factors_on_device = opt.setup_on_device == 1;
    int rc = build_layout(v, h->lay, err, threads);
    if (rc) {
        delete h;
        return set_err(nullptr, rc, err);
    }
    h->LP = h->lay.waves * kWave;
    h->user_stream = (hipStream_t)hip_stream;
    h->xcd_remap = opt.workgroup_order == 1 ? 1 : 0;
    h->wpb = h->lay.block_waves;
    auto fail = [&](int code) {
        std::string m = h->err;
        opf_admm_destroy(h);
        return set_err(nullptr, code, m);
    };
    if (hipGetDevice(&h->device) != hipSuccess) return fail(set_err(h, OPF_EHIP, "hipGetDevice failed"));
    if (h->user_stream) {
        h->stream = h->user_stream;          // all work on the caller's stream
    } else if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) {
        return fail(set_err(h, OPF_EHIP, "hipStreamCreate failed"));
    }
    if (hipHostMalloc((void**)&h->ctrl_host, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess)
        return fail(set_err(h, OPF_ENOMEM, "hipHostMalloc failed"));
    if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess)
        return fail(set_err(h, OPF_EHIP, "hipEventCreate failed"));
    std::memset(h->ctrl_host, 0, sizeof(Ctrl));
    const HostLayout& L = h->lay;
    std::vector<int2> wi(L.waves);
    for (int w = 0; w < L.waves; ++w) wi[w] = make_int2(L.wave_maxn[w], (int)(L.wave_foff[w] / kWave));
    if ((rc = upload(h, &h->winfo, wi))) return fail(rc);
    if ((rc = upload(h, &h->var, L.var))) return fail(rc);
    if ((rc = upload(h, &h->meta, L.meta))) return fail(rc);
    if ((rc = upload(h, &h->cstart, L.copy_start))) return fail(rc);
    if ((rc = upload(h, &h->ccnt, L.copy_cnt))) return fail(rc);
    if ((rc = upload(h, &h->clist, L.copy_list))) return fail(rc);
    if ((rc = upload(h, &h->user_slot, L.user_slot))) return fail(rc);
    if ((rc = upload(h, &h->user_to_dev, L.user_to_dev))) return fail(rc);
    if ((rc = upload(h, &h->z0, L.z0))) return fail(rc);
    if ((rc = upload(h, &h->c, L.c_full))) return fail(rc);
    if (L.factors_on_device && (rc = device_factors(h, p))) return fail(rc);
    if ((rc = dalloc(h, &h->warm_z, h->LP))) return fail(rc);
    if ((rc = dalloc(h, &h->warm_l, h->LP))) return fail(rc);
    if ((rc = dalloc(h, &h->user_z, L.L))) return fail(rc);
    if ((rc = dalloc(h, &h->user_l, L.L))) return fail(rc);
    if ((rc = dalloc(h, &h->xo, L.n))) return fail(rc);
    const int blocks = L.blocks;
    h->grid_blocks = blocks;
    // residual partials of the step kernel; tagged records of the persistent kernel
    Work& w = h->work;
    if ((rc = dalloc(h, &w.partials, step_partials_count(blocks)))) return fail(rc);
    // the arrival counters behind the partials start at 0 and return to 0 every iteration
    if (hipMemsetAsync(w.partials, 0, sizeof(double) * step_partials_count(blocks), h->stream) != hipSuccess)
        return fail(set_err(h, OPF_EHIP, "memset"));
    if ((rc = dalloc(h, &w.pub, (size_t)h->LP * 4))) return fail(rc);
    if ((rc = dalloc(h, &w.records, (size_t)blocks * 10 * kDecisionLag))) return fail(rc);
    if ((rc = dalloc(h, &w.dec_iter, 1))) return fail(rc);
    if ((rc = dalloc(h, &w.dec_stop, 1))) return fail(rc);
    if ((rc = dalloc(h, &w.dev_error, 1))) return fail(rc);
    if (hipHostMalloc((void**)&h->error_host, sizeof(int), hipHostMallocDefault) != hipSuccess)
        return fail(set_err(h, OPF_ENOMEM, "hipHostMalloc failed"));
    *h->error_host = 0;
    // factors stay in LDS when the grid still fits the device with that much
    // dynamic shared memory per workgroup (else they are read through the caches)
    for (int b2 = 0; b2 < blocks; ++b2) {
        int cols = 0;
        for (int q = 0; q < h->wpb; ++q) cols += L.wave_maxn[(size_t)b2 * h->wpb + q];
        h->lds_cols = std::max(h->lds_cols, cols);
    }
    const size_t lds_limit = 64 * 1024;
    const size_t l32 = (size_t)h->lds_cols * 64 * 4;
    const int ad = opt.rho_every > 0;
    const int cap32_lds = l32 <= lds_limit ? persistent_capacity<float>(h->wpb, l32, ad) : 0;
    h->lds32 = cap32_lds >= blocks + 1;
    const int cap32 = h->lds32 ? cap32_lds : persistent_capacity<float>(h->wpb, 0, ad);
    // FP64: the largest column budget (every workgroup's columns, else a
    // multiple of 8) with which the grid still fits; workgroups within it
    // hold their factors in LDS
    int cap64 = persistent_capacity<double>(h->wpb, 0, ad);
    h->lds64 = 0;
    h->lds64_cols = 0;
    std::vector<int> budgets{h->lds_cols};
    for (int c = h->lds_cols / 8 * 8; c >= 8; c -= 8)
        if (c < h->lds_cols) budgets.push_back(c);
    for (int cols : budgets) {
        if (cols < 1) break;
        const size_t l64 = (size_t)cols * 64 * 8;
        if (l64 > lds_limit) continue;
        const int c = persistent_capacity<double>(h->wpb, l64, ad);
        if (c >= blocks + 1) {
            h->lds64 = cols;
            h->lds64_cols = cols;
            cap64 = c;
            break;
        }
    }
    h->capacity = opt.precision == OPF_PREC_MIXED ? std::min(cap32, cap64) : cap64;
    if (opt.kernel == OPF_KERNEL_PERSISTENT && h->capacity < blocks + 1)
        return fail(set_err(h, OPF_EINVAL, "persistent kernel needs " + std::to_string(blocks + 1) +
                                              " co-resident workgroups, the device holds " +
                                              std::to_string(h->capacity)));
    // tiled schedule: as many co-resident workgroups as needed for an even
    // share of tiles (plus the reducer)
    // (per precision: the FP32 and FP64 kernels hold different numbers of
    // workgroups).  When every workgroup can take at most two tiles, the
    // two-tile kernel (both tiles in flight) runs with ceil(tiles / 2)
    // workgroups; otherwise the loop kernel with an even share each.
    if (opt.tiled_workgroups < 0) return fail(set_err(h, OPF_EINVAL, "tiled_workgroups must be >= 0"));
    auto tiled_grid = [&](int cap_loop, int cap_pair, int* pair) {
        int gmax = std::min(cap_loop - 1, blocks);
        if (opt.tiled_workgroups > 0) gmax = std::min(gmax, opt.tiled_workgroups);
        const int gpair = (blocks + 1) / 2;
        if (blocks >= 2 && gpair + 1 <= cap_pair && (opt.tiled_workgroups == 0 || opt.tiled_workgroups >= gpair)) {
            *pair = 1;
            return gpair;
        }
        *pair = 0;
        const int per = (blocks + gmax - 1) / gmax;
        return (blocks + per - 1) / per;
    };
    const int tcap64 = tiled_capacity<double>(h->wpb, 0);
    const int tcap32 = opt.precision == OPF_PREC_MIXED ? tiled_capacity<float>(h->wpb, 0) : tcap64;
    const int pcap64 = tiled_capacity<double>(h->wpb, 1);
    const int pcap32 = opt.precision == OPF_PREC_MIXED ? tiled_capacity<float>(h->wpb, 1) : pcap64;
    const bool tiled_ok = std::min(tcap64, tcap32) >= 2 && opt.rho_every == 0;
    if (tiled_ok) {
        h->tiled_G = tiled_grid(tcap64, pcap64, &h->tiled_pair64);
        h->tiled_G32 = tiled_grid(tcap32, pcap32, &h->tiled_pair32);
        // two-tile kernel: the largest column budget of dynamic shared memory
        // (every workgroup's two tiles, else a multiple of 8) with which its
        // grid still fits; workgroups within it keep their factors in LDS
        auto pair_budget = [&](int G, size_t elem, bool fp32) {
            int most = 0;
            for (int b2 = 0; b2 < G; ++b2) {
                int cols = 0;
                for (int q = 0; q < 2 && b2 + q * G < blocks; ++q)
                    for (int v = 0; v < h->wpb; ++v) cols += L.wave_maxn[(size_t)(b2 + q * G) * h->wpb + v];
                most = std::max(most, cols);
            }
            std::vector<int> budgets{most};
            for (int c = most / 8 * 8; c >= 8; c -= 8)
                if (c < most) budgets.push_back(c);
            for (int cols : budgets) {
                const size_t bytes = (size_t)cols * 64 * elem;
                if (cols < 1 || bytes > lds_limit) continue;
                const int cap = fp32 ? tiled_capacity<float>(h->wpb, 1, bytes) : tiled_capacity<double>(h->wpb, 1, bytes);
                if (cap >= G + 1) return cols;
            }
            return 0;
        };
        if (h->tiled_pair64) h->tiled_lds64 = pair_budget(h->tiled_G, 8, false);
        if (h->tiled_pair32) h->tiled_lds32 = pair_budget(h->tiled_G32, 4, true);
    }
    if (opt.kernel == OPF_KERNEL_TILED && !tiled_ok)
        return fail(set_err(h, OPF_EINVAL, "the tiled schedule runs a fixed penalty on a device holding at least "
                                           "two of its workgroups"));
    if (opt.kernel == OPF_KERNEL_STEP) h->kernel = OPF_KERNEL_STEP;
    else if (opt.kernel == OPF_KERNEL_PERSISTENT) h->kernel = OPF_KERNEL_PERSISTENT;
    else if (opt.kernel == OPF_KERNEL_TILED) h->kernel = OPF_KERNEL_TILED;
    else if (h->capacity >= blocks + 1) h->kernel = OPF_KERNEL_PERSISTENT;
    else h->kernel = tiled_ok ? OPF_KERNEL_TILED : OPF_KERNEL_STEP;
    if ((rc = dalloc(h, &h->hist, (size_t)std::max(1, opt.history_cap) * 4))) return fail(rc);
    if ((rc = dalloc(h, &h->ctrl, 1))) return fail(rc);
    if (hipMemsetAsync(h->ctrl, 0, sizeof(Ctrl), h->stream) != hipSuccess) return fail(set_err(h, OPF_EHIP, "memset"));
    if ((rc = make_prec<double>(h, h->s64))) return fail(rc);
    if (opt.precision == OPF_PREC_MIXED) {
        if ((rc = make_prec<float>(h, h->s32))) return fail(rc);
        h->has32 = true;
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(set_err(h, OPF_EHIP, "sync"));
    h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h;
    return OPF_OK;
}

int opf_admm_solve(opf_admm_handle* h, const opf_warm* warm, opf_result* r) {
    if (!h) return set_err(nullptr, OPF_EINVAL, "null handle");
    const int rc = solve_impl(h, warm, r, 0, h->work);
    if ((rc >= 0 || rc == OPF_ENUMERIC) && metrics_on()) record_solve(h, r, "solve");
    return rc;
}

int opf_admm_run_fixed(opf_admm_handle* h, const opf_warm* warm, int64_t iters, opf_result* r) {
    if (!h) return set_err(nullptr, OPF_EINVAL, "null handle");
    if (iters < 1) return set_err(h, OPF_EINVAL, "iters must be >= 1");
    const int rc = solve_impl(h, warm, r, iters, h->work);
    if ((rc >= 0 || rc == OPF_ENUMERIC) && metrics_on()) record_solve(h, r, "fixed");
    return rc;
}

int opf_admm_solve_noalloc(opf_admm_handle* h, const opf_warm* warm, opf_result* r) {
    if (!h) return set_err(nullptr, OPF_EINVAL, "null handle");
    Work w;
    int rc = static_work(h, &w);
    if (rc) return rc;
    return solve_impl(h, warm, r, 0, w);
}

int opf_admm_residuals(const opf_admm_handle* hc, opf_residuals* out, double* hist, int hist_cap) {
    opf_admm_handle* h = const_cast<opf_admm_handle*>(hc);
    if (!h) return set_err(nullptr, OPF_EINVAL, "null handle");
    HIPCHK(hipMemcpyAsync(h->ctrl_host, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    const Ctrl& c = *h->ctrl_host;
    if (out) {
        out->iterations = c.iter;
        out->pres = c.res[0];
        out->dres = c.res[1];
        out->eps_prim = c.res[2];
        out->eps_dual = c.res[3];
    }
    int rows = 0;
    if (hist && hist_cap > 0) {
        rows = (int)std::min<long long>({(long long)hist_cap, (long long)h->opt.history_cap, c.iter});
        if (rows > 0) {
            HIPCHK(hipMemcpyAsync(hist, h->hist, sizeof(double) * 4 * rows, hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
        }
    }
    return rows;
}

int opf_admm_get_info(const opf_admm_handle* h, opf_admm_info* info) {
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
    info->grid_blocks = h->kernel != OPF_KERNEL_TILED ? h->grid_blocks
                        : (h->opt.precision == OPF_PREC_MIXED ? h->tiled_G32 : h->tiled_G);
    info->block_waves = h->wpb;
    info->kernel = h->kernel;
    info->persistent_capacity = h->capacity;
    info->max_neighbours = h->lay.max_nbrs;
    info->factors_in_lds = (h->lds32 ? 1 : 0) | (h->lds64 ? 2 : 0);
    if (h->lds64) {
        int in = 0;
        for (int b2 = 0; b2 < h->lay.blocks; ++b2) {
            int cols = 0;
            for (int q = 0; q < h->wpb; ++q) cols += h->lay.wave_maxn[(size_t)b2 * h->wpb + q];
            in += cols <= h->lds64;
        }
        info->fp64_lds_workgroups = in;
    }
    if (h->kernel == OPF_KERNEL_TILED)
        info->tiled_pair = h->opt.precision == OPF_PREC_MIXED ? h->tiled_pair32 : h->tiled_pair64;
    return 0;
}

void opf_admm_destroy(opf_admm_handle* h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->graph64) (void)hipGraphExecDestroy(h->graph64);
    if (h->graph32) (void)hipGraphExecDestroy(h->graph32);
    for (auto& b : h->bufs) (void)hipFree(b.p);
    if (h->ctrl_host) (void)hipHostFree(h->ctrl_host);
    if (h->error_host) (void)hipHostFree(h->error_host);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->stream && h->stream != h->user_stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

const char* opf_admm_last_error(const opf_admm_handle* h) {
    if (h) return h->err.c_str();
    std::lock_guard<std::mutex> lk(g_err_mu);
    return g_setup_err.c_str();
}

}  // extern "C"
