// Host set-up of the componentwise ADMM: validation, row reduction and the
// FP64 projection factors of every component, copy lists of B^T, and the
// packing of components into 64-lane wavefronts.
//
// Factors (closed_2 and the precomputation of Algorithm 1): for the
// row-reduced, full-row-rank A_s (Section IV-B),
//     F_s    = I - A_s^T (A_s A_s^T)^{-1} A_s      (the paper's Abar_s is -F_s)
//     bbar_s = A_s^T (A_s A_s^T)^{-1} b_s
// so that the local update is x_s = F_s (B_s x + lambda_s / rho) + bbar_s.
#include "opf_layout.h"

#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <deque>
#include <thread>

#include "../../include/opf_admm.h"

namespace opf {

int component_factor(int m, int n, const double* A, const double* b, double* F, double* bbar,
                     int* rank_out) {
    return component_factor_multi(m, n, A, 1, b, F, bbar, rank_out);
}

int component_rhs_map(int m, int n, const double* A, double* F, double* Wmap) {
    std::vector<double> I((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) I[(size_t)i * m + i] = 1.0;
    int rank = 0;
    // identity right-hand sides: rows that reduce to zero carry the consistency
    // conditions of b, not a contradiction, so they are not checked here
    return component_factor_multi(m, n, A, -m, I.data(), F, Wmap, &rank);
}

int component_factor_multi(int m, int n, const double* A, int r_in, const double* Bm, double* F,
                           double* bbar, int* rank_out) {
    const bool check = r_in > 0;
    const int r = r_in > 0 ? r_in : -r_in;
    const int w = n + r;
    std::vector<double> M((size_t)m * w);
    double amax = 0.0, bmax = 0.0;
    for (int rr = 0; rr < m; ++rr) {
        for (int c = 0; c < n; ++c) {
            M[(size_t)rr * w + c] = A[(size_t)rr * n + c];
            amax = std::max(amax, std::fabs(A[(size_t)rr * n + c]));
        }
        for (int c = 0; c < r; ++c) {
            M[(size_t)rr * w + n + c] = Bm[(size_t)rr * r + c];
            bmax = std::max(bmax, std::fabs(Bm[(size_t)rr * r + c]));
        }
    }
    const double tol = std::max(m, n) * DBL_EPSILON * std::max(amax, 1e-300);
    // Gauss-Jordan elimination with partial pivoting (reduced row echelon form)
    int row = 0;
    for (int col = 0; col < n && row < m; ++col) {
        int p = row;
        double best = std::fabs(M[(size_t)row * w + col]);
        for (int r = row + 1; r < m; ++r) {
            double v = std::fabs(M[(size_t)r * w + col]);
            if (v > best) { best = v; p = r; }
        }
        if (best <= tol) {
            for (int r = row; r < m; ++r) M[(size_t)r * w + col] = 0.0;
            continue;
        }
        if (p != row)
            for (int c = 0; c < w; ++c) std::swap(M[(size_t)p * w + c], M[(size_t)row * w + c]);
        const double inv = 1.0 / M[(size_t)row * w + col];
        for (int c = 0; c < w; ++c) M[(size_t)row * w + c] *= inv;
        M[(size_t)row * w + col] = 1.0;
        for (int r = 0; r < m; ++r) {
            if (r == row) continue;
            const double f = M[(size_t)r * w + col];
            if (f == 0.0) continue;
            for (int c = 0; c < w; ++c) M[(size_t)r * w + c] -= f * M[(size_t)row * w + c];
            M[(size_t)r * w + col] = 0.0;
        }
        ++row;
    }
    const double bscale = std::max(1.0, bmax);
    if (check)
        for (int rr = row; rr < m; ++rr)
            for (int c = 0; c < r; ++c)
                if (std::fabs(M[(size_t)rr * w + n + c]) > tol * bscale) return OPF_EINFEASIBLE_COMPONENT;
    const int k = row;
    if (rank_out) *rank_out = k;
    std::fill(F, F + (size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) F[(size_t)i * n + i] = 1.0;
    std::fill(bbar, bbar + (size_t)n * r, 0.0);
    if (k == 0) return 0;
    // G = Ahat Ahat^T and its Cholesky factor (lower, in place)
    std::vector<double> G((size_t)k * k);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = 0.0;
            for (int c = 0; c < n; ++c) s += M[(size_t)i * w + c] * M[(size_t)j * w + c];
            G[(size_t)i * k + j] = s;
        }
    for (int j = 0; j < k; ++j) {
        double d = G[(size_t)j * k + j];
        for (int q = 0; q < j; ++q) d -= G[(size_t)j * k + q] * G[(size_t)j * k + q];
        if (!(d > 0.0)) return OPF_EINFEASIBLE_COMPONENT;
        d = std::sqrt(d);
        G[(size_t)j * k + j] = d;
        for (int i = j + 1; i < k; ++i) {
            double s = G[(size_t)i * k + j];
            for (int q = 0; q < j; ++q) s -= G[(size_t)i * k + q] * G[(size_t)j * k + q];
            G[(size_t)i * k + j] = s / d;
        }
    }
    // solve G W = [Ahat | bhat] column by column (W is k x (n+r))
    std::vector<double> W((size_t)k * w);
    std::vector<double> y(k);
    for (int c = 0; c < w; ++c) {
        for (int i = 0; i < k; ++i) {
            double s = M[(size_t)i * w + c];
            for (int q = 0; q < i; ++q) s -= G[(size_t)i * k + q] * y[q];
            y[i] = s / G[(size_t)i * k + i];
        }
        for (int i = k - 1; i >= 0; --i) {
            double s = y[i];
            for (int q = i + 1; q < k; ++q) s -= G[(size_t)q * k + i] * W[(size_t)q * w + c];
            W[(size_t)i * w + c] = s / G[(size_t)i * k + i];
        }
    }
    // F = I - Ahat^T W[:, :n] (symmetrised), bbar = Ahat^T W[:, n:]
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int q = 0; q < k; ++q) s += M[(size_t)q * w + i] * W[(size_t)q * w + j];
            F[(size_t)i * n + j] -= s;
        }
        for (int c = 0; c < r; ++c) {
            double s = 0.0;
            for (int q = 0; q < k; ++q) s += M[(size_t)q * w + i] * W[(size_t)q * w + n + c];
            bbar[(size_t)i * r + c] = s;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double a = 0.5 * (F[(size_t)i * n + j] + F[(size_t)j * n + i]);
            F[(size_t)i * n + j] = a;
            F[(size_t)j * n + i] = a;
        }
    return 0;
}

static std::string fmt(const char* what, long a) { return std::string(what) + " " + std::to_string(a); }

int build_layout(const ProblemView& p, HostLayout& out, std::string& err, int threads) {
    if (p.n < 1 || p.S < 1) { err = "n and S must be positive"; return OPF_EINVAL; }
    if (!p.c || !p.lb || !p.ub || !p.comp_m || !p.comp_n || !p.idx || !p.b || !p.A) {
        err = "null array in problem"; return OPF_EINVAL;
    }
    const int n = p.n, S = p.S;
    std::vector<int64_t> aoff(S + 1), boff(S + 1), ioff(S + 1);
    aoff[0] = boff[0] = ioff[0] = 0;
    for (int s = 0; s < S; ++s) {
        const int m = p.comp_m[s], k = p.comp_n[s];
        if (m < 0 || k < 1 || k > kWave) {
            err = fmt("component size out of range (need 0 <= m_s, 1 <= n_s <= 64) at component", s);
            return OPF_EINVAL;
        }
        aoff[s + 1] = aoff[s] + (int64_t)m * k;
        boff[s + 1] = boff[s] + m;
        ioff[s + 1] = ioff[s] + k;
    }
    if (ioff[S] > INT32_MAX / 2) { err = "too many slots"; return OPF_EINVAL; }
    const int L = (int)ioff[S];
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(p.c[i])) { err = fmt("non-finite c at", i); return OPF_EINVAL; }
        if (std::isnan(p.lb[i]) || std::isnan(p.ub[i])) { err = fmt("NaN bound at", i); return OPF_EBOUNDS; }
        if (p.lb[i] > p.ub[i]) { err = fmt("lb > ub at", i); return OPF_EBOUNDS; }
        if (p.lb[i] == INFINITY || p.ub[i] == -INFINITY) { err = fmt("empty bound interval at", i); return OPF_EBOUNDS; }
    }
    for (int64_t q = 0; q < aoff[S]; ++q)
        if (!std::isfinite(p.A[q])) { err = fmt("non-finite entry of A at", (long)q); return OPF_EINVAL; }
    for (int64_t q = 0; q < boff[S]; ++q)
        if (!std::isfinite(p.b[q])) { err = fmt("non-finite entry of b at", (long)q); return OPF_EINVAL; }
    std::vector<int32_t> cnt(n, 0), mark(n, -1);
    for (int s = 0; s < S; ++s)
        for (int64_t q = ioff[s]; q < ioff[s + 1]; ++q) {
            const int g = p.idx[q];
            if (g < 0 || g >= n) { err = fmt("index out of range in component", s); return OPF_EINVAL; }
            if (mark[g] == s) { err = fmt("duplicate index inside component", s); return OPF_EINVAL; }
            mark[g] = s;
            cnt[g]++;
        }
    for (int i = 0; i < n; ++i)
        if (cnt[i] == 0) { err = fmt("global variable has no local copy:", i); return OPF_EUNCOVERED; }

    // ---- factors, in parallel over components (unless the device computes them)
    const bool host_factors = !out.factors_on_device;
    std::vector<int64_t> foff(S + 1);
    foff[0] = 0;
    for (int s = 0; s < S; ++s) foff[s + 1] = host_factors ? foff[s] + (int64_t)p.comp_n[s] * p.comp_n[s] : 0;
    std::vector<double> Fs(foff[S]), bb(host_factors ? L : 0);
    std::atomic<int> next(0), bad(-1), badcode(0);
    auto work = [&]() {
        for (;;) {
            const int s = next.fetch_add(16);
            if (s >= S) break;
            for (int u = s; u < std::min(S, s + 16); ++u) {
                int rank = 0;
                int rc = component_factor(p.comp_m[u], p.comp_n[u], p.A + aoff[u], p.b + boff[u],
                                          Fs.data() + foff[u], bb.data() + ioff[u], &rank);
                if (rc) { bad.store(u); badcode.store(rc); }
            }
        }
    };
    threads = std::max(1, std::min(threads, 64));
    if (host_factors) {
        std::vector<std::thread> pool;
        for (int t = 1; t < threads; ++t) pool.emplace_back(work);
        work();
        for (auto& th : pool) th.join();
    }
    if (bad.load() >= 0) {
        err = fmt("row reduction found 0 = nonzero (inconsistent equations) in component", bad.load());
        return badcode.load();
    }

    // ---- order components so that neighbours in the network sit together:
    // depth-first over the component graph (two components are adjacent when
    // they copy a common variable)
    std::vector<int32_t> vptr0(n + 1, 0);
    for (int i = 0; i < n; ++i) vptr0[i + 1] = vptr0[i] + cnt[i];
    std::vector<int32_t> vcomp(L);
    {
        std::vector<int32_t> f(vptr0.begin(), vptr0.end() - 1);
        for (int s2 = 0; s2 < S; ++s2)
            for (int64_t q = ioff[s2]; q < ioff[s2 + 1]; ++q) vcomp[f[p.idx[q]]++] = s2;
    }
    std::vector<int> order;
    order.reserve(S);
    {
        std::vector<char> seen(S, 0);
        std::vector<int> stack;
        for (int root = 0; root < S; ++root) {
            if (seen[root]) continue;
            stack.push_back(root);
            seen[root] = 1;
            while (!stack.empty()) {
                const int u = stack.back();
                stack.pop_back();
                order.push_back(u);
                for (int64_t q = ioff[u + 1] - 1; q >= ioff[u]; --q) {
                    const int g = p.idx[q];
                    for (int r = vptr0[g + 1] - 1; r >= vptr0[g]; --r) {
                        const int v2 = vcomp[r];
                        if (!seen[v2]) { seen[v2] = 1; stack.push_back(v2); }
                    }
                }
            }
        }
    }
    // components of group 1 first (each group keeps its depth-first order)
    const bool grouped = (int)out.comp_group.size() == S;
    if (grouped)
        std::stable_partition(order.begin(), order.end(), [&](int c2) { return out.comp_group[c2] == 1; });
    // ---- cut the order into workgroups of `block_waves` wavefronts; inside a
    // workgroup components are packed largest first with holes filled from the
    // small end, and a component never straddles two wavefronts
    const int B = out.block_waves > 0 ? out.block_waves : 4;
    auto pack = [&](const std::vector<int>& chunk, std::vector<std::vector<int>>& ws) {
        std::vector<int> srt(chunk);
        std::stable_sort(srt.begin(), srt.end(), [&](int a, int b2) { return p.comp_n[a] > p.comp_n[b2]; });
        std::deque<int> dq(srt.begin(), srt.end());
        ws.clear();
        while (!dq.empty()) {
            std::vector<int> w;
            int used = 0;
            while (!dq.empty() && used + p.comp_n[dq.front()] <= kWave) {
                used += p.comp_n[dq.front()];
                w.push_back(dq.front());
                dq.pop_front();
            }
            while (!dq.empty() && used + p.comp_n[dq.back()] <= kWave) {
                used += p.comp_n[dq.back()];
                w.push_back(dq.back());
                dq.pop_back();
            }
            ws.push_back(std::move(w));
        }
        return (int)ws.size() <= B;
    };
    std::vector<std::vector<int>> waves;
    std::vector<int> comp_block(S, -1);
    {
        std::vector<int> cur;
        std::vector<std::vector<int>> ws;
        int cur_lanes = 0;
        auto emit = [&]() {
            pack(cur, ws);
            const int blk = (int)(waves.size() / B);
            for (auto& w : ws) {
                for (int c2 : w) comp_block[c2] = blk;
                waves.push_back(w);
            }
            for (int e = (int)ws.size(); e < B; ++e) waves.push_back({});
            cur.clear();
            cur_lanes = 0;
        };
        for (int s2 : order) {
            if (grouped && !cur.empty() && out.comp_group[cur.back()] != out.comp_group[s2]) emit();
            cur.push_back(s2);
            cur_lanes += p.comp_n[s2];
            if (cur_lanes > B * kWave * 3 / 4 && !pack(cur, ws)) {
                cur.pop_back();
                emit();
                cur.push_back(s2);
                cur_lanes = p.comp_n[s2];
            }
        }
        if (!cur.empty()) emit();
    }
    out.block_waves = B;
    out.blocks = (int)(waves.size() / B);
    const int W = (int)waves.size();
    const int LP = W * kWave;
    out.n = n; out.S = S; out.L = L; out.waves = W;
    out.wave_maxn.assign(W, 0);
    out.wave_foff.assign(W, 0);
    out.var.assign(LP, -1);
    out.meta.assign(LP, 0);
    out.copy_start.assign(LP, 0);
    out.copy_cnt.assign(LP, 0);
    out.user_slot.assign(LP, -1);
    out.bbar.assign(LP, 0.0);
    out.lo.assign(LP, 0.0);
    out.hi.assign(LP, 0.0);
    out.cost.assign(LP, 0.0);
    out.z0.assign(LP, 0.0);
    out.user_to_dev.assign(L, -1);
    int64_t ftotal = 0;
    for (int wi = 0; wi < W; ++wi) {
        int maxn = 0;
        for (int s : waves[wi]) maxn = std::max(maxn, (int)p.comp_n[s]);
        out.wave_maxn[wi] = maxn;
        out.wave_foff[wi] = ftotal;
        ftotal += (int64_t)maxn * kWave;
    }
    out.F.assign(host_factors ? ftotal : 0, 0.0);
    if (!host_factors) {
        out.comp_dev.assign(S, -1);
        out.comp_aoff.assign(aoff.begin(), aoff.end() - 1);
        out.comp_boff.assign(boff.begin(), boff.end() - 1);
    }
    out.max_ns = 0;
    out.sum_ns2 = 0;
    for (int wi = 0; wi < W; ++wi) {
        int lane = 0;
        const int64_t fb = out.wave_foff[wi];
        for (int s : waves[wi]) {
            const int k = p.comp_n[s];
            out.max_ns = std::max(out.max_ns, k);
            out.sum_ns2 += (int64_t)k * k;
            if (!host_factors) out.comp_dev[s] = wi * kWave + lane;
            for (int j = 0; j < k; ++j) {
                const int d = wi * kWave + lane + j;
                const int us = (int)(ioff[s] + j);
                out.var[d] = p.idx[us];
                out.meta[d] = lane | (k << 8);
                out.user_slot[d] = us;
                out.user_to_dev[us] = d;
                if (!host_factors) continue;
                out.bbar[d] = bb[us];
                for (int q = 0; q < k; ++q)
                    out.F[fb + (int64_t)q * kWave + lane + j] = Fs[foff[s] + (int64_t)j * k + q];
            }
            lane += k;
        }
    }
    // ---- copy lists of B^T (device slots of each variable, ascending)
    std::vector<int32_t> vptr(n + 1, 0);
    for (int i = 0; i < n; ++i) vptr[i + 1] = vptr[i] + cnt[i];
    out.copy_list.assign(L, 0);
    std::vector<int32_t> fill(vptr.begin(), vptr.end() - 1);
    for (int d = 0; d < LP; ++d)
        if (out.var[d] >= 0) out.copy_list[fill[out.var[d]]++] = d;   // d ascending
    out.owner_slot.assign(n, -1);
    out.max_copies = 0;
    for (int i = 0; i < n; ++i) {
        out.owner_slot[i] = out.copy_list[vptr[i]];
        out.max_copies = std::max(out.max_copies, (int)cnt[i]);
    }
    // workgroups that own a copy of any variable of workgroup b (excluding b)
    {
        const int G = out.blocks;
        std::vector<std::vector<int>> nb(G);
        for (int i = 0; i < n; ++i) {
            for (int r = vptr[i]; r < vptr[i + 1]; ++r) {
                const int bi = out.copy_list[r] / (B * kWave);
                for (int r2 = vptr[i]; r2 < vptr[i + 1]; ++r2) {
                    const int bj = out.copy_list[r2] / (B * kWave);
                    if (bi != bj) nb[bi].push_back(bj);
                }
            }
        }
        out.nbr_ptr.assign(G + 1, 0);
        out.nbr_list.clear();
        for (int b2 = 0; b2 < G; ++b2) {
            std::sort(nb[b2].begin(), nb[b2].end());
            nb[b2].erase(std::unique(nb[b2].begin(), nb[b2].end()), nb[b2].end());
            out.nbr_list.insert(out.nbr_list.end(), nb[b2].begin(), nb[b2].end());
            out.nbr_ptr[b2 + 1] = (int32_t)out.nbr_list.size();
            out.max_nbrs = std::max(out.max_nbrs, (int)nb[b2].size());
        }
    }
    for (int d = 0; d < LP; ++d) {
        const int g = out.var[d];
        if (g < 0) continue;
        out.copy_start[d] = vptr[g];
        out.copy_cnt[d] = cnt[g];
        if (out.owner_slot[g] == d) out.meta[d] |= (1 << 16);
        out.lo[d] = p.lb[g];
        out.hi[d] = p.ub[g];
        out.cost[d] = p.c[g];
        double z0 = 0.0;
        const int kind = p.var_kind ? p.var_kind[g] : 0;
        if (kind == 2) z0 = 1.0;
        else if (std::isfinite(p.lb[g]) && std::isfinite(p.ub[g])) z0 = 0.5 * (p.lb[g] + p.ub[g]);
        out.z0[d] = z0;
    }
    out.c_full.assign(p.c, p.c + n);
    return 0;
}

int build_batch_rhs(const ProblemView& p, const HostLayout& lay, const double* b_scen, int K, int Kp,
                    std::vector<float>& out, std::string& err, int threads, const std::vector<int8_t>* skip) {
    const int S = p.S;
    std::vector<int64_t> aoff(S + 1), boff(S + 1), ioff(S + 1);
    aoff[0] = boff[0] = ioff[0] = 0;
    for (int s = 0; s < S; ++s) {
        aoff[s + 1] = aoff[s] + (int64_t)p.comp_m[s] * p.comp_n[s];
        boff[s + 1] = boff[s] + p.comp_m[s];
        ioff[s + 1] = ioff[s] + p.comp_n[s];
    }
    const int64_t M = boff[S];
    for (int64_t q = 0; q < M * K; ++q)
        if (!std::isfinite(b_scen[q])) { err = "non-finite scenario right-hand side"; return OPF_EINVAL; }
    out.assign((size_t)lay.waves * kWave * Kp, 0.0f);
    std::atomic<int> next(0), bad(-1);
    auto work = [&]() {
        std::vector<double> F, Wm, bb;
        for (;;) {
            const int s = next.fetch_add(8);
            if (s >= S) break;
            for (int u = s; u < std::min(S, s + 8); ++u) {
                if (skip && (*skip)[u]) continue;      // factored per scenario elsewhere
                const int m = p.comp_m[u], n = p.comp_n[u];
                F.assign((size_t)n * n, 0.0);
                Wm.assign((size_t)n * std::max(m, 1), 0.0);
                if (m > 0) component_rhs_map(m, n, p.A + aoff[u], F.data(), Wm.data());
                bb.assign(n, 0.0);
                for (int k = 0; k < K; ++k) {
                    const double* b = b_scen + (size_t)k * M + boff[u];
                    for (int i = 0; i < n; ++i) {
                        double acc = 0.0;
                        for (int j = 0; j < m; ++j) acc += Wm[(size_t)i * m + j] * b[j];
                        bb[i] = acc;
                    }
                    // the scenario's equations must hold at bbar (consistent right-hand side)
                    double bmax = 1.0, rmax = 0.0, amax = 0.0;
                    for (int j = 0; j < m; ++j) {
                        double acc = 0.0;
                        for (int i = 0; i < n; ++i) {
                            acc += p.A[aoff[u] + (size_t)j * n + i] * bb[i];
                            amax = std::max(amax, std::fabs(p.A[aoff[u] + (size_t)j * n + i]));
                        }
                        rmax = std::max(rmax, std::fabs(acc - b[j]));
                        bmax = std::max(bmax, std::fabs(b[j]));
                    }
                    if (rmax > 1e-9 * bmax * std::max(1.0, amax)) bad.store(u);
                    for (int i = 0; i < n; ++i) {
                        const int d = lay.user_to_dev[ioff[u] + i];
                        out[(size_t)d * Kp + k] = (float)bb[i];
                    }
                }
            }
        }
    };
    threads = std::max(1, std::min(threads, 64));
    std::vector<std::thread> pool;
    for (int t = 1; t < threads; ++t) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
    if (bad.load() >= 0) {
        err = fmt("scenario right-hand side inconsistent with the equations of component", bad.load());
        return OPF_EINFEASIBLE_COMPONENT;
    }
    return 0;
}

static uint16_t to_bf16(double v) {
    float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    const uint32_t rounding = 0x7fffu + ((u >> 16) & 1u);              // nearest even
    return (uint16_t)((u + rounding) >> 16);
}
static double from_bf16(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}

void build_dense_planes(const HostLayout& lay, int terms, std::vector<uint16_t>& planes) {
    const size_t per = (size_t)kWave * kWave;
    planes.assign((size_t)terms * lay.waves * per, 0);
    for (int w = 0; w < lay.waves; ++w) {
        for (int r = 0; r < kWave; ++r) {
            const int d = w * kWave + r;
            if (lay.var[d] < 0) continue;
            const int b0 = lay.meta[d] & 255, ns = (lay.meta[d] >> 8) & 255;
            for (int k = 0; k < ns; ++k) {
                double rem = lay.F[lay.wave_foff[w] + (int64_t)k * kWave + r];
                for (int t = 0; t < terms; ++t) {
                    const uint16_t h = to_bf16(rem);
                    planes[(size_t)t * lay.waves * per + (size_t)w * per + (size_t)r * kWave + b0 + k] = h;
                    rem -= from_bf16(h);
                }
            }
        }
    }
}

}  // namespace opf
