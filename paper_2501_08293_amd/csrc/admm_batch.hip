// Batched same-topology scenarios on MFMA (gfx950).
//
// K load scenarios share every A_s (constant-power loads), so they share the
// projection factors F_s and differ only in bbar_s.  One iteration of
// Algorithm 1 for all scenarios at once:
//   phase 1  per slot and scenario, the clipped consensus average of the slot's
//            variable (global_sparse) and the projection input
//            V = B_s x + lambda_s / rho, staged in LDS as a 64-slot x 64-scenario tile;
//   phase 2  the local update (closed_2) of every component of a packed
//            wavefront as one dense product Z = F_w V with F_w the 64 x 64
//            block-diagonal factor of the wavefront: four 32 x 32 output tiles,
//            one per wave, each accumulated by v_mfma_f32_32x32x16_bf16 over
//            K = 64 in FP32.  F_w and V are split into bfloat16 terms
//            (F = F1 + F2 + F3, V likewise) and the products with term order
//            i + j <= terms + 1 are summed (6 products for 3 terms), which keeps
//            FP32-level accuracy; a two-term split leaves a rounding floor above
//            the paper's dual-residual test at 1e-4;
//   phase 3  z = Z + bbar, the dual update (ADMM-3) and per-scenario FP64
//            residual partial sums.
// Wavefronts of components whose A_s changes with the scenario (ZIP loads)
// take phase 2 as a per-scenario product with their own FP32 factors instead.
// A second launch reduces the partials per scenario, applies the termination
// test per scenario and records each scenario's solution at its own stop
// iteration; the batch runs until every scenario has stopped.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/opf_admm.h"
#include "admm_batch.h"
#include "admm_kernels.h"

namespace opf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 as_bf16x8(const uint16_t (&h)[8]) {
    bf16x8 r;
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = __builtin_bit_cast(__bf16, h[i]);
    return r;
}

// Element at a 32-bit byte offset from a base address that is the same for
// the whole workgroup (one base register pair instead of a 64-bit address per
// load in flight).
__device__ __forceinline__ float ld32(const float* base, uint32_t off) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + off);
}
__device__ __forceinline__ void st32(float* base, uint32_t off, float v) {
    *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + off) = v;
}

__device__ __forceinline__ double wave_sum_b(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// grid W * Kp / 64, 256 threads: workgroup (wavefront w of the packing,
// scenarios [kc, kc + 64)).  Order (tuned per problem, every order computes
// the same values): bit 0 set, each XCD runs a contiguous range of packing
// positions, so the copies of a variable (in nearby wavefronts) and the
// scenario tiles of one factor tile meet in one L2; bit 1 set, positions run
// scenario-chunk-major (all wavefronts of one 64-scenario chunk, then the
// next) instead of wavefront-major.  The workgroups of the scenario-varying
// wavefronts (the slowest, packed first) are dealt over all XCDs and start
// first.
//
// Phases 1 and 3 share one layout (wave wv: slots 16 wv .. 16 wv + 15, lane:
// scenario), so x and the slot's own lambda, loaded in phase 1, stay in
// registers until phase 3; the product Z comes back from the matrix cores
// through the V tile's LDS.  LDS 30 KiB.  Four wavefronts per SIMD (at most
// 128 registers; the matrix-core accumulators live in ordinary VGPRs): the
// kernel is bound by the latency of its dependent memory rounds, so the
// fourth workgroup per CU is worth more than a few registers.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void admm_batch_step_kernel(BatchArgs a) {
    if (a.ctrl->stop) return;
    const long long t = a.ctrl->iter + 1;
    const bool odd = (t & 1) != 0;
    const size_t Kp = (size_t)a.Kp;

    __shared__ __align__(16) float vs[64][65];   // V = B x + lambda / rho, then Z = F_w V   [slot][scenario]
    __shared__ double red[4][5][64];              // residual partials per wave and scenario

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int KB = a.nc;                       // chunks of this launch
    const int nvb = a.vary_waves * KB, bx = (int)blockIdx.x;
    const int rest = (int)gridDim.x - nvb;
    int pos = bx < nvb ? bx : nvb + logical_block(bx - nvb, rest, a.order & 1);
    if ((a.order & 2) && pos >= nvb) {
        // chunk-major over the wavefronts after the scenario-varying ones
        const int q = pos - nvb, wr = rest / KB;
        pos = nvb + (q % wr) * KB + q / wr;
    }
    const int w = pos / KB;
    const int chunk = a.c0 + (pos - w * KB), kc = chunk * 64;
    // state of this 64-scenario chunk: [slot][64] (x: [variable][64])
    const size_t sb = (size_t)chunk * a.W * 64 * 64, xb = (size_t)chunk * a.n * 64;
    const float* zp = (odd ? a.z0 : a.z1) + sb;
    const float* lp = (odd ? a.l0 : a.l1) + sb;
    float* zq = (odd ? a.z1 : a.z0) + sb;
    float* lq = (odd ? a.l1 : a.l0) + sb;
    float* xq = (odd ? a.x1 : a.x0) + xb;
    const float* bbar = a.bbar + sb;

    // ---- slot descriptors of this wavefront staged in LDS: one 16-byte
    // record per slot and its first copies, loaded side by side
    __shared__ int s_var[64], s_cn[64], s_cs[64], s_owner[64];
    __shared__ float s_cost[64], s_lo[64], s_hi[64];
    __shared__ int s_copy[64][kBatchCopies];
    if (tid < 64) {
        const int d = w * 64 + tid;
        const int4 sd = a.sdesc[d];
        const float4 sv = a.sval[d];
        s_var[tid] = sd.x;
        s_cn[tid] = sd.y;
        s_cs[tid] = sd.z;
        s_owner[tid] = sd.w;
        s_cost[tid] = sv.x * a.inv_rho;
        s_lo[tid] = sv.y;
        s_hi[tid] = sv.z;
    } else if (tid < 128) {
        const int r = tid - 64;
        const int4 c0 = a.scopy[(size_t)(w * 64 + r) * 2];
        const int4 c1 = a.scopy[(size_t)(w * 64 + r) * 2 + 1];
        const int c[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
        for (int q = 0; q < kBatchCopies; ++q) s_copy[r][q] = c[q];
    }
    __syncthreads();

    // ---- phase 1: consensus average and projection input, 16 slots per
    // wave in groups of eight: copies 0 and 1 of the eight slots are gathered
    // together, then copies 2-3 and 4-5 only where some of the eight slots
    // have them (a slot's copy count is the same on every lane); each slot's
    // terms are summed in copy order
    const uint32_t lane4 = 4u * lane;
    float xr[16], lr[16];
#pragma unroll
    for (int r0 = 0; r0 < 16; r0 += 8) {
        float acc[8];
        int cmax = 0;
#pragma unroll
        for (int q0 = 0; q0 < kBatchCopies; q0 += 2) {
            if (q0 > 0 && q0 >= cmax) break;
            float zz[8][2], ll[8][2];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int r = wv * 16 + r0 + j;
                const int cn = s_cn[r];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const uint32_t e = (uint32_t)s_copy[r][q0 + q] * 256u + lane4;
                    zz[j][q] = q0 + q < cn ? ld32(zp, e) : 0.0f;
                    ll[j][q] = q0 + q < cn ? ld32(lp, e) : 0.0f;
                }
                if (q0 == 0) {
                    const uint32_t dk = (uint32_t)(w * 64 + r) * 256u + lane4;
                    lr[r0 + j] = s_var[r] >= 0 ? ld32(lp, dk) : 0.0f;
                    cmax = cn > cmax ? cn : cmax;
                }
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int cn = s_cn[wv * 16 + r0 + j];
                if (q0 == 0) acc[j] = 0.0f;
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    if (q0 + q < cn) acc[j] += zz[j][q] - ll[j][q] * a.inv_rho;
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int r = wv * 16 + r0 + j;
            const int g = s_var[r];
            const int cn = s_cn[r];
            float xv = 0.0f, vv = 0.0f;
            if (g >= 0) {
                float sum = acc[j];
                for (int q = kBatchCopies; q < cn; ++q) {
                    const uint32_t e = (uint32_t)a.clist[s_cs[r] + q] * 256u + lane4;
                    sum += ld32(zp, e) - ld32(lp, e) * a.inv_rho;
                }
                const float xh = (sum - s_cost[r]) / (float)cn;
                xv = xh < s_lo[r] ? s_lo[r] : (xh > s_hi[r] ? s_hi[r] : xh);
                vv = xv + lr[r0 + j] * a.inv_rho;
                if (s_owner[r]) st32(xq, (uint32_t)g * 256u + lane4, xv);
            }
            xr[r0 + j] = xv;
            vs[r][lane] = vv;
        }
    }
    __syncthreads();

    // ---- phase 2: Z (64 x 64) = F_w (64 x 64) V (64 x 64); wave wv owns the
    // 32 x 32 tile (rows 32 m .., scenarios 32 nt ..)
    const int m = wv & 1, nt = wv >> 1;
    const int grp = lane >> 5, l32 = lane & 31;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    const int vw = a.wave_var ? a.wave_var[w] : -1;
    if (vw >= 0) {
        // per-scenario factors: output (row r, scenario col) of this lane's
        // sixteen tile positions, each summed over the component's columns in
        // order; the sixteen factor loads of one column are in flight together
        const int col = 32 * nt + l32;
        const int r0 = 32 * m + 4 * grp;     // row of tile position v: r0 + 8 (v / 4) + v % 4
        // column base lanes of the sixteen rows (< 64), four to a register, and
        // the largest component size among the wavefront's rows: the factors of
        // a row are zero past its component's columns, so the columns beyond
        // every row's size are skipped
        unsigned bases[4] = {0u, 0u, 0u, 0u};
        int ncol = 0;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int mt = a.meta[(size_t)w * 64 + r0 + 8 * (v >> 2) + (v & 3)];
            bases[v >> 2] |= (unsigned)(mt & 255) << (8 * (v & 3));
            ncol = max(ncol, (mt >> 8) & 255);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) ncol = max(ncol, __shfl_xor(ncol, o, 64));
        ncol = min(__builtin_amdgcn_readfirstlane(ncol), a.fv_cols);
        // this wavefront's factors [column][row][scenario] from one base, at 32-bit
        // byte offsets (at most 64 x 64 x 4096 floats)
        const float* Fw = a.Fv + (size_t)vw * a.fv_cols * 64 * Kp;
        const uint32_t rs = (uint32_t)Kp * 4u, js = 64u * rs;
        const uint32_t o0 = (uint32_t)r0 * rs + (uint32_t)(kc + col) * 4u;
        for (int j = 0; j < ncol; ++j) {
            const uint32_t oj = o0 + (uint32_t)j * js;
            float f[16];
#pragma unroll
            for (int v = 0; v < 16; ++v) f[v] = ld32(Fw, oj + (uint32_t)(8 * (v >> 2) + (v & 3)) * rs);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int bv = (int)((bases[v >> 2] >> (8 * (v & 3))) & 255u);
                acc[v] = fmadd(f[v], vs[(bv + j) & 63][col], acc[v]);
            }
        }
    } else {
    const size_t plane = (size_t)a.W * 64 * 64;
    const uint16_t* Fw = a.Fp + (size_t)w * 64 * 64 + (size_t)(32 * m + l32) * 64;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k0 = 16 * q + 8 * grp;
        // B operand: V[k0 + i][32 nt + l32], split into bf16 terms
        uint16_t b1[8], b2[8], b3[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float v = vs[k0 + i][32 * nt + l32];
            b1[i] = bf16_bits(v);
            const float r1 = v - bf16_val(b1[i]);
            b2[i] = bf16_bits(r1);
            const float r2 = r1 - bf16_val(b2[i]);
            b3[i] = bf16_bits(r2);
        }
        // A operand: F_w[32 m + l32][k0 .. k0 + 7] of each plane (16 bytes)
        uint16_t a1[8], a2[8], a3[8];
        {
            const uint4 u1 = *reinterpret_cast<const uint4*>(Fw + k0);
            const uint4 u2 = *reinterpret_cast<const uint4*>(Fw + plane + k0);
            __builtin_memcpy(a1, &u1, 16);
            __builtin_memcpy(a2, &u2, 16);
            if (a.terms >= 3) {
                const uint4 u3 = *reinterpret_cast<const uint4*>(Fw + 2 * plane + k0);
                __builtin_memcpy(a3, &u3, 16);
            }
        }
        const bf16x8 A1 = as_bf16x8(a1), A2 = as_bf16x8(a2), B1 = as_bf16x8(b1), B2 = as_bf16x8(b2);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, B1, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, B2, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A2, B1, acc, 0, 0, 0);
        if (a.terms >= 3) {
            const bf16x8 A3 = as_bf16x8(a3), B3 = as_bf16x8(b3);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, B3, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A2, B2, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A3, B1, acc, 0, 0, 0);
        }
    }
    }

    // ---- Z into the V tile's LDS once every wave has read V
    // D[row][col] of a 32 x 32 tile: col = lane % 32, row = 8 (v / 4) + 4 (lane / 32) + v % 4
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 16; ++v) vs[32 * m + 8 * (v >> 2) + 4 * grp + (v & 3)][32 * nt + l32] = acc[v];
    __syncthreads();

    // ---- phase 3: z = Z + bbar, dual update, residual partials (phase 1's layout).
    // The old z and bbar of all sixteen slots are loaded before any store (a
    // load after a store to a possibly aliasing address would wait for it),
    // unconditionally: padding slots have state too, and a conditional load
    // would wait at its branch's join.
    float zo16[16], bb16[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t dk = (uint32_t)(w * 64 + wv * 16 + j) * 256u + lane4;
        zo16[j] = ld32(zp, dk);
        bb16[j] = ld32(bbar, dk);
    }
    double s[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int r = wv * 16 + j;
        if (s_var[r] >= 0) {
            const uint32_t dk = (uint32_t)(w * 64 + r) * 256u + lane4;
            const float zo = zo16[j];
            const float zn = vs[r][lane] + bb16[j];
            const float xv = xr[j];
            const float ln = lr[j] + a.rho * (xv - zn);
            st32(zq, dk, zn);
            st32(lq, dk, ln);
            const double xd = xv, zd = zn;
            s[0] += (xd - zd) * (xd - zd);
            s[1] += (zd - (double)zo) * (zd - (double)zo);
            s[2] += xd * xd;
            s[3] += zd * zd;
            s[4] += (double)ln * (double)ln;
        }
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) red[wv][i][lane] = s[i];
    __syncthreads();
    if (wv == 0) {
        const size_t k = (size_t)(kc + lane);
#pragma unroll
        for (int i = 0; i < 5; ++i)
            a.part[((size_t)i * Kp + k) * a.W + w] = (red[0][i][lane] + red[1][i][lane]) + (red[2][i][lane] + red[3][i][lane]);
    }
}

// grid K, 256 threads: reduction of scenario blockIdx.x, its stop decision and
// the snapshot of its solution; the last workgroup advances the iteration.
__global__ __launch_bounds__(256) void admm_batch_reduce_kernel(BatchRedArgs r) {
    BatchCtrl* ctrl = r.ctrl;
    if (ctrl->stop) return;
    const long long t = ctrl->iter + 1;
    const int k = r.k0 + (int)blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __shared__ double red[4][5];
    __shared__ int decide;
    double a[5] = {0, 0, 0, 0, 0};
    for (int w = threadIdx.x; w < r.W; w += 256)
#pragma unroll
        for (int i = 0; i < 5; ++i) a[i] += r.part[((size_t)i * r.Kp + k) * r.W + w];
#pragma unroll
    for (int i = 0; i < 5; ++i) a[i] = wave_sum_b(a[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 5; ++i) red[wv][i] = a[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        double S[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) S[i] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
        const double pres = sqrt(S[0]);
        const double dres = r.rho * sqrt(S[1]);
        const double ep = r.eps_rel * fmax(sqrt(S[2]), sqrt(S[3]));
        const double ed = r.eps_rel * sqrt(S[4]);
        int st = 0;
        if (r.state[k] == 0) {
            if (!(isfinite(pres) && isfinite(dres) && isfinite(ep) && isfinite(ed))) st = 3;
            else if (pres <= ep && dres <= ed) st = 1;
            else if (t >= ctrl->max_iter) st = 2;
            if (st) {
                r.state[k] = st;
                r.iters[k] = t;
                r.res[k * 4 + 0] = pres;
                r.res[k * 4 + 1] = dres;
                r.res[k * 4 + 2] = ep;
                r.res[k * 4 + 3] = ed;
                __hip_atomic_fetch_add(&ctrl->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        decide = st;
    }
    __syncthreads();
    if (decide) {
        // snapshot x of this scenario at its stop iteration and its objective
        const float* xs = ((t & 1) ? r.x1 : r.x0) + (size_t)(k >> 6) * r.n * 64 + (k & 63);
        double obj = 0.0;
        for (int i = threadIdx.x; i < r.n; i += 256) {
            const double xv = (double)xs[(size_t)i * 64];
            r.xout[(size_t)k * r.n + i] = xv;
            obj += r.c[i] * xv;
        }
        obj = wave_sum_b(obj);
        __syncthreads();
        if (lane == 0) red[wv][0] = obj;
        __syncthreads();
        if (threadIdx.x == 0) r.objective[k] = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    }
    if (threadIdx.x == 0) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const unsigned old = __hip_atomic_fetch_add(&ctrl->arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old == gridDim.x - 1) {
            const int done = __hip_atomic_load(&ctrl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ctrl->iter = t;
            if (done >= (int)gridDim.x || t >= ctrl->max_iter) ctrl->stop = 1;
            ctrl->arrive = 0u;
        }
    }
}

__global__ void batch_init_kernel(const double* z0, float* z, float* l, int LP, int Kp, BatchCtrl* ctrl,
                                  int groups, int* state, int K, long long max_iter) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t tot = (size_t)LP * Kp;
    if (i < tot) {
        // chunk-major: [Kp / 64][LP][64]
        z[i] = (float)z0[(i >> 6) % (size_t)LP];
        l[i] = 0.0f;
    }
    if (i < (size_t)K) state[i] = 0;
    if (i < (size_t)groups) {
        ctrl[i].iter = 0;
        ctrl[i].max_iter = max_iter;
        ctrl[i].stop = 0;
        ctrl[i].done = 0;
        ctrl[i].arrive = 0u;
    }
}

hipError_t launch_batch_iteration(const BatchArgs& a, const BatchRedArgs& r, int kn, hipStream_t st) {
    if (a.nc < 1 || kn < 1 || a.c0 < 0 || a.c0 + a.nc > a.Kp / 64 || r.k0 < 0 || r.k0 + kn > r.K)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(admm_batch_step_kernel, dim3(a.W * a.nc), dim3(256), 0, st, a);
    hipLaunchKernelGGL(admm_batch_reduce_kernel, dim3(kn), dim3(256), 0, st, r);
    return hipGetLastError();
}

hipError_t launch_batch_init(const double* z0, float* z, float* l, int LP, int Kp, BatchCtrl* ctrl, int groups,
                             int* state, int K, long long max_iter, hipStream_t st) {
    const size_t tot = std::max((size_t)LP * Kp, (size_t)std::max(K, groups));
    hipLaunchKernelGGL(batch_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, z0, z, l, LP, Kp,
                       ctrl, groups, state, K, max_iter);
    return hipGetLastError();
}

}  // namespace opf
