// Device-side set-up (gfx950): the per-component factors of the local update,
// computed on the GPU instead of the host threads.
//
// One 64-lane workgroup per component, working in LDS:
//   1. row reduction of [A_s | b_s] to reduced row echelon form with partial
//      pivoting (Section IV-B); rows that vanish are dropped, and a vanishing
//      row with a nonzero right-hand side marks the component infeasible;
//   2. G = Ahat Ahat^T and its Cholesky factor;
//   3. W = G^{-1} [Ahat | bhat] by forward and back substitution;
//   4. F_s = I - Ahat^T W[:, :n] (symmetrised) and bbar_s = Ahat^T W[:, n]
//      (closed_2: the projection onto {A_s y = b_s}),
// written straight into the packed [k][lane] factor layout of the iteration
// kernels.  Pivot tolerance and inconsistency test are the host set-up's:
// tol = max(m, n) * eps * max|A_s|, |rhs| > tol * max(1, max|b_s|).
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstdint>

#include "../../include/opf_admm.h"
#include "admm_kernels.h"
#include "setup_device.h"

namespace opf {

namespace {

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// (value, row) with the largest value, ties to the smaller row
__device__ __forceinline__ void wave_argmax(double& v, int& r) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double v2 = __shfl_xor(v, o, 64);
        const int r2 = __shfl_xor(r, o, 64);
        if (v2 > v || (v2 == v && r2 < r)) {
            v = v2;
            r = r2;
        }
    }
}

}  // namespace

__global__ __launch_bounds__(64) void factor_kernel(FactorJob j) {
    extern __shared__ __align__(16) double sm[];
    const int s = blockIdx.x;
    if (s >= j.S) return;
    const int lane = threadIdx.x;
    const int m = j.comp_m[s], n = j.comp_n[s], w = n + 1;
    double* M = sm;                         // [m][w]
    double* G = M + (size_t)m * w;          // [m][m]
    double* Wm = G + (size_t)m * m;         // [m][w]
    double* fcol = Wm + (size_t)m * w;      // [m]
    const double* A = j.A + j.aoff[s];
    const double* b = j.b + j.boff[s];

    double amax = 0.0, bmax = 0.0;
    for (int q = lane; q < m * w; q += 64) {
        const int r = q / w, c = q - r * w;
        const double v = c < n ? A[(size_t)r * n + c] : b[r];
        M[q] = v;
        if (c < n) amax = fmax(amax, fabs(v));
        else bmax = fmax(bmax, fabs(v));
    }
    amax = wave_max_d(amax);
    bmax = wave_max_d(bmax);
    __syncthreads();
    const double tol = (double)(m > n ? m : n) * DBL_EPSILON * fmax(amax, 1e-300);

    // ---- Gauss-Jordan elimination with partial pivoting
    int row = 0;
    for (int col = 0; col < n && row < m; ++col) {
        double best = -1.0;
        int p = m;
        for (int r = row + lane; r < m; r += 64) {
            const double v = fabs(M[(size_t)r * w + col]);
            if (v > best) {
                best = v;
                p = r;
            }
        }
        wave_argmax(best, p);
        if (best <= tol) {
            for (int r = row + lane; r < m; r += 64) M[(size_t)r * w + col] = 0.0;
            __syncthreads();
            continue;
        }
        if (p != row) {
            for (int c = lane; c < w; c += 64) {
                const double t = M[(size_t)p * w + c];
                M[(size_t)p * w + c] = M[(size_t)row * w + c];
                M[(size_t)row * w + c] = t;
            }
            __syncthreads();
        }
        const double inv = 1.0 / M[(size_t)row * w + col];
        __syncthreads();
        for (int c = lane; c < w; c += 64) M[(size_t)row * w + c] *= inv;
        __syncthreads();
        if (lane == 0) M[(size_t)row * w + col] = 1.0;
        for (int r = lane; r < m; r += 64) fcol[r] = (r == row) ? 0.0 : M[(size_t)r * w + col];
        __syncthreads();
        for (int q = lane; q < m * w; q += 64) {
            const int r = q / w, c = q - r * w;
            const double f = fcol[r];
            if (f != 0.0) M[q] = fmadd(-f, M[(size_t)row * w + c], M[q]);
        }
        __syncthreads();
        for (int r = lane; r < m; r += 64)
            if (r != row && fcol[r] != 0.0) M[(size_t)r * w + col] = 0.0;
        __syncthreads();
        ++row;
    }
    const int k = row;
    // ---- rows that vanished must have a vanishing right-hand side
    int bad = 0;
    const double bscale = fmax(1.0, bmax);
    for (int r = k + lane; r < m; r += 64) bad |= fabs(M[(size_t)r * w + n]) > tol * bscale;
    if (__syncthreads_or(bad)) {
        if (lane == 0) j.status[s] = OPF_EINFEASIBLE_COMPONENT;
        return;
    }
    // ---- G = Ahat Ahat^T (lower triangle), Cholesky in place
    for (int q = lane; q < k * k; q += 64) {
        const int r = q / k, c = q - r * k;
        if (c > r) continue;
        double acc = 0.0;
        for (int t = 0; t < n; ++t) acc = fmadd(M[(size_t)r * w + t], M[(size_t)c * w + t], acc);
        G[(size_t)r * k + c] = acc;
    }
    __syncthreads();
    for (int c = 0; c < k; ++c) {
        double d = G[(size_t)c * k + c];
        for (int q = 0; q < c; ++q) d = fmadd(-G[(size_t)c * k + q], G[(size_t)c * k + q], d);
        if (!(d > 0.0)) {
            if (lane == 0) j.status[s] = OPF_EINFEASIBLE_COMPONENT;
            return;                              // uniform: every lane computed the same d
        }
        d = sqrt(d);
        for (int r = c + 1 + lane; r < k; r += 64) {
            double acc = G[(size_t)r * k + c];
            for (int q = 0; q < c; ++q) acc = fmadd(-G[(size_t)r * k + q], G[(size_t)c * k + q], acc);
            G[(size_t)r * k + c] = acc / d;
        }
        __syncthreads();
        if (lane == 0) G[(size_t)c * k + c] = d;
        __syncthreads();
    }
    // ---- W = G^{-1} [Ahat | bhat], one column per lane
    for (int c = lane; c < w; c += 64) {
        for (int i = 0; i < k; ++i) {
            double acc = M[(size_t)i * w + c];
            for (int q = 0; q < i; ++q) acc = fmadd(-G[(size_t)i * k + q], Wm[(size_t)q * w + c], acc);
            Wm[(size_t)i * w + c] = acc / G[(size_t)i * k + i];
        }
        for (int i = k - 1; i >= 0; --i) {
            double acc = Wm[(size_t)i * w + c];
            for (int q = i + 1; q < k; ++q) acc = fmadd(-G[(size_t)q * k + i], Wm[(size_t)q * w + c], acc);
            Wm[(size_t)i * w + c] = acc / G[(size_t)i * k + i];
        }
    }
    __syncthreads();
    // ---- F = I - Ahat^T W[:, :n] (symmetrised), bbar = Ahat^T W[:, n]
    const int d0 = j.comp_dev[s];
    const int base = d0 & 63;
    double* Fw = j.F + j.wave_foff[d0 >> 6];
    for (int q = lane; q < n * n; q += 64) {
        const int r = q / n, c = q - r * n;
        double sa = 0.0, sb = 0.0;
        for (int t = 0; t < k; ++t) {
            sa = fmadd(M[(size_t)t * w + r], Wm[(size_t)t * w + c], sa);
            sb = fmadd(M[(size_t)t * w + c], Wm[(size_t)t * w + r], sb);
        }
        const double id = (r == c) ? 1.0 : 0.0;
        Fw[(size_t)c * 64 + base + r] = 0.5 * ((id - sa) + (id - sb));
    }
    for (int r = lane; r < n; r += 64) {
        double acc = 0.0;
        for (int t = 0; t < k; ++t) acc = fmadd(M[(size_t)t * w + r], Wm[(size_t)t * w + n], acc);
        j.bbar[d0 + r] = acc;
    }
    if (lane == 0) j.status[s] = 0;
}

// FP32 copies of the factors and bbar for the mixed-precision bulk phase.
__global__ void narrow_kernel(const double* src, float* dst, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = (float)src[i];
}

// LDS bytes the factor kernel needs for an m x n component.
size_t factor_lds_bytes(int m, int n) {
    return sizeof(double) * ((size_t)2 * m * (n + 1) + (size_t)m * m + (size_t)m);
}

hipError_t launch_factors(const FactorJob& job, size_t lds_bytes, hipStream_t st) {
    if (job.S < 1) return hipSuccess;
    hipLaunchKernelGGL(factor_kernel, dim3(job.S), dim3(64), lds_bytes, st, job);
    return hipGetLastError();
}

hipError_t launch_narrow(const double* src, float* dst, int64_t count, hipStream_t st) {
    if (count < 1) return hipSuccess;
    hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, src, dst, count);
    return hipGetLastError();
}

}  // namespace opf
