// Device set-up of the component factors (internal header; see setup_device.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace opf {

// ---- device set-up of the component factors (see setup_device.hip)
struct FactorJob {
    const double* A;          // concatenated row-major m_s x n_s blocks
    const double* b;          // concatenated m_s entries
    const int64_t* aoff;      // [S]
    const int64_t* boff;      // [S]
    const int* comp_m;        // [S]
    const int* comp_n;        // [S]
    const int* comp_dev;      // [S] first device slot of the component
    const int64_t* wave_foff; // [waves] element offset of each wave's factor block
    double* F;                // packed factors (zeroed before the launch)
    double* bbar;             // [lanes]
    int* status;              // [S] 0 or OPF_EINFEASIBLE_COMPONENT
    int S;
};
size_t factor_lds_bytes(int m, int n);
hipError_t launch_factors(const FactorJob& job, size_t lds_bytes, hipStream_t st);
hipError_t launch_narrow(const double* src, float* dst, int64_t count, hipStream_t st);

}  // namespace opf
